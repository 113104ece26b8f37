// tm_scan.hip -- stages a2 and a3: the integral images of v and v^2 (Eq. 5) and the
// integral histogram (Eq. 7-8), built in one pass over the luminance.
//
// Decomposition (reduce, then scan; no workgroup ever waits on another):
//   stage 1  every 64-lane wave owns a tile of th rows x 64*VEC columns and writes the
//            tile's row totals RS[y][tx], column totals CS[ty][x] and total TT[ty][tx];
//   stage 2  three families of independent 1-D exclusive scans over those aggregates:
//            XC  = prefix of RS along tx, CSE = prefix of CS along ty,
//            TTE = prefix of TT along tx;
//   stage 3  every tile re-reads its pixels and forms
//              I(x, y) = sum_{ty'<ty} TTE[ty'][tx] + sum_{x0<=x'<=x} CSE[ty][x']
//                        + sum_{y0<=y'<=y} (XC[y'][tx] + sum_{x0<=x'<=x} q(x', y')),
//            i.e. the sums above the tile plus the tile's own 2-D prefix.  Row prefixes
//            use an in-lane prefix over the lane's VEC consecutive columns and a DPP wave
//            scan of the lane totals; column prefixes run down the tile in registers.
// The image is read twice (4 bytes/pixel each) and every table entry is written once; the
// aggregates are 1/th and 1/(64 VEC) of the image.  Histogram counts are exact uint32; the
// integral image accumulates in the precision's own arithmetic (FP32, compensated FP32
// pairs, or FP64), in a fixed order, so results are bit-reproducible.
#include <float.h>
#include <math.h>

#include "tm_device.h"
#include "tm_internal.h"

namespace tmo {

namespace {

constexpr int kBlock = 256;
constexpr int kWavesPerBlock = kBlock / kWave;


// ---------------------------------------------------------------- table entries
template <int P>
struct Entry;
template <>
struct Entry<kF32> {
    using T = float2;
    __device__ static T make(float a, float b) { return make_float2(a, b); }
    __device__ static T zero() { return make_float2(0.f, 0.f); }
};
template <>
struct Entry<kC32x2> {
    using T = float4;
    __device__ static T make(f2 a, f2 b) { return make_float4(a.hi, a.lo, b.hi, b.lo); }
    __device__ static T zero() { return make_float4(0.f, 0.f, 0.f, 0.f); }
};
template <>
struct Entry<kF64> {
    using T = double2;
    __device__ static T make(double a, double b) { return make_double2(a, b); }
    __device__ static T zero() { return make_double2(0.0, 0.0); }
};

// Load the lane's VEC consecutive pixels of row y (zeros outside the image).  wide: the
// whole tile lies inside the image and its rows are 16-byte aligned.  The choice is
// tile-uniform, so the two forms are separate paths rather than one masked sequence (where
// the element loads would have to wait for the vector load into the same registers).
template <int VEC>
__device__ __forceinline__ void load_row(const ScanK &k, int y, int xl, bool wide,
                                         float (&v)[VEC]) {
    const TM_GLOBAL float *row = gptr(k.v) + (int64_t)y * k.ld_v;
    if ((VEC % 4 == 0) && wide) {
#pragma unroll
        for (int i = 0; i < VEC; i += 4) {
            float4 t = *reinterpret_cast<const TM_GLOBAL float4 *>(row + xl + i);
            v[i] = t.x; v[i + 1] = t.y; v[i + 2] = t.z; v[i + 3] = t.w;
        }
    } else {
#pragma unroll
        for (int i = 0; i < VEC; ++i) v[i] = (xl + i < k.W) ? row[xl + i] : 0.f;
    }
}

// Histogram plane indicator: cumulative plane p counts bins < p+1 (v < edge[p]);
// per-bin plane p counts bin p (edge[p-1] <= v < edge[p]).
template <int CHUNK>
struct PlaneEdges {
    float lo[CHUNK], hi[CHUNK];
    int np;   // planes in this chunk
};
template <int CHUNK>
__device__ __forceinline__ PlaneEdges<CHUNK> chunk_edges(const ScanK &k, int p0) {
    PlaneEdges<CHUNK> e;
    e.np = k.n_planes - p0 < CHUNK ? k.n_planes - p0 : CHUNK;
#pragma unroll
    for (int c = 0; c < CHUNK; ++c) {
        const int p = p0 + c;
        if (k.layout == 1) {
            e.lo[c] = -INFINITY;
            e.hi[c] = (p < k.n_planes) ? k.edges[p] : -INFINITY;
        } else {
            e.lo[c] = (p == 0) ? -INFINITY : ((p < k.n_planes) ? k.edges[p - 1] : INFINITY);
            e.hi[c] = (p == k.n_bins - 1) ? INFINITY : ((p < k.n_planes) ? k.edges[p] : -INFINITY);
        }
    }
    return e;
}

__device__ __forceinline__ uint32_t ind(float v, float lo, float hi, bool in) {
    return (in && v >= lo && v < hi) ? 1u : 0u;
}

// One row of scan input: the luminance in table mode; in adjoint mode the deposit pair of
// the row and the luminance at the mirrored output pixels.  Tiles load row r+1 before they
// process row r, so the loads of the next row are in flight during the row's wave scans and
// stores.
template <int VEC, bool ADJ>
struct RowIn {
    float v[VEC];
    double2 d[ADJ ? VEC : 1];
};

// wide: table mode, the tile's columns are all in the image and its rows 16-byte aligned;
// adjoint mode, the tile's columns are all in the image.  A wide adjoint row is loaded
// entry-major (load i of lane l reads entry i*64 + l, so each load instruction covers 64
// consecutive entries) and put into the scan's lane-major order by adj_lane_major.
template <int VEC, bool ADJ, bool OUT_V = ADJ>
__device__ __forceinline__ void load_in(const ScanK &k, int y, int xl, bool wide,
                                        RowIn<VEC, ADJ> &r) {
    if constexpr (ADJ) {
        const TM_GLOBAL double2 *row = gptr(k.dsrc) + (int64_t)y * k.ld_d;
        const TM_GLOBAL float *vr = gptr(k.v) + (int64_t)(k.H - 1 - y) * k.ld_v;
        if (wide) {
            const int lane = lane_id();
            const int xe = xl - lane * VEC + lane;   // entry of load 0
#pragma unroll
            for (int i = 0; i < VEC; ++i) {
                r.d[i] = row[xe + i * kWave];
                if (OUT_V) r.v[i] = vr[k.W - 1 - (xe + i * kWave)];
            }
            return;
        }
#pragma unroll
        for (int i = 0; i < VEC; ++i) {
            const bool in = xl + i < k.W;
            r.d[i] = in ? make_double2(row[xl + i].x, row[xl + i].y) : make_double2(0.0, 0.0);
            if (OUT_V) r.v[i] = in ? vr[k.W - 1 - (xl + i)] : 0.f;
        }
    } else {
        load_row<VEC>(k, y, xl, wide, r.v);
    }
}

// LDS accesses of one wave happen in issue order; this keeps the compiler from moving the
// staging writes and reads of a row across each other.
__device__ __forceinline__ void wave_lds_sync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Entry-major row (element i of lane l is entry i*64 + l) to lane-major (element i of lane l
// is entry l*VEC + i), through the wave's LDS slice st of 64*VEC pairs.
template <int VEC, bool OUT_V>
__device__ __forceinline__ void adj_lane_major(RowIn<VEC, true> &r, double2 *st, int lane) {
#pragma unroll
    for (int i = 0; i < VEC; ++i) st[i * kWave + lane] = r.d[i];
    wave_lds_sync();
#pragma unroll
    for (int i = 0; i < VEC; ++i) r.d[i] = st[lane * VEC + i];
    wave_lds_sync();
    if constexpr (OUT_V) {
        float *sv = reinterpret_cast<float *>(st);
#pragma unroll
        for (int i = 0; i < VEC; ++i) sv[i * kWave + lane] = r.v[i];
        wave_lds_sync();
#pragma unroll
        for (int i = 0; i < VEC; ++i) r.v[i] = sv[lane * VEC + i];
        wave_lds_sync();
    }
}

// Per-pixel terms of the two scanned quantities: (v - mu1, v^2 - mu2) of the luminance in
// table mode; the two FP64 deposit planes in adjoint mode.  Zero outside the image.
template <int P, int VEC, bool ADJ>
__device__ __forceinline__ void sat_terms(const ScanK &k, int xl, const RowIn<VEC, ADJ> &in,
                                          float mu1, float mu2, typename Acc<P>::T (&q1)[VEC],
                                          typename Acc<P>::T (&q2)[VEC]) {
    using A = Acc<P>;
    if constexpr (ADJ) {
#pragma unroll
        for (int i = 0; i < VEC; ++i) {
            q1[i] = in.d[i].x;
            q2[i] = in.d[i].y;
        }
    } else {
        float x[VEC];
#pragma unroll
        for (int i = 0; i < VEC; ++i) x[i] = in.v[i];
        if (k.log_src) {   // the log plane's own expression
#pragma unroll
            for (int i = 0; i < VEC; ++i) x[i] = logf(fmaxf(x[i], FLT_MIN));
        }
#pragma unroll
        for (int i = 0; i < VEC; ++i) {
            const bool ok = xl + i < k.W;
            q1[i] = ok ? A::of_v(x[i], mu1) : A::zero();
            q2[i] = ok ? A::of_v2(x[i], mu2) : A::zero();
        }
    }
}

// Store of a table value (4, 8 or 16 bytes), non-temporal when nt.  Tables larger than the
// memory-side cache cannot stay there for the query anyway; streaming them out keeps them
// from displacing the lines the scans and the query still read.  Smaller tables are stored
// normally, so the query finds them in that cache.
template <typename T>
__device__ __forceinline__ void st_tab(TM_GLOBAL T *p, const T &v, bool nt) {
    if (!nt) {
        *p = v;
    } else if constexpr (sizeof(T) == 4) {
        uint32_t w;
        __builtin_memcpy(&w, &v, 4);
        __builtin_nontemporal_store(w, reinterpret_cast<TM_GLOBAL uint32_t *>(p));
    } else {
        using V = uint32_t __attribute__((ext_vector_type(sizeof(T) / 4)));
        V w;
        __builtin_memcpy(&w, &v, sizeof(T));
        __builtin_nontemporal_store(w, reinterpret_cast<TM_GLOBAL V *>(p));
    }
}

// Store a lane's VEC consecutive counts of one row: 16-byte stores inside the image (the
// row pitch is a multiple of 64 entries and xl a multiple of VEC, so they are aligned),
// element stores on the ragged last tile.
template <int VEC>
__device__ __forceinline__ void store_counts(TM_GLOBAL uint32_t *out, int xl, int W, bool full,
                                             const uint32_t (&c)[VEC], bool nt) {
    if (full && VEC % 4 == 0) {
#pragma unroll
        for (int i = 0; i < VEC; i += 4)
            st_tab(reinterpret_cast<TM_GLOBAL uint4 *>(out + xl + i),
                   make_uint4(c[i], c[i + 1], c[i + 2], c[i + 3]), nt);
    } else if (full) {
#pragma unroll
        for (int i = 0; i < VEC; ++i) st_tab(out + xl + i, c[i], nt);
    } else {
#pragma unroll
        for (int i = 0; i < VEC; ++i)
            if (xl + i < W) st_tab(out + xl + i, c[i], nt);
    }
}

// Store a lane's VEC consecutive integral-image entries of one full-width row.  A lane owns
// VEC consecutive columns, so a direct store instruction would write every VEC-th entry; the
// row is staged through the wave's LDS slice instead and written back so that each store
// instruction covers 64 consecutive entries.
template <int VEC, typename ET>
__device__ __forceinline__ void store_entries_full(TM_GLOBAL ET *out, int x0, int lane,
                                                   const ET (&e)[VEC], ET *st, bool nt) {
    if constexpr (VEC == 1) {
        st_tab(out + x0 + lane, e[0], nt);
    } else {
#pragma unroll
        for (int i = 0; i < VEC; ++i) st[lane * VEC + i] = e[i];
        wave_lds_sync();
#pragma unroll
        for (int i = 0; i < VEC; ++i) st_tab(out + x0 + i * kWave + lane, st[i * kWave + lane], nt);
        wave_lds_sync();
    }
}

// ================================================================ stage 1
// Rows are processed in groups of G; the loads of the next group are issued before the
// current group is processed, so a tile waits for memory once per group rather than once per
// row (the wave scans and stores of a row do not depend on the next rows).  The adjoint's rows
// are 64 bytes per lane, so it keeps two in flight.
template <int VEC, bool ADJ, bool THIRD>
__host__ __device__ constexpr int row_group() {
    return ADJ ? 2 : (VEC >= 8 || THIRD ? 4 : 8);
}

// Row totals of a group of eight rows without a wave reduction per row.  Each lane writes
// its in-lane sums of the eight rows to the wave's LDS slice (row-major, pitch 65); lane l
// then adds the eight entries [8p, 8p + 8) of row l & 7 (p = l >> 3), and the eight parts
// of a row (lanes differing in bits 3, 4 and 5) are added by a rotation of 8 inside each
// 16-lane row and gfx950's 16- and 32-lane swaps.  Every lane then holds the total of row
// l & 7; lanes 0..7 hold rows 0..7.  Per group and quantity this costs seven additions and
// three cross-lane steps, where a wave reduction per row cost eight times six steps.
constexpr int kRtRows = 8;
constexpr int kRtPitch = kWave + 1;

__device__ __forceinline__ void lane_swap16(uint32_t x, uint32_t &a, uint32_t &b) {
    const auto r = __builtin_amdgcn_permlane16_swap(x, x, false, false);
    a = r[0];
    b = r[1];
}
__device__ __forceinline__ void lane_swap32(uint32_t x, uint32_t &a, uint32_t &b) {
    const auto r = __builtin_amdgcn_permlane32_swap(x, x, false, false);
    a = r[0];
    b = r[1];
}

// {value of this lane, value of lane l ^ 16} (H16) or {.., lane l ^ 32}, in a lane-independent
// order, for each scan value type.
template <bool H16>
__device__ __forceinline__ void swap_pair(uint32_t x, uint32_t &a, uint32_t &b) {
    if constexpr (H16) lane_swap16(x, a, b); else lane_swap32(x, a, b);
}
template <bool H16>
__device__ __forceinline__ void swap_pair(float x, float &a, float &b) {
    uint32_t u, v;
    swap_pair<H16>(__float_as_uint(x), u, v);
    a = __uint_as_float(u);
    b = __uint_as_float(v);
}
template <bool H16>
__device__ __forceinline__ void swap_pair(double x, double &a, double &b) {
    const uint64_t bits = __double_as_longlong(x);
    uint32_t l0, l1, h0, h1;
    swap_pair<H16>((uint32_t)bits, l0, l1);
    swap_pair<H16>((uint32_t)(bits >> 32), h0, h1);
    a = __longlong_as_double((long long)(((uint64_t)h0 << 32) | l0));
    b = __longlong_as_double((long long)(((uint64_t)h1 << 32) | l1));
}
template <bool H16>
__device__ __forceinline__ void swap_pair(f2 x, f2 &a, f2 &b) {
    swap_pair<H16>(x.hi, a.hi, b.hi);
    swap_pair<H16>(x.lo, a.lo, b.lo);
}

template <class A, class T>
__device__ __forceinline__ T group_row_total(const T *row_part) {
    T s = row_part[0];
#pragma unroll
    for (int e = 1; e < kRtRows; ++e) s = A::add(s, row_part[e]);
    s = A::add(s, dpp<0x128>(s));   // row_ror:8, the partner l ^ 8 inside the 16-lane row
    T a, b;
    swap_pair<true>(s, a, b);
    s = A::add(a, b);
    swap_pair<false>(s, a, b);
    return A::add(a, b);
}

template <int G, int VEC, bool ADJ, bool OUT_V>
__device__ __forceinline__ void load_group(const ScanK &k, int y, int n, int xl, bool wide,
                                           RowIn<VEC, ADJ> (&b)[G]) {
#pragma unroll
    for (int u = 0; u < G; ++u)
        if (u < n) load_in<VEC, ADJ, OUT_V>(k, y + u, xl, wide, b[u]);
}

template <int P, int VEC, int CHUNK, bool SAT, bool HIST, bool ADJ>
__device__ __forceinline__ void stage1_tile(const ScanK &k, const int tile, int cb = 0,
                                            int ce = 1 << 30) {
    using A = Acc<P>;
    using T = typename A::T;
    constexpr int G = row_group<VEC, ADJ, false>();
    const int ty = tile / k.tiles_x, tx = tile % k.tiles_x;
    const int lane = lane_id();
    const int TW = kWave * VEC;
    const int x0 = tx * TW, y0 = ty * k.th;
    const int rows = min(k.th, k.H - y0);
    const int xl = x0 + lane * VEC;
    const int nchunks = HIST ? (k.n_planes + CHUNK - 1) / CHUNK : 0;
    const bool full = x0 + TW <= k.W;   // tile-uniform
    const bool wide = ADJ ? full : (k.vec_load && full);
    __shared__ double2 sh_adj[ADJ ? kWavesPerBlock * kWave * VEC : 1];
    constexpr bool kLdsRows = SAT && !ADJ && G == kRtRows;
    __shared__ T sh_rt[kLdsRows ? kWavesPerBlock * 2 * kRtRows * kRtPitch : 1];
    T *rt = sh_rt + (kLdsRows ? wave_id() * 2 * kRtRows * kRtPitch : 0);

    // a histogram-only work item covers the plane chunks [cb, ce)
    const int ch0 = SAT ? 0 : cb, ch1 = SAT ? (nchunks > 1 ? nchunks : 1) : min(ce, nchunks);
    for (int ch = ch0; ch < ch1; ++ch) {
        const bool do_sat = SAT && ch == 0;
        const bool do_h = HIST && ch < nchunks;
        const int p0 = ch * CHUNK;
        float mu1 = 0.f, mu2 = 0.f;
        if (do_sat && P == kC32x2) { mu1 = k.offsets[0]; mu2 = k.offsets[1]; }
        PlaneEdges<CHUNK> pe;
        if (do_h) pe = chunk_edges<CHUNK>(k, p0);

        T c1[VEC], c2[VEC], t1 = A::zero(), t2 = A::zero();
        uint32_t cc[CHUNK][VEC], tc[CHUNK];
#pragma unroll
        for (int i = 0; i < VEC; ++i) { c1[i] = A::zero(); c2[i] = A::zero(); }
#pragma unroll
        for (int c = 0; c < CHUNK; ++c) {
            tc[c] = 0u;
#pragma unroll
            for (int i = 0; i < VEC; ++i) cc[c][i] = 0u;
        }

        RowIn<VEC, ADJ> nb[G];
        load_group<G, VEC, ADJ, false>(k, y0, rows, xl, wide, nb);
        for (int r0 = 0; r0 < rows; r0 += G) {
            const int n = min(G, rows - r0);
            RowIn<VEC, ADJ> cb[G];
#pragma unroll
            for (int u = 0; u < G; ++u) cb[u] = nb[u];
            if (r0 + G < rows)
                load_group<G, VEC, ADJ, false>(k, y0 + r0 + G, rows - r0 - G, xl, wide, nb);
            // lane u keeps the totals of the group's row u; they are stored after the group
            T k1 = A::zero(), k2 = A::zero();
            uint32_t kh[CHUNK];
#pragma unroll
            for (int c = 0; c < CHUNK; ++c) kh[c] = 0u;
#pragma unroll
            for (int u = 0; u < G; ++u) {
                if (u >= n) break;
                if constexpr (ADJ)
                    if (wide) adj_lane_major<VEC, false>(cb[u], sh_adj + wave_id() * (kWave * VEC), lane);
                const float(&v)[VEC] = cb[u].v;
                if (do_sat) {
                    T s1 = A::zero(), s2 = A::zero();
                    T q1[VEC], q2[VEC];
                    sat_terms<P, VEC, ADJ>(k, xl, cb[u], mu1, mu2, q1, q2);
#pragma unroll
                    for (int i = 0; i < VEC; ++i) {
                        c1[i] = A::add(c1[i], q1[i]);
                        c2[i] = A::add(c2[i], q2[i]);
                        s1 = A::add(s1, q1[i]);
                        s2 = A::add(s2, q2[i]);
                    }
                    if constexpr (kLdsRows) {
                        rt[u * kRtPitch + lane] = s1;
                        rt[(kRtRows + u) * kRtPitch + lane] = s2;
                    } else {
                        if constexpr (P == kF64) {
                            wave_sum2(s1, s2, s1, s2);
                        } else {
                            s1 = wave_sum<A>(s1);
                            s2 = wave_sum<A>(s2);
                        }
                        t1 = A::add(t1, s1);
                        t2 = A::add(t2, s2);
                        if (lane == u) { k1 = s1; k2 = s2; }
                    }
                }
                if (do_h) {
                    uint32_t lc[CHUNK];
#pragma unroll
                    for (int c = 0; c < CHUNK; ++c) {
                        lc[c] = 0u;
#pragma unroll
                        for (int i = 0; i < VEC; ++i) {
                            const uint32_t b = ind(v[i], pe.lo[c], pe.hi[c], xl + i < k.W);
                            cc[c][i] += b;
                            lc[c] += b;
                        }
                    }
                    // row totals <= 64*VEC < 2^16: two planes per 32-bit lane value
#pragma unroll
                    for (int c = 0; c < CHUNK; c += 2) {
                        const uint32_t pk = lc[c] | (c + 1 < CHUNK ? lc[c + 1] << 16 : 0u);
                        const uint32_t s = wave_sum<AddU32>(pk);
                        const uint32_t a = s & 0xffffu, b = s >> 16;
                        tc[c] += a;
                        if (c + 1 < CHUNK) tc[c + 1] += b;
                        if (lane == u) {
                            kh[c] = a;
                            if (c + 1 < CHUNK) kh[c + 1] = b;
                        }
                    }
                }
            }
            if constexpr (kLdsRows) {
                if (do_sat) {   // rows u >= n of the slice are stale; their totals go unused
                    wave_lds_sync();
                    const int ru = lane & (kRtRows - 1), part = lane >> 3;
                    k1 = group_row_total<A>(rt + ru * kRtPitch + part * kRtRows);
                    k2 = group_row_total<A>(rt + (kRtRows + ru) * kRtPitch + part * kRtRows);
                    wave_lds_sync();
                }
            }
            if (lane < n) {
                const int64_t y = y0 + r0 + lane;
                if (do_sat) {
                    TM_GLOBAL T *rs = reinterpret_cast<TM_GLOBAL T *>(gptr(k.rs_sat));
                    rs[y * k.tiles_x + tx] = k1;
                    rs[((int64_t)k.H + y) * k.tiles_x + tx] = k2;
                }
                if (do_h) {
#pragma unroll
                    for (int c = 0; c < CHUNK; ++c)
                        if (c < pe.np) gptr(k.rs_h)[((int64_t)(p0 + c) * k.H + y) * k.tiles_x + tx] = kh[c];
                }
            }
        }
        if constexpr (kLdsRows) {
            if (do_sat) {   // tile totals from the column totals
                T a = c1[0], b = c2[0];
#pragma unroll
                for (int i = 1; i < VEC; ++i) {
                    a = A::add(a, c1[i]);
                    b = A::add(b, c2[i]);
                }
                t1 = wave_sum<A>(a);
                t2 = wave_sum<A>(b);
            }
        }
        if (do_sat) {
            T *cs = reinterpret_cast<T *>(k.cs_sat);
#pragma unroll
            for (int i = 0; i < VEC; ++i) {
                if (xl + i < k.W) {
                    cs[(int64_t)ty * k.W + xl + i] = c1[i];
                    cs[((int64_t)k.tiles_y + ty) * k.W + xl + i] = c2[i];
                }
            }
            if (lane == 0) {
                T *tt = reinterpret_cast<T *>(k.tt_sat);
                tt[(int64_t)ty * k.tiles_x + tx] = t1;
                tt[((int64_t)k.tiles_y + ty) * k.tiles_x + tx] = t2;
            }
        }
        if (do_h) {
#pragma unroll
            for (int c = 0; c < CHUNK; ++c) {
                if (c < pe.np) {
                    const int64_t q = p0 + c;
#pragma unroll
                    for (int i = 0; i < VEC; ++i)
                        if (xl + i < k.W) k.cs_h[(q * k.tiles_y + ty) * k.W + xl + i] = cc[c][i];
                    if (lane == 0) k.tt_h[(q * k.tiles_y + ty) * k.tiles_x + tx] = tc[c];
                }
            }
        }
    }
}

// ================================================================ stage 2
// Exclusive prefix of n values at stride `stride`, one thread, the loads issued 32 at a time
// so that the scan's add chain does not serialise the memory latency (stage 2 runs far fewer
// threads than the GPU holds, so its time is the number of load round trips in the longest
// chain).  Used for the chains along tx (tiles_x long); the long chains along ty are split
// across lanes below.  src and dst do not overlap.
template <class A, class T>
__device__ __forceinline__ void excl_scan(const T *__restrict__ src, T *__restrict__ dst, int n,
                                          int64_t stride) {
    constexpr int kB = 32;
    T run = A::zero();
    int t = 0;
    for (; t + kB <= n; t += kB) {
        T a[kB];
#pragma unroll
        for (int u = 0; u < kB; ++u) a[u] = src[(int64_t)(t + u) * stride];
#pragma unroll
        for (int u = 0; u < kB; ++u) {
            dst[(int64_t)(t + u) * stride] = run;
            run = A::add(run, a[u]);
        }
    }
    for (; t + 8 <= n; t += 8) {
        T a[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) a[u] = src[(int64_t)(t + u) * stride];
#pragma unroll
        for (int u = 0; u < 8; ++u) {
            dst[(int64_t)(t + u) * stride] = run;
            run = A::add(run, a[u]);
        }
    }
    for (; t < n; ++t) {
        const T a = src[(int64_t)t * stride];
        dst[(int64_t)t * stride] = run;
        run = A::add(run, a);
    }
}

// The column chains (one per quantity and image column, tiles_y long) are the long ones:
// each is split into kSegs segments on lanes c, c + 8, ..., c + 56 of one wave (8 chains per
// wave).  A lane loads its segment (up to kSegMax values held in registers) and sums it, the
// segment totals get an exclusive prefix across the chain's lanes (three shuffle steps), and
// the lane scans its segment from that carry: one round trip of loads instead of tiles_y / 32.
// Longer segments are summed and then rescanned from memory.
constexpr int kSegs = 8;
constexpr int kChainsPerWave = kWave / kSegs;
constexpr int kSegMax = 48;

__device__ __forceinline__ float shfl_up_v(float v, int d) { return __shfl_up(v, d); }
__device__ __forceinline__ double shfl_up_v(double v, int d) { return __shfl_up(v, d); }
__device__ __forceinline__ uint32_t shfl_up_v(uint32_t v, int d) {
    return (uint32_t)__shfl_up((int)v, d);
}
__device__ __forceinline__ f2 shfl_up_v(f2 v, int d) {
    return f2{shfl_up_v(v.hi, d), shfl_up_v(v.lo, d)};
}

// Sum of src[t * stride] for t in [b, e), loads issued 32 at a time, added in order.
template <class A, class T>
__device__ __forceinline__ T range_sum(const T *__restrict__ src, int b, int e, int64_t stride) {
    constexpr int kB = 32;
    T run = A::zero();
    int t = b;
    for (; t + kB <= e; t += kB) {
        T a[kB];
#pragma unroll
        for (int u = 0; u < kB; ++u) a[u] = src[(int64_t)(t + u) * stride];
#pragma unroll
        for (int u = 0; u < kB; ++u) run = A::add(run, a[u]);
    }
    for (; t < e; ++t) run = A::add(run, src[(int64_t)t * stride]);
    return run;
}

// Exclusive prefix of src over [b, e) starting from `run`, written to dst.
template <class A, class T>
__device__ __forceinline__ void range_scan(const T *__restrict__ src, T *__restrict__ dst, int b,
                                           int e, int64_t stride, T run) {
    constexpr int kB = 32;
    int t = b;
    for (; t + kB <= e; t += kB) {
        T a[kB];
#pragma unroll
        for (int u = 0; u < kB; ++u) a[u] = src[(int64_t)(t + u) * stride];
#pragma unroll
        for (int u = 0; u < kB; ++u) {
            dst[(int64_t)(t + u) * stride] = run;
            run = A::add(run, a[u]);
        }
    }
    for (; t < e; ++t) {
        const T a = src[(int64_t)t * stride];
        dst[(int64_t)t * stride] = run;
        run = A::add(run, a);
    }
}

// One lane's part of a segmented column chain of n values (seg = lane / 16).  Every lane of
// the wave calls this (inactive lanes with active = false) so that the shuffles see all.
template <class A, class T>
__device__ __forceinline__ T seg_carry(T total, int seg) {
    T inc = total;
#pragma unroll
    for (int d = 1; d < kSegs; d *= 2) {
        const T up = shfl_up_v(inc, d * kChainsPerWave);
        if (seg >= d) inc = A::add(up, inc);
    }
    const T carry = shfl_up_v(inc, kChainsPerWave);
    return seg == 0 ? A::zero() : carry;
}

template <class A, class T>
__device__ __forceinline__ void seg_excl_scan(const T *__restrict__ src, T *__restrict__ dst,
                                              int n, int64_t stride, int seg, bool active) {
    const int len = (n + kSegs - 1) / kSegs;   // chain-uniform
    const int b = min(n, seg * len), e = min(n, b + len);
    if (len <= kSegMax) {
        T a[kSegMax];
        T tot = A::zero();
#pragma unroll
        for (int u = 0; u < kSegMax; ++u)
            a[u] = (active && b + u < e) ? src[(int64_t)(b + u) * stride] : A::zero();
#pragma unroll
        for (int u = 0; u < kSegMax; ++u) tot = A::add(tot, a[u]);
        T run = seg_carry<A>(tot, seg);
        if (active) {
#pragma unroll
            for (int u = 0; u < kSegMax; ++u) {
                if (b + u < e) dst[(int64_t)(b + u) * stride] = run;
                run = A::add(run, a[u]);
            }
        }
    } else {
        const T tot = active ? range_sum<A>(src, b, e, stride) : A::zero();
        const T carry = seg_carry<A>(tot, seg);
        if (active) range_scan<A>(src, dst, b, e, stride, carry);
    }
}

__host__ __device__ constexpr int64_t round64(int64_t a) { return (a + 63) / 64 * 64; }

// Stage-2 work items of one image: [0, n1) scan RS along tx for one (quantity, row), padded
// to whole waves; then waves of 16 column chains x 4 segments scan CS along ty; then items
// scan TT along tx for one (quantity, ty).  The total is a whole number of waves, so in a
// batch every image's items start on a wave boundary.
struct Stage2Split {
    int64_t n1, n1p, groups, n2, n3, total;
};
__host__ __device__ inline Stage2Split stage2_split(const ScanK &k, bool sat) {
    Stage2Split q;
    const int64_t nq = (sat ? 2 : 0) + k.n_planes;
    q.n1 = nq * k.H;
    q.n1p = round64(q.n1);
    q.groups = (k.W + kChainsPerWave - 1) / kChainsPerWave;
    q.n2 = nq * q.groups * kWave;
    q.n3 = nq * k.tiles_y;
    q.total = round64(q.n1p + q.n2 + q.n3);
    return q;
}

template <int P, bool SAT>
__device__ __forceinline__ void stage2_item(const ScanK &k, int64_t idx) {
    using A = Acc<P>;
    using T = typename A::T;
    const int nq_sat = SAT ? 2 : 0;
    const Stage2Split sp = stage2_split(k, SAT);
    const int64_t n1 = sp.n1;
    if (idx < n1) {
        // XC[q][y][tx] = sum_{tx' < tx} RS[q][y][tx']
        const int q = (int)(idx / k.H);
        const int64_t y = idx % k.H;
        if (q < nq_sat) {
            const int64_t o = ((int64_t)q * k.H + y) * k.tiles_x;
            excl_scan<A>(reinterpret_cast<const T *>(k.rs_sat) + o,
                         reinterpret_cast<T *>(k.xc_sat) + o, k.tiles_x, 1);
        } else {
            const int64_t o = ((int64_t)(q - nq_sat) * k.H + y) * k.tiles_x;
            excl_scan<AddU32>(k.rs_h + o, k.xc_h + o, k.tiles_x, 1);
        }
    } else if (idx < sp.n1p) {
        return;   // padding to a whole wave
    } else if (idx < sp.n1p + sp.n2) {
        // CSE[q][ty][x] = sum_{ty' < ty} CS[q][ty'][x], one wave per (q, 16 columns)
        const int64_t id = idx - sp.n1p;
        const int lane = (int)(id & (kWave - 1));
        const int64_t wv = id >> 6;
        const int q = (int)(wv / sp.groups);
        const int64_t x = (wv % sp.groups) * kChainsPerWave + (lane & (kChainsPerWave - 1));
        const int seg = lane / kChainsPerWave;
        const bool active = x < k.W;
        const int64_t xa = active ? x : 0;
        if (q < nq_sat) {   // wave-uniform
            const int64_t o = (int64_t)q * k.tiles_y * k.W + xa;
            seg_excl_scan<A>(reinterpret_cast<const T *>(k.cs_sat) + o,
                             reinterpret_cast<T *>(k.cse_sat) + o, k.tiles_y, k.W, seg, active);
        } else {
            const int64_t o = (int64_t)(q - nq_sat) * k.tiles_y * k.W + xa;
            seg_excl_scan<AddU32>(k.cs_h + o, k.cse_h + o, k.tiles_y, k.W, seg, active);
        }
    } else {
        // TTE[q][ty][tx] = sum_{tx' < tx} TT[q][ty][tx']
        const int64_t id = idx - sp.n1p - sp.n2;
        if (id >= sp.n3) return;
        const int q = (int)(id / k.tiles_y);
        const int64_t ty = id % k.tiles_y;
        if (q < nq_sat) {
            const int64_t o = ((int64_t)q * k.tiles_y + ty) * k.tiles_x;
            excl_scan<A>(reinterpret_cast<const T *>(k.tt_sat) + o,
                         reinterpret_cast<T *>(k.tte_sat) + o, k.tiles_x, 1);
        } else {
            const int64_t o = ((int64_t)(q - nq_sat) * k.tiles_y + ty) * k.tiles_x;
            excl_scan<AddU32>(k.tt_h + o, k.tte_h + o, k.tiles_x, 1);
        }
    }
}

// ================================================================ stage 3
// Adjoint output of one pixel from its suffix sums s1, s2: dv = s1 + 2 v s2.  In the
// log-domain variant v is the image i, the moments were those of l = ln max(i, FLT_MIN) (the
// same expression as the log pass), so the gradient w.r.t. l is s1 + 2 l s2 and the chain
// rule gives (s1 + 2 l s2) / i, or 0 where the floor constant is taken.
__device__ __forceinline__ float adj_grad(const ScanK &k, float v, double s1, double s2) {
    if (!k.log_chain) return (float)(s1 + 2.0 * (double)v * s2);
    const float l = logf(fmaxf(v, FLT_MIN));
    const float gl = (float)(s1 + 2.0 * (double)l * s2);
    return v > FLT_MIN ? gl / v : 0.f;
}

// Column carries at the top of the tile for the lane's VEC columns, for every quantity of
// the pass:  sum_{ty'<ty} TTE[ty'][tx] + inclusive prefix over the tile of CSE[ty][.].
// All loads are issued before the first sum (one memory round trip per 256 tile rows above,
// not one per quantity and 64 rows); each lane sums the rows t = lane (mod 64) in ascending
// order, then the wave adds the lanes' sums.
// col = (sum over the wave of above_lane) + (sum of e over the lanes to the left) +
// (inclusive prefix of the lane's own e).
template <class O, int VEC, class T>
__device__ __forceinline__ void carry_finish(T above_lane, const T (&e)[VEC], T (&col)[VEC]) {
    const T above = wave_sum<O>(above_lane);
    T p[VEC];
#pragma unroll
    for (int i = 0; i < VEC; ++i) p[i] = i ? O::add(p[i - 1], e[i]) : e[i];
    const T ex = wave_shr1(wave_inclusive<O>(p[VEC - 1]));
    const T base = O::add(above, ex);
#pragma unroll
    for (int i = 0; i < VEC; ++i) col[i] = O::add(base, p[i]);
}

template <class A, int VEC, int CHUNK, class T>
__device__ __forceinline__ void tile_carries(const ScanK &k, bool do_sat, bool do_h, int p0,
                                             int np, int ty, int tx, int xl, T (&c1)[VEC],
                                             T (&c2)[VEC], uint32_t (&cc)[CHUNK][VEC]) {
    const int lane = lane_id();
    const int64_t ntt = (int64_t)k.tiles_y * k.tiles_x;
    const T *tte = reinterpret_cast<const T *>(k.tte_sat);
    const T *cse = reinterpret_cast<const T *>(k.cse_sat);
    // the tile row's column sums above it
    T e1[VEC], e2[VEC];
    uint32_t eh[CHUNK][VEC];
#pragma unroll
    for (int i = 0; i < VEC; ++i) {
        const bool in = xl + i < k.W;
        e1[i] = A::zero();
        e2[i] = A::zero();
        if (do_sat && in) {
            const T a = cse[(int64_t)ty * k.W + xl + i];
            const T b = cse[((int64_t)k.tiles_y + ty) * k.W + xl + i];
            e1[i] = a;
            e2[i] = b;
        }
#pragma unroll
        for (int c = 0; c < CHUNK; ++c)
            eh[c][i] = (do_h && in && c < np)
                           ? k.cse_h[((int64_t)(p0 + c) * k.tiles_y + ty) * k.W + xl + i]
                           : 0u;
    }
    // the tiles above, in this tile column
    T a1 = A::zero(), a2 = A::zero();
    uint32_t ah[CHUNK];
#pragma unroll
    for (int c = 0; c < CHUNK; ++c) ah[c] = 0u;
    for (int t0 = 0; t0 < ty; t0 += 4 * kWave) {
        T l1[4], l2[4];
        uint32_t lh[4][CHUNK];
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            const int t = t0 + u * kWave + lane;
            const int64_t o = (int64_t)t * k.tiles_x + tx;
            l1[u] = A::zero();
            l2[u] = A::zero();
            if (do_sat && t < ty) {
                const T a = tte[o];
                const T b = tte[ntt + o];
                l1[u] = a;
                l2[u] = b;
            }
#pragma unroll
            for (int c = 0; c < CHUNK; ++c)
                lh[u][c] = (do_h && t < ty && c < np) ? k.tte_h[(int64_t)(p0 + c) * ntt + o] : 0u;
        }
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            if (t0 + u * kWave + lane < ty) {
                a1 = A::add(a1, l1[u]);
                a2 = A::add(a2, l2[u]);
#pragma unroll
                for (int c = 0; c < CHUNK; ++c) ah[c] += lh[u][c];
            }
        }
    }
    if (do_sat) {
        carry_finish<A, VEC>(a1, e1, c1);
        carry_finish<A, VEC>(a2, e2, c2);
    }
    if (do_h) {
#pragma unroll
        for (int c = 0; c < CHUNK; ++c) carry_finish<AddU32, VEC>(ah[c], eh[c], cc[c]);
    }
}

template <int P, int VEC, int CHUNK, bool SAT, bool HIST, bool ADJ>
__device__ __forceinline__ void stage3_tile(const ScanK &k, const int tile, int cb = 0,
                                            int ce = 1 << 30) {
    using A = Acc<P>;
    using T = typename A::T;
    using E = Entry<P>;
    using ET = typename E::T;
    const int ty = tile / k.tiles_x, tx = tile % k.tiles_x;
    const int lane = lane_id();
    const int TW = kWave * VEC;
    const int x0 = tx * TW, y0 = ty * k.th;
    const int rows = min(k.th, k.H - y0);
    const int xl = x0 + lane * VEC;
    const int nchunks = HIST ? (k.n_planes + CHUNK - 1) / CHUNK : 0;
    const bool last_tx = tx == k.tiles_x - 1;
    const bool full = x0 + TW <= k.W;   // tile-uniform: every lane's columns are in the image
    // each wave's staging slice for the entry stores of one row
    __shared__ ET sh_stage[(ADJ || !SAT) ? 1 : kWavesPerBlock * kWave * VEC];
    __shared__ double2 sh_adj[ADJ ? kWavesPerBlock * kWave * VEC : 1];

    // a histogram-only work item covers the plane chunks [cb, ce)
    const int ch0 = SAT ? 0 : cb, ch1 = SAT ? (nchunks > 1 ? nchunks : 1) : min(ce, nchunks);
    for (int ch = ch0; ch < ch1; ++ch) {
        const bool do_sat = SAT && ch == 0;
        const bool do_h = HIST && ch < nchunks;
        const int p0 = ch * CHUNK;
        float mu1 = 0.f, mu2 = 0.f;
        if (do_sat && P == kC32x2) { mu1 = k.offsets[0]; mu2 = k.offsets[1]; }
        PlaneEdges<CHUNK> pe;
        if (do_h) pe = chunk_edges<CHUNK>(k, p0);

        // the tile's first rows (and their row carries) are requested before the column
        // carries, so both are in flight together; lane u holds the row carries of the
        // group's row u
        constexpr int G = row_group<VEC, ADJ, true>();
        RowIn<VEC, ADJ> nb[G];
        T nx1 = A::zero(), nx2 = A::zero();
        uint32_t nxh[CHUNK];
        auto load_rows = [&](int r0) {
            const int n = rows - r0;
            load_group<G, VEC, ADJ, ADJ>(k, y0 + r0, n, xl, ADJ ? full : (full && k.vec_load), nb);
            const int64_t y = y0 + r0 + lane;
            if (do_sat) {
                const TM_GLOBAL T *xc = reinterpret_cast<const TM_GLOBAL T *>(gptr(k.xc_sat));
                nx1 = A::zero();
                nx2 = A::zero();
                if (lane < n) {
                    const T a = xc[y * k.tiles_x + tx];
                    const T b = xc[((int64_t)k.H + y) * k.tiles_x + tx];
                    nx1 = a;
                    nx2 = b;
                }
            }
            if (do_h) {
#pragma unroll
                for (int c = 0; c < CHUNK; ++c)
                    nxh[c] = (lane < n && c < pe.np)
                                 ? gptr(k.xc_h)[((int64_t)(p0 + c) * k.H + y) * k.tiles_x + tx]
                                 : 0u;
            }
        };
        if (rows > 0) load_rows(0);
        T c1[VEC], c2[VEC];
        uint32_t cc[CHUNK][VEC];
        tile_carries<A, VEC, CHUNK>(k, do_sat, do_h, p0, do_h ? pe.np : 0, ty, tx, xl, c1, c2, cc);

        for (int r0 = 0; r0 < rows; r0 += G) {
            const int n = min(G, rows - r0);
            RowIn<VEC, ADJ> cb[G];
#pragma unroll
            for (int u = 0; u < G; ++u) cb[u] = nb[u];
            const T gx1 = nx1, gx2 = nx2;
            uint32_t gxh[CHUNK];
#pragma unroll
            for (int c = 0; c < CHUNK; ++c) gxh[c] = nxh[c];
            if (r0 + G < rows) load_rows(r0 + G);
#pragma unroll
            for (int u = 0; u < G; ++u) {
                if (u >= n) break;
                const int y = y0 + r0 + u;
                if constexpr (ADJ)
                    if (full) adj_lane_major<VEC, true>(cb[u], sh_adj + wave_id() * (kWave * VEC), lane);
                const RowIn<VEC, ADJ> &cur = cb[u];
                const float(&v)[VEC] = cur.v;
                if (do_sat) {
                    const T xc1 = readlane(gx1, u);
                    const T xc2 = readlane(gx2, u);
                    T p1[VEC], p2[VEC];
                    sat_terms<P, VEC, ADJ>(k, xl, cur, mu1, mu2, p1, p2);
#pragma unroll
                    for (int i = 1; i < VEC; ++i) {
                        p1[i] = A::add(p1[i - 1], p1[i]);
                        p2[i] = A::add(p2[i - 1], p2[i]);
                    }
                    const T b1 = A::add(xc1, wave_shr1(wave_inclusive<A>(p1[VEC - 1])));
                    const T b2 = A::add(xc2, wave_shr1(wave_inclusive<A>(p2[VEC - 1])));
#pragma unroll
                    for (int i = 0; i < VEC; ++i) {
                        c1[i] = A::add(c1[i], A::add(b1, p1[i]));
                        c2[i] = A::add(c2[i], A::add(b2, p2[i]));
                    }
                    if constexpr (ADJ) {
                        // virtual (x', y) is pixel (W-1-x', H-1-y): dv = s1 + 2 v s2
                        const int yo = k.H - 1 - y;
                        TM_GLOBAL float *gr = gptr(k.gv) + (int64_t)yo * k.ld_gv;
                        if (full) {
                            // staged so that each store covers 64 consecutive outputs
                            float *sv = reinterpret_cast<float *>(sh_adj + wave_id() * (kWave * VEC));
#pragma unroll
                            for (int i = 0; i < VEC; ++i)
                                sv[lane * VEC + i] = adj_grad(k, cur.v[i], c1[i], c2[i]);
                            wave_lds_sync();
#pragma unroll
                            for (int i = 0; i < VEC; ++i)
                                gr[k.W - 1 - (x0 + i * kWave + lane)] = sv[i * kWave + lane];
                            wave_lds_sync();
                        } else {
#pragma unroll
                            for (int i = 0; i < VEC; ++i) {
                                const int xo = k.W - 1 - (xl + i);
                                if (xo >= 0) gr[xo] = adj_grad(k, cur.v[i], c1[i], c2[i]);
                            }
                        }
                    } else {
                        TM_GLOBAL ET *out = reinterpret_cast<TM_GLOBAL ET *>(gptr(k.sat)) + (int64_t)y * k.ld_sat;
                        if (full) {
                            ET e[VEC];
#pragma unroll
                            for (int i = 0; i < VEC; ++i) e[i] = E::make(c1[i], c2[i]);
                            store_entries_full<VEC, ET>(out, x0, lane, e,
                                                        sh_stage + wave_id() * (kWave * VEC),
                                                        k.stream_out != 0);
                        } else {
#pragma unroll
                            for (int i = 0; i < VEC; ++i)
                                if (xl + i < k.W) st_tab(out + xl + i, E::make(c1[i], c2[i]), k.stream_out != 0);
                        }
                    }
                }
                if (do_h) {
#pragma unroll
                    for (int c = 0; c < CHUNK; c += 2) {
                        uint32_t pa[VEC], pb[VEC];
#pragma unroll
                        for (int i = 0; i < VEC; ++i) {
                            const bool in = xl + i < k.W;
                            const uint32_t a = ind(v[i], pe.lo[c], pe.hi[c], in);
                            const uint32_t b = (c + 1 < CHUNK) ? ind(v[i], pe.lo[c + 1], pe.hi[c + 1], in) : 0u;
                            pa[i] = i ? pa[i - 1] + a : a;
                            pb[i] = i ? pb[i - 1] + b : b;
                        }
                        // lane-exclusive prefix of both planes packed in 16-bit halves (<= 64*VEC)
                        const uint32_t pk = pa[VEC - 1] | (pb[VEC - 1] << 16);
                        const uint32_t ex = wave_shr1(wave_inclusive<AddU32>(pk));
                        const uint32_t exa = ex & 0xffffu, exb = ex >> 16;
                        if (c < pe.np) {
                            const uint32_t xc = readlane(gxh[c], u);
                            TM_GLOBAL uint32_t *out = gptr(k.hist) + (int64_t)(p0 + c) * k.plane_stride + (int64_t)y * k.ld_hist;
#pragma unroll
                            for (int i = 0; i < VEC; ++i) cc[c][i] += xc + exa + pa[i];
                            store_counts<VEC>(out, xl, k.W, full, cc[c], k.stream_out != 0);
                        }
                        if (c + 1 < CHUNK && c + 1 < pe.np) {
                            const uint32_t xc = readlane(gxh[c + 1], u);
                            TM_GLOBAL uint32_t *out = gptr(k.hist) + (int64_t)(p0 + c + 1) * k.plane_stride + (int64_t)y * k.ld_hist;
#pragma unroll
                            for (int i = 0; i < VEC; ++i) cc[c + 1][i] += xc + exb + pb[i];
                            store_counts<VEC>(out, xl, k.W, full, cc[c + 1], k.stream_out != 0);
                        }
                    }
                }
            }
        }

        // zero border: row -1 over this tile's columns (plus x = -1 on the first tile) and
        // the padding columns [W, ld) on the last tile column (rows y0..y0+rows-1, and
        // row -1 when ty == 0).
        if (do_sat && !ADJ) {
            ET *t0 = reinterpret_cast<ET *>(k.sat);
            if (ty == 0) {
                for (int x = x0 - (tx == 0 ? 1 : 0) + lane; x < x0 + TW && x < k.W; x += kWave)
                    t0[-k.ld_sat + x] = E::zero();
            }
            if (last_tx) {
                for (int r = (ty == 0 ? -1 : 0); r < rows; ++r)
                    for (int x = k.W + lane; x < k.ld_sat; x += kWave)
                        t0[(int64_t)(y0 + r) * k.ld_sat + x] = E::zero();
            }
        }
        if (do_h) {
            for (int c = 0; c < pe.np; ++c) {
                uint32_t *t0 = k.hist + (int64_t)(p0 + c) * k.plane_stride;
                if (ty == 0) {
                    for (int x = x0 - (tx == 0 ? 1 : 0) + lane; x < x0 + TW && x < k.W; x += kWave)
                        t0[-k.ld_hist + x] = 0u;
                }
                if (last_tx) {
                    for (int r = (ty == 0 ? -1 : 0); r < rows; ++r)
                        for (int x = k.W + lane; x < k.ld_hist; x += kWave)
                            t0[(int64_t)(y0 + r) * k.ld_hist + x] = 0u;
                }
            }
        }
    }
}

// ---------------------------------------------------------------- single-image kernels
// Work items of a tile: its integral image (one item, when built) and its histogram planes
// (k.hist_items items, each k.hist_chunks plane chunks), on neighbouring waves, so that every
// wave holds the state of one kind of table only and the tile's luminance rows are read from
// the cache after the first.
template <bool SAT, bool HIST>
__host__ __device__ __forceinline__ int items_per_tile(const ScanK &k) {
    return (SAT ? 1 : 0) + (HIST ? k.hist_items : 0);
}

// HSRC: histogram items bin k.vh (single-image launches); the batch bins each image's own
// luminance (vh == v) and reads its parameters from global memory, where a modified copy
// would cost registers.
template <int P, int VEC, int CHUNK, bool SAT, bool HIST, bool ADJ, bool THIRD, bool HSRC = true>
__device__ __forceinline__ void tile_item(const ScanK &k, int item) {
    const int ipt = items_per_tile<SAT, HIST>(k);
    const int tile = item / ipt, r = item - tile * ipt;
    if constexpr (SAT) {
        if (r == 0) {
            if (THIRD) stage3_tile<P, VEC, CHUNK, true, false, ADJ>(k, tile);
            else stage1_tile<P, VEC, CHUNK, true, false, ADJ>(k, tile);
            return;
        }
    }
    if constexpr (HIST) {
        const int h = r - (SAT ? 1 : 0);
        const int cb = h * k.hist_chunks, ce = cb + k.hist_chunks;
        if constexpr (HSRC) {
            // histogram items bin their own source plane (the same one unless given another)
            ScanK kh = k;
            kh.v = k.vh;
            kh.ld_v = k.ld_vh;
            kh.vec_load = k.vec_load_h;
            if (THIRD) stage3_tile<P, VEC, CHUNK, false, true, ADJ>(kh, tile, cb, ce);
            else stage1_tile<P, VEC, CHUNK, false, true, ADJ>(kh, tile, cb, ce);
        } else {
            if (THIRD) stage3_tile<P, VEC, CHUNK, false, true, ADJ>(k, tile, cb, ce);
            else stage1_tile<P, VEC, CHUNK, false, true, ADJ>(k, tile, cb, ce);
        }
    }
}

template <int P, int VEC, int CHUNK, bool SAT, bool HIST, bool ADJ>
__global__ void __launch_bounds__(kBlock) scan_stage1(ScanK k) {
    const int item = blockIdx.x * kWavesPerBlock + wave_id();
    if (item >= k.tiles_x * k.tiles_y * items_per_tile<SAT, HIST>(k)) return;
    tile_item<P, VEC, CHUNK, SAT, HIST, ADJ, false>(k, item);
}

template <int P, bool SAT>
__global__ void __launch_bounds__(kBlock) scan_stage2(ScanK k, int64_t items) {
    const int64_t idx = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (idx < items) stage2_item<P, SAT>(k, idx);
}

template <int P, int VEC, int CHUNK, bool SAT, bool HIST, bool ADJ>
__global__ void __launch_bounds__(kBlock) scan_stage3(ScanK k) {
    const int item = blockIdx.x * kWavesPerBlock + wave_id();
    if (item >= k.tiles_x * k.tiles_y * items_per_tile<SAT, HIST>(k)) return;
    tile_item<P, VEC, CHUNK, SAT, HIST, ADJ, true>(k, item);
}

// ---------------------------------------------------------------- batched kernels
// A grid walks one flattened list of work items spanning images [0, count) of ks; prefix
// points at the first image's entry of the batch-wide prefix sums, so the walk covers
// [prefix[0], prefix[count]).  The batch launches one item per wave (one wave per item is
// handed out in order by the hardware); the loop also serves smaller grids.
template <int P, int VEC, int CHUNK, bool SAT, bool HIST, bool THIRD>
__global__ void __launch_bounds__(kBlock) scan_tiles_batch(const ScanK *__restrict__ ks,
                                                           const int64_t *__restrict__ prefix,
                                                           int count) {
    const int64_t total = prefix[count];
    const int64_t step = (int64_t)gridDim.x * kWavesPerBlock;
    int64_t g = prefix[0] + (int64_t)blockIdx.x * kWavesPerBlock + wave_id();
    // g only grows, so the image index only advances (no search per tile)
    int i = g < total ? __builtin_amdgcn_readfirstlane(find_image(prefix, count, g)) : 0;
    for (; g < total; g += step) {
        while (g >= prefix[i + 1]) ++i;
        tile_item<P, VEC, CHUNK, SAT, HIST, false, THIRD, false>(ks[i], (int)(g - prefix[i]));
    }
}

template <int P, bool SAT>
__global__ void __launch_bounds__(kBlock) scan_stage2_batch(const ScanK *__restrict__ ks,
                                                           const int64_t *__restrict__ prefix,
                                                            int count) {
    const int64_t total = prefix[count];
    const int64_t step = (int64_t)gridDim.x * kBlock;
    for (int64_t g = prefix[0] + (int64_t)blockIdx.x * kBlock + threadIdx.x; g < total;
         g += step) {
        const int i = find_image(prefix, count, g);
        stage2_item<P, SAT>(ks[i], g - prefix[i]);
    }
}

template <int P, int VEC, int CHUNK, bool SAT, bool HIST, bool ADJ = false>
hipError_t run3(const ScanK &k, hipStream_t s) {
    const int items = k.tiles_x * k.tiles_y * items_per_tile<SAT, HIST>(k);
    const int grid = (items + kWavesPerBlock - 1) / kWavesPerBlock;
    hipLaunchKernelGGL((scan_stage1<P, VEC, CHUNK, SAT, HIST, ADJ>), dim3(grid), dim3(kBlock), 0, s, k);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    const int64_t items2 = scan_stage2_items(k, SAT);
    hipLaunchKernelGGL((scan_stage2<P, SAT>), dim3((unsigned)((items2 + kBlock - 1) / kBlock)),
                       dim3(kBlock), 0, s, k, items2);
    e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL((scan_stage3<P, VEC, CHUNK, SAT, HIST, ADJ>), dim3(grid), dim3(kBlock), 0, s, k);
    return hipGetLastError();
}

template <int P, int VEC, int CHUNK>
hipError_t dispatch_sh(const ScanK &k, bool sat, bool hist, hipStream_t s) {
    if (sat && hist) return run3<P, VEC, CHUNK, true, true>(k, s);
    if (sat) return run3<P, VEC, CHUNK, true, false>(k, s);
    return run3<P, VEC, CHUNK, false, true>(k, s);
}

template <int P, int VEC>
hipError_t dispatch_chunk(const ScanK &k, int chunk, bool sat, bool hist, hipStream_t s) {
    switch (chunk) {
        case 2: return dispatch_sh<P, VEC, 2>(k, sat, hist, s);
        case 4: return dispatch_sh<P, VEC, 4>(k, sat, hist, s);
        default: return dispatch_sh<P, VEC, 8>(k, sat, hist, s);
    }
}

template <int P>
hipError_t dispatch_vec(const ScanK &k, int vec, int chunk, bool sat, bool hist, hipStream_t s) {
    switch (vec) {
        case 2: return dispatch_chunk<P, 2>(k, chunk, sat, hist, s);
        case 4: return dispatch_chunk<P, 4>(k, chunk, sat, hist, s);
        default: return dispatch_chunk<P, 8>(k, chunk, sat, hist, s);
    }
}

template <int P, int VEC, int CHUNK>
hipError_t batch3(const BatchScan &b, hipStream_t s) {
    hipLaunchKernelGGL((scan_tiles_batch<P, VEC, CHUNK, true, true, false>), dim3(b.grid_tiles),
                       dim3(kBlock), 0, s, b.ks, b.tile_prefix, b.count);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL((scan_stage2_batch<P, true>), dim3(b.grid_items), dim3(kBlock), 0, s, b.ks,
                       b.item_prefix, b.count);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    hipLaunchKernelGGL((scan_tiles_batch<P, VEC, CHUNK, true, true, true>), dim3(b.grid_tiles),
                       dim3(kBlock), 0, s, b.ks, b.tile_prefix, b.count);
    return hipGetLastError();
}

template <int P, int VEC>
hipError_t batch_chunk(const BatchScan &b, hipStream_t s) {
    switch (b.chunk) {
        case 2: return batch3<P, VEC, 2>(b, s);
        case 4: return batch3<P, VEC, 4>(b, s);
        default: return batch3<P, VEC, 8>(b, s);
    }
}

template <int P>
hipError_t batch_vec(const BatchScan &b, hipStream_t s) {
    switch (b.vec) {
        case 2: return batch_chunk<P, 2>(b, s);
        case 4: return batch_chunk<P, 4>(b, s);
        default: return batch_chunk<P, 8>(b, s);
    }
}

size_t round_up(size_t a, size_t b) { return (a + b - 1) / b * b; }

}  // namespace

hipError_t launch_tables_batch(const BatchScan &b, hipStream_t s) {
    switch (b.prec) {
        case kF32: return batch_vec<kF32>(b, s);
        case kC32x2: return batch_vec<kC32x2>(b, s);
        default: return batch_vec<kF64>(b, s);
    }
}

// Default tiling, from a sweep of every candidate over shapes 360..4000 per side: rows per
// tile grow with the image height (taller tiles shorten the column-carry chains and amortise
// each tile's carries), halved while the image would have fewer than 512 tiles.  32-row
// tiles were up to 6 % faster from 2600 rows but raised the 12 MP output error by a third,
// so tiles stop at 16 rows.  From 33 bins the column aggregates of the histogram planes
// dominate the scan's traffic (W x H / th x planes x 4 bytes), so the rows per tile double
// (at most 32): 8-21 % faster with 33 and 64 bins at 1080p and 12 MP, the same up to 17.
ScanTune scan_tune_default(int H, int W, int n_bins) {
    ScanTune t;
    t.vec = W >= 2048 ? 4 : 2;
    t.th = H < 900 ? 4 : H < 1800 ? 8 : 16;
    if (n_bins >= 33) t.th = t.th * 2 < 32 ? t.th * 2 : 32;
    const int64_t tw = 64 * t.vec;
    const int64_t tiles_x = (W + tw - 1) / tw;
    while (t.th > 4 && tiles_x * ((H + t.th - 1) / t.th) < 512) t.th /= 2;
    t.chunk = 4;
    return t;
}

// Tiling of the adjoint scans of the backward (FP64 deposit pairs in, gradient out): 16 rows
// per tile, halved (not below 4) while the image has fewer than 2048 tiles.
ScanTune scan_tune_adjoint(int H, int W) {
    ScanTune t;
    t.vec = W >= 2048 ? 4 : 2;
    t.th = 16;
    const int64_t tw = 64 * t.vec;
    const int64_t tiles_x = (W + tw - 1) / tw;
    while (t.th > 4 && tiles_x * ((H + t.th - 1) / t.th) < 2048) t.th /= 2;
    t.chunk = 4;
    return t;
}

bool scan_tune_valid(const ScanTune &t) {
    return (t.vec == 2 || t.vec == 4 || t.vec == 8) && t.th >= 1 && t.th <= 256 &&
           (t.chunk == 2 || t.chunk == 4 || t.chunk == 8);
}

ScanPlan make_scan_plan(int H, int W, int sat_prec, int n_planes, const ScanTune &t) {
    ScanPlan p{};
    p.H = H;
    p.W = W;
    p.vec = t.vec;
    p.th = t.th;
    p.chunk = t.chunk;
    p.tiles_x = (W + 64 * t.vec - 1) / (64 * t.vec);
    p.tiles_y = (H + t.th - 1) / t.th;
    p.sat_prec = sat_prec;
    p.n_planes = n_planes;
    p.acc_bytes = sat_prec < 0 ? 0 : (sat_prec == kF32 ? 4 : 8);
    size_t off = 0;
    auto take = [&](size_t bytes) {
        size_t o = off;
        off = round_up(off + bytes, 256);
        return o;
    };
    const size_t rs = (size_t)H * p.tiles_x, cs = (size_t)p.tiles_y * W,
                 tt = (size_t)p.tiles_y * p.tiles_x;
    const size_t a2 = 2 * p.acc_bytes, hq = (size_t)n_planes * 4;
    p.rs_sat = take(rs * a2);
    p.cs_sat = take(cs * a2);
    p.tt_sat = take(tt * a2);
    p.xc_sat = take(rs * a2);
    p.cse_sat = take(cs * a2);
    p.tte_sat = take(tt * a2);
    p.rs_h = take(rs * hq);
    p.cs_h = take(cs * hq);
    p.tt_h = take(tt * hq);
    p.xc_h = take(rs * hq);
    p.cse_h = take(cs * hq);
    p.tte_h = take(tt * hq);
    p.total = off;
    return p;
}

ScanK make_scank(const ScanArgs &a, const ScanPlan &plan, void *ws) {
    ScanK k{};
    char *w = static_cast<char *>(ws);
    k.v = a.v;
    k.ld_v = a.ld_v;
    k.H = a.H;
    k.W = a.W;
    k.th = plan.th;
    k.tiles_x = plan.tiles_x;
    k.tiles_y = plan.tiles_y;
    k.vec_load = (((uintptr_t)a.v & 15u) == 0) && (a.ld_v % 4 == 0);
    k.vh = a.v_hist ? a.v_hist : a.v;
    k.ld_vh = a.v_hist ? a.ld_v_hist : a.ld_v;
    k.vec_load_h = (((uintptr_t)k.vh & 15u) == 0) && (k.ld_vh % 4 == 0);
    k.log_src = a.log_src;
    k.offsets = a.offsets;
    k.sat = a.sat;
    k.ld_sat = a.ld_sat;
    k.edges = a.edges;
    k.n_bins = a.n_bins;
    k.layout = a.layout;
    k.n_planes = (a.n_planes > 0 && a.hist != nullptr) ? a.n_planes : 0;
    // histogram work items per tile: many planes are spread over up to kMaxHistItems waves
    const int nchunks = (k.n_planes + plan.chunk - 1) / plan.chunk;
    k.hist_items = nchunks < kMaxHistItems ? nchunks : kMaxHistItems;
    k.hist_chunks = k.hist_items > 0 ? (nchunks + k.hist_items - 1) / k.hist_items : 0;
    if (k.hist_chunks > 0) k.hist_items = (nchunks + k.hist_chunks - 1) / k.hist_chunks;
    k.hist = a.hist;
    k.ld_hist = a.ld_hist;
    k.plane_stride = a.plane_stride;
    // the memory-side cache (Infinity Cache) of MI355X holds 256 MiB
    constexpr int64_t kMallBytes = (int64_t)256 << 20;
    const int64_t sat_bytes =
        (a.sat && a.sat_prec >= 0) ? (int64_t)(a.sat_prec == kF32 ? 8 : 16) * (a.H + 1) * a.ld_sat : 0;
    const int64_t hist_bytes = (int64_t)k.n_planes * a.plane_stride * 4;
    k.stream_out = sat_bytes + hist_bytes > kMallBytes;
    k.rs_sat = w + plan.rs_sat;
    k.cs_sat = w + plan.cs_sat;
    k.tt_sat = w + plan.tt_sat;
    k.xc_sat = w + plan.xc_sat;
    k.cse_sat = w + plan.cse_sat;
    k.tte_sat = w + plan.tte_sat;
    k.rs_h = reinterpret_cast<uint32_t *>(w + plan.rs_h);
    k.cs_h = reinterpret_cast<uint32_t *>(w + plan.cs_h);
    k.tt_h = reinterpret_cast<uint32_t *>(w + plan.tt_h);
    k.xc_h = reinterpret_cast<uint32_t *>(w + plan.xc_h);
    k.cse_h = reinterpret_cast<uint32_t *>(w + plan.cse_h);
    k.tte_h = reinterpret_cast<uint32_t *>(w + plan.tte_h);
    return k;
}

int64_t scan_stage2_items(const ScanK &k, bool sat) { return stage2_split(k, sat).total; }

hipError_t launch_tables(const ScanArgs &a, const ScanPlan &plan, void *ws, hipStream_t s) {
    const ScanK k = make_scank(a, plan, ws);
    const bool sat = a.sat_prec >= 0 && a.sat != nullptr;
    const bool hist = k.n_planes > 0;
    if (!sat && !hist) return hipSuccess;
    switch (sat ? a.sat_prec : kF32) {
        case kF32: return dispatch_vec<kF32>(k, plan.vec, plan.chunk, sat, hist, s);
        case kC32x2: return dispatch_vec<kC32x2>(k, plan.vec, plan.chunk, sat, hist, s);
        default: return dispatch_vec<kF64>(k, plan.vec, plan.chunk, sat, hist, s);
    }
}

hipError_t launch_suffix_adjoint(const double2 *d, int64_t ld_d, const float *v, int64_t ld_v,
                                 int H, int W, float *gv, int64_t ld_gv, const ScanPlan &plan,
                                 void *ws, hipStream_t s, bool log_chain) {
    ScanK k{};
    char *w = static_cast<char *>(ws);
    k.v = v;
    k.ld_v = ld_v;
    k.vh = v;
    k.ld_vh = ld_v;
    k.H = H;
    k.W = W;
    k.th = plan.th;
    k.tiles_x = plan.tiles_x;
    k.tiles_y = plan.tiles_y;
    k.n_planes = 0;
    k.rs_sat = w + plan.rs_sat;
    k.cs_sat = w + plan.cs_sat;
    k.tt_sat = w + plan.tt_sat;
    k.xc_sat = w + plan.xc_sat;
    k.cse_sat = w + plan.cse_sat;
    k.tte_sat = w + plan.tte_sat;
    k.dsrc = d;
    k.ld_d = ld_d;
    k.gv = gv;
    k.ld_gv = ld_gv;
    k.log_chain = log_chain ? 1 : 0;
    switch (plan.vec) {
        case 2: return run3<kF64, 2, 2, true, false, true>(k, s);
        case 4: return run3<kF64, 4, 2, true, false, true>(k, s);
        default: return run3<kF64, 8, 2, true, false, true>(k, s);
    }
}

}  // namespace tmo
