// tm_lookback.hip -- the integral histogram (Eq. 7-8) in one pass over the image, with the
// tiles' carries exchanged by decoupled look-back.
//
// The counts are exact integers, so the carries may be summed in whatever order the
// look-back finds them: the result does not depend on timing.  (The floating-point integral
// image has no such freedom; it keeps the three-stage build.)
//
// One wave per tile of 128 columns (two per lane) x TH rows, the tiles taken in row-major
// order from a ticket counter, so a wave waits only on tiles whose waves already run.  A wave
//   1. reads its rows (eight at a time, the next eight in flight meanwhile) and, per row and
//      group of four planes, forms its two pixels' indicators as 8-bit fields of one word,
//      scans them over the lanes (giving the in-row prefix and the row total) and adds them
//      to its column totals; the prefix and the indicator bits go to LDS for step 4; it then
//      publishes the row and column totals as "aggregate" records;
//   2. looks back up its tile column for the column carries (the counts above the tile, per
//      column) and along its tile row for the row carries (the counts left of the tile, per
//      row): it adds aggregates until it meets an "inclusive" record, which already holds
//      everything before it, and publishes its own inclusive records.  Each poll requests
//      the records of two tiles at once (one with more than four planes);
//   3. publishes its total column carry and looks back along the tile row for the corner
//      carry (everything above and to the left of the tile), 16 or 8 tiles per poll;
//   4. writes every plane entry: the tile's own 2-D prefix (a running column sum of the
//      in-row prefixes) plus the row carries summed down to the row, the column carries
//      summed across to the column and the corner carry.
// Row and column records are 32-bit words {state:2, count:30}, corner records 64-bit
// {state, count}; all are written and read with agent-scope atomics, so each word is either
// absent (state 0) or whole and no fence is needed.  A small clearing kernel resets them (and
// the ticket counter) before each pass.  Every wait is bounded: if a word does not arrive in
// time the wave counts it as an inclusive zero and raises the status word at the start of
// the workspace, so the kernel always finishes.
#include "tm_device.h"
#include "tm_internal.h"

namespace tmo {

namespace {

constexpr int kLbVec = 2;                   // columns per lane
constexpr int kLbTw = kWave * kLbVec;       // columns per tile
constexpr int kLbBlock = 128;               // 2 waves, 2 independent tiles
constexpr uint32_t kAgg = 1, kIncl = 2;     // record states
constexpr uint32_t kCountMask = (1u << 30) - 1;

struct LbK {
    const float *v;
    int64_t ld_v;
    int H, W;
    const float *edges;
    int n_bins, np, layout;
    uint32_t *hist;
    int64_t ld_hist, plane_stride;
    int tiles_x, tiles_y;
    uint32_t *counter;   // ticket counter
    uint32_t *status;    // 0, or 1 if a wait ran out
    uint32_t *rowrec;    // [tile][TH][np]
    uint32_t *colrec;    // [tile][np][kLbTw]
    uint64_t *cornrec;   // [tile][np]
    int nt;              // non-temporal plane stores
    uint32_t spin;       // bound on the polls of one window (about a second by default)
};

__device__ __forceinline__ void put32(uint32_t *p, uint32_t state, uint32_t count) {
    __hip_atomic_store(p, (state << 30) | count, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ uint32_t get32(uint32_t *p) {
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ void put64(uint64_t *p, uint64_t state, uint32_t count) {
    __hip_atomic_store(p, (state << 32) | count, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ uint64_t get64(uint64_t *p) {
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

__device__ __forceinline__ void raise_status(const LbK &k) {
    __hip_atomic_store(k.status, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Plane p's indicator (the tables' convention): cumulative plane p counts bins <= p
// (v < edge[p]); per-bin plane p counts bin p (edge[p-1] <= v < edge[p]).
__device__ __forceinline__ void plane_edges(const LbK &k, int p, float &lo, float &hi) {
    if (k.layout == 1) {
        lo = -INFINITY;
        hi = k.edges[p];
    } else {
        lo = p == 0 ? -INFINITY : k.edges[p - 1];
        hi = p == k.n_bins - 1 ? INFINITY : k.edges[p];
    }
}

// Polls a window of J x S record words, slot s of the j-th tile back at bp[j] + off(s), until
// every wanted one (j < jn and slot s still open) is present.  Unwanted words read as
// inclusive zeros.  All wanted words are requested together, so one round trip covers the
// window.
template <int J, int S, class Off>
__device__ __forceinline__ void poll32(const LbK &k, uint32_t (&w)[J][S], uint32_t *const (&bp)[J],
                                       int jn, const bool (&open)[S], Off off) {
#pragma unroll
    for (int j = 0; j < J; ++j)
#pragma unroll
        for (int s = 0; s < S; ++s)
            w[j][s] = (j < jn && open[s]) ? get32(bp[j] + off(s)) : (kIncl << 30);
    for (uint32_t it = 0;; ++it) {
        bool miss = false;
#pragma unroll
        for (int j = 0; j < J; ++j)
#pragma unroll
            for (int s = 0; s < S; ++s) miss = miss || (w[j][s] >> 30) == 0;
        if (!__any(miss)) return;
        if (it == k.spin) {
#pragma unroll
            for (int j = 0; j < J; ++j)
#pragma unroll
                for (int s = 0; s < S; ++s)
                    if ((w[j][s] >> 30) == 0) w[j][s] = kIncl << 30;
            if (miss) raise_status(k);
            return;
        }
        __builtin_amdgcn_s_sleep(1);
#pragma unroll
        for (int j = 0; j < J; ++j)
#pragma unroll
            for (int s = 0; s < S; ++s)
                if ((w[j][s] >> 30) == 0) w[j][s] = get32(bp[j] + off(s));
    }
}

// Pass 2 over a tile's rows: the plane entries from the in-row prefixes kept in LDS.
// FULL: the tile lies inside the image (8-byte stores); NT: non-temporal stores.
template <int NP, int TH, bool FULL, bool NT>
__device__ __forceinline__ void write_rows(const LbK &k, const uint32_t (*ls)[kWave], int y0,
                                           int rows, int xl, const uint32_t (&xc)[NP],
                                           const uint32_t (&cpre)[NP][kLbVec]) {
    constexpr int NG = NP / 4;
    const int lane = lane_id();
    const int np = k.np;
    uint32_t tp[NP][kLbVec];     // the tile's own 2-D prefix, row by row
    uint32_t bsum[NP];           // row carries summed down to the row
#pragma unroll
    for (int p = 0; p < NP; ++p) {
        bsum[p] = 0u;
        tp[p][0] = tp[p][1] = 0u;
    }
    TM_GLOBAL uint32_t *out = gptr(k.hist) + (int64_t)y0 * k.ld_hist + xl;
    for (int r = 0; r < rows; ++r, out += k.ld_hist) {
#pragma unroll
        for (int g = 0; g < NG; ++g) {
            const uint32_t ex = ls[(r * NG + g) * 2][lane];        // exclusive in-row prefix
            const uint32_t bits = ls[(r * NG + g) * 2 + 1][lane];  // column 0 bit 0, column 1 bit 1
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const int p = 4 * g + q;
                const uint32_t e = (ex >> (8 * q)) & 0xffu;
                const uint32_t b0 = (bits >> (8 * q)) & 1u, b1 = (bits >> (8 * q + 1)) & 1u;
                tp[p][0] += e + b0;
                tp[p][1] += e + b0 + b1;
                bsum[p] += readlane(xc[p], r);
                if (p >= np) continue;
                const uint32_t o0 = tp[p][0] + bsum[p] + cpre[p][0];
                const uint32_t o1 = tp[p][1] + bsum[p] + cpre[p][1];
                TM_GLOBAL uint32_t *o = out + (int64_t)p * k.plane_stride;
                if (FULL) {   // 8-byte stores: the pitch is a multiple of 64 entries
                    typedef uint32_t u2v __attribute__((ext_vector_type(2)));
                    u2v wv;
                    wv.x = o0;
                    wv.y = o1;
                    TM_GLOBAL u2v *dst = reinterpret_cast<TM_GLOBAL u2v *>(o);
                    if (NT) __builtin_nontemporal_store(wv, dst);
                    else *dst = wv;
                } else {
                    if (xl < k.W) o[0] = o0;
                    if (xl + 1 < k.W) o[1] = o1;
                }
            }
        }
    }
}

template <int NP, int TH, bool CUM>
__device__ void lookback_tile(const LbK &k, int t, uint32_t (*ls)[kWave]) {
    constexpr int NG = NP / 4;                  // groups of four planes
    // look-back windows in tiles: two with four planes, one with eight (larger windows hold
    // more words in registers; measured slower through the lower occupancy)
    constexpr int JC = 8 / NP;                  // column look-back window (tiles)
    constexpr int JR = 8 / NP;                  // row look-back window (tiles)
    constexpr int JK = kWave / NP;              // corner look-back window (tiles)
    const int lane = lane_id();
    const int tx = t % k.tiles_x, ty = t / k.tiles_x;
    const int x0 = tx * kLbTw, y0 = ty * TH;
    const int rows = min(TH, k.H - y0);
    const int xl = x0 + lane * kLbVec;
    const int np = k.np;

    // 1. per row and group of four planes: the indicators of the lane's two pixels as 8-bit
    //    fields (one word per column), their in-row scan over the lanes (exclusive prefix and
    //    row total) and the column totals; the prefix and the indicator bits go to LDS for
    //    pass 2 (each lane reads back only its own slots: no barrier)
    uint32_t rtp[NG], ccp[NG][kLbVec];
    {
        float lo[NP], hi[NP];
#pragma unroll
        for (int p = 0; p < NP; ++p) {
            lo[p] = INFINITY;
            hi[p] = -INFINITY;
            if (p < np) plane_edges(k, p, lo[p], hi[p]);
        }
#pragma unroll
        for (int g = 0; g < NG; ++g) {
            rtp[g] = 0u;
#pragma unroll
            for (int i = 0; i < kLbVec; ++i) ccp[g][i] = 0u;
        }
        // loads are clamped into the image (no branches); pixels outside count nowhere
        int xcl[kLbVec];
        bool xin[kLbVec];
#pragma unroll
        for (int i = 0; i < kLbVec; ++i) {
            xin[i] = xl + i < k.W;
            xcl[i] = min(xl + i, k.W - 1);
        }
        auto load8 = [&](float (&v)[8][kLbVec], int r0) {
#pragma unroll
            for (int rr = 0; rr < 8; ++rr) {
                const float *row = k.v + (int64_t)min(y0 + r0 + rr, k.H - 1) * k.ld_v;
#pragma unroll
                for (int i = 0; i < kLbVec; ++i) v[rr][i] = row[xcl[i]];
            }
        };
        float cur[8][kLbVec];
        load8(cur, 0);
#pragma unroll 1
        for (int r0 = 0; r0 < TH; r0 += 8) {
            float nxt[8][kLbVec];
            if (r0 + 8 < TH) load8(nxt, r0 + 8);   // the next rows are in flight meanwhile
#pragma unroll
            for (int rr = 0; rr < 8; ++rr) {
                const int r = r0 + rr;
                const bool rin = r < rows;
#pragma unroll
                for (int g = 0; g < NG; ++g) {
                    uint32_t f[kLbVec];
#pragma unroll
                    for (int i = 0; i < kLbVec; ++i) {
                        f[i] = 0u;
#pragma unroll
                        for (int q = 0; q < 4; ++q) {
                            const int p = 4 * g + q;
                            const bool c = CUM ? cur[rr][i] < hi[p]
                                               : (cur[rr][i] >= lo[p] && cur[rr][i] < hi[p]);
                            f[i] |= c ? (1u << (8 * q)) : 0u;
                        }
                        f[i] = (rin && xin[i]) ? f[i] : 0u;
                        ccp[g][i] += f[i];
                    }
                    const uint32_t inc = wave_inclusive<AddU32>(f[0] + f[1]);
                    const uint32_t tot = readlane(inc, kWave - 1);
                    if (lane == r) rtp[g] = tot;
                    ls[(r * NG + g) * 2][lane] = wave_shr1(inc);
                    ls[(r * NG + g) * 2 + 1][lane] = f[0] | (f[1] << 1);
                }
            }
#pragma unroll
            for (int rr = 0; rr < 8; ++rr)
#pragma unroll
                for (int i = 0; i < kLbVec; ++i) cur[rr][i] = nxt[rr][i];
        }
    }
    uint32_t cc[NP][kLbVec], rt[NP];
#pragma unroll
    for (int p = 0; p < NP; ++p) {
        rt[p] = (rtp[p / 4] >> (8 * (p % 4))) & 0xffu;
#pragma unroll
        for (int i = 0; i < kLbVec; ++i) cc[p][i] = (ccp[p / 4][i] >> (8 * (p % 4))) & 0xffu;
    }

    // publish the aggregates
    uint32_t *rrec = k.rowrec + (int64_t)t * TH * np;
    uint32_t *crec = k.colrec + (int64_t)t * np * kLbTw;
    if (lane < rows) {
#pragma unroll
        for (int p = 0; p < NP; ++p)
            if (p < np) put32(rrec + lane * np + p, kAgg, rt[p]);
    }
#pragma unroll
    for (int p = 0; p < NP; ++p)
        if (p < np) {
#pragma unroll
            for (int i = 0; i < kLbVec; ++i) put32(crec + p * kLbTw + lane * kLbVec + i, kAgg, cc[p][i]);
        }

    // 2a. column carries: look back up the tile column, JC tiles per poll
    uint32_t cse[NP][kLbVec];
    {
        bool done[NP * kLbVec];
#pragma unroll
        for (int s = 0; s < NP * kLbVec; ++s) {
            cse[s / kLbVec][s % kLbVec] = 0u;
            done[s] = s / kLbVec >= np || ty == 0;
        }
        for (int base = ty - 1; base >= 0; base -= JC) {
            bool open = false;
#pragma unroll
            for (int s = 0; s < NP * kLbVec; ++s) open = open || !done[s];
            if (!__any(open)) break;
            bool op[NP * kLbVec];
#pragma unroll
            for (int s = 0; s < NP * kLbVec; ++s) op[s] = !done[s];
            uint32_t *bp[JC];
#pragma unroll
            for (int j = 0; j < JC; ++j)
                bp[j] = k.colrec + ((int64_t)(base - j) * k.tiles_x + tx) * np * kLbTw + lane * kLbVec;
            uint32_t w[JC][NP * kLbVec];
            poll32<JC, NP * kLbVec>(k, w, bp, min(JC, base + 1), op, [](int s) {
                return (s / kLbVec) * kLbTw + s % kLbVec;
            });
#pragma unroll
            for (int j = 0; j < JC; ++j)
#pragma unroll
                for (int s = 0; s < NP * kLbVec; ++s)
                    if (!done[s]) {
                        cse[s / kLbVec][s % kLbVec] += w[j][s] & kCountMask;
                        done[s] = (w[j][s] >> 30) == kIncl;
                    }
        }
    }
#pragma unroll
    for (int p = 0; p < NP; ++p)
        if (p < np) {
#pragma unroll
            for (int i = 0; i < kLbVec; ++i)
                put32(crec + p * kLbTw + lane * kLbVec + i, kIncl, cse[p][i] + cc[p][i]);
        }

    // 2b. row carries: look back along the tile row (lane r, its row's planes), JR tiles per
    //     poll
    uint32_t xc[NP];
    {
        bool done[NP];
#pragma unroll
        for (int p = 0; p < NP; ++p) {
            xc[p] = 0u;
            done[p] = p >= np || lane >= rows || tx == 0;
        }
        for (int base = tx - 1; base >= 0; base -= JR) {
            bool open = false;
#pragma unroll
            for (int p = 0; p < NP; ++p) open = open || !done[p];
            if (!__any(open)) break;
            bool op[NP];
#pragma unroll
            for (int p = 0; p < NP; ++p) op[p] = !done[p];
            uint32_t *bp[JR];
#pragma unroll
            for (int j = 0; j < JR; ++j)
                bp[j] = k.rowrec + ((int64_t)ty * k.tiles_x + base - j) * TH * np + lane * np;
            uint32_t w[JR][NP];
            poll32<JR, NP>(k, w, bp, min(JR, base + 1), op, [](int p) { return p; });
#pragma unroll
            for (int j = 0; j < JR; ++j)
#pragma unroll
                for (int p = 0; p < NP; ++p)
                    if (!done[p]) {
                        xc[p] += w[j][p] & kCountMask;
                        done[p] = (w[j][p] >> 30) == kIncl;
                    }
        }
    }
    if (lane < rows) {
#pragma unroll
        for (int p = 0; p < NP; ++p)
            if (p < np) put32(rrec + lane * np + p, kIncl, xc[p] + rt[p]);
    }

    // 3. corner carry: the tile's total column carry, then a look-back along the tile row;
    //    lane l reads plane l % NP of the (l / NP)-th tile back
    uint32_t corner[NP];
    {
        uint32_t ct[NP];
#pragma unroll
        for (int p = 0; p < NP; ++p) ct[p] = wave_sum<AddU32>(cse[p][0] + cse[p][1]);
        uint64_t *kr = k.cornrec + (int64_t)t * np;
        uint32_t mine = 0u;
#pragma unroll
        for (int p = 0; p < NP; ++p)
            if (lane == p) mine = ct[p];
        if (lane < np) put64(kr + lane, kAgg, mine);
        const int jj = lane / NP, pp = lane % NP;
        uint64_t same = 0ull;   // the lanes reading plane pp, nearer tiles first
#pragma unroll
        for (int j = 0; j < JK; ++j) same |= 1ull << (j * NP + pp);
        const uint64_t before = same & ((1ull << lane) - 1ull);
        uint32_t open = 0u;     // planes still looking back (bit p)
#pragma unroll
        for (int p = 0; p < NP; ++p) {
            corner[p] = 0u;
            if (p < np && tx > 0) open |= 1u << p;
        }
        for (int base = tx - 1; base >= 0 && open; base -= JK) {
            const int tt = base - jj;
            const bool want = tt >= 0 && ((open >> pp) & 1u);
            uint64_t *src = k.cornrec + ((int64_t)ty * k.tiles_x + tt) * np + pp;
            uint64_t w = want ? get64(src) : (uint64_t)kIncl << 32;
            for (uint32_t it = 0;; ++it) {
                const bool miss = (w >> 32) == 0;
                if (!__any(miss)) break;
                if (it == k.spin) {
                    if (miss) {
                        w = (uint64_t)kIncl << 32;
                        raise_status(k);
                    }
                    break;
                }
                __builtin_amdgcn_s_sleep(1);
                if (miss) w = get64(src);
            }
            const uint64_t incl = __ballot((w >> 32) == kIncl);
            // a lane counts if no nearer tile of its plane is inclusive
            const uint32_t c = ((incl & before) == 0ull && ((open >> pp) & 1u)) ? (uint32_t)w : 0u;
#pragma unroll
            for (int p = 0; p < NP; ++p) {
                if (!((open >> p) & 1u)) continue;
                corner[p] += wave_sum<AddU32>(pp == p ? c : 0u);
                uint64_t samep = 0ull;
#pragma unroll
                for (int j = 0; j < JK; ++j) samep |= 1ull << (j * NP + p);
                if (incl & samep) open &= ~(1u << p);
            }
        }
        uint32_t sum = 0u;
#pragma unroll
        for (int p = 0; p < NP; ++p)
            if (lane == p) sum = corner[p] + ct[p];
        if (lane < np) put64(kr + lane, kIncl, sum);
    }

    // 4. the plane entries
    uint32_t cpre[NP][kLbVec];   // corner + column carries summed across to each column
#pragma unroll
    for (int p = 0; p < NP; ++p) {
        const uint32_t s = cse[p][0] + cse[p][1];
        const uint32_t ex = wave_shr1(wave_inclusive<AddU32>(s));
        cpre[p][0] = corner[p] + ex + cse[p][0];
        cpre[p][1] = cpre[p][0] + cse[p][1];
    }
    if (x0 + kLbTw <= k.W) {
        if (k.nt) write_rows<NP, TH, true, true>(k, ls, y0, rows, xl, xc, cpre);
        else write_rows<NP, TH, true, false>(k, ls, y0, rows, xl, xc, cpre);
    } else {
        write_rows<NP, TH, false, false>(k, ls, y0, rows, xl, xc, cpre);
    }
    // zero border: row -1 over the tile's columns (and x = -1 on the first tile column), the
    // padding columns [W, ld) on the last tile column (rows y0-1.. on the first tile row)
    for (int p = 0; p < np; ++p) {
        uint32_t *t0 = k.hist + (int64_t)p * k.plane_stride;
        if (ty == 0)
            for (int x = x0 - (tx == 0 ? 1 : 0) + lane; x < x0 + kLbTw && x < k.W; x += kWave)
                t0[-k.ld_hist + x] = 0u;
        if (tx == k.tiles_x - 1)
            for (int r = (ty == 0 ? -1 : 0); r < rows; ++r)
                for (int x = k.W + lane; x < k.ld_hist; x += kWave)
                    t0[(int64_t)(y0 + r) * k.ld_hist + x] = 0u;
    }
}

template <int NP, int TH, bool CUM>
__global__ void __launch_bounds__(kLbBlock) lookback_hist_kernel(LbK k) {
    uint32_t t = 0u;
    if (lane_id() == 0)
        t = __hip_atomic_fetch_add(k.counter, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    t = (uint32_t)__builtin_amdgcn_readfirstlane((int)t);
    if (t >= (uint32_t)(k.tiles_x * k.tiles_y)) return;
    // per wave and row: the in-row prefix and the indicator bits of each group of planes
    __shared__ uint32_t rowdata[kLbBlock / kWave][TH * (NP / 4) * 2][kWave];
    lookback_tile<NP, TH, CUM>(k, (int)t, rowdata[wave_id()]);
}

// Clears the records and the ticket counter (a fill kernel: the pass may be captured into a
// graph, where memset nodes are avoided).
__global__ void __launch_bounds__(kLbBlock) lookback_clear_kernel(uint4 *rec, int64_t n,
                                                                  uint32_t *hdr) {
    const int64_t i = (int64_t)blockIdx.x * kLbBlock + threadIdx.x;
    if (i < n) rec[i] = make_uint4(0u, 0u, 0u, 0u);
    if (i < 2) hdr[i] = 0u;
}

// Polls of one look-back window before it counts as timed out (settable for tests of that
// path; 0 selects the default of 2^20, about a second).
uint32_t g_lookback_spin = 0;

}  // namespace

void set_lookback_spin_limit(uint32_t polls) { g_lookback_spin = polls; }

// Rows per tile: 32, or 16 while 32 would leave fewer than about two waves per compute unit,
// and always 16 for more than four planes (their rows take twice the LDS).
int lookback_rows(int H, int W, int n_planes) {
    const int64_t tx = (W + kLbTw - 1) / kLbTw;
    return n_planes <= 4 && tx * ((H + 31) / 32) >= 480 ? 32 : 16;
}

LookbackPlan make_lookback_plan(int H, int W, int n_planes, int th) {
    LookbackPlan p{};
    p.th = th;
    p.tiles_x = (W + kLbTw - 1) / kLbTw;
    p.tiles_y = (H + p.th - 1) / p.th;
    const int64_t tiles = (int64_t)p.tiles_x * p.tiles_y;
    auto up = [](int64_t b) { return (size_t)((b + 255) / 256) * 256; };
    p.rowrec = 256;
    p.colrec = p.rowrec + up(tiles * p.th * n_planes * 4);
    p.cornrec = p.colrec + up(tiles * n_planes * kLbTw * 4);
    p.total = p.cornrec + up(tiles * n_planes * 8);
    return p;
}

hipError_t launch_lookback_hist(const LookbackArgs &a, const LookbackPlan &plan, void *ws,
                                hipStream_t s) {
    if (plan.th != 16 && (plan.th != 32 || a.n_planes > 4)) return hipErrorInvalidValue;
    char *w = static_cast<char *>(ws);
    LbK k{};
    k.v = a.v;
    k.ld_v = a.ld_v;
    k.H = a.H;
    k.W = a.W;
    k.edges = a.edges;
    k.n_bins = a.n_bins;
    k.np = a.n_planes;
    k.layout = a.layout;
    k.hist = a.hist;
    k.ld_hist = a.ld_hist;
    k.plane_stride = a.plane_stride;
    k.tiles_x = plan.tiles_x;
    k.tiles_y = plan.tiles_y;
    k.counter = reinterpret_cast<uint32_t *>(w);
    k.status = reinterpret_cast<uint32_t *>(w) + 1;
    k.rowrec = reinterpret_cast<uint32_t *>(w + plan.rowrec);
    k.colrec = reinterpret_cast<uint32_t *>(w + plan.colrec);
    k.cornrec = reinterpret_cast<uint64_t *>(w + plan.cornrec);
    k.nt = a.nt;
    k.spin = g_lookback_spin ? g_lookback_spin : (1u << 20);
    // the record area is a whole number of 256-byte blocks: cleared 16 bytes per thread
    const int64_t n16 = (int64_t)(plan.total - plan.rowrec) / 16;
    hipLaunchKernelGGL(lookback_clear_kernel, dim3((unsigned)((n16 + kLbBlock - 1) / kLbBlock)),
                       dim3(kLbBlock), 0, s, reinterpret_cast<uint4 *>(k.rowrec), n16, k.counter);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    const int64_t tiles = (int64_t)plan.tiles_x * plan.tiles_y;
    const unsigned grid = (unsigned)((tiles + kLbBlock / kWave - 1) / (kLbBlock / kWave));
    const bool cum = a.layout == 1;
    if (a.n_planes > 4) {   // eight planes: 16-row tiles only
        if (cum) hipLaunchKernelGGL((lookback_hist_kernel<8, 16, true>), dim3(grid), dim3(kLbBlock), 0, s, k);
        else hipLaunchKernelGGL((lookback_hist_kernel<8, 16, false>), dim3(grid), dim3(kLbBlock), 0, s, k);
    } else if (plan.th == 32) {
        if (cum) hipLaunchKernelGGL((lookback_hist_kernel<4, 32, true>), dim3(grid), dim3(kLbBlock), 0, s, k);
        else hipLaunchKernelGGL((lookback_hist_kernel<4, 32, false>), dim3(grid), dim3(kLbBlock), 0, s, k);
    } else {
        if (cum) hipLaunchKernelGGL((lookback_hist_kernel<4, 16, true>), dim3(grid), dim3(kLbBlock), 0, s, k);
        else hipLaunchKernelGGL((lookback_hist_kernel<4, 16, false>), dim3(grid), dim3(kLbBlock), 0, s, k);
    }
    return hipGetLastError();
}

}  // namespace tmo
