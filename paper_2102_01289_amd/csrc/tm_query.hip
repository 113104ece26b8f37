// tm_query.hip -- stage a4: the fused per-pixel query and blend.
//
// One thread per pixel, all receptive fields in one launch (the paper launches three
// kernels per field, Section III-A).  For each field j the thread reads the four clamped
// window corners (Algorithm 1) of the interleaved integral image {I(v), I(v^2)} and of the
// cumulative histogram plane G_b selected by its own bin b, then forms
//   N (clamped window area), S1, S2 (Eq. 6), c = G_b box (Eq. 9 summed as in Eq. 1),
//   P = c / N (Eq. 1), L_j = min L_d + (max L_d - min L_d) P (Eq. 2),
//   var = max(0, S2/N - (S1/N)^2) (Eq. 10), W_j = var / (var + eps) (Eq. 4),
// and accumulates sum W_j L_j, sum W_j in registers for Eq. 3.  Per-field maps never touch
// memory.  The variance is formed in FP64 for the compensated and FP64 tables.
#include "tm_device.h"
#include "tm_internal.h"

namespace tmo {

namespace {

constexpr int kBlock = 256;
constexpr int kRows = kQueryRows;   // a block covers 64 columns x 4 rows
constexpr int kMaxS = 8;            // TM_MAX_SCALES


// Table entry types per integral-image precision.
template <int P> struct SatEntry { using T = float2; };     // {I1, I2}
template <> struct SatEntry<kC32x2> { using T = float4; };  // {I1.hi, I1.lo, I2.hi, I2.lo}
template <> struct SatEntry<kF64> { using T = double2; };

// Window mean m and variance var (Eq. 10 read as the population variance, not yet clamped)
// from the four corner entries of the interleaved integral image and the reciprocal of the
// window area.  The corner sums cancel heavily (large quadrant sums, small window sums), so
// for the compensated and FP64 tables they are combined in FP64.
template <int P>
__device__ __forceinline__ void window_moments(const typename SatEntry<P>::T &A,
                                               const typename SatEntry<P>::T &B,
                                               const typename SatEntry<P>::T &C,
                                               const typename SatEntry<P>::T &D, double inv_n,
                                               float mu1, float mu2, double &m, double &var) {
    if constexpr (P == kF32) {
        const float inv = (float)inv_n;
        const float mf = ((A.x + C.x) - (B.x + D.x)) * inv;
        const float vf = __builtin_fmaf((A.y + C.y) - (B.y + D.y), inv, -(mf * mf));
        m = (double)mf;
        var = (double)vf;
    } else if constexpr (P == kC32x2) {
        // leading parts exactly in FP64; trailing parts (2^-24 smaller) summed in FP32
        const double h1 = ((double)A.x + (double)C.x) - ((double)B.x + (double)D.x);
        const double h2 = ((double)A.z + (double)C.z) - ((double)B.z + (double)D.z);
        const float l1 = (A.y + C.y) - (B.y + D.y);
        const float l2 = (A.w + C.w) - (B.w + D.w);
        m = __builtin_fma(h1 + (double)l1, inv_n, (double)mu1);
        const double e2 = __builtin_fma(h2 + (double)l2, inv_n, (double)mu2);
        var = __builtin_fma(-m, m, e2);
    } else {
        m = ((A.x + C.x) - (B.x + D.x)) * inv_n;
        var = __builtin_fma(-m, m, ((A.y + C.y) - (B.y + D.y)) * inv_n);
    }
}

// 1/N for an integer window area N: hardware reciprocal refined by one Newton step
// (relative error ~2^-50, far below the table error it multiplies).
__device__ __forceinline__ double recip_area(int N) {
    const double d = (double)N;
    double r = __builtin_amdgcn_rcp(d);
    r = __builtin_fma(__builtin_fma(-d, r, 1.0), r, r);
    return r;
}

// One 64 x 4 tile of one image.  sh_edges is the block's copy of the image's bin edges.
// A wave covers 64 columns of one row, so every row index and row address is wave-uniform
// (scalar registers) and the lanes only add their column offsets.  H32: every histogram
// byte offset fits in 32 bits, so a lane's plane is folded into its 32-bit column offset.
// RESID: also write the per-pixel residual planes the backward needs (their derivation is
// in the backward's header): the pair {R1_j, R2_j} = {-2 c_j m_j / N_j, c_j / N_j} with
// c_j = (L_j - L)/D eps/(var_j + eps)^2 (zero where var_j was clamped or D = 0), one
// interleaved pair plane per field, then E = sum_j (L_j - L)/D (-var_j/(var_j + eps)^2) and
// Pbar = sum_j W_j P_j / D.
// Outputs and residual planes are written with streaming (non-temporal) stores so that
// they do not evict table lines the neighbouring tiles still read.
template <int P, bool RESID, bool H32>
__device__ __forceinline__ void forward_tile(const FwdK &k, uint32_t tile, float *sh_edges) {
    using ST = typename SatEntry<P>::T;
    constexpr uint32_t ES = sizeof(ST);
    const int ne = k.p.n_bins - 1;
    __syncthreads();   // the previous tile of this block may still read sh_edges
    for (int i = threadIdx.x; i < ne; i += kBlock) sh_edges[i] = gptr(k.edges)[i];
    __syncthreads();

    int tx, rg;
    comb_map(tile, k.tiles_x, k.p4, k.teeth, tx, rg);
    const int x = tx * kWave + lane_id();
    const int y = rg * kRows + wave_id();
    if (y >= k.H || x >= k.W) return;

    const float v = gptr(k.v)[(int64_t)y * k.ld_v + x];
    // bin b = #{edges <= v} (edges ascending)
    int lo = 0, hi = ne;
    while (lo < hi) {
        const int mid = (lo + hi) >> 1;
        if (sh_edges[mid] <= v) lo = mid + 1; else hi = mid;
    }
    const int b = lo;
    // histogram addressing: the plane G_b of this pixel, entry (-1, -1) at byte 0 of a row
    // base, lanes add their plane (H32) and column offsets
    const int64_t hplane = (int64_t)(b > 0 ? b - 1 : 0) * k.plane_stride;
    const uint32_t hplane_b = H32 ? (uint32_t)(hplane * 4) : 0u;
    const uint32_t *hlane = H32 ? nullptr : k.hist + hplane;
    const char *sat0 = static_cast<const char *>(k.sat) - (k.ld_sat + 1) * (int64_t)ES;
    const char *hist0 = reinterpret_cast<const char *>(k.hist - (k.ld_hist + 1));

    const int s = k.p.n_scales;
    // eps and the display range: the launch's values, or device values read at run time
    float eps = k.p.eps, ld_min = k.p.ld_min, ld_max = k.p.ld_max;
    if (k.p.scalars) {
        const TM_GLOBAL float *sc = gptr(k.p.scalars);
        eps = sc[0];
        ld_min = sc[1];
        ld_max = sc[2];
    }
    const float ldr = ld_max - ld_min;
    const float mu1 = P == kC32x2 ? gptr(k.offsets)[0] : 0.f;
    const float mu2 = P == kC32x2 ? gptr(k.offsets)[1] : 0.f;
    float num = 0.f, den = 0.f, lsum = 0.f, pn = 0.f, psum = 0.f;
    float vj[kMaxS], mj[kMaxS], lj[kMaxS], nj[kMaxS];
    bool clj[kMaxS];
#pragma unroll
    for (int j = 0; j < kMaxS; ++j) {
        if (j < s) {
            const int rx = k.p.rx[j], ry = k.p.ry[j];
            const int xm = max(x - rx - 1, -1), xp = min(x + rx, k.W - 1);
            const int ym = max(y - ry - 1, -1), yp = min(y + ry, k.H - 1);   // uniform
            const int N = (xp - xm) * (yp - ym);
            const double inv_n = recip_area(N);
            const char *sm = sat0 + (int64_t)(ym + 1) * k.ld_sat * ES;
            const char *sp = sat0 + (int64_t)(yp + 1) * k.ld_sat * ES;
            const uint32_t oxm = (uint32_t)(xm + 1) * ES, oxp = (uint32_t)(xp + 1) * ES;
            double m, vr;
            window_moments<P>(load_at<ST>(sm, oxm), load_at<ST>(sm, oxp), load_at<ST>(sp, oxp),
                              load_at<ST>(sp, oxm), inv_n, mu1, mu2, m, vr);
            // a one-pixel window has zero variance by definition (its rounding noise would
            // otherwise reach the gradient through the clamp)
            const bool clamped = !(vr > 0.0) || N == 1;
            const float var = clamped ? 0.f : (float)vr;
            uint32_t c = 0u;
            if (b > 0) {
                if constexpr (H32) {
                    const char *hm = hist0 + (int64_t)(ym + 1) * k.ld_hist * 4;
                    const char *hp = hist0 + (int64_t)(yp + 1) * k.ld_hist * 4;
                    const uint32_t hxm = hplane_b + (uint32_t)(xm + 1) * 4u;
                    const uint32_t hxp = hplane_b + (uint32_t)(xp + 1) * 4u;
                    c = load_at<uint32_t>(hp, hxp) + load_at<uint32_t>(hm, hxm) -
                        load_at<uint32_t>(hm, hxp) - load_at<uint32_t>(hp, hxm);
                } else {
                    const TM_GLOBAL uint32_t *pm = gptr(hlane) + (int64_t)ym * k.ld_hist;
                    const TM_GLOBAL uint32_t *pp = gptr(hlane) + (int64_t)yp * k.ld_hist;
                    c = pp[xp] + pm[xm] - pm[xp] - pp[xm];
                }
            }
            const float Pj = (float)c * (float)inv_n;
            const float Lj = __builtin_fmaf(ldr, Pj, ld_min);
            // Eq. 4 with the hardware reciprocal, held in [0, 1] (the reciprocal's last-bit
            // error could otherwise lift W_j of a very large variance one ulp above 1)
            const float Wj = fminf(var * __builtin_amdgcn_rcpf(var + eps), 1.f);
            if (k.maps) {
                TM_GLOBAL float *mp = gptr(k.maps) + (int64_t)y * k.W + x;
                __builtin_nontemporal_store(Lj, mp + (int64_t)j * k.mstride);
                __builtin_nontemporal_store(Wj, mp + (int64_t)(s + j) * k.mstride);
            }
            num = __builtin_fmaf(Wj, Lj, num);
            den += Wj;
            lsum += Lj;
            if (RESID) {
                pn = __builtin_fmaf(Wj, Pj, pn);
                psum += Pj;
                vj[j] = var;
                mj[j] = (float)m;
                lj[j] = Lj;
                nj[j] = (float)inv_n;
                clj[j] = clamped;
            }
        }
    }
    const float L = den > 0.f ? num / den : lsum / (float)s;
    if (k.out) __builtin_nontemporal_store(L, gptr(k.out) + (int64_t)y * k.ld_out + x);
    if (k.rgb_out) {
        // Eq. 12: each channel keeps its ratio to the input luminance, compressed by sat
        const TM_GLOBAL float *ci = gptr(k.rgb) + (int64_t)y * k.rgb_ld + x;
        TM_GLOBAL float *co = gptr(k.rgb_out) + (int64_t)y * k.out_ld + x;
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            const float cin = fmaxf(ci[c * k.rgb_cs], 0.f);
            const float r = v > 0.f ? cin / v : 1.f;
            __builtin_nontemporal_store(powf(r, k.saturation) * L, co + c * k.out_cs);
        }
    }
    if (RESID) {
        TM_GLOBAL float *ro = gptr(k.resid) + (int64_t)y * k.W + x;
        const int64_t ps = k.rstride;
        const float inv_d = den > 0.f ? 1.0f / den : 0.f;
        float E = 0.f;
#pragma unroll
        for (int j = 0; j < kMaxS; ++j) {
            if (j < s) {
                const float d = (lj[j] - L) * inv_d;
                const float r = __builtin_amdgcn_rcpf(vj[j] + eps);
                const float r2 = r * r;
                E = __builtin_fmaf(d, -vj[j] * r2, E);
                const float c = clj[j] ? 0.f : d * eps * r2;
                const float cn = c * nj[j];
                TM_GLOBAL float *pr = gptr(k.resid) + 2 * ((int64_t)j * ps + (int64_t)y * k.W + x);
                __builtin_nontemporal_store(-2.0f * cn * mj[j], pr);
                __builtin_nontemporal_store(cn, pr + 1);
            }
        }
        __builtin_nontemporal_store(E, ro + (int64_t)(2 * s) * ps);
        __builtin_nontemporal_store(den > 0.f ? pn / den : psum / (float)s,
                                    ro + (int64_t)(2 * s + 1) * ps);
    }
}

template <int P, bool RESID, bool H32>
__global__ void __launch_bounds__(kBlock) forward_kernel(FwdK k) {
    __shared__ float sh_edges[256];
    forward_tile<P, RESID, H32>(k, xcd_tile(blockIdx.x, gridDim.x), sh_edges);
}

// Batched query over the tiles of images [0, count) of ks: one block per tile of the
// flattened list (tiles of image i are prefix[i] .. prefix[i+1]-1, each image's in comb
// order), remapped like the single-image launch so that each XCD gets one contiguous eighth
// of the list.  The hardware hands the blocks out in order, so the tiles in flight stay a
// compact window of the list: a persistent grid with a static split lets its blocks drift
// apart, which was measured 34 % slower on the same image.
template <int P, bool H32>
__global__ void __launch_bounds__(kBlock) forward_batch(const FwdK *__restrict__ ks,
                                                       const int64_t *__restrict__ prefix,
                                                       int count) {
    __shared__ float sh_edges[256];
    const int64_t g = prefix[0] + xcd_tile(blockIdx.x, gridDim.x);
    const int i = find_image(prefix, count, g);
    forward_tile<P, false, H32>(ks[i], (uint32_t)(g - prefix[i]), sh_edges);
}

}  // namespace

int64_t query_blocks(const FwdK &k) { return (int64_t)k.tiles_x * k.p4 * k.teeth; }

template <bool H32>
hipError_t launch_fwd_batch(const FwdK *ks, const int64_t *tile_prefix, int count, int prec,
                            unsigned grid, hipStream_t s) {
    switch (prec) {
        case kF32:
            hipLaunchKernelGGL((forward_batch<kF32, H32>), dim3(grid), dim3(kBlock), 0, s, ks, tile_prefix, count);
            break;
        case kC32x2:
            hipLaunchKernelGGL((forward_batch<kC32x2, H32>), dim3(grid), dim3(kBlock), 0, s, ks, tile_prefix, count);
            break;
        default:
            hipLaunchKernelGGL((forward_batch<kF64, H32>), dim3(grid), dim3(kBlock), 0, s, ks, tile_prefix, count);
            break;
    }
    return hipGetLastError();
}

hipError_t launch_forward_batch(const FwdK *ks, const int64_t *tile_prefix, int count, int prec,
                                bool h32, unsigned grid, hipStream_t s) {
    return h32 ? launch_fwd_batch<true>(ks, tile_prefix, count, prec, grid, s)
               : launch_fwd_batch<false>(ks, tile_prefix, count, prec, grid, s);
}

void comb_params(int H, int rows, const int *ry, int n_scales, int *p4, int *teeth) {
    const int groups = (H + rows - 1) / rows;
    int rmin = ry[0];
    for (int j = 1; j < n_scales; ++j) rmin = ry[j] < rmin ? ry[j] : rmin;
    const int p = (2 * rmin + 1 + rows / 2) / rows;
    if (p >= 4 && p < groups) {
        *p4 = p;
        *teeth = (groups + p - 1) / p;
    } else {
        *p4 = groups;
        *teeth = 1;
    }
}

FwdK make_fwdk(const float *v, int64_t ld_v, int H, int W, const void *sat, int64_t ld_sat,
                const float *offsets, const uint32_t *hist, int64_t ld_hist,
                int64_t plane_stride, const float *edges, const QueryParams &p, float *out,
                int64_t ld_out) {
    FwdK k;
    k.v = v;
    k.ld_v = ld_v;
    k.H = H;
    k.W = W;
    k.sat = sat;
    k.ld_sat = ld_sat;
    k.offsets = offsets;
    k.hist = hist;
    k.ld_hist = ld_hist;
    k.plane_stride = plane_stride;
    k.edges = edges;
    k.p = p;
    k.out = out;
    k.ld_out = ld_out;
    k.tiles_x = (W + kWave - 1) / kWave;
    k.resid = nullptr;
    k.rstride = 0;
    k.rgb = nullptr;
    k.rgb_cs = k.rgb_ld = 0;
    k.rgb_out = nullptr;
    k.out_cs = k.out_ld = 0;
    k.saturation = 0.f;
    k.maps = nullptr;
    k.mstride = 0;
    comb_params(H, kRows, p.ry, p.n_scales, &k.p4, &k.teeth);
    return k;
}

template <bool RESID, bool H32>
hipError_t launch_fwd(const FwdK &k, int prec, hipStream_t s) {
    const unsigned tiles = (unsigned)query_blocks(k);
    switch (prec) {
        case kF32:
            hipLaunchKernelGGL((forward_kernel<kF32, RESID, H32>), dim3(tiles), dim3(kBlock), 0, s, k);
            break;
        case kC32x2:
            hipLaunchKernelGGL((forward_kernel<kC32x2, RESID, H32>), dim3(tiles), dim3(kBlock), 0, s, k);
            break;
        default:
            hipLaunchKernelGGL((forward_kernel<kF64, RESID, H32>), dim3(tiles), dim3(kBlock), 0, s, k);
            break;
    }
    return hipGetLastError();
}

// Largest histogram byte offset a lane forms relative to entry (-1, -1) of plane 0.
bool hist_offsets_fit_32(const FwdK &k) {
    if (!k.hist || k.p.n_bins < 2) return true;
    const int64_t last = (int64_t)(k.p.n_bins - 2) * k.plane_stride + (int64_t)k.W + 1;
    return last * 4 < ((int64_t)1 << 32);
}

hipError_t launch_forward_maps(const float *v, int64_t ld_v, int H, int W, const void *sat,
                               int64_t ld_sat, int prec, const float *offsets,
                               const uint32_t *hist, int64_t ld_hist, int64_t plane_stride,
                               const float *edges, const QueryParams &p, float *out,
                               int64_t ld_out, float *maps, hipStream_t s) {
    FwdK k = make_fwdk(v, ld_v, H, W, sat, ld_sat, offsets, hist, ld_hist, plane_stride, edges,
                       p, out, ld_out);
    k.maps = maps;
    k.mstride = (int64_t)H * W;
    return hist_offsets_fit_32(k) ? launch_fwd<false, true>(k, prec, s)
                                  : launch_fwd<false, false>(k, prec, s);
}

hipError_t launch_forward_rgb(const float *v, int64_t ld_v, int H, int W, const void *sat_tab,
                              int64_t ld_sat, int prec, const float *offsets,
                              const uint32_t *hist, int64_t ld_hist, int64_t plane_stride,
                              const float *edges, const QueryParams &p, float *out,
                              int64_t ld_out, const float *rgb, int64_t rgb_cs, int64_t rgb_ld,
                              float *rgb_out, int64_t out_cs, int64_t out_ld, float sat,
                              hipStream_t s) {
    FwdK k = make_fwdk(v, ld_v, H, W, sat_tab, ld_sat, offsets, hist, ld_hist, plane_stride,
                       edges, p, out, ld_out);
    k.rgb = rgb;
    k.rgb_cs = rgb_cs;
    k.rgb_ld = rgb_ld;
    k.rgb_out = rgb_out;
    k.out_cs = out_cs;
    k.out_ld = out_ld;
    k.saturation = sat;
    return hist_offsets_fit_32(k) ? launch_fwd<false, true>(k, prec, s)
                                  : launch_fwd<false, false>(k, prec, s);
}

hipError_t launch_forward(const float *v, int64_t ld_v, int H, int W, const void *sat,
                          int64_t ld_sat, int prec, const float *offsets, const uint32_t *hist,
                          int64_t ld_hist, int64_t plane_stride, const float *edges,
                          const QueryParams &p, float *out, int64_t ld_out, float *resid,
                          hipStream_t s) {
    FwdK k = make_fwdk(v, ld_v, H, W, sat, ld_sat, offsets, hist, ld_hist, plane_stride, edges,
                       p, out, ld_out);
    k.resid = resid;
    k.rstride = (int64_t)H * W;
    if (hist_offsets_fit_32(k))
        return resid ? launch_fwd<true, true>(k, prec, s) : launch_fwd<false, true>(k, prec, s);
    return resid ? launch_fwd<true, false>(k, prec, s) : launch_fwd<false, false>(k, prec, s);
}

}  // namespace tmo
