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


// Window mean m and variance var (Eq. 10 read as the population variance, not yet clamped)
// from the four corner entries of the interleaved integral image and the reciprocal of the
// window area.  The corner sums cancel heavily (large quadrant sums, small window sums), so
// for the compensated and FP64 tables they are combined in FP64.
template <int P>
__device__ __forceinline__ void window_moments(const FwdK &k, int64_t oA, int64_t oB,
                                               int64_t oC, int64_t oD, double inv_n, float mu1,
                                               float mu2, double &m, double &var) {
    if constexpr (P == kF32) {
        const float2 *t = static_cast<const float2 *>(k.sat);
        const float2 A = t[oA], B = t[oB], C = t[oC], D = t[oD];
        const float inv = (float)inv_n;
        const float mf = ((A.x + C.x) - (B.x + D.x)) * inv;
        const float vf = __builtin_fmaf((A.y + C.y) - (B.y + D.y), inv, -(mf * mf));
        m = (double)mf;
        var = (double)vf;
    } else if constexpr (P == kC32x2) {
        const float4 *t = static_cast<const float4 *>(k.sat);
        const float4 A = t[oA], B = t[oB], C = t[oC], D = t[oD];
        // leading parts exactly in FP64; trailing parts (2^-24 smaller) summed in FP32
        const double h1 = ((double)A.x + (double)C.x) - ((double)B.x + (double)D.x);
        const double h2 = ((double)A.z + (double)C.z) - ((double)B.z + (double)D.z);
        const float l1 = (A.y + C.y) - (B.y + D.y);
        const float l2 = (A.w + C.w) - (B.w + D.w);
        m = __builtin_fma(h1 + (double)l1, inv_n, (double)mu1);
        const double e2 = __builtin_fma(h2 + (double)l2, inv_n, (double)mu2);
        var = __builtin_fma(-m, m, e2);
    } else {
        const double2 *t = static_cast<const double2 *>(k.sat);
        const double2 A = t[oA], B = t[oB], C = t[oC], D = t[oD];
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
// RESID: also write the per-pixel residual planes the backward needs (their derivation is
// in the backward's header): R1_j = -2 c_j m_j / N_j and R2_j = c_j / N_j with
// c_j = (L_j - L)/D eps/(var_j + eps)^2 (zero where var_j was clamped or D = 0),
// E = sum_j (L_j - L)/D (-var_j/(var_j + eps)^2) and Pbar = sum_j W_j P_j / D.
template <int P, bool RESID>
__device__ __forceinline__ void forward_tile(const FwdK &k, uint32_t tile, float *sh_edges) {
    const int ne = k.p.n_bins - 1;
    __syncthreads();   // the previous tile of this block may still read sh_edges
    for (int i = threadIdx.x; i < ne; i += kBlock) sh_edges[i] = k.edges[i];
    __syncthreads();

    int tx, rg;
    comb_map(tile, k.tiles_x, k.p4, k.teeth, tx, rg);
    const int x = tx * kWave + lane_id();
    const int y = rg * kRows + (int)(threadIdx.x / kWave);
    if (x >= k.W || y >= k.H) return;

    const float v = k.v[(int64_t)y * k.ld_v + x];
    // bin b = #{edges <= v} (edges ascending)
    int lo = 0, hi = ne;
    while (lo < hi) {
        const int mid = (lo + hi) >> 1;
        if (sh_edges[mid] <= v) lo = mid + 1; else hi = mid;
    }
    const int b = lo;
    const uint32_t *plane = b > 0 ? k.hist + (int64_t)(b - 1) * k.plane_stride : nullptr;

    const int s = k.p.n_scales;
    const float ldr = k.p.ld_max - k.p.ld_min;
    const float mu1 = P == kC32x2 ? k.offsets[0] : 0.f;
    const float mu2 = P == kC32x2 ? k.offsets[1] : 0.f;
    float num = 0.f, den = 0.f, lsum = 0.f, pn = 0.f, psum = 0.f;
    float vj[kMaxS], mj[kMaxS], lj[kMaxS], nj[kMaxS];
    bool clj[kMaxS];
#pragma unroll
    for (int j = 0; j < kMaxS; ++j) {
        if (j < s) {
            const int rx = k.p.rx[j], ry = k.p.ry[j];
            const int xm = max(x - rx - 1, -1), xp = min(x + rx, k.W - 1);
            const int ym = max(y - ry - 1, -1), yp = min(y + ry, k.H - 1);
            const int N = (xp - xm) * (yp - ym);
            const double inv_n = recip_area(N);
            double m, vr;
            window_moments<P>(k, (int64_t)ym * k.ld_sat + xm, (int64_t)ym * k.ld_sat + xp,
                              (int64_t)yp * k.ld_sat + xp, (int64_t)yp * k.ld_sat + xm, inv_n,
                              mu1, mu2, m, vr);
            // a one-pixel window has zero variance by definition (its rounding noise would
            // otherwise reach the gradient through the clamp)
            const bool clamped = !(vr > 0.0) || N == 1;
            const float var = clamped ? 0.f : (float)vr;
            uint32_t c = 0u;
            if (plane) {
                c = plane[(int64_t)yp * k.ld_hist + xp] + plane[(int64_t)ym * k.ld_hist + xm] -
                    plane[(int64_t)ym * k.ld_hist + xp] - plane[(int64_t)yp * k.ld_hist + xm];
            }
            const float Pj = (float)c * (float)inv_n;
            const float Lj = __builtin_fmaf(ldr, Pj, k.p.ld_min);
            const float Wj = var * __builtin_amdgcn_rcpf(var + k.p.eps);
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
    const int64_t pix = (int64_t)y * k.ld_out + x;
    if (k.out) k.out[pix] = L;
    if (RESID) {
        const int64_t o = (int64_t)y * k.W + x, ps = k.rstride;
        const float inv_d = den > 0.f ? 1.0f / den : 0.f;
        float E = 0.f;
#pragma unroll
        for (int j = 0; j < kMaxS; ++j) {
            if (j < s) {
                const float d = (lj[j] - L) * inv_d;
                const float r = __builtin_amdgcn_rcpf(vj[j] + k.p.eps);
                const float r2 = r * r;
                E = __builtin_fmaf(d, -vj[j] * r2, E);
                const float c = clj[j] ? 0.f : d * k.p.eps * r2;
                const float cn = c * nj[j];
                k.resid[(int64_t)j * ps + o] = -2.0f * cn * mj[j];
                k.resid[(int64_t)(s + j) * ps + o] = cn;
            }
        }
        k.resid[(int64_t)(2 * s) * ps + o] = E;
        k.resid[(int64_t)(2 * s + 1) * ps + o] = den > 0.f ? pn / den : psum / (float)s;
    }
}

template <int P, bool RESID>
__global__ void __launch_bounds__(kBlock) forward_kernel(FwdK k) {
    __shared__ float sh_edges[256];
    forward_tile<P, RESID>(k, xcd_tile(blockIdx.x, gridDim.x), sh_edges);
}

// Batched query: a persistent grid whose blocks on XCD x (block % 8) walk the x-th eighth of
// the flattened tile list, so each XCD's L2 sees one contiguous run of tiles.
template <int P>
__global__ void __launch_bounds__(kBlock) forward_batch(const FwdK *ks, const int64_t *prefix,
                                                       int count) {
    __shared__ float sh_edges[256];
    const int64_t total = prefix[count];
    const int64_t per = (total + 7) / 8;
    const int64_t xcd = blockIdx.x % 8, nb = gridDim.x / 8;
    const int64_t end = min(total, (xcd + 1) * per);
    for (int64_t g = xcd * per + blockIdx.x / 8; g < end; g += nb) {
        const int i = find_image(prefix, count, g);
        forward_tile<P, false>(ks[i], (uint32_t)(g - prefix[i]), sh_edges);
    }
}

}  // namespace

int64_t query_blocks(const FwdK &k) { return (int64_t)k.tiles_x * k.p4 * k.teeth; }

hipError_t launch_forward_batch(const FwdK *ks, const int64_t *tile_prefix, int count, int prec,
                                unsigned grid, hipStream_t s) {
    switch (prec) {
        case kF32:
            hipLaunchKernelGGL(forward_batch<kF32>, dim3(grid), dim3(kBlock), 0, s, ks, tile_prefix, count);
            break;
        case kC32x2:
            hipLaunchKernelGGL(forward_batch<kC32x2>, dim3(grid), dim3(kBlock), 0, s, ks, tile_prefix, count);
            break;
        default:
            hipLaunchKernelGGL(forward_batch<kF64>, dim3(grid), dim3(kBlock), 0, s, ks, tile_prefix, count);
            break;
    }
    return hipGetLastError();
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
    comb_params(H, kRows, p.ry, p.n_scales, &k.p4, &k.teeth);
    return k;
}

template <bool RESID>
hipError_t launch_fwd(const FwdK &k, int prec, hipStream_t s) {
    const unsigned tiles = (unsigned)query_blocks(k);
    switch (prec) {
        case kF32:
            hipLaunchKernelGGL((forward_kernel<kF32, RESID>), dim3(tiles), dim3(kBlock), 0, s, k);
            break;
        case kC32x2:
            hipLaunchKernelGGL((forward_kernel<kC32x2, RESID>), dim3(tiles), dim3(kBlock), 0, s, k);
            break;
        default:
            hipLaunchKernelGGL((forward_kernel<kF64, RESID>), dim3(tiles), dim3(kBlock), 0, s, k);
            break;
    }
    return hipGetLastError();
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
    return resid ? launch_fwd<true>(k, prec, s) : launch_fwd<false>(k, prec, s);
}

}  // namespace tmo
