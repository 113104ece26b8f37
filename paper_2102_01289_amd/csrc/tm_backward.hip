// tm_backward.hip -- stage a5: the adjoint of the fused forward with respect to the
// luminance v and the scalars (eps, min L_d, max L_d).
//
// The bin counts are piecewise constant in v and the bin edges are held fixed, so v reaches
// L only through the window variances var_j = S2_j/N_j - (S1_j/N_j)^2 (Eq. 10).  With
// D = sum_j W_j and a_j = g (L_j - L)/D * eps/(var_j + eps)^2 (Eq. 3, Eq. 4; zero where var_j
// was clamped or D = 0) the gradient is
//   dv(q) = sum_j sum_{p : q in w_j(p)} ( A1_j(p) + 2 v(q) A2_j(p) ),
//   A1_j = -2 a_j S1_j / N_j^2,   A2_j = a_j / N_j.
// Each window sum is four corner reads of an integral image (Eq. 6), so its adjoint deposits
// +-A at those four corners and the integral image's adjoint is a suffix sum:
//   dv = suffix2D(D1) + 2 v suffix2D(D2),   D = sum_j sum_corners +-A_j.
// Kernels: (1) per-pixel coefficients A1_j, A2_j and block partials of the scalar
// gradients; (2) the deposits that clamping piles onto the last column / row, as row and
// column range sums; (3) the deposit gather D1, D2, written in reversed pixel order so that
// (4) the ordinary three-stage prefix scan, run in adjoint mode, yields the suffix sums and
// writes dv; (5) a fixed-order reduction of the scalar partials.  No atomics anywhere, so
// every result is bit-reproducible.
#include "tm_device.h"
#include "tm_internal.h"

namespace tmo {

namespace {

constexpr int kBlock = 256;
constexpr int kRows = kBlock / kWave;
constexpr int kS = 8;   // TM_MAX_SCALES

struct BwdK {
    const float *v;
    int64_t ld_v;
    int H, W;
    const void *sat;
    int64_t ld_sat;
    const float *offsets;
    const uint32_t *hist;
    int64_t ld_hist, plane_stride;
    const float *edges;
    QueryParams p;
    const float *g;
    int64_t ld_g;
    double *A;       // [2][s][H][W]: A1_j then A2_j
    double *Rb;      // [2][s][H]  row range sums
    double *Cb;      // [2][s][W]  column range sums
    double2 *Dr;     // [H][W] deposits {D1, D2} in reversed order
    double *part;    // [nblocks][3] scalar partials
    int tiles_x;
};

__device__ __forceinline__ int64_t plane_off(const BwdK &k, int q, int j) {
    return ((int64_t)q * k.p.n_scales + j) * (int64_t)k.H * k.W;
}

// Window sums S1, S2 from the four corners of the interleaved integral image.
template <int P>
__device__ __forceinline__ void box_sums(const BwdK &k, int64_t oA, int64_t oB, int64_t oC,
                                         int64_t oD, double dN, double &s1, double &s2) {
    if constexpr (P == kF32) {
        const float2 *t = static_cast<const float2 *>(k.sat);
        const float2 A = t[oA], B = t[oB], C = t[oC], D = t[oD];
        s1 = (double)((A.x + C.x) - (B.x + D.x));
        s2 = (double)((A.y + C.y) - (B.y + D.y));
    } else if constexpr (P == kC32x2) {
        const float4 *t = static_cast<const float4 *>(k.sat);
        const float4 A = t[oA], B = t[oB], C = t[oC], D = t[oD];
        const double h1 = ((double)A.x + (double)C.x) - ((double)B.x + (double)D.x);
        const double l1 = ((double)A.y + (double)C.y) - ((double)B.y + (double)D.y);
        const double h2 = ((double)A.z + (double)C.z) - ((double)B.z + (double)D.z);
        const double l2 = ((double)A.w + (double)C.w) - ((double)B.w + (double)D.w);
        s1 = (h1 + l1) + dN * (double)k.offsets[0];
        s2 = (h2 + l2) + dN * (double)k.offsets[1];
    } else {
        const double2 *t = static_cast<const double2 *>(k.sat);
        const double2 A = t[oA], B = t[oB], C = t[oC], D = t[oD];
        s1 = (A.x + C.x) - (B.x + D.x);
        s2 = (A.y + C.y) - (B.y + D.y);
    }
}

struct Sum3 {
    double a, b, c;
};

__device__ Sum3 block_sum3(Sum3 v) {
    for (int m = 32; m >= 1; m >>= 1) {
        v.a += __shfl_xor(v.a, m);
        v.b += __shfl_xor(v.b, m);
        v.c += __shfl_xor(v.c, m);
    }
    __shared__ Sum3 sh[kRows];
    if (lane_id() == 0) sh[threadIdx.x / kWave] = v;
    __syncthreads();
    Sum3 r = sh[0];
    for (int i = 1; i < kRows; ++i) {
        r.a += sh[i].a;
        r.b += sh[i].b;
        r.c += sh[i].c;
    }
    return r;
}

// (1) per-pixel adjoint coefficients
template <int P>
__global__ void __launch_bounds__(kBlock) adjoint_kernel(BwdK k) {
    __shared__ float sh_edges[256];
    const int ne = k.p.n_bins - 1;
    for (int i = threadIdx.x; i < ne; i += kBlock) sh_edges[i] = k.edges[i];
    __syncthreads();

    const int tx = (int)(blockIdx.x % (uint32_t)k.tiles_x), ty = (int)(blockIdx.x / (uint32_t)k.tiles_x);
    const int x = tx * kWave + lane_id();
    const int y = ty * kRows + (int)(threadIdx.x / kWave);
    const bool in = x < k.W && y < k.H;
    Sum3 acc{0.0, 0.0, 0.0};
    if (in) {
        const float v = k.v[(int64_t)y * k.ld_v + x];
        int lo = 0, hi = ne;
        while (lo < hi) {
            const int mid = (lo + hi) >> 1;
            if (sh_edges[mid] <= v) lo = mid + 1; else hi = mid;
        }
        const uint32_t *plane = lo > 0 ? k.hist + (int64_t)(lo - 1) * k.plane_stride : nullptr;
        const int s = k.p.n_scales;
        const double eps = (double)k.p.eps, lmin = (double)k.p.ld_min;
        const double ldr = (double)k.p.ld_max - lmin;
        double Lj[kS], Wj[kS], var[kS], m[kS], Nj[kS], Pj[kS];
        bool clamped[kS];
        double num = 0.0, den = 0.0, pn = 0.0, lsum = 0.0, psum = 0.0;
#pragma unroll
        for (int j = 0; j < kS; ++j) {
            if (j < s) {
                const int rx = k.p.rx[j], ry = k.p.ry[j];
                const int xm = max(x - rx - 1, -1), xp = min(x + rx, k.W - 1);
                const int ym = max(y - ry - 1, -1), yp = min(y + ry, k.H - 1);
                const int N = (xp - xm) * (yp - ym);
                const double dN = (double)N;
                double s1, s2;
                box_sums<P>(k, (int64_t)ym * k.ld_sat + xm, (int64_t)ym * k.ld_sat + xp,
                            (int64_t)yp * k.ld_sat + xp, (int64_t)yp * k.ld_sat + xm, dN, s1, s2);
                uint32_t c = 0u;
                if (plane)
                    c = plane[(int64_t)yp * k.ld_hist + xp] + plane[(int64_t)ym * k.ld_hist + xm] -
                        plane[(int64_t)ym * k.ld_hist + xp] - plane[(int64_t)yp * k.ld_hist + xm];
                m[j] = s1 / dN;
                const double vr = s2 / dN - m[j] * m[j];
                clamped[j] = !(vr > 0.0);
                var[j] = clamped[j] ? 0.0 : vr;
                Nj[j] = dN;
                Pj[j] = (double)c / dN;
                Lj[j] = lmin + ldr * Pj[j];
                Wj[j] = var[j] / (var[j] + eps);
                num += Wj[j] * Lj[j];
                pn += Wj[j] * Pj[j];
                den += Wj[j];
                lsum += Lj[j];
                psum += Pj[j];
            }
        }
        const double L = den > 0.0 ? num / den : lsum / s;
        const double Pbar = den > 0.0 ? pn / den : psum / s;
        const double gp = (double)k.g[(int64_t)y * k.ld_g + x];
        const int64_t pix = (int64_t)y * k.W + x;
#pragma unroll
        for (int j = 0; j < kS; ++j) {
            if (j < s) {
                double a = 0.0;
                if (den > 0.0) {
                    const double dLdW = (Lj[j] - L) / den;
                    const double dd = var[j] + eps;
                    acc.a += gp * dLdW * (-var[j] / (dd * dd));
                    if (!clamped[j]) a = gp * dLdW * eps / (dd * dd);
                }
                k.A[plane_off(k, 0, j) + pix] = -2.0 * a * m[j] / Nj[j];
                k.A[plane_off(k, 1, j) + pix] = a / Nj[j];
            }
        }
        acc.b = gp * (1.0 - Pbar);
        acc.c = gp * Pbar;
    }
    const Sum3 r = block_sum3(acc);
    if (threadIdx.x == 0) {
        k.part[3 * (int64_t)blockIdx.x + 0] = r.a;
        k.part[3 * (int64_t)blockIdx.x + 1] = r.b;
        k.part[3 * (int64_t)blockIdx.x + 2] = r.c;
    }
}

// (2) clamped-corner aggregates.  Blocks [0, nrow) compute Rb[q][j][y] = sum of A_qj over
// the columns whose window reaches the last column (x >= W-1-rx_j), one wave per row;
// the remaining blocks compute Cb[q][j][x] = sum over the rows y >= H-1-ry_j, 64 columns per
// block with the row range split over the 4 waves and combined in a fixed order.
__global__ void __launch_bounds__(kBlock) border_kernel(BwdK k, int nrow_blocks) {
    const int s = k.p.n_scales;
    if ((int)blockIdx.x < nrow_blocks) {
        const int64_t item = (int64_t)blockIdx.x * kRows + threadIdx.x / kWave;
        if (item >= (int64_t)2 * s * k.H) return;
        const int q = (int)(item / ((int64_t)s * k.H));
        const int j = (int)((item / k.H) % s);
        const int y = (int)(item % k.H);
        const int x0 = max(k.W - 1 - k.p.rx[j], 0);
        const double *row = k.A + plane_off(k, q, j) + (int64_t)y * k.W;
        double acc = 0.0;
        for (int x = x0 + lane_id(); x < k.W; x += kWave) acc += row[x];
        acc = wave_sum<Acc<kF64>>(acc);
        if (lane_id() == 0) k.Rb[((int64_t)q * s + j) * k.H + y] = acc;
        return;
    }
    __shared__ double sh[kRows][kWave];
    const int cb = (int)blockIdx.x - nrow_blocks;
    const int ncol_tiles = (k.W + kWave - 1) / kWave;
    const int q = cb / (s * ncol_tiles);
    const int j = (cb / ncol_tiles) % s;
    const int x = (cb % ncol_tiles) * kWave + lane_id();
    const int w = threadIdx.x / kWave;
    const int y0 = max(k.H - 1 - k.p.ry[j], 0);
    double acc = 0.0;
    if (x < k.W) {
        const double *col = k.A + plane_off(k, q, j) + x;
        for (int y = y0 + w; y < k.H; y += kRows) acc += col[(int64_t)y * k.W];
    }
    sh[w][lane_id()] = acc;
    __syncthreads();
    if (w == 0 && x < k.W) {
        double r = sh[0][lane_id()];
        for (int i = 1; i < kRows; ++i) r += sh[i][lane_id()];
        k.Cb[((int64_t)q * s + j) * k.W + x] = r;
    }
}

// (3) deposits.  Virtual pixel (x', y') holds the deposit at corner c = (W-1-x', H-1-y').
// For field j the corners that equal c come from at most one pixel per corner type,
// except where clamping maps a whole range of pixels onto the last column / row; those
// ranges use Rb, Cb and (for the bottom-right corner) their total K, which the first block
// forms cooperatively before use.
__global__ void __launch_bounds__(kBlock) deposit_kernel(BwdK k) {
    const int s = k.p.n_scales;
    __shared__ double shK[2][kS];
    if (blockIdx.x == 0) {
        __shared__ double shp[kRows][2 * kS];
        const int w = threadIdx.x / kWave;
        for (int qj = 0; qj < 2 * s; ++qj) {
            const int q = qj / s, j = qj % s;
            const int y0 = max(k.H - 1 - k.p.ry[j], 0);
            double acc = 0.0;
            for (int y = y0 + (int)threadIdx.x; y < k.H; y += kBlock)
                acc += k.Rb[((int64_t)q * s + j) * k.H + y];
            acc = wave_sum<Acc<kF64>>(acc);
            if (lane_id() == 0) shp[w][qj] = acc;
        }
        __syncthreads();
        if (threadIdx.x < 2 * s) {
            double r = shp[0][threadIdx.x];
            for (int i = 1; i < kRows; ++i) r += shp[i][threadIdx.x];
            shK[threadIdx.x / s][threadIdx.x % s] = r;
        }
        __syncthreads();
    }
    const int tiles_x = k.tiles_x;
    const int xv = (int)(blockIdx.x % (uint32_t)tiles_x) * kWave + lane_id();
    const int yv = (int)(blockIdx.x / (uint32_t)tiles_x) * kRows + (int)(threadIdx.x / kWave);
    if (xv >= k.W || yv >= k.H) return;
    const int cx = k.W - 1 - xv, cy = k.H - 1 - yv;
    const bool lastx = cx == k.W - 1, lasty = cy == k.H - 1;
    double d[2] = {0.0, 0.0};
    for (int j = 0; j < s; ++j) {
        const int rx = k.p.rx[j], ry = k.p.ry[j];
        const int pxp = cx - rx;            // pixel whose x+ corner is cx (cx < W-1)
        const int pxm = cx + rx + 1;        // pixel whose x- corner is cx
        const int pyp = cy - ry;
        const int pym = cy + ry + 1;
        const bool vxm = pxm <= k.W - 1, vym = pym <= k.H - 1;
#pragma unroll
        for (int q = 0; q < 2; ++q) {
            const double *A = k.A + plane_off(k, q, j);
            const double *R = k.Rb + ((int64_t)q * s + j) * k.H;
            const double *C = k.Cb + ((int64_t)q * s + j) * k.W;
            auto at = [&](int px, int py) { return A[(int64_t)py * k.W + px]; };
            double t = 0.0;
            // (x+, y+) corner
            if (!lastx && !lasty) {
                if (pxp >= 0 && pyp >= 0) t += at(pxp, pyp);
            } else if (lastx && !lasty) {
                if (pyp >= 0) t += R[pyp];
            } else if (!lastx && lasty) {
                if (pxp >= 0) t += C[pxp];
            } else {
                t += shK[q][j];
            }
            // (x-, y+) corner, sign -
            if (vxm) {
                if (!lasty) {
                    if (pyp >= 0) t -= at(pxm, pyp);
                } else {
                    t -= C[pxm];
                }
            }
            // (x+, y-) corner, sign -
            if (vym) {
                if (!lastx) {
                    if (pxp >= 0) t -= at(pxp, pym);
                } else {
                    t -= R[pym];
                }
            }
            // (x-, y-) corner
            if (vxm && vym) t += at(pxm, pym);
            d[q] += t;
        }
    }
    k.Dr[(int64_t)yv * k.W + xv] = make_double2(d[0], d[1]);
}

// (5) scalar gradients: fixed-order reduction of the per-block partials.
__global__ void __launch_bounds__(kBlock) scalar_finalize_kernel(const double *part, int nparts,
                                                                 double *out) {
    Sum3 acc{0.0, 0.0, 0.0};
    for (int i = threadIdx.x; i < nparts; i += kBlock) {
        acc.a += part[3 * (int64_t)i];
        acc.b += part[3 * (int64_t)i + 1];
        acc.c += part[3 * (int64_t)i + 2];
    }
    const Sum3 r = block_sum3(acc);
    if (threadIdx.x == 0) {
        out[0] = r.a;
        out[1] = r.b;
        out[2] = r.c;
    }
}

size_t round_up(size_t a, size_t b) { return (a + b - 1) / b * b; }

}  // namespace

BwdPlan make_bwd_plan(int H, int W, int n_scales) {
    BwdPlan b{};
    const int tiles_x = (W + kWave - 1) / kWave;
    b.nblocks = (int64_t)tiles_x * ((H + kRows - 1) / kRows);
    size_t off = 0;
    auto take = [&](size_t bytes) {
        size_t o = off;
        off = round_up(off + bytes, 256);
        return o;
    };
    const size_t hw = (size_t)H * W;
    b.A = take(2 * (size_t)n_scales * hw * sizeof(double));
    b.Rb = take(2 * (size_t)n_scales * H * sizeof(double));
    b.Cb = take(2 * (size_t)n_scales * W * sizeof(double));
    b.Dr = take(hw * sizeof(double2));
    b.part = take((size_t)b.nblocks * 3 * sizeof(double));
    b.scan_plan = make_scan_plan(H, W, kF64, 0, scan_tune_default(H, W));
    b.scan = take(b.scan_plan.total);
    b.total = off;
    return b;
}

hipError_t launch_backward(const BwdArgs &a, const BwdPlan &plan, void *ws, hipStream_t s) {
    char *w = static_cast<char *>(ws);
    BwdK k;
    k.v = a.v;
    k.ld_v = a.ld_v;
    k.H = a.H;
    k.W = a.W;
    k.sat = a.sat;
    k.ld_sat = a.ld_sat;
    k.offsets = a.offsets;
    k.hist = a.hist;
    k.ld_hist = a.ld_hist;
    k.plane_stride = a.plane_stride;
    k.edges = a.edges;
    k.p = a.p;
    k.g = a.g;
    k.ld_g = a.ld_g;
    k.A = reinterpret_cast<double *>(w + plan.A);
    k.Rb = reinterpret_cast<double *>(w + plan.Rb);
    k.Cb = reinterpret_cast<double *>(w + plan.Cb);
    k.Dr = reinterpret_cast<double2 *>(w + plan.Dr);
    k.part = reinterpret_cast<double *>(w + plan.part);
    k.tiles_x = (a.W + kWave - 1) / kWave;
    const unsigned nb = (unsigned)plan.nblocks;
    switch (a.prec) {
        case kF32: hipLaunchKernelGGL(adjoint_kernel<kF32>, dim3(nb), dim3(kBlock), 0, s, k); break;
        case kC32x2: hipLaunchKernelGGL(adjoint_kernel<kC32x2>, dim3(nb), dim3(kBlock), 0, s, k); break;
        default: hipLaunchKernelGGL(adjoint_kernel<kF64>, dim3(nb), dim3(kBlock), 0, s, k); break;
    }
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    const int S = a.p.n_scales;
    const int nrow = (int)(((int64_t)2 * S * a.H + kRows - 1) / kRows);
    const int ncol = 2 * S * ((a.W + kWave - 1) / kWave);
    hipLaunchKernelGGL(border_kernel, dim3(nrow + ncol), dim3(kBlock), 0, s, k, nrow);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    hipLaunchKernelGGL(deposit_kernel, dim3(nb), dim3(kBlock), 0, s, k);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    e = launch_suffix_adjoint(k.Dr, a.W, a.v, a.ld_v, a.H, a.W, a.grad_v, a.ld_gv,
                              plan.scan_plan, w + plan.scan, s);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(scalar_finalize_kernel, dim3(1), dim3(kBlock), 0, s, k.part, (int)nb,
                       a.grad_params);
    return hipGetLastError();
}

}  // namespace tmo
