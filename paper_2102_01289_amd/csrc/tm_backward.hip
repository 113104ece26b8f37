// tm_backward.hip -- stage a5: the adjoint of the fused forward with respect to the
// luminance v and the scalars (eps, min L_d, max L_d).
//
// The bin counts are piecewise constant in v and the bin edges are held fixed, so v reaches
// L only through the window variances var_j = S2_j/N_j - (S1_j/N_j)^2 (Eq. 10).  With
// D = sum_j W_j and c_j = (L_j - L)/D * eps/(var_j + eps)^2 (Eq. 3, Eq. 4; zero where var_j
// was clamped or D = 0) the gradient of sum_p g(p) L(p) is
//   dv(q) = sum_j sum_{p : q in w_j(p)} g(p) ( R1_j(p) + 2 v(q) R2_j(p) ),
//   R1_j = -2 c_j S1_j / N_j^2,   R2_j = c_j / N_j,
// and d/d eps = sum_p g E, d/d min L_d = sum_p g (1 - Pbar), d/d max L_d = sum_p g Pbar with
// E = sum_j (L_j - L)/D (-var_j/(var_j + eps)^2) and Pbar = sum_j W_j P_j / D.  None of
// R1, R2, E, Pbar depends on g: the training forward writes them as FP32 "residual" planes
// (or the table-based entry point rebuilds them from the tables), and the backward reads no
// table at all.
// Each window sum is four corner reads of an integral image (Eq. 6), so its adjoint deposits
// +-g R at those four corners and the integral image's adjoint is a suffix sum:
//   dv = suffix2D(D1) + 2 v suffix2D(D2),   D = sum_j sum_corners +-g R_j.
// Kernels: (1) the deposits that clamping piles onto the last column / row, as row sums and
// (two-level) column sums; (2) the deposit gather D1, D2 (FP64, comb block order), written in
// reversed pixel order so that (3) the ordinary three-stage prefix scan, run in adjoint
// mode, yields the suffix sums and writes dv; (4) a streaming two-level fixed-order reduction
// of the scalar gradients.  No atomics anywhere, so every result is bit-reproducible.
#include "tm_device.h"
#include "tm_internal.h"

namespace tmo {

namespace {

constexpr int kBlock = 256;
constexpr int kRows = kBlock / kWave;
constexpr int kS = 8;            // TM_MAX_SCALES
constexpr int kChunk = 64;       // rows per partial of the column sums
constexpr int kScalarBlocks = 1024;

struct BwdK {
    const float *v;
    int64_t ld_v;
    int H, W;
    QueryParams p;
    const float *g;
    int64_t ld_g;
    const float *R;  // residual planes: R1_j at j, R2_j at s + j, E at 2s, Pbar at 2s + 1
    double *Rb;      // [2][s][H]  row range sums of g R
    double *Cp;      // [2][s][nchunks][W] partial column range sums
    double *Cb;      // [2][s][W]  column range sums
    double2 *Dr;     // [H][W] deposits {D1, D2} in reversed order
    double *part;    // [kScalarBlocks][3] scalar partials
    int tiles_x, p4, teeth, nchunks;
};

__device__ __forceinline__ const float *rplane(const BwdK &k, int q, int j) {
    return k.R + ((int64_t)q * k.p.n_scales + j) * (int64_t)k.H * k.W;
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
    __syncthreads();
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

// (1a) Rb[q][j][y] = sum over x >= W-1-rx_j of g R_qj at (x, y): one block per row, every
// field and both planes in one pass, combined in a fixed order.
__global__ void __launch_bounds__(kBlock) border_rows_kernel(BwdK k) {
    const int s = k.p.n_scales, y = blockIdx.x;
    int lo[kS], x0 = k.W;
    double acc[2][kS];
#pragma unroll
    for (int j = 0; j < kS; ++j) {
        acc[0][j] = acc[1][j] = 0.0;
        lo[j] = j < s ? max(k.W - 1 - k.p.rx[j], 0) : k.W;
        x0 = min(x0, lo[j]);
    }
    const int64_t row = (int64_t)y * k.W;
    for (int x = x0 + (int)threadIdx.x; x < k.W; x += kBlock) {
        const double gx = (double)k.g[(int64_t)y * k.ld_g + x];
#pragma unroll
        for (int j = 0; j < kS; ++j) {
            if (j < s && x >= lo[j]) {
                acc[0][j] = __builtin_fma(gx, (double)rplane(k, 0, j)[row + x], acc[0][j]);
                acc[1][j] = __builtin_fma(gx, (double)rplane(k, 1, j)[row + x], acc[1][j]);
            }
        }
    }
    __shared__ double sh[kRows][2 * kS];
#pragma unroll
    for (int j = 0; j < kS; ++j)
        for (int m = 32; m >= 1; m >>= 1) {
            acc[0][j] += __shfl_xor(acc[0][j], m);
            acc[1][j] += __shfl_xor(acc[1][j], m);
        }
    if (lane_id() == 0) {
#pragma unroll
        for (int j = 0; j < kS; ++j) {
            sh[threadIdx.x / kWave][j] = acc[0][j];
            sh[threadIdx.x / kWave][kS + j] = acc[1][j];
        }
    }
    __syncthreads();
    if (threadIdx.x < (unsigned)(2 * s)) {
        const int q = threadIdx.x / s, j = threadIdx.x % s;
        double r = sh[0][q * kS + j];
        for (int w = 1; w < kRows; ++w) r += sh[w][q * kS + j];
        k.Rb[((int64_t)q * s + j) * k.H + y] = r;
    }
}

// (1b) partial column sums over y >= H-1-ry_j of g R_qj, one block per (64 columns, 64
// rows): Cp[q][j][chunk][x].
__global__ void __launch_bounds__(kBlock) border_cols_kernel(BwdK k) {
    const int s = k.p.n_scales;
    const int ncol = (k.W + kWave - 1) / kWave;
    const int ct = blockIdx.x % ncol, ch = blockIdx.x / ncol;
    const int x = ct * kWave + lane_id(), w = threadIdx.x / kWave;
    int lo[kS];
    double acc[2][kS];
#pragma unroll
    for (int j = 0; j < kS; ++j) {
        acc[0][j] = acc[1][j] = 0.0;
        lo[j] = j < s ? max(k.H - 1 - k.p.ry[j], 0) : k.H;
    }
    if (x < k.W) {
        const int y1 = min(k.H, (ch + 1) * kChunk);
        for (int y = ch * kChunk + w; y < y1; y += kRows) {
            const double gx = (double)k.g[(int64_t)y * k.ld_g + x];
            const int64_t o = (int64_t)y * k.W + x;
#pragma unroll
            for (int j = 0; j < kS; ++j) {
                if (j < s && y >= lo[j]) {
                    acc[0][j] = __builtin_fma(gx, (double)rplane(k, 0, j)[o], acc[0][j]);
                    acc[1][j] = __builtin_fma(gx, (double)rplane(k, 1, j)[o], acc[1][j]);
                }
            }
        }
    }
    __shared__ double sh[kRows][2 * kS][kWave];
#pragma unroll
    for (int j = 0; j < kS; ++j) {
        sh[w][j][lane_id()] = acc[0][j];
        sh[w][kS + j][lane_id()] = acc[1][j];
    }
    __syncthreads();
    if (w == 0 && x < k.W) {
        for (int q = 0; q < 2; ++q)
            for (int j = 0; j < s; ++j) {
                double r = sh[0][q * kS + j][lane_id()];
                for (int i = 1; i < kRows; ++i) r += sh[i][q * kS + j][lane_id()];
                k.Cp[(((int64_t)q * s + j) * k.nchunks + ch) * k.W + x] = r;
            }
    }
}

// (1c) Cb[q][j][x] = sum over chunks of Cp (loads issued 8 at a time).
__global__ void __launch_bounds__(kBlock) border_cols_reduce_kernel(BwdK k) {
    const int s = k.p.n_scales;
    const int64_t id = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (id >= (int64_t)2 * s * k.W) return;
    const int64_t qj = id / k.W, x = id % k.W;
    const double *src = k.Cp + qj * k.nchunks * k.W + x;
    double r = 0.0;
    int c = 0;
    for (; c + 8 <= k.nchunks; c += 8) {
        double a[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) a[u] = src[(int64_t)(c + u) * k.W];
#pragma unroll
        for (int u = 0; u < 8; ++u) r += a[u];
    }
    for (; c < k.nchunks; ++c) r += src[(int64_t)c * k.W];
    k.Cb[qj * k.W + x] = r;
}

// (2) deposits.  Virtual pixel (x', y') holds the deposit at corner c = (W-1-x', H-1-y').
// For field j the corners that equal c come from at most one pixel per corner type,
// except where clamping maps a whole range of pixels onto the last column / row; those
// ranges use Rb, Cb and (for the bottom-right corner) their total K, which the block holding
// virtual pixel (0, 0) forms cooperatively before use.
__global__ void __launch_bounds__(kBlock) deposit_kernel(BwdK k) {
    const int s = k.p.n_scales;
    __shared__ double shK[2][kS];
    int tx, rg;
    comb_map(blockIdx.x, k.tiles_x, k.p4, k.teeth, tx, rg);
    if (tx == 0 && rg == 0) {
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
        if (threadIdx.x < (unsigned)(2 * s)) {
            double r = shp[0][threadIdx.x];
            for (int i = 1; i < kRows; ++i) r += shp[i][threadIdx.x];
            shK[threadIdx.x / s][threadIdx.x % s] = r;
        }
        __syncthreads();
    }
    const int xv = tx * kWave + lane_id();
    const int yv = rg * kRows + (int)(threadIdx.x / kWave);
    if (xv >= k.W || yv >= k.H) return;
    const int cx = k.W - 1 - xv, cy = k.H - 1 - yv;
    const bool lastx = cx == k.W - 1, lasty = cy == k.H - 1;
    double d0 = 0.0, d1 = 0.0;
    // g R1 and g R2 at pixel (px, py), added with sign sg
    auto add = [&](int j, int px, int py, double sg) {
        const int64_t o = (int64_t)py * k.W + px;
        const double gs = sg * (double)k.g[(int64_t)py * k.ld_g + px];
        d0 = __builtin_fma(gs, (double)rplane(k, 0, j)[o], d0);
        d1 = __builtin_fma(gs, (double)rplane(k, 1, j)[o], d1);
    };
    for (int j = 0; j < s; ++j) {
        const int rx = k.p.rx[j], ry = k.p.ry[j];
        const int pxp = cx - rx;            // pixel whose x+ corner is cx (cx < W-1)
        const int pxm = cx + rx + 1;        // pixel whose x- corner is cx
        const int pyp = cy - ry;
        const int pym = cy + ry + 1;
        const bool vxm = pxm <= k.W - 1, vym = pym <= k.H - 1;
        const double *R0 = k.Rb + (int64_t)j * k.H, *R1 = k.Rb + ((int64_t)s + j) * k.H;
        const double *C0 = k.Cb + (int64_t)j * k.W, *C1 = k.Cb + ((int64_t)s + j) * k.W;
        // (x+, y+) corner
        if (!lastx && !lasty) {
            if (pxp >= 0 && pyp >= 0) add(j, pxp, pyp, 1.0);
        } else if (lastx && !lasty) {
            if (pyp >= 0) { d0 += R0[pyp]; d1 += R1[pyp]; }
        } else if (!lastx && lasty) {
            if (pxp >= 0) { d0 += C0[pxp]; d1 += C1[pxp]; }
        } else {
            d0 += shK[0][j];
            d1 += shK[1][j];
        }
        // (x-, y+) corner, sign -
        if (vxm) {
            if (!lasty) {
                if (pyp >= 0) add(j, pxm, pyp, -1.0);
            } else {
                d0 -= C0[pxm];
                d1 -= C1[pxm];
            }
        }
        // (x+, y-) corner, sign -
        if (vym) {
            if (!lastx) {
                if (pxp >= 0) add(j, pxp, pym, -1.0);
            } else {
                d0 -= R0[pym];
                d1 -= R1[pym];
            }
        }
        // (x-, y-) corner
        if (vxm && vym) add(j, pxm, pym, 1.0);
    }
    k.Dr[(int64_t)yv * k.W + xv] = make_double2(d0, d1);
}

// (4) scalar gradients: per-block partials of sum g E, sum g (1 - Pbar), sum g Pbar over a
// fixed pixel assignment, then one block adds them in a fixed order.
__global__ void __launch_bounds__(kBlock) scalar_partial_kernel(BwdK k) {
    const int s = k.p.n_scales;
    const int64_t n = (int64_t)k.H * k.W, ps = n;
    const float *E = k.R + (int64_t)(2 * s) * ps, *Pb = k.R + (int64_t)(2 * s + 1) * ps;
    Sum3 acc{0.0, 0.0, 0.0};
    for (int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * kBlock) {
        const int64_t y = i / k.W, x = i % k.W;
        const double gx = (double)k.g[y * k.ld_g + x];
        const double pb = (double)Pb[i];
        acc.a = __builtin_fma(gx, (double)E[i], acc.a);
        acc.b = __builtin_fma(gx, 1.0 - pb, acc.b);
        acc.c = __builtin_fma(gx, pb, acc.c);
    }
    const Sum3 r = block_sum3(acc);
    if (threadIdx.x == 0) {
        k.part[3 * blockIdx.x] = r.a;
        k.part[3 * blockIdx.x + 1] = r.b;
        k.part[3 * blockIdx.x + 2] = r.c;
    }
}

__global__ void __launch_bounds__(kBlock) scalar_finalize_kernel(const double *part, int nparts,
                                                                 double *out) {
    Sum3 acc{0.0, 0.0, 0.0};
    for (int i = threadIdx.x; i < nparts; i += kBlock) {
        acc.a += part[3 * i];
        acc.b += part[3 * i + 1];
        acc.c += part[3 * i + 2];
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

BwdPlan make_bwd_plan(int H, int W, int n_scales, const int *ry, bool with_resid) {
    BwdPlan b{};
    const int tiles_x = (W + kWave - 1) / kWave;
    comb_params(H, kRows, ry, n_scales, &b.p4, &b.teeth);
    b.nblocks = (int64_t)tiles_x * b.p4 * b.teeth;
    b.nchunks = (H + kChunk - 1) / kChunk;
    size_t off = 0;
    auto take = [&](size_t bytes) {
        size_t o = off;
        off = round_up(off + bytes, 256);
        return o;
    };
    const size_t hw = (size_t)H * W;
    b.resid = with_resid ? take((2 * (size_t)n_scales + 2) * hw * sizeof(float)) : 0;
    b.Rb = take(2 * (size_t)n_scales * H * sizeof(double));
    b.Cp = take(2 * (size_t)n_scales * b.nchunks * (size_t)W * sizeof(double));
    b.Cb = take(2 * (size_t)n_scales * W * sizeof(double));
    b.Dr = take(hw * sizeof(double2));
    b.part = take((size_t)kScalarBlocks * 3 * sizeof(double));
    b.scan_plan = make_scan_plan(H, W, kF64, 0, scan_tune_default(H, W));
    b.scan = take(b.scan_plan.total);
    b.total = off;
    return b;
}

hipError_t launch_backward_resid(const BwdResidArgs &a, const BwdPlan &plan, void *ws,
                                 hipStream_t s) {
    char *w = static_cast<char *>(ws);
    BwdK k;
    k.v = a.v;
    k.ld_v = a.ld_v;
    k.H = a.H;
    k.W = a.W;
    k.p = a.p;
    k.g = a.g;
    k.ld_g = a.ld_g;
    k.R = a.resid;
    k.Rb = reinterpret_cast<double *>(w + plan.Rb);
    k.Cp = reinterpret_cast<double *>(w + plan.Cp);
    k.Cb = reinterpret_cast<double *>(w + plan.Cb);
    k.Dr = reinterpret_cast<double2 *>(w + plan.Dr);
    k.part = reinterpret_cast<double *>(w + plan.part);
    k.tiles_x = (a.W + kWave - 1) / kWave;
    k.p4 = plan.p4;
    k.teeth = plan.teeth;
    k.nchunks = plan.nchunks;
    const int S = a.p.n_scales;
    hipLaunchKernelGGL(border_rows_kernel, dim3(a.H), dim3(kBlock), 0, s, k);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    const unsigned ncol = (unsigned)((a.W + kWave - 1) / kWave);
    hipLaunchKernelGGL(border_cols_kernel, dim3(ncol * plan.nchunks), dim3(kBlock), 0, s, k);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    const unsigned nred = (unsigned)(((int64_t)2 * S * a.W + kBlock - 1) / kBlock);
    hipLaunchKernelGGL(border_cols_reduce_kernel, dim3(nred), dim3(kBlock), 0, s, k);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    hipLaunchKernelGGL(deposit_kernel, dim3((unsigned)plan.nblocks), dim3(kBlock), 0, s, k);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    e = launch_suffix_adjoint(k.Dr, a.W, a.v, a.ld_v, a.H, a.W, a.grad_v, a.ld_gv,
                              plan.scan_plan, w + plan.scan, s);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(scalar_partial_kernel, dim3(kScalarBlocks), dim3(kBlock), 0, s, k);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    hipLaunchKernelGGL(scalar_finalize_kernel, dim3(1), dim3(kBlock), 0, s, k.part,
                       kScalarBlocks, a.grad_params);
    return hipGetLastError();
}

}  // namespace tmo
