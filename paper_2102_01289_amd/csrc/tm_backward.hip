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
constexpr int kChunkMax = 64;    // rows per partial of the column sums, at most

struct BwdK {
    const float *v;
    int64_t ld_v;
    int H, W;
    QueryParams p;
    const float *g;
    int64_t ld_g;
    const float *R;  // residuals: pair planes {R1_j, R2_j} for j < s, then E, then Pbar
    double *Rp;      // [2][s][ncol][H] row range sums of g R per 64-column tile
    double *Rb;      // [2][s][H]  row range sums of g R
    double *Cp;      // [2][s][nchunks][W] partial column range sums
    double *Cb;      // [2][s][W]  column range sums
    double2 *Dr;     // [H][W] deposits {D1, D2} in reversed order
    double *part;    // [ncol * nchunks][3] scalar partials
    int tiles_x, p4, teeth, nchunks, chunk;
};

// Residual pair plane of field j: {R1_j, R2_j} per pixel, pitch W.
__device__ __forceinline__ const float2 *rpair(const BwdK &k, int j) {
    return reinterpret_cast<const float2 *>(k.R) + (int64_t)j * k.H * k.W;
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

// (1) One streaming pass over g, the residual pairs, E and Pbar, one block per (64 columns,
// chunk rows):
//   Rp[q][j][ct][y] = sum over the tile's columns x >= W-1-rx_j of g R_qj(x, y),
//   Cp[q][j][chunk][x] = sum over the tile's rows y >= H-1-ry_j of g R_qj(x, y),
//   part[block] = {sum g E, sum g (1 - Pbar), sum g Pbar},
// each combined in a fixed order.  A residual pair is loaded only where some field needs it.
// S: the number of fields, fixed at compile time so that a row's state holds only the fields
// in use.
template <int S>
__global__ void __launch_bounds__(kBlock) border_scalar_kernel(BwdK k) {
    constexpr int s = S;
    const int ncol = (k.W + kWave - 1) / kWave;
    const int ct = blockIdx.x % ncol, ch = blockIdx.x / ncol;
    const int x = ct * kWave + lane_id(), w = wave_id();
    const int y0 = ch * k.chunk, y1 = min(k.H, y0 + k.chunk);
    const int64_t hw = (int64_t)k.H * k.W;
    const float *E = k.R + 2 * (int64_t)s * hw, *Pb = E + hw;
    int lox[S], loy[S];
    double cacc[2][S];
#pragma unroll
    for (int j = 0; j < S; ++j) {
        lox[j] = max(k.W - 1 - k.p.rx[j], 0);
        loy[j] = max(k.H - 1 - k.p.ry[j], 0);
        cacc[0][j] = cacc[1][j] = 0.0;
    }
    __shared__ double shr[2 * S][kChunkMax];
    Sum3 sacc{0.0, 0.0, 0.0};
    const int xc = min(x, k.W - 1);      // in-image address for the lanes past the edge
    const bool in = x < k.W;
    const int tile_end = min(ct * kWave + kWave, k.W);
    // every load of a row in one phase; the next row of this wave is loaded before the
    // current one is reduced
    struct Row {
        float g, e, p;
        float2 r[S];
    };
    auto load_row = [&](int y, Row &q) {
        const int64_t o = (int64_t)y * k.W + xc;
        q.g = k.g[(int64_t)y * k.ld_g + xc];
        q.e = E[o];
        q.p = Pb[o];
#pragma unroll
        for (int j = 0; j < S; ++j) {
            q.r[j] = make_float2(0.f, 0.f);
            // wave-uniform: does any field-j range sum need this tile row?
            if (tile_end > lox[j] || y >= loy[j]) q.r[j] = rpair(k, j)[o];
        }
    };
    Row cur, nxt;
    int y = y0 + w;   // wave-uniform
    if (y < y1) load_row(y, cur);
    for (; y < y1; y += kRows) {
        const bool more = y + kRows < y1;
        if (more) load_row(y + kRows, nxt);
        const double gx = in ? (double)cur.g : 0.0;
        const double pb = (double)cur.p;
        sacc.a = __builtin_fma(gx, (double)cur.e, sacc.a);
        sacc.b = __builtin_fma(gx, 1.0 - pb, sacc.b);
        sacc.c = __builtin_fma(gx, pb, sacc.c);
#pragma unroll
        for (int j = 0; j < S; ++j) {
            const double a = gx * (double)cur.r[j].x, b = gx * (double)cur.r[j].y;
            if (y >= loy[j]) { cacc[0][j] += a; cacc[1][j] += b; }
            double ra = 0.0, rb = 0.0;
            if (tile_end > lox[j]) {   // block-uniform: the row range reaches this tile
                const bool inr = x >= lox[j];
                ra = wave_sum<Acc<kF64>>(inr ? a : 0.0);
                rb = wave_sum<Acc<kF64>>(inr ? b : 0.0);
            }
            if (lane_id() == 0) {
                shr[j][y - y0] = ra;
                shr[S + j][y - y0] = rb;
            }
        }
        if (more) cur = nxt;
    }
    // column partials: the four waves' sums in a fixed order
    __shared__ double shc[kRows][kWave];
    for (int qj = 0; qj < 2 * s; ++qj) {
        const int q = qj / s, j = qj % s;
        double v = 0.0;
#pragma unroll
        for (int jj = 0; jj < S; ++jj)
            if (jj == j) v = q ? cacc[1][jj] : cacc[0][jj];
        __syncthreads();
        shc[w][lane_id()] = v;
        __syncthreads();
        if (w == 0 && x < k.W) {
            double r = shc[0][lane_id()];
            for (int i = 1; i < kRows; ++i) r += shc[i][lane_id()];
            k.Cp[(((int64_t)q * s + j) * k.nchunks + ch) * k.W + x] = r;
        }
    }
    // row partials, coalesced along y
    for (int t = threadIdx.x; t < 2 * s * (y1 - y0); t += kBlock) {
        const int qj = t / (y1 - y0), r = t % (y1 - y0);
        const int q = qj / s, j = qj % s;
        k.Rp[(((int64_t)q * s + j) * ncol + ct) * k.H + y0 + r] = shr[q * S + j][r];
    }
    const Sum3 tot = block_sum3(sacc);
    if (threadIdx.x == 0) {
        k.part[3 * blockIdx.x] = tot.a;
        k.part[3 * blockIdx.x + 1] = tot.b;
        k.part[3 * blockIdx.x + 2] = tot.c;
    }
}

// (1') Rb[q][j][y] = sum over column tiles of Rp and Cb[q][j][x] = sum over row chunks of Cp,
// in a fixed order, loads issued 16 at a time (the pass is a few memory round trips long).
__device__ __forceinline__ double strided_sum(const double *src, int n, int64_t stride) {
    constexpr int kB = 16;
    double r = 0.0;
    int c = 0;
    for (; c + kB <= n; c += kB) {
        double a[kB];
#pragma unroll
        for (int u = 0; u < kB; ++u) a[u] = src[(int64_t)(c + u) * stride];
#pragma unroll
        for (int u = 0; u < kB; ++u) r += a[u];
    }
    double a[kB];
#pragma unroll
    for (int u = 0; u < kB; ++u) a[u] = c + u < n ? src[(int64_t)(c + u) * stride] : 0.0;
#pragma unroll
    for (int u = 0; u < kB; ++u)
        if (c + u < n) r += a[u];
    return r;
}

__global__ void __launch_bounds__(kBlock) border_reduce_kernel(BwdK k) {
    const int s = k.p.n_scales;
    const int ncol = (k.W + kWave - 1) / kWave;
    const int64_t id = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    const int64_t nr = (int64_t)2 * s * k.H, nc = (int64_t)2 * s * k.W;
    if (id < nr) {
        const int64_t qj = id / k.H, y = id % k.H;
        k.Rb[qj * k.H + y] = strided_sum(k.Rp + qj * ncol * k.H + y, ncol, k.H);
    } else if (id < nr + nc) {
        const int64_t i = id - nr, qj = i / k.W, x = i % k.W;
        k.Cb[qj * k.W + x] = strided_sum(k.Cp + qj * k.nchunks * k.W + x, k.nchunks, k.W);
    }
}

// (2) deposits.  Virtual pixel (x', y') holds the deposit at corner c = (W-1-x', H-1-y').
// For field j the corners that equal c come from at most one pixel per corner type,
// except where clamping maps a whole range of pixels onto the last column / row; those
// ranges use Rb, Cb and (for the bottom-right corner) their total K, which the block holding
// virtual pixel (0, 0) forms cooperatively before use.  The four gathers of a field are
// issued together, branch-free: a corner that does not exist reads a clamped in-image
// address with weight 0 (such lanes share one cache line).  Rows are wave-uniform.
// S: the number of fields, fixed at compile time so that the gathers of every field are
// issued together (a loop with a run-time bound keeps one field's loads in flight at a time).
template <int S>
__global__ void __launch_bounds__(kBlock) deposit_kernel(BwdK k) {
    constexpr int s = S;
    __shared__ double shK[2][kS];
    int tx, rg;
    comb_map(xcd_tile(blockIdx.x, gridDim.x), k.tiles_x, k.p4, k.teeth, tx, rg);
    if (tx == 0 && rg == 0) {
        __shared__ double shp[kRows][2 * kS];
        const int w = wave_id();
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
    const int yv = rg * kRows + wave_id();
    if (xv >= k.W || yv >= k.H) return;
    const int cx = k.W - 1 - xv, cy = k.H - 1 - yv;   // cy is wave-uniform
    const bool lastx = cx == k.W - 1, lasty = cy == k.H - 1;
    double d0 = 0.0, d1 = 0.0;
    // gather phase: all loads of all fields first (issued unconditionally: skipping the
    // corner types no lane of a wave has, behind wave-uniform branches, was measured 2.8x
    // slower, because the branches stop the loads of later fields from being in flight)
    float2 rv[S][4];
    float gw[S][4];
#pragma unroll
    for (int j = 0; j < S; ++j) {
        const int rx = k.p.rx[j], ry = k.p.ry[j];
        const int ax = max(cx - rx, 0), bx = min(cx + rx + 1, k.W - 1);
        const int ay = max(cy - ry, 0), by = min(cy + ry + 1, k.H - 1);
        // corner rows are wave-uniform: scalar row bases, 32-bit lane offsets
        const char *Rj = reinterpret_cast<const char *>(rpair(k, j));
        const char *Ra = Rj + (int64_t)ay * k.W * 8, *Rb_ = Rj + (int64_t)by * k.W * 8;
        const char *ga = reinterpret_cast<const char *>(k.g + (int64_t)ay * k.ld_g);
        const char *gb = reinterpret_cast<const char *>(k.g + (int64_t)by * k.ld_g);
        const uint32_t oa = (uint32_t)ax, ob = (uint32_t)bx;
        rv[j][0] = load_at<float2>(Ra, oa * 8u);
        rv[j][1] = load_at<float2>(Ra, ob * 8u);
        rv[j][2] = load_at<float2>(Rb_, oa * 8u);
        rv[j][3] = load_at<float2>(Rb_, ob * 8u);
        gw[j][0] = load_at<float>(ga, oa * 4u);
        gw[j][1] = load_at<float>(ga, ob * 4u);
        gw[j][2] = load_at<float>(gb, oa * 4u);
        gw[j][3] = load_at<float>(gb, ob * 4u);
    }
#pragma unroll
    for (int j = 0; j < S; ++j) {
        {
            const int rx = k.p.rx[j], ry = k.p.ry[j];
            const int pxp = cx - rx;        // pixel whose x+ corner is cx (cx < W-1)
            const int pxm = cx + rx + 1;    // pixel whose x- corner is cx
            const int pyp = cy - ry;
            const int pym = cy + ry + 1;
            const bool okxp = !lastx && pxp >= 0, okxm = pxm <= k.W - 1;
            const bool okyp = !lasty && pyp >= 0, okym = pym <= k.H - 1;
            const float2 r_pp = rv[j][0], r_mp = rv[j][1], r_pm = rv[j][2], r_mm = rv[j][3];
            const float g_pp = gw[j][0], g_mp = gw[j][1], g_pm = gw[j][2], g_mm = gw[j][3];
            const double w_pp = okxp && okyp ? (double)g_pp : 0.0;
            const double w_mp = okxm && okyp ? -(double)g_mp : 0.0;
            const double w_pm = okxp && okym ? -(double)g_pm : 0.0;
            const double w_mm = okxm && okym ? (double)g_mm : 0.0;
            d0 = __builtin_fma(w_pp, (double)r_pp.x, d0);
            d1 = __builtin_fma(w_pp, (double)r_pp.y, d1);
            d0 = __builtin_fma(w_mp, (double)r_mp.x, d0);
            d1 = __builtin_fma(w_mp, (double)r_mp.y, d1);
            d0 = __builtin_fma(w_pm, (double)r_pm.x, d0);
            d1 = __builtin_fma(w_pm, (double)r_pm.y, d1);
            d0 = __builtin_fma(w_mm, (double)r_mm.x, d0);
            d1 = __builtin_fma(w_mm, (double)r_mm.y, d1);
            if (lastx || lasty) {
                // clamped corners: whole ranges of pixels deposit on the last column / row
                const double *R0 = k.Rb + (int64_t)j * k.H, *R1 = k.Rb + ((int64_t)s + j) * k.H;
                const double *C0 = k.Cb + (int64_t)j * k.W, *C1 = k.Cb + ((int64_t)s + j) * k.W;
                if (lastx && !lasty && pyp >= 0) { d0 += R0[pyp]; d1 += R1[pyp]; }
                if (lasty && !lastx && pxp >= 0) { d0 += C0[pxp]; d1 += C1[pxp]; }
                if (lastx && lasty) { d0 += shK[0][j]; d1 += shK[1][j]; }
                if (lasty && okxm) { d0 -= C0[pxm]; d1 -= C1[pxm]; }
                if (lastx && okym) { d0 -= R0[pym]; d1 -= R1[pym]; }
            }
        }
    }
    __builtin_nontemporal_store(d0, &k.Dr[(int64_t)yv * k.W + xv].x);
    __builtin_nontemporal_store(d1, &k.Dr[(int64_t)yv * k.W + xv].y);
}

// (4) scalar gradients: one block adds the per-block partials of (1) in a fixed order.
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
    // rows per block of the border pass: 64, halved (down to 16) while the pass would have
    // fewer than 2048 blocks, so that smaller images still fill the GPU
    b.chunk = kChunkMax;
    while (b.chunk > 16 && (int64_t)tiles_x * ((H + b.chunk - 1) / b.chunk) < 2048) b.chunk /= 2;
    b.nchunks = (H + b.chunk - 1) / b.chunk;
    size_t off = 0;
    auto take = [&](size_t bytes) {
        size_t o = off;
        off = round_up(off + bytes, 256);
        return o;
    };
    const size_t hw = (size_t)H * W;
    b.resid = with_resid ? take((2 * (size_t)n_scales + 2) * hw * sizeof(float)) : 0;
    b.Rp = take(2 * (size_t)n_scales * tiles_x * (size_t)H * sizeof(double));
    b.Rb = take(2 * (size_t)n_scales * H * sizeof(double));
    b.Cp = take(2 * (size_t)n_scales * b.nchunks * (size_t)W * sizeof(double));
    b.Cb = take(2 * (size_t)n_scales * W * sizeof(double));
    b.Dr = take(hw * sizeof(double2));
    b.part = take((size_t)tiles_x * b.nchunks * 3 * sizeof(double));
    b.scan_plan = make_scan_plan(H, W, kF64, 0, scan_tune_adjoint(H, W));
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
    k.Rp = reinterpret_cast<double *>(w + plan.Rp);
    k.Rb = reinterpret_cast<double *>(w + plan.Rb);
    k.Cp = reinterpret_cast<double *>(w + plan.Cp);
    k.Cb = reinterpret_cast<double *>(w + plan.Cb);
    k.Dr = reinterpret_cast<double2 *>(w + plan.Dr);
    k.part = reinterpret_cast<double *>(w + plan.part);
    k.tiles_x = (a.W + kWave - 1) / kWave;
    k.p4 = plan.p4;
    k.teeth = plan.teeth;
    k.nchunks = plan.nchunks;
    k.chunk = plan.chunk;
    const int S = a.p.n_scales;
    const unsigned nbs = (unsigned)(k.tiles_x * plan.nchunks);
    switch (S) {
#define TM_BORDER(n)                                                                            \
    case n:                                                                                    \
        hipLaunchKernelGGL(border_scalar_kernel<n>, dim3(nbs), dim3(kBlock), 0, s, k);         \
        break;
        TM_BORDER(1) TM_BORDER(2) TM_BORDER(3) TM_BORDER(4)
        TM_BORDER(5) TM_BORDER(6) TM_BORDER(7) TM_BORDER(8)
#undef TM_BORDER
        default: return hipErrorInvalidValue;
    }
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    const unsigned nred = (unsigned)(((int64_t)2 * S * (a.H + a.W) + kBlock - 1) / kBlock);
    hipLaunchKernelGGL(border_reduce_kernel, dim3(nred), dim3(kBlock), 0, s, k);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    hipLaunchKernelGGL(scalar_finalize_kernel, dim3(1), dim3(kBlock), 0, s, k.part, (int)nbs,
                       a.grad_params);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    switch (S) {
#define TM_DEPOSIT(n)                                                                           \
    case n:                                                                                    \
        hipLaunchKernelGGL(deposit_kernel<n>, dim3((unsigned)plan.nblocks), dim3(kBlock), 0, s, k); \
        break;
        TM_DEPOSIT(1) TM_DEPOSIT(2) TM_DEPOSIT(3) TM_DEPOSIT(4)
        TM_DEPOSIT(5) TM_DEPOSIT(6) TM_DEPOSIT(7) TM_DEPOSIT(8)
#undef TM_DEPOSIT
        default: return hipErrorInvalidValue;
    }
    if ((e = hipGetLastError()) != hipSuccess) return e;
    return launch_suffix_adjoint(k.Dr, a.W, a.v, a.ld_v, a.H, a.W, a.grad_v, a.ld_gv,
                                 plan.scan_plan, w + plan.scan, s);
}

}  // namespace tmo
