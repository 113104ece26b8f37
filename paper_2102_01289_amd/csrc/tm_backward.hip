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
// Kernels: (1) one launch that interleaves two independent kinds of block: border blocks,
// which stream g, E, Pbar and the residual pairs and form the deposits that clamping piles
// onto the last column / row (row sums and partial column sums) and the scalar partials,
// and deposit blocks, which gather D1, D2 (FP64, comb block order) at every virtual pixel
// off the last column and row, written in reversed pixel order; (2) fixed-order sums of the
// border partials and of the scalar gradients; (3) the deposits of the last column and row
// (only clamped ranges reach them); (4) the ordinary three-stage prefix scan, run in adjoint
// mode, which yields the suffix sums and writes dv.  No atomics anywhere, so every result is
// bit-reproducible.
#include "tm_device.h"
#include "tm_internal.h"

namespace tmo {

namespace {

constexpr int kBlock = 256;
constexpr int kRows = kBlock / kWave;
constexpr int kS = 8;            // TM_MAX_SCALES
constexpr int kChunkMax = 64;    // rows per partial of the column sums, at most
constexpr int kKParts = 8;       // blocks per corner total K

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
    double *gp;      // [3] scalar gradients
    double *K;       // [2][s][kKParts] partial totals of the row range sums over each
                     // field's clamped rows
    int tiles_x, p4, teeth, nchunks, chunk;
    uint32_t ndep, nbor;  // deposit and border blocks of the interleaved launch
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

// (1a) Border block bid (64 columns, chunk rows): streaming passes over g, E, Pbar and the
// residual pairs.  First the scalar partials
//   part[bid] = {sum g E, sum g (1 - Pbar), sum g Pbar},
// then, one field at a time (so the per-row state stays a few registers), only where the
// field's clamped ranges reach this block:
//   Rp[q][j][ct][y] = sum over the tile's columns x >= W-1-rx_j of g R_qj(x, y)
//                     (tiles that end right of W-1-rx_j),
//   Cp[q][j][chunk][x] = sum over the chunk's rows y >= H-1-ry_j of g R_qj(x, y)
//                     (chunks that end below H-1-ry_j).
// Entries of Rp and Cp outside those ranges are never written nor read.  Every sum is in a
// fixed order.  Rows are wave-uniform (scalar row bases, 32-bit lane offsets), two rows in
// flight per wave.  The scalar pass keeps the block's g tile in LDS, where every field's pass
// reads it back instead of streaming g again.
template <int S>
__device__ __forceinline__ void border_block(const BwdK &k, int bid) {
    const int ncol = (k.W + kWave - 1) / kWave;
    const int ct = bid % ncol, ch = bid / ncol;
    const int x = ct * kWave + lane_id(), w = wave_id();
    const int y0 = ch * k.chunk, y1 = min(k.H, y0 + k.chunk);
    const int64_t hw = (int64_t)k.H * k.W;
    const float *E = k.R + 2 * (int64_t)S * hw, *Pb = E + hw;
    const int xc = min(x, k.W - 1);      // in-image address for the lanes past the edge
    const bool in = x < k.W;
    const int tile_end = min(ct * kWave + kWave, k.W);
    const uint32_t o4 = (uint32_t)xc * 4u, o8 = (uint32_t)xc * 8u;
    auto grow = [&](int y) { return reinterpret_cast<const char *>(k.g + (int64_t)y * k.ld_g); };
    __shared__ float shg[kChunkMax][kWave];   // g of the block's rows [y0, y1)
    {
        Sum3 sacc{0.0, 0.0, 0.0};
        float g[2], e[2], pb[2];
        auto load = [&](int y, int u) {
            const int64_t ro = (int64_t)y * k.W;
            g[u] = load_at<float>(grow(y), o4);
            e[u] = load_at<float>(reinterpret_cast<const char *>(E + ro), o4);
            pb[u] = load_at<float>(reinterpret_cast<const char *>(Pb + ro), o4);
        };
        auto use = [&](int y, int u) {
            shg[y - y0][lane_id()] = g[u];
            const double gx = in ? (double)g[u] : 0.0;
            const double pv = (double)pb[u];
            sacc.a = __builtin_fma(gx, (double)e[u], sacc.a);
            sacc.b = __builtin_fma(gx, 1.0 - pv, sacc.b);
            sacc.c = __builtin_fma(gx, pv, sacc.c);
        };
        int y = y0 + w;   // wave-uniform; the waves together cover every row of [y0, y1)
        if (y < y1) load(y, 0);
        while (y < y1) {
            if (y + kRows < y1) load(y + kRows, 1);
            use(y, 0);
            y += kRows;
            if (y >= y1) break;
            if (y + kRows < y1) load(y + kRows, 0);
            use(y, 1);
            y += kRows;
        }
        // block_sum3 passes two block barriers: the g tile is complete after it
        const Sum3 tot = block_sum3(sacc);
        if (threadIdx.x == 0) {
            k.part[3 * bid] = tot.a;
            k.part[3 * bid + 1] = tot.b;
            k.part[3 * bid + 2] = tot.c;
        }
    }
    __shared__ double shr[2][kChunkMax];
    __shared__ double shc[kRows][kWave];
    for (int j = 0; j < S; ++j) {
        const int lox = max(k.W - 1 - k.p.rx[j], 0), loy = max(k.H - 1 - k.p.ry[j], 0);
        const bool rows = tile_end > lox, cols = y1 > loy;   // block-uniform
        if (!rows && !cols) continue;
        const bool inr = in && x >= lox;
        const char *Rj = reinterpret_cast<const char *>(rpair(k, j));
        double c0 = 0.0, c1 = 0.0;
        float g[2];
        float2 r[2];
        auto load = [&](int y, int u) {
            g[u] = shg[y - y0][lane_id()];
            r[u] = load_at<float2>(Rj + (int64_t)y * k.W * 8, o8);
        };
        auto use = [&](int y, int u) {
            const double gx = in ? (double)g[u] : 0.0;
            const double a = gx * (double)r[u].x, b = gx * (double)r[u].y;
            if (y >= loy) {
                c0 += a;
                c1 += b;
            }
            if (rows) {
                double ra, rb;
                wave_sum2(inr ? a : 0.0, inr ? b : 0.0, ra, rb);
                if (lane_id() == 0) {
                    shr[0][y - y0] = ra;
                    shr[1][y - y0] = rb;
                }
            }
        };
        int y = (rows ? y0 : max(y0, loy)) + w;   // wave-uniform
        if (y < y1) load(y, 0);
        while (y < y1) {
            if (y + kRows < y1) load(y + kRows, 1);
            use(y, 0);
            y += kRows;
            if (y >= y1) break;
            if (y + kRows < y1) load(y + kRows, 0);
            use(y, 1);
            y += kRows;
        }
        if (cols) {   // the four waves' column sums in a fixed order
            for (int q = 0; q < 2; ++q) {
                __syncthreads();
                shc[w][lane_id()] = q ? c1 : c0;
                __syncthreads();
                if (w == 0 && x < k.W) {
                    double v = shc[0][lane_id()];
                    for (int i = 1; i < kRows; ++i) v += shc[i][lane_id()];
                    k.Cp[(((int64_t)q * S + j) * k.nchunks + ch) * k.W + x] = v;
                }
            }
        }
        __syncthreads();
        if (rows) {   // row sums, coalesced along y
            for (int t = threadIdx.x; t < 2 * (y1 - y0); t += kBlock) {
                const int q = t / (y1 - y0), rr = t % (y1 - y0);
                k.Rp[(((int64_t)q * S + j) * ncol + ct) * k.H + y0 + rr] = shr[q][rr];
            }
        }
        __syncthreads();
    }
}

// (2) Sums of border partials over column tiles / row chunks in a fixed order, loads issued
// 16 at a time (the pass is a few memory round trips long).
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

// (2) Rb[q][j][y] = sum over column tiles of Rp and Cb[q][j][x] = sum over row chunks of Cp;
// 2s kKParts blocks form parts of the totals K of the range sums over each field's clamped
// rows (for the bottom-right corner), and the last block adds the border blocks' scalar
// partials into the three scalar gradients.  All in a fixed order.
__global__ void __launch_bounds__(kBlock) border_reduce_kernel(BwdK k) {
    const int s = k.p.n_scales;
    const int ncol = (k.W + kWave - 1) / kWave;
    const int nK = 2 * s * kKParts;
    if (blockIdx.x >= gridDim.x - 1 - nK && blockIdx.x < gridDim.x - 1) {
        // part kp of K[q][j] = sum over y >= H-1-ry_j and column tiles ct >= ct0_j of Rp,
        // the (tile, row) pairs taken in a fixed order, split evenly over kKParts blocks
        const int kb = (int)(blockIdx.x - (gridDim.x - 1 - nK));
        const int qj = kb / kKParts, kp = kb % kKParts, j = qj % s;
        const int ct0 = max(k.W - 1 - k.p.rx[j], 0) / kWave;
        const int y0 = max(k.H - 1 - k.p.ry[j], 0), ny = k.H - y0;
        const int64_t n = (int64_t)(ncol - ct0) * ny;
        const int64_t e0 = n * kp / kKParts, e1 = n * (kp + 1) / kKParts;
        const double *base = k.Rp + ((int64_t)qj * ncol + ct0) * k.H + y0;
        constexpr int kB = 8;
        double acc = 0.0;
        for (int64_t e = e0 + threadIdx.x; e < e1; e += (int64_t)kB * kBlock) {
            double a[kB];
#pragma unroll
            for (int u = 0; u < kB; ++u) {
                const int64_t f = e + (int64_t)u * kBlock;
                a[u] = f < e1 ? base[(f / ny) * k.H + f % ny] : 0.0;
            }
#pragma unroll
            for (int u = 0; u < kB; ++u) acc += a[u];
        }
        acc = wave_sum<Acc<kF64>>(acc);
        __shared__ double shp[kRows];
        if (lane_id() == 0) shp[wave_id()] = acc;
        __syncthreads();
        if (threadIdx.x == 0) {
            double r = shp[0];
            for (int i = 1; i < kRows; ++i) r += shp[i];
            k.K[kb] = r;
        }
        return;
    }
    if (blockIdx.x == gridDim.x - 1) {
        Sum3 acc{0.0, 0.0, 0.0};
        for (uint32_t i = threadIdx.x; i < k.nbor; i += kBlock) {
            acc.a += k.part[3 * i];
            acc.b += k.part[3 * i + 1];
            acc.c += k.part[3 * i + 2];
        }
        const Sum3 r = block_sum3(acc);
        if (threadIdx.x == 0) {
            k.gp[0] = r.a;
            k.gp[1] = r.b;
            k.gp[2] = r.c;
        }
        return;
    }
    const int64_t id = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    const int64_t nr = (int64_t)2 * s * k.H, nc = (int64_t)2 * s * k.W;
    // only the tiles / chunks that the field's clamped range reaches hold partials
    if (id < nr) {
        const int64_t qj = id / k.H, y = id % k.H;
        const int j = (int)(qj % s), ct0 = max(k.W - 1 - k.p.rx[j], 0) / kWave;
        k.Rb[qj * k.H + y] =
            strided_sum(k.Rp + (qj * ncol + ct0) * k.H + y, ncol - ct0, k.H);
    } else if (id < nr + nc) {
        const int64_t i = id - nr, qj = i / k.W, x = i % k.W;
        const int j = (int)(qj % s), ch0 = max(k.H - 1 - k.p.ry[j], 0) / k.chunk;
        k.Cb[qj * k.W + x] =
            strided_sum(k.Cp + (qj * k.nchunks + ch0) * k.W + x, k.nchunks - ch0, k.W);
    }
}

// (1b) Deposit block: virtual pixel (x', y') holds the deposit at corner c = (W-1-x',
// H-1-y').  For field j the corners that equal c come from at most one pixel per corner type,
// except where clamping maps a whole range of pixels onto the last column / row; the last
// column and row receive nothing else, and (3) writes them.  The four gathers of a field are
// issued together, branch-free: a corner that does not exist reads a clamped in-image
// address with weight 0 (such lanes share one cache line).  Rows are wave-uniform.
// S: the number of fields, fixed at compile time so that the gathers of every field are
// issued together (a loop with a run-time bound keeps one field's loads in flight at a time).
template <int S>
__device__ __forceinline__ void deposit_block(const BwdK &k, uint32_t tile) {
    int tx, rg;
    comb_map(tile, k.tiles_x, k.p4, k.teeth, tx, rg);
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
        const int rx = k.p.rx[j], ry = k.p.ry[j];
        const int pxp = cx - rx;        // pixel whose x+ corner is cx (cx < W-1)
        const int pxm = cx + rx + 1;    // pixel whose x- corner is cx
        const int pyp = cy - ry;
        const int pym = cy + ry + 1;
        const bool okxp = !lastx && pxp >= 0, okxm = pxm <= k.W - 1;
        const bool okyp = !lasty && pyp >= 0, okym = pym <= k.H - 1;
        const float2 r_pp = rv[j][0], r_mp = rv[j][1], r_pm = rv[j][2], r_mm = rv[j][3];
        const double w_pp = okxp && okyp ? (double)gw[j][0] : 0.0;
        const double w_mp = okxm && okyp ? -(double)gw[j][1] : 0.0;
        const double w_pm = okxp && okym ? -(double)gw[j][2] : 0.0;
        const double w_mm = okxm && okym ? (double)gw[j][3] : 0.0;
        d0 = __builtin_fma(w_pp, (double)r_pp.x, d0);
        d1 = __builtin_fma(w_pp, (double)r_pp.y, d1);
        d0 = __builtin_fma(w_mp, (double)r_mp.x, d0);
        d1 = __builtin_fma(w_mp, (double)r_mp.y, d1);
        d0 = __builtin_fma(w_pm, (double)r_pm.x, d0);
        d1 = __builtin_fma(w_pm, (double)r_pm.y, d1);
        d0 = __builtin_fma(w_mm, (double)r_mm.x, d0);
        d1 = __builtin_fma(w_mm, (double)r_mm.y, d1);
    }
    // one 16-byte non-temporal store per lane (the last column and row get zero here)
    typedef double dbl2 __attribute__((ext_vector_type(2)));
    dbl2 d;
    d.x = d0;
    d.y = d1;
    __builtin_nontemporal_store(d, reinterpret_cast<dbl2 *>(k.Dr + (int64_t)yv * k.W + xv));
}

// (1) The interleaved launch.  Blocks reach the 8 XCDs round-robin by index; XCD x receives
// one contiguous range of the deposit tiles (in comb order) and one of the border blocks,
// and its i-th block is a border block exactly when floor((i+1) nb / t) > floor(i nb / t)
// (nb border and t blocks in all on that XCD), which spreads the border blocks evenly
// between the deposit blocks.  The two kinds use different units (arithmetic against memory
// latency), so each covers the other's stalls.  Every block index maps to one work item or
// none (the grid is rounded up to whole rounds of 8).
template <int S>
__global__ void __launch_bounds__(kBlock) border_deposit_kernel(BwdK k) {
    constexpr uint32_t kXcd = 8;
    const uint32_t xcd = blockIdx.x % kXcd, i = blockIdx.x / kXcd;
    const uint32_t qd = k.ndep / kXcd, rd = k.ndep % kXcd;
    const uint32_t qb = k.nbor / kXcd, rb = k.nbor % kXcd;
    const uint32_t cd = qd + (xcd < rd ? 1u : 0u), cb = qb + (xcd < rb ? 1u : 0u);
    const uint32_t t = cd + cb;
    if (i >= t) return;
    const uint32_t nb0 = (uint32_t)((uint64_t)i * cb / t);
    const uint32_t nb1 = (uint32_t)((uint64_t)(i + 1) * cb / t);
    if (nb1 > nb0)
        border_block<S>(k, (int)(xcd * qb + min(xcd, rb) + nb0));
    else
        deposit_block<S>(k, xcd * qd + min(xcd, rd) + (i - nb0));
}

// (3) The last column and row of the deposits (virtual column 0 and row 0): only clamped
// ranges reach them, through Rb, Cb and (for the bottom-right corner) the total K.
// Overwrites the zeros that (1) left there.
template <int S>
__global__ void __launch_bounds__(kBlock) edge_deposit_kernel(BwdK k) {
    const int e = (int)(blockIdx.x * kBlock + threadIdx.x);
    if (e >= k.W + k.H - 1) return;
    const int xv = e < k.W ? e : 0, yv = e < k.W ? 0 : e - k.W + 1;
    const int cx = k.W - 1 - xv, cy = k.H - 1 - yv;
    const bool lastx = xv == 0, lasty = yv == 0;
    // every load of every field first, at clamped in-range indices (a term that does not
    // exist is selected away), then the terms in a fixed order
    double t[S][4][2];
#pragma unroll
    for (int j = 0; j < S; ++j) {
        const int rx = k.p.rx[j], ry = k.p.ry[j];
        const int pxp = cx - rx, pxm = cx + rx + 1, pyp = cy - ry, pym = cy + ry + 1;
        const double *R0 = k.Rb + (int64_t)j * k.H, *R1 = k.Rb + ((int64_t)S + j) * k.H;
        const double *C0 = k.Cb + (int64_t)j * k.W, *C1 = k.Cb + ((int64_t)S + j) * k.W;
        const int iy0 = min(max(pyp, 0), k.H - 1), ix0 = min(max(pxp, 0), k.W - 1);
        const int ix1 = min(pxm, k.W - 1), iy1 = min(pym, k.H - 1);
        t[j][0][0] = R0[iy0];
        t[j][0][1] = R1[iy0];
        t[j][1][0] = C0[ix0];
        t[j][1][1] = C1[ix0];
        t[j][2][0] = C0[ix1];
        t[j][2][1] = C1[ix1];
        t[j][3][0] = R0[iy1];
        t[j][3][1] = R1[iy1];
    }
    double d0 = 0.0, d1 = 0.0;
#pragma unroll
    for (int j = 0; j < S; ++j) {
        const int rx = k.p.rx[j], ry = k.p.ry[j];
        const int pxp = cx - rx, pxm = cx + rx + 1, pyp = cy - ry, pym = cy + ry + 1;
        const bool okxm = pxm <= k.W - 1, okym = pym <= k.H - 1;
        if (lastx && !lasty && pyp >= 0) { d0 += t[j][0][0]; d1 += t[j][0][1]; }
        if (lasty && !lastx && pxp >= 0) { d0 += t[j][1][0]; d1 += t[j][1][1]; }
        if (lastx && lasty) {   // the corner totals from their parts, in a fixed order
            double k0 = k.K[j * kKParts], k1 = k.K[(S + j) * kKParts];
            for (int u = 1; u < kKParts; ++u) {
                k0 += k.K[j * kKParts + u];
                k1 += k.K[(S + j) * kKParts + u];
            }
            d0 += k0;
            d1 += k1;
        }
        if (lasty && okxm) { d0 -= t[j][2][0]; d1 -= t[j][2][1]; }
        if (lastx && okym) { d0 -= t[j][3][0]; d1 -= t[j][3][1]; }
    }
    k.Dr[(int64_t)yv * k.W + xv] = make_double2(d0, d1);
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
    b.K = take(2 * kS * kKParts * sizeof(double));
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
    k.gp = a.grad_params;
    k.K = reinterpret_cast<double *>(w + plan.K);
    k.tiles_x = (a.W + kWave - 1) / kWave;
    k.p4 = plan.p4;
    k.teeth = plan.teeth;
    k.nchunks = plan.nchunks;
    k.chunk = plan.chunk;
    k.ndep = (uint32_t)plan.nblocks;
    k.nbor = (uint32_t)(k.tiles_x * plan.nchunks);
    const int S = a.p.n_scales;
    // XCD 0 holds the most work items: ceil of each kind's share
    const uint32_t per_xcd = (k.ndep + 7) / 8 + (k.nbor + 7) / 8;
    const unsigned nfused = 8u * per_xcd;
    switch (S) {
#define TM_FUSED(n)                                                                             \
    case n:                                                                                    \
        hipLaunchKernelGGL(border_deposit_kernel<n>, dim3(nfused), dim3(kBlock), 0, s, k);     \
        break;
        TM_FUSED(1) TM_FUSED(2) TM_FUSED(3) TM_FUSED(4)
        TM_FUSED(5) TM_FUSED(6) TM_FUSED(7) TM_FUSED(8)
#undef TM_FUSED
        default: return hipErrorInvalidValue;
    }
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    const unsigned nred =
        (unsigned)(((int64_t)2 * S * (a.H + a.W) + kBlock - 1) / kBlock) + 2 * S * kKParts + 1;
    hipLaunchKernelGGL(border_reduce_kernel, dim3(nred), dim3(kBlock), 0, s, k);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    const unsigned nedge = (unsigned)((a.W + a.H - 1 + kBlock - 1) / kBlock);
    switch (S) {
#define TM_EDGE(n)                                                                              \
    case n:                                                                                    \
        hipLaunchKernelGGL(edge_deposit_kernel<n>, dim3(nedge), dim3(kBlock), 0, s, k);        \
        break;
        TM_EDGE(1) TM_EDGE(2) TM_EDGE(3) TM_EDGE(4)
        TM_EDGE(5) TM_EDGE(6) TM_EDGE(7) TM_EDGE(8)
#undef TM_EDGE
        default: return hipErrorInvalidValue;
    }
    if ((e = hipGetLastError()) != hipSuccess) return e;
    return launch_suffix_adjoint(k.Dr, a.W, a.v, a.ld_v, a.H, a.W, a.grad_v, a.ld_gv,
                                 plan.scan_plan, w + plan.scan, s, a.log_chain);
}

}  // namespace tmo
