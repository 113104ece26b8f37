// tm_hdr.hip -- the multi-exposure front end: the step before the tone mapping in the
// paper's application (Section III), which recovers the WDR radiance image from several
// 8-bit exposures with the method of Debevec and Malik.
//
// For 8-bit values z, pixel i and exposure j of time dt_j, the inverse log response
// g(z) = ln f^-1(z) obeys g(Z_ij) = ln E_i + ln dt_j.  With the hat weight w(z) = z for
// z <= 127, 255 - z above:
//   * the response minimises sum_ij [w(Z_ij)(g(Z_ij) - ln E_i - ln dt_j)]^2
//     + lam sum_{z=1..254} [w(z)(g(z-1) - 2 g(z) + g(z+1))]^2 with g(128) = 0;
//   * the radiance map is ln E_i = sum_j w(Z_ij)(g(Z_ij) - ln dt_j) / sum_j w(Z_ij)
//     (the unweighted mean where every weight is 0).
//
// Response: the per-sample unknowns ln E_i enter the least squares only through their own
// rows, so they are eliminated in closed form (for sample i with a_j = w(Z_ij)^2 and
// S = sum a_j, the data term is (P g - t)^T Q (P g - t) with Q = diag(a) - a a^T / S, P the
// 0/1 map from g to the sample's values and t the log times).  That leaves one 255 x 255
// symmetric positive definite system for g (g(128) removed), assembled row by row and
// factored by Cholesky in FP64, one workgroup per colour channel.
// Merge: a streaming pass, 8 pixels per thread, the three response tables in LDS.
#include <math.h>

#include "tm_device.h"
#include "tm_internal.h"

namespace tmo {

namespace {

constexpr int kBlock = 256;
constexpr int kZ = 256;           // 8-bit code values
constexpr int kMid = 128;         // g(kMid) = 0 fixes the scale
constexpr int kN = kZ - 1;        // unknowns once g(kMid) is removed
constexpr int kLd = kZ;           // row pitch of the normal matrix (doubles)

__device__ __forceinline__ int hat(int z) { return z <= 127 ? z : 255 - z; }
// unknown index of g(z), z != kMid
__device__ __forceinline__ int col_of(int z) { return z < kMid ? z : z - 1; }

struct RespK {
    const uint8_t *stack;
    int64_t exp_stride, ch_stride, ld;
    int P, H, W;
    const int32_t *samples;
    int N;
    const float *log_dt;
    float lam;
    float *g;        // [3][256]
    double *ws;      // per channel: kN x kLd normal matrix, then kLd right-hand side
};

// One workgroup per channel (blockIdx.x).
__global__ void __launch_bounds__(kBlock) hdr_response_kernel(RespK k) {
    const int c = blockIdx.x;
    const int tid = threadIdx.x;
    double *M = k.ws + (size_t)c * (kN * kLd + kLd);
    double *rhs = M + kN * kLd;
    extern __shared__ uint8_t sh_z[];            // [N][P] sample values of this channel
    __shared__ double sh_t[16];
    __shared__ double sh_v[kLd];                 // pivot column / solve vector
    __shared__ int sh_bad;
    const int np = k.N * k.P;
    const int64_t hw = (int64_t)k.H * k.W;
    const uint8_t *base = k.stack + (int64_t)c * k.ch_stride;
    for (int q = tid; q < np; q += kBlock) {
        const int i = q / k.P, j = q % k.P;
        const int64_t s = k.samples[i];
        // an index outside the image marks the sample unusable (weight 0 in every exposure)
        uint8_t z = 0;
        if (s >= 0 && s < hw) z = base[(int64_t)j * k.exp_stride + (s / k.W) * k.ld + s % k.W];
        sh_z[q] = z;
    }
    if (tid < k.P) sh_t[tid] = (double)k.log_dt[tid];
    if (tid == 0) sh_bad = 0;
    for (int e = tid; e < kN * kLd; e += kBlock) M[e] = 0.0;   // coalesced, before the rows fill
    __syncthreads();

    // ---- assembly: thread z owns row col_of(z) of the reduced normal equations
    const int z = tid;
    if (z != kMid) {
        double *row = M + (size_t)col_of(z) * kLd;   // zeroed above
        double r = 0.0;
        // samples in chunks of 32: first the chunk's samples that hold code value z (a bit
        // mask), then only those, in sample order; a wave then runs as many rounds as its
        // busiest lane has hits, not one per sample that any lane hits
        for (int i0 = 0; i0 < k.N; i0 += 32) {
            const int nch = min(32, k.N - i0);
            uint32_t hits = 0u;
            for (int u = 0; u < nch; ++u) {
                const uint8_t *zu = sh_z + (i0 + u) * k.P;
                bool h = false;
                for (int j = 0; j < k.P; ++j) h |= zu[j] == z;
                hits |= h ? 1u << u : 0u;
            }
            while (hits) {
                const int i = i0 + __builtin_ctz(hits);
                hits &= hits - 1u;
                const uint8_t *zi = sh_z + i * k.P;
                double S = 0.0;
                for (int j = 0; j < k.P; ++j) {
                    const double w = (double)hat(zi[j]);
                    S += w * w;
                }
                if (S == 0.0) continue;
                for (int j = 0; j < k.P; ++j) {
                    if (zi[j] != z) continue;
                    const double wj = (double)hat(z);
                    const double aj = wj * wj;
                    for (int jj = 0; jj < k.P; ++jj) {
                        const double wjj = (double)hat(zi[jj]);
                        const double q = (jj == j ? aj : 0.0) - aj * (wjj * wjj) / S;
                        if (zi[jj] != kMid) row[col_of(zi[jj])] += q;
                        r += q * sh_t[jj];
                    }
                }
            }
        }
        // smoothness rows z' = z-1, z, z+1 (those in 1..254) with stencil (1, -2, 1)
        for (int zp = z - 1; zp <= z + 1; ++zp) {
            if (zp < 1 || zp > 254) continue;
            const double wz = (double)hat(zp);
            const double a = (double)k.lam * wz * wz;
            const double dz = zp == z ? -2.0 : 1.0;   // stencil weight of g(z) in row z'
            for (int cc = zp - 1; cc <= zp + 1; ++cc) {
                if (cc == kMid) continue;
                const double dc = cc == zp ? -2.0 : 1.0;
                row[col_of(cc)] += a * dz * dc;
            }
        }
        rhs[col_of(z)] = r;
    }
    __syncthreads();

    // ---- Cholesky M = L L^T in place (lower triangle), right-looking, in panels of kPb
    // columns.  Each entry receives the updates of the pivots before it one at a time, in
    // pivot order, exactly as in the unblocked elimination: a panel is factored in LDS, then
    // the trailing update applies the panel's pivots to every later entry in turn, reading
    // the entry from memory once per panel rather than once per pivot.  A pivot at or below
    // kN 2^-52 of the largest diagonal entry marks the system singular (rank-deficient up to
    // rounding).
    constexpr int kBatch = 16;                   // rows requested per round trip
    constexpr int kPb = 16;                      // panel width
    constexpr int kPs = kPb + 1;                 // LDS row pitch of the panel (odd)
    __shared__ double sh_tol;
    __shared__ double sh_pan[kN * kPs];          // the panel's columns, rows c0 .. kN-1
    __shared__ double sh_d[kLd];                 // diagonal of L
    if (tid == 0) {
        double mx = 0.0;
        for (int q = 0; q < kN; ++q) mx = fmax(mx, M[(size_t)q * kLd + q]);
        sh_tol = (double)kN * 0x1p-52 * mx;
    }
    __syncthreads();
    for (int c0 = 0; c0 < kN; c0 += kPb) {
        const int nc = min(kPb, kN - c0);        // columns of this panel
        const int nr = kN - c0;                  // its rows: c0 .. kN-1
        for (int e = tid; e < nr * kPb; e += kBlock) {
            const int r = e / kPb, q = e % kPb;
            if (q < nc) sh_pan[r * kPs + q] = M[(size_t)(c0 + r) * kLd + c0 + q];
        }
        __syncthreads();
        for (int q = 0; q < nc; ++q) {           // pivot p = c0 + q
            const int p = c0 + q;
            if (tid == 0) {
                const double d = sh_pan[q * kPs + q];
                if (!(d > sh_tol)) sh_bad = 1;
                const double sq = sqrt(d > 0.0 ? d : 1.0);
                sh_pan[q * kPs + q] = sq;
                sh_d[p] = sq;
            }
            __syncthreads();
            const double piv = sh_d[p];
            for (int r = q + 1 + tid; r < nr; r += kBlock) sh_pan[r * kPs + q] /= piv;
            __syncthreads();
            const int rest = nc - q - 1;         // later columns of the panel
            if (rest > 0) {
                for (int r = q + 1 + tid; r < nr; r += kBlock) {
                    const double lr = sh_pan[r * kPs + q];
                    for (int q2 = q + 1; q2 < nc && q2 <= r; ++q2)
                        sh_pan[r * kPs + q2] -= lr * sh_pan[q2 * kPs + q];
                }
            }
            __syncthreads();
        }
        // the factored panel's lower part back to memory (the solves read L there)
        for (int e = tid; e < nr * kPb; e += kBlock) {
            const int r = e / kPb, q = e % kPb;
            if (q < nc && r >= q) M[(size_t)(c0 + r) * kLd + c0 + q] = sh_pan[r * kPs + q];
        }
        // trailing update: thread t owns column j = c0 + nc + t (rows i >= j); every thread
        // walks the rows in the same order, so each LDS read is a broadcast
        const int j = c0 + nc + tid;
        if (j < kN) {
            double lj[kPb];
#pragma unroll
            for (int q = 0; q < kPb; ++q) lj[q] = q < nc ? sh_pan[(j - c0) * kPs + q] : 0.0;
            for (int i0 = c0 + nc; i0 < kN; i0 += kBatch) {
                // kBatch rows advance together, pivot by pivot (each entry's updates stay in
                // pivot order); rows past the matrix or above the diagonal are not stored
                double acc[kBatch];
#pragma unroll
                for (int u = 0; u < kBatch; ++u) {
                    const int i = i0 + u;
                    acc[u] = (i < kN && i >= j) ? M[(size_t)i * kLd + j] : 0.0;
                }
#pragma unroll
                for (int q = 0; q < kPb; ++q) {
                    if (q < nc) {
#pragma unroll
                        for (int u = 0; u < kBatch; ++u) {
                            const int r = min(i0 + u, kN - 1) - c0;
                            acc[u] -= sh_pan[r * kPs + q] * lj[q];
                        }
                    }
                }
#pragma unroll
                for (int u = 0; u < kBatch; ++u) {
                    const int i = i0 + u;
                    if (i < kN && i >= j) M[(size_t)i * kLd + j] = acc[u];
                }
            }
        }
        __syncthreads();
    }

    // ---- L y = rhs, then L^T x = y (in sh_v).  Thread i owns unknown i and requests the
    // entries of kBatch steps at once: row i of L going forward, column i going back.
    for (int q = tid; q < kN; q += kBlock) sh_v[q] = rhs[q];
    __syncthreads();
    const int ri = tid;   // kBlock >= kN: one unknown per thread
    for (int p0 = 0; p0 < kN; p0 += kBatch) {
        double lr[kBatch];
#pragma unroll
        for (int u = 0; u < kBatch; ++u) {
            const int p = p0 + u;
            lr[u] = (ri < kN && p < ri) ? M[(size_t)ri * kLd + p] : 0.0;
        }
#pragma unroll
        for (int u = 0; u < kBatch; ++u) {
            const int p = p0 + u;
            if (p >= kN) break;
            if (ri == p) sh_v[p] /= sh_d[p];
            __syncthreads();
            if (ri < kN && ri > p) sh_v[ri] -= lr[u] * sh_v[p];
        }
    }
    __syncthreads();
    for (int p0 = kN - 1; p0 >= 0; p0 -= kBatch) {
        double lc[kBatch];
#pragma unroll
        for (int u = 0; u < kBatch; ++u) {
            const int p = p0 - u;
            lc[u] = (p >= 0 && ri < p) ? M[(size_t)p * kLd + ri] : 0.0;
        }
#pragma unroll
        for (int u = 0; u < kBatch; ++u) {
            const int p = p0 - u;
            if (p < 0) break;
            if (ri == p) sh_v[p] /= sh_d[p];
            __syncthreads();
            if (ri < p) sh_v[ri] -= lc[u] * sh_v[p];
        }
    }
    __syncthreads();
    // a singular system (too few distinct sample values) leaves NaN
    const float nan = __builtin_nanf("");
    k.g[c * kZ + z] = sh_bad ? nan : (z == kMid ? 0.f : (float)sh_v[col_of(z)]);
}

struct MergeK {
    const uint8_t *stack;
    int64_t exp_stride, ch_stride, ld;
    int P, H, W;
    const float *log_dt;
    const float *g;
    float *out;
    int64_t ch_out, ld_out;
    int groups;      // kPx-pixel groups per row
    int vec;         // 8-byte loads and 16-byte stores are aligned for every full group
};

constexpr int kPx = 8;   // pixels per thread: one 8-byte load per exposure and channel
typedef float f32x4 __attribute__((ext_vector_type(4)));

// ln E of one pixel value set: weighted mean, or the plain mean where every weight is 0.
__device__ __forceinline__ float merge_px(float num, float den, float plain, float inv_p) {
    return den > 0.f ? num / den : plain * inv_p;
}

// The running sums of one group of kPx pixels: sum w (g - ln dt), sum w, sum (g - ln dt).
struct Acc8 {
    float num[kPx], den[kPx], plain[kPx];
};

__device__ __forceinline__ void acc_init(Acc8 &a) {
#pragma unroll
    for (int u = 0; u < kPx; ++u) a.num[u] = a.den[u] = a.plain[u] = 0.f;
}

// Add one exposure's eight values (packed in v, pixel u in byte u) to the sums of a group.
__device__ __forceinline__ void acc_add(Acc8 &a, const float *gc, float tj, const uint2 v) {
    const uint32_t wv[2] = {v.x, v.y};
#pragma unroll
    for (int u = 0; u < kPx; ++u) {
        const int zv = (int)((wv[u >> 2] >> (8 * (u & 3))) & 0xffu);
        const float term = gc[zv] - tj;
        const float w = (float)hat(zv);
        a.num[u] = __builtin_fmaf(w, term, a.num[u]);
        a.den[u] += w;
        a.plain[u] += term;
    }
}

// Eight values of one row; byte by byte (zero past the image edge, n < 8) where the group is
// not full or the row not 8-byte aligned.
__device__ __forceinline__ uint2 load8(const uint8_t *row, bool wide, int n) {
    if (wide) return *reinterpret_cast<const TM_GLOBAL uint2 *>(gptr(row));
    uint32_t w[2] = {0u, 0u};
    for (int u = 0; u < n; ++u) w[u >> 2] |= (uint32_t)row[u] << (8 * (u & 3));
    return make_uint2(w[0], w[1]);
}

// PC > 0: the exposure count is PC and every load of a full, aligned group is issued before
// any arithmetic (3 PC 8-byte loads in flight per thread); PC = 0: any count, the loads of
// one exposure at a time.
template <int PC>
__global__ void __launch_bounds__(kBlock) hdr_merge_kernel(MergeK k) {
    __shared__ float sh_g[3 * kZ];
    __shared__ float sh_t[16];
    for (int q = threadIdx.x; q < 3 * kZ; q += kBlock) sh_g[q] = k.g[q];
    if ((int)threadIdx.x < k.P) sh_t[threadIdx.x] = k.log_dt[threadIdx.x];
    __syncthreads();
    const int64_t item = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    const int64_t nitems = (int64_t)k.H * k.groups;
    if (item >= nitems) return;
    const int y = (int)(item / k.groups);
    const int x0 = (int)(item % k.groups) * kPx;
    const int n = min(kPx, k.W - x0);
    const int P = PC > 0 ? PC : k.P;
    const float inv_p = 1.0f / (float)P;
    const bool wide = n == kPx && k.vec;
    const uint8_t *src = k.stack + (int64_t)y * k.ld + x0;
    float *dst0 = k.out + (int64_t)y * k.ld_out + x0;
    auto finish = [&](int c, const Acc8 &a) {
        float e[kPx];
#pragma unroll
        for (int u = 0; u < kPx; ++u) e[u] = expf(merge_px(a.num[u], a.den[u], a.plain[u], inv_p));
        float *dst = dst0 + (int64_t)c * k.ch_out;
        if (wide) {
#pragma unroll
            for (int u = 0; u < kPx; u += 4) {
                const f32x4 q = {e[u], e[u + 1], e[u + 2], e[u + 3]};
                __builtin_nontemporal_store(q, reinterpret_cast<TM_GLOBAL f32x4 *>(gptr(dst + u)));
            }
        } else {
            for (int u = 0; u < n; ++u) dst[u] = e[u];
        }
    };
    if constexpr (PC > 0) {
        if (wide) {
            uint2 raw[3][PC];
#pragma unroll
            for (int c = 0; c < 3; ++c)
#pragma unroll
                for (int j = 0; j < PC; ++j)
                    raw[c][j] = *reinterpret_cast<const TM_GLOBAL uint2 *>(
                        gptr(src + (int64_t)c * k.ch_stride + (int64_t)j * k.exp_stride));
            // channel after channel: the barriers keep the scheduler from interleaving the
            // three channels' sums (which would hold all of them in registers at once)
#pragma unroll
            for (int c = 0; c < 3; ++c) {
                Acc8 a;
                acc_init(a);
#pragma unroll
                for (int j = 0; j < PC; ++j) acc_add(a, sh_g + c * kZ, sh_t[j], raw[c][j]);
                finish(c, a);
                __builtin_amdgcn_sched_barrier(0);
            }
            return;
        }
    }
    for (int c = 0; c < 3; ++c) {
        Acc8 a;
        acc_init(a);
        for (int j = 0; j < P; ++j)
            acc_add(a, sh_g + c * kZ, sh_t[j],
                    load8(src + (int64_t)c * k.ch_stride + (int64_t)j * k.exp_stride, wide, n));
        finish(c, a);
    }
}

}  // namespace

size_t hdr_response_ws_bytes() { return 3 * ((size_t)kN * kLd + kLd) * sizeof(double); }

hipError_t launch_hdr_response(const uint8_t *stack, int64_t exp_stride, int64_t ch_stride,
                               int64_t ld, int P, int H, int W, const int32_t *samples, int N,
                               const float *log_dt, float lam, float *g, void *ws,
                               hipStream_t s) {
    RespK k;
    k.stack = stack;
    k.exp_stride = exp_stride;
    k.ch_stride = ch_stride;
    k.ld = ld;
    k.P = P;
    k.H = H;
    k.W = W;
    k.samples = samples;
    k.N = N;
    k.log_dt = log_dt;
    k.lam = lam;
    k.g = g;
    k.ws = static_cast<double *>(ws);
    hipLaunchKernelGGL(hdr_response_kernel, dim3(3), dim3(kBlock), (size_t)N * P, s, k);
    return hipGetLastError();
}

hipError_t launch_hdr_merge(const uint8_t *stack, int64_t exp_stride, int64_t ch_stride,
                            int64_t ld, int P, int H, int W, const float *log_dt, const float *g,
                            float *out, int64_t ch_out, int64_t ld_out, hipStream_t s) {
    MergeK k;
    k.stack = stack;
    k.exp_stride = exp_stride;
    k.ch_stride = ch_stride;
    k.ld = ld;
    k.P = P;
    k.H = H;
    k.W = W;
    k.log_dt = log_dt;
    k.g = g;
    k.out = out;
    k.ch_out = ch_out;
    k.ld_out = ld_out;
    k.groups = (W + kPx - 1) / kPx;
    k.vec = ((uintptr_t)stack % 8 == 0) && exp_stride % 8 == 0 && ch_stride % 8 == 0 &&
            ld % 8 == 0 && ((uintptr_t)out % 16 == 0) && ch_out % 4 == 0 && ld_out % 4 == 0;
    const int64_t items = (int64_t)H * k.groups;
    const dim3 grid((unsigned)((items + kBlock - 1) / kBlock));
    switch (P) {
        case 2: hipLaunchKernelGGL(hdr_merge_kernel<2>, grid, dim3(kBlock), 0, s, k); break;
        case 3: hipLaunchKernelGGL(hdr_merge_kernel<3>, grid, dim3(kBlock), 0, s, k); break;
        case 4: hipLaunchKernelGGL(hdr_merge_kernel<4>, grid, dim3(kBlock), 0, s, k); break;
        case 5: hipLaunchKernelGGL(hdr_merge_kernel<5>, grid, dim3(kBlock), 0, s, k); break;
        default: hipLaunchKernelGGL(hdr_merge_kernel<0>, grid, dim3(kBlock), 0, s, k); break;
    }
    return hipGetLastError();
}

}  // namespace tmo
