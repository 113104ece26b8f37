// tm_prologue.hip -- stage a1: luminance (Eq. 11) and the image statistics the later stages
// need: min / max of the luminance (range of the log-domain bins, Section II-A), the bin
// edges, and the FP32 mean offsets of the compensated integral images.
//
// One streaming pass reads RGB (or luminance), writes luminance and leaves per-block
// partials (min, max, FP64 sums of v and v^2); a one-block finalize kernel reduces the
// partials in a fixed order (bit-reproducible) and places the bin edges.
#include <float.h>
#include <math.h>

#include <mutex>

#include "tm_device.h"
#include "tm_internal.h"

namespace tmo {

namespace {

constexpr int kBlock = 256;
constexpr int kSeg = kBlock * 4;   // pixels of one row segment handled by a block step

// Eq. 11 in FP32, left to right with fused multiply-adds.
__device__ __forceinline__ float luminance(float r, float g, float b) {
    float t = 0.2126f * r;
    t = __builtin_fmaf(0.7152f, g, t);
    return __builtin_fmaf(0.0722f, b, t);
}

struct Stat {
    float mn, mx;
    double s1, s2;
};

__device__ __forceinline__ void stat_add(Stat &a, float v) {
    a.mn = fminf(a.mn, v);
    a.mx = fmaxf(a.mx, v);
    double d = (double)v;
    a.s1 += d;
    a.s2 += d * d;
}

// Range of v, sums of l (the log-domain variant's prologue).
__device__ __forceinline__ void stat_add_split(Stat &a, float v, float l) {
    a.mn = fminf(a.mn, v);
    a.mx = fmaxf(a.mx, v);
    double d = (double)l;
    a.s1 += d;
    a.s2 += d * d;
}

__device__ __forceinline__ Stat stat_merge(Stat a, Stat b) {
    return Stat{fminf(a.mn, b.mn), fmaxf(a.mx, b.mx), a.s1 + b.s1, a.s2 + b.s2};
}

// Deterministic block reduction (butterfly within waves, fixed order across waves).
__device__ Stat block_reduce(Stat st) {
    for (int m = 32; m >= 1; m >>= 1) {
        Stat o{__shfl_xor(st.mn, m), __shfl_xor(st.mx, m), __shfl_xor(st.s1, m),
               __shfl_xor(st.s2, m)};
        st = stat_merge(st, o);
    }
    __shared__ Stat sh[kBlock / kWave];
    const int w = threadIdx.x / kWave;
    if (lane_id() == 0) sh[w] = st;
    __syncthreads();
    Stat r = sh[0];
    for (int i = 1; i < kBlock / kWave; ++i) r = stat_merge(r, sh[i]);
    return r;
}

// One reduction part of one image: row segments part, part + nparts, ... (so the partials,
// and hence the statistics, do not depend on how parts are scheduled).
// LOG, luminance input: the pass writes l = ln(max(v, FLT_MIN)) to lum_out and the
// statistics are those of l.  LOG, colour input: the pass writes the luminance to lum_out and
// l to log_out (when given); the range is the luminance's, the sums are l's.
template <bool FROM_RGB, bool STATS, bool LOG = false>
__device__ void stats_part(const StatsK &k, int part, int nparts) {
    Stat st{INFINITY, -INFINITY, 0.0, 0.0};
    const int H = k.H, W = k.W;
    const int segs_per_row = (W + kSeg - 1) / kSeg;
    const int64_t nseg = (int64_t)H * segs_per_row;
    for (int64_t seg = part; seg < nseg; seg += nparts) {
        const int y = (int)(seg / segs_per_row);
        const int x = (int)(seg % segs_per_row) * kSeg + (int)threadIdx.x * 4;
        if (x >= W) continue;
        float v[4];
        const bool full = x + 4 <= W;
        if (FROM_RGB) {
            const float *R = k.rgb + (int64_t)y * k.ld_rgb + x;
            const float *G = R + k.ch_stride;
            const float *B = G + k.ch_stride;
            if (full && k.vec_in) {
                // read once: non-temporal, so the colour planes do not displace cached tables
                typedef float f4v __attribute__((ext_vector_type(4)));
                const f4v r = __builtin_nontemporal_load(reinterpret_cast<const f4v *>(R));
                const f4v g = __builtin_nontemporal_load(reinterpret_cast<const f4v *>(G));
                const f4v b = __builtin_nontemporal_load(reinterpret_cast<const f4v *>(B));
                v[0] = luminance(r.x, g.x, b.x);
                v[1] = luminance(r.y, g.y, b.y);
                v[2] = luminance(r.z, g.z, b.z);
                v[3] = luminance(r.w, g.w, b.w);
            } else {
                for (int i = 0; i < 4; ++i)
                    v[i] = (x + i < W) ? luminance(R[i], G[i], B[i]) : 0.f;
            }
            float *o = k.lum_out + (int64_t)y * k.ld_out + x;
            if (full && k.vec_out) {
                *reinterpret_cast<float4 *>(o) = make_float4(v[0], v[1], v[2], v[3]);
            } else {
                for (int i = 0; i < 4; ++i)
                    if (x + i < W) o[i] = v[i];
            }
            if (LOG) {
                float l[4];
                for (int i = 0; i < 4; ++i) l[i] = logf(fmaxf(v[i], FLT_MIN));
                if (k.log_out) {   // the plane is optional: the sums are always formed
                    float *ol = k.log_out + (int64_t)y * k.ld_log + x;
                    if (full && k.vec_log) {
                        *reinterpret_cast<float4 *>(ol) = make_float4(l[0], l[1], l[2], l[3]);
                    } else {
                        for (int i = 0; i < 4; ++i)
                            if (x + i < W) ol[i] = l[i];
                    }
                }
                if (STATS) {
                    for (int i = 0; i < 4; ++i)
                        if (x + i < W) stat_add_split(st, v[i], l[i]);
                }
                continue;
            }
        } else {
            const float *L = k.lum_in + (int64_t)y * k.ld_in + x;
            if (full && k.vec_in) {
                float4 l = *reinterpret_cast<const float4 *>(L);
                v[0] = l.x; v[1] = l.y; v[2] = l.z; v[3] = l.w;
            } else {
                for (int i = 0; i < 4; ++i) v[i] = (x + i < W) ? L[i] : 0.f;
            }
            if (LOG) {
                for (int i = 0; i < 4; ++i) v[i] = logf(fmaxf(v[i], FLT_MIN));
                if (k.lum_out) {   // the plane is optional: the statistics are always formed
                    float *o = k.lum_out + (int64_t)y * k.ld_out + x;
                    if (full && k.vec_out) {
                        *reinterpret_cast<float4 *>(o) = make_float4(v[0], v[1], v[2], v[3]);
                    } else {
                        for (int i = 0; i < 4; ++i)
                            if (x + i < W) o[i] = v[i];
                    }
                }
            }
        }
        if (STATS) {
            for (int i = 0; i < 4; ++i)
                if (x + i < W) stat_add(st, v[i]);
        }
    }
    if (STATS) {
        Stat r = block_reduce(st);
        if (threadIdx.x == 0) {
            StatsPartial p;
            p.mn = r.mn;
            p.mx = r.mx;
            p.s1 = r.s1;
            p.s2 = r.s2;
            p.pad = 0.0;
            k.partials[part] = p;
        }
    }
}

template <bool FROM_RGB, bool STATS, bool LOG = false>
__global__ void __launch_bounds__(kBlock) lum_stats_kernel(StatsK k) {
    stats_part<FROM_RGB, STATS, LOG>(k, blockIdx.x, gridDim.x);
}

// Batched prologue over images [0, count) of ks: item g in [prefix[0], prefix[count]) is part
// (g - prefix[i]) of image i.  LOG: the log-domain variant's statistics (range of the
// luminance, sums of its log plane; no plane is written).
template <bool LOG>
__global__ void __launch_bounds__(kBlock) lum_stats_batch(const StatsK *__restrict__ ks,
                                                          const int64_t *__restrict__ prefix,
                                                          int count) {
    const int64_t total = prefix[count];
    int64_t g = prefix[0] + blockIdx.x;
    int i = g < total ? find_image(prefix, count, g) : 0;   // advances with g
    for (; g < total; g += gridDim.x) {
        while (g >= prefix[i + 1]) ++i;
        stats_part<true, true, LOG>(ks[i], (int)(g - prefix[i]), ks[i].nparts);
        __syncthreads();
    }
}

// ---------------------------------------------------------------- exact edge placement
// Unsigned big integers (little-endian 32-bit limbs), enough for x^n with 24-bit x and
// n <= 256 shifted by up to n + 2 bits.
constexpr int kLimbs = 208;
struct Big {
    uint32_t w[kLimbs];
    int len;
};

__device__ void big_one(Big &a) {
    a.w[0] = 1u;
    a.len = 1;
}
__device__ void big_mul_small(Big &a, uint32_t m) {
    uint64_t carry = 0;
    for (int i = 0; i < a.len; ++i) {
        uint64_t t = (uint64_t)a.w[i] * m + carry;
        a.w[i] = (uint32_t)t;
        carry = t >> 32;
    }
    if (carry && a.len < kLimbs) a.w[a.len++] = (uint32_t)carry;
}
__device__ void big_shl(Big &a, int d) {
    const int ws = d >> 5, bs = d & 31;
    int nl = a.len + ws + 1;
    if (nl > kLimbs) nl = kLimbs;
    for (int i = nl - 1; i >= 0; --i) {
        const int s = i - ws;
        uint64_t hi = (s >= 0 && s < a.len) ? a.w[s] : 0u;
        uint64_t lo = (s - 1 >= 0 && s - 1 < a.len) ? a.w[s - 1] : 0u;
        a.w[i] = bs ? (uint32_t)((hi << bs) | (lo >> (32 - bs))) : (uint32_t)hi;
    }
    a.len = nl;
}
__device__ int big_cmp(Big &a, Big &b) {
    while (a.len > 1 && a.w[a.len - 1] == 0) --a.len;
    while (b.len > 1 && b.w[b.len - 1] == 0) --b.len;
    if (a.len != b.len) return a.len < b.len ? -1 : 1;
    for (int i = a.len - 1; i >= 0; --i)
        if (a.w[i] != b.w[i]) return a.w[i] < b.w[i] ? -1 : 1;
    return 0;
}

// x = m * 2^e for a positive finite FP32 x (m < 2^24).
__device__ void f32_split(float x, uint32_t &m, int &e) {
    const uint32_t bits = __float_as_uint(x);
    const uint32_t be = (bits >> 23) & 0xffu;
    if (be == 0) {
        m = bits & 0x7fffffu;
        e = -149;
    } else {
        m = (bits & 0x7fffffu) | 0x800000u;
        e = (int)be - 150;
    }
}

// c^n >= a^(n-k) b^k, exactly (a, b, c positive finite FP32).
__device__ bool pow_ge(float c, int n, int k, float a, float b, Big &X, Big &Y) {
    uint32_t mc, ma, mb;
    int ec, ea, eb;
    f32_split(c, mc, ec);
    f32_split(a, ma, ea);
    f32_split(b, mb, eb);
    big_one(X);
    for (int i = 0; i < n; ++i) big_mul_small(X, mc);
    big_one(Y);
    for (int i = 0; i < n - k; ++i) big_mul_small(Y, ma);
    for (int i = 0; i < k; ++i) big_mul_small(Y, mb);
    const int d = ((n - k) * ea + k * eb) - n * ec;   // compare X vs Y * 2^d
    if (d >= 0)
        big_shl(Y, d);
    else
        big_shl(X, -d);
    return big_cmp(X, Y) >= 0;
}

__device__ __forceinline__ float f32_next(float x) { return __uint_as_float(__float_as_uint(x) + 1u); }
__device__ __forceinline__ float f32_prev(float x) { return __uint_as_float(__float_as_uint(x) - 1u); }

// Smallest FP32 >= i_min^(1-k/n) i_max^(k/n).  An FP64 estimate decides unless an FP32
// value lies within 2^-36 (relative) of it -- far wider than the estimate's own error --
// in which case the candidates are tested exactly with big integers.
__device__ float edge_value(int k, int n, float a, float b) {
    const double la = log((double)a), lb = log((double)b);
    const double e = exp(la + ((double)k / (double)n) * (lb - la));
    float c = (float)e;
    if (!(c < INFINITY)) c = FLT_MAX;
    if ((double)c < e) c = f32_next(c);
    const float p = f32_prev(c);
    const double tol = e * 0x1p-36;
    if ((double)c - e > tol && e - (double)p > tol) return c;
    Big X, Y;
    if (p > 0.f && pow_ge(p, n, k, a, b, X, Y)) return p;
    if (pow_ge(c, n, k, a, b, X, Y)) return c;
    return f32_next(c);
}

__device__ void finalize_body(const StatsK &k) {
    Stat st{INFINITY, -INFINITY, 0.0, 0.0};
    for (int i = threadIdx.x; i < k.nparts; i += kBlock) {
        StatsPartial p = k.partials[i];
        st = stat_merge(st, Stat{p.mn, p.mx, p.s1, p.s2});
    }
    const Stat r = block_reduce(st);
    const double np = (double)k.H * (double)k.W;
    if (threadIdx.x == 0) {
        if (k.offsets) {
            k.offsets[0] = (float)(r.s1 / np);
            k.offsets[1] = (float)(r.s2 / np);
        }
        if (k.minmax) {
            k.minmax[0] = r.mn;
            k.minmax[1] = r.mx;
        }
    }
    const float a = fmaxf(r.mn, FLT_MIN);
    const float b = r.mx;
    for (int kk = 1 + (int)threadIdx.x; kk < k.n_bins; kk += kBlock) {
        float e = INFINITY;
        if (b > a) e = edge_value(kk, k.n_bins, a, b);
        k.edges[kk - 1] = e;
    }
}

__global__ void __launch_bounds__(kBlock) stats_finalize_kernel(StatsK k) { finalize_body(k); }

__global__ void __launch_bounds__(kBlock) stats_finalize_batch(const StatsK *__restrict__ ks, int count) {
    for (int i = blockIdx.x; i < count; i += gridDim.x) {
        finalize_body(ks[i]);
        __syncthreads();
    }
}

}  // namespace

int stats_blocks(int H, int W) {
    const int64_t nseg = (int64_t)H * ((W + kSeg - 1) / kSeg);
    return (int)(nseg < kStatsMaxBlocks ? nseg : kStatsMaxBlocks);
}

static bool aligned16(const void *p) { return ((uintptr_t)p & 15u) == 0; }

StatsK make_statsk(const float *rgb, int64_t ch_stride, int64_t ld_rgb, const float *lum_in,
                   int64_t ld_in, float *lum_out, int64_t ld_out, int H, int W, int n_bins,
                   float *edges, float *offsets, float *minmax, StatsPartial *partials) {
    StatsK k{};
    k.rgb = rgb;
    k.ch_stride = ch_stride;
    k.ld_rgb = ld_rgb;
    k.lum_in = lum_in;
    k.ld_in = ld_in;
    k.lum_out = lum_out;
    k.ld_out = ld_out;
    k.H = H;
    k.W = W;
    k.vec_in = rgb ? (aligned16(rgb) && ld_rgb % 4 == 0 && ch_stride % 4 == 0)
                   : (aligned16(lum_in) && ld_in % 4 == 0);
    k.vec_out = lum_out && aligned16(lum_out) && ld_out % 4 == 0;
    k.nparts = stats_blocks(H, W);
    k.n_bins = n_bins;
    k.partials = partials;
    k.edges = edges;
    k.offsets = offsets;
    k.minmax = minmax;
    return k;
}

hipError_t launch_luminance(const float *rgb, int64_t ch_stride, int64_t ld_rgb, int H, int W,
                            float *lum, int64_t ld_lum, hipStream_t s) {
    StatsK k = make_statsk(rgb, ch_stride, ld_rgb, nullptr, 0, lum, ld_lum, H, W, 1, nullptr,
                           nullptr, nullptr, nullptr);
    const int64_t nseg = (int64_t)H * ((W + kSeg - 1) / kSeg);
    const int grid = (int)(nseg < 65536 ? nseg : 65536);
    hipLaunchKernelGGL((lum_stats_kernel<true, false>), dim3(grid), dim3(kBlock), 0, s, k);
    return hipGetLastError();
}

hipError_t launch_stats(const float *rgb, int64_t ch_stride, int64_t ld_rgb, const float *lum_in,
                        int64_t ld_lum_in, float *lum_out, int64_t ld_lum_out, int H, int W,
                        int n_bins, float *edges, float *offsets, float *minmax,
                        StatsPartial *partials, hipStream_t s) {
    StatsK k = make_statsk(rgb, ch_stride, ld_rgb, lum_in, ld_lum_in, lum_out, ld_lum_out, H, W,
                           n_bins, edges, offsets, minmax, partials);
    if (rgb)
        hipLaunchKernelGGL((lum_stats_kernel<true, true>), dim3(k.nparts), dim3(kBlock), 0, s, k);
    else
        hipLaunchKernelGGL((lum_stats_kernel<false, true>), dim3(k.nparts), dim3(kBlock), 0, s, k);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(stats_finalize_kernel, dim3(1), dim3(kBlock), 0, s, k);
    return hipGetLastError();
}

hipError_t launch_stats_log(const float *rgb, int64_t ch_stride, int64_t ld_rgb, float *lum,
                            int64_t ld_lum, float *logv, int64_t ld_log, int H, int W, int n_bins,
                            float *edges, float *offsets, float *minmax, StatsPartial *partials,
                            hipStream_t s) {
    StatsK k = make_statsk(rgb, ch_stride, ld_rgb, nullptr, 0, lum, ld_lum, H, W, n_bins, edges,
                           offsets, minmax, partials);
    k.log_out = logv;
    k.ld_log = ld_log;
    k.vec_log = aligned16(logv) && ld_log % 4 == 0;
    hipLaunchKernelGGL((lum_stats_kernel<true, true, true>), dim3(k.nparts), dim3(kBlock), 0, s,
                       k);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(stats_finalize_kernel, dim3(1), dim3(kBlock), 0, s, k);
    return hipGetLastError();
}

hipError_t launch_log_stats(const float *lum, int64_t ld_lum, float *logv, int64_t ld_log, int H,
                            int W, float *offsets, float *minmax, StatsPartial *partials,
                            hipStream_t s) {
    StatsK k = make_statsk(nullptr, 0, 0, lum, ld_lum, logv, ld_log, H, W, 1, nullptr, offsets,
                           minmax, partials);
    hipLaunchKernelGGL((lum_stats_kernel<false, true, true>), dim3(k.nparts), dim3(kBlock), 0, s,
                       k);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(stats_finalize_kernel, dim3(1), dim3(kBlock), 0, s, k);
    return hipGetLastError();
}

// The chain rule through the log plane of the log-domain variance variant: from the gradient
// with respect to l = ln(max(i, FLT_MIN)) the gradient with respect to i, grad_l / i where
// i > FLT_MIN and 0 where the floor constant is taken.  Elementwise (one correctly rounded
// FP32 division); gi may be gl itself, so neither is restrict-qualified.
namespace {
__global__ void __launch_bounds__(kBlock) log_chain_kernel(const float *lum, int64_t ld_lum,
                                                           const float *gl, int64_t ld_gl,
                                                           float *gi, int64_t ld_gi, int H,
                                                           int W) {
    const int x = blockIdx.x * kBlock + threadIdx.x;
    if (x >= W) return;
    for (int64_t y = blockIdx.y; y < H; y += gridDim.y) {
        const float v = lum[y * ld_lum + x];
        const float g = gl[y * ld_gl + x];
        gi[y * ld_gi + x] = v > FLT_MIN ? g / v : 0.f;
    }
}
}  // namespace

hipError_t launch_log_chain(const float *lum, int64_t ld_lum, const float *grad_l, int64_t ld_gl,
                            float *grad_i, int64_t ld_gi, int H, int W, hipStream_t s) {
    const dim3 grid((unsigned)((W + kBlock - 1) / kBlock), (unsigned)(H < 4096 ? H : 4096));
    hipLaunchKernelGGL(log_chain_kernel, grid, dim3(kBlock), 0, s, lum, ld_lum, grad_l, ld_gl,
                       grad_i, ld_gi, H, W);
    return hipGetLastError();
}

// ---------------------------------------------------------------- prologue without workspace
// The reduction partials of tm_prologue_noalloc live in this file-scope device array (one
// copy per GPU, for the life of the process).  Host code must not pass the array's name to a
// kernel: in host code it is only a stand-in for the symbol.  Its device address is looked up
// once per device with hipGetSymbolAddress, with that device current, and kept here.  Every
// partial the stats kernel needs is written by its own block before the finalize kernel reads
// it, so nothing has to be cleared between calls; calls that overlap on one GPU share the
// array and race.
static __device__ __align__(256) StatsPartial scratch[kPrologueScratchBytes / sizeof(StatsPartial)];
static_assert(kPrologueScratchBytes / sizeof(StatsPartial) >= (size_t)kStatsMaxBlocks,
              "the scratch array holds the largest number of partials");

namespace {
constexpr int kMaxDevices = 64;
std::mutex scratch_mu;
StatsPartial *scratch_ptr[kMaxDevices] = {};
}  // namespace

static hipError_t scratch_address(StatsPartial **out) {
    int dev = -1;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lock(scratch_mu);
    if (!scratch_ptr[dev]) {
        void *p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return e;
        if (!p) return hipErrorInvalidSymbol;
        scratch_ptr[dev] = static_cast<StatsPartial *>(p);
    }
    *out = scratch_ptr[dev];
    return hipSuccess;
}

hipError_t launch_stats_noalloc(const float *rgb, int64_t ch_stride, int64_t ld_rgb,
                                float *lum_out, int64_t ld_lum_out, int H, int W, int n_bins,
                                float *edges, float *offsets, float *minmax, hipStream_t s) {
    if ((size_t)stats_blocks(H, W) * sizeof(StatsPartial) > kPrologueScratchBytes)
        return hipErrorInvalidValue;
    StatsPartial *part = nullptr;
    const hipError_t e = scratch_address(&part);
    if (e != hipSuccess) return e;
    return launch_stats(rgb, ch_stride, ld_rgb, nullptr, 0, lum_out, ld_lum_out, H, W, n_bins,
                        edges, offsets, minmax, part, s);
}

hipError_t launch_stats_batch(const StatsK *ks, const int64_t *part_prefix, int count,
                              unsigned grid, hipStream_t s, bool log) {
    if (log)
        hipLaunchKernelGGL(lum_stats_batch<true>, dim3(grid), dim3(kBlock), 0, s, ks,
                           part_prefix, count);
    else
        hipLaunchKernelGGL(lum_stats_batch<false>, dim3(grid), dim3(kBlock), 0, s, ks,
                           part_prefix, count);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    const unsigned fg = (unsigned)(count < 4096 ? count : 4096);
    hipLaunchKernelGGL(stats_finalize_batch, dim3(fg), dim3(kBlock), 0, s, ks, count);
    return hipGetLastError();
}

}  // namespace tmo
