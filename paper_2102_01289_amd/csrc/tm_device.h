// tm_device.h -- device helpers shared by the HIP kernels of the tone-mapping library:
// wave64 prefix primitives built on GFX9 DPP, error-free FP32 transforms, the accumulator
// types of the three integral-image precisions, and the table-layout conventions.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace tmo {

constexpr int kWave = 64;

// Global-address-space view of a pointer.  Pointers that a kernel reads from a descriptor in
// memory (the batched launches) are generic to the compiler, which then emits flat loads
// and stores with 64-bit lane addresses; through this view it emits global memory
// instructions, including the scalar-base + 32-bit-offset form.
// (The host compilation pass of a .hip file parses device code but has no such address
// space; there the view is the plain pointer.)
#if defined(__HIP_DEVICE_COMPILE__)
#define TM_GLOBAL __attribute__((address_space(1)))
#else
#define TM_GLOBAL
#endif
template <typename T>
__device__ __forceinline__ const TM_GLOBAL T *gptr(const T *p) {
    return (const TM_GLOBAL T *)p;
}
template <typename T>
__device__ __forceinline__ TM_GLOBAL T *gptr(T *p) {
    return (TM_GLOBAL T *)p;
}

// Load at a wave-uniform row base plus a per-lane unsigned 32-bit byte offset, the form
// the global_load "saddr + voffset" addressing takes directly (no 64-bit lane arithmetic).
template <typename T>
__device__ __forceinline__ T load_at(const char *row, uint32_t off) {
    return *reinterpret_cast<const TM_GLOBAL T *>(gptr(row) + off);
}

// ------------------------------------------------------------------ DPP moves (GFX9)
// dpp_ctrl encodings: row_shr:n = 0x110 + n, wave_shr:1 = 0x138, row_bcast:15 = 0x142,
// row_bcast:31 = 0x143.  Lanes whose source is outside the row/wave, or that row_mask /
// bank_mask switch off, receive 0 (old = 0, bound_ctrl set), which is the identity of
// every scan operator used here.
template <int CTRL, int ROW_MASK = 0xf, int BANK_MASK = 0xf>
__device__ __forceinline__ uint32_t dpp32(uint32_t v) {
    return (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, CTRL, ROW_MASK, BANK_MASK, true);
}

// Shift-by-DPP of the value types the scans carry.
template <int CTRL, int RM = 0xf, int BM = 0xf>
__device__ __forceinline__ float dpp(float v) {
    return __uint_as_float(dpp32<CTRL, RM, BM>(__float_as_uint(v)));
}
template <int CTRL, int RM = 0xf, int BM = 0xf>
__device__ __forceinline__ uint32_t dpp(uint32_t v) {
    return dpp32<CTRL, RM, BM>(v);
}
template <int CTRL, int RM = 0xf, int BM = 0xf>
__device__ __forceinline__ double dpp(double v) {
    uint64_t b = __double_as_longlong(v);
    uint32_t lo = dpp32<CTRL, RM, BM>((uint32_t)b);
    uint32_t hi = dpp32<CTRL, RM, BM>((uint32_t)(b >> 32));
    return __longlong_as_double((long long)(((uint64_t)hi << 32) | lo));
}

// ------------------------------------------------------------------ compensated FP32
// Unevaluated sum hi + lo of two FP32 values.
struct f2 {
    float hi, lo;
};

template <int CTRL, int RM = 0xf, int BM = 0xf>
__device__ __forceinline__ f2 dpp(f2 v) {
    return f2{dpp<CTRL, RM, BM>(v.hi), dpp<CTRL, RM, BM>(v.lo)};
}

// Knuth's TwoSum: s + e == a + b exactly.
__device__ __forceinline__ f2 two_sum(float a, float b) {
    float s = a + b;
    float bb = s - a;
    float e = (a - (s - bb)) + (b - bb);
    return f2{s, e};
}
// Dekker's FastTwoSum (|a| >= |b|).
__device__ __forceinline__ f2 fast_two_sum(float a, float b) {
    float s = a + b;
    return f2{s, b - (s - a)};
}
// a - b exactly as a pair.
__device__ __forceinline__ f2 two_diff(float a, float b) { return two_sum(a, -b); }
// a * a exactly as a pair (fused multiply-add recovers the rounding error).
__device__ __forceinline__ f2 two_sqr(float a) {
    float p = a * a;
    return f2{p, __builtin_fmaf(a, a, -p)};
}
// Sum of two pairs: TwoSum of the leading parts, the trailing parts added in, renormalised.
// Error below 2^-44 of |a| + |b|.
__device__ __forceinline__ f2 add22(f2 a, f2 b) {
    f2 s = two_sum(a.hi, b.hi);
    s.lo += a.lo + b.lo;
    return fast_two_sum(s.hi, s.lo);
}

// ------------------------------------------------------------------ accumulators
// Accumulator of one integral-image quantity for each tm_sat_prec:
//   T        the running-sum type; Store the table entry component type.
//   of_v(v, mu) / of_v2(v, mu2): the per-pixel term (v or v^2, minus the offset for C32X2).
enum SatPrec { kF32 = 0, kC32x2 = 1, kF64 = 2 };

template <int P>
struct Acc;

template <>
struct Acc<kF32> {
    using T = float;
    __device__ static T zero() { return 0.f; }
    __device__ static T add(T a, T b) { return a + b; }
    __device__ static T of_v(float v, float) { return v; }
    __device__ static T of_v2(float v, float) { return v * v; }
};

template <>
struct Acc<kC32x2> {
    using T = f2;
    __device__ static T zero() { return f2{0.f, 0.f}; }
    __device__ static T add(T a, T b) { return add22(a, b); }
    __device__ static T of_v(float v, float mu) { return two_diff(v, mu); }
    __device__ static T of_v2(float v, float mu2) {
        f2 sq = two_sqr(v);
        f2 d = two_diff(sq.hi, mu2);
        d.lo += sq.lo;
        return fast_two_sum(d.hi, d.lo);
    }
};

template <>
struct Acc<kF64> {
    using T = double;
    __device__ static T zero() { return 0.0; }
    __device__ static T add(T a, T b) { return a + b; }
    __device__ static T of_v(float v, float) { return (double)v; }
    __device__ static T of_v2(float v, float) { return (double)v * (double)v; }
};

struct AddU32 {
    __device__ static uint32_t zero() { return 0u; }
    __device__ static uint32_t add(uint32_t a, uint32_t b) { return a + b; }
};

// ------------------------------------------------------------------ wave64 scans
// Inclusive prefix over the 64 lanes with Op::add (Hillis-Steele inside each 16-lane row
// with row_shr 1/2/4/8, then row_bcast:15 and row_bcast:31 across rows).
template <class Op, class T>
__device__ __forceinline__ T wave_inclusive(T v) {
    v = Op::add(v, dpp<0x111>(v));
    v = Op::add(v, dpp<0x112>(v));
    v = Op::add(v, dpp<0x114>(v));
    v = Op::add(v, dpp<0x118>(v));
    v = Op::add(v, dpp<0x142, 0xa>(v));
    v = Op::add(v, dpp<0x143, 0xc>(v));
    return v;
}
// The value of lane l-1 (lane 0 receives zero): turns an inclusive scan into an exclusive one.
template <class T>
__device__ __forceinline__ T wave_shr1(T v) {
    return dpp<0x138>(v);
}

__device__ __forceinline__ float readlane(float v, int l) {
    return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), l));
}
__device__ __forceinline__ uint32_t readlane(uint32_t v, int l) {
    return (uint32_t)__builtin_amdgcn_readlane((int)v, l);
}
__device__ __forceinline__ double readlane(double v, int l) {
    uint64_t b = __double_as_longlong(v);
    uint32_t lo = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)b, l);
    uint32_t hi = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)(b >> 32), l);
    return __longlong_as_double((long long)(((uint64_t)hi << 32) | lo));
}
__device__ __forceinline__ f2 readlane(f2 v, int l) {
    return f2{readlane(v.hi, l), readlane(v.lo, l)};
}

// Sum over the wave (same value in every lane).
template <class Op, class T>
__device__ __forceinline__ T wave_sum(T v) {
    return readlane(wave_inclusive<Op>(v), kWave - 1);
}

// FP64 sums over the wave of a and b at once.  gfx950's permlane32_swap trades lanes 32-63 of its
// first operand for lanes 0-31 of its second, so one exchange (two per FP64 value) and one
// addition leave the half-sums of a in lanes 0-31 and those of b in lanes 32-63; four row
// shifts and one row broadcast finish both.  A fixed order of additions; half the steps of
// two separate wave sums.
__device__ __forceinline__ void wave_sum2(double a, double b, double &sa, double &sb) {
    const uint64_t ua = (uint64_t)__double_as_longlong(a);
    const uint64_t ub = (uint64_t)__double_as_longlong(b);
    const auto lo = __builtin_amdgcn_permlane32_swap((uint32_t)ua, (uint32_t)ub, false, false);
    const auto hi =
        __builtin_amdgcn_permlane32_swap((uint32_t)(ua >> 32), (uint32_t)(ub >> 32), false, false);
    const double x = __longlong_as_double((long long)(((uint64_t)hi[0] << 32) | lo[0]));
    const double y = __longlong_as_double((long long)(((uint64_t)hi[1] << 32) | lo[1]));
    double v = x + y;
    v += dpp<0x111>(v);
    v += dpp<0x112>(v);
    v += dpp<0x114>(v);
    v += dpp<0x118>(v);
    v += dpp<0x142, 0xa>(v);
    sa = readlane(v, 31);
    sb = readlane(v, 63);
}

__device__ __forceinline__ int lane_id() { return (int)(threadIdx.x & (kWave - 1)); }

// Index of the calling wave inside its block, as a wave-uniform (scalar) value.
__device__ __forceinline__ int wave_id() {
    return __builtin_amdgcn_readfirstlane((int)(threadIdx.x / kWave));
}

// ------------------------------------------------------------------ blockIdx -> tile
// Workgroups are dispatched to the 8 XCDs round-robin by block index.  Remap so that each
// XCD receives one contiguous range of tiles, keeping neighbouring tiles (which share
// table rows) in one XCD's L2.  The map is a bijection on [0, nblocks).
__device__ __forceinline__ uint32_t xcd_tile(uint32_t b, uint32_t nblocks) {
    constexpr uint32_t kXcd = 8;
    uint32_t q = nblocks / kXcd, r = nblocks % kXcd;
    uint32_t k = b % kXcd, i = b / kXcd;
    return k * q + (k < r ? k : r) + i;
}

// Comb schedule of the per-pixel kernels that read window corners: block b covers column
// tile tx and row group rg, ordered by phase inside a period of p4 row groups, then tooth,
// then column tile (see comb_params).
__device__ __forceinline__ void comb_map(uint32_t b, int tiles_x, int p4, int teeth, int &tx,
                                         int &rg) {
    tx = (int)(b % (uint32_t)tiles_x);
    const uint32_t r = b / (uint32_t)tiles_x;
    rg = (int)(r % (uint32_t)teeth) * p4 + (int)(r / (uint32_t)teeth);
}

// Batched launches walk one flattened list of work items spanning a range of images; the
// image of item g is the last i with prefix[i] <= g (prefix has count+1 entries and
// prefix[0] <= g).
__device__ __forceinline__ int find_image(const int64_t *prefix, int count, int64_t g) {
    int lo = 0, hi = count - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (prefix[mid] <= g) lo = mid; else hi = mid - 1;
    }
    return lo;
}

}  // namespace tmo
