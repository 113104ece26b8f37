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


template <int P>
struct Box;

template <>
struct Box<kF32> {
    // returns the window variance (clamped) from four float2 entries
    __device__ static float var(const FwdK &k, int64_t oA, int64_t oB, int64_t oC, int64_t oD,
                                int N) {
        const float2 *t = static_cast<const float2 *>(k.sat);
        const float2 A = t[oA], B = t[oB], C = t[oC], D = t[oD];
        const float s1 = (A.x + C.x) - (B.x + D.x);
        const float s2 = (A.y + C.y) - (B.y + D.y);
        const float inv = 1.0f / (float)N;
        const float m = s1 * inv;
        const float var = s2 * inv - m * m;
        return var > 0.f ? var : 0.f;
    }
};

template <>
struct Box<kC32x2> {
    __device__ static float var(const FwdK &k, int64_t oA, int64_t oB, int64_t oC, int64_t oD,
                                int N) {
        const float4 *t = static_cast<const float4 *>(k.sat);
        const float4 A = t[oA], B = t[oB], C = t[oC], D = t[oD];
        const double dN = (double)N;
        const double h1 = ((double)A.x + (double)C.x) - ((double)B.x + (double)D.x);
        const double l1 = ((double)A.y + (double)C.y) - ((double)B.y + (double)D.y);
        const double h2 = ((double)A.z + (double)C.z) - ((double)B.z + (double)D.z);
        const double l2 = ((double)A.w + (double)C.w) - ((double)B.w + (double)D.w);
        const double s1 = (h1 + l1) + dN * (double)k.offsets[0];
        const double s2 = (h2 + l2) + dN * (double)k.offsets[1];
        const double m = s1 / dN;
        const double var = s2 / dN - m * m;
        return var > 0.0 ? (float)var : 0.f;
    }
};

template <>
struct Box<kF64> {
    __device__ static float var(const FwdK &k, int64_t oA, int64_t oB, int64_t oC, int64_t oD,
                                int N) {
        const double2 *t = static_cast<const double2 *>(k.sat);
        const double2 A = t[oA], B = t[oB], C = t[oC], D = t[oD];
        const double dN = (double)N;
        const double s1 = (A.x + C.x) - (B.x + D.x);
        const double s2 = (A.y + C.y) - (B.y + D.y);
        const double m = s1 / dN;
        const double var = s2 / dN - m * m;
        return var > 0.0 ? (float)var : 0.f;
    }
};

// One 64 x 4 tile of one image.  sh_edges is the block's copy of the image's bin edges.
template <int P>
__device__ __forceinline__ void forward_tile(const FwdK &k, uint32_t tile, float *sh_edges) {
    const int ne = k.p.n_bins - 1;
    __syncthreads();   // the previous tile of this block may still read sh_edges
    for (int i = threadIdx.x; i < ne; i += kBlock) sh_edges[i] = k.edges[i];
    __syncthreads();

    const int tx = (int)(tile % (uint32_t)k.tiles_x), ty = (int)(tile / (uint32_t)k.tiles_x);
    const int x = tx * kWave + lane_id();
    const int y = ty * kRows + (int)(threadIdx.x / kWave);
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

    const float ldr = k.p.ld_max - k.p.ld_min;
    float num = 0.f, den = 0.f, lsum = 0.f;
    for (int j = 0; j < k.p.n_scales; ++j) {
        const int rx = k.p.rx[j], ry = k.p.ry[j];
        const int xm = max(x - rx - 1, -1), xp = min(x + rx, k.W - 1);
        const int ym = max(y - ry - 1, -1), yp = min(y + ry, k.H - 1);
        const int N = (xp - xm) * (yp - ym);
        const float var = Box<P>::var(k, (int64_t)ym * k.ld_sat + xm, (int64_t)ym * k.ld_sat + xp,
                                      (int64_t)yp * k.ld_sat + xp, (int64_t)yp * k.ld_sat + xm, N);
        uint32_t c = 0u;
        if (plane) {
            c = plane[(int64_t)yp * k.ld_hist + xp] + plane[(int64_t)ym * k.ld_hist + xm] -
                plane[(int64_t)ym * k.ld_hist + xp] - plane[(int64_t)yp * k.ld_hist + xm];
        }
        const float Pj = (float)c / (float)N;
        const float Lj = k.p.ld_min + ldr * Pj;
        const float Wj = var / (var + k.p.eps);
        num += Wj * Lj;
        den += Wj;
        lsum += Lj;
    }
    k.out[(int64_t)y * k.ld_out + x] = den > 0.f ? num / den : lsum / (float)k.p.n_scales;
}

template <int P>
__global__ void __launch_bounds__(kBlock) forward_kernel(FwdK k) {
    __shared__ float sh_edges[256];
    forward_tile<P>(k, xcd_tile(blockIdx.x, gridDim.x), sh_edges);
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
        forward_tile<P>(ks[i], (uint32_t)(g - prefix[i]), sh_edges);
    }
}

}  // namespace

int64_t query_tiles(int H, int W) {
    return (int64_t)((W + kWave - 1) / kWave) * ((H + kRows - 1) / kRows);
}

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
    return k;
}

hipError_t launch_forward(const float *v, int64_t ld_v, int H, int W, const void *sat,
                          int64_t ld_sat, int prec, const float *offsets, const uint32_t *hist,
                          int64_t ld_hist, int64_t plane_stride, const float *edges,
                          const QueryParams &p, float *out, int64_t ld_out, hipStream_t s) {
    const FwdK k = make_fwdk(v, ld_v, H, W, sat, ld_sat, offsets, hist, ld_hist, plane_stride,
                             edges, p, out, ld_out);
    const unsigned tiles = (unsigned)query_tiles(H, W);
    switch (prec) {
        case kF32:
            hipLaunchKernelGGL(forward_kernel<kF32>, dim3(tiles), dim3(kBlock), 0, s, k);
            break;
        case kC32x2:
            hipLaunchKernelGGL(forward_kernel<kC32x2>, dim3(tiles), dim3(kBlock), 0, s, k);
            break;
        default:
            hipLaunchKernelGGL(forward_kernel<kF64>, dim3(tiles), dim3(kBlock), 0, s, k);
            break;
    }
    return hipGetLastError();
}

}  // namespace tmo
