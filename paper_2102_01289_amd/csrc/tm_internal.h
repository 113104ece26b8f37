// tm_internal.h -- host-side launchers shared between the kernel files and the C ABI.
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

namespace tmo {

// ---------------------------------------------------------------- prologue (a1)
struct StatsPartial {          // one per reduction block, 32 bytes
    float mn, mx;
    double s1, s2;
    double pad;
};
// One image of the prologue: RGB (or luminance) in, luminance out, nparts partials.
struct StatsK {
    const float *rgb;
    int64_t ch_stride, ld_rgb;
    const float *lum_in;
    int64_t ld_in;
    float *lum_out;
    int64_t ld_out;
    int H, W, vec_in, vec_out, nparts, n_bins;
    StatsPartial *partials;
    float *edges, *offsets, *minmax;
    // colour input, log-domain variant: also write l = ln max(lum, FLT_MIN) here; the sums
    // (offsets) are then those of l, the range (edges, minmax) still that of lum
    float *log_out;
    int64_t ld_log;
    int vec_log;
};
constexpr int kStatsMaxBlocks = 1024;
int stats_blocks(int H, int W);
StatsK make_statsk(const float *rgb, int64_t ch_stride, int64_t ld_rgb, const float *lum_in,
                   int64_t ld_in, float *lum_out, int64_t ld_out, int H, int W, int n_bins,
                   float *edges, float *offsets, float *minmax, StatsPartial *partials);
// Prologue of a batch: the parts of images [0, count) in one launch, then one finalize
// block per image (device arrays ks[count], part_prefix[count+1]).
hipError_t launch_stats_batch(const StatsK *ks, const int64_t *part_prefix, int count,
                              unsigned grid, hipStream_t s, bool log = false);

hipError_t launch_luminance(const float *rgb, int64_t ch_stride, int64_t ld_rgb, int H, int W,
                            float *lum, int64_t ld_lum, hipStream_t s);
// rgb == nullptr: reduce lum only.  Otherwise compute lum from rgb and reduce it.
hipError_t launch_stats(const float *rgb, int64_t ch_stride, int64_t ld_rgb, const float *lum_in,
                        int64_t ld_lum_in, float *lum_out, int64_t ld_lum_out, int H, int W,
                        int n_bins, float *edges, float *offsets, float *minmax,
                        StatsPartial *partials, hipStream_t s);
// logv = ln(max(lum, FLT_MIN)) and the statistics (offsets, minmax) of logv.
// tm_prologue and tm_log_luminance in one pass over the colour planes (see StatsK::log_out).
hipError_t launch_stats_log(const float *rgb, int64_t ch_stride, int64_t ld_rgb, float *lum,
                            int64_t ld_lum, float *logv, int64_t ld_log, int H, int W, int n_bins,
                            float *edges, float *offsets, float *minmax, StatsPartial *partials,
                            hipStream_t s);
hipError_t launch_log_stats(const float *lum, int64_t ld_lum, float *logv, int64_t ld_log, int H,
                            int W, float *offsets, float *minmax, StatsPartial *partials,
                            hipStream_t s);
hipError_t launch_log_chain(const float *lum, int64_t ld_lum, const float *grad_l, int64_t ld_gl,
                            float *grad_i, int64_t ld_gi, int H, int W, hipStream_t s);
// launch_stats from RGB with the partials in the library's static per-device scratch array
// (no workspace).  Fails with hipErrorInvalidValue if the partials would not fit.
constexpr size_t kPrologueScratchBytes = 32768;
hipError_t launch_stats_noalloc(const float *rgb, int64_t ch_stride, int64_t ld_rgb,
                                float *lum_out, int64_t ld_lum_out, int H, int W, int n_bins,
                                float *edges, float *offsets, float *minmax, hipStream_t s);

// ---------------------------------------------------------------- multi-exposure front end
size_t hdr_response_ws_bytes();
hipError_t launch_hdr_response(const uint8_t *stack, int64_t exp_stride, int64_t ch_stride,
                               int64_t ld, int P, int H, int W, const int32_t *samples, int N,
                               const float *log_dt, float lam, float *g, void *ws,
                               hipStream_t s);
hipError_t launch_hdr_merge(const uint8_t *stack, int64_t exp_stride, int64_t ch_stride,
                            int64_t ld, int P, int H, int W, const float *log_dt, const float *g,
                            float *out, int64_t ch_out, int64_t ld_out, hipStream_t s);

// ---------------------------------------------------------------- scans (a2, a3)
struct ScanTune {
    int vec;        // columns per lane: 1, 2, 4, 8
    int th;         // rows per tile
    int chunk;      // histogram planes per pass: 2, 4, 8
};
ScanTune scan_tune_default(int H, int W, int n_bins);   // n_bins: of the histogram built with it
ScanTune scan_tune_adjoint(int H, int W);   // the backward's suffix scans
bool scan_tune_valid(const ScanTune &t);

// Workspace carve-up of the three-stage scan (a pure function of the shape and options).
struct ScanPlan {
    int H, W, tiles_x, tiles_y, vec, th, chunk;
    int sat_prec;      // -1: no integral image
    int n_planes;      // 0: no histogram
    size_t acc_bytes;  // bytes of one accumulator element (4 or 8)
    // byte offsets into ws
    size_t rs_sat, cs_sat, tt_sat, xc_sat, cse_sat, tte_sat;  // each holds 2 quantities
    size_t rs_h, cs_h, tt_h, xc_h, cse_h, tte_h;              // n_planes quantities
    size_t total;
};
ScanPlan make_scan_plan(int H, int W, int sat_prec, int n_planes, const ScanTune &t);

// Kernel parameters of one image's three-stage scan (device-side copy in batched mode).
struct ScanK {
    const float *v;
    int64_t ld_v;
    int H, W, th, tiles_x, tiles_y;
    int vec_load;                 // rows of v are 16-byte aligned
    // the plane the histogram items bin (v itself unless the caller gives another one)
    const float *vh;
    int64_t ld_vh;
    int vec_load_h;
    // the integral image is of l = ln max(v, FLT_MIN), formed as each pixel is read (the
    // log-domain variant; the histogram items still bin v)
    int log_src;
    const float *offsets;
    void *sat;
    int64_t ld_sat;
    const float *edges;
    int n_bins, layout, n_planes;
    uint32_t *hist;
    int64_t ld_hist, plane_stride;
    int stream_out;               // tables larger than the memory-side cache: non-temporal stores
    int hist_items, hist_chunks;  // histogram work items per tile, plane chunks per item
    // aggregates (each an array of quantities; see ScanPlan)
    void *rs_sat, *cs_sat, *tt_sat, *xc_sat, *cse_sat, *tte_sat;
    uint32_t *rs_h, *cs_h, *tt_h, *xc_h, *cse_h, *tte_h;
    // adjoint mode: the two FP64 planes to scan (row-major, pitch ld_d, already in reversed
    // pixel order) and the gradient written back in forward order, dv = s1 + 2 v s2
    const double2 *dsrc;
    int64_t ld_d;
    float *gv;
    int64_t ld_gv;
    // adjoint mode, log-domain variant: v is the image i whose log plane l = ln max(i,
    // FLT_MIN) the moments were taken of; the pass forms l itself and writes the gradient
    // with respect to i, (s1 + 2 l s2) / i, or 0 where the floor constant is taken
    int log_chain;
};

struct ScanArgs {
    const float *v;
    int64_t ld_v;
    const float *v_hist;     // plane the histogram bins; null: v
    int64_t ld_v_hist;
    int log_src;             // integral image of ln max(v, FLT_MIN) (see ScanK)
    int H, W;
    int sat_prec;            // -1 none
    const float *offsets;    // C32X2
    void *sat;               // table origin
    int64_t ld_sat;
    const float *edges;
    int n_bins;
    int layout;              // 0 per-bin, 1 cumulative
    int n_planes;
    uint32_t *hist;
    int64_t ld_hist, plane_stride;
};
hipError_t launch_tables(const ScanArgs &a, const ScanPlan &plan, void *ws, hipStream_t s);
ScanK make_scank(const ScanArgs &a, const ScanPlan &plan, void *ws);

// Integral image + cumulative histogram of images [0, count): three launches over flattened
// work lists (device arrays: ks[count], tile_prefix[count+1], item_prefix[count+1]).
// A scan tile that builds both tables is 1 + k.hist_items work items (ScanK): its integral
// image, then its histogram planes split into at most kMaxHistItems items, on neighbouring
// waves, so each wave holds the state of one kind of table only (fewer registers, more waves
// in flight) and the later reads of the tile's luminance rows are served by the cache.
constexpr int kMaxHistItems = 8;

struct BatchScan {
    const ScanK *ks;
    const int64_t *tile_prefix, *item_prefix;
    int count, prec, vec, chunk;
    unsigned grid_tiles, grid_items;
};
hipError_t launch_tables_batch(const BatchScan &b, hipStream_t s);

// Items of stage 2 of one image (thread-level): nq*H + nq*W + nq*tiles_y.
int64_t scan_stage2_items(const ScanK &k, bool sat);

// ---------------------------------------------------------------- comb schedule
// Output rows y and y + 2r + 1 read the same table row at the field of radius r, and the
// pyramid's halving radii put the other fields' shared rows a few rows apart.  Ordering
// blocks by phase within a period of the smallest window height, then by tooth, keeps every
// shared corner row in flight at once.  p4 = period in row groups of `rows` rows; teeth =
// number of periods; one tooth (plain row-major order) for short windows.
void comb_params(int H, int rows, const int *ry, int n_scales, int *p4, int *teeth);

// ---------------------------------------------------------------- query (a4)
struct QueryParams {
    int n_bins, n_scales;
    int rx[8], ry[8];          // clamped to the image's width and height
    float eps, ld_min, ld_max;
    const float *scalars;      // null, or device {eps, ld_min, ld_max} read at run time
};

struct FwdK {
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
    float *out;
    int64_t ld_out;
    int tiles_x;
    int p4, teeth;      // comb schedule: period in 4-row groups, number of teeth
    float *resid;       // training forward: 2s + 2 residual planes of H*W (else null)
    int64_t rstride;
    // colour restoration (Eq. 12), when rgb_out is not null: planar RGB in and out
    const float *rgb;
    int64_t rgb_cs, rgb_ld;
    float *rgb_out;
    int64_t out_cs, out_ld;
    float saturation;
    // per-field maps (Fig. 3), when not null: L_j at plane j, W_j at plane s + j (pitch W)
    float *maps;
    int64_t mstride;
};
constexpr int kQueryRows = 4;   // a query block covers 64 columns x 4 rows
// Blocks of one image's fused query (the comb schedule may include idle blocks).
int64_t query_blocks(const FwdK &k);
// Fused query of a batch: one block per tile of images [0, count) (device arrays ks[count],
// tile_prefix[count+1]; the grid is tile_prefix[count] - tile_prefix[0]).
hipError_t launch_forward_batch(const FwdK *ks, const int64_t *tile_prefix, int count, int prec,
                                bool h32, unsigned grid, hipStream_t s);
// Every histogram byte offset of the query of k fits in 32 bits.
bool hist_offsets_fit_32(const FwdK &k);
FwdK make_fwdk(const float *v, int64_t ld_v, int H, int W, const void *sat, int64_t ld_sat,
                const float *offsets, const uint32_t *hist, int64_t ld_hist,
                int64_t plane_stride, const float *edges, const QueryParams &p, float *out,
                int64_t ld_out);
// The fused query that also writes the per-field tone values L_j (Eq. 2) and weights W_j
// (Eq. 4): maps holds 2s planes of H*W (plane stride H*W, pitch W).
hipError_t launch_forward_maps(const float *v, int64_t ld_v, int H, int W, const void *sat,
                               int64_t ld_sat, int prec, const float *offsets,
                               const uint32_t *hist, int64_t ld_hist, int64_t plane_stride,
                               const float *edges, const QueryParams &p, float *out,
                               int64_t ld_out, float *maps, hipStream_t s);
// The fused query followed by colour restoration (Eq. 12): c_out = (c_in / v)^sat L for
// c = R, G, B (the ratio taken as 1 where v = 0, inputs clamped at 0); out may be null.
hipError_t launch_forward_rgb(const float *v, int64_t ld_v, int H, int W, const void *sat_tab,
                              int64_t ld_sat, int prec, const float *offsets,
                              const uint32_t *hist, int64_t ld_hist, int64_t plane_stride,
                              const float *edges, const QueryParams &p, float *out,
                              int64_t ld_out, const float *rgb, int64_t rgb_cs, int64_t rgb_ld,
                              float *rgb_out, int64_t out_cs, int64_t out_ld, float sat,
                              hipStream_t s);
hipError_t launch_forward(const float *v, int64_t ld_v, int H, int W, const void *sat,
                          int64_t ld_sat, int prec, const float *offsets, const uint32_t *hist,
                          int64_t ld_hist, int64_t plane_stride, const float *edges,
                          const QueryParams &p, float *out, int64_t ld_out, float *resid,
                          hipStream_t s);

// Prefix scan of two FP64 planes stored in reversed pixel order (pitch ld_d), written back as
// dv = s1 + 2 v s2 in forward order: the suffix sums of the backward.
hipError_t launch_suffix_adjoint(const double2 *d, int64_t ld_d, const float *v, int64_t ld_v,
                                 int H, int W, float *gv, int64_t ld_gv, const ScanPlan &plan,
                                 void *ws, hipStream_t s, bool log_chain = false);

// ---------------------------------------------------------------- backward (a5)
struct BwdResidArgs {
    const float *v;
    int64_t ld_v;
    int H, W;
    QueryParams p;
    const float *resid;      // 2s + 2 planes of H*W (pitch W)
    const float *g;
    int64_t ld_g;
    float *grad_v;
    int64_t ld_gv;
    double *grad_params;
    bool log_chain;          // v is the image i of the log-domain variant (see ScanK)
};
struct BwdPlan {
    int64_t nblocks;
    int p4, teeth, nchunks, chunk;
    size_t resid, Rp, Rb, Cp, Cb, Dr, part, K, scan, total;
    ScanPlan scan_plan;
};
// with_resid: also reserve the residual planes (the table-based backward rebuilds them).
BwdPlan make_bwd_plan(int H, int W, int n_scales, const int *ry, bool with_resid);
hipError_t launch_backward_resid(const BwdResidArgs &a, const BwdPlan &plan, void *ws,
                                 hipStream_t s);

// ---------------------------------------------------------------- single-pass histogram
struct LookbackArgs {
    const float *v;
    int64_t ld_v;
    int H, W;
    const float *edges;
    int n_bins, n_planes, layout;   // layout: 0 per bin, 1 cumulative
    uint32_t *hist;
    int64_t ld_hist, plane_stride;
    int nt;                         // non-temporal plane stores
};
struct LookbackPlan {
    int th, tiles_x, tiles_y;
    size_t rowrec, colrec, cornrec, total;   // byte offsets in the workspace; header at 0
};
void set_lookback_spin_limit(uint32_t polls);   // 0: the default bound
int lookback_rows(int H, int W, int n_planes);   // rows per look-back tile (16 or 32)
LookbackPlan make_lookback_plan(int H, int W, int n_planes, int th);
hipError_t launch_lookback_hist(const LookbackArgs &a, const LookbackPlan &plan, void *ws,
                                hipStream_t s);

}  // namespace tmo
