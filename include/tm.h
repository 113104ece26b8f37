/*
 * tm.h -- C ABI of the MI355X (gfx950) implementation of multi-receptive-field local tone
 * mapping with integral images and integral histograms (Yang, Lin, Liu, Shahnovich,
 * Yadid-Pecht, "Mobile-end Tone Mapping based on Integral Image and Integral Histogram",
 * arXiv 2102.01289).
 *
 * The method (Section II): the luminance image i is compressed to l = log i and split into
 * n equal-width bins (Eq. 7); an integral histogram (Eq. 8) and integral images of i and
 * i^2 (Eq. 5) are built once; then every pixel, for each of s receptive fields w_j centred
 * on it, reads O(1) box queries (Eq. 6, Eq. 9) to get the window histogram's CDF at its own
 * bin (Eq. 1), a tone value (Eq. 2), the window variance (Eq. 10) and a weight (Eq. 4), and
 * the per-field tone values are fused by the weights (Eq. 3).
 *
 * Conventions shared by every entry point
 *   - All data pointers are DEVICE pointers owned by the caller (hipMalloc or framework
 *     tensors).  The library never allocates, frees or keeps caller memory.  Scratch space
 *     comes from the caller's workspace `ws` of `ws_bytes` bytes; the size an entry point
 *     needs is returned by the matching tm_*_workspace_bytes function.  ws must be 256-byte
 *     aligned and is clobbered.
 *   - `stream` is a hipStream_t (NULL = the null stream).  Every call only enqueues kernels
 *     on it and returns without synchronising; no call uses hipMemset, so a sequence of
 *     calls can be captured into a HIP graph.
 *   - Images are row-major FP32 with a row pitch `ld_*` counted in elements (ld >= W).
 *     Pixel (x, y) is column x of row y.
 *   - Integral tables use one layout ("table layout"): a pointer T0 to the entry of pixel
 *     (0, 0) and a row pitch ld >= W + 1.  The entry for (x, y) is T0[y*ld + x] for
 *     -1 <= x < W and -1 <= y < H; the entries with x = -1 or y = -1 are the zero border of
 *     Eq. 5 (the sums over an empty range).  x = -1 of row y aliases column ld-1 of row y-1,
 *     which is padding.  The producing call writes every entry of this region, the zeros
 *     included: row -1 (ld + 1 entries starting at T0 - ld - 1) and the padding columns
 *     [W, ld) of every row.  tm_table_geometry() returns an ld, the offset of T0 from the
 *     start of an allocation and the element count to allocate.
 *   - Every argument is checked on the host before anything is launched; a failed check
 *     returns a negative tm_status and launches nothing.  HIP launch errors map to
 *     TM_ERR_HIP.  No C++ exception crosses this interface.
 *   - Sizes: 1 <= H; 1 <= W <= TM_MAX_WIDTH (2^24, so that every per-lane byte offset
 *     along a table row fits in 32 bits); H*W < 2^31; every table and plane holds
 *     < 2^31 entries.
 */
#ifndef TM_H
#define TM_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    TM_OK = 0,
    TM_ERR_ARG = -1,          /* null pointer, bad enum, bad parameter value */
    TM_ERR_SHAPE = -2,        /* H, W, ld or plane stride out of range */
    TM_ERR_ALIGN = -3,        /* pointer not aligned as documented */
    TM_ERR_WORKSPACE = -4,    /* ws NULL, misaligned or smaller than required */
    TM_ERR_HIP = -5,          /* a HIP runtime call failed */
    TM_ERR_UNSUPPORTED = -6   /* valid request the library does not implement */
} tm_status;

/* Storage and accumulation of the integral images of i and i^2 (Eq. 5).
 *   TM_SAT_F32   plain FP32 sums, no offset; entry = float2 {I(i), I(i^2)} (8 bytes).
 *   TM_SAT_C32X2 sums of (i - mu1) and (i^2 - mu2) accumulated with compensated FP32
 *                (TwoSum) arithmetic and stored as unevaluated pairs hi + lo;
 *                entry = float4 {I1.hi, I1.lo, I2.hi, I2.lo} (16 bytes).  mu1, mu2 are
 *                the FP32 offsets from tm_image_stats (the image means of i and i^2).
 *   TM_SAT_F64   plain FP64 sums, no offset; entry = double2 {I(i), I(i^2)} (16 bytes). */
typedef enum { TM_SAT_F32 = 0, TM_SAT_C32X2 = 1, TM_SAT_F64 = 2 } tm_sat_prec;

/* Integral-histogram planes (Eq. 8), uint32 each, in the table layout.
 *   TM_HIST_PER_BIN     n planes H_k, k = 0..n-1: counts of pixels in bin k (Eq. 8).
 *   TM_HIST_CUMULATIVE  n-1 planes G_k, k = 1..n-1: counts of pixels in bins below k,
 *                       G_k = sum_{j<k} H_j.  The CDF of Eq. 1 at a pixel of bin b is then
 *                       one box query on G_b (G_0 = 0 is not stored).
 * Plane p (0-based) starts at hist + p * plane_stride. */
typedef enum { TM_HIST_PER_BIN = 0, TM_HIST_CUMULATIVE = 1 } tm_hist_layout;

#define TM_MAX_WIDTH (1 << 24)
#define TM_MAX_SCALES 8
#define TM_MAX_BINS 256

/* Method parameters (Section II-C).  Paper setting: n = 5, s = 5, eps = 0.1 (Section IV),
 * radii halving from the image size (tm_paper_radii), display range [0, 1].
 *   n_bins   n, 1..256 (number of equal-width log-luminance bins, Eq. 7)
 *   n_scales s, 1..8   (number of receptive fields, Eq. 3)
 *   rx, ry   per-field half-widths >= 0; field j covers x-(rx+1) < x' <= x+rx and the same
 *            in y (Algorithm 1), clamped to the image.  Any radius >= the image's width
 *            (height) gives the whole row (column), so larger radii act as that size.
 *   eps      the regulariser of Eq. 4, > 0, in units of luminance squared
 *   ld_min, ld_max  display luminance range of Eq. 2, ld_max > ld_min
 *   scalars  NULL, or a DEVICE pointer to float[3] = {eps, ld_min, ld_max} that the kernels
 *            read when they run, in place of the three fields above (which are then neither
 *            used nor checked).  It lets a caller whose parameters live in device memory (an
 *            autograd graph, a captured HIP graph) change them without a host
 *            synchronisation.  The device values must meet the same conditions (eps > 0,
 *            ld_max > ld_min, finite); the library cannot check them.  4-byte aligned, else
 *            TM_ERR_ALIGN.  The batch entry points ignore it. */
typedef struct {
    int32_t n_bins;
    int32_t n_scales;
    int32_t rx[TM_MAX_SCALES];
    int32_t ry[TM_MAX_SCALES];
    float eps;
    float ld_min;
    float ld_max;
    const float *scalars;
} tm_params;

/* Scan tiling (chosen by the autotuner; NULL anywhere means the built-in default).
 *   tile_w_vec  columns per lane of one 64-lane tile: 2, 4 or 8 (tile width 64*vec)
 *   tile_h      rows per tile, 1..256
 *   bin_chunk   histogram planes accumulated per pass over the image tile: 2, 4 or 8 */
typedef struct {
    int32_t tile_w_vec;
    int32_t tile_h;
    int32_t bin_chunk;
} tm_tune;

const char *tm_status_string(tm_status s);

/* The scan tiling an H x W image with an n_bins-bin histogram gets when an entry point is
 * passed tune = NULL (host function; n_bins is the entry point's own n_bins argument, 0 for
 * an integral image alone): 4 columns per lane from width 2048 up, else 2; rows per tile 4
 * (H < 900), 8 (H < 1800) or 16, doubled (at most 32) from 33 bins, then halved (not below 4)
 * while the image has fewer than 512 tiles; 4 planes per pass.  TM_ERR_ARG if t is NULL or
 * n_bins is outside [0, TM_MAX_BINS]. */
tm_status tm_default_tune(int32_t H, int32_t W, int32_t n_bins, tm_tune *t);

/* Radii of the receptive-field pyramid (Section II-C): the largest field is the image and
 * each next one is half as wide, rx[j] = W >> (j+1), ry[j] = H >> (j+1) for j < n_scales.
 * Host function; fills p->rx, p->ry only. */
tm_status tm_paper_radii(int32_t H, int32_t W, tm_params *p);

/* Table layout helper (host): for an H x W image returns the row pitch ld (elements, a
 * multiple of 64, >= W + 1), the offset in elements of T0 from the start of an allocation
 * (a multiple of 64, >= ld + 1) and the elements one table or plane needs (origin offset +
 * H * ld, rounded up to 64).  Use the same element count as the plane stride. */
tm_status tm_table_geometry(int32_t H, int32_t W, int64_t *ld, int64_t *origin_offset,
                            int64_t *elems);

/* ---------------------------------------------------------------- stage a1: prologue */

/* Luminance (Section III, Eq. 11): i = 0.2126 R + 0.7152 G + 0.0722 B from planar FP32
 * RGB (channel c of pixel (x, y) at rgb[c*ch_stride + y*ld_rgb + x]).  Evaluated in FP32
 * left to right with fused multiply-adds, i = fma(0.0722, B, fma(0.7152, G, 0.2126*R)).
 * lum: H x W, pitch ld_lum.  No workspace. */
tm_status tm_luminance(const float *rgb, int64_t ch_stride, int64_t ld_rgb, int32_t H,
                       int32_t W, float *lum, int64_t ld_lum, void *stream);

/* Image statistics the later stages need, in one reduction over lum:
 *   edges[0..n_bins-2] (FP32, device): bin edges of n_bins equal-width bins of log i over
 *       [log i_min, log i_max] (Section II-A, Eq. 7).  Edge k sits at the real number
 *       e_k = i_min^(1-k/n) i_max^(k/n); the stored value is the smallest FP32 >= e_k, so
 *       `i >= edges[k-1]` decides bin >= k exactly.  i_min is floored at the smallest
 *       normal FP32.  If i_max <= i_min all edges are +inf.  n_bins = 1 writes nothing.
 *   offsets[2] (FP32, device, nullable): {mu1, mu2} = FP32-rounded means of i and i^2
 *       (FP64 sums), the offsets of TM_SAT_C32X2 tables.
 *   minmax[2] (FP32, device, nullable): {min i, max i}.
 * Deterministic (fixed reduction order).  Workspace: tm_image_stats_workspace_bytes. */
size_t tm_image_stats_workspace_bytes(int32_t H, int32_t W);
tm_status tm_image_stats(const float *lum, int64_t ld_lum, int32_t H, int32_t W,
                         int32_t n_bins, float *edges, float *offsets, float *minmax,
                         void *ws, size_t ws_bytes, void *stream);

/* Eq. 11 and the statistics above fused in one pass over the RGB image. */
tm_status tm_prologue(const float *rgb, int64_t ch_stride, int64_t ld_rgb, int32_t H,
                      int32_t W, int32_t n_bins, float *lum, int64_t ld_lum, float *edges,
                      float *offsets, float *minmax, void *ws, size_t ws_bytes, void *stream);

/* tm_prologue without a workspace, for callers that cannot allocate device memory (code
 * under HIP graph capture, tight serving loops, harnesses that forbid hipMalloc).  The
 * per-block partials of the reduction live in a static device array of the library,
 * TM_PROLOGUE_SCRATCH_BYTES (32 KiB) per GPU, held until the process ends; every image size
 * tm_prologue accepts fits (the reduction never uses more than 1024 partials), and a
 * request that would need more returns TM_ERR_UNSUPPORTED.  No memory is allocated or
 * freed.  Every call on one GPU shares that GPU's array: calls that overlap in time on one
 * GPU (on different streams, or from different threads before their work is ordered) race
 * and give wrong statistics; calls ordered on one stream are safe.  Results are bitwise
 * those of tm_prologue.  The first call on a device looks up the array's device address
 * (a host-side query, not a stream operation); a failure there returns TM_ERR_HIP. */
#define TM_PROLOGUE_SCRATCH_BYTES 32768
tm_status tm_prologue_noalloc(const float *rgb, int64_t ch_stride, int64_t ld_rgb, int32_t H,
                              int32_t W, int32_t n_bins, float *lum, int64_t ld_lum,
                              float *edges, float *offsets, float *minmax, void *stream);

/* Log-domain variance variant.  Section II-A builds the integral images of the image and of
 * its square (Eq. 5) for Eq. 10's window variance; the method is also defined with that
 * variance taken of the logarithmic image l the bins are cut from.  This call writes
 *   logv = ln(max(i, FLT_MIN))   (FP32, the device logf, within 2 ulp of the exact value)
 * (H x W, pitch ld_log; must not overlap lum; NULL: no plane, the statistics only) and, in
 * the same pass, the statistics of l:
 * offsets[2] (device, nullable) = FP32-rounded means of l and l^2 (FP64 sums), the offsets a
 * TM_SAT_C32X2 integral image of l needs, and minmax[2] (device, nullable) = {min l, max l}.
 * The variant is then: tm_integral_image of logv with these offsets, the integral histogram
 * of i as usual (or both from i alone: tm_integral_tables_log), and tm_tonemap_forward (or
 * _maps, _rgb) given i itself (its bins decide Eq. 1) with the table and offsets of l; eps
 * is then in units of l^2.  From colour input tm_prologue_log forms the offsets in the
 * prologue's own pass, with no log plane needed.  Its gradient:
 * tm_tonemap_forward_train given i with the table and offsets of l, then
 * tm_tonemap_backward_resid_log given i (or, in two steps, tm_tonemap_backward_resid given
 * logv as its image, which returns the gradient with respect to l since the residual
 * backward uses its image only in the final dv = s1 + 2 v s2, then
 * tm_log_luminance_backward); from the tables, tm_tonemap_backward_log.
 * Deterministic.  Workspace: tm_image_stats_workspace_bytes. */
tm_status tm_log_luminance(const float *lum, int64_t ld_lum, int32_t H, int32_t W, float *logv,
                           int64_t ld_log, float *offsets, float *minmax, void *ws,
                           size_t ws_bytes, void *stream);

/* tm_prologue and tm_log_luminance in one pass over the colour planes: lum (Eq. 11), edges
 * and minmax of lum exactly as tm_prologue writes them, and logv and log_offsets (means of l
 * and l^2) exactly as tm_log_luminance of that lum writes its plane and offsets, bit for bit.
 * The log plane's range and the luminance's offsets are not produced.  logv may be NULL
 * (then only its offsets are formed); else lum and logv must be disjoint (else TM_ERR_ARG).
 * Other arguments and errors as for tm_prologue.  Workspace: tm_image_stats_workspace_bytes.
 * The log-domain variant's forward is then tm_integral_tables_log of lum (which needs no
 * log plane) and the fused query. */
tm_status tm_prologue_log(const float *rgb, int64_t ch_stride, int64_t ld_rgb, int32_t H,
                          int32_t W, int32_t n_bins, float *lum, int64_t ld_lum, float *logv,
                          int64_t ld_log, float *edges, float *log_offsets, float *minmax,
                          void *ws, size_t ws_bytes, void *stream);

/* The chain rule through l = ln(max(i, FLT_MIN)) for the log-domain variant's gradient:
 *   grad_i = grad_l / i   where i > FLT_MIN,   0 where the floor constant is taken
 * (FP32, one correctly rounded division per pixel).  lum is the image i given to
 * tm_log_luminance; grad_l the gradient with respect to its logv.  grad_i may be grad_l
 * itself (then with the same pitch); any other overlap is TM_ERR_ARG.  No workspace. */
tm_status tm_log_luminance_backward(const float *lum, int64_t ld_lum, int32_t H, int32_t W,
                                    const float *grad_l, int64_t ld_gl, float *grad_i,
                                    int64_t ld_gi, void *stream);

/* ---------------------------------------------------------------- stages a2, a3: tables */

/* Integral images (Eq. 5) of v and v^2 in one interleaved table (entry type per
 * tm_sat_prec), table layout, pitch ld_sat.  offsets: device float[2] for TM_SAT_C32X2
 * (required), ignored otherwise.  Workspace: tm_tables_workspace_bytes. */
tm_status tm_integral_image(const float *v, int64_t ld_v, int32_t H, int32_t W,
                            tm_sat_prec prec, const float *offsets, void *sat,
                            int64_t ld_sat, const tm_tune *tune, void *ws, size_t ws_bytes,
                            void *stream);

/* Integral histogram (Eq. 7-8) of v's bins under `edges` (as from tm_image_stats), uint32
 * planes in the table layout.  Counts are exact.  Workspace: tm_tables_workspace_bytes. */
tm_status tm_integral_histogram(const float *v, int64_t ld_v, int32_t H, int32_t W,
                                const float *edges, int32_t n_bins, tm_hist_layout layout,
                                uint32_t *hist, int64_t ld_hist, int64_t plane_stride,
                                const tm_tune *tune, void *ws, size_t ws_bytes,
                                void *stream);

/* The same integral histogram in one pass over v: each tile's carries come from the tiles
 * before it by decoupled look-back ({state, count} records published and polled with
 * agent-scope atomics; exact integers, so the result does not depend on the order they
 * arrive in and equals tm_integral_histogram's bit for bit).  Up to 8 planes (n_bins <= 8
 * per bin, <= 9 cumulative) and H < 2^30 (the records hold 30-bit counts);
 * TM_ERR_UNSUPPORTED beyond.  Tiles of 128 columns by 16 or 32 rows.  Workspace:
 * tm_lookback_workspace_bytes (0 for an unsupported shape); its first 8 bytes are a header
 * the call resets: a ticket counter, then a status word that is 0 after the call, or 1 if
 * some wait for a record ran out (bounded, about a second; the planes are then invalid).
 * Every wait is bounded, so the call always completes.  Calls that share a workspace must
 * not overlap. */
size_t tm_lookback_workspace_bytes(int32_t H, int32_t W, int32_t n_bins, tm_hist_layout layout);
/* Test hook for the bounded waits of tm_integral_histogram_lookback: the polls of one
 * look-back window before it counts as timed out (then the status word is raised and the pass
 * still completes), for the calls made after it in this process; 0 restores the default
 * (2^20 polls, about a second).  Not thread-safe against concurrent calls. */
void tm_lookback_set_spin_limit(uint32_t polls);
tm_status tm_integral_histogram_lookback(const float *v, int64_t ld_v, int32_t H, int32_t W,
                                         const float *edges, int32_t n_bins,
                                         tm_hist_layout layout, uint32_t *hist, int64_t ld_hist,
                                         int64_t plane_stride, void *ws, size_t ws_bytes,
                                         void *stream);

/* Both tables in one pass over v (sat or hist may be NULL to skip that table). */
tm_status tm_integral_tables(const float *v, int64_t ld_v, int32_t H, int32_t W,
                             tm_sat_prec prec, const float *offsets, void *sat,
                             int64_t ld_sat, const float *edges, int32_t n_bins,
                             tm_hist_layout layout, uint32_t *hist, int64_t ld_hist,
                             int64_t plane_stride, const tm_tune *tune, void *ws,
                             size_t ws_bytes, void *stream);

size_t tm_tables_workspace_bytes(int32_t H, int32_t W, int32_t n_bins, tm_sat_prec prec,
                                 const tm_tune *tune);

/* The log-domain variant's two tables from the image i alone: the integral images (Eq. 5)
 * of l = ln max(i, FLT_MIN), formed as each pixel is read with tm_log_luminance's own
 * expression, and the integral histogram (Eq. 7-8) of i's bins.  log_offsets as
 * tm_log_luminance or tm_prologue_log write them (required for TM_SAT_C32X2).  Results equal
 * tm_integral_tables_split of (tm_log_luminance's plane, i) bit for bit, without reading a
 * log plane.  sat is required (else TM_ERR_ARG); hist may be NULL; other arguments,
 * workspace and errors as for tm_integral_tables. */
tm_status tm_integral_tables_log(const float *lum, int64_t ld_lum, int32_t H, int32_t W,
                                 tm_sat_prec prec, const float *log_offsets, void *sat,
                                 int64_t ld_sat, const float *edges, int32_t n_bins,
                                 tm_hist_layout layout, uint32_t *hist, int64_t ld_hist,
                                 int64_t plane_stride, const tm_tune *tune, void *ws,
                                 size_t ws_bytes, void *stream);

/* Both tables in one pass, each of its own plane of the same H x W: the integral images
 * (Eq. 5) of v_sat and the integral histogram (Eq. 7-8) of v_hist's bins under edges.  For
 * the log-domain variant, whose local statistics are those of l = ln i (tm_log_luminance)
 * while the bins stay those of i (Eq. 9).  Results equal tm_integral_image of v_sat and
 * tm_integral_histogram of v_hist bit for bit; sat and hist are both required (else
 * TM_ERR_ARG), other arguments as for tm_integral_tables, whose workspace size applies. */
tm_status tm_integral_tables_split(const float *v_sat, int64_t ld_v_sat, const float *v_hist,
                                   int64_t ld_v_hist, int32_t H, int32_t W, tm_sat_prec prec,
                                   const float *offsets, void *sat, int64_t ld_sat,
                                   const float *edges, int32_t n_bins, tm_hist_layout layout,
                                   uint32_t *hist, int64_t ld_hist, int64_t plane_stride,
                                   const tm_tune *tune, void *ws, size_t ws_bytes,
                                   void *stream);

/* ---------------------------------------------------------------- stage a4: forward */

/* Tone-mapped luminance (Eq. 1-4, 6, 9, 10 and the fusion of Eq. 3) of v, from its
 * integral images `sat` (precision prec, offsets as used to build it) and its cumulative
 * integral histogram `hist_cum` (n_bins-1 planes, may be NULL when n_bins = 1).
 * For each pixel p and field j: the clamped window (Algorithm 1's corners), its pixel
 * count N, S1 = sum v and S2 = sum v^2 (Eq. 6), the count c of window pixels in bins below
 * p's bin (Eq. 9 summed as in Eq. 1, one query on G_b), P = c/N (Eq. 1; the histogram
 * total equals N), L_j = ld_min + (ld_max - ld_min) P (Eq. 2), var = max(0, S2/N -
 * (S1/N)^2) (Eq. 10 as the population variance), W_j = var/(var + eps) (Eq. 4); then
 * L = sum W_j L_j / sum W_j (Eq. 3), or the mean of the L_j where every W_j = 0.
 * out: FP32 H x W, pitch ld_out.  No workspace.  One launch for all fields. */
tm_status tm_tonemap_forward(const float *v, int64_t ld_v, int32_t H, int32_t W,
                             const void *sat, int64_t ld_sat, tm_sat_prec prec,
                             const float *offsets, const uint32_t *hist_cum, int64_t ld_hist,
                             int64_t plane_stride, const float *edges, const tm_params *p,
                             float *out, int64_t ld_out, void *stream);

/* The forward of tm_tonemap_forward that also writes, for every field j, its tone value
 * L_j (Eq. 2) and its weight W_j (Eq. 4), the maps Fig. 3 shows: maps holds 2 * n_scales
 * planes of H*W FP32 (pitch W, plane stride H*W), L_j at plane j and W_j at plane
 * n_scales + j; caller-owned. */
tm_status tm_tonemap_forward_maps(const float *v, int64_t ld_v, int32_t H, int32_t W,
                                  const void *sat, int64_t ld_sat, tm_sat_prec prec,
                                  const float *offsets, const uint32_t *hist_cum,
                                  int64_t ld_hist, int64_t plane_stride, const float *edges,
                                  const tm_params *p, float *out, int64_t ld_out, float *maps,
                                  void *stream);

/* Colour restoration (Sec. II-D, Eq. 12) fused into the forward: after L (the tone-mapped
 * luminance of tm_tonemap_forward) each output channel is
 *   c_out = (c_in / v)^saturation * L,   c = R, G, B,
 * with v the input luminance (the image the tables were built from, normally Eq. 11 of the
 * same rgb).  Readings: inputs are clamped at 0, and where v = 0 the ratio is taken as 1 (a
 * neutral pixel).  The paper uses saturation = 0.6; any finite saturation >= 0 is accepted
 * (0 gives a grey image of value L).  rgb / rgb_out: planar FP32, channel c at
 * rgb + c*ch_stride, row pitch ld_rgb (ch_stride >= H*ld_rgb), caller-owned device memory.
 * out (tone-mapped luminance, pitch ld_out) may be NULL. */
tm_status tm_tonemap_forward_rgb(const float *v, int64_t ld_v, int32_t H, int32_t W,
                                 const void *sat, int64_t ld_sat, tm_sat_prec prec,
                                 const float *offsets, const uint32_t *hist_cum,
                                 int64_t ld_hist, int64_t plane_stride, const float *edges,
                                 const tm_params *p, const float *rgb, int64_t ch_stride,
                                 int64_t ld_rgb, float saturation, float *rgb_out,
                                 int64_t ch_stride_out, int64_t ld_rgb_out, float *out,
                                 int64_t ld_out, void *stream);

/* The whole path RGB -> RGB on one image: prologue (Eq. 11, edges, offsets), integral image
 * of precision prec and cumulative integral histogram (default tiling), fused query with
 * colour restoration.  Every intermediate lives in ws (tm_tonemap_rgb_workspace_bytes). */
size_t tm_tonemap_rgb_workspace_bytes(int32_t H, int32_t W, const tm_params *p,
                                      tm_sat_prec prec);
tm_status tm_tonemap_rgb(const float *rgb, int64_t ch_stride, int64_t ld_rgb, int32_t H,
                         int32_t W, const tm_params *p, tm_sat_prec prec, float saturation,
                         float *rgb_out, int64_t ch_stride_out, int64_t ld_rgb_out, void *ws,
                         size_t ws_bytes, void *stream);

/* Number of FP32 residual planes a training forward writes: 2 * n_scales + 2 (0 if
 * n_scales is out of range). */
int32_t tm_residual_planes(int32_t n_scales);

/* The forward of tm_tonemap_forward plus, for the backward, per-pixel residual planes that
 * do not depend on the upstream gradient (Eq. 3, 4, 10 differentiated): with
 * c_j = (L_j - L)/D eps/(var_j + eps)^2 (zero where var_j was clamped or D = 0),
 *   R1_j = -2 c_j (S1_j/N_j) / N_j,  R2_j = c_j / N_j          (j < s)
 *   E    = sum_j (L_j - L)/D (-var_j/(var_j + eps)^2)
 *   Pbar = sum_j W_j P_j / D (mean of P_j where D = 0)
 * resid: tm_residual_planes(s) * H * W FP32 values, caller-owned, 8-byte aligned (else
 * TM_ERR_ALIGN), laid out as s interleaved pair planes (pair plane j starts at
 * resid + 2*j*H*W and holds {R1_j, R2_j} of pixel (x, y) at offset 2*(y*W + x)), then the
 * E plane at resid + 2*s*H*W and the Pbar plane at resid + (2*s + 1)*H*W (pitch W).
 * A window of one pixel has zero variance by definition. */
tm_status tm_tonemap_forward_train(const float *v, int64_t ld_v, int32_t H, int32_t W,
                                   const void *sat, int64_t ld_sat, tm_sat_prec prec,
                                   const float *offsets, const uint32_t *hist_cum,
                                   int64_t ld_hist, int64_t plane_stride, const float *edges,
                                   const tm_params *p, float *out, int64_t ld_out, float *resid,
                                   void *stream);

/* ---------------------------------------------------------------- stage a5: backward */

/* Gradient from the residual planes of tm_tonemap_forward_train: no integral table is read.
 *   dv(q) = sum_j sum_{p: q in w_j(p)} g(p) (R1_j(p) + 2 v(q) R2_j(p)),
 *   grad_params = {sum g E, sum g (1 - Pbar), sum g Pbar}.
 * v: the luminance the training forward read (pitch ld_v); resid: its residual planes as laid
 * out above; grad_out: FP32 H x W, pitch ld_g; grad_v: FP32 H x W, pitch ld_gv (only its H x W
 * entries are written); grad_params: device double[3] = {d/d eps, d/d ld_min, d/d ld_max}.
 * Every sum is taken in a fixed order (no atomics), so results are bit-reproducible.
 * Workspace: tm_backward_resid_workspace_bytes. */
size_t tm_backward_resid_workspace_bytes(int32_t H, int32_t W, const tm_params *p);
tm_status tm_tonemap_backward_resid(const float *v, int64_t ld_v, int32_t H, int32_t W,
                                    const tm_params *p, const float *resid,
                                    const float *grad_out, int64_t ld_g, float *grad_v,
                                    int64_t ld_gv, double *grad_params, void *ws,
                                    size_t ws_bytes, void *stream);

/* The same residual backward for the log-domain variance variant (tm_log_luminance), given
 * the image i itself: the last scan pass forms l = ln max(i, FLT_MIN) with the expression
 * tm_log_luminance uses and writes the gradient with respect to i,
 *   grad_lum = (s1 + 2 l s2) / i  where i > FLT_MIN,  0 where the floor constant is taken,
 * which equals tm_tonemap_backward_resid given logv followed by tm_log_luminance_backward
 * bit for bit, without the log plane and without the extra pass.  resid from
 * tm_tonemap_forward_train given i with l's table and offsets; other arguments, workspace
 * (tm_backward_resid_workspace_bytes) and errors as for tm_tonemap_backward_resid. */
tm_status tm_tonemap_backward_resid_log(const float *lum, int64_t ld_lum, int32_t H, int32_t W,
                                        const tm_params *p, const float *resid,
                                        const float *grad_out, int64_t ld_g, float *grad_lum,
                                        int64_t ld_gl, double *grad_params, void *ws,
                                        size_t ws_bytes, void *stream);


/* Gradient of sum_p g(p) L(p) (g = grad_out) with respect to v and to (eps, ld_min,
 * ld_max), from the same tables the forward read.  The histogram terms are piecewise
 * constant in v and the bin edges are held fixed, so v enters only through the window
 * variances: with D = sum_j W_j and a_j = g (L_j - L)/D eps/(var_j + eps)^2 (zero where
 * var_j was clamped or D = 0),
 *   dv(q) = sum_j sum_{p: q in w_j(p)} (-2 a_j S1_j/N_j^2 + 2 v(q) a_j/N_j),
 * evaluated by depositing the per-pixel coefficients at the window corners and taking two
 * reverse (suffix) 2-D scans.  grad_v: FP32 H x W, pitch ld_gv.  grad_params: device
 * double[3] = {d/d eps, d/d ld_min, d/d ld_max}, deterministic.  This entry point rebuilds
 * the residual planes of tm_tonemap_forward_train from the tables in its workspace and then
 * runs tm_tonemap_backward_resid.  Workspace: tm_backward_workspace_bytes. */
size_t tm_backward_workspace_bytes(int32_t H, int32_t W, const tm_params *p);
tm_status tm_tonemap_backward(const float *v, int64_t ld_v, int32_t H, int32_t W,
                              const void *sat, int64_t ld_sat, tm_sat_prec prec,
                              const float *offsets, const uint32_t *hist_cum,
                              int64_t ld_hist, int64_t plane_stride, const float *edges,
                              const tm_params *p, const float *grad_out, int64_t ld_g,
                              float *grad_v, int64_t ld_gv, double *grad_params, void *ws,
                              size_t ws_bytes, void *stream);

/* The same table-based backward for the log-domain variance variant: lum is the image i,
 * sat and log_offsets the integral image of l and its offsets (tm_integral_tables_log,
 * tm_prologue_log), hist_cum and edges those of i.  The residual planes are rebuilt from
 * these tables, then tm_tonemap_backward_resid_log gives the gradient with respect to i.
 * Equal bit for bit to tm_tonemap_forward_train of the same tables followed by
 * tm_tonemap_backward_resid_log.  Workspace, arguments and errors as for
 * tm_tonemap_backward. */
tm_status tm_tonemap_backward_log(const float *lum, int64_t ld_lum, int32_t H, int32_t W,
                                  const void *sat, int64_t ld_sat, tm_sat_prec prec,
                                  const float *log_offsets, const uint32_t *hist_cum,
                                  int64_t ld_hist, int64_t plane_stride, const float *edges,
                                  const tm_params *p, const float *grad_out, int64_t ld_g,
                                  float *grad_lum, int64_t ld_gl, double *grad_params, void *ws,
                                  size_t ws_bytes, void *stream);

/* ---------------------------------------------------------------- multi-exposure input */

/* The step before the method in the paper's application (Section III): the WDR image is
 * recovered from several 8-bit exposures with the method of Debevec and Malik.  For 8-bit
 * values z, pixel i and exposure j of time dt_j, the inverse log camera response
 * g(z) = ln f^-1(z) obeys g(Z_ij) = ln E_i + ln dt_j; values are trusted by the hat weight
 * w(z) = z (z <= 127), 255 - z (z >= 128).
 *
 * Exposure stacks: uint8, exposure j, channel c (R, G, B) of pixel (x, y) at
 * stack[j*exp_stride + c*ch_stride + y*ld + x], with ld >= W, ch_stride >= H*ld,
 * exp_stride >= 3*ch_stride; 1 <= P <= TM_HDR_MAX_EXPOSURES.  log_dt: device float[P], the
 * natural logs of the exposure times.  g: device float[3][256], one inverse log response
 * per channel. */
#define TM_HDR_MAX_EXPOSURES 16
#define TM_HDR_MAX_SAMPLE_VALUES 32768

/* Response recovery: per channel, g minimising
 *   sum_ij [w(Z_ij)(g(Z_ij) - ln E_i - ln dt_j)]^2 + lambda sum_{z=1..254} [w(z) g''(z)]^2,
 * g''(z) = g(z-1) - 2 g(z) + g(z+1), with g(128) = 0, over the n_samples pixels whose flat
 * indices y*W + x are in samples (device int32[n_samples]; an index outside the image makes
 * that sample count for nothing).  n_samples * P <= TM_HDR_MAX_SAMPLE_VALUES, lambda >= 0.
 * Solved in FP64 on the device (the per-sample ln E_i eliminated in closed form, then a
 * Cholesky factorisation); g is written as FP32.  If the samples leave the system singular
 * (too few distinct values) the channel's g is NaN.  Deterministic.
 * Workspace: tm_hdr_response_workspace_bytes(). */
size_t tm_hdr_response_workspace_bytes(void);
tm_status tm_hdr_response(const uint8_t *stack, int64_t exp_stride, int64_t ch_stride,
                          int64_t ld, int32_t P, int32_t H, int32_t W, const int32_t *samples,
                          int32_t n_samples, const float *log_dt, float lambda, float *g,
                          void *ws, size_t ws_bytes, void *stream);

/* Radiance map: per pixel and channel, ln E = sum_j w(Z_j)(g(Z_j) - ln dt_j) / sum_j w(Z_j)
 * (where every weight is 0, i.e. each value is 0 or 255, the unweighted mean of
 * g(Z_j) - ln dt_j), written as E = exp(ln E) in FP32 to the planar image rgb (channel c at
 * rgb + c*ch_stride_out, pitch ld_out), ready for tm_prologue / tm_tonemap_rgb.  No
 * workspace. */
tm_status tm_hdr_merge(const uint8_t *stack, int64_t exp_stride, int64_t ch_stride, int64_t ld,
                       int32_t P, int32_t H, int32_t W, const float *log_dt, const float *g,
                       float *rgb, int64_t ch_stride_out, int64_t ld_out, void *stream);

/* ---------------------------------------------------------------- batched forward */

/* One image of a batch.  The method (Section II) is applied to each image independently,
 * with its own statistics, tables and fields. */
typedef struct {
    const float *rgb;       /* planar RGB: channel c of (x, y) at rgb[c*ch_stride + y*ld_rgb + x] */
    int64_t ch_stride, ld_rgb;
    float *out;             /* tone-mapped luminance, H x W, row pitch ld_out */
    int64_t ld_out;
    int32_t H, W;
    int32_t rx[TM_MAX_SCALES], ry[TM_MAX_SCALES];   /* this image's fields (tm_paper_radii) */
} tm_image_desc;

/* Opaque host object holding a batch's layout in the caller's workspace, the device-side
 * descriptor tables and (after tm_batch_capture) an instantiated HIP graph. */
typedef struct tm_batch tm_batch;

/* Workspace for a batch: every image's luminance, statistics, integral image (prec),
 * cumulative histogram (p->n_bins - 1 planes) and scan aggregates, plus the descriptor
 * tables.  p supplies n_bins, n_scales, eps, ld_min, ld_max (its rx, ry are ignored). */
size_t tm_batch_workspace_bytes(const tm_image_desc *descs, int32_t count, const tm_params *p,
                                tm_sat_prec prec, const tm_tune *tune);

/* Lay the batch out in ws and upload its descriptor tables on `stream`: the copies are
 * enqueued and the call returns without synchronising; the object keeps their host source
 * buffers alive until tm_batch_destroy, so the caller must not destroy the batch before the
 * stream has passed those copies (any later synchronisation of the stream ensures it; the
 * batch's own launches on the same stream are ordered after them).  This call cannot be
 * captured into a HIP graph (it copies from pageable host memory).  descs is read during
 * the call only.  tune: one scan
 * tiling for all images, except that tile_w_vec = 0 and tile_h = 0 give every image the
 * library default for its own shape (NULL: {0, 0, 4}).  The images are processed in groups
 * of equal columns per lane; outputs go to each descriptor's own buffer. */
tm_status tm_batch_create(const tm_image_desc *descs, int32_t count, const tm_params *p,
                          tm_sat_prec prec, const tm_tune *tune, void *ws, size_t ws_bytes,
                          void *stream, tm_batch **batch);

/* The forward of every image.  The images are taken in consecutive groups whose integral
 * tables together stay within 160 MiB (so that the fused query finds them still in the
 * memory-side cache); for each group, one launch per phase covers all its images (prologue
 * parts, per-image finalize, scan stages 1-3, fused query) -- 6 launches per group, no host
 * sync.  With concurrency set (tm_batch_set_concurrency), the groups are dealt to internal
 * streams that start after the work already queued on `stream` and that `stream` waits for
 * at the end, so phases of different groups overlap; the call stays ordered on `stream` and
 * capturable into a graph. */
tm_status tm_batch_forward(tm_batch *batch, void *stream);

/* How tm_batch_forward spreads the work: `streams` (1..TM_BATCH_MAX_STREAMS) internal
 * streams (1: everything on the caller's stream, the default), created here at the default
 * priority and owned by the batch; at most `images_per_group` images per group (0: only the
 * table rule, 160 MiB divided by the number of streams).  Groups are dealt, in order, to the
 * stream with the fewest pixels so far.  Host call; not capturable itself.  Outputs are the
 * same bit for bit for any setting. */
#define TM_BATCH_MAX_STREAMS 8
tm_status tm_batch_set_concurrency(tm_batch *batch, int32_t streams, int32_t images_per_group);

/* Variance domain of the batch's forwards: 0 linear (Eq. 10 of i, the default), 1 the
 * log-domain variant (of l = ln max(i, FLT_MIN), as tm_prologue_log and
 * tm_integral_tables_log form it; the bins stay those of i).  Each image's output then equals
 * ToneMapper-style single-image calls of that variant bit for bit.  The device descriptor
 * table is updated by a copy on stream, and the call waits for the stream (so for the work
 * queued on it before); order any forward on another stream after it.  A graph captured
 * before is released: call tm_batch_capture again before replaying.  Host call; not
 * capturable itself. */
tm_status tm_batch_set_variance(tm_batch *batch, int32_t log_domain, void *stream);

/* Record tm_batch_forward into a HIP graph (stream must not be the null stream; nothing is
 * executed).  A later call replaces the graph. */
tm_status tm_batch_capture(tm_batch *batch, void *stream);

/* Launch the captured graph on stream. */
tm_status tm_batch_replay(tm_batch *batch, void *stream);

tm_status tm_batch_destroy(tm_batch *batch);

/* Device buffers of image i inside the workspace (luminance with its pitch, bin edges, the
 * C32X2 offsets, the integral image origin and pitch, the cumulative planes). */
tm_status tm_batch_image_buffers(const tm_batch *batch, int32_t i, float **lum, int64_t *ld_lum,
                                 float **edges, float **offsets, void **sat, int64_t *ld_sat,
                                 uint32_t **hist, int64_t *ld_hist, int64_t *plane_stride);

#ifdef __cplusplus
}
#endif

#endif /* TM_H */
