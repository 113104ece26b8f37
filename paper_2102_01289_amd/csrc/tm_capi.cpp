// tm_capi.cpp -- the C ABI declared in include/tm.h: host-side argument checks, workspace
// sizing and kernel dispatch.  Nothing here computes on the host.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdint>

#include "../../include/tm.h"
#include "tm_internal.h"

using namespace tmo;

namespace {

constexpr int64_t kMaxEntries = (int64_t)1 << 31;

bool aligned(const void *p, uintptr_t a) { return ((uintptr_t)p & (a - 1)) == 0; }

tm_status check_image(int32_t H, int32_t W) {
    if (H < 1 || W < 1 || W > TM_MAX_WIDTH) return TM_ERR_SHAPE;
    if ((int64_t)H * W >= kMaxEntries) return TM_ERR_SHAPE;
    return TM_OK;
}

tm_status check_plane(int32_t H, int32_t W, int64_t ld) {
    if (ld < W) return TM_ERR_SHAPE;
    if ((int64_t)H * ld >= kMaxEntries) return TM_ERR_SHAPE;
    return TM_OK;
}

// A table in the documented layout: ld >= W+1, ld % 4 == 0, < 2^31 entries incl. border.
tm_status check_table(int32_t H, int32_t W, int64_t ld, const void *t0) {
    if (ld < (int64_t)W + 1 || ld % 4 != 0) return TM_ERR_SHAPE;
    if (((int64_t)H + 1) * ld + 1 >= kMaxEntries) return TM_ERR_SHAPE;
    if (!t0) return TM_ERR_ARG;
    if (!aligned(t0, 16)) return TM_ERR_ALIGN;
    return TM_OK;
}

tm_status check_hist(int32_t H, int32_t W, int64_t ld, int64_t stride, const void *h,
                     int planes) {
    tm_status s = check_table(H, W, ld, h);
    if (s != TM_OK) return s;
    if (planes > 1) {
        if (stride < ((int64_t)H + 1) * ld + 1 || stride % 4 != 0) return TM_ERR_SHAPE;
        if (stride * (planes - 1) + (int64_t)H * ld >= ((int64_t)1 << 40)) return TM_ERR_SHAPE;
    }
    return TM_OK;
}

tm_status check_ws(void *ws, size_t have, size_t need) {
    if (need == 0) return TM_OK;
    if (!ws) return TM_ERR_WORKSPACE;
    if (!aligned(ws, 256)) return TM_ERR_WORKSPACE;
    if (have < need) return TM_ERR_WORKSPACE;
    return TM_OK;
}

tm_status check_params(const tm_params *p) {
    if (!p) return TM_ERR_ARG;
    if (p->n_bins < 1 || p->n_bins > TM_MAX_BINS) return TM_ERR_ARG;
    if (p->n_scales < 1 || p->n_scales > TM_MAX_SCALES) return TM_ERR_ARG;
    for (int j = 0; j < p->n_scales; ++j)
        if (p->rx[j] < 0 || p->ry[j] < 0) return TM_ERR_ARG;
    if (p->scalars) {   // device values: read by the kernels, not checkable here
        if (!aligned(p->scalars, 4)) return TM_ERR_ALIGN;
        return TM_OK;
    }
    if (!(p->eps > 0.f) || !std::isfinite(p->eps)) return TM_ERR_ARG;
    if (!std::isfinite(p->ld_min) || !std::isfinite(p->ld_max) || !(p->ld_max > p->ld_min))
        return TM_ERR_ARG;
    return TM_OK;
}

bool valid_prec(int prec) { return prec == TM_SAT_F32 || prec == TM_SAT_C32X2 || prec == TM_SAT_F64; }

tm_status from_hip(hipError_t e) { return e == hipSuccess ? TM_OK : TM_ERR_HIP; }

ScanTune resolve_tune(const tm_tune *t, int H, int W, int n_bins, tm_status *st) {
    *st = TM_OK;
    if (!t) return scan_tune_default(H, W, n_bins);
    ScanTune r{t->tile_w_vec, t->tile_h, t->bin_chunk};
    if (!scan_tune_valid(r)) *st = TM_ERR_ARG;
    return r;
}

size_t round256(size_t a) { return (a + 255) / 256 * 256; }

// Kernel parameters of an H x W image.  A radius of at least the image's width (height)
// already covers the whole row (column) at every pixel under Algorithm 1's clamping, so radii
// are clamped to W and H: the windows are the same and every index expression of the kernels
// (x + rx, 2 rmin + 1, ...) stays far from int32 overflow.
QueryParams to_query(const tm_params *p, int32_t H, int32_t W) {
    QueryParams q{};
    q.n_bins = p->n_bins;
    q.n_scales = p->n_scales;
    for (int j = 0; j < TM_MAX_SCALES; ++j) {
        q.rx[j] = j < p->n_scales ? (p->rx[j] < W ? p->rx[j] : W) : 0;
        q.ry[j] = j < p->n_scales ? (p->ry[j] < H ? p->ry[j] : H) : 0;
    }
    q.eps = p->eps;
    q.ld_min = p->ld_min;
    q.ld_max = p->ld_max;
    q.scalars = p->scalars;
    return q;
}

#define TM_TRY(expr)                      \
    do {                                  \
        tm_status _s = (expr);            \
        if (_s != TM_OK) return _s;       \
    } while (0)

}  // namespace

extern "C" {

const char *tm_status_string(tm_status s) {
    switch (s) {
        case TM_OK: return "ok";
        case TM_ERR_ARG: return "invalid argument";
        case TM_ERR_SHAPE: return "invalid shape, pitch or stride";
        case TM_ERR_ALIGN: return "misaligned pointer";
        case TM_ERR_WORKSPACE: return "workspace missing, misaligned or too small";
        case TM_ERR_HIP: return "HIP runtime error";
        case TM_ERR_UNSUPPORTED: return "unsupported";
    }
    return "unknown status";
}

tm_status tm_paper_radii(int32_t H, int32_t W, tm_params *p) {
    if (!p) return TM_ERR_ARG;
    TM_TRY(check_image(H, W));
    if (p->n_scales < 1 || p->n_scales > TM_MAX_SCALES) return TM_ERR_ARG;
    for (int j = 0; j < p->n_scales; ++j) {
        p->rx[j] = W >> (j + 1);
        p->ry[j] = H >> (j + 1);
    }
    return TM_OK;
}

tm_status tm_default_tune(int32_t H, int32_t W, int32_t n_bins, tm_tune *t) {
    if (!t || n_bins < 0 || n_bins > TM_MAX_BINS) return TM_ERR_ARG;
    TM_TRY(check_image(H, W));
    const ScanTune d = scan_tune_default(H, W, n_bins);
    t->tile_w_vec = d.vec;
    t->tile_h = d.th;
    t->bin_chunk = d.chunk;
    return TM_OK;
}

tm_status tm_table_geometry(int32_t H, int32_t W, int64_t *ld, int64_t *origin_offset,
                            int64_t *elems) {
    TM_TRY(check_image(H, W));
    const int64_t l = ((int64_t)W + 1 + 63) / 64 * 64;
    const int64_t o = (l + 1 + 63) / 64 * 64;
    const int64_t e = (o + (int64_t)H * l + 63) / 64 * 64;
    if (e >= kMaxEntries) return TM_ERR_SHAPE;
    if (ld) *ld = l;
    if (origin_offset) *origin_offset = o;
    if (elems) *elems = e;
    return TM_OK;
}

// ------------------------------------------------------------------ a1
tm_status tm_luminance(const float *rgb, int64_t ch_stride, int64_t ld_rgb, int32_t H,
                       int32_t W, float *lum, int64_t ld_lum, void *stream) {
    TM_TRY(check_image(H, W));
    if (!rgb || !lum) return TM_ERR_ARG;
    TM_TRY(check_plane(H, W, ld_rgb));
    TM_TRY(check_plane(H, W, ld_lum));
    if (ch_stride < (int64_t)H * ld_rgb) return TM_ERR_SHAPE;
    return from_hip(launch_luminance(rgb, ch_stride, ld_rgb, H, W, lum, ld_lum,
                                     (hipStream_t)stream));
}

size_t tm_image_stats_workspace_bytes(int32_t H, int32_t W) {
    if (check_image(H, W) != TM_OK) return 0;
    return round256((size_t)stats_blocks(H, W) * sizeof(StatsPartial));
}

tm_status tm_image_stats(const float *lum, int64_t ld_lum, int32_t H, int32_t W,
                         int32_t n_bins, float *edges, float *offsets, float *minmax,
                         void *ws, size_t ws_bytes, void *stream) {
    TM_TRY(check_image(H, W));
    if (!lum || n_bins < 1 || n_bins > TM_MAX_BINS) return TM_ERR_ARG;
    if (n_bins > 1 && !edges) return TM_ERR_ARG;
    TM_TRY(check_plane(H, W, ld_lum));
    TM_TRY(check_ws(ws, ws_bytes, tm_image_stats_workspace_bytes(H, W)));
    return from_hip(launch_stats(nullptr, 0, 0, lum, ld_lum, nullptr, 0, H, W, n_bins, edges,
                                 offsets, minmax, static_cast<StatsPartial *>(ws),
                                 (hipStream_t)stream));
}

tm_status tm_prologue(const float *rgb, int64_t ch_stride, int64_t ld_rgb, int32_t H,
                      int32_t W, int32_t n_bins, float *lum, int64_t ld_lum, float *edges,
                      float *offsets, float *minmax, void *ws, size_t ws_bytes, void *stream) {
    TM_TRY(check_image(H, W));
    if (!rgb || !lum || n_bins < 1 || n_bins > TM_MAX_BINS) return TM_ERR_ARG;
    if (n_bins > 1 && !edges) return TM_ERR_ARG;
    TM_TRY(check_plane(H, W, ld_rgb));
    TM_TRY(check_plane(H, W, ld_lum));
    if (ch_stride < (int64_t)H * ld_rgb) return TM_ERR_SHAPE;
    TM_TRY(check_ws(ws, ws_bytes, tm_image_stats_workspace_bytes(H, W)));
    return from_hip(launch_stats(rgb, ch_stride, ld_rgb, nullptr, 0, lum, ld_lum, H, W, n_bins,
                                 edges, offsets, minmax, static_cast<StatsPartial *>(ws),
                                 (hipStream_t)stream));
}

tm_status tm_prologue_noalloc(const float *rgb, int64_t ch_stride, int64_t ld_rgb, int32_t H,
                              int32_t W, int32_t n_bins, float *lum, int64_t ld_lum,
                              float *edges, float *offsets, float *minmax, void *stream) {
    TM_TRY(check_image(H, W));
    if (!rgb || !lum || n_bins < 1 || n_bins > TM_MAX_BINS) return TM_ERR_ARG;
    if (n_bins > 1 && !edges) return TM_ERR_ARG;
    TM_TRY(check_plane(H, W, ld_rgb));
    TM_TRY(check_plane(H, W, ld_lum));
    if (ch_stride < (int64_t)H * ld_rgb) return TM_ERR_SHAPE;
    static_assert(TM_PROLOGUE_SCRATCH_BYTES == kPrologueScratchBytes, "scratch size");
    if (tm_image_stats_workspace_bytes(H, W) > kPrologueScratchBytes) return TM_ERR_UNSUPPORTED;
    return from_hip(launch_stats_noalloc(rgb, ch_stride, ld_rgb, lum, ld_lum, H, W, n_bins,
                                         edges, offsets, minmax, (hipStream_t)stream));
}

tm_status tm_prologue_log(const float *rgb, int64_t ch_stride, int64_t ld_rgb, int32_t H,
                          int32_t W, int32_t n_bins, float *lum, int64_t ld_lum, float *logv,
                          int64_t ld_log, float *edges, float *log_offsets, float *minmax,
                          void *ws, size_t ws_bytes, void *stream) {
    TM_TRY(check_image(H, W));
    if (!rgb || !lum || n_bins < 1 || n_bins > TM_MAX_BINS) return TM_ERR_ARG;
    if (n_bins > 1 && !edges) return TM_ERR_ARG;
    TM_TRY(check_plane(H, W, ld_rgb));
    TM_TRY(check_plane(H, W, ld_lum));
    if (logv) TM_TRY(check_plane(H, W, ld_log));
    if (ch_stride < (int64_t)H * ld_rgb) return TM_ERR_SHAPE;
    if (logv) {   // the two output planes must be disjoint
        const char *a0 = reinterpret_cast<const char *>(lum);
        const char *a1 = a0 + (((int64_t)H - 1) * ld_lum + W) * 4;
        const char *b0 = reinterpret_cast<const char *>(logv);
        const char *b1 = b0 + (((int64_t)H - 1) * ld_log + W) * 4;
        if (a0 < b1 && b0 < a1) return TM_ERR_ARG;
    }
    TM_TRY(check_ws(ws, ws_bytes, tm_image_stats_workspace_bytes(H, W)));
    return from_hip(launch_stats_log(rgb, ch_stride, ld_rgb, lum, ld_lum, logv, ld_log, H, W,
                                     n_bins, edges, log_offsets, minmax,
                                     static_cast<StatsPartial *>(ws), (hipStream_t)stream));
}

tm_status tm_log_luminance(const float *lum, int64_t ld_lum, int32_t H, int32_t W, float *logv,
                           int64_t ld_log, float *offsets, float *minmax, void *ws,
                           size_t ws_bytes, void *stream) {
    TM_TRY(check_image(H, W));
    if (!lum) return TM_ERR_ARG;
    TM_TRY(check_plane(H, W, ld_lum));
    if (logv) TM_TRY(check_plane(H, W, ld_log));
    TM_TRY(check_ws(ws, ws_bytes, tm_image_stats_workspace_bytes(H, W)));
    return from_hip(launch_log_stats(lum, ld_lum, logv, ld_log, H, W, offsets, minmax,
                                     static_cast<StatsPartial *>(ws), (hipStream_t)stream));
}

tm_status tm_log_luminance_backward(const float *lum, int64_t ld_lum, int32_t H, int32_t W,
                                    const float *grad_l, int64_t ld_gl, float *grad_i,
                                    int64_t ld_gi, void *stream) {
    TM_TRY(check_image(H, W));
    if (!lum || !grad_l || !grad_i) return TM_ERR_ARG;
    TM_TRY(check_plane(H, W, ld_lum));
    TM_TRY(check_plane(H, W, ld_gl));
    TM_TRY(check_plane(H, W, ld_gi));
    // in place (same buffer, same pitch) or disjoint: a partial overlap would let one pixel's
    // result land on another pixel's unread input
    if (grad_i != grad_l) {
        const char *a0 = reinterpret_cast<const char *>(grad_l);
        const char *a1 = a0 + (((int64_t)H - 1) * ld_gl + W) * 4;
        const char *b0 = reinterpret_cast<const char *>(grad_i);
        const char *b1 = b0 + (((int64_t)H - 1) * ld_gi + W) * 4;
        if (a0 < b1 && b0 < a1) return TM_ERR_ARG;
    } else if (ld_gi != ld_gl) {
        return TM_ERR_ARG;
    }
    return from_hip(launch_log_chain(lum, ld_lum, grad_l, ld_gl, grad_i, ld_gi, H, W,
                                     (hipStream_t)stream));
}

// ------------------------------------------------------------------ exposures
namespace {
tm_status check_stack(const uint8_t *stack, int64_t exp_stride, int64_t ch_stride, int64_t ld,
                      int32_t P, int32_t H, int32_t W) {
    TM_TRY(check_image(H, W));
    if (!stack) return TM_ERR_ARG;
    if (P < 1 || P > TM_HDR_MAX_EXPOSURES) return TM_ERR_ARG;
    if (ld < W || ch_stride < (int64_t)H * ld || exp_stride < 3 * ch_stride) return TM_ERR_SHAPE;
    if (exp_stride > ((int64_t)1 << 40) / P) return TM_ERR_SHAPE;
    return TM_OK;
}
}  // namespace

size_t tm_hdr_response_workspace_bytes(void) { return round256(hdr_response_ws_bytes()); }

tm_status tm_hdr_response(const uint8_t *stack, int64_t exp_stride, int64_t ch_stride,
                          int64_t ld, int32_t P, int32_t H, int32_t W, const int32_t *samples,
                          int32_t n_samples, const float *log_dt, float lambda, float *g,
                          void *ws, size_t ws_bytes, void *stream) {
    TM_TRY(check_stack(stack, exp_stride, ch_stride, ld, P, H, W));
    if (!samples || !log_dt || !g) return TM_ERR_ARG;
    if (n_samples < 1 || (int64_t)n_samples * P > TM_HDR_MAX_SAMPLE_VALUES) return TM_ERR_ARG;
    if (!(lambda >= 0.f) || !std::isfinite(lambda)) return TM_ERR_ARG;
    TM_TRY(check_ws(ws, ws_bytes, tm_hdr_response_workspace_bytes()));
    return from_hip(launch_hdr_response(stack, exp_stride, ch_stride, ld, P, H, W, samples,
                                        n_samples, log_dt, lambda, g, ws, (hipStream_t)stream));
}

tm_status tm_hdr_merge(const uint8_t *stack, int64_t exp_stride, int64_t ch_stride, int64_t ld,
                       int32_t P, int32_t H, int32_t W, const float *log_dt, const float *g,
                       float *rgb, int64_t ch_stride_out, int64_t ld_out, void *stream) {
    TM_TRY(check_stack(stack, exp_stride, ch_stride, ld, P, H, W));
    if (!log_dt || !g || !rgb) return TM_ERR_ARG;
    TM_TRY(check_plane(H, W, ld_out));
    if (ch_stride_out < (int64_t)H * ld_out) return TM_ERR_SHAPE;
    if (3 * ch_stride_out >= ((int64_t)1 << 40)) return TM_ERR_SHAPE;
    return from_hip(launch_hdr_merge(stack, exp_stride, ch_stride, ld, P, H, W, log_dt, g, rgb,
                                     ch_stride_out, ld_out, (hipStream_t)stream));
}

// ------------------------------------------------------------------ a2, a3
size_t tm_tables_workspace_bytes(int32_t H, int32_t W, int32_t n_bins, tm_sat_prec prec,
                                 const tm_tune *tune) {
    if (check_image(H, W) != TM_OK || !valid_prec(prec) || n_bins < 1 || n_bins > TM_MAX_BINS)
        return 0;
    tm_status st;
    ScanTune t = resolve_tune(tune, H, W, n_bins, &st);
    if (st != TM_OK) return 0;
    return make_scan_plan(H, W, (int)prec, n_bins, t).total;
}

// v_hist: the plane the histogram bins (null: v); log_src: the integral image is of
// ln max(v, FLT_MIN)
static tm_status run_tables(const float *v, int64_t ld_v, const float *v_hist,
                            int64_t ld_v_hist, int32_t H, int32_t W, tm_sat_prec prec,
                            const float *offsets, void *sat, int64_t ld_sat,
                            const float *edges, int32_t n_bins, tm_hist_layout layout,
                            uint32_t *hist, int64_t ld_hist, int64_t plane_stride,
                            const tm_tune *tune, void *ws, size_t ws_bytes, void *stream,
                            bool log_src = false) {
    TM_TRY(check_image(H, W));
    if (!v) return TM_ERR_ARG;
    TM_TRY(check_plane(H, W, ld_v));
    if (v_hist) TM_TRY(check_plane(H, W, ld_v_hist));
    if (!sat && !hist) return TM_ERR_ARG;
    int n_planes = 0;
    if (sat) {
        if (!valid_prec(prec)) return TM_ERR_ARG;
        TM_TRY(check_table(H, W, ld_sat, sat));
        if (prec == TM_SAT_C32X2 && !offsets) return TM_ERR_ARG;
    }
    if (hist) {
        if (n_bins < 1 || n_bins > TM_MAX_BINS) return TM_ERR_ARG;
        if (layout != TM_HIST_PER_BIN && layout != TM_HIST_CUMULATIVE) return TM_ERR_ARG;
        n_planes = layout == TM_HIST_PER_BIN ? n_bins : n_bins - 1;
        if (n_planes > 0) {
            if (n_bins > 1 && !edges) return TM_ERR_ARG;
            TM_TRY(check_hist(H, W, ld_hist, plane_stride, hist, n_planes));
        }
    }
    tm_status st;
    ScanTune t = resolve_tune(tune, H, W, n_bins, &st);
    TM_TRY(st);
    const int sp = sat ? (int)prec : -1;
    ScanPlan plan = make_scan_plan(H, W, sp, n_planes, t);
    // the workspace query assumes a full-precision integral image and n_bins planes
    TM_TRY(check_ws(ws, ws_bytes, plan.total));
    if (!sat && n_planes == 0) return TM_OK;
    ScanArgs a{};
    a.v = v;
    a.ld_v = ld_v;
    a.v_hist = v_hist;
    a.ld_v_hist = ld_v_hist;
    a.log_src = log_src ? 1 : 0;
    a.H = H;
    a.W = W;
    a.sat_prec = sp;
    a.offsets = offsets;
    a.sat = sat;
    a.ld_sat = ld_sat;
    a.edges = edges;
    a.n_bins = n_bins;
    a.layout = (int)layout;
    a.n_planes = n_planes;
    a.hist = n_planes > 0 ? hist : nullptr;
    a.ld_hist = ld_hist;
    a.plane_stride = plane_stride;
    return from_hip(launch_tables(a, plan, ws, (hipStream_t)stream));
}

tm_status tm_integral_tables(const float *v, int64_t ld_v, int32_t H, int32_t W,
                             tm_sat_prec prec, const float *offsets, void *sat,
                             int64_t ld_sat, const float *edges, int32_t n_bins,
                             tm_hist_layout layout, uint32_t *hist, int64_t ld_hist,
                             int64_t plane_stride, const tm_tune *tune, void *ws,
                             size_t ws_bytes, void *stream) {
    return run_tables(v, ld_v, nullptr, 0, H, W, prec, offsets, sat, ld_sat, edges, n_bins,
                      layout, hist, ld_hist, plane_stride, tune, ws, ws_bytes, stream);
}

tm_status tm_integral_tables_split(const float *v_sat, int64_t ld_v_sat, const float *v_hist,
                                   int64_t ld_v_hist, int32_t H, int32_t W, tm_sat_prec prec,
                                   const float *offsets, void *sat, int64_t ld_sat,
                                   const float *edges, int32_t n_bins, tm_hist_layout layout,
                                   uint32_t *hist, int64_t ld_hist, int64_t plane_stride,
                                   const tm_tune *tune, void *ws, size_t ws_bytes,
                                   void *stream) {
    if (!v_sat || !v_hist || !sat || !hist) return TM_ERR_ARG;
    return run_tables(v_sat, ld_v_sat, v_hist, ld_v_hist, H, W, prec, offsets, sat, ld_sat,
                      edges, n_bins, layout, hist, ld_hist, plane_stride, tune, ws, ws_bytes,
                      stream);
}

tm_status tm_integral_tables_log(const float *lum, int64_t ld_lum, int32_t H, int32_t W,
                                 tm_sat_prec prec, const float *log_offsets, void *sat,
                                 int64_t ld_sat, const float *edges, int32_t n_bins,
                                 tm_hist_layout layout, uint32_t *hist, int64_t ld_hist,
                                 int64_t plane_stride, const tm_tune *tune, void *ws,
                                 size_t ws_bytes, void *stream) {
    if (!sat) return TM_ERR_ARG;
    return run_tables(lum, ld_lum, nullptr, 0, H, W, prec, log_offsets, sat, ld_sat, edges,
                      n_bins, layout, hist, ld_hist, plane_stride, tune, ws, ws_bytes, stream,
                      true);
}

tm_status tm_integral_image(const float *v, int64_t ld_v, int32_t H, int32_t W,
                            tm_sat_prec prec, const float *offsets, void *sat,
                            int64_t ld_sat, const tm_tune *tune, void *ws, size_t ws_bytes,
                            void *stream) {
    if (!sat) return TM_ERR_ARG;
    return tm_integral_tables(v, ld_v, H, W, prec, offsets, sat, ld_sat, nullptr, 1,
                              TM_HIST_CUMULATIVE, nullptr, 0, 0, tune, ws, ws_bytes, stream);
}

tm_status tm_integral_histogram(const float *v, int64_t ld_v, int32_t H, int32_t W,
                                const float *edges, int32_t n_bins, tm_hist_layout layout,
                                uint32_t *hist, int64_t ld_hist, int64_t plane_stride,
                                const tm_tune *tune, void *ws, size_t ws_bytes,
                                void *stream) {
    if (!hist) return TM_ERR_ARG;
    return tm_integral_tables(v, ld_v, H, W, TM_SAT_F32, nullptr, nullptr, 0, edges, n_bins,
                              layout, hist, ld_hist, plane_stride, tune, ws, ws_bytes, stream);
}

// the single-pass histogram: planes of a layout; counts in its records take 30 bits, so
// H < 2^30 (row counts are below W <= 2^24)
namespace {
int lookback_planes(int32_t n_bins, tm_hist_layout layout) {
    return layout == TM_HIST_PER_BIN ? n_bins : n_bins - 1;
}
}  // namespace

size_t tm_lookback_workspace_bytes(int32_t H, int32_t W, int32_t n_bins, tm_hist_layout layout) {
    if (check_image(H, W) != TM_OK || n_bins < 1 || n_bins > TM_MAX_BINS) return 0;
    if (layout != TM_HIST_PER_BIN && layout != TM_HIST_CUMULATIVE) return 0;
    const int np = lookback_planes(n_bins, layout);
    if (np < 1 || np > 8 || H >= (1 << 30)) return 0;
    return make_lookback_plan(H, W, np, lookback_rows(H, W, np)).total;
}

void tm_lookback_set_spin_limit(uint32_t polls) { set_lookback_spin_limit(polls); }

tm_status tm_integral_histogram_lookback(const float *v, int64_t ld_v, int32_t H, int32_t W,
                                         const float *edges, int32_t n_bins,
                                         tm_hist_layout layout, uint32_t *hist, int64_t ld_hist,
                                         int64_t plane_stride, void *ws, size_t ws_bytes,
                                         void *stream) {
    TM_TRY(check_image(H, W));
    if (!v || !hist) return TM_ERR_ARG;
    TM_TRY(check_plane(H, W, ld_v));
    if (n_bins < 1 || n_bins > TM_MAX_BINS) return TM_ERR_ARG;
    if (layout != TM_HIST_PER_BIN && layout != TM_HIST_CUMULATIVE) return TM_ERR_ARG;
    const int np = lookback_planes(n_bins, layout);
    if (np == 0) return TM_OK;
    if (np > 8 || H >= (1 << 30)) return TM_ERR_UNSUPPORTED;
    if (n_bins > 1 && !edges) return TM_ERR_ARG;
    TM_TRY(check_hist(H, W, ld_hist, plane_stride, hist, np));
    const LookbackPlan plan = make_lookback_plan(H, W, np, lookback_rows(H, W, np));
    TM_TRY(check_ws(ws, ws_bytes, plan.total));
    LookbackArgs a{};
    a.v = v;
    a.ld_v = ld_v;
    a.H = H;
    a.W = W;
    a.edges = edges;
    a.n_bins = n_bins;
    a.n_planes = np;
    a.layout = layout == TM_HIST_PER_BIN ? 0 : 1;
    a.hist = hist;
    a.ld_hist = ld_hist;
    a.plane_stride = plane_stride;
    // planes larger than the memory-side cache are written non-temporally, as by the scan
    a.nt = (int64_t)np * plane_stride * 4 > ((int64_t)256 << 20);
    return from_hip(launch_lookback_hist(a, plan, ws, static_cast<hipStream_t>(stream)));
}

// ------------------------------------------------------------------ a4
tm_status tm_tonemap_forward(const float *v, int64_t ld_v, int32_t H, int32_t W,
                             const void *sat, int64_t ld_sat, tm_sat_prec prec,
                             const float *offsets, const uint32_t *hist_cum, int64_t ld_hist,
                             int64_t plane_stride, const float *edges, const tm_params *p,
                             float *out, int64_t ld_out, void *stream) {
    TM_TRY(check_image(H, W));
    TM_TRY(check_params(p));
    if (!v || !out || !valid_prec(prec)) return TM_ERR_ARG;
    TM_TRY(check_plane(H, W, ld_v));
    TM_TRY(check_plane(H, W, ld_out));
    TM_TRY(check_table(H, W, ld_sat, sat));
    if (prec == TM_SAT_C32X2 && !offsets) return TM_ERR_ARG;
    if (p->n_bins > 1) {
        if (!edges) return TM_ERR_ARG;
        TM_TRY(check_hist(H, W, ld_hist, plane_stride, hist_cum, p->n_bins - 1));
    }
    const QueryParams q = to_query(p, H, W);
    return from_hip(launch_forward(v, ld_v, H, W, sat, ld_sat, (int)prec, offsets, hist_cum,
                                   ld_hist, plane_stride, edges, q, out, ld_out, nullptr,
                                   (hipStream_t)stream));
}

tm_status tm_tonemap_forward_maps(const float *v, int64_t ld_v, int32_t H, int32_t W,
                                  const void *sat, int64_t ld_sat, tm_sat_prec prec,
                                  const float *offsets, const uint32_t *hist_cum,
                                  int64_t ld_hist, int64_t plane_stride, const float *edges,
                                  const tm_params *p, float *out, int64_t ld_out, float *maps,
                                  void *stream) {
    TM_TRY(check_image(H, W));
    TM_TRY(check_params(p));
    if (!v || !out || !maps || !valid_prec(prec)) return TM_ERR_ARG;
    if (!aligned(maps, 4)) return TM_ERR_ALIGN;
    TM_TRY(check_plane(H, W, ld_v));
    TM_TRY(check_plane(H, W, ld_out));
    TM_TRY(check_table(H, W, ld_sat, sat));
    if (prec == TM_SAT_C32X2 && !offsets) return TM_ERR_ARG;
    if (p->n_bins > 1) {
        if (!edges) return TM_ERR_ARG;
        TM_TRY(check_hist(H, W, ld_hist, plane_stride, hist_cum, p->n_bins - 1));
    }
    const QueryParams q = to_query(p, H, W);
    return from_hip(launch_forward_maps(v, ld_v, H, W, sat, ld_sat, (int)prec, offsets, hist_cum,
                                        ld_hist, plane_stride, edges, q, out, ld_out, maps,
                                        (hipStream_t)stream));
}

tm_status tm_tonemap_forward_rgb(const float *v, int64_t ld_v, int32_t H, int32_t W,
                                 const void *sat, int64_t ld_sat, tm_sat_prec prec,
                                 const float *offsets, const uint32_t *hist_cum,
                                 int64_t ld_hist, int64_t plane_stride, const float *edges,
                                 const tm_params *p, const float *rgb, int64_t ch_stride,
                                 int64_t ld_rgb, float saturation, float *rgb_out,
                                 int64_t ch_stride_out, int64_t ld_rgb_out, float *out,
                                 int64_t ld_out, void *stream) {
    TM_TRY(check_image(H, W));
    TM_TRY(check_params(p));
    if (!v || !rgb || !rgb_out || !valid_prec(prec)) return TM_ERR_ARG;
    if (!(saturation >= 0.f) || !std::isfinite(saturation)) return TM_ERR_ARG;
    TM_TRY(check_plane(H, W, ld_v));
    TM_TRY(check_plane(H, W, ld_rgb));
    TM_TRY(check_plane(H, W, ld_rgb_out));
    if (ch_stride < (int64_t)H * ld_rgb || ch_stride_out < (int64_t)H * ld_rgb_out)
        return TM_ERR_SHAPE;
    if (out) TM_TRY(check_plane(H, W, ld_out));
    TM_TRY(check_table(H, W, ld_sat, sat));
    if (prec == TM_SAT_C32X2 && !offsets) return TM_ERR_ARG;
    if (p->n_bins > 1) {
        if (!edges) return TM_ERR_ARG;
        TM_TRY(check_hist(H, W, ld_hist, plane_stride, hist_cum, p->n_bins - 1));
    }
    const QueryParams q = to_query(p, H, W);
    return from_hip(launch_forward_rgb(v, ld_v, H, W, sat, ld_sat, (int)prec, offsets, hist_cum,
                                       ld_hist, plane_stride, edges, q, out, ld_out, rgb,
                                       ch_stride, ld_rgb, rgb_out, ch_stride_out, ld_rgb_out,
                                       saturation, (hipStream_t)stream));
}

// Buffers of the end-to-end RGB call, carved from its workspace (offsets in bytes).
struct RgbPlan {
    int64_t ld_lum, ld, org, elems;
    size_t lum, edges, stats, sat, hist, scan, total;
    size_t stats_bytes, scan_bytes;
};

static bool rgb_plan(int32_t H, int32_t W, const tm_params *p, tm_sat_prec prec, RgbPlan &r) {
    if (check_image(H, W) != TM_OK || check_params(p) != TM_OK || !valid_prec(prec)) return false;
    if (tm_table_geometry(H, W, &r.ld, &r.org, &r.elems) != TM_OK) return false;
    r.ld_lum = ((int64_t)W + 63) / 64 * 64;
    const size_t es = prec == TM_SAT_F32 ? 8 : 16;
    const int planes = p->n_bins > 1 ? p->n_bins - 1 : 0;
    r.stats_bytes = tm_image_stats_workspace_bytes(H, W);
    r.scan_bytes = tm_tables_workspace_bytes(H, W, p->n_bins, prec, nullptr);
    size_t off = 0;
    auto take = [&](size_t bytes) {
        const size_t o = off;
        off = (off + bytes + 255) / 256 * 256;
        return o;
    };
    r.lum = take(sizeof(float) * (size_t)H * (size_t)r.ld_lum);
    r.edges = take(sizeof(float) * 260);
    r.stats = take(r.stats_bytes);
    r.sat = take(es * (size_t)r.elems);
    r.hist = take(4 * (size_t)r.elems * (size_t)(planes > 0 ? planes : 1));
    r.scan = take(r.scan_bytes);
    r.total = off;
    return true;
}

size_t tm_tonemap_rgb_workspace_bytes(int32_t H, int32_t W, const tm_params *p,
                                      tm_sat_prec prec) {
    RgbPlan r;
    return rgb_plan(H, W, p, prec, r) ? r.total : 0;
}

tm_status tm_tonemap_rgb(const float *rgb, int64_t ch_stride, int64_t ld_rgb, int32_t H,
                         int32_t W, const tm_params *p, tm_sat_prec prec, float saturation,
                         float *rgb_out, int64_t ch_stride_out, int64_t ld_rgb_out, void *ws,
                         size_t ws_bytes, void *stream) {
    RgbPlan r;
    if (!rgb_plan(H, W, p, prec, r)) {
        TM_TRY(check_image(H, W));
        TM_TRY(check_params(p));
        return TM_ERR_ARG;
    }
    if (!rgb || !rgb_out) return TM_ERR_ARG;
    TM_TRY(check_ws(ws, ws_bytes, r.total));
    char *w = static_cast<char *>(ws);
    float *lum = reinterpret_cast<float *>(w + r.lum);
    float *edges = reinterpret_cast<float *>(w + r.edges);
    float *offsets = edges + 256, *minmax = edges + 258;
    const size_t es = prec == TM_SAT_F32 ? 8 : 16;
    void *sat = w + r.sat + (size_t)r.org * es;
    uint32_t *hist = p->n_bins > 1 ? reinterpret_cast<uint32_t *>(w + r.hist) + r.org : nullptr;
    TM_TRY(tm_prologue(rgb, ch_stride, ld_rgb, H, W, p->n_bins, lum, r.ld_lum, edges, offsets,
                       minmax, w + r.stats, r.stats_bytes, stream));
    TM_TRY(tm_integral_tables(lum, r.ld_lum, H, W, prec, offsets, sat, r.ld, edges, p->n_bins,
                              TM_HIST_CUMULATIVE, hist, r.ld, r.elems, nullptr, w + r.scan,
                              r.scan_bytes, stream));
    return tm_tonemap_forward_rgb(lum, r.ld_lum, H, W, sat, r.ld, prec, offsets, hist, r.ld,
                                  r.elems, edges, p, rgb, ch_stride, ld_rgb, saturation, rgb_out,
                                  ch_stride_out, ld_rgb_out, nullptr, 0, stream);
}

int32_t tm_residual_planes(int32_t n_scales) {
    return (n_scales < 1 || n_scales > TM_MAX_SCALES) ? 0 : 2 * n_scales + 2;
}

tm_status tm_tonemap_forward_train(const float *v, int64_t ld_v, int32_t H, int32_t W,
                                   const void *sat, int64_t ld_sat, tm_sat_prec prec,
                                   const float *offsets, const uint32_t *hist_cum,
                                   int64_t ld_hist, int64_t plane_stride, const float *edges,
                                   const tm_params *p, float *out, int64_t ld_out, float *resid,
                                   void *stream) {
    if (!resid) return TM_ERR_ARG;
    if (!aligned(resid, 8)) return TM_ERR_ALIGN;   // pair planes are read as 8-byte pairs
    TM_TRY(check_image(H, W));
    TM_TRY(check_params(p));
    if (!v || !out || !valid_prec(prec)) return TM_ERR_ARG;
    TM_TRY(check_plane(H, W, ld_v));
    TM_TRY(check_plane(H, W, ld_out));
    TM_TRY(check_table(H, W, ld_sat, sat));
    if (prec == TM_SAT_C32X2 && !offsets) return TM_ERR_ARG;
    if (p->n_bins > 1) {
        if (!edges) return TM_ERR_ARG;
        TM_TRY(check_hist(H, W, ld_hist, plane_stride, hist_cum, p->n_bins - 1));
    }
    const QueryParams q = to_query(p, H, W);
    return from_hip(launch_forward(v, ld_v, H, W, sat, ld_sat, (int)prec, offsets, hist_cum,
                                   ld_hist, plane_stride, edges, q, out, ld_out, resid,
                                   (hipStream_t)stream));
}

// ------------------------------------------------------------------ a5
size_t tm_backward_workspace_bytes(int32_t H, int32_t W, const tm_params *p) {
    if (check_image(H, W) != TM_OK || check_params(p) != TM_OK) return 0;
    return make_bwd_plan(H, W, p->n_scales, to_query(p, H, W).ry, true).total;
}

size_t tm_backward_resid_workspace_bytes(int32_t H, int32_t W, const tm_params *p) {
    if (check_image(H, W) != TM_OK || check_params(p) != TM_OK) return 0;
    return make_bwd_plan(H, W, p->n_scales, to_query(p, H, W).ry, false).total;
}

static tm_status run_backward_resid(const float *v, int64_t ld_v, int32_t H, int32_t W,
                                    const tm_params *p, const float *resid,
                                    const float *grad_out, int64_t ld_g, float *grad_v,
                                    int64_t ld_gv, double *grad_params, const BwdPlan &plan,
                                    void *ws, hipStream_t s, bool log_chain = false) {
    BwdResidArgs a{};
    a.v = v;
    a.ld_v = ld_v;
    a.H = H;
    a.W = W;
    a.p = to_query(p, H, W);
    a.resid = resid;
    a.g = grad_out;
    a.ld_g = ld_g;
    a.grad_v = grad_v;
    a.ld_gv = ld_gv;
    a.grad_params = grad_params;
    a.log_chain = log_chain;
    return from_hip(launch_backward_resid(a, plan, ws, s));
}

static tm_status check_bwd_common(const float *v, int64_t ld_v, int32_t H, int32_t W,
                                  const tm_params *p, const float *grad_out, int64_t ld_g,
                                  float *grad_v, int64_t ld_gv, double *grad_params) {
    TM_TRY(check_image(H, W));
    TM_TRY(check_params(p));
    if (!v || !grad_out || !grad_v || !grad_params) return TM_ERR_ARG;
    TM_TRY(check_plane(H, W, ld_v));
    TM_TRY(check_plane(H, W, ld_g));
    TM_TRY(check_plane(H, W, ld_gv));
    if (!aligned(grad_params, 8)) return TM_ERR_ALIGN;
    return TM_OK;
}

tm_status tm_tonemap_backward_resid(const float *v, int64_t ld_v, int32_t H, int32_t W,
                                    const tm_params *p, const float *resid,
                                    const float *grad_out, int64_t ld_g, float *grad_v,
                                    int64_t ld_gv, double *grad_params, void *ws,
                                    size_t ws_bytes, void *stream) {
    TM_TRY(check_bwd_common(v, ld_v, H, W, p, grad_out, ld_g, grad_v, ld_gv, grad_params));
    if (!resid) return TM_ERR_ARG;
    if (!aligned(resid, 8)) return TM_ERR_ALIGN;   // pair planes are read as 8-byte pairs
    BwdPlan plan = make_bwd_plan(H, W, p->n_scales, to_query(p, H, W).ry, false);
    TM_TRY(check_ws(ws, ws_bytes, plan.total));
    return run_backward_resid(v, ld_v, H, W, p, resid, grad_out, ld_g, grad_v, ld_gv,
                              grad_params, plan, ws, (hipStream_t)stream);
}

tm_status tm_tonemap_backward_resid_log(const float *lum, int64_t ld_lum, int32_t H, int32_t W,
                                        const tm_params *p, const float *resid,
                                        const float *grad_out, int64_t ld_g, float *grad_lum,
                                        int64_t ld_gl, double *grad_params, void *ws,
                                        size_t ws_bytes, void *stream) {
    TM_TRY(check_bwd_common(lum, ld_lum, H, W, p, grad_out, ld_g, grad_lum, ld_gl, grad_params));
    if (!resid) return TM_ERR_ARG;
    if (!aligned(resid, 8)) return TM_ERR_ALIGN;
    BwdPlan plan = make_bwd_plan(H, W, p->n_scales, to_query(p, H, W).ry, false);
    TM_TRY(check_ws(ws, ws_bytes, plan.total));
    return run_backward_resid(lum, ld_lum, H, W, p, resid, grad_out, ld_g, grad_lum, ld_gl,
                              grad_params, plan, ws, (hipStream_t)stream, true);
}

static tm_status run_backward_tables(const float *v, int64_t ld_v, int32_t H, int32_t W,
                                     const void *sat, int64_t ld_sat, tm_sat_prec prec,
                                     const float *offsets, const uint32_t *hist_cum,
                                     int64_t ld_hist, int64_t plane_stride, const float *edges,
                                     const tm_params *p, const float *grad_out, int64_t ld_g,
                                     float *grad_v, int64_t ld_gv, double *grad_params, void *ws,
                                     size_t ws_bytes, void *stream, bool log_chain) {
    TM_TRY(check_bwd_common(v, ld_v, H, W, p, grad_out, ld_g, grad_v, ld_gv, grad_params));
    if (!valid_prec(prec)) return TM_ERR_ARG;
    TM_TRY(check_table(H, W, ld_sat, sat));
    if (prec == TM_SAT_C32X2 && !offsets) return TM_ERR_ARG;
    if (p->n_bins > 1) {
        if (!edges) return TM_ERR_ARG;
        TM_TRY(check_hist(H, W, ld_hist, plane_stride, hist_cum, p->n_bins - 1));
    }
    BwdPlan plan = make_bwd_plan(H, W, p->n_scales, to_query(p, H, W).ry, true);
    TM_TRY(check_ws(ws, ws_bytes, plan.total));
    float *resid = reinterpret_cast<float *>(static_cast<char *>(ws) + plan.resid);
    hipStream_t s = (hipStream_t)stream;
    // the residual planes from the tables (the query in training mode, no tone output)
    const QueryParams q = to_query(p, H, W);
    tm_status st = from_hip(launch_forward(v, ld_v, H, W, sat, ld_sat, (int)prec, offsets,
                                           hist_cum, ld_hist, plane_stride, edges, q, nullptr,
                                           W, resid, s));
    if (st != TM_OK) return st;
    return run_backward_resid(v, ld_v, H, W, p, resid, grad_out, ld_g, grad_v, ld_gv,
                              grad_params, plan, ws, s, log_chain);
}

tm_status tm_tonemap_backward(const float *v, int64_t ld_v, int32_t H, int32_t W,
                              const void *sat, int64_t ld_sat, tm_sat_prec prec,
                              const float *offsets, const uint32_t *hist_cum,
                              int64_t ld_hist, int64_t plane_stride, const float *edges,
                              const tm_params *p, const float *grad_out, int64_t ld_g,
                              float *grad_v, int64_t ld_gv, double *grad_params, void *ws,
                              size_t ws_bytes, void *stream) {
    return run_backward_tables(v, ld_v, H, W, sat, ld_sat, prec, offsets, hist_cum, ld_hist,
                               plane_stride, edges, p, grad_out, ld_g, grad_v, ld_gv,
                               grad_params, ws, ws_bytes, stream, false);
}

tm_status tm_tonemap_backward_log(const float *lum, int64_t ld_lum, int32_t H, int32_t W,
                                  const void *sat, int64_t ld_sat, tm_sat_prec prec,
                                  const float *log_offsets, const uint32_t *hist_cum,
                                  int64_t ld_hist, int64_t plane_stride, const float *edges,
                                  const tm_params *p, const float *grad_out, int64_t ld_g,
                                  float *grad_lum, int64_t ld_gl, double *grad_params, void *ws,
                                  size_t ws_bytes, void *stream) {
    return run_backward_tables(lum, ld_lum, H, W, sat, ld_sat, prec, log_offsets, hist_cum,
                               ld_hist, plane_stride, edges, p, grad_out, ld_g, grad_lum, ld_gl,
                               grad_params, ws, ws_bytes, stream, true);
}

}  // extern "C"
