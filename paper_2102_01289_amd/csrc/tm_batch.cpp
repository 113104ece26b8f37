// tm_batch.cpp -- batched forward: many images of uneven size, one launch per phase and image
// group, recordable as one HIP graph.
//
// tm_batch_create lays every image's buffers out in the caller's workspace, builds the
// per-image kernel descriptors (StatsK, ScanK, FwdK) and prefix sums of each phase's work
// items, and uploads them.  It also cuts the image list into consecutive groups whose
// integral tables together stay within kGroupTableBytes: the fused query reads every table
// entry twenty times (four corners, five fields), and it runs at about twice the speed when
// the tables it reads were just written and still sit in the 256 MB memory-side cache.
// tm_batch_forward then launches, group after group, six kernels whose grids cover the
// flattened work of the group's images (statistics, edges, three scan phases, query), one
// work item per block (per wave for the scan tiles), so the hardware hands the items out in
// order and the items in flight stay a compact window of the list.
// Every image keeps exactly the reduction structure and scan tiling of a single-image call
// with the same tiling, so batched outputs equal per-image outputs bit for bit.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstring>
#include <new>
#include <vector>

#include "../../include/tm.h"
#include "tm_internal.h"

using namespace tmo;

struct tm_batch {
    int count = 0, prec = 0;
    ScanTune tune{};
    std::vector<StatsK> sk;
    std::vector<ScanK> ck;
    std::vector<FwdK> fk;
    std::vector<int> vec;   // columns per lane of the scan of descriptor k
    std::vector<int64_t> parts, tiles, items, qtiles;   // prefixes, count + 1 each
    StatsK *d_sk = nullptr;
    ScanK *d_ck = nullptr;
    FwdK *d_fk = nullptr;
    int64_t *d_parts = nullptr, *d_tiles = nullptr, *d_items = nullptr, *d_qtiles = nullptr;
    struct Group {
        int i0, i1;                                  // descriptors [i0, i1)
        int vec;                                     // their scans' columns per lane
        unsigned g_stats, g_tiles, g_items, g_query;   // grid sizes
    };
    std::vector<Group> groups;
    bool h32 = true;   // every image's histogram offsets fit the 32-bit query addressing
    bool log = false;  // log-domain variance variant (tm_batch_set_variance)
    struct Bufs {
        float *lum, *edges, *offsets;
        int64_t ld_lum;
        void *sat;
        int64_t ld_sat;
        uint32_t *hist;
        int64_t ld_hist, plane_stride;
    };
    std::vector<Bufs> bufs;
    std::vector<char> host_tables;   // staging of the uploaded descriptor tables
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    // concurrency: groups dealt to internal streams (forked from and joined back to the
    // caller's stream), at most images_per_group images per group (0: table bytes only)
    size_t per_entry = 0;
    int images_per_group = 0;
    std::vector<hipStream_t> streams;
    std::vector<int> group_stream;
    hipEvent_t ev_fork = nullptr;
    std::vector<hipEvent_t> ev_join;
};

namespace {

constexpr size_t kAlign = 256;
// Integral-table bytes of one image group: well inside the 256 MB memory-side cache, leaving
// room for the luminance, outputs and scan aggregates that stream past it.
constexpr size_t kGroupTableBytes = (size_t)160 << 20;
size_t up(size_t a, size_t b) { return (a + b - 1) / b * b; }

size_t entry_bytes(int prec) { return prec == TM_SAT_F32 ? 8 : 16; }

struct Carver {
    char *base;
    size_t off = 0;
    size_t take(size_t bytes) {
        size_t o = off;
        off = up(off + bytes, kAlign);
        return o;
    }
    template <class T>
    T *ptr(size_t o) const {
        return base ? reinterpret_cast<T *>(base + o) : nullptr;
    }
};

tm_status check(const tm_image_desc *d, int32_t count, const tm_params *p, tm_sat_prec prec,
                const tm_tune *tune, ScanTune &t) {
    if (!d || count < 1 || !p) return TM_ERR_ARG;
    if (prec != TM_SAT_F32 && prec != TM_SAT_C32X2 && prec != TM_SAT_F64) return TM_ERR_ARG;
    if (p->n_bins < 1 || p->n_bins > TM_MAX_BINS || p->n_scales < 1 ||
        p->n_scales > TM_MAX_SCALES)
        return TM_ERR_ARG;
    if (!(p->eps > 0.f) || !(p->ld_max > p->ld_min)) return TM_ERR_ARG;
    // tile_w_vec 0 / tile_h 0: every image takes the default for its own shape
    t = tune ? ScanTune{tune->tile_w_vec, tune->tile_h, tune->bin_chunk} : ScanTune{0, 0, 4};
    if (!scan_tune_valid(ScanTune{t.vec ? t.vec : 4, t.th ? t.th : 16, t.chunk}))
        return TM_ERR_ARG;
    for (int i = 0; i < count; ++i) {
        const tm_image_desc &x = d[i];
        if (x.H < 1 || x.W < 1 || x.W > TM_MAX_WIDTH || (int64_t)x.H * x.W >= ((int64_t)1 << 31))
            return TM_ERR_SHAPE;
        if (!x.rgb || !x.out) return TM_ERR_ARG;
        if (x.ld_rgb < x.W || x.ld_out < x.W || x.ch_stride < (int64_t)x.H * x.ld_rgb)
            return TM_ERR_SHAPE;
        for (int j = 0; j < p->n_scales; ++j)
            if (x.rx[j] < 0 || x.ry[j] < 0) return TM_ERR_ARG;
    }
    return TM_OK;
}

// The scan tiling of one image: the batch's, with 0 fields taken from the image's default.
ScanTune image_tiling(const ScanTune &t, int H, int W, int n_bins) {
    const ScanTune def = scan_tune_default(H, W, n_bins);
    return ScanTune{t.vec ? t.vec : def.vec, t.th ? t.th : def.th, t.chunk};
}

// Processing order: the images sorted (stably) by columns per lane, so that a group of
// consecutive images shares one compiled scan variant (columns per lane do not depend on the
// bin count).
std::vector<int> processing_order(const tm_image_desc *d, int32_t count, const ScanTune &t) {
    std::vector<int> order(count);
    for (int i = 0; i < count; ++i) order[i] = i;
    std::stable_sort(order.begin(), order.end(), [&](int a, int b) {
        return image_tiling(t, d[a].H, d[a].W, 0).vec < image_tiling(t, d[b].H, d[b].W, 0).vec;
    });
    return order;
}

// Lays the batch out from `base` (nullptr: sizing only) and fills the host descriptors, in
// processing order (descriptor k is image order[k]; bufs stay indexed by image).
size_t layout(const tm_image_desc *d, int32_t count, const tm_params *p, int prec,
              const ScanTune &t, char *base, tm_batch *b) {
    const std::vector<int> order = processing_order(d, count, t);
    Carver c{base};
    const size_t o_sk = c.take(sizeof(StatsK) * count);
    const size_t o_ck = c.take(sizeof(ScanK) * count);
    const size_t o_fk = c.take(sizeof(FwdK) * count);
    const size_t o_pf = c.take(sizeof(int64_t) * 4 * (count + 1));
    const int n = p->n_bins;
    QueryParams q{};
    q.n_bins = n;
    q.n_scales = p->n_scales;
    q.eps = p->eps;
    q.ld_min = p->ld_min;
    q.ld_max = p->ld_max;
    if (b) {
        b->sk.resize(count);
        b->ck.resize(count);
        b->fk.resize(count);
        b->vec.resize(count);
        b->bufs.resize(count);
        b->parts.assign(count + 1, 0);
        b->tiles.assign(count + 1, 0);
        b->items.assign(count + 1, 0);
        b->qtiles.assign(count + 1, 0);
    }
    for (int i = 0; i < count; ++i) {
        const int img = order[i];
        const tm_image_desc &x = d[img];
        const int H = x.H, W = x.W;
        int64_t ld, org, elems;
        tm_table_geometry(H, W, &ld, &org, &elems);
        const int64_t ld_lum = (W + 63) / 64 * 64;
        const size_t o_lum = c.take(sizeof(float) * (size_t)H * ld_lum);
        const size_t o_edges = c.take(sizeof(float) * 260);
        const size_t o_part = c.take(sizeof(StatsPartial) * (size_t)stats_blocks(H, W));
        const size_t o_sat = c.take(entry_bytes(prec) * (size_t)elems);
        const size_t o_hist = c.take(4 * (size_t)elems * (size_t)(n > 1 ? n - 1 : 1));
        const ScanTune ti = image_tiling(t, H, W, n);
        const ScanPlan sp = make_scan_plan(H, W, prec, n - 1, ti);
        const size_t o_scan = c.take(sp.total);
        if (!b) continue;
        float *lum = c.ptr<float>(o_lum);
        float *edges = c.ptr<float>(o_edges);
        float *offsets = edges + 256;
        float *minmax = edges + 258;
        void *sat = c.ptr<char>(o_sat) + org * entry_bytes(prec);
        uint32_t *hist = c.ptr<uint32_t>(o_hist) + org;
        b->bufs[img] = {lum, edges, offsets, ld_lum, sat, ld, hist, ld, elems};
        b->vec[i] = ti.vec;
        b->sk[i] = make_statsk(x.rgb, x.ch_stride, x.ld_rgb, nullptr, 0, lum, ld_lum, H, W, n,
                               edges, offsets, minmax, c.ptr<StatsPartial>(o_part));
        ScanArgs a{};
        a.v = lum;
        a.ld_v = ld_lum;
        a.H = H;
        a.W = W;
        a.sat_prec = prec;
        a.offsets = offsets;
        a.sat = sat;
        a.ld_sat = ld;
        a.edges = edges;
        a.n_bins = n;
        a.layout = TM_HIST_CUMULATIVE;
        a.n_planes = n - 1;
        a.hist = n > 1 ? hist : nullptr;
        a.ld_hist = ld;
        a.plane_stride = elems;
        b->ck[i] = make_scank(a, sp, c.ptr<char>(o_scan));
        QueryParams qi = q;
        for (int j = 0; j < TM_MAX_SCALES; ++j) {
            // radii beyond the image act as the image's size (Algorithm 1's clamping); held
            // there so that no index expression of the kernels can overflow
            qi.rx[j] = j < p->n_scales ? (x.rx[j] < x.W ? x.rx[j] : x.W) : 0;
            qi.ry[j] = j < p->n_scales ? (x.ry[j] < x.H ? x.ry[j] : x.H) : 0;
        }
        b->fk[i] = make_fwdk(lum, ld_lum, H, W, sat, ld, offsets, n > 1 ? hist : nullptr, ld,
                             elems, edges, qi, x.out, x.ld_out);
        b->parts[i + 1] = b->parts[i] + b->sk[i].nparts;
        // scan work items: each tile is its integral image plus hist_items histogram items
        b->tiles[i + 1] = b->tiles[i] + (int64_t)(1 + b->ck[i].hist_items) * sp.tiles_x * sp.tiles_y;
        b->items[i + 1] = b->items[i] + scan_stage2_items(b->ck[i], true);
        b->qtiles[i + 1] = b->qtiles[i] + query_blocks(b->fk[i]);
    }
    if (b) {
        b->d_sk = c.ptr<StatsK>(o_sk);
        b->d_ck = c.ptr<ScanK>(o_ck);
        b->d_fk = c.ptr<FwdK>(o_fk);
        int64_t *pf = c.ptr<int64_t>(o_pf);
        b->d_parts = pf;
        b->d_tiles = pf + (count + 1);
        b->d_items = pf + 2 * (count + 1);
        b->d_qtiles = pf + 3 * (count + 1);
    }
    return c.off;
}

tm_status from_hip(hipError_t e) { return e == hipSuccess ? TM_OK : TM_ERR_HIP; }

unsigned clampu(int64_t v, int64_t lo, int64_t hi) {
    return (unsigned)(v < lo ? lo : (v > hi ? hi : v));
}

// Image groups: consecutive descriptors whose integral tables together stay within
// kGroupTableBytes divided by the number of streams (so that the groups in flight together
// still fit the memory-side cache), of one scan variant, at most images_per_group images
// (0: no limit), at
// least one image each; their grids give one work item per block (per wave for the scan
// tiles), handed out in order by the hardware, so the items in flight stay a compact window
// of the list.  With several streams the groups are dealt in list order, each to the stream
// with the fewest pixels so far (dealing them largest first measured no better).
void make_groups(tm_batch *b) {
    b->groups.clear();
    b->group_stream.clear();
    const size_t limit = kGroupTableBytes / (b->streams.empty() ? 1 : b->streams.size());
    for (int i0 = 0; i0 < b->count;) {
        int i1 = i0;
        size_t bytes = 0;
        while (i1 < b->count) {
            const size_t bi = (size_t)b->fk[i1].plane_stride * b->per_entry;
            if (i1 > i0 && (bytes + bi > limit || b->vec[i1] != b->vec[i0])) break;
            if (b->images_per_group > 0 && i1 - i0 >= b->images_per_group) break;
            bytes += bi;
            ++i1;
        }
        tm_batch::Group g;
        g.i0 = i0;
        g.i1 = i1;
        g.vec = b->vec[i0];
        const int64_t kMaxGrid = ((int64_t)1 << 31) - 1;
        g.g_stats = clampu(b->parts[i1] - b->parts[i0], 1, kMaxGrid);
        g.g_tiles = clampu((b->tiles[i1] - b->tiles[i0] + 3) / 4, 1, kMaxGrid);
        g.g_items = clampu((b->items[i1] - b->items[i0] + 255) / 256, 1, kMaxGrid);
        g.g_query = clampu(b->qtiles[i1] - b->qtiles[i0], 1, kMaxGrid);   // one block per tile
        b->groups.push_back(g);
        i0 = i1;
    }
    const size_t ng = b->groups.size();
    std::vector<int64_t> px(ng, 0);
    for (size_t gi = 0; gi < ng; ++gi)
        for (int i = b->groups[gi].i0; i < b->groups[gi].i1; ++i)
            px[gi] += (int64_t)b->fk[i].H * b->fk[i].W;
    std::vector<int64_t> load(b->streams.empty() ? 1 : b->streams.size(), 0);
    b->group_stream.assign(ng, 0);
    for (size_t gi = 0; gi < ng; ++gi) {
        int best = 0;
        for (int k = 1; k < (int)load.size(); ++k)
            if (load[k] < load[best]) best = k;
        load[best] += px[gi];
        b->group_stream[gi] = best;
    }
}

void release_streams(tm_batch *b) {
    for (hipStream_t s : b->streams) hipStreamDestroy(s);
    for (hipEvent_t e : b->ev_join) hipEventDestroy(e);
    if (b->ev_fork) hipEventDestroy(b->ev_fork);
    b->streams.clear();
    b->ev_join.clear();
    b->ev_fork = nullptr;
}

}  // namespace

extern "C" {

size_t tm_batch_workspace_bytes(const tm_image_desc *descs, int32_t count, const tm_params *p,
                                tm_sat_prec prec, const tm_tune *tune) {
    ScanTune t;
    if (check(descs, count, p, prec, tune, t) != TM_OK) return 0;
    return layout(descs, count, p, (int)prec, t, nullptr, nullptr);
}

tm_status tm_batch_create(const tm_image_desc *descs, int32_t count, const tm_params *p,
                          tm_sat_prec prec, const tm_tune *tune, void *ws, size_t ws_bytes,
                          void *stream, tm_batch **batch) {
    if (!batch) return TM_ERR_ARG;
    *batch = nullptr;
    ScanTune t;
    tm_status st = check(descs, count, p, prec, tune, t);
    if (st != TM_OK) return st;
    const size_t need = layout(descs, count, p, (int)prec, t, nullptr, nullptr);
    if (!ws || ((uintptr_t)ws & (kAlign - 1)) || ws_bytes < need) return TM_ERR_WORKSPACE;
    tm_batch *b = new (std::nothrow) tm_batch;
    if (!b) return TM_ERR_HIP;
    b->count = count;
    b->prec = (int)prec;
    b->tune = t;
    layout(descs, count, p, (int)prec, t, static_cast<char *>(ws), b);
    for (int i = 0; i < count; ++i) b->h32 = b->h32 && hist_offsets_fit_32(b->fk[i]);
    b->per_entry = entry_bytes((int)prec) + 4 * (size_t)(p->n_bins > 1 ? p->n_bins - 1 : 0);
    make_groups(b);
    // upload the descriptor tables (contiguous in ws from d_sk to the end of the prefixes)
    const size_t n_sk = sizeof(StatsK) * count, n_ck = sizeof(ScanK) * count,
                 n_fk = sizeof(FwdK) * count, n_pf = sizeof(int64_t) * (count + 1);
    hipStream_t s = (hipStream_t)stream;
    hipError_t e = hipMemcpyAsync(b->d_sk, b->sk.data(), n_sk, hipMemcpyHostToDevice, s);
    if (e == hipSuccess) e = hipMemcpyAsync(b->d_ck, b->ck.data(), n_ck, hipMemcpyHostToDevice, s);
    if (e == hipSuccess) e = hipMemcpyAsync(b->d_fk, b->fk.data(), n_fk, hipMemcpyHostToDevice, s);
    if (e == hipSuccess) e = hipMemcpyAsync(b->d_parts, b->parts.data(), n_pf, hipMemcpyHostToDevice, s);
    if (e == hipSuccess) e = hipMemcpyAsync(b->d_tiles, b->tiles.data(), n_pf, hipMemcpyHostToDevice, s);
    if (e == hipSuccess) e = hipMemcpyAsync(b->d_items, b->items.data(), n_pf, hipMemcpyHostToDevice, s);
    if (e == hipSuccess) e = hipMemcpyAsync(b->d_qtiles, b->qtiles.data(), n_pf, hipMemcpyHostToDevice, s);
    // no synchronisation: the host vectors backing the copies live until tm_batch_destroy
    if (e != hipSuccess) {
        delete b;
        return TM_ERR_HIP;
    }
    *batch = b;
    return TM_OK;
}

tm_status tm_batch_set_concurrency(tm_batch *b, int32_t streams, int32_t images_per_group) {
    if (!b || streams < 1 || streams > TM_BATCH_MAX_STREAMS || images_per_group < 0)
        return TM_ERR_ARG;
    release_streams(b);
    if (streams > 1) {
        b->streams.resize(streams, nullptr);
        b->ev_join.resize(streams, nullptr);
        bool ok = hipEventCreateWithFlags(&b->ev_fork, hipEventDisableTiming) == hipSuccess;
        for (int k = 0; ok && k < streams; ++k) {
            ok = hipStreamCreateWithFlags(&b->streams[k], hipStreamNonBlocking) == hipSuccess &&
                 hipEventCreateWithFlags(&b->ev_join[k], hipEventDisableTiming) == hipSuccess;
        }
        if (!ok) {
            release_streams(b);
            make_groups(b);
            return TM_ERR_HIP;
        }
    }
    b->images_per_group = images_per_group;
    make_groups(b);
    return TM_OK;
}

tm_status tm_batch_set_variance(tm_batch *b, int32_t log_domain, void *stream) {
    if (!b || (log_domain != 0 && log_domain != 1)) return TM_ERR_ARG;
    b->log = log_domain != 0;
    for (ScanK &k : b->ck) k.log_src = log_domain;
    // the scan descriptors on the device follow; the copy has completed when the call
    // returns, so a later call may change the host table without racing it
    if (hipMemcpyAsync(b->d_ck, b->ck.data(), sizeof(ScanK) * b->count, hipMemcpyHostToDevice,
                       (hipStream_t)stream) != hipSuccess ||
        hipStreamSynchronize((hipStream_t)stream) != hipSuccess)
        return TM_ERR_HIP;
    // a graph captured before holds the other variant's prologue: it must be captured again
    if (b->exec) hipGraphExecDestroy(b->exec);
    if (b->graph) hipGraphDestroy(b->graph);
    b->exec = nullptr;
    b->graph = nullptr;
    return TM_OK;
}

tm_status tm_batch_forward(tm_batch *b, void *stream) {
    if (!b) return TM_ERR_ARG;
    hipStream_t s0 = (hipStream_t)stream;
    const bool fork = !b->streams.empty();
    if (fork) {   // the internal streams start after everything already queued on stream
        if (hipEventRecord(b->ev_fork, s0) != hipSuccess) return TM_ERR_HIP;
        for (hipStream_t t : b->streams)
            if (hipStreamWaitEvent(t, b->ev_fork, 0) != hipSuccess) return TM_ERR_HIP;
    }
    for (size_t gi = 0; gi < b->groups.size(); ++gi) {
        const tm_batch::Group &g = b->groups[gi];
        hipStream_t s = fork ? b->streams[b->group_stream[gi]] : s0;
        const int n = g.i1 - g.i0;
        hipError_t e =
            launch_stats_batch(b->d_sk + g.i0, b->d_parts + g.i0, n, g.g_stats, s, b->log);
        if (e != hipSuccess) return TM_ERR_HIP;
        BatchScan bs{b->d_ck + g.i0, b->d_tiles + g.i0, b->d_items + g.i0, n, b->prec,
                     g.vec, b->tune.chunk, g.g_tiles, g.g_items};
        e = launch_tables_batch(bs, s);
        if (e != hipSuccess) return TM_ERR_HIP;
        e = launch_forward_batch(b->d_fk + g.i0, b->d_qtiles + g.i0, n, b->prec, b->h32,
                                 g.g_query, s);
        if (e != hipSuccess) return TM_ERR_HIP;
    }
    if (fork) {   // and stream waits for all of them
        for (size_t k = 0; k < b->streams.size(); ++k) {
            if (hipEventRecord(b->ev_join[k], b->streams[k]) != hipSuccess) return TM_ERR_HIP;
            if (hipStreamWaitEvent(s0, b->ev_join[k], 0) != hipSuccess) return TM_ERR_HIP;
        }
    }
    return TM_OK;
}

tm_status tm_batch_capture(tm_batch *b, void *stream) {
    if (!b || !stream) return TM_ERR_ARG;
    hipStream_t s = (hipStream_t)stream;
    if (hipStreamBeginCapture(s, hipStreamCaptureModeRelaxed) != hipSuccess) return TM_ERR_HIP;
    tm_status st = tm_batch_forward(b, stream);
    hipGraph_t g = nullptr;
    hipError_t e = hipStreamEndCapture(s, &g);
    if (st != TM_OK || e != hipSuccess) {
        if (g) hipGraphDestroy(g);
        return st != TM_OK ? st : TM_ERR_HIP;
    }
    hipGraphExec_t x = nullptr;
    if (hipGraphInstantiate(&x, g, nullptr, nullptr, 0) != hipSuccess) {
        hipGraphDestroy(g);
        return TM_ERR_HIP;
    }
    if (b->exec) hipGraphExecDestroy(b->exec);
    if (b->graph) hipGraphDestroy(b->graph);
    b->graph = g;
    b->exec = x;
    return TM_OK;
}

tm_status tm_batch_replay(tm_batch *b, void *stream) {
    if (!b || !b->exec) return TM_ERR_ARG;
    return from_hip(hipGraphLaunch(b->exec, (hipStream_t)stream));
}

tm_status tm_batch_destroy(tm_batch *b) {
    if (!b) return TM_ERR_ARG;
    if (b->exec) hipGraphExecDestroy(b->exec);
    if (b->graph) hipGraphDestroy(b->graph);
    release_streams(b);
    delete b;
    return TM_OK;
}

tm_status tm_batch_image_buffers(const tm_batch *b, int32_t i, float **lum, int64_t *ld_lum,
                                 float **edges, float **offsets, void **sat, int64_t *ld_sat,
                                 uint32_t **hist, int64_t *ld_hist, int64_t *plane_stride) {
    if (!b || i < 0 || i >= b->count) return TM_ERR_ARG;
    const auto &x = b->bufs[i];
    if (lum) *lum = x.lum;
    if (ld_lum) *ld_lum = x.ld_lum;
    if (edges) *edges = x.edges;
    if (offsets) *offsets = x.offsets;
    if (sat) *sat = x.sat;
    if (ld_sat) *ld_sat = x.ld_sat;
    if (hist) *hist = x.hist;
    if (ld_hist) *ld_hist = x.ld_hist;
    if (plane_stride) *plane_stride = x.plane_stride;
    return TM_OK;
}

}  // extern "C"
