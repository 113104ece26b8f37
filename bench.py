"""Benchmark of the tone-mapping hot path on one MI355X.

A step is one pass of the whole path over one synthetic 4000x3000 WDR image (inputs
resident in HBM): prologue (Eq. 11 + image statistics), integral image and integral
histogram (Eq. 5, 8), the fused per-pixel query/blend over all fields (Eq. 1-4), and the
backward (adjoint of the same path) when it is enabled.  Prints one JSON line.

    python bench.py [--steps K] [--warmup W] [--prec c32x2|f32|f64] [--no-backward]
                    [--no-cpu-baseline] [--kernel-only query|tables|backward]
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

WORKLOAD = "wdr_4000x3000"        # the image the metric is quoted on
PEAK_HBM_GBS = 8000.0
# PMC summary of the roofline kernel (FETCH_SIZE and WRITE_SIZE per dispatch, calibrated on a
# plain copy kernel), and the sources whose digest it records
IMAGES = ("wdr_4000x3000", "wdr_1920x1080", "wdr_256x256")


def traffic_profile(workload: str) -> str:
    """The committed counter summary of the fused query on one workload."""
    return os.path.join(ROOT, "profiles", f"forward_kernel_{workload}_traffic.md")
QUERY_SOURCES = ("paper_2102_01289_amd/csrc/tm_query.hip", "paper_2102_01289_amd/csrc/tm_device.h")
# the kernel's parameter struct lives in the shared internal header
QUERY_STRUCT = ("paper_2102_01289_amd/csrc/tm_internal.h", "struct FwdK {")


def _parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--prec", default="c32x2", choices=["c32x2", "f32", "f64"])
    ap.add_argument("--n-bins", type=int, default=5)
    ap.add_argument("--n-scales", type=int, default=5)
    ap.add_argument("--eps", type=float, default=0.1)
    ap.add_argument("--no-backward", action="store_true")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--kernel-only", choices=["query", "tables", "backward"], default=None,
                    help="launch only that stage in the timed loop (profiling runs)")
    ap.add_argument("--no-extras", action="store_true",
                    help="leave out the batch, stress-set and log-variance blocks of the "
                         "default line (profiling runs)")
    ap.add_argument("--copy-probe", action="store_true",
                    help="after the timed loop, copy 1 GiB device-to-device once (a plain copy "
                         "kernel of known size, for calibrating HBM counters) and report its "
                         "bandwidth")
    ap.add_argument("--workload", choices=["image", "batch", "sweep", "hdr", "stress", "scan",
                                           "logvar"],
                    default="image",
                    help="image: one image (--image, 4000x3000 by default); batch: 64 images "
                         "of uneven size, launches replayed from a HIP graph; sweep: the "
                         "paper's Table IV grid (n, s in {3, 4, 5} at 480x640, 720x1280, "
                         "1080x1920) with a per-stage split; hdr: the multi-exposure front end "
                         "at 4000x3000; stress: 64 bins and radii 4/16/64 at 4000x3000; scan: "
                         "the integral histogram built in three stages and in one look-back "
                         "pass, at 1080p and 4000x3000; logvar: the log-domain variance "
                         "variant's stages (forward and backward) beside the linear form")
    ap.add_argument("--image", choices=IMAGES, default=WORKLOAD,
                    help="the image of the image workload (the metric is quoted on "
                         "wdr_4000x3000)")
    return ap.parse_args()


# The paper's Table IV: whole tone-mapping time in ms on its phone GPU (an iPhone 6 Plus
# through Metal), by bins n, fields s and resolution.  Context only: other hardware and an
# unstated precision.
PAPER_TABLE_IV_MS = {
    (3, 3): (122.11, 303.79, 637.90), (3, 4): (145.82, 351.13, 788.27),
    (3, 5): (166.91, 402.36, 865.69), (4, 3): (130.33, 284.74, 677.69),
    (4, 4): (174.73, 359.80, 793.60), (4, 5): (175.14, 422.65, 920.95),
    (5, 3): (139.69, 293.37, 869.33), (5, 4): (187.64, 355.05, 886.96),
    (5, 5): (212.44, 432.90, 1016.26)}
SWEEP_SHAPES = ((480, 640), (720, 1280), (1080, 1920))


def bench_sweep(args):
    """Forward time of one image over the Table IV grid, with the per-stage split (prologue,
    tables, query; the paper's Fig. 7 splits its own time the same way) and each stage's
    algorithmic bytes over its time."""
    import torch

    import paper_2102_01289_amd as tm
    from synth import gen_wdr

    dev = torch.device("cuda:0")
    stream = torch.cuda.current_stream()
    rows = []
    for k, (H, W) in enumerate(SWEEP_SHAPES):
        rgb = torch.from_numpy(gen_wdr(H, W, 32, -2.0, 4.0, 202 + k).rgb).to(dev)
        for (n, s), paper in PAPER_TABLE_IV_MS.items():
            p = tm.make_params(n, s, eps=0.1, H=H, W=W)
            m = tm.ToneMapper(H, W, p, args.prec, device=dev)
            m.run(rgb)
            stage = {}
            for name, fn in (("prologue", lambda: m.prologue(rgb)), ("tables", m.tables),
                             ("query", m.query)):
                for _ in range(args.warmup):
                    fn()
                a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
                a.record(stream)
                for _ in range(args.steps):
                    fn()
                b.record(stream)
                torch.cuda.synchronize()
                stage[name] = a.elapsed_time(b) / args.steps
            ms = sum(stage.values())
            sat_b = {"f32": 8, "c32x2": 16, "f64": 16}[args.prec]
            bytes_px = {"prologue": 16, "tables": 4 + sat_b + 4 * (n - 1),
                        "query": query_bytes_per_px(args.prec, n)}
            rows.append({
                "height": H, "width": W, "n_bins": n, "n_scales": s,
                "ms": round(ms, 4), "mp_s": round(H * W / (ms * 1e-3) / 1e6, 1),
                "stage_ms": {k2: round(v, 4) for k2, v in stage.items()},
                "stage_share": {k2: round(v / ms, 3) for k2, v in stage.items()},
                "stage_algorithmic_gb_s": {k2: round(bytes_px[k2] * H * W / (v * 1e-3) / 1e9, 1)
                                           for k2, v in stage.items()},
                "paper_ms_iphone6plus": paper[k],
                "speedup_vs_paper_context": round(paper[k] / ms, 1)})
            print(f"sweep: {H}x{W} n={n} s={s}: {ms:.3f} ms", file=sys.stderr, flush=True)
    print(json.dumps({"metric": "forward ms and MP/s over the Table IV grid (n, s, resolution)",
                      "data": "synthetic", "sat_precision": args.prec, "steps": args.steps,
                      "rows": rows}), flush=True)


STRESS_BINS = 64
STRESS_RADII = (4, 16, 64)


def bench_stress(args):
    print(json.dumps(stress_line(args)), flush=True)


def stress_line(args) -> dict:
    """The stress parameter set (n = 64 bins, fields of radius 4, 16 and 64 on both axes,
    eps = 0.1) on the 4000x3000 image: forward MP/s, per-stage split and each stage's
    algorithmic bytes over its time.  Algorithmic bytes per pixel (every input read once,
    every table written once and read once): prologue 16; tables 4 + E + 4 (n - 1) with E the
    integral-image entry; query 4 + E + 4 (n - 1) + 4; forward 564 B/px with C32X2 tables."""
    import torch

    import paper_2102_01289_amd as tm
    from synth import WORKLOADS, gen_wdr

    cfg = WORKLOADS[WORKLOAD]
    H, W = cfg["H"], cfg["W"]
    dev = torch.device("cuda:0")
    rgb = torch.from_numpy(gen_wdr(H, W, cfg["K"], cfg["lo"], cfg["hi"], cfg["seed"]).rgb).to(dev)
    n, r = STRESS_BINS, list(STRESS_RADII)
    p = tm.make_params(n, len(r), r, r, args.eps)
    m = tm.ToneMapper(H, W, p, args.prec, device=dev)
    m.run(rgb)
    stream = torch.cuda.current_stream()
    stage = {}
    for name, fn in (("prologue", lambda: m.prologue(rgb)), ("tables", m.tables),
                     ("query", m.query)):
        for _ in range(args.warmup):
            fn()
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record(stream)
        for _ in range(args.steps):
            fn()
        b.record(stream)
        torch.cuda.synchronize()
        stage[name] = a.elapsed_time(b) / args.steps
    ms = sum(stage.values())
    esz = {"f32": 8, "c32x2": 16, "f64": 16}[args.prec]
    bpx = {"prologue": 16, "tables": 4 + esz + 4 * (n - 1),
           "query": 4 + esz + 4 * (n - 1) + 4}
    total_b = sum(bpx.values())
    dom = max(stage, key=stage.get)
    gbs = {k: bpx[k] * H * W / (v * 1e-3) / 1e9 for k, v in stage.items()}
    line = {
        "metric": "megapixels/s, forward with the stress parameter set (64 bins, radii 4/16/64)",
        "value": round(H * W / 1e6 / (ms * 1e-3), 3), "unit": "megapixels/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(ms, 4),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": {"c32x2": "f32x2", "f32": "f32", "f64": "f64"}[args.prec], "data": "synthetic",
        "config": {"workload": f"{WORKLOAD}_stress", "height": H, "width": W, "n_bins": n,
                   "radii": r, "eps": args.eps, "sat_precision": args.prec},
        "stage_ms": {k: round(v, 4) for k, v in stage.items()},
        "stage_algorithmic_gb_s": {k: round(v, 1) for k, v in gbs.items()},
        "algorithmic_bytes_per_px": {**bpx, "forward": total_b},
        "forward_algorithmic_frac": round(total_b * H * W / (ms * 1e-3) / 1e9 / PEAK_HBM_GBS, 4),
        "roofline": {"bound": "hbm", "kernel": {"prologue": "lum_stats_kernel",
                                                 "tables": "scan_stage1-3 (one table build)",
                                                 "query": "forward_kernel"}[dom],
                     "achieved": round(gbs[dom], 1), "peak": PEAK_HBM_GBS, "unit": "GB/s",
                     "frac": round(gbs[dom] / PEAK_HBM_GBS, 4), "traffic": None,
                     "algorithmic_bytes_per_launch": bpx[dom] * H * W,
                     "avg_kernel_ms": round(stage[dom], 4)},
    }
    return line


def _median_ms(fn, reps=10, warmup=2):
    """Median over reps of one call of fn, timed with events on torch's current stream (the
    stream the ToneMapper calls launch on)."""
    import torch
    for _ in range(warmup):
        fn()
    ts = []
    for _ in range(reps):
        a = torch.cuda.Event(enable_timing=True)
        b = torch.cuda.Event(enable_timing=True)
        a.record()
        fn()
        b.record()
        b.synchronize()
        ts.append(a.elapsed_time(b))
    return sorted(ts)[len(ts) // 2]


def bench_hdr(args):
    """The multi-exposure front end at 4000x3000: four 8-bit exposures of the 12 MP workload's
    radiance (seeded camera model), response recovery from 200 sampled pixels, the radiance
    merge (HBM-bound: P*3 B in, 12 B out per pixel) and the chain exposures -> tone-mapped
    RGB (merge, prologue, tables, fused query with colour restoration).  The oracle's merge
    is timed on the host beside it."""
    import numpy as np
    import torch

    import paper_2102_01289_amd as tm
    from oracle import hdr
    from synth import WORKLOADS, exposure_times, gen_exposure_stack, gen_sample_pixels, gen_wdr

    c = WORKLOADS["wdr_4000x3000"]
    H, W, P = c["H"], c["W"], 4
    img = gen_wdr(H, W, c["K"], c["lo"], c["hi"], c["seed"])
    times = exposure_times(P)
    stack = gen_exposure_stack(img.rgb, times, seed=c["seed"] + 1000)
    del img
    print("bench: exposure stack generated", file=sys.stderr, flush=True)
    dev = torch.device("cuda:0")
    st = torch.from_numpy(stack).to(dev)
    t = torch.from_numpy(np.log(times).astype(np.float32)).to(dev)
    idx = torch.from_numpy(gen_sample_pixels(H, W, 200, seed=c["seed"] + 2000)).to(dev)
    g = torch.empty((3, 256), dtype=torch.float32, device=dev)
    ws = torch.empty(tm._lib().tm_hdr_response_workspace_bytes(), dtype=torch.uint8, device=dev)
    E = torch.empty((3, H, W), dtype=torch.float32, device=dev)
    resp_ms = _median_ms(lambda: tm.tm_hdr_response(st, t, idx, 100.0, g=g, ws=ws), reps=5)
    merge_ms = _median_ms(lambda: tm.tm_hdr_merge(st, t, g, out=E), reps=args.steps)
    p = tm.make_params(args.n_bins, args.n_scales, eps=args.eps, H=H, W=W)
    m = tm.ToneMapper(H, W, p, args.prec, device=dev)

    def chain():
        tm.tm_hdr_merge(st, t, g, out=E)
        m.run_rgb(E)

    chain_ms = _median_ms(chain, reps=args.steps)
    algo = (3 * P + 12) * H * W
    # the oracle on the host: its own response from the same samples, then its merge (timed)
    Z = [stack[:, ch].reshape(P, -1)[:, idx.cpu().numpy()].T for ch in range(3)]
    g_host = np.stack([hdr.response(z, np.log(times), 100.0) for z in Z])
    t0 = time.perf_counter()
    hdr.merge(stack, g_host, np.log(times))
    orc_s = time.perf_counter() - t0
    out = {"metric": "megapixels/s, exposure merge (Debevec-Malik) and exposures -> "
                     "tone-mapped RGB", "value": round(H * W / merge_ms / 1e3, 1),
           "unit": "megapixels/s", "n_gpus": 1, "steps": args.steps,
           "higher_is_better": True, "data": "synthetic", "dtype": "u8->f32",
           "config": {"workload": "wdr_4000x3000_exposures4", "height": H, "width": W,
                      "exposures": P, "exposure_ratio": 16, "samples": 200, "lambda": 100.0},
           "merge_ms": round(merge_ms, 4), "response_ms": round(resp_ms, 3),
           "chain_ms": round(chain_ms, 4), "chain_mp_s": round(H * W / chain_ms / 1e3, 1),
           "roofline": {"bound": "hbm", "kernel": "hdr_merge_kernel",
                        "achieved": round(algo / merge_ms / 1e6, 1), "peak": 8000.0,
                        "unit": "GB/s", "frac": round(algo / merge_ms / 1e6 / 8000.0, 4),
                        "algorithmic_bytes_per_launch": algo},
           "cpu_baseline": {"value": round(H * W / orc_s / 1e6, 2), "unit": "megapixels/s",
                            "cores": 1, "kind": "oracle",
                            "sample": f"numpy merge of the full stack, {orc_s:.1f} s"}}
    print(json.dumps(out), flush=True)


def bench_batch(args):
    """64 images with H, W ~ U{360..4000}: aggregate MP/s of the graph-replayed batched
    forward, the eager batched forward and 64 per-image launch sequences."""
    import numpy as np
    import torch

    import paper_2102_01289_amd as tm
    from paper_2102_01289_amd import autotune
    from synth import WORKLOADS, gen_batch_shapes, gen_wdr

    cfg = WORKLOADS["wdr_batch64_uneven"]
    shapes = gen_batch_shapes(cfg["count"], 360, 4000, seed=cfg["shape_seed"])
    dev = torch.device("cuda:0")
    imgs = []
    for i, (h, w) in enumerate(shapes):
        imgs.append(torch.from_numpy(gen_wdr(h, w, cfg["K"], cfg["lo"], cfg["hi"],
                                             cfg["seed"] + i).rgb).to(dev))
        print(f"bench: generated image {i + 1}/{len(shapes)} ({h}x{w})", file=sys.stderr,
              flush=True)
    mpx = sum(h * w for h, w in shapes) / 1e6
    # (0 = each image's own default for its shape)
    cands = [(0, 0, 4), (0, 16, 4), (4, 0, 4), (2, 0, 4), (4, 16, 4), (2, 16, 4), (4, 8, 4),
             (4, 32, 4)]
    t, _ = autotune.tune_batch(imgs, args.n_bins, args.n_scales, args.prec, reps=3,
                               use_cache=False, cands=cands)
    b = tm.Batch(imgs, args.n_bins, args.n_scales, args.eps, prec=args.prec, tune=t)

    def timed(fn, stream=None):
        for _ in range(args.warmup):
            fn()
        torch.cuda.synchronize()
        a, e = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record(stream)
        for _ in range(args.steps):
            fn()
        e.record(stream)
        torch.cuda.synchronize()
        return a.elapsed_time(e) / args.steps

    eager_ms = timed(b.forward)
    s = torch.cuda.Stream()
    b.capture(s)
    graph1_ms = timed(lambda: b.replay(s), s)
    # concurrency: groups spread over internal streams (phases of different groups overlap);
    # each setting captured into its own graph and replayed
    conc = {}
    for streams, per_group in ((2, 0), (3, 0), (4, 0), (3, 1), (4, 1), (6, 1)):
        key = f"{streams}x{per_group}"
        b.set_concurrency(streams, per_group)
        b.capture(s)
        conc[key] = timed(lambda: b.replay(s), s)
        print(f"bench: batch concurrency {key}: {conc[key]:.3f} ms", file=sys.stderr,
              flush=True)
    best = min(conc, key=conc.get)
    graph_ms = min(graph1_ms, conc[best])
    best_cfg = best if conc[best] < graph1_ms else "1x0"
    st, pg = (int(v) for v in best_cfg.split("x"))
    b.set_concurrency(st, pg)
    b.capture(s)
    mappers = []
    for rgb in imgs:
        _, H, W = rgb.shape
        mappers.append(tm.ToneMapper(H, W, tm.make_params(args.n_bins, args.n_scales,
                                                          eps=args.eps, H=H, W=W),
                                     args.prec, tune=tm.image_tune(t, H, W, args.n_bins), device=dev))
    per_ms = timed(lambda: [m.run(r) for m, r in zip(mappers, imgs)])
    line = {
        "metric": "aggregate megapixels/s, batched forward (HIP graph) vs per-image launches",
        "value": round(mpx / (graph_ms * 1e-3), 3), "unit": "megapixels/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(graph_ms, 4),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": {"c32x2": "f32x2", "f32": "f32", "f64": "f64"}[args.prec],
        "data": "synthetic",
        "config": {"workload": "wdr_batch64_uneven", "images": len(shapes),
                   "megapixels": round(mpx, 3), "n_bins": args.n_bins,
                   "n_scales": args.n_scales, "eps": args.eps, "sat_precision": args.prec,
                   "tune": [t.tile_w_vec, t.tile_h, t.bin_chunk]},
        "concurrency": {"streams": st, "images_per_group": pg,
                        "graph_ms": {"1x0": round(graph1_ms, 4),
                                     **{k: round(v, 4) for k, v in conc.items()}}},
        "eager_batched_mp_s": round(mpx / (eager_ms * 1e-3), 3),
        "per_image_launches_mp_s": round(mpx / (per_ms * 1e-3), 3),
        "graph_over_per_image": round(per_ms / graph_ms, 4),
    }
    print(json.dumps(line), flush=True)


def bench_scan(args):
    """The integral histogram alone (n = 5, cumulative planes): the three-stage build against
    the single pass with decoupled look-back, at 1080p and 12 MP, plus the combined table
    build (integral image and histogram) for reference.  Algorithmic bytes: read v once (4)
    and write 4 (n - 1) per pixel."""
    import torch

    import paper_2102_01289_amd as tm
    from synth import WORKLOADS, gen_wdr

    dev = torch.device("cuda:0")
    n = args.n_bins
    rows = []
    for img in ("wdr_1920x1080", "wdr_4000x3000"):
        cfg = WORKLOADS[img]
        H, W = cfg["H"], cfg["W"]
        rgb = torch.from_numpy(gen_wdr(H, W, cfg["K"], cfg["lo"], cfg["hi"], cfg["seed"]).rgb).to(dev)
        m = tm.ToneMapper(H, W, tm.make_params(n, 5, eps=args.eps, H=H, W=W), args.prec, device=dev)
        m.run(rgb)
        v, edges = m.lum, m.edges
        hist = tm.Table(H, W, "u32", n - 1, dev)
        ws3 = torch.empty(max(tm._lib().tm_tables_workspace_bytes(H, W, n, 0, None), 1),
                          dtype=torch.uint8, device=dev)
        _, wsl = tm.tm_integral_histogram_lookback(v, edges, n, hist=hist)

        def three():
            tm._ck("tm_integral_histogram", tm._lib().tm_integral_histogram(
                tm._vp(v), v.stride(0), H, W, tm._vp(edges), n, 1, tm._vp(hist.ptr), hist.ld,
                hist.plane_stride, None, tm._vp(ws3), ws3.numel(), None))

        def single():
            tm.tm_integral_histogram_lookback(v, edges, n, hist=hist, ws=wsl)

        res = {}
        for name, fn in (("three_stage", three), ("lookback", single), ("tables", m.tables)):
            for _ in range(args.warmup):
                fn()
            torch.cuda.synchronize()
            a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            a.record()
            for _ in range(args.steps):
                fn()
            b.record()
            torch.cuda.synchronize()
            res[name] = a.elapsed_time(b) / args.steps * 1e3
        status = int(wsl[4:8].cpu().view(torch.int32)[0])
        hb = (4 + 4 * (n - 1)) * H * W
        rows.append({"workload": img, "three_stage_us": round(res["three_stage"], 1),
                     "lookback_us": round(res["lookback"], 1),
                     "tables_us": round(res["tables"], 1),
                     "hist_algorithmic_gb_s": {k: round(hb / (res[k] * 1e-6) / 1e9, 1)
                                               for k in ("three_stage", "lookback")},
                     "lookback_status": status})
        print(f"scan: {img}: three-stage {res['three_stage']:.1f} us, look-back "
              f"{res['lookback']:.1f} us", file=sys.stderr, flush=True)
    print(json.dumps({"metric": "integral histogram build, three-stage vs single-pass look-back",
                      "unit": "us", "n_bins": n, "steps": args.steps, "rows": rows}), flush=True)


def log_variance_extra(args, rgb, g, H, W):
    """The log-domain variance variant's forward+backward step on the headline image, for
    the default line: same parameters, steps timed as the headline's."""
    import torch

    import paper_2102_01289_amd as tm

    p = tm.make_params(args.n_bins, args.n_scales, eps=args.eps, H=H, W=W)
    m = tm.ToneMapper(H, W, p, args.prec, device=rgb.device, variance="log")
    stream = torch.cuda.current_stream()

    def step():
        m.run_train(rgb)
        m.backward_resid(g)

    def fwd():
        m.run(rgb)

    out = {}
    for name, fn in (("fwd_bwd", step), ("fwd", fwd)):
        for _ in range(args.warmup):
            fn()
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record(stream)
        for _ in range(args.steps):
            fn()
        b.record(stream)
        torch.cuda.synchronize()
        out[name + "_ms"] = round(a.elapsed_time(b) / args.steps, 4)
    mpx = H * W / 1e6
    out["fwd_bwd_mp_s"] = round(mpx / (out["fwd_bwd_ms"] * 1e-3), 3)
    out["fwd_mp_s"] = round(mpx / (out["fwd_ms"] * 1e-3), 3)
    return out


def bench_logvar(args):
    """The log-domain variance variant (Eq. 10's window variance of l = ln i, bins of i) beside
    the linear form, per stage, forward and forward+backward, at 4000x3000 and 1920x1080.
    The variant's backward is the residual backward given l followed by the chain rule
    through the logarithm."""
    import torch

    import paper_2102_01289_amd as tm
    from synth import WORKLOADS, gen_upstream_grad, gen_wdr

    dev = torch.device("cuda:0")
    stream = torch.cuda.current_stream()
    rows = []
    for img in ("wdr_4000x3000", "wdr_1920x1080"):
        cfg = WORKLOADS[img]
        H, W = cfg["H"], cfg["W"]
        rgb = torch.from_numpy(gen_wdr(H, W, cfg["K"], cfg["lo"], cfg["hi"], cfg["seed"]).rgb).to(dev)
        g = torch.from_numpy(gen_upstream_grad((H, W), seed=cfg["seed"] + 1)).to(dev)
        p = tm.make_params(args.n_bins, args.n_scales, eps=args.eps, H=H, W=W)
        for dom in ("linear", "log"):
            m = tm.ToneMapper(H, W, p, args.prec, device=dev, variance=dom)
            m.run_train(rgb)
            m.backward_resid(g)
            st = {}
            for name, fn in (("prologue", lambda: m.prologue(rgb)), ("tables", m.tables),
                             ("query", m.query), ("query_train", m.query_train),
                             ("backward", lambda: m.backward_resid(g))):
                for _ in range(args.warmup):
                    fn()
                a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
                a.record(stream)
                for _ in range(args.steps):
                    fn()
                b.record(stream)
                torch.cuda.synchronize()
                st[name] = round(a.elapsed_time(b) / args.steps, 4)
            fwd = st["prologue"] + st["tables"] + st["query"]
            step = fwd - st["query"] + st["query_train"] + st["backward"]
            mpx = H * W / 1e6
            rows.append({"workload": img, "variance": dom, "stage_ms": st,
                         "fwd_ms": round(fwd, 4), "fwd_bwd_ms": round(step, 4),
                         "fwd_mp_s": round(mpx / (fwd * 1e-3), 1),
                         "fwd_bwd_mp_s": round(mpx / (step * 1e-3), 1)})
            print(f"logvar: {img} {dom}: fwd {fwd:.3f} ms, fwd+bwd {step:.3f} ms",
                  file=sys.stderr, flush=True)
            del m
    print(json.dumps({"metric": "log-domain variance variant beside the linear form, per stage",
                      "unit": "ms", "sat_precision": args.prec, "n_bins": args.n_bins,
                      "n_scales": args.n_scales, "steps": args.steps, "rows": rows}), flush=True)


def batch_extra(args, streams: int = 3, tune=(0, 16, 4)) -> dict:
    """The 64-image batch in the default bench line: the graph-replayed batched forward with
    its groups on `streams` internal streams, against per-image launch sequences, both with
    the scan tiling `tune` (0 = each image's default), no autotuner."""
    import torch

    import paper_2102_01289_amd as tm
    from synth import WORKLOADS, gen_batch_shapes, gen_wdr

    cfg = WORKLOADS["wdr_batch64_uneven"]
    shapes = gen_batch_shapes(cfg["count"], 360, 4000, seed=cfg["shape_seed"])
    dev = torch.device("cuda:0")
    imgs = [torch.from_numpy(gen_wdr(h, w, cfg["K"], cfg["lo"], cfg["hi"], cfg["seed"] + i).rgb)
            .to(dev) for i, (h, w) in enumerate(shapes)]
    mpx = sum(h * w for h, w in shapes) / 1e6
    t = tm.tune(*tune)
    b = tm.Batch(imgs, args.n_bins, args.n_scales, args.eps, prec=args.prec, tune=t)
    b.set_concurrency(streams, 0)
    s = torch.cuda.Stream()
    b.capture(s)

    def timed(fn, stream, steps=5, warmup=2):
        for _ in range(warmup):
            fn()
        torch.cuda.synchronize()
        a, e = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record(stream)
        for _ in range(steps):
            fn()
        e.record(stream)
        torch.cuda.synchronize()
        return a.elapsed_time(e) / steps

    graph_ms = timed(lambda: b.replay(s), s)
    mappers = [tm.ToneMapper(r.shape[1], r.shape[2],
                             tm.make_params(args.n_bins, args.n_scales, eps=args.eps,
                                            H=r.shape[1], W=r.shape[2]),
                             args.prec, tune=tm.image_tune(t, r.shape[1], r.shape[2], args.n_bins),
                             device=dev)
               for r in imgs]
    per_ms = timed(lambda: [m.run(r) for m, r in zip(mappers, imgs)],
                   torch.cuda.current_stream())
    del b, mappers, imgs
    torch.cuda.synchronize()
    return {"workload": "wdr_batch64_uneven", "images": len(shapes), "megapixels": round(mpx, 3),
            "graph_ms": round(graph_ms, 4), "mp_s": round(mpx / (graph_ms * 1e-3), 3),
            "per_image_launches_ms": round(per_ms, 4),
            "graph_over_per_image": round(per_ms / graph_ms, 4), "streams": streams,
            "tune": list(tune)}


def query_bytes_per_px(prec: str, n_bins: int, resid_planes: int = 0) -> int:
    """Algorithmic bytes of the fused query per pixel: luminance in, every table entry read
    once (interleaved integral image + n-1 cumulative planes), tone value out, and in the
    training form the FP32 residual planes out."""
    sat = {"f32": 8, "c32x2": 16, "f64": 16}[prec]
    return 4 + sat + 4 * (n_bins - 1) + 4 + 4 * resid_planes


def query_source_digest() -> str:
    """Digest of everything the fused query kernel is built from: its source file, the device
    header, the compiler flags and its parameter struct."""
    from paper_2102_01289_amd import build as hip_build
    h = hashlib.sha256()
    for f in QUERY_SOURCES:
        with open(os.path.join(ROOT, f), "rb") as fh:
            h.update(fh.read())
    h.update(" ".join(hip_build.COMMON[:-1]).encode())   # the flags, without the include path
    with open(os.path.join(ROOT, QUERY_STRUCT[0])) as fh:
        text = fh.read()
    i = text.index(QUERY_STRUCT[1])
    h.update(text[i:text.index("};", i)].encode())
    return h.hexdigest()[:16]


def measured_traffic(variant: str, prec: str, n_bins: int, n_scales: int,
                     workload: str = WORKLOAD):
    """HBM bytes per launch of the fused query from the committed counter summary: FETCH_SIZE
    and WRITE_SIZE (KiB per dispatch) each times its copy-kernel calibration factor.  None when
    no record matches this configuration or the kernel's sources changed since the counters
    were taken."""
    try:
        with open(traffic_profile(workload)) as f:
            lines = f.read().splitlines()
    except OSError:
        return None
    digest = query_source_digest()
    for ln in lines:
        if not ln.startswith("traffic-record: "):
            continue
        r = json.loads(ln[len("traffic-record: "):])
        if (r["variant"], r["prec"], r["n_bins"], r["n_scales"], r["workload"]) != (
                variant, prec, n_bins, n_scales, workload):
            continue
        if r["source_digest"] != digest:
            return None
        return int(round(r["fetch_kib"] * 1024 * r["fetch_factor"] +
                         r["write_kib"] * 1024 * r["write_factor"]))
    return None


def host_threads() -> int:
    """Host threads this process may use: its CPU affinity, capped by OMP_NUM_THREADS when
    that is set (the share of the host given to one GPU)."""
    try:
        n = len(os.sched_getaffinity(0))
    except (AttributeError, OSError):
        n = os.cpu_count() or 1
    cap = os.environ.get("OMP_NUM_THREADS", "")
    if cap.isdigit() and int(cap) > 0:
        n = min(n, int(cap))
    return max(n, 1)


def cpu_model() -> str:
    try:
        with open("/proc/cpuinfo") as f:
            for ln in f:
                if ln.startswith("model name"):
                    return ln.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(rgb, params_np, backward: bool, gpu_outputs=None):
    """The oracle on the full image, on all the host threads this process may use and on one
    thread (the forward's per-pixel loops and the adjoint's box sums run on OpenMP threads;
    the double-double tables are built serially either way).  gpu_outputs: {name: L} device
    forwards of the same image, whose max-abs and p99.9 error against the oracle's FP64 L are
    reported beside the timing."""
    import numpy as np

    import oracle
    from synth import gen_upstream_grad
    n, s, eps, seed = params_np
    H, W = rgb.shape[1:]
    g = gen_upstream_grad((H, W), seed=seed).astype(np.float64) if backward else None

    def run(threads):
        oracle.set_threads(threads)
        t0 = time.perf_counter()
        lum = oracle.luminance(rgb)
        e = oracle.exact_edges(lum.min(), lum.max(), n)
        rx, ry = oracle.paper_radii(H, W, s)
        L = oracle.forward(lum, e, rx, ry, eps)
        if backward:
            oracle.backward(lum, e, rx, ry, g, eps)
        return time.perf_counter() - t0, L

    threads = host_threads()
    dt, L = run(threads)
    dt1, _ = run(1) if threads > 1 else (dt, None)
    oracle.set_threads(1)
    what = "forward+backward" if backward else "forward"
    out = {"value": round(H * W / dt / 1e6, 4), "unit": "megapixels/s", "cores": threads,
           "kind": "oracle",
           "sample": (f"full {W}x{H} {what} (luminance, exact edges, FP64 double-double "
                      f"tables, per-pixel pass{', adjoint' if backward else ''}) on {threads} "
                      f"OpenMP threads, {dt:.1f} s; one thread {dt1:.1f} s"),
           "single_thread_value": round(H * W / dt1 / 1e6, 4),
           "host_cpus": os.cpu_count(), "cpu_model": cpu_model()}
    if gpu_outputs:
        err = {}
        for name, Lg in gpu_outputs.items():
            d = np.abs(Lg.astype(np.float64) - L)
            err[name] = {"max_abs": float(f"{d.max():.3e}"),
                         "p99_9": float(f"{np.quantile(d, 0.999):.3e}")}
        out["forward_error_vs_oracle"] = err
    return out


def main():
    args = _parse()
    if args.gpus != 1:
        print(f"bench.py: the tone-mapping path runs on one GPU only (asked for --gpus "
              f"{args.gpus}); sharding across GPUs is not implemented", file=sys.stderr)
        sys.exit(2)
    if args.workload == "batch":
        bench_batch(args)
        return
    if args.workload == "sweep":
        bench_sweep(args)
        return
    if args.workload == "hdr":
        bench_hdr(args)
        return
    if args.workload == "stress":
        bench_stress(args)
        return
    if args.workload == "scan":
        bench_scan(args)
        return
    if args.workload == "logvar":
        bench_logvar(args)
        return

    import numpy as np
    import torch

    import paper_2102_01289_amd as tm
    from synth import WORKLOADS, gen_upstream_grad, gen_wdr

    cfg = WORKLOADS[args.image]
    H, W = cfg["H"], cfg["W"]
    img = gen_wdr(H, W, cfg["K"], cfg["lo"], cfg["hi"], cfg["seed"])
    dev = torch.device("cuda:0")
    rgb = torch.from_numpy(img.rgb).to(dev)
    params = tm.make_params(args.n_bins, args.n_scales, eps=args.eps, H=H, W=W)
    mapper = tm.ToneMapper(H, W, params, args.prec, device=dev)
    stream = torch.cuda.current_stream()

    g = torch.from_numpy(gen_upstream_grad((H, W), seed=cfg["seed"] + 1)).to(dev)
    do_bwd = not args.no_backward

    # forward+backward: the training forward writes the residual planes the backward reads
    query = mapper.query_train if do_bwd else mapper.query

    def step(ev=None):
        ko = args.kernel_only
        if ko in (None, "tables"):
            mapper.prologue(rgb)
            mapper.tables()
        if ko in (None, "query"):
            if ev is not None:
                ev[0].record(stream)
            query()
            if ev is not None:
                ev[1].record(stream)
        if do_bwd and ko in (None, "backward"):
            mapper.backward_resid(g)

    # warm-up (also produces the tables a query-only or backward-only loop reads)
    mapper.run_train(rgb) if do_bwd else mapper.run(rgb)
    if do_bwd:
        mapper.backward_resid(g)
    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()

    evs = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
           for _ in range(args.steps)]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i in range(args.steps):
        step(evs[i])
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ms_step = wall * 1e3 / args.steps
    q_ms = float(np.mean([a.elapsed_time(b) for a, b in evs])) if args.kernel_only in (
        None, "query") else float("nan")

    # per-stage split (outside the timed loop)
    stage = {}
    stages = [("prologue", lambda: mapper.prologue(rgb)), ("tables", mapper.tables),
              ("query", mapper.query)]
    if do_bwd:
        stages += [("query_train", mapper.query_train),
                   ("backward", lambda: mapper.backward_resid(g))]
    for name, fn in stages:
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record(stream)
        for _ in range(5):
            fn()
        b.record(stream)
        torch.cuda.synchronize()
        stage[name] = round(a.elapsed_time(b) / 5, 4)
    fwd_ms = stage["prologue"] + stage["tables"] + stage["query"]
    step_ms = fwd_ms + (stage["query_train"] - stage["query"] + stage["backward"] if do_bwd else 0)

    copy_gbs = None
    if args.copy_probe:
        src = torch.empty(1 << 28, dtype=torch.float32, device=dev).fill_(1.0)
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record(stream)
        dst.copy_(src)
        b.record(stream)
        torch.cuda.synchronize()
        copy_gbs = round(2 * src.numel() * 4 / (a.elapsed_time(b) * 1e-3) / 1e9, 1)
        del src, dst

    mpx = H * W / 1e6
    qbytes = query_bytes_per_px(args.prec, args.n_bins,
                                tm.residual_planes(args.n_scales) if do_bwd else 0) * H * W
    achieved = qbytes / (q_ms * 1e-3) / 1e9
    traffic = measured_traffic("train" if do_bwd else "forward", args.prec, args.n_bins,
                               args.n_scales, args.image)
    # counted HBM rate: the calibrated counter bytes per launch over the live duration
    traffic_gbs = traffic / (q_ms * 1e-3) / 1e9 if traffic else None
    line = {
        "metric": "megapixels/s fwd and fwd+bwd at 12MP vs plain fwd; HBM GB/s fraction",
        "value": round(mpx / (ms_step * 1e-3), 3),
        "unit": "megapixels/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_step, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": {"c32x2": "f32x2", "f32": "f32", "f64": "f64"}[args.prec],
        "data": "synthetic",
        "config": {"workload": args.image, "height": H, "width": W, "n_bins": args.n_bins,
                   "n_scales": args.n_scales, "eps": args.eps, "sat_precision": args.prec,
                   "radii_x": list(params.rx[:args.n_scales]),
                   "radii_y": list(params.ry[:args.n_scales]),
                   "step": ("forward+backward" if do_bwd else "forward")
                   if args.kernel_only is None else args.kernel_only},
        "fwd_mp_s": round(mpx / (fwd_ms * 1e-3), 3),
        "fwd_bwd_mp_s": round(mpx / (step_ms * 1e-3), 3) if do_bwd else None,
        "fwd_bwd_over_fwd": round(fwd_ms / step_ms, 4) if do_bwd else None,
        "stage_ms": stage,
        "copy_probe_gbs": copy_gbs,
        "roofline": {"bound": "hbm",
                     "kernel": ("forward_kernel (fused query+blend, training form writing the "
                                "residual planes)") if do_bwd else
                     "forward_kernel (fused query+blend)",
                     "achieved": round(achieved, 1), "peak": PEAK_HBM_GBS, "unit": "GB/s",
                     "frac": round(achieved / PEAK_HBM_GBS, 4),
                     "traffic": traffic,
                     "traffic_gbs": round(traffic_gbs, 1) if traffic_gbs else None,
                     "traffic_frac": round(traffic_gbs / PEAK_HBM_GBS, 4) if traffic_gbs
                     else None,
                     "algorithmic_bytes_per_launch": qbytes,
                     "avg_kernel_ms": round(q_ms, 4)},
    }
    # the FP64-table forward of the same image beside the default precision (same stages)
    other = None
    if args.prec != "f64" and args.kernel_only is None:
        m64 = tm.ToneMapper(H, W, params, "f64", device=dev)
        m64.run(rgb)
        st64 = {}
        for name, fn in (("prologue", lambda: m64.prologue(rgb)), ("tables", m64.tables),
                         ("query", m64.query)):
            a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            a.record(stream)
            for _ in range(5):
                fn()
            b.record(stream)
            torch.cuda.synchronize()
            st64[name] = round(a.elapsed_time(b) / 5, 4)
        f64_ms = sum(st64.values())
        line["f64_tables"] = {"fwd_mp_s": round(mpx / (f64_ms * 1e-3), 3), "stage_ms": st64}
        m64.run(rgb)
        other = m64
    if not args.no_cpu_baseline:
        outs = {args.prec: mapper.run(rgb).cpu().numpy()}
        if other is not None:
            outs["f64"] = other.run(rgb).cpu().numpy()
        torch.cuda.synchronize()
        line["cpu_baseline"] = cpu_baseline(img.rgb, (args.n_bins, args.n_scales, args.eps,
                                                      cfg["seed"] + 1), do_bwd, outs)
    if (not args.no_extras and args.kernel_only is None and args.image == WORKLOAD
            and not args.copy_probe):
        # the secondary workloads, so that every run of the default line records them
        for key, fn in (("batch", lambda: batch_extra(args)),
                        ("stress", lambda: stress_line(args)),
                        ("log_variance", lambda: log_variance_extra(args, rgb, g, H, W))):
            try:
                line[key] = fn()
            except Exception as e:   # a secondary block never loses the headline line
                line[key] = {"error": f"{type(e).__name__}: {e}"}
            torch.cuda.synchronize()
        st = line.get("stress", {})
        if "value" in st:
            line["stress"] = {k: st[k] for k in ("value", "unit", "ms_per_step", "stage_ms",
                                                  "forward_algorithmic_frac", "config")}
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
