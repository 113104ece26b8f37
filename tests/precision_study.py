"""Precision study (run as a script on a machine with the GPU, not collected by pytest): the output error
of each integral-image precision against the FP64 oracle on whole images -- the paper set at
4000x3000 (10^8:1) and the n = 64, radii {4, 16, 64} stress set at 1920x1080 -- and, for
the paper set, the log-domain variance variant against the oracle's FP64 log-variance form.
Each variant's whole forward (prologue, tables, query) is timed beside its error.  Prints
one JSON object.

    python tests/precision_study.py > precision.json
"""
from __future__ import annotations

import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def _median_ms(fn, reps=10, warmup=2):
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


def main():
    import numpy as np
    import torch

    import oracle
    import paper_2102_01289_amd as tm
    from synth import WORKLOADS, gen_wdr

    dev = torch.device("cuda:0")
    cases = [("wdr_4000x3000", 5, None), ("wdr_1920x1080", 64, [4, 16, 64])]
    out = {"metric": "max-abs / p99.9 output error vs FP64 oracle per integral-image precision",
           "data": "synthetic", "cases": []}
    for name, n, radii in cases:
        c = WORKLOADS[name]
        H, W = c["H"], c["W"]
        rgb = gen_wdr(H, W, c["K"], c["lo"], c["hi"], c["seed"]).rgb
        lum = oracle.luminance(rgb)
        e = oracle.exact_edges(lum.min(), lum.max(), n)
        if radii is None:
            rx, ry = oracle.paper_radii(H, W, 5)
        else:
            rx, ry = radii, radii
        t0 = time.perf_counter()
        ref = oracle.forward(lum, e, rx, ry, 0.1)
        t_orc = time.perf_counter() - t0
        p = tm.make_params(n, len(rx), rx, ry, 0.1)
        case = {"workload": name, "n_bins": n, "radii_x": list(rx), "radii_y": list(ry),
                "dynamic_range": float(lum.max() / lum.min()), "oracle_s": round(t_orc, 2),
                "variants": {}}
        refs = {"linear": ref}
        variants = [(prec, "linear") for prec in ("f32", "c32x2", "f64")]
        if radii is None:
            refs["log"] = oracle.forward(lum, e, rx, ry, 0.1, var_domain="log")
            variants += [(prec, "log") for prec in ("f32", "c32x2", "f64")]
        x = torch.from_numpy(rgb).to(dev)
        G_ref = oracle.integral_histogram(oracle.bins(lum, e), n, cumulative=True)
        for prec, dom in variants:
            m = tm.ToneMapper(H, W, p, prec, device=dev, variance=dom)
            L = m.run(x).cpu().numpy().astype(np.float64)
            G = m.hist.padded()[..., 0].numpy().astype(np.uint64)
            err = np.abs(L - refs[dom])
            ms = _median_ms(lambda: m.run(x), reps=10)
            key = prec if dom == "linear" else f"log_{prec}"
            case["variants"][key] = {
                "max_abs": float(err.max()), "p99_9": float(np.quantile(err, 0.999)),
                "mean_abs": float(err.mean()), "frac_above_1_255": float(np.mean(err > 1 / 255)),
                "histogram_bit_exact": bool(np.array_equal(G, G_ref)),
                "forward_ms": round(ms, 4), "forward_mp_s": round(H * W / ms / 1e3, 1)}
            del m
            print(f"precision: {name} {key} max {err.max():.3e} {ms:.3f} ms", file=sys.stderr,
                  flush=True)
        out["cases"].append(case)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
