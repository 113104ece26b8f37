"""Autotuner of the scan tiling (columns per lane, rows per tile, histogram planes per pass).

Candidates are timed on the device with HIP events (median of `reps` runs after a warm-up);
the winner is cached in a JSON file keyed by device, workload signature, bin count and
integral-image precision.  Only the scans depend on the tiling, so single images time the
table build alone and batches time the whole batched forward.
"""
from __future__ import annotations

import json
import os
import statistics

import torch

from . import Batch, ToneMapper, make_params, tune

__all__ = ["candidates", "tune_image", "tune_batch", "cache_path", "cached_image_tune"]


def cache_path() -> str:
    return os.environ.get("TM355_TUNE_CACHE",
                          os.path.join(os.path.expanduser("~"), ".cache", "tm355", "tune.json"))


def _load() -> dict:
    try:
        with open(cache_path()) as f:
            return json.load(f)
    except (OSError, ValueError):
        return {}


def _store(key: str, value) -> None:
    path = cache_path()
    os.makedirs(os.path.dirname(path), exist_ok=True)
    d = _load()
    d[key] = value
    tmp = path + ".tmp"
    with open(tmp, "w") as f:
        json.dump(d, f, indent=1, sort_keys=True)
    os.replace(tmp, path)


def candidates(n_bins: int, batch: bool = False):
    """Tilings to time: columns per lane x rows per tile x planes per pass.  For batches,
    0 columns per lane or 0 rows per tile means each image takes the default for its own
    shape."""
    planes = n_bins - 1
    chunks = [c for c in (2, 4, 8) if c <= max(planes, 2) or c == 4]
    rows = (0, 4, 8, 16, 32) if batch else (4, 8, 16, 32)
    vecs = (0, 2, 4, 8) if batch else (2, 4, 8)
    return [(v, th, c) for v in vecs for th in rows for c in chunks]


def _time(fn, reps: int, warmup: int = 2) -> float:
    for _ in range(warmup):
        fn()
    torch.cuda.synchronize()
    ts = []
    for _ in range(reps):
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record()
        fn()
        b.record()
        torch.cuda.synchronize()
        ts.append(a.elapsed_time(b))
    return statistics.median(ts)


def _device_key(device=None) -> str:
    p = torch.cuda.get_device_properties(
        torch.cuda.current_device() if device is None or device.index is None else device)
    return f"{p.name}|{getattr(p, 'gcnArchName', '')}|cu{p.multi_processor_count}"


def _bucket(H: int, W: int) -> str:
    # shapes within a factor of ~1.4 per axis share a tuning
    import math
    return f"{int(round(2 * math.log2(H)))}x{int(round(2 * math.log2(W)))}"


def _image_key(H: int, W: int, n_bins: int, prec: str, device=None) -> str:
    return f"image|{_device_key(device)}|{_bucket(H, W)}|n{n_bins}|{prec}"


def cached_image_tune(H: int, W: int, n_bins: int = 5, prec: str = "c32x2", device=None):
    """The tiling tune_image stored for this device, shape bucket, bin count and precision,
    or None (the shape's default) when none is stored.  Looks up only; never times."""
    hit = _load().get(_image_key(H, W, n_bins, prec, device))
    return tune(*hit[:3]) if hit else None


def tune_image(rgb: torch.Tensor, n_bins: int = 5, prec: str = "c32x2", reps: int = 5,
               use_cache: bool = True, cands=None):
    """Best tiling for the table build of one image shape: (TmTune, ms)."""
    _, H, W = rgb.shape
    key = _image_key(H, W, n_bins, prec, rgb.device)
    if use_cache and cands is None:
        hit = _load().get(key)
        if hit:
            return tune(*hit[:3]), hit[3]
    p = make_params(n_bins, 1, [0], [0])
    best = None
    for c in (cands or candidates(n_bins)):
        m = ToneMapper(H, W, p, prec, tune=tune(*c), device=rgb.device)
        m.prologue(rgb)
        ms = _time(m.tables, reps)
        if best is None or ms < best[1]:
            best = (c, ms)
        del m
    if use_cache and cands is None:
        _store(key, [*best[0], best[1]])
    return tune(*best[0]), best[1]


def tune_batch(rgbs, n_bins: int = 5, n_scales: int = 5, prec: str = "c32x2", reps: int = 3,
               use_cache: bool = True, cands=None):
    """Best tiling for a batched forward: (TmTune, ms)."""
    shapes = sorted((int(r.shape[1]), int(r.shape[2])) for r in rgbs)
    mp = sum(h * w for h, w in shapes) / 1e6
    key = f"batch|{_device_key()}|{len(shapes)}|{mp:.0f}MP|n{n_bins}|s{n_scales}|{prec}"
    if use_cache and cands is None:
        hit = _load().get(key)
        if hit:
            return tune(*hit[:3]), hit[3]
    best = None
    for c in (cands or candidates(n_bins, batch=True)):
        b = Batch(rgbs, n_bins, n_scales, prec=prec, tune=tune(*c))
        ms = _time(b.forward, reps)
        b.close()
        del b
        if best is None or ms < best[1]:
            best = (c, ms)
    if use_cache and cands is None:
        _store(key, [*best[0], best[1]])
    return tune(*best[0]), best[1]
