"""Shared helpers of the GPU parity tests: seeded inputs and oracle references."""
from __future__ import annotations

import numpy as np
import torch

import oracle
from synth import gen_wdr

U32 = np.uint32


def rgb_case(H, W, K=6, lo=-2.0, hi=4.0, seed=0):
    return gen_wdr(H, W, K, lo, hi, seed).rgb


def to_dev(a: np.ndarray) -> torch.Tensor:
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def lum_ref(rgb):
    return oracle.luminance(rgb)


def edges_ref(lum, n):
    return oracle.exact_edges(lum.min(), lum.max(), n)


def fill_garbage(t) -> None:
    """Overwrite a Table's whole buffer with a non-zero pattern so that the border zeros the
    producing call must write are really checked."""
    buf = t.buf
    if buf.dtype in (torch.float32, torch.float64):
        buf.fill_(float("nan"))
    else:
        buf.view(torch.int32).fill_(-559038737)


def hist_ref(lum, edges, n, layout):
    b = oracle.bins(lum, edges)
    return oracle.integral_histogram(b, n, cumulative=(layout == "cumulative"))


def check_gradient(lum, edges, rx, ry, eps, g, gv, sat, offsets, prec, ld=(0.0, 1.0),
                   oracle_fwd=None, oracle_bwd=None):
    """Device gradient gv (float64 [H, W]) of sum(g L) against the FP64 oracle, at every pixel,
    within the derived per-pixel bound of tests/_bounds.backward_bound, with the integral
    image's entry errors measured on the device's own table (sat, a Table) against the
    oracle's double-double tables.  Returns the oracle's (dv, (d eps, d min L_d, d max L_d))
    and the per-field forward arrays, for further checks."""
    from _bounds import backward_bound, measured_entry_errors, window_sums
    g64 = np.asarray(g, dtype=np.float64)
    if oracle_bwd is None:
        oracle_bwd = oracle.backward(lum, edges, rx, ry, g64, eps, ld[0], ld[1])
    dv, gref = oracle_bwd
    if oracle_fwd is None:
        oracle_fwd = oracle.forward(lum, edges, rx, ry, eps, ld[0], ld[1], per_scale=True)
    Lr, Lj, Wj, varj = oracle_fwd
    mu = offsets.cpu().numpy().astype(np.float64) if prec == "c32x2" else (0.0, 0.0)
    err = measured_entry_errors(sat.padded(), lum, prec, float(mu[0]), float(mu[1]))
    B, bad = backward_bound(lum, g64, Lr, Lj, Wj, varj, window_sums(lum, rx, ry), rx, ry, eps,
                            prec, 1, 1, float(mu[0]), float(mu[1]), dv_ref=dv, entry_err=err)
    # pixels whose fusion weights are too uncertain for a first-order bound (every window
    # nearly flat) leave the pixels of their windows unchecked: they must stay rare
    H, W = lum.shape
    assert bad <= max(2, H * W // 1000), f"{bad} pixels with uncertain fusion weights"
    assert np.mean(np.isinf(B)) <= 0.05, np.mean(np.isinf(B))
    over = np.abs(gv - dv) / B
    worst = np.unravel_index(int(np.argmax(over)), over.shape)
    assert np.all(over <= 1.0), (f"gradient outside the derived bound at {int(np.sum(over > 1))} "
                                 f"pixels; worst {worst}: gpu {gv[worst]:.6e} oracle "
                                 f"{dv[worst]:.6e} bound {B[worst]:.3e}")
    return dv, gref, oracle_fwd


def check_scalar_gradients(gp, gref, g, oracle_fwd, eps, ld=(0.0, 1.0)):
    """d/d min L_d and d/d max L_d (sums of g (1 - Pbar), g Pbar, Pbar from exact counts)
    within 2e-4 relative; d/d eps = sum_p g E, a sum that cancels by up to four decades under
    N(0, 1) weights, held to its condition: E is evaluated in FP32 (tens of roundings, < 1e-5
    relative) from variances bounded per pixel, so |d| <= 1e-5 sum |g E| + 2e-4 |value|."""
    gp = np.asarray(gp, dtype=np.float64)
    gref = np.asarray(gref, dtype=np.float64)
    assert np.allclose(gp[1:], gref[1:], rtol=2e-4, atol=1e-6), (gp, gref)
    Lr, Lj, Wj, varj = oracle_fwd
    Dw = Wj.sum(axis=0)
    with np.errstate(invalid="ignore", divide="ignore"):
        E = np.where(Dw > 0, np.sum(-varj / (varj + eps) ** 2 * (Lj - Lr[None]), axis=0)
                     / np.where(Dw > 0, Dw, 1.0), 0.0)
    cond = float(np.sum(np.abs(np.asarray(g, dtype=np.float64) * E)))
    assert abs(gp[0] - gref[0]) <= 1e-5 * cond + 2e-4 * abs(gref[0]) + 1e-6, \
        (gp[0], gref[0], cond)
