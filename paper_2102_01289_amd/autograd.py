"""torch.autograd.Function over the C ABI: forward = tables + fused query, backward = the
hand-written adjoint (tm_tonemap_backward).

Differentiable inputs: the luminance image and the scalars (eps, min L_d, max L_d).  The bin
edges are statistics of the image held fixed in the backward (stop-gradient), and the bin
counts are piecewise constant in the luminance, so their derivative is zero almost
everywhere.  recompute=False (fastest): the forward writes the backward's residual planes
(2s + 2 FP32 per pixel) and the backward reads no table.  recompute=True (least memory kept
between the passes): only the luminance, edges and offsets are kept; the backward rebuilds
the integral tables and derives the residual planes from them.

The three scalars reach the kernels through device memory (tm_params.scalars), so neither
pass synchronises with the host and both can be recorded into a CUDA/HIP graph.

variance="log": Eq. 10's variance is that of l = ln(max(lum, FLT_MIN)) (the bins still come
from lum).  The residual backward given lum forms l in its last pass and applies the chain
rule through the logarithm there (tm_tonemap_backward_resid_log).  With recompute=True the
backward rebuilds l's integral image (l formed on load, with the offsets the forward kept)
and lum's histogram, then runs the table-based form (tm_tonemap_backward_log).
"""
from __future__ import annotations

import torch

from . import (make_params, tm_image_stats, tm_integral_tables, tm_integral_tables_log,
               tm_log_luminance, tm_tonemap_backward, tm_tonemap_backward_log,
               tm_tonemap_backward_resid, tm_tonemap_backward_resid_log, tm_tonemap_forward,
               tm_tonemap_forward_train)

__all__ = ["TonemapFn", "tonemap_luminance"]


def _log_tables(lum, prec, edges, n_bins):
    """The log-domain variant's tables: integral image of l = ln(max(lum, FLT_MIN)) (formed
    on load) with l's offsets, integral histogram of lum.  (loff, sat, hist)."""
    _, loff, _ = tm_log_luminance(lum, write_plane=False)   # the offsets; no plane needed
    sat, hist = tm_integral_tables_log(lum, prec, loff, edges, n_bins,
                                       "cumulative" if n_bins > 1 else None)
    return loff, sat, hist


class TonemapFn(torch.autograd.Function):
    @staticmethod
    def forward(ctx, lum, eps, ld_min, ld_max, n_bins: int, rx, ry, prec: str = "c32x2",
                recompute: bool = True, variance: str = "linear"):
        H, W = lum.shape
        # device copy of (eps, ld_min, ld_max) that the kernels read when they run
        scal = torch.stack([t.detach().reshape(()).to(device=lum.device, dtype=torch.float32)
                            for t in (eps, ld_min, ld_max)]).contiguous()
        p = make_params(n_bins, len(rx), rx, ry, H=H, W=W, scalars=scal)
        edges, offsets, _ = tm_image_stats(lum, n_bins)
        log = variance == "log"
        if log:
            offsets, sat, hist = _log_tables(lum, prec, edges, n_bins)
        else:
            sat, hist = tm_integral_tables(lum, prec, offsets, edges, n_bins, "cumulative")
        if recompute:
            out = tm_tonemap_forward(lum, sat, hist, edges, p, offsets)
            ctx.resid = None
        else:
            out, ctx.resid = tm_tonemap_forward_train(lum, sat, hist, edges, p, offsets)
        del sat, hist
        ctx.meta = (p, prec, n_bins, eps.dtype, log)
        ctx.scal = scal            # p points into it
        ctx.save_for_backward(lum, edges, offsets)
        return out

    @staticmethod
    def backward(ctx, g):
        lum, edges, offsets = ctx.saved_tensors
        p, prec, n_bins, sdt, log = ctx.meta
        g = g.contiguous().float()
        if log and ctx.resid is None:
            # offsets saved by the forward are l's: rebuild l's table (formed on load) and
            # lum's histogram, then the table-based backward with the chain rule to lum
            sat, hist = tm_integral_tables_log(lum, prec, offsets, edges, n_bins,
                                               "cumulative" if n_bins > 1 else None)
            gv, gp = tm_tonemap_backward_log(lum, sat, hist, edges, p, g, offsets)
        elif log:
            gv, gp = tm_tonemap_backward_resid_log(lum, p, ctx.resid, g)
            ctx.resid = None
        elif ctx.resid is None:
            sat, hist = tm_integral_tables(lum, prec, offsets, edges, n_bins, "cumulative")
            gv, gp = tm_tonemap_backward(lum, sat, hist, edges, p, g, offsets)
        else:
            gv, gp = tm_tonemap_backward_resid(lum, p, ctx.resid, g)
            ctx.resid = None
        return (gv, gp[0].to(sdt), gp[1].to(sdt), gp[2].to(sdt), None, None, None, None, None,
                None)


def tonemap_luminance(lum, eps, ld_min, ld_max, n_bins=5, rx=None, ry=None, n_scales=5,
                      prec="c32x2", recompute=True, variance="linear"):
    """Differentiable tone mapping of a luminance image [H, W] (CUDA float32).  eps, ld_min,
    ld_max are 0-d tensors; radii default to the paper's pyramid; variance "linear" or "log"
    (Eq. 10's variance of l = ln lum)."""
    if variance not in ("linear", "log"):
        raise ValueError('variance must be "linear" or "log"')
    H, W = lum.shape
    if rx is None or ry is None:
        from . import paper_radii
        rx, ry = paper_radii(H, W, n_scales)
    return TonemapFn.apply(lum, eps, ld_min, ld_max, n_bins, tuple(rx), tuple(ry), prec,
                           recompute, variance)
