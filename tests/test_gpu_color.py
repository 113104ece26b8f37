"""Colour restoration (Eq. 12) fused into the query, and the end-to-end RGB -> RGB call,
against the FP64 oracle."""
import numpy as np
import pytest
import torch

import oracle
import paper_2102_01289_amd as tm
from _bounds import forward_bound, tiling, window_sums
from _cases import edges_ref, lum_ref, rgb_case, to_dev

pytestmark = pytest.mark.gpu

SHAPES = [(96, 130), (37, 123), (1, 1), (1, 300), (130, 1030)]


def colour_tolerance(rgb, lum, Lbound, ref, sat):
    """|c_gpu - c_oracle| per value: the channel ratio (c/v)^sat times the derived bound on
    |L_gpu - L_oracle|, plus the FP32 colour arithmetic (a division, powf and a product:
    1e-6 relative)."""
    c = np.maximum(rgb.astype(np.float64), 0.0)
    lv = lum.astype(np.float64)
    ratio = np.where(lv > 0, c / np.where(lv > 0, lv, 1.0), 1.0) ** sat
    return ratio * Lbound[None] + 1e-6 * np.abs(ref) + 1e-30


@pytest.mark.parametrize("H,W", SHAPES)
@pytest.mark.parametrize("prec", ["c32x2", "f64"])
@pytest.mark.parametrize("sat", [0.6, 0.0, 1.0, 0.35])
def test_fused_colour_restoration(H, W, prec, sat):
    rgb = rgb_case(H, W, 5, seed=H + W)
    p = tm.make_params(5, 5, eps=0.1, H=H, W=W)
    m = tm.ToneMapper(H, W, p, prec)
    L_plain = m.run(to_dev(rgb)).clone()
    out = m.run_rgb(to_dev(rgb), sat).clone()
    torch.cuda.synchronize()
    assert torch.equal(m.out, L_plain)             # the fused colour stage leaves L unchanged
    # against the oracle chain (luminance, exact edges, FP64 forward, Eq. 12); the tolerance
    # carries the derived per-pixel bound of the fused forward through Eq. 12
    lum = lum_ref(rgb)
    e = edges_ref(lum, 5)
    rx, ry = oracle.paper_radii(H, W, 5)
    Lref, Lj, Wj, varj = oracle.forward(lum, e, rx, ry, 0.1, per_scale=True)
    vd = lum.astype(np.float64)
    mu = (float(np.float32(vd.mean())), float(np.float32((vd * vd).mean())))
    vec, th = tiling(H, W)
    Lb = forward_bound(lum, Lref, Lj, Wj, varj, window_sums(lum, rx, ry), rx, ry, 0.1, prec,
                       vec, th, *(mu if prec == "c32x2" else (0.0, 0.0)))
    ref = oracle.color_restore(rgb, lum, Lref, sat)
    got = out.cpu().numpy().astype(np.float64)
    assert np.all(np.abs(got - ref) <= colour_tolerance(rgb, lum, Lb, ref, sat))


@pytest.mark.parametrize("prec", ["c32x2", "f64"])
def test_end_to_end_rgb(prec):
    H, W = 160, 210
    rgb = rgb_case(H, W, 6, seed=4)
    rgb[:, 10:20, 30:60] = 0.0                     # a black patch (luminance 0)
    d = to_dev(rgb)
    out = tm.tonemap_rgb(d, prec=prec, ld_min=0.1, ld_max=0.9)
    p = tm.make_params(5, 5, eps=0.1, ld_min=0.1, ld_max=0.9, H=H, W=W)
    staged = tm.ToneMapper(H, W, p, prec).run_rgb(d, 0.6)
    torch.cuda.synchronize()
    assert torch.equal(out, staged)                # one call = the three stages
    # against the whole FP64 oracle chain: luminance, exact edges, FP64 forward, Eq. 12
    lum = lum_ref(rgb)
    e = edges_ref(lum, 5)
    rx, ry = oracle.paper_radii(H, W, 5)
    Lref = oracle.forward(lum, e, rx, ry, 0.1, ldmin=0.1, ldmax=0.9)
    ref = oracle.color_restore(rgb, lum, Lref, 0.6)
    got = out.cpu().numpy().astype(np.float64)
    c = np.maximum(rgb.astype(np.float64), 0.0)
    ratio = np.where(lum > 0, c / np.where(lum > 0, lum, 1.0), 1.0) ** 0.6
    assert np.all(np.abs(got - ref) <= ratio * 1e-4 + 1e-6 * np.abs(ref))
    # the black patch is neutral: every channel equals the tone-mapped luminance
    blk = got[:, 10:20, 30:60]
    assert np.all(blk == blk[0:1]) and np.allclose(blk[0], Lref[10:20, 30:60], atol=1e-4)
