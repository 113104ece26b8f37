"""The closed-form bound of the size-limit test against the general per-pixel bound, on a
small row-invariant image (CPU only): for such an image the quadrant sums of |q| are the
row's prefix sums times the row count, so the two must agree row by row, and the bound taken
at its largest over the rows must cover every row."""
import numpy as np
import pytest

import oracle
from _bounds import forward_bound, tiling, window_sums
from _cases import edges_ref
from synth import gen_wdr_row
from test_gpu_limits import EPS, N_BINS, N_SCALES, _row_bound


@pytest.mark.parametrize("prec", ["c32x2", "f64"])
def test_closed_form_bound_matches_the_general_bound(prec):
    H, W = 23, 700
    row = gen_wdr_row(W, K=6, lo=-2.0, hi=4.0, seed=5)
    img = np.repeat(row[None, :], H, axis=0)
    e = edges_ref(img, N_BINS)
    rx, ry = oracle.paper_radii(H, W, N_SCALES)
    Lref, Lj, Wj, varj = oracle.forward(img, e, rx, ry, EPS, per_scale=True)
    # the forward of the repeated row is the row's forward on every row
    Lrow, Ljr, Wjr, varjr = oracle.forward(row[None, :], e, rx, ry, EPS, per_scale=True)
    assert np.allclose(Lref, Lrow, rtol=0, atol=1e-12)
    vd = img.astype(np.float64)
    mu = (float(np.float32(vd.mean())), float(np.float32((vd * vd).mean())))
    vec, th = tiling(H, W)
    general = forward_bound(img, Lref, Lj, Wj, varj, window_sums(img, rx, ry), rx, ry, EPS,
                            prec, vec, th, *(mu if prec == "c32x2" else (0.0, 0.0)))
    ys = list(range(H))
    closed = _row_bound(row, H, rx, ry, Lrow, Ljr, Wjr, varjr, prec, ys)
    for y in ys:
        assert np.allclose(closed[y], general[y], rtol=1e-9, atol=0), y
    assert np.all(closed[-1] >= general.max(axis=0) * (1 - 1e-12))
