"""The per-pixel gradient bound the GPU backward tests use (tests/_bounds.backward_bound) is
not vacuous: on WDR images it sits below half the gradient's own size at almost every pixel,
and mistakes planted in the oracle's gradient -- a zeroed dark region, a wrong radius, a
dropped field, a wrong eps -- exceed it at most pixels.  (The bound is derived from the
arithmetic; these checks show it is tight enough to catch what the looser
max-relative tolerance let through.)"""
import numpy as np
import pytest

import oracle
from _bounds import backward_bound, tiling, window_sums
from synth import gen_wdr


@pytest.fixture(scope="module", params=[(96, 128, 21), (256, 256, 101)])
def case(request):
    H, W, seed = request.param
    lum = oracle.luminance(gen_wdr(H, W, 6, -2.0, 4.0, seed).rgb)
    e = oracle.exact_edges(lum.min(), lum.max(), 5)
    rx, ry = oracle.paper_radii(H, W, 5)
    g = np.random.default_rng(4).standard_normal((H, W))
    dv, _ = oracle.backward(lum, e, rx, ry, g, 0.1)
    Lr, Lj, Wj, varj = oracle.forward(lum, e, rx, ry, 0.1, per_scale=True)
    vec, th = tiling(H, W)
    B, bad = backward_bound(lum, g, Lr, Lj, Wj, varj, window_sums(lum, rx, ry), rx, ry, 0.1,
                            "f64", vec, th, dv_ref=dv)
    return dict(lum=lum, e=e, rx=rx, ry=ry, g=g, dv=dv, B=B, bad=bad)


def test_bound_is_tight(case):
    assert case["bad"] == 0
    assert np.mean(case["B"] < 0.5 * np.abs(case["dv"])) >= 0.95


def test_zeroed_dark_gradient_is_caught(case):
    dark = case["lum"] <= np.quantile(case["lum"], 0.1)
    assert np.mean(np.abs(case["dv"][dark]) > case["B"][dark]) >= 0.99


@pytest.mark.parametrize("mistake", ["radius", "dropped_field", "eps"])
def test_planted_oracle_mistakes_are_caught(case, mistake):
    c = case
    rx, ry, eps = list(c["rx"]), list(c["ry"]), 0.1
    if mistake == "radius":
        rx[4] -= 1
    elif mistake == "dropped_field":
        rx, ry = rx[:4], ry[:4]
    else:
        eps = 0.1001
    wrong, _ = oracle.backward(c["lum"], c["e"], rx, ry, c["g"], eps)
    frac = np.mean(np.abs(wrong - c["dv"]) > c["B"])
    assert frac >= (0.4 if mistake == "eps" else 0.95), frac
