"""Pins for the CPU oracle: each check ties it to something other than itself -- a
hand-worked example, exact rational brute force, closed forms, invariants or symmetries
of the method (Section II, Eq. 1-11, Algorithm 1)."""
import json
import math
import os
from decimal import Decimal, getcontext
from fractions import Fraction

import numpy as np
import pytest

from oracle import brute
from synth import gen_wdr

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _lum(orc, H, W, K=4, seed=0, lo=-2.0, hi=4.0):
    return orc.luminance(gen_wdr(H, W, K, lo, hi, seed).rgb)


def _edges(orc, v, n):
    return orc.exact_edges(v.min(), v.max(), n)


# ----------------------------------------------------------------------------- Eq. 11
def test_luminance_matches_exact_fused_steps(orc):
    rng = np.random.default_rng(5)
    rgb = (10.0 ** rng.uniform(-3, 5, size=(3, 12, 11))).astype(np.float32)
    lum = orc.luminance(rgb)
    naive_differs = False
    for y in range(12):
        for x in range(11):
            want = brute.luminance_px(*rgb[:, y, x])
            assert lum[y, x] == want, (y, x)
            naive = np.float32(np.float32(np.float32(0.2126) * rgb[0, y, x])
                               + np.float32(np.float32(0.7152) * rgb[1, y, x]))
            naive = np.float32(naive + np.float32(np.float32(0.0722) * rgb[2, y, x]))
            naive_differs |= bool(naive != want)
    # the pin is sensitive to the rounding order: unfused evaluation differs somewhere
    assert naive_differs


# ----------------------------------------------------------------------------- edges
def _decimal_edges(a, b, n):
    getcontext().prec = 80
    la, lb = Decimal(float(a)).ln(), Decimal(float(b)).ln()
    out = []
    for k in range(1, n):
        ek = (la + (lb - la) * Decimal(k) / Decimal(n)).exp()
        c = np.float32(float(ek))
        while Decimal(float(c)) < ek:
            c = np.nextafter(c, np.float32(np.inf))
        while Decimal(float(np.nextafter(c, np.float32(-np.inf)))) >= ek:
            c = np.nextafter(c, np.float32(-np.inf))
        out.append(c)
    return np.array(out, dtype=np.float32)


@pytest.mark.parametrize("a,b,n", [(0.001, 1e5, 5), (0.0040625315, 15334.056, 64),
                                   (1.0, 3.0, 7), (2.5e-3, 2.5e-3 * 1.0001, 5),
                                   (1e-30, 1e30, 256), (0.5, 0.75, 3)])
def test_edges_match_high_precision_logs(orc, a, b, n):
    got = orc.exact_edges(np.float32(a), np.float32(b), n)
    want = _decimal_edges(np.float32(a), np.float32(b), n)
    assert np.array_equal(got, want)
    assert np.all(np.diff(got) >= 0)


def test_edges_closed_forms(orc):
    # i_min = 1, i_max = 2^n: the log-domain edges fall on exact powers of two
    for n in (2, 5, 8, 31):
        e = orc.exact_edges(np.float32(1.0), np.float32(2.0 ** n), n)
        assert np.array_equal(e, np.float32(2.0) ** np.arange(1, n, dtype=np.float32))
    # i_min = 3, i_max = 3 * 4^4, n = 4 -> 3 * 4^k, exact
    e = orc.exact_edges(np.float32(3.0), np.float32(3.0 * 256), 4)
    assert np.array_equal(e, np.float32([12.0, 48.0, 192.0]))
    assert orc.exact_edges(1.0, 5.0, 1).size == 0                  # one bin: no edges
    assert np.all(np.isinf(orc.exact_edges(2.0, 2.0, 5)))           # flat image: one bin
    # a non-positive minimum is floored at the smallest normal FP32
    e0 = orc.exact_edges(np.float32(0.0), np.float32(1.0), 2)
    assert e0[0] == orc.exact_edges(np.float32(orc.FLT_MIN), np.float32(1.0), 2)[0]


def test_bins_match_exact_log_criterion(orc):
    v = _lum(orc, 14, 13, seed=3)
    for n in (2, 3, 5, 16, 64):
        b = orc.bins(v, _edges(orc, v, n))
        vmin, vmax = v.min(), v.max()
        for y in range(v.shape[0]):
            for x in range(v.shape[1]):
                assert b[y, x] == brute.bin_of(v[y, x], vmin, vmax, n)
        assert b.flat[np.argmin(v)] == 0 and b.flat[np.argmax(v)] == n - 1
        order = np.argsort(v, axis=None, kind="stable")
        assert np.all(np.diff(b.flat[order]) >= 0)


# ----------------------------------------------------------------------------- Eq. 8, 9
@pytest.mark.parametrize("n", [1, 2, 5, 64])
def test_integral_histogram_vs_window_counts(orc, n):
    rng = np.random.default_rng(11 + n)
    H, W = 13, 17
    b = rng.integers(0, n, size=(H, W)).astype(np.int32)
    Hk = orc.integral_histogram(b, n, cumulative=False)
    assert Hk.shape == (n, H + 1, W + 1)
    assert np.all(Hk[:, 0, :] == 0) and np.all(Hk[:, :, 0] == 0)
    # sum over bins of H_k is the pixel count (x+1)(y+1); last cell is H*W
    tot = Hk.sum(axis=0)
    yy, xx = np.mgrid[0:H + 1, 0:W + 1]
    assert np.array_equal(tot, (yy * xx).astype(np.uint64))
    assert np.array_equal(Hk[:, H, W], np.bincount(b.ravel(), minlength=n))
    for _ in range(40):  # Eq. 9 on random windows vs a direct count
        x0, x1 = sorted(rng.integers(-1, W, size=2))
        y0, y1 = sorted(rng.integers(-1, H, size=2))
        f = (Hk[:, y0 + 1, x0 + 1] + Hk[:, y1 + 1, x1 + 1]
             - Hk[:, y0 + 1, x1 + 1] - Hk[:, y1 + 1, x0 + 1])
        want = brute.window_hist(b, n, x0 + 1, x1, y0 + 1, y1) if x1 > x0 and y1 > y0 \
            else np.zeros(n)
        assert np.array_equal(f.astype(np.int64), want.astype(np.int64))
    if n > 1:
        G = orc.integral_histogram(b, n, cumulative=True)
        assert G.shape == (n - 1, H + 1, W + 1)
        for k in range(1, n):
            assert np.array_equal(G[k - 1], Hk[:k].sum(axis=0))


# ----------------------------------------------------------------------------- Eq. 5, 6
def test_integral_image_is_exact_window_sum(orc):
    rng = np.random.default_rng(2)
    H, W = 9, 12
    v = (10.0 ** rng.uniform(-3, 5, size=(H, W))).astype(np.float32)
    for square in (False, True):
        hi, lo = orc.integral_image(v, square)
        assert np.all(hi[0] == 0) and np.all(hi[:, 0] == 0)
        vv = [[Fraction(float(v[y, x])) ** (2 if square else 1) for x in range(W)]
              for y in range(H)]
        for y in range(H):
            for x in range(W):
                exact = sum(vv[yy][xx] for yy in range(y + 1) for xx in range(x + 1))
                got = Fraction(hi[y + 1, x + 1]) + Fraction(lo[y + 1, x + 1])
                assert abs(got - exact) <= abs(exact) * Fraction(1, 2 ** 100)
        # corner equals the image sum (correctly rounded)
        flat = [float(t) for row in vv for t in row]
        assert hi[H, W] == math.fsum(flat)


def test_integral_image_differencing_recovers_image(orc):
    v = np.arange(30, dtype=np.float32).reshape(5, 6) * 3 + 1   # integer-valued: exact
    hi, lo = orc.integral_image(v)
    assert np.all(lo == 0)
    rec = hi[1:, 1:] - hi[:-1, 1:] - hi[1:, :-1] + hi[:-1, :-1]
    assert np.array_equal(rec, v.astype(np.float64))


# ----------------------------------------------------------------------------- forward
def test_hand_worked_example(orc):
    g = json.load(open(os.path.join(GOLDEN, "hand_worked_1x4.json")))
    v = np.array([g["v"]], dtype=np.float32)
    e = orc.exact_edges(v.min(), v.max(), g["n_bins"])
    L = orc.forward(v, e, g["rx"], g["ry"], g["eps"], g["ld_min"], g["ld_max"])
    want = np.array([n / d for n, d in zip(g["L_num"], g["L_den"])])
    assert np.allclose(L[0], want, rtol=0, atol=1e-15)
    Lb = brute.forward(v, g["n_bins"], g["rx"], g["ry"], g["eps"], g["ld_min"], g["ld_max"])
    assert np.allclose(Lb[0], want, rtol=0, atol=1e-15)


@pytest.mark.parametrize("H,W,n,rx,ry,seed", [
    (6, 7, 5, [3, 1], [3, 1], 0),
    (5, 9, 3, [4, 2, 1], [2, 1, 0], 1),
    (8, 8, 2, [4, 2, 1], [4, 2, 1], 2),
    (7, 5, 4, [20], [20], 3),          # window larger than the image
    (1, 9, 5, [4, 2], [0, 0], 4),
    (9, 1, 5, [0, 0], [4, 2], 5),
    (6, 6, 64, [3, 1], [3, 1], 6),
])
def test_forward_matches_exact_brute_force(orc, H, W, n, rx, ry, seed):
    v = _lum(orc, H, W, seed=seed)
    L, Ls, Ws, _ = orc.forward(v, _edges(orc, v, n), rx, ry, per_scale=True)
    Lb, Lsb, Wsb = brute.forward(v, n, rx, ry, per_scale=True)
    assert np.max(np.abs(L - Lb)) <= 1e-12
    assert np.max(np.abs(Ls - Lsb)) <= 1e-15
    assert np.max(np.abs(Ws - Wsb)) <= 1e-12


def test_forward_tables_equal_direct_windows(orc):
    v = _lum(orc, 37, 45, K=6, seed=9, lo=-3, hi=5)
    rx, ry = orc.paper_radii(37, 45, 5)
    e = _edges(orc, v, 5)
    L = orc.forward(v, e, rx, ry)
    pix = np.arange(v.size)
    Ld = orc.forward_direct(v, e, rx, ry, pix)
    assert np.max(np.abs(L.ravel() - Ld)) <= 1e-13


def test_special_cases(orc):
    v = _lum(orc, 20, 24, seed=12)
    rx, ry = orc.paper_radii(20, 24, 3)
    # n = 1: every pixel is in the lowest bin, so every L_j is min L_d
    assert np.all(orc.forward(v, _edges(orc, v, 1), rx, ry, 0.1, 0.25, 0.75) == 0.25)
    # constant image: one bin and zero variance
    c = np.full((9, 11), 3.5, dtype=np.float32)
    assert np.all(orc.forward(c, _edges(orc, c, 5), [4, 2], [4, 2], 0.1, 0.2, 0.9) == 0.2)
    # s = 1 with a field covering the image: global histogram equalisation (closed form)
    n = 5
    e = _edges(orc, v, n)
    b = orc.bins(v, e)
    counts = np.bincount(b.ravel(), minlength=n)
    below = np.concatenate([[0], np.cumsum(counts)[:-1]])
    L = orc.forward(v, e, [100], [100], 0.1, 0.0, 1.0)
    assert np.allclose(L, below[b] / v.size, rtol=0, atol=1e-15)


def test_range_affinity_and_symmetry(orc):
    v = _lum(orc, 18, 23, seed=21)
    rx, ry = orc.paper_radii(18, 23, 4)
    e = _edges(orc, v, 5)
    L01 = orc.forward(v, e, rx, ry, 0.1, 0.0, 1.0)
    assert L01.min() >= 0.0 and L01.max() <= 1.0
    Lab = orc.forward(v, e, rx, ry, 0.1, 0.2, 0.7)
    assert np.allclose(Lab, 0.2 + 0.5 * L01, rtol=0, atol=1e-14)
    # mirror and transpose equivariance (Algorithm 1's window is symmetric)
    Lf = orc.forward(v[:, ::-1].copy(), e, rx, ry)
    assert np.allclose(Lf[:, ::-1], L01, rtol=0, atol=1e-13)
    Lt = orc.forward(v.T.copy(), e, ry, rx)
    assert np.allclose(Lt.T, L01, rtol=0, atol=1e-13)


def test_power_of_two_covariance_is_bit_exact(orc):
    v = _lum(orc, 16, 21, seed=30)
    rx, ry = orc.paper_radii(16, 21, 3)
    L = orc.forward(v, _edges(orc, v, 5), rx, ry, 0.1)
    for k in (-3, 2, 5):
        vs = (v * np.float32(2.0 ** k)).astype(np.float32)
        Ls = orc.forward(vs, _edges(orc, vs, 5), rx, ry, 0.1 * 4.0 ** k)
        assert np.array_equal(L, Ls)


# ------------------------------------------------------------- log-domain variance variant
@pytest.mark.parametrize("H,W,n,rx,ry,seed", [
    (5, 9, 3, [4, 2, 1], [2, 1, 0], 41),
    (8, 8, 5, [4, 2, 1], [4, 2, 1], 42),
    (6, 6, 64, [3, 1], [3, 1], 43),
])
def test_log_variance_matches_exact_brute_force(orc, H, W, n, rx, ry, seed):
    v = _lum(orc, H, W, seed=seed, lo=-3, hi=5)
    e = _edges(orc, v, n)
    L, Ls, Ws, var = orc.forward(v, e, rx, ry, per_scale=True, var_domain="log")
    Lb, Lsb, Wsb = brute.forward(v, n, rx, ry, per_scale=True, var_domain="log")
    assert np.max(np.abs(L - Lb)) <= 1e-12
    assert np.max(np.abs(Ls - Lsb)) <= 1e-15
    assert np.max(np.abs(Ws - Wsb)) <= 1e-12
    # the variant is a different method: the linear-domain weights differ
    _, _, Wlin, _ = orc.forward(v, e, rx, ry, per_scale=True)
    assert np.max(np.abs(Ws - Wlin)) > 1e-3


def test_log_variance_equals_numpy_window_variance(orc):
    # Eq. 10 of the log image, window by window with numpy (population variance)
    v = _lum(orc, 11, 14, seed=44, lo=-3, hi=5)
    rx, ry = [5, 2], [3, 1]
    _, _, _, var = orc.forward(v, _edges(orc, v, 5), rx, ry, per_scale=True, var_domain="log")
    lg = np.log(np.maximum(v.astype(np.float64), 2.0 ** -126))
    for j in range(2):
        for y in range(11):
            for x in range(14):
                win = lg[max(y - ry[j], 0):y + ry[j] + 1, max(x - rx[j], 0):x + rx[j] + 1]
                assert abs(var[j, y, x] - max(np.var(win), 0.0)) <= 1e-12


def test_log_variance_tables_equal_direct_windows(orc):
    v = _lum(orc, 29, 41, K=6, seed=45, lo=-3, hi=5)
    rx, ry = orc.paper_radii(29, 41, 5)
    e = _edges(orc, v, 5)
    L = orc.forward(v, e, rx, ry, var_domain="log")
    Ld = orc.forward_direct(v, e, rx, ry, np.arange(v.size), var_domain="log")
    assert np.max(np.abs(L.ravel() - Ld)) <= 1e-12


def test_log_variance_is_scale_invariant(orc):
    # scaling the luminance by 2^k moves the bin edges with it (the bins are unchanged)
    # and shifts every log value by k ln 2, which leaves every window variance unchanged:
    # the same eps gives the same L, while the linear variance needs eps * 4^k
    v = _lum(orc, 16, 21, seed=46, lo=-3, hi=5)
    rx, ry = orc.paper_radii(16, 21, 3)
    L = orc.forward(v, _edges(orc, v, 5), rx, ry, 0.1, var_domain="log")
    Llin = orc.forward(v, _edges(orc, v, 5), rx, ry, 0.1)
    for k in (-3, 4):
        vs = (v * np.float32(2.0 ** k)).astype(np.float32)
        e = _edges(orc, vs, 5)
        assert np.max(np.abs(orc.forward(vs, e, rx, ry, 0.1, var_domain="log") - L)) <= 1e-10
        assert np.max(np.abs(orc.forward(vs, e, rx, ry, 0.1) - Llin)) > 1e-3
    # a constant image has zero log variance: every L_j is min L_d
    c = np.full((7, 9), 0.37, dtype=np.float32)
    assert np.all(orc.forward(c, _edges(orc, c, 5), [3, 1], [3, 1], 0.1, 0.2, 0.9,
                              var_domain="log") == 0.2)


# ----------------------------------------------------------------------------- backward
def test_box_filter_is_self_adjoint(orc):
    rng = np.random.default_rng(4)
    a = rng.standard_normal((11, 14))
    b = rng.standard_normal((11, 14))
    for rx, ry in [(0, 0), (2, 1), (5, 3), (13, 20)]:
        lhs = np.dot(orc.box_filter(a, rx, ry).ravel(), b.ravel())
        rhs = np.dot(a.ravel(), orc.box_filter(b, rx, ry).ravel())
        assert abs(lhs - rhs) <= 1e-12 * (abs(lhs) + 1)
        # and it is the clamped window sum
        x, y = 3, 7
        want = a[max(y - ry, 0):y + ry + 1, max(x - rx, 0):x + rx + 1].sum()
        assert abs(orc.box_filter(a, rx, ry)[y, x] - want) <= 1e-12


def _safe_mask(v, edges, h):
    lv = np.log(v.astype(np.float64))
    safe = np.ones(v.shape, dtype=bool)
    for e in edges:
        safe &= np.abs(lv - np.log(float(e))) > 4 * h
    safe &= lv > np.log(float(v.min())) + 4 * h
    safe &= lv < np.log(float(v.max())) - 4 * h
    return safe


def test_backward_matches_central_differences(orc):
    H, W = 20, 26
    v = _lum(orc, H, W, K=5, seed=41)
    rx, ry = orc.paper_radii(H, W, 3)
    e = _edges(orc, v, 5)
    g = np.random.default_rng(7).standard_normal((H, W))
    dv, (geps, gmin, gmax) = orc.backward(v, e, rx, ry, g)
    h = 1e-3
    safe = _safe_mask(v, e, h)
    rng = np.random.default_rng(8)
    for _ in range(4):
        d = rng.standard_normal((H, W)) * safe
        vp = (v * np.exp(h * d)).astype(np.float32)
        vm = (v * np.exp(-h * d)).astype(np.float32)
        assert np.array_equal(orc.bins(vp, e), orc.bins(v, e))
        fp = np.sum(g * orc.forward(vp, e, rx, ry))
        fm = np.sum(g * orc.forward(vm, e, rx, ry))
        lin = np.sum(dv * (vp.astype(np.float64) - vm.astype(np.float64)))
        assert abs((fp - fm) - lin) <= 2e-4 * abs(fp - fm) + 1e-12
    # scalar gradients: L is affine in (min L_d, max L_d), so differences are exact
    L = orc.forward(v, e, rx, ry, 0.1, 0.0, 1.0)
    d_lo = np.sum(g * (orc.forward(v, e, rx, ry, 0.1, 0.5, 1.0) - L)) / 0.5
    d_hi = np.sum(g * (orc.forward(v, e, rx, ry, 0.1, 0.0, 2.0) - L)) / 1.0
    assert abs(d_lo - gmin) <= 1e-10 * (1 + abs(gmin))
    assert abs(d_hi - gmax) <= 1e-10 * (1 + abs(gmax))
    he = 1e-5
    d_eps = (np.sum(g * orc.forward(v, e, rx, ry, 0.1 + he))
             - np.sum(g * orc.forward(v, e, rx, ry, 0.1 - he))) / (2 * he)
    assert abs(d_eps - geps) <= 1e-6 * (1 + abs(geps))


def test_log_backward_matches_central_differences(orc):
    # the log-domain variant's gradient against central differences of its own forward
    H, W = 18, 23
    v = _lum(orc, H, W, K=5, seed=43)
    rx, ry = orc.paper_radii(H, W, 3)
    e = _edges(orc, v, 5)
    g = np.random.default_rng(9).standard_normal((H, W))
    dv, (geps, gmin, gmax) = orc.backward(v, e, rx, ry, g, var_domain="log")
    h = 1e-3
    safe = _safe_mask(v, e, h)
    rng = np.random.default_rng(10)
    for _ in range(4):
        d = rng.standard_normal((H, W)) * safe
        vp = (v * np.exp(h * d)).astype(np.float32)
        vm = (v * np.exp(-h * d)).astype(np.float32)
        assert np.array_equal(orc.bins(vp, e), orc.bins(v, e))
        fp = np.sum(g * orc.forward(vp, e, rx, ry, var_domain="log"))
        fm = np.sum(g * orc.forward(vm, e, rx, ry, var_domain="log"))
        lin = np.sum(dv * (vp.astype(np.float64) - vm.astype(np.float64)))
        assert abs((fp - fm) - lin) <= 2e-4 * abs(fp - fm) + 1e-12
    L = orc.forward(v, e, rx, ry, 0.1, 0.0, 1.0, var_domain="log")
    d_lo = np.sum(g * (orc.forward(v, e, rx, ry, 0.1, 0.5, 1.0, var_domain="log") - L)) / 0.5
    d_hi = np.sum(g * (orc.forward(v, e, rx, ry, 0.1, 0.0, 2.0, var_domain="log") - L)) / 1.0
    assert abs(d_lo - gmin) <= 1e-10 * (1 + abs(gmin))
    assert abs(d_hi - gmax) <= 1e-10 * (1 + abs(gmax))
    he = 1e-5
    d_eps = (np.sum(g * orc.forward(v, e, rx, ry, 0.1 + he, var_domain="log"))
             - np.sum(g * orc.forward(v, e, rx, ry, 0.1 - he, var_domain="log"))) / (2 * he)
    assert abs(d_eps - geps) <= 1e-6 * (1 + abs(geps))


def test_log_backward_follows_the_scale_law(orc):
    # scaling v and the edges by 2^k leaves the log-domain L unchanged (the log values shift
    # by k ln 2), so dL/dv at 2^k v is 2^-k times dL/dv at v; the scalar gradients are equal
    H, W = 15, 19
    v = _lum(orc, H, W, K=4, seed=47)
    rx, ry = orc.paper_radii(H, W, 3)
    e = _edges(orc, v, 5)
    g = np.random.default_rng(11).standard_normal((H, W))
    dv, gp = orc.backward(v, e, rx, ry, g, var_domain="log")
    scale = float(np.abs(dv).max())
    for k in (-3, 2, 5):
        f = np.float32(2.0 ** k)
        dvs, gps = orc.backward(v * f, e * f, rx, ry, g, var_domain="log")
        assert np.max(np.abs(dvs * float(f) - dv)) <= 1e-9 * scale
        for a, b in zip(gps, gp):
            assert abs(a - b) <= 1e-9 * (1 + abs(b))


def test_log_backward_is_zero_where_the_floor_is_taken(orc):
    # below the smallest normal FP32 the log plane is the constant ln(FLT_MIN)
    H, W = 9, 11
    v = _lum(orc, H, W, K=3, seed=53)
    v[2, 3] = 0.0
    v[5, 7] = np.float32(2.0 ** -140)
    rx, ry = [3, 1], [2, 1]
    e = _edges(orc, v[v > 2.0 ** -126], 4)
    g = np.random.default_rng(12).standard_normal((H, W))
    dv, _ = orc.backward(v, e, rx, ry, g, var_domain="log")
    assert dv[2, 3] == 0.0 and dv[5, 7] == 0.0
    # the same pixels just above the floor do carry a gradient
    v2 = v.copy()
    v2[2, 3] = np.float32(2.0 ** -120)
    v2[5, 7] = np.float32(2.0 ** -110)
    dv2, _ = orc.backward(v2, e, rx, ry, g, var_domain="log")
    assert dv2[2, 3] != 0.0 and dv2[5, 7] != 0.0


# ---------------------------------------------------------------- Eq. 12 colour restoration
def _color_case(seed=3, H=7, W=9):
    import oracle
    rng = np.random.default_rng(seed)
    rgb = rng.uniform(0.0, 3.0, (3, H, W)).astype(np.float32)
    rgb[:, 0, 0] = 0.0                       # black pixel: v = 0, ratio taken as 1
    rgb[:, 1, 1] = (2.0, -0.01, 1.0)         # a negative channel counts as 0
    lum = oracle.luminance(rgb)
    L = rng.uniform(0.0, 1.0, (H, W))
    return rgb, lum, L


def test_color_sat_one_is_the_plain_ratio(orc):
    oracle = orc
    # sat = 1: each channel is scaled by L / v
    rgb, lum, L = _color_case()
    out = oracle.color_restore(rgb, lum, L, 1.0)
    c = np.maximum(rgb.astype(np.float64), 0.0)
    v = lum.astype(np.float64)
    want = np.where(v > 0, c / np.where(v > 0, v, 1.0), 1.0) * L
    assert np.allclose(out, want, rtol=1e-15, atol=0)


def test_color_sat_zero_is_grey(orc):
    oracle = orc
    rgb, lum, L = _color_case()
    out = oracle.color_restore(rgb, lum, L, 0.0)
    assert np.array_equal(out, np.broadcast_to(L, out.shape))


def test_color_channel_ratios_and_exponent_law(orc):
    oracle = orc
    rgb, lum, L = _color_case(seed=8)
    a, b = 0.35, 0.25
    oa = oracle.color_restore(rgb, lum, L, a)
    ob = oracle.color_restore(rgb, lum, L, b)
    oab = oracle.color_restore(rgb, lum, L, a + b)
    ok = (lum > 0) & (L > 0)
    # (c/v)^(a+b) L = (c/v)^a L (c/v)^b L / L
    assert np.allclose(oab[:, ok], (oa * ob)[:, ok] / L[ok], rtol=1e-13)
    # channel ratios are the input ratios raised to sat (where both channels are positive)
    c = rgb.astype(np.float64)
    pos = ok & (c[0] > 0) & (c[2] > 0)
    assert np.allclose(oa[0, pos] / oa[2, pos], (c[0, pos] / c[2, pos]) ** a, rtol=1e-13)
    # the black pixel is neutral and the negative channel is zero
    assert np.all(oa[:, 0, 0] == L[0, 0]) and oa[1, 1, 1] == 0.0


def test_paper_radii_reproduce_the_paper_pyramid_example():
    import oracle
    # Section II-C: on a 2048 x 2048 image with five fields, the largest field is the image
    # and the smallest is 128 x 128.  With r_j = floor(dim / 2^j) the smallest window spans
    # 2 r_5 + 1 = 129 pixels (r_5 = 64) -- the paper's 128 up to the centre pixel -- and the
    # largest (r_1 = 1024) covers the whole image from every pixel once clamped.
    rx, ry = oracle.paper_radii(2048, 2048, 5)
    assert rx == ry == [1024, 512, 256, 128, 64]
    assert 2 * rx[-1] + 1 == 129
    assert all(2 * a == b for a, b in zip(rx[1:], rx[:-1]))      # each field half the last
    assert 2 * rx[0] + 1 >= 2048


def test_oracle_results_do_not_depend_on_thread_count():
    import oracle
    lum = oracle.luminance(gen_wdr(45, 67, 5, -2.0, 4.0, 3).rgb)
    e = oracle.exact_edges(lum.min(), lum.max(), 5)
    rx, ry = oracle.paper_radii(45, 67, 4)
    g = np.random.default_rng(0).standard_normal(lum.shape)
    try:
        oracle.set_threads(1)
        a = oracle.forward(lum, e, rx, ry, 0.1, per_scale=True)
        da, ga = oracle.backward(lum, e, rx, ry, g, 0.1)
        oracle.set_threads(4)
        b = oracle.forward(lum, e, rx, ry, 0.1, per_scale=True)
        db, gb = oracle.backward(lum, e, rx, ry, g, 0.1)
    finally:
        oracle.set_threads(1)
    for x, y in zip(a, b):
        assert np.array_equal(x, y)
    assert np.array_equal(da, db) and ga == gb
