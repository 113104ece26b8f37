"""GPU parity of every stage against the CPU oracle (on the same seeded inputs):
bit-exact luminance, bin edges and integral histograms; integral images and the fused
forward within the bounds derived in tests/_bounds.py."""
import numpy as np
import pytest
import torch

import oracle
import paper_2102_01289_amd as tm
from _bounds import entry_bound, forward_bound, tiling, window_sums
from _cases import edges_ref, fill_garbage, hist_ref, lum_ref, rgb_case, to_dev

pytestmark = pytest.mark.gpu

SHAPES = [(256, 256), (37, 123), (1, 1), (1, 300), (300, 1), (65, 257), (130, 1030)]


def _lum_dev(H, W, seed=0, K=6, lo=-2.0, hi=4.0):
    rgb = rgb_case(H, W, K, lo, hi, seed)
    return rgb, lum_ref(rgb)


# --------------------------------------------------------------------------- a1
@pytest.mark.parametrize("H,W", SHAPES)
def test_luminance_bit_exact(H, W):
    rgb, ref = _lum_dev(H, W, seed=H * 7 + W)
    got = tm.tm_luminance(to_dev(rgb)).cpu().numpy()
    assert np.array_equal(got.view(np.uint32), ref.view(np.uint32))


@pytest.mark.parametrize("H,W", [(256, 256), (37, 123), (1, 1), (130, 1030)])
@pytest.mark.parametrize("n", [1, 2, 5, 64, 256])
def test_prologue_edges_bit_exact(H, W, n):
    rgb, ref = _lum_dev(H, W, seed=n + H)
    lum, edges, offsets, minmax = tm.tm_prologue(to_dev(rgb), n)
    torch.cuda.synchronize()
    assert np.array_equal(lum.cpu().numpy().view(np.uint32), ref.view(np.uint32))
    assert np.array_equal(edges.cpu().numpy(), edges_ref(ref, n))
    assert minmax.cpu().numpy().tolist() == [float(ref.min()), float(ref.max())]
    v = ref.astype(np.float64)
    want = np.float32([v.mean(), (v * v).mean()])
    assert np.allclose(offsets.cpu().numpy(), want, rtol=2e-7, atol=0)
    # the stats-only entry point agrees with the fused one
    e2, o2, m2 = tm.tm_image_stats(lum, n)
    assert torch.equal(e2, edges) and torch.equal(o2, offsets) and torch.equal(m2, minmax)


@pytest.mark.parametrize("n,top", [(5, 32.0), (8, 256.0), (3, 27.0), (2, 4.0)])
def test_edges_on_exact_powers(n, top):
    # i_min = 1 and i_max = top: some edges are exact FP32 values, which forces the exact
    # big-integer tie-break on the device
    rng = np.random.default_rng(n)
    lum = rng.uniform(1.0, top, size=(33, 47)).astype(np.float32)
    lum[3, 4], lum[20, 30] = 1.0, top
    edges, _, _ = tm.tm_image_stats(to_dev(lum), n)
    assert np.array_equal(edges.cpu().numpy(), edges_ref(lum, n))


def test_edges_degenerate_image():
    lum = np.full((9, 70), 2.5, dtype=np.float32)
    edges, _, _ = tm.tm_image_stats(to_dev(lum), 5)
    assert np.all(np.isinf(edges.cpu().numpy()))


# --------------------------------------------------------------------------- a3
TUNES = [None, (2, 1, 2), (8, 3, 8), (4, 16, 4), (2, 64, 8)]
# every shape with the default tiling; the explicit tilings are swept on three shapes
SHAPE_TUNES = [(H, W, 0) for H, W in SHAPES] + [
    (H, W, ti) for H, W in [(256, 256), (37, 123), (65, 257)] for ti in range(1, len(TUNES))]


@pytest.mark.parametrize("H,W,ti", SHAPE_TUNES)
@pytest.mark.parametrize("n", [2, 5, 64])
@pytest.mark.parametrize("layout", ["cumulative", "per_bin"])
def test_integral_histogram_bit_exact(H, W, n, layout, ti):
    _, ref = _lum_dev(H, W, seed=3 * n + W)
    v = to_dev(ref)
    edges = to_dev(edges_ref(ref, n))
    planes = n if layout == "per_bin" else n - 1
    hist = tm.Table(H, W, "u32", planes)
    fill_garbage(hist)
    t = tm.tune(*TUNES[ti]) if TUNES[ti] else None
    tm.tm_integral_tables(v, None, None, edges, n, layout, tune=t, hist=hist)
    got = hist.padded()[..., 0].numpy().astype(np.uint64)
    want = hist_ref(ref, edges_ref(ref, n), n, layout)
    assert np.array_equal(got, want)


# --------------------------------------------------------------------------- a2
@pytest.mark.parametrize("prec", ["f32", "c32x2", "f64"])
@pytest.mark.parametrize("H,W,ti", SHAPE_TUNES)
def test_integral_image_within_bound(prec, H, W, ti):
    _, ref = _lum_dev(H, W, seed=11 + W, lo=-3.0, hi=5.0)
    v = to_dev(ref)
    vd = ref.astype(np.float64)
    mu = np.float32([vd.mean(), (vd * vd).mean()]) if prec == "c32x2" else np.float32([0, 0])
    offs = to_dev(mu)
    sat = tm.Table(H, W, prec)
    fill_garbage(sat)
    t = tm.tune(*TUNES[ti]) if TUNES[ti] else None
    tm.tm_integral_tables(v, prec, offs, None, 1, None, tune=t, sat=sat)
    got = sat.padded()[0].numpy().astype(np.float64)
    hi1, lo1 = oracle.integral_image(ref, False)
    hi2, lo2 = oracle.integral_image(ref, True)
    yy, xx = np.mgrid[0:H + 1, 0:W + 1]
    cnt = (yy * xx).astype(np.float64)
    if prec == "c32x2":
        g1 = got[..., 0] + got[..., 1] + cnt * float(mu[0])
        g2 = got[..., 2] + got[..., 3] + cnt * float(mu[1])
    else:
        g1, g2 = got[..., 0], got[..., 1]
    vec, th = (TUNES[ti][0], TUNES[ti][1]) if TUNES[ti] else tiling(H, W)
    b1, b2 = entry_bound(ref, prec, vec, th, float(mu[0]), float(mu[1]))
    # the reconstruction above rounds once more in FP64
    b1 = b1 + 4 * 2.0 ** -53 * (np.abs(hi1) + cnt * abs(float(mu[0])))
    b2 = b2 + 4 * 2.0 ** -53 * (np.abs(hi2) + cnt * abs(float(mu[1])))
    assert np.all(np.abs(g1 - (hi1 + lo1)) <= b1)
    assert np.all(np.abs(g2 - (hi2 + lo2)) <= b2)
    assert np.all(got[0] == 0) and np.all(got[:, 0] == 0)


@pytest.mark.parametrize("prec", ["f32", "f64"])
def test_integral_image_exact_on_integers(prec):
    # integer pixels with every quadrant sum below 2^24: each variant is exact
    rng = np.random.default_rng(1)
    lum = rng.integers(1, 16, size=(200, 300)).astype(np.float32)
    sat = tm.tm_integral_image(to_dev(lum), prec)
    got = sat.padded()[0].numpy().astype(np.float64)
    hi1, lo1 = oracle.integral_image(lum, False)
    hi2, lo2 = oracle.integral_image(lum, True)
    assert np.array_equal(got[..., 0], hi1) and np.array_equal(got[..., 1], hi2)


# --------------------------------------------------------------------------- a4
def _run_forward(rgb, params, prec, tune=None):
    H, W = rgb.shape[1:]
    m = tm.ToneMapper(H, W, params, prec, tune=tune)
    out = m.run(to_dev(rgb))
    torch.cuda.synchronize()
    return m, out.cpu().numpy().astype(np.float64)


def _check_forward(rgb, n, s, rx, ry, eps, prec, ld=(0.0, 1.0), tune=None):
    H, W = rgb.shape[1:]
    p = tm.make_params(n, s, rx, ry, eps, ld[0], ld[1])
    m, L = _run_forward(rgb, p, prec, tune)
    lum = lum_ref(rgb)
    e = edges_ref(lum, n)
    assert np.array_equal(m.lum.cpu().numpy().view(np.uint32), lum.view(np.uint32))
    assert np.array_equal(m.edges.cpu().numpy()[:n - 1], e)
    Lref, Lj, Wj, varj = oracle.forward(lum, e, rx, ry, eps, ld[0], ld[1], per_scale=True)
    vd = lum.astype(np.float64)
    mu = (float(np.float32(vd.mean())), float(np.float32((vd * vd).mean())))
    vec, th = (tune.tile_w_vec, tune.tile_h) if tune is not None else tiling(H, W, n_bins=n)
    bound = forward_bound(lum, Lref, Lj, Wj, varj, window_sums(lum, rx, ry), rx, ry, eps,
                          prec, vec, th, *(mu if prec == "c32x2" else (0.0, 0.0)))
    bound *= (ld[1] - ld[0])
    err = np.abs(L - Lref)
    worst = np.unravel_index(np.argmax(err - bound), err.shape)
    assert np.all(err <= bound), (f"max err {err.max():.3e}; worst excess at {worst}: "
                                  f"err {err[worst]:.3e} bound {bound[worst]:.3e}")
    return L, Lref, err


@pytest.mark.parametrize("prec", ["c32x2", "f64", "f32"])
def test_forward_paper_set_256(prec):
    rgb = rgb_case(256, 256, 8, -2.0, 4.0, seed=101)
    rx, ry = oracle.paper_radii(256, 256, 5)
    L, Lref, err = _check_forward(rgb, 5, 5, rx, ry, 0.1, prec)
    if prec != "f32":
        assert err.max() <= 1e-4 and np.quantile(err, 0.999) <= 1e-5


@pytest.mark.parametrize("H,W,n,rx,ry", [
    (37, 123, 5, [61, 30, 15], [18, 9, 4]),
    (65, 257, 3, [0, 3, 100], [0, 7, 100]),
    (1, 300, 5, [150, 10], [0, 0]),
    (300, 1, 4, [0, 0], [150, 10]),
    (1, 1, 5, [0], [0]),
    (130, 1030, 64, [4, 16, 64], [4, 16, 64]),
    (96, 200, 256, [50, 25, 12, 6, 3, 1, 0, 2], [48, 24, 12, 6, 3, 1, 0, 2]),
])
@pytest.mark.parametrize("prec", ["c32x2", "f64"])
def test_forward_ragged_and_parameters(H, W, n, rx, ry, prec):
    rgb = rgb_case(H, W, 5, -2.0, 4.0, seed=H + 3 * W + n)
    _check_forward(rgb, n, len(rx), rx, ry, 0.1, prec, ld=(0.1, 0.9))


def test_forward_tunes_agree():
    rgb = rgb_case(130, 700, 6, -2.0, 4.0, seed=9)
    rx, ry = oracle.paper_radii(130, 700, 5)
    for t in [(2, 1, 2), (8, 3, 8), (4, 64, 4)]:
        _check_forward(rgb, 5, 5, rx, ry, 0.1, "c32x2", tune=tm.tune(*t))


def test_forward_special_cases():
    H, W = 70, 90
    rgb = rgb_case(H, W, 5, seed=4)
    rx, ry = oracle.paper_radii(H, W, 4)
    # one bin: every L_j is min L_d
    _, L = _run_forward(rgb, tm.make_params(1, 4, rx, ry, 0.1, 0.25, 0.75), "c32x2")
    assert np.all(L == np.float32(0.25))
    # constant image
    c = np.full((3, H, W), 2.0, dtype=np.float32)
    _, L = _run_forward(c, tm.make_params(5, 4, rx, ry, 0.1, 0.2, 0.9), "c32x2")
    assert np.all(L == np.float32(0.2))
    # one field covering the image: global histogram equalisation, closed form
    lum = lum_ref(rgb)
    e = edges_ref(lum, 5)
    b = oracle.bins(lum, e)
    below = np.concatenate([[0], np.cumsum(np.bincount(b.ravel(), minlength=5))[:-1]])
    _, L = _run_forward(rgb, tm.make_params(5, 1, [W], [H], 0.1), "c32x2")
    assert np.max(np.abs(L - below[b] / (H * W))) <= 2 ** -23


@pytest.mark.parametrize("prec", ["f32", "c32x2", "f64"])
def test_forward_power_of_two_covariance_bit_exact(prec):
    H, W = 90, 130
    rgb = rgb_case(H, W, 5, seed=12)
    rx, ry = oracle.paper_radii(H, W, 4)
    _, L = _run_forward(rgb, tm.make_params(5, 4, rx, ry, 0.1), prec)
    for k in (-2, 3):
        _, Ls = _run_forward((rgb * np.float32(2.0 ** k)).astype(np.float32),
                             tm.make_params(5, 4, rx, ry, 0.1 * 4.0 ** k), prec)
        assert np.array_equal(L, Ls)


def test_forward_is_deterministic():
    rgb = rgb_case(256, 384, 6, seed=77)
    p = tm.make_params(5, 5, eps=0.1, H=256, W=384)
    _, a = _run_forward(rgb, p, "c32x2")
    _, b = _run_forward(rgb, p, "c32x2")
    assert np.array_equal(a, b)


def test_mirror_equivariance():
    H, W = 64, 96
    rgb = rgb_case(H, W, 5, seed=31)
    p = tm.make_params(5, 4, eps=0.1, H=H, W=W)
    _, L = _run_forward(rgb, p, "f64")
    _, Lf = _run_forward(rgb[:, :, ::-1].copy(), p, "f64")
    assert np.max(np.abs(Lf[:, ::-1] - L)) <= 1e-5


@pytest.mark.parametrize("prec", ["c32x2", "f64"])
@pytest.mark.parametrize("H,W", [(256, 256), (37, 123), (1, 300)])
def test_per_field_maps(prec, H, W):
    # Fig. 3: the per-field tone values L_j (Eq. 2) and weights W_j (Eq. 4)
    rgb = rgb_case(H, W, 8, -2.0, 4.0, seed=H + W)
    lum = lum_ref(rgb)
    e = edges_ref(lum, 5)
    rx, ry = oracle.paper_radii(H, W, 5)
    p = tm.make_params(5, 5, eps=0.1, H=H, W=W)
    m = tm.ToneMapper(H, W, p, prec)
    L_plain = m.run(to_dev(rgb)).clone()
    L, maps = m.query_maps()
    torch.cuda.synchronize()
    assert torch.equal(L, L_plain)                    # the maps change no output bit
    Lref, Lj, Wj, varj = oracle.forward(lum, e, rx, ry, 0.1, per_scale=True)
    mp = maps.cpu().numpy().astype(np.float64)
    # tone values: exact counts over the exact area, one FP32 division and one FMA
    assert np.max(np.abs(mp[:5] - Lj)) <= 2e-7
    # weights: W_j = var/(var + eps) moves by eps/(var + eps)^2 times the variance error
    assert np.max(np.abs(mp[5:] - Wj)) <= 1e-4
    assert np.all((mp[5:] >= 0) & (mp[5:] <= 1))
