"""GPU parity of the log-domain variance variant (Eq. 10's window variance taken of the log
image l = ln i rather than of i, the bins still cut from i) against the oracle's FP64 form:
the device log plane within 2 ulp of the exact logarithm, histograms bit-exact, the fused
output within the derived per-pixel bound and a stated envelope, and its gradient (the
residual backward given l, then the chain rule through the logarithm) within the derived
backward bound."""
import numpy as np
import pytest
import torch

import oracle
import paper_2102_01289_amd as tm
from _bounds import backward_bound, forward_bound, tiling, window_sums
from _cases import (check_scalar_gradients, edges_ref, fill_garbage, lum_ref, rgb_case,
                    to_dev)
from synth import WORKLOADS, gen_wdr

pytestmark = pytest.mark.gpu

FLT_MIN = float(np.finfo(np.float32).tiny)


def _ulp32(x):
    return np.spacing(np.abs(x).astype(np.float32)).astype(np.float64)


def _log_ref(lum):
    return np.log(np.maximum(lum.astype(np.float64), FLT_MIN))


@pytest.mark.parametrize("H,W", [(1, 1), (37, 123), (256, 256), (130, 1030)])
def test_log_luminance_plane_and_offsets(H, W):
    lum = lum_ref(rgb_case(H, W, 5, -3.0, 5.0, seed=H + W))
    lum.flat[0] = 0.0                 # floored at FLT_MIN
    if lum.size > 2:
        lum.flat[1] = 1.0             # ln 1 = 0 exactly
        lum.flat[2] = np.float32(1e-40)   # a subnormal, also floored
    logv, off, mm = tm.tm_log_luminance(to_dev(lum))
    torch.cuda.synchronize()
    got = logv.cpu().numpy().astype(np.float64)
    ref = _log_ref(lum)
    assert np.all(np.abs(got - ref) <= 2 * _ulp32(ref))
    if lum.size > 2:
        assert got.flat[1] == 0.0 and got.flat[0] == got.flat[2] == np.float32(np.log(FLT_MIN))
    # the offsets and range are those of the plane the call wrote (FP64 sums, FP32 result)
    want = np.float32([got.mean(), (got * got).mean()])
    assert np.allclose(off.cpu().numpy(), want, rtol=2e-7, atol=1e-7)
    assert mm.cpu().numpy().tolist() == [float(got.min()), float(got.max())]
    # without the plane: the same statistics, bit for bit
    none, off2, mm2 = tm.tm_log_luminance(to_dev(lum), write_plane=False)
    torch.cuda.synchronize()
    assert none is None and torch.equal(off2, off) and torch.equal(mm2, mm)


def _check_log_forward(rgb, n, rx, ry, eps, prec, ld=(0.0, 1.0)):
    H, W = rgb.shape[1:]
    p = tm.make_params(n, len(rx), rx, ry, eps, ld[0], ld[1])
    m = tm.ToneMapper(H, W, p, prec, variance="log")
    L = m.run(to_dev(rgb)).cpu().numpy().astype(np.float64)
    lum = lum_ref(rgb)
    e = edges_ref(lum, n)
    assert np.array_equal(m.edges.cpu().numpy()[:n - 1], e)
    if n > 1:
        G = m.hist.padded()[..., 0].numpy().astype(np.uint64)
        assert np.array_equal(G, oracle.integral_histogram(oracle.bins(lum, e), n,
                                                           cumulative=True))
    Lref, Lj, Wj, varj = oracle.forward(lum, e, rx, ry, eps, ld[0], ld[1], per_scale=True,
                                        var_domain="log")
    lg = _log_ref(lum)
    mu = (float(np.float32(lg.mean())), float(np.float32((lg * lg).mean())))
    dl = 2 * _ulp32(lg)
    vec, th = tiling(H, W)
    bound = forward_bound(lg, Lref, Lj, Wj, varj, window_sums(lg, rx, ry), rx, ry, eps, prec,
                          vec, th, *(mu if prec == "c32x2" else (0.0, 0.0)),
                          input_err=(dl, 2 * np.abs(lg) * dl + dl * dl))
    bound *= (ld[1] - ld[0])
    err = np.abs(L - Lref)
    worst = np.unravel_index(np.argmax(err - bound), err.shape)
    assert np.all(err <= bound), (f"max err {err.max():.3e}; worst excess at {worst}: "
                                  f"err {err[worst]:.3e} bound {bound[worst]:.3e}")
    # the variant differs from the linear-variance method
    Llin = oracle.forward(lum, e, rx, ry, eps, ld[0], ld[1])
    assert np.max(np.abs(Llin - Lref)) > 1e-3
    return err


@pytest.mark.parametrize("prec", ["c32x2", "f64"])
def test_log_forward_paper_set_256(prec):
    rgb = rgb_case(256, 256, 8, -2.0, 4.0, seed=101)
    rx, ry = oracle.paper_radii(256, 256, 5)
    err = _check_log_forward(rgb, 5, rx, ry, 0.1, prec)
    assert err.max() <= 1e-5 and np.quantile(err, 0.999) <= 2e-6


@pytest.mark.parametrize("H,W,n,rx,ry", [
    (37, 123, 5, [61, 30, 15], [18, 9, 4]),
    (65, 257, 3, [0, 3, 100], [0, 7, 100]),
    (1, 300, 5, [150, 10], [0, 0]),
    (130, 1030, 64, [4, 16, 64], [4, 16, 64]),
])
@pytest.mark.parametrize("prec", ["c32x2", "f64"])
def test_log_forward_ragged_and_parameters(H, W, n, rx, ry, prec):
    rgb = rgb_case(H, W, 5, -3.0, 5.0, seed=2 * H + W + n)
    _check_log_forward(rgb, n, rx, ry, 0.1, prec, ld=(0.1, 0.9))


def test_log_forward_1920x1080():
    c = WORKLOADS["wdr_1920x1080"]
    rgb = gen_wdr(c["H"], c["W"], c["K"], c["lo"], c["hi"], c["seed"]).rgb
    rx, ry = oracle.paper_radii(c["H"], c["W"], 5)
    err = _check_log_forward(rgb, 5, rx, ry, 0.1, "c32x2")
    assert err.max() <= 1e-5 and np.quantile(err, 0.999) <= 2e-6


def test_log_forward_special_cases():
    H, W = 48, 80
    rx, ry = oracle.paper_radii(H, W, 4)
    # constant image: zero log variance everywhere, every L_j = min L_d
    c = np.full((3, H, W), 0.37, dtype=np.float32)
    m = tm.ToneMapper(H, W, tm.make_params(5, 4, rx, ry, 0.1, 0.2, 0.9), "c32x2",
                      variance="log")
    assert np.all(m.run(to_dev(c)).cpu().numpy() == np.float32(0.2))
    # scaling by 2^k keeps the bins and shifts l by k ln 2: L changes by rounding only
    rgb = rgb_case(H, W, 5, -3.0, 5.0, seed=17)
    p = tm.make_params(5, 4, rx, ry, 0.1)
    a = tm.ToneMapper(H, W, p, "c32x2", variance="log").run(to_dev(rgb)).cpu().numpy()
    b = tm.ToneMapper(H, W, p, "c32x2", variance="log").run(
        to_dev((rgb * np.float32(8.0)).astype(np.float32))).cpu().numpy()
    assert np.max(np.abs(a.astype(np.float64) - b)) <= 1e-5
    # the table-based backward of the variant equals the residual one bit for bit
    m = tm.ToneMapper(H, W, p, "c32x2", variance="log")
    g = to_dev(np.random.default_rng(4).standard_normal((H, W)).astype(np.float32))
    m.run_train(to_dev(rgb))
    gr, pr = (t.clone() for t in m.backward_resid(g))
    gt, pt = (t.clone() for t in m.backward(g))
    gf, pf = tm.tm_tonemap_backward_log(m.lum, m.sat, m.hist, m.edges, p, g, m.log_offsets)
    torch.cuda.synchronize()
    assert torch.equal(gt, gr) and torch.equal(pt, pr)
    assert torch.equal(gf, gr) and torch.equal(pf, pr)


def test_log_variance_maps_and_colour():
    # the per-field maps (Fig. 3) and the colour stage (Eq. 12) run on the log-variance
    # tables too: same L as the plain query, weights of the log variance
    H, W = 120, 200
    rgb = rgb_case(H, W, 6, -3.0, 5.0, seed=23)
    lum = lum_ref(rgb)
    e = edges_ref(lum, 5)
    rx, ry = oracle.paper_radii(H, W, 5)
    p = tm.make_params(5, 5, eps=0.1, H=H, W=W)
    m = tm.ToneMapper(H, W, p, "c32x2", variance="log")
    L_plain = m.run(to_dev(rgb)).clone()
    L, maps = m.query_maps()
    torch.cuda.synchronize()
    assert torch.equal(L, L_plain)
    _, Lj, Wj, _ = oracle.forward(lum, e, rx, ry, 0.1, per_scale=True, var_domain="log")
    mp = maps.cpu().numpy().astype(np.float64)
    assert np.max(np.abs(mp[:5] - Lj)) <= 2e-7
    # log variances are well conditioned: the FP32 log plane's rounding dominates
    assert np.max(np.abs(mp[5:] - Wj)) <= 1e-5
    out = m.query_rgb(to_dev(rgb), 0.6)
    torch.cuda.synchronize()
    assert torch.equal(m.out, L_plain)
    # against the oracle chain, with the log-variance forward bound carried through Eq. 12
    Lref, Lj2, Wj2, varj2 = oracle.forward(lum, e, rx, ry, 0.1, per_scale=True,
                                           var_domain="log")
    lg = _log_ref(lum)
    mu = (float(np.float32(lg.mean())), float(np.float32((lg * lg).mean())))
    dl = 2 * _ulp32(lg)
    vec, th = tiling(H, W)
    Lb = forward_bound(lg, Lref, Lj2, Wj2, varj2, window_sums(lg, rx, ry), rx, ry, 0.1, "c32x2",
                       vec, th, *mu, input_err=(dl, 2 * np.abs(lg) * dl + dl * dl))
    ref = oracle.color_restore(rgb, lum, Lref, 0.6)
    got = out.cpu().numpy().astype(np.float64)
    c = np.maximum(rgb.astype(np.float64), 0.0)
    lv = lum.astype(np.float64)
    ratio = np.where(lv > 0, c / np.where(lv > 0, lv, 1.0), 1.0) ** 0.6
    assert np.all(np.abs(got - ref) <= ratio * Lb[None] + 1e-6 * np.abs(ref) + 1e-30)


@pytest.mark.slow
def test_log_forward_4000x3000():
    # the 12 MP, 10^8:1 workload: whole image against the oracle's FP64 log-variance form
    c = WORKLOADS["wdr_4000x3000"]
    rgb = gen_wdr(c["H"], c["W"], c["K"], c["lo"], c["hi"], c["seed"]).rgb
    rx, ry = oracle.paper_radii(c["H"], c["W"], 5)
    err = _check_log_forward(rgb, 5, rx, ry, 0.1, "c32x2")
    assert err.max() <= 1e-5 and np.quantile(err, 0.999) <= 2e-6


# ------------------------------------------------------------------------ gradient
@pytest.mark.parametrize("H,W,n,layout", [(1, 1, 2, "cumulative"), (37, 123, 5, "cumulative"),
                                           (130, 1030, 9, "cumulative"), (256, 256, 5, "per_bin"),
                                           (61, 517, 3, "per_bin"), (1080, 1920, 5, "cumulative")])
@pytest.mark.parametrize("prec", ["c32x2", "f64"])
def test_split_tables_equal_the_two_single_builds(H, W, n, layout, prec):
    # one three-stage pass with the integral image of l and the histogram of i: bit-identical
    # to the separate builds, and the histogram exact against the oracle's (Eq. 7-8).  The
    # luminance plane has a pitch of W+3 (rows not 16-byte aligned) while l's rows are.
    lum = lum_ref(rgb_case(H, W, 5, -3.0, 5.0, seed=H * 7 + W))
    big = torch.zeros((H, W + 3), dtype=torch.float32, device="cuda")
    big[:, :W] = to_dev(lum)
    lum_d = big[:, :W]
    l, loff, _ = tm.tm_log_luminance(lum_d)
    e = edges_ref(lum, n)
    edges = to_dev(e)
    sat = tm.Table(H, W, prec, 1)
    hist = tm.Table(H, W, "u32", n if layout == "per_bin" else n - 1)
    fill_garbage(sat)
    fill_garbage(hist)         # the border zeros must be written too
    tm.tm_integral_tables_split(l, lum_d, prec, loff, edges, n, layout, sat=sat, hist=hist)
    sat1 = tm.tm_integral_image(l, prec, loff)
    hist1 = tm.tm_integral_histogram(lum_d, edges, n, layout)
    torch.cuda.synchronize()
    assert torch.equal(sat.raw_region(), sat1.raw_region())
    assert torch.equal(hist.raw_region(), hist1.raw_region())
    # and from lum alone, l formed as each pixel is read
    sat2 = tm.Table(H, W, prec, 1)
    hist2 = tm.Table(H, W, "u32", n if layout == "per_bin" else n - 1)
    fill_garbage(sat2)
    fill_garbage(hist2)
    tm.tm_integral_tables_log(lum_d, prec, loff, edges, n, layout, sat=sat2, hist=hist2)
    torch.cuda.synchronize()
    assert torch.equal(sat2.raw_region(), sat1.raw_region())
    assert torch.equal(hist2.raw_region(), hist1.raw_region())
    G = hist.padded()[..., 0]
    if H * W <= 256 * 256:
        want = oracle.integral_histogram(oracle.bins(lum, e), n,
                                         cumulative=layout == "cumulative")
        assert np.array_equal(G.numpy().astype(np.uint64), want)


@pytest.mark.parametrize("prec", ["f32", "c32x2", "f64"])
def test_log_tables_without_histogram(prec):
    # one bin: only the integral image of l (formed on load), equal to that of the log plane
    H, W = 45, 333
    lum = lum_ref(rgb_case(H, W, 5, -3.0, 5.0, seed=9))
    lum[3, :4] = [0.0, 1e-40, 1.1754944e-38, 7.0]
    d = to_dev(lum)
    l, loff, _ = tm.tm_log_luminance(d)
    sat, hist = tm.tm_integral_tables_log(d, prec, loff, None, 1, None)
    assert hist is None
    ref = tm.tm_integral_image(l, prec, loff)
    torch.cuda.synchronize()
    assert torch.equal(sat.raw_region(), ref.raw_region())


@pytest.mark.parametrize("t", [(2, 4, 4), (4, 16, 2), (8, 32, 8), (8, 8, 2)])
@pytest.mark.parametrize("prec", ["c32x2", "f64"])
def test_log_tables_every_tiling(t, prec):
    # every scan variant (columns per lane, tile height, planes per item) forms l on load
    # exactly as the log pass does: equal to the tables of the stored plane and of i
    H, W = 203, 1301
    lum = lum_ref(rgb_case(H, W, 5, -3.0, 5.0, seed=sum(t)))
    lum[5, :3] = [0.0, 1e-40, 1.1754944e-38]
    d = to_dev(lum)
    e = to_dev(edges_ref(lum, 9))
    l, loff, _ = tm.tm_log_luminance(d)
    tn = tm.tune(*t)
    sat, hist = tm.tm_integral_tables_log(d, prec, loff, e, 9, "cumulative", tune=tn)
    ref = tm.tm_integral_image(l, prec, loff, tune=tn)
    href = tm.tm_integral_histogram(d, e, 9, "cumulative", tune=tn)
    torch.cuda.synchronize()
    assert torch.equal(sat.raw_region(), ref.raw_region())
    assert torch.equal(hist.raw_region(), href.raw_region())


def test_split_tables_shape_mismatch_rejected():
    a = torch.zeros((8, 8), device="cuda")
    with pytest.raises(ValueError):
        tm.tm_integral_tables_split(a, torch.zeros((8, 9), device="cuda"), "f64", None,
                                    torch.zeros(4, device="cuda"), 5)


@pytest.mark.parametrize("H,W,n", [(1, 1, 1), (37, 123, 5), (130, 1030, 9), (1080, 1920, 5),
                                   (3000, 4000, 5)])
def test_log_prologue_equals_prologue_then_log_pass(H, W, n):
    # one pass over the colour planes gives the luminance, edges and range of tm_prologue and
    # the log plane and offsets of tm_log_luminance, bit for bit (black and subnormal pixels
    # included: they take the floor constant)
    rgb = rgb_case(H, W, 5, -3.0, 5.0, seed=H + 5 * W)
    rgb[:, 0, :min(W, 3)] = np.float32([0.0, 1e-40, 1.0])[:min(W, 3)]
    d = to_dev(rgb)
    lum, logv, edges, loff, mm = tm.tm_prologue_log(d, n)
    lum1, edges1, _, mm1 = tm.tm_prologue(d, n)
    logv1, loff1, _ = tm.tm_log_luminance(lum1)
    torch.cuda.synchronize()
    assert torch.equal(lum, lum1) and torch.equal(mm, mm1)
    assert torch.equal(edges, edges1)
    assert torch.equal(logv, logv1) and torch.equal(loff, loff1)
    # without the plane: the same offsets and luminance
    lum2, none, edges2, loff2, _ = tm.tm_prologue_log(d, n, write_log=False)
    torch.cuda.synchronize()
    assert none is None
    assert torch.equal(lum2, lum1) and torch.equal(edges2, edges1) and torch.equal(loff2, loff1)


@pytest.mark.parametrize("pad_lum,pad_log", [(3, 1), (0, 5), (2, 0)])
def test_log_prologue_with_pitched_planes(pad_lum, pad_log):
    # rows of the luminance and log planes that are not 16-byte aligned take the element
    # stores; the results equal the contiguous call's
    import ctypes
    from paper_2102_01289_amd import _capi
    H, W, n = 37, 517, 5
    d = to_dev(rgb_case(H, W, 5, -3.0, 5.0, seed=pad_lum * 7 + pad_log))
    lum, logv, edges, loff, mm = tm.tm_prologue_log(d, n)
    lb = torch.full((H, W + pad_lum), -7.0, device="cuda")
    gb = torch.full((H, W + pad_log), -7.0, device="cuda")
    e2 = torch.empty(n - 1, device="cuda")
    o2 = torch.empty(2, device="cuda")
    m2 = torch.empty(2, device="cuda")
    lib = _capi.load()
    ws = torch.empty(max(int(lib.tm_image_stats_workspace_bytes(H, W)), 1), dtype=torch.uint8,
                     device="cuda")
    vp = lambda t: ctypes.c_void_p(t.data_ptr())
    st = lib.tm_prologue_log(vp(d), d.stride(0), d.stride(1), H, W, n, vp(lb), lb.stride(0),
                             vp(gb), gb.stride(0), vp(e2), vp(o2), vp(m2), vp(ws), ws.numel(),
                             ctypes.c_void_p(torch.cuda.current_stream().cuda_stream))
    torch.cuda.synchronize()
    assert st == 0
    assert torch.equal(lb[:, :W], lum) and torch.equal(gb[:, :W], logv)
    assert torch.all(lb[:, W:] == -7.0) and torch.all(gb[:, W:] == -7.0)   # padding untouched
    assert torch.equal(e2, edges) and torch.equal(o2, loff) and torch.equal(m2, mm)


def test_tonemap_convenience_takes_the_variance():
    rgb = to_dev(rgb_case(40, 70, 5, -3.0, 5.0, seed=3))
    p = tm.make_params(5, 5, eps=0.1, H=40, W=70)
    want = tm.ToneMapper(40, 70, p, "c32x2", variance="log").run(rgb).clone()
    got = tm.tonemap(rgb, variance="log")
    torch.cuda.synchronize()
    assert torch.equal(got, want)
    assert not torch.equal(got, tm.tonemap(rgb))
    rgb_log = tm.tonemap_rgb(rgb, variance="log")
    want_rgb = tm.ToneMapper(40, 70, p, "c32x2", variance="log").run_rgb(rgb)
    torch.cuda.synchronize()
    assert torch.equal(rgb_log, want_rgb)
    assert not torch.equal(rgb_log, tm.tonemap_rgb(rgb))


def test_log_chain_rule_kernel():
    # grad_i = grad_l / i (one correctly rounded FP32 division) above the floor, 0 below;
    # in place too
    H, W = 37, 301
    lum = lum_ref(rgb_case(H, W, 5, -3.0, 5.0, seed=71))
    lum[0, :5] = [0.0, 1e-40, FLT_MIN, 2.0 * FLT_MIN, 1.0]
    gl = np.random.default_rng(3).standard_normal((H, W)).astype(np.float32)
    want = np.where(lum > FLT_MIN, gl / np.where(lum > FLT_MIN, lum, 1.0), 0.0).astype(np.float32)
    got = tm.tm_log_luminance_backward(to_dev(lum), to_dev(gl)).cpu().numpy()
    assert np.array_equal(got, want)
    t = to_dev(gl)
    tm.tm_log_luminance_backward(to_dev(lum), t, t)
    assert np.array_equal(t.cpu().numpy(), want)
    assert got[0, 0] == got[0, 1] == got[0, 2] == 0.0 and got[0, 3] != 0.0


def _check_log_backward(rgb, n, rx, ry, eps, prec, seed, ld=(0.0, 1.0)):
    H, W = rgb.shape[1:]
    p = tm.make_params(n, len(rx), rx, ry, eps, ld[0], ld[1])
    m = tm.ToneMapper(H, W, p, prec, variance="log")
    L_plain = m.run(to_dev(rgb)).clone()
    L_train = m.run_train(to_dev(rgb)).clone()
    assert torch.equal(L_plain, L_train)       # the training form writes the same L
    g = np.random.default_rng(seed).standard_normal((H, W)).astype(np.float32)
    gv, gp = m.backward_resid(to_dev(g))
    gv, gp = gv.clone(), gp.clone()
    # the fused chain rule equals the two-step form (residual backward given the log plane,
    # then the chain-rule pass) bit for bit
    gl, gp2 = tm.tm_tonemap_backward_resid(tm.tm_log_luminance(m.lum)[0], p, m.resid,
                                           to_dev(g))
    tm.tm_log_luminance_backward(m.lum, gl, gl)
    torch.cuda.synchronize()
    assert torch.equal(gv, gl) and torch.equal(gp, gp2)
    gv = gv.cpu().numpy().astype(np.float64)
    gp = gp.cpu().numpy()
    lum = lum_ref(rgb)
    e = edges_ref(lum, n)
    g64 = g.astype(np.float64)
    dv, gref = oracle.backward(lum, e, rx, ry, g64, eps, ld[0], ld[1], var_domain="log")
    fwd = oracle.forward(lum, e, rx, ry, eps, ld[0], ld[1], per_scale=True, var_domain="log")
    Lr, Lj, Wj, varj = fwd
    # the bound of the gradient with respect to l (the variance's image), with the device log
    # plane's rounding (2 ulp) as input error, then carried through the FP32 division by i
    lg = _log_ref(lum)
    i64 = lum.astype(np.float64)
    above = i64 > FLT_MIN
    dl_ref = np.where(above, dv * i64, 0.0)
    mu = (float(np.float32(lg.mean())), float(np.float32((lg * lg).mean())))
    d1 = 2 * _ulp32(lg)
    vec, th = tiling(H, W)
    B, bad = backward_bound(lg, g64, Lr, Lj, Wj, varj, window_sums(lg, rx, ry), rx, ry, eps,
                            prec, vec, th, *(mu if prec == "c32x2" else (0.0, 0.0)),
                            dv_ref=dl_ref, input_err=(d1, 2 * np.abs(lg) * d1 + d1 * d1))
    assert bad <= max(2, H * W // 1000), f"{bad} pixels with uncertain fusion weights"
    assert np.mean(np.isinf(B)) <= 0.05
    with np.errstate(invalid="ignore", divide="ignore"):
        Bv = np.where(above, B / np.where(above, i64, 1.0), 0.0)
        Bv = Bv + 2.0 ** -24 * (np.abs(dv) + Bv)
        over = np.where(above, np.abs(gv - dv) / Bv, 0.0)
    worst = np.unravel_index(int(np.argmax(over)), over.shape)
    assert np.all(over <= 1.0), (f"gradient outside the derived bound at {int(np.sum(over > 1))} "
                                 f"pixels; worst {worst}: gpu {gv[worst]:.6e} oracle "
                                 f"{dv[worst]:.6e} bound {Bv[worst]:.3e}")
    assert np.all(gv[~above] == 0.0)
    check_scalar_gradients(gp, gref, g64, fwd, eps, ld)
    # the variant's gradient differs from the linear-variance one
    dlin, _ = oracle.backward(lum, e, rx, ry, g64, eps, ld[0], ld[1])
    assert np.max(np.abs(dlin - dv)) > 1e-3 * np.max(np.abs(dv))
    return gv, dv


@pytest.mark.parametrize("prec", ["c32x2", "f64"])
@pytest.mark.parametrize("H,W,n,s", [(48, 64, 5, 3), (96, 128, 5, 5), (37, 123, 3, 4),
                                     (1, 200, 5, 2), (150, 1, 5, 2), (64, 64, 64, 3)])
def test_log_backward_matches_oracle(prec, H, W, n, s):
    rgb = rgb_case(H, W, 5, -3.0, 5.0, seed=3 * H + W + n)
    rx, ry = oracle.paper_radii(H, W, s)
    _check_log_backward(rgb, n, rx, ry, 0.1, prec, seed=s)


@pytest.mark.parametrize("rx,ry", [([0, 3, 100], [0, 7, 100]), ([5, 1], [0, 9]),
                                   ([30, 15, 8, 4, 2, 1, 0], [20, 10, 5, 2, 1, 0, 1])])
def test_log_backward_radii_clamping_and_floor(rx, ry):
    rgb = rgb_case(60, 80, 5, -3.0, 5.0, seed=len(rx) + 30)
    rgb[:, 7, 9] = 0.0                   # a black pixel: l is the floor, its gradient 0
    _check_log_backward(rgb, 5, rx, ry, 0.05, "c32x2", seed=5, ld=(0.2, 0.8))


@pytest.mark.parametrize("H,W,s", [(1, 1, 1), (3, 700, 2), (1080, 1920, 5), (3000, 4000, 5)])
def test_log_backward_fused_chain_rule_equals_the_two_steps(H, W, s):
    # ragged, tiny and full-size shapes (the adjoint tiling changes with the shape), pixels at
    # and around the floor: the fused pass equals residual backward given l + chain rule
    rgb = rgb_case(H, W, 5, -3.0, 5.0, seed=H + 3 * W)
    rgb[:, 0, :min(W, 6)] = np.float32([0.0, 1e-40, 1.1754944e-38, 2.4e-38, 1.0, 5.0])[:min(W, 6)]
    rx, ry = oracle.paper_radii(H, W, s)
    p = tm.make_params(5, s, rx, ry, 0.05)
    m = tm.ToneMapper(H, W, p, "c32x2", variance="log")
    m.run_train(to_dev(rgb))
    g = to_dev(np.random.default_rng(W).standard_normal((H, W)).astype(np.float32))
    gv, gp = (t.clone() for t in m.backward_resid(g))
    gl, gp2 = tm.tm_tonemap_backward_resid(tm.tm_log_luminance(m.lum)[0], p, m.resid, g)
    tm.tm_log_luminance_backward(m.lum, gl, gl)
    torch.cuda.synchronize()
    assert torch.equal(gv, gl) and torch.equal(gp, gp2)
    assert torch.all(gv[m.lum <= FLT_MIN] == 0)


def test_log_backward_paper_set_256():
    rgb = rgb_case(256, 256, 8, -2.0, 4.0, seed=101)
    rx, ry = oracle.paper_radii(256, 256, 5)
    _check_log_backward(rgb, 5, rx, ry, 0.1, "c32x2", seed=9)


@pytest.mark.parametrize("recompute", [False, True])
def test_log_backward_through_autograd(recompute):
    from paper_2102_01289_amd.autograd import tonemap_luminance
    H, W = 70, 90
    rgb = rgb_case(H, W, 5, -3.0, 5.0, seed=77)
    rx, ry = oracle.paper_radii(H, W, 4)
    p = tm.make_params(5, 4, rx, ry, 0.1, 0.0, 1.0)
    m = tm.ToneMapper(H, W, p, "c32x2", variance="log")
    L = m.run_train(to_dev(rgb)).clone()
    g = to_dev(np.random.default_rng(4).standard_normal((H, W)).astype(np.float32))
    gv, gp = (t.clone() for t in m.backward_resid(g))
    lum = m.lum.clone().requires_grad_(True)
    scal = [torch.tensor(x, dtype=torch.float64, device="cuda", requires_grad=True)
            for x in (0.1, 0.0, 1.0)]
    out = tonemap_luminance(lum, *scal, n_bins=5, rx=rx, ry=ry, prec="c32x2",
                            recompute=recompute, variance="log")
    assert torch.equal(out, L)
    (out * g).sum().backward()
    assert torch.equal(lum.grad, gv)
    assert [float(t.grad) for t in scal] == gp.cpu().tolist()


def test_log_backward_1920x1080():
    c = WORKLOADS["wdr_1920x1080"]
    rgb = gen_wdr(c["H"], c["W"], c["K"], c["lo"], c["hi"], c["seed"]).rgb
    rx, ry = oracle.paper_radii(c["H"], c["W"], 5)
    _check_log_backward(rgb, 5, rx, ry, 0.1, "c32x2", seed=13)
