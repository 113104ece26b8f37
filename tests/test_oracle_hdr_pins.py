"""Pins for the oracle of the multi-exposure front end (Debevec-Malik response recovery and
radiance merge, the step before the tone mapping in the paper's application, Section III):
exactly consistent data with a known response, stationarity of the objective written out
term by term, exact rational brute force of the merge, closed forms."""
from fractions import Fraction

import numpy as np

from oracle import hdr
from synth import exposure_times, gen_exposure_stack, gen_sample_pixels, gen_wdr


def _consistent_samples(a=0.05, P=4, N=40, seed=0):
    # g_true(z) = a (z - 128) is linear, so its second differences vanish; integer offsets
    # for ln E_i / a and ln dt_j / a make every Z_ij = 128 + k_i + s_j an exact code value
    rng = np.random.default_rng(seed)
    s = np.array([0, 15, 30, 45][:P])
    k = rng.integers(-120, 80, size=N)
    Z = (128 + k[:, None] + s[None, :]).astype(np.int64)
    assert Z.min() >= 1 and Z.max() <= 254
    return Z.astype(np.uint8), a * s.astype(np.float64), a * k.astype(np.float64)


def test_response_recovers_an_exact_linear_log_response():
    a = 0.05
    Z, t, lnE = _consistent_samples(a)
    for lam in (0.1, 10.0, 1000.0):
        g, e = hdr.response(Z, t, lam, return_lnE=True)
        assert np.max(np.abs(g - a * (np.arange(256) - 128))) <= 1e-9
        assert np.max(np.abs(e - lnE)) <= 1e-9
        assert g[128] == 0.0


def test_response_is_a_stationary_point_of_the_objective():
    img = gen_wdr(40, 50, 5, -2.0, 4.0, seed=3)
    t = np.log(exposure_times(4))
    st = gen_exposure_stack(img.rgb, np.exp(t), seed=4)
    idx = gen_sample_pixels(40, 50, 90, seed=5)
    Z = st[:, 0].reshape(4, -1)[:, idx].T
    lam = 20.0
    g, e = hdr.response(Z, t, lam, return_lnE=True)
    base = hdr.objective(g, e, Z, t, lam)
    h = 1e-4
    # the objective is quadratic: central differences are its exact gradient
    for z in [1, 5, 40, 100, 127, 129, 200, 254]:
        gp, gm = g.copy(), g.copy()
        gp[z] += h
        gm[z] -= h
        d = (hdr.objective(gp, e, Z, t, lam) - hdr.objective(gm, e, Z, t, lam)) / (2 * h)
        assert abs(d) <= 1e-6 * max(base, 1.0), (z, d)
    for i in [0, 17, 89]:
        ep, em = e.copy(), e.copy()
        ep[i] += h
        em[i] -= h
        d = (hdr.objective(g, ep, Z, t, lam) - hdr.objective(g, em, Z, t, lam)) / (2 * h)
        assert abs(d) <= 1e-6 * max(base, 1.0), (i, d)
    # moving g(128) off zero would lower nothing the constraint allows: it stays pinned
    assert g[128] == 0.0


def test_merge_matches_exact_rational_brute_force():
    rng = np.random.default_rng(7)
    P, H, W = 3, 4, 5
    st = rng.integers(0, 256, size=(P, 3, H, W)).astype(np.uint8)
    st[:, 0, 0, 0] = 255          # saturated in every exposure: the unweighted mean
    st[:, 1, 1, 1] = [0, 255, 0]  # every weight zero, mixed
    g = np.cumsum(rng.uniform(0.01, 0.1, size=(3, 256)), axis=1)
    g -= g[:, 128:129]
    t = np.log(np.array([1 / 64, 1 / 8, 1.0]))
    got = hdr.merge(st, g, t)
    for c in range(3):
        for y in range(H):
            for x in range(W):
                num = den = Fraction(0)
                plain = Fraction(0)
                for j in range(P):
                    z = int(st[j, c, y, x])
                    w = z if z <= 127 else 255 - z
                    term = Fraction(float(g[c, z])) - Fraction(float(t[j]))
                    num += w * term
                    den += w
                    plain += term
                want = num / den if den else plain / P
                assert abs(got[c, y, x] - float(want)) <= 1e-14


def test_merge_closed_forms():
    rng = np.random.default_rng(8)
    g = np.sort(rng.uniform(-5, 2, size=(3, 256)), axis=1)
    # one exposure: ln E = g(Z) - ln dt at every pixel, whatever the weight
    st = rng.integers(0, 256, size=(1, 3, 6, 7)).astype(np.uint8)
    t = np.array([np.log(0.01)])
    want = np.stack([g[c][st[0, c].astype(int)] for c in range(3)]) - t[0]
    assert np.max(np.abs(hdr.merge(st, g, t) - want)) <= 1e-15
    # exposures in any order give the same map
    st3 = rng.integers(0, 256, size=(3, 3, 6, 7)).astype(np.uint8)
    t3 = np.log(np.array([0.01, 0.1, 1.0]))
    perm = [2, 0, 1]
    assert np.max(np.abs(hdr.merge(st3, g, t3) - hdr.merge(st3[perm], g, t3[perm]))) <= 1e-14
    # the hat weight
    assert hdr.weight(0) == 0 and hdr.weight(127) == 127 and hdr.weight(128) == 127
    assert hdr.weight(255) == 0


def test_recovery_of_a_noise_free_camera_is_a_constant_log_shift():
    # the recovered map equals the true radiance up to one global factor (g(128) = 0 fixes
    # the scale) wherever some exposure is mid-range
    img = gen_wdr(48, 64, 5, -2.0, 3.0, seed=9)
    times = exposure_times(4)
    st = gen_exposure_stack(img.rgb, times, noise=0.0, seed=10)
    idx = gen_sample_pixels(48, 64, 200, seed=11)
    t = np.log(times)
    g = np.stack([hdr.response(st[:, c].reshape(4, -1)[:, idx].T, t, 100.0)
                  for c in range(3)])
    lnE = hdr.merge(st, g, t)
    good = ((st > 20) & (st < 235)).any(axis=0)
    d = (lnE - np.log(img.rgb.astype(np.float64)))[good]
    assert np.std(d) <= 0.05
