"""GPU parity of the multi-exposure front end (Debevec-Malik response recovery and radiance
merge, the step before the tone mapping in the paper's application, Section III) against
the FP64 oracle, on seeded synthetic exposure stacks."""
import numpy as np
import pytest
import torch

import paper_2102_01289_amd as tm
from _cases import to_dev
from oracle import hdr
from synth import exposure_times, gen_exposure_stack, gen_sample_pixels, gen_wdr

pytestmark = pytest.mark.gpu

U = 2.0 ** -24


def _stack(H, W, P=4, seed=0, noise=0.5):
    img = gen_wdr(H, W, 5, -2.0, 4.0, seed=seed)
    times = exposure_times(P, ratio=16.0 if P > 1 else 1.0)
    return gen_exposure_stack(img.rgb, times, noise=noise, seed=seed + 1), times


def _samples(stack, idx):
    P = stack.shape[0]
    flat = stack.reshape(P, 3, -1)
    return [flat[:, c, idx].T for c in range(3)]


def _merge_bound(stack, g, t, lnE):
    """Per-value bound on |E_gpu / E_oracle - 1|: the FP32 weighted sum of P terms
    (each term one rounding, each fused step one), the division, then expf (2 ulp)."""
    P = stack.shape[0]
    A = np.zeros(lnE.shape)
    Sw = np.zeros(lnE.shape)
    Sp = np.zeros(lnE.shape)
    for j in range(P):
        for c in range(3):
            z = stack[j, c].astype(np.int64)
            term = np.abs(g[c][z] - t[j])
            w = hdr.weight(z)
            A[c] += w * term
            Sw[c] += w
            Sp[c] += term
    with np.errstate(invalid="ignore", divide="ignore"):
        d = np.where(Sw > 0, (P + 2) * U * A / np.where(Sw > 0, Sw, 1.0), (P + 2) * U * Sp / P)
    d += 2 * U * np.abs(lnE)
    return 1.01 * d + 4 * U


@pytest.mark.parametrize("H,W,P", [(1, 1, 1), (37, 123, 3), (64, 256, 4), (301, 417, 4),
                                   (96, 2048, 5), (32, 512, 3), (16, 64, 2), (8, 72, 7),
                                   (5, 1000, 16)])
def test_merge_vs_oracle(H, W, P):
    stack, times = _stack(H, W, P, seed=H + W)
    rng = np.random.default_rng(P)
    g = np.sort(rng.uniform(-9.0, 2.0, size=(3, 256)), axis=1).astype(np.float32)
    g -= g[:, 128:129]
    t = np.log(times).astype(np.float32)
    E = tm.tm_hdr_merge(to_dev(stack), to_dev(t), to_dev(g)).cpu().numpy().astype(np.float64)
    lnE = hdr.merge(stack, g.astype(np.float64), t.astype(np.float64))
    ref = np.exp(lnE)
    bound = _merge_bound(stack, g.astype(np.float64), t.astype(np.float64), lnE)
    rel = np.abs(E / ref - 1.0)
    assert np.all(rel <= bound), f"max rel {rel.max():.3e}"


def test_merge_strided_stack_and_output():
    # a stack that is a view with row and channel padding, and an output with padding
    H, W, P = 45, 77, 3
    stack, times = _stack(H, W, P, seed=5)
    big = np.zeros((P, 4, H + 3, W + 9), dtype=np.uint8)
    big[:, :3, :H, :W] = stack
    dev = to_dev(big)[:, :3, :H, :W]
    out = torch.full((3, H + 2, W + 5), -1.0, device="cuda")
    g = np.cumsum(np.full((3, 256), 0.03, dtype=np.float32), axis=1)
    g -= g[:, 128:129]
    t = np.log(times).astype(np.float32)
    tm.tm_hdr_merge(dev, to_dev(t), to_dev(g), out=out[:, :H, :W])
    o = out.cpu().numpy()
    assert np.all(o[:, H:, :] == -1.0) and np.all(o[:, :, W:] == -1.0)
    lnE = hdr.merge(stack, g.astype(np.float64), t.astype(np.float64))
    bound = _merge_bound(stack, g.astype(np.float64), t.astype(np.float64), lnE)
    assert np.all(np.abs(o[:, :H, :W] / np.exp(lnE) - 1.0) <= bound)


def _response_bound(Z, t, lam, g_ref):
    """Both sides solve the same FP64 least squares (the oracle on the full system, the
    device through the eliminated normal equations, whose condition number is at most
    cond(A)^2); the device result is then rounded to FP32."""
    A, _ = hdr.system(Z, t, lam)
    keep = np.any(A != 0.0, axis=0)         # samples saturated everywhere carry no column
    k = np.linalg.cond(A[:, keep])
    return U * np.abs(g_ref) + 64 * k * k * 2.0 ** -53 * np.max(np.abs(g_ref)) + 1e-30


@pytest.mark.parametrize("H,W,P,N,lam", [(64, 96, 4, 120, 100.0), (300, 400, 3, 300, 20.0),
                                         (128, 128, 5, 80, 1000.0)])
def test_response_vs_oracle(H, W, P, N, lam):
    stack, times = _stack(H, W, P, seed=7 * P + N)
    idx = gen_sample_pixels(H, W, N, seed=N)
    t = np.log(times).astype(np.float32)
    g = tm.tm_hdr_response(to_dev(stack), to_dev(t), to_dev(idx), lam).cpu().numpy()
    assert np.all(g[:, 128] == 0.0)
    for c, Z in enumerate(_samples(stack, idx)):
        ref = hdr.response(Z, t.astype(np.float64), lam)
        err = np.abs(g[c].astype(np.float64) - ref)
        bound = _response_bound(Z, t.astype(np.float64), lam, ref)
        assert np.all(err <= bound), f"channel {c}: max err {err.max():.3e}"


def test_response_exact_linear_log_response():
    # every Z_ij = 128 + k_i + s_j with ln E_i = a k_i, ln dt_j = a s_j: the data are exactly
    # consistent with g(z) = a (z - 128), which the device must recover to FP32 rounding
    a = 0.05
    rng = np.random.default_rng(3)
    N, s = 60, np.array([0, 15, 30, 45])
    k = rng.integers(-120, 80, size=N)
    Z = (128 + k[:, None] + s[None, :]).astype(np.uint8)          # [N, P]
    stack = np.zeros((4, 3, 1, N), dtype=np.uint8)
    for c in range(3):
        stack[:, c, 0, :] = Z.T
    t = (a * s).astype(np.float32)
    idx = np.arange(N, dtype=np.int32)
    g = tm.tm_hdr_response(to_dev(stack), to_dev(t), to_dev(idx), 100.0).cpu().numpy()
    want = a * (np.arange(256) - 128.0)
    assert np.max(np.abs(g - want[None, :])) <= 1e-5


def test_response_skips_samples_outside_the_image_and_flags_singular_systems():
    H, W, P = 50, 60, 3
    stack, times = _stack(H, W, P, seed=11)
    t = np.log(times).astype(np.float32)
    idx = gen_sample_pixels(H, W, 100, seed=12)
    bad = np.concatenate([idx[:50], [-1, H * W, 2 ** 31 - 1], idx[50:]]).astype(np.int32)
    g1 = tm.tm_hdr_response(to_dev(stack), to_dev(t), to_dev(idx), 50.0).cpu().numpy()
    g2 = tm.tm_hdr_response(to_dev(stack), to_dev(t), to_dev(bad), 50.0).cpu().numpy()
    for c, Z in enumerate(_samples(stack, idx)):
        ref = hdr.response(Z, t.astype(np.float64), 50.0)
        bound = _response_bound(Z, t.astype(np.float64), 50.0, ref)
        assert np.all(np.abs(g2[c] - ref) <= bound)
        assert np.all(np.abs(g1[c] - ref) <= bound)
    # one exposure: the data never constrain g, the slope stays free -> NaN
    g = tm.tm_hdr_response(to_dev(stack[:1]), to_dev(t[:1]), to_dev(idx), 50.0).cpu().numpy()
    assert np.all(np.isnan(g))


def test_exposures_to_tonemapped_rgb():
    # the whole application chain on the device: response, merge, then the tone mapping
    # with colour restoration; each stage is checked above, here the chain's output range
    H, W = 240, 320
    stack, times = _stack(H, W, 4, seed=21)
    t = to_dev(np.log(times).astype(np.float32))
    st = to_dev(stack)
    g = tm.tm_hdr_response(st, t, to_dev(gen_sample_pixels(H, W, 200, seed=22)), 100.0)
    E = tm.tm_hdr_merge(st, t, g)
    p = tm.make_params(5, 5, eps=0.1, H=H, W=W)
    m = tm.ToneMapper(H, W, p, "c32x2")
    out = m.run_rgb(E).cpu().numpy()
    L = m.out.cpu().numpy()
    assert np.all(np.isfinite(out)) and np.all(np.isfinite(L))
    assert L.min() >= 0.0 and L.max() <= 1.0
    assert np.all(out >= 0.0)
