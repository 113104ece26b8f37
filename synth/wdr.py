"""Seeded synthetic WDR images standing in for the paper's captured scenes.

The paper evaluates on captured WDR photographs that are not available here, so every
input is drawn from a seeded generator with the structure of such scenes: smooth bright
and dark regions spanning six to eight decades of luminance, fine texture on top, and a
per-region colour cast.

Recipe (numpy PCG64, draws in this order):
  * K Gaussian blobs: centre uniform over the image, sigma ~ U(0.03, 0.25) * min(H, W),
    amplitude a ~ U(0.2, 1), chroma ~ U(0.5, 1.5)^3;
  * F = sum_k a_k g_k, min-max normalised to [0, 1];
  * log10 Y = lo + (hi - lo) * F + N(0, 0.05) i.i.d. per pixel;
  * every pixel takes the chroma of its dominant blob (argmax_k a_k g_k);
  * RGB = Y * chroma, float32, planar [3, H, W].
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np

__all__ = ["WdrImage", "gen_wdr", "gen_wdr_row", "gen_batch_shapes", "gen_upstream_grad", "WORKLOADS"]


@dataclass(frozen=True)
class WdrImage:
    rgb: np.ndarray  # float32 [3, H, W], planar
    seed: int
    blobs: int
    lo: float
    hi: float


def _row_chunks(n: int, step: int):
    for a in range(0, n, step):
        yield a, min(n, a + step)


def gen_wdr(H: int, W: int, K: int = 8, lo: float = -2.0, hi: float = 4.0,
            seed: int = 0) -> WdrImage:
    """Draw one seeded RGB WDR image of shape [3, H, W] (float32, planar)."""
    if H < 1 or W < 1 or K < 1:
        raise ValueError("H, W and K must be positive")
    rng = np.random.Generator(np.random.PCG64(seed))
    cx = rng.uniform(0.0, W, size=K)
    cy = rng.uniform(0.0, H, size=K)
    sig = rng.uniform(0.03, 0.25, size=K) * min(H, W)
    amp = rng.uniform(0.2, 1.0, size=K)
    chroma = rng.uniform(0.5, 1.5, size=(K, 3))

    xs = np.arange(W, dtype=np.float64)
    ys = np.arange(H, dtype=np.float64)
    inv2s2 = 1.0 / (2.0 * sig * sig)
    # separable Gaussians: log g_k(x, y) = lx[k, x] + ly[k, y]
    lx = -((xs[None, :] - cx[:, None]) ** 2) * inv2s2[:, None]  # [K, W]
    ly = -((ys[None, :] - cy[:, None]) ** 2) * inv2s2[:, None]  # [K, H]
    gx = np.exp(lx)
    gy = np.exp(ly)
    F = (gy * amp[:, None]).T @ gx  # [H, W] = sum_k a_k gy_k(y) gx_k(x)
    fmin, fmax = float(F.min()), float(F.max())
    F = (F - fmin) / (fmax - fmin) if fmax > fmin else np.zeros_like(F)

    noise = rng.standard_normal((H, W)) * 0.05
    Y = np.power(10.0, lo + (hi - lo) * F + noise)
    del F, noise

    # dominant blob per pixel: argmax_k (log a_k + ly[k, y] + lx[k, x])
    la = np.log(amp).astype(np.float32)
    lx32 = lx.astype(np.float32)
    ly32 = (ly + np.log(amp)[:, None]).astype(np.float32)
    dom = np.empty((H, W), dtype=np.int16)
    step = max(1, (1 << 22) // (K * W))
    for a, b in _row_chunks(H, step):
        score = ly32[:, a:b].T[:, :, None] + lx32[None, :, :]  # [rows, K, W]
        dom[a:b] = np.argmax(score, axis=1)
    del la

    rgb = np.empty((3, H, W), dtype=np.float32)
    for c in range(3):
        rgb[c] = (Y * chroma[dom, c]).astype(np.float32)
    return WdrImage(rgb=rgb, seed=seed, blobs=K, lo=lo, hi=hi)


def gen_wdr_row(W: int, K: int = 8, lo: float = -2.0, hi: float = 4.0,
                seed: int = 0) -> np.ndarray:
    """One seeded WDR luminance row [W] (float32): the recipe above along one axis, with
    sigma ~ U(0.03, 0.25) * W and no colour.  Broadcast down the rows, it gives an image whose
    every row is the same, for tests at sizes the oracle cannot cover in two dimensions."""
    if W < 1 or K < 1:
        raise ValueError("W and K must be positive")
    rng = np.random.Generator(np.random.PCG64(seed))
    cx = rng.uniform(0.0, W, size=K)
    sig = rng.uniform(0.03, 0.25, size=K) * W
    amp = rng.uniform(0.2, 1.0, size=K)
    xs = np.arange(W, dtype=np.float64)
    F = np.zeros(W)
    for k in range(K):
        F += amp[k] * np.exp(-((xs - cx[k]) ** 2) / (2.0 * sig[k] * sig[k]))
    fmin, fmax = float(F.min()), float(F.max())
    F = (F - fmin) / (fmax - fmin) if fmax > fmin else np.zeros_like(F)
    noise = rng.standard_normal(W) * 0.05
    return np.power(10.0, lo + (hi - lo) * F + noise).astype(np.float32)


def gen_batch_shapes(count: int, lo: int = 360, hi: int = 4000, seed: int = 0):
    """(H, W) pairs with H, W ~ U{lo..hi} each, seeded."""
    rng = np.random.Generator(np.random.PCG64(seed))
    hw = rng.integers(lo, hi + 1, size=(count, 2))
    return [(int(h), int(w)) for h, w in hw]


def gen_upstream_grad(shape, seed: int = 0) -> np.ndarray:
    """Upstream gradient g ~ N(0, 1), float32."""
    rng = np.random.Generator(np.random.PCG64(seed))
    return rng.standard_normal(shape).astype(np.float32)


# Named workloads: (H, W, blobs, lo, hi, seed).  The batch entries list their own shapes.
WORKLOADS = {
    "wdr_256x256": dict(H=256, W=256, K=8, lo=-2.0, hi=4.0, seed=101),
    "wdr_1920x1080": dict(H=1080, W=1920, K=32, lo=-2.0, hi=4.0, seed=102),
    "wdr_4000x3000": dict(H=3000, W=4000, K=64, lo=-3.0, hi=5.0, seed=103),
    "wdr_batch64_uneven": dict(count=64, K=32, lo=-2.0, hi=4.0, seed=104, shape_seed=1104),
    "wdr_batch8_1024": dict(count=8, H=1024, W=1024, K=32, lo=-2.0, hi=4.0, seed=105),
}
