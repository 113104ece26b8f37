"""Seeded synthetic exposure stacks standing in for the paper's multi-exposure captures.

The paper's application captures four exposures and recovers a WDR image from them
(Section III, with the method of Debevec and Malik).  Those captures are not available, so a
stack is drawn from a synthetic WDR radiance image through a simple camera model.  This
module holds the camera, not the recovery: none of the recovery's arithmetic is here.

Camera (numpy PCG64, draws in this order):
  * exposure times dt_j = dt_0 * ratio^j, j = 0..P-1;
  * a scale k that maps the image's median radiance, under the middle exposure, to the
    middle of the 8-bit range;
  * per exposure and channel, Z = clip(round(255 (E dt_j / k)^(1/gamma) + N(0, noise)),
    0, 255) as uint8, so dark pixels underflow in the short exposures and bright ones
    saturate in the long ones.
"""
from __future__ import annotations

import numpy as np

__all__ = ["exposure_times", "gen_exposure_stack", "gen_sample_pixels"]


def exposure_times(P: int = 4, ratio: float = 16.0, dt0: float = 1.0 / 1024) -> np.ndarray:
    """dt_j = dt0 * ratio^j (float64, seconds)."""
    return dt0 * ratio ** np.arange(P, dtype=np.float64)


def gen_exposure_stack(radiance: np.ndarray, times, gamma: float = 2.2, noise: float = 0.5,
                       seed: int = 0) -> np.ndarray:
    """uint8 stack [P, 3, H, W] of the planar float32 radiance [3, H, W]."""
    rad = np.asarray(radiance, dtype=np.float64)
    times = np.asarray(times, dtype=np.float64)
    if rad.ndim != 3 or rad.shape[0] != 3:
        raise ValueError("radiance must be planar [3, H, W]")
    rng = np.random.Generator(np.random.PCG64(seed))
    k = float(np.median(rad)) * float(times[len(times) // 2]) / 0.5 ** gamma
    out = np.empty((len(times),) + rad.shape, dtype=np.uint8)
    for j, dt in enumerate(times):
        x = np.clip(rad * (dt / k), 0.0, None) ** (1.0 / gamma)
        z = np.rint(255.0 * x + rng.standard_normal(rad.shape) * noise)
        out[j] = np.clip(z, 0, 255).astype(np.uint8)
    return out


def gen_sample_pixels(H: int, W: int, N: int, seed: int = 0) -> np.ndarray:
    """N distinct flat pixel indices y*W + x (int32, ascending), drawn uniformly."""
    rng = np.random.Generator(np.random.PCG64(seed))
    N = min(N, H * W)
    return np.sort(rng.choice(H * W, size=N, replace=False)).astype(np.int32)
