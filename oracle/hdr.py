"""CPU oracle of the multi-exposure front end: camera response recovery and radiance-map
merge of Debevec and Malik (the method the paper's application uses to build its WDR input
from four exposures, Section III).

TEST INFRASTRUCTURE ONLY (tests, smoke, bench CPU leg).  Plain numpy in FP64; the least
squares is solved with numpy's lstsq on the full system, written out row by row.

The method, for 8-bit values z in [0, 255], pixel i, exposure j of time dt_j:
  * reciprocity: the inverse log response g(z) = ln f^-1(z) satisfies
    g(Z_ij) = ln E_i + ln dt_j;
  * hat weight w(z) = z for z <= 127, 255 - z for z >= 128 (trusting mid-range values);
  * response: minimise
        sum_ij [w(Z_ij) (g(Z_ij) - ln E_i - ln dt_j)]^2
      + lam * sum_{z=1..254} [w(z) (g(z-1) - 2 g(z) + g(z+1))]^2
    over g(0..255) and ln E_i, with g(128) = 0 fixing the scale;
  * radiance map: ln E_i = sum_j w(Z_ij) (g(Z_ij) - ln dt_j) / sum_j w(Z_ij).
Readings: lam multiplies the squared smoothness term (the objective as written, so each
smoothness row carries sqrt(lam) w(z)); a pixel whose every exposure has weight 0 (each value
0 or 255) takes the unweighted mean of g(Z_ij) - ln dt_j.
"""
from __future__ import annotations

import numpy as np

ZMID = 128


def weight(z) -> np.ndarray:
    """Hat weight of 8-bit values (float64)."""
    z = np.asarray(z, dtype=np.int64)
    return np.where(z <= 127, z, 255 - z).astype(np.float64)


def system(Z, log_dt, lam: float):
    """The least-squares system (A, b) of the response: columns g(0..255) without g(128),
    then ln E_0..ln E_{N-1}; one row per sample value, then one per smoothness term."""
    Z = np.asarray(Z, dtype=np.int64)
    t = np.asarray(log_dt, dtype=np.float64)
    N, P = Z.shape
    if t.shape != (P,):
        raise ValueError("log_dt must have one entry per exposure")
    # columns: g(0..255) without g(128), then ln E_0..ln E_{N-1}
    gcol = {z: (z if z < ZMID else z - 1) for z in range(256) if z != ZMID}
    ncol = 255 + N
    rows = N * P + 254
    A = np.zeros((rows, ncol))
    b = np.zeros(rows)
    r = 0
    for i in range(N):
        for j in range(P):
            w = float(weight(Z[i, j]))
            z = int(Z[i, j])
            if z != ZMID:
                A[r, gcol[z]] = w
            A[r, 255 + i] = -w
            b[r] = w * t[j]
            r += 1
    s = np.sqrt(lam)
    for z in range(1, 255):
        w = float(weight(z))
        for dz, c in ((-1, 1.0), (0, -2.0), (1, 1.0)):
            if z + dz != ZMID:
                A[r, gcol[z + dz]] = s * w * c
        r += 1
    return A, b


def response(Z, log_dt, lam: float, return_lnE: bool = False):
    """Inverse log response g[256] (float64, g[128] = 0) from samples Z [N, P] (uint8)
    and log exposure times log_dt [P]; with return_lnE also the samples' ln E [N]."""
    A, b = system(Z, log_dt, lam)
    gcol = {z: (z if z < ZMID else z - 1) for z in range(256) if z != ZMID}
    x = np.linalg.lstsq(A, b, rcond=None)[0]
    g = np.zeros(256)
    for z, c in gcol.items():
        g[z] = x[c]
    return (g, x[255:].copy()) if return_lnE else g


def objective(g, lnE, Z, log_dt, lam: float) -> float:
    """The minimised objective, written out term by term (for pinning)."""
    Z = np.asarray(Z, dtype=np.int64)
    total = 0.0
    for i in range(Z.shape[0]):
        for j in range(Z.shape[1]):
            z = int(Z[i, j])
            total += (float(weight(z)) * (g[z] - lnE[i] - log_dt[j])) ** 2
    for z in range(1, 255):
        total += lam * (float(weight(z)) * (g[z - 1] - 2.0 * g[z] + g[z + 1])) ** 2
    return total


def merge(stack, g, log_dt) -> np.ndarray:
    """ln E (float64 [3, H, W]) of a uint8 stack [P, 3, H, W] under per-channel inverse log
    responses g [3, 256] and log exposure times log_dt [P]."""
    stack = np.asarray(stack)
    g = np.asarray(g, dtype=np.float64)
    t = np.asarray(log_dt, dtype=np.float64)
    P = stack.shape[0]
    num = np.zeros(stack.shape[1:])
    den = np.zeros(stack.shape[1:])
    plain = np.zeros(stack.shape[1:])
    for j in range(P):
        for c in range(3):
            z = stack[j, c].astype(np.int64)
            term = g[c][z] - t[j]
            w = weight(z)
            num[c] += w * term
            den[c] += w
            plain[c] += term
    with np.errstate(invalid="ignore", divide="ignore"):
        return np.where(den > 0, num / np.where(den > 0, den, 1.0), plain / P)
