"""Error bounds used by the parity tests, derived from the arithmetic (no fitting).

Integral images.  Every stored entry is a sum of the pixel terms q over its quadrant,
formed by a fixed tree of additions in the table's arithmetic.  Along any root-to-leaf path
the tree has at most
    depth = 2 tiles_x + 2 tiles_y + th + 2 vec + 28
additions (in-lane prefix, 6 DPP levels, row and column carries, the tile's column run; a
row total of a group of eight rows takes 8 + 3 levels across the lanes),
so the entry's error is at most depth * u * sum |q| over the quadrant, with u = 2^-24
(FP32), 2^-44 (compensated FP32 pairs: TwoSum of the leading parts plus the trailing parts)
or 2^-53 (FP64).  For TM_SAT_C32X2, q = v - mu1 (and v^2 - mu2), |q| <= v + mu1.

Log-domain variance variant.  The device's log plane is FP32 logf, within 2 ulp of the
exact logarithm; the oracle's is FP64.  That input difference enters the window sums as
|dS1| <= sum |dl| and |dS2| <= sum (2 |l| |dl| + dl^2) over the window.

Fused output.  A perturbation d_j of the window variance of field j moves
L = sum W_j L_j / D (D = sum W_j, W_j = var_j/(var_j + eps)) by
    dL = sum_j (L_j - L)/D * eps/(var_j + eps)^2 * d_j        (first order),
and var_j = S2/N - (S1/N)^2 gives |d_j| <= (|dS2| + 2 |S1/N| |dS1|)/N with |dS| bounded by
the four corners' entry bounds.  The per-pixel bound is 4 * that first-order term (margin
for second order) plus 4e-6 for the FP32 blend (W_j, P, L_j, the fusion division: a few
FP32 roundings of values in [0, 1])."""
from __future__ import annotations

import numpy as np

U = {"f32": 2.0 ** -24, "c32x2": 2.0 ** -44, "f64": 2.0 ** -53}


def tiling(H, W, vec=None, th=None):
    """The scan tiling the library picks by default (mirrors scan_tune_default)."""
    if vec is None:
        vec = 4 if W >= 2048 else 2
    if th is None:
        th = 16
        tx = -(-W // (64 * vec))
        while th > 4 and tx * (-(-H // th)) < 2048:
            th //= 2
    return vec, th


def sat_depth(H, W, vec, th):
    tx = -(-W // (64 * vec))
    ty = -(-H // th)
    return 2 * tx + 2 * ty + th + 2 * vec + 28


def abs_tables(lum, prec, mu1=0.0, mu2=0.0):
    """Quadrant sums of |q| for q = v and q = v^2 (upper bounds for C32X2), shape (H+1, W+1)."""
    v = np.abs(lum.astype(np.float64))
    H, W = v.shape
    a1 = np.zeros((H + 1, W + 1))
    a2 = np.zeros((H + 1, W + 1))
    a1[1:, 1:] = np.cumsum(np.cumsum(v, 0), 1)
    a2[1:, 1:] = np.cumsum(np.cumsum(v * v, 0), 1)
    if prec == "c32x2":
        yy, xx = np.mgrid[0:H + 1, 0:W + 1]
        cnt = (yy * xx).astype(np.float64)
        a1 += cnt * abs(mu1)
        a2 += cnt * abs(mu2)
    return a1, a2


def entry_bound(lum, prec, vec, th, mu1=0.0, mu2=0.0):
    H, W = lum.shape
    d = sat_depth(H, W, vec, th)
    a1, a2 = abs_tables(lum, prec, mu1, mu2)
    return d * U[prec] * a1, d * U[prec] * a2


def corners(H, W, rx, ry):
    """Per-pixel clamped corner indices in the (H+1, W+1) padded layout."""
    ys, xs = np.mgrid[0:H, 0:W]
    xm = np.maximum(xs - rx - 1, -1) + 1
    xp = np.minimum(xs + rx, W - 1) + 1
    ym = np.maximum(ys - ry - 1, -1) + 1
    yp = np.minimum(ys + ry, H - 1) + 1
    N = ((xp - xm) * (yp - ym)).astype(np.float64)
    return xm, xp, ym, yp, N


def _box_table(a):
    t = np.zeros((a.shape[0] + 1, a.shape[1] + 1))
    t[1:, 1:] = np.cumsum(np.cumsum(a, 0), 1)
    return t


def var_bounds(lum, S1j, rx, ry, prec, vec, th, mu1=0.0, mu2=0.0, input_err=None):
    """Per field, the per-pixel bound on |var_gpu - var_oracle| propagated from the four
    corners' entry bounds (and input_err, see forward_bound)."""
    H, W = lum.shape
    e1, e2 = entry_bound(lum, prec, vec, th, mu1, mu2)
    b1 = b2 = None
    if input_err is not None:
        b1, b2 = _box_table(input_err[0]), _box_table(input_err[1])
    out = []
    for j in range(len(rx)):
        xm, xp, ym, yp, N = corners(H, W, rx[j], ry[j])
        c1 = e1[ym, xm] + e1[ym, xp] + e1[yp, xm] + e1[yp, xp]
        c2 = e2[ym, xm] + e2[ym, xp] + e2[yp, xm] + e2[yp, xp]
        if b1 is not None:
            c1 = c1 + (b1[yp, xp] - b1[ym, xp] - b1[yp, xm] + b1[ym, xm])
            c2 = c2 + (b2[yp, xp] - b2[ym, xp] - b2[yp, xm] + b2[ym, xm])
        out.append((c2 + 2.0 * np.abs(S1j[j] / N) * c1) / N)
    return out


def forward_bound(lum, Lref, Lj, Wj, varj, S1j, rx, ry, eps, prec, vec, th, mu1=0.0,
                  mu2=0.0, input_err=None):
    """Per-pixel bound on |L_gpu - L_oracle| (see module docstring).  lum is the image whose
    window variance is taken.  input_err = (d1, d2): per-pixel bounds on how far the device's
    terms q = v and q = v^2 may lie from the oracle's (when the two do not start from the
    same values), added to the table bounds through window sums."""
    H, W = lum.shape
    dv = var_bounds(lum, S1j, rx, ry, prec, vec, th, mu1, mu2, input_err)
    D = Wj.sum(axis=0)
    out = np.zeros((H, W))
    with np.errstate(divide="ignore", invalid="ignore"):
        for j in range(len(rx)):
            sens = np.abs(Lj[j] - Lref) / D * eps / (varj[j] + eps) ** 2
            # with every weight near zero the first-order term is not a bound: count the whole
            # range as possible there
            term = np.where(D > 0, sens * dv[j], 1.0)
            out += term
    return 4.0 * out + 4e-6


def window_sums(lum, rx, ry):
    """S1 per field (FP64, exact enough for the bound's |S1/N| factor)."""
    v = lum.astype(np.float64)
    H, W = v.shape
    a = np.zeros((H + 1, W + 1))
    a[1:, 1:] = np.cumsum(np.cumsum(v, 0), 1)
    out = []
    for j in range(len(rx)):
        xm, xp, ym, yp, _ = corners(H, W, rx[j], ry[j])
        out.append(a[yp, xp] - a[ym, xp] - a[yp, xm] + a[ym, xm])
    return np.stack(out)
