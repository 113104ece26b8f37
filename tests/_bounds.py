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


def tiling(H, W, vec=None, th=None, n_bins=0):
    """The scan tiling the library picks by default (mirrors scan_tune_default)."""
    if vec is None:
        vec = 4 if W >= 2048 else 2
    if th is None:
        th = 4 if H < 900 else 8 if H < 1800 else 16
        if n_bins >= 33:
            th = min(2 * th, 32)
        tx = -(-W // (64 * vec))
        while th > 4 and tx * (-(-H // th)) < 512:
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


# ------------------------------------------------------------------------ backward
def _suffix2d(a):
    """S[y, x] = sum of a over y' >= y, x' >= x."""
    return np.cumsum(np.cumsum(a[::-1, ::-1], 0), 1)[::-1, ::-1]


def _box(a, xm, xp, ym, yp):
    t = _box_table(a)
    return t[yp, xp] - t[ym, xp] - t[yp, xm] + t[ym, xm]


def measured_entry_errors(table, lum, prec, mu1=0.0, mu2=0.0):
    """Per-entry error bounds of a device integral image read back with Table.padded()
    ([1, H+1, W+1, comps]), from its exact difference to the oracle's double-double tables:
    |device - exact| plus the rounding of that FP64 difference itself (4 * 2^-53 of the
    magnitudes involved), and the FP64 rounding of the device's own four-corner combination
    (another 4 * 2^-53 |entry|).  For TM_SAT_C32X2 the device entry is the offset sum
    hi + lo (exact in FP64) and the exact one is sum (v - mu1) = I(v) - mu1 (x+1)(y+1)."""
    import oracle
    t = table[0].numpy().astype(np.float64)
    H, W = lum.shape
    h1, l1 = oracle.integral_image(lum, square=False)
    h2, l2 = oracle.integral_image(lum, square=True)
    u53 = 2.0 ** -53
    if prec == "c32x2":
        d1, d2 = t[..., 0] + t[..., 1], t[..., 2] + t[..., 3]
        yy, xx = np.mgrid[0:H + 1, 0:W + 1]
        cnt = (yy * xx).astype(np.float64)
        o1, o2 = mu1 * cnt, mu2 * cnt
    elif prec == "f64":
        d1, d2 = t[..., 0], t[..., 1]
        o1 = o2 = 0.0
    else:
        d1, d2 = t[..., 0], t[..., 1]
        o1 = o2 = 0.0
    e1 = np.abs((d1 + o1 - h1) - l1) + 8.0 * u53 * (np.abs(d1) + np.abs(h1) + np.abs(o1))
    e2 = np.abs((d2 + o2 - h2) - l2) + 8.0 * u53 * (np.abs(d2) + np.abs(h2) + np.abs(o2))
    return e1, e2


def backward_bound(lum, g, Lref, Lj, Wj, varj, S1j, rx, ry, eps, prec, vec, th, mu1=0.0,
                   mu2=0.0, dv_ref=None, entry_err=None, input_err=None):
    """Per-pixel bound on |dv_gpu - dv_oracle| for the gradient of sum(g L) wrt v.

    dv(q) = sum_j sum_{p: q in w_j(p)} g(p) (R1_j(p) + 2 v(q) R2_j(p)) with
    R2_j = c_j / N_j, R1_j = -2 m_j R2_j, c_j = (L_j - L)/D eps/(var_j + eps)^2.  The device
    forms R1, R2 per pixel in FP32 from its own window moments, then sums them exactly as
    above in FP64.  Error of one pixel's residuals:
      - c_j relative: ~16 FP32 roundings, 2 dvar_j/(var_j + eps) through the squared
        denominator, dD/D through the fusion weight sum (dD = sum_k eps/(var_k+eps)^2 dvar_k
        plus the FP32 rounding of every W_k);
      - c_j absolute: eps/(var_j+eps)^2/D times the error of L_j - L: twice the first-order
        variance part of the forward bound, plus the FP32 fusion (num/den, each a sum of s
        rounded products: (2s + 6) u |L|) and the rounding of L_j (u |L_j|).  Where every
        field has the same tone value (a pixel of the lowest bin) the device's L_j - L is
        exactly that of the oracle in every term but the fusion's rounding;
      - a possible flip of the clamp var_j > 0 where dvar_j >= var_j: the whole |c_j| at
        its largest, |L_j - L| + dL over D eps;
      - R1 adds 2 |R2| dm_j (dm_j = dS1/N) and the rounding of the product.
    The window of p contains q exactly when p is in the window of q (clamped windows of
    radius r are symmetric), so each field's part is a box sum of |g| dR1 and of
    2 |v(q)| |g| dR2.  The FP64 deposits and suffix scans add at most depth 2^-53 times the
    quadrant sums of the absolute deposits; the final FP32 store adds 2^-24 |dv|.  The
    first-order part carries a margin of 2.  Where dD reaches a quarter of D (a pixel whose
    every window is nearly flat, so that the fusion is close to 0/0), first order does not
    hold for that pixel's residuals: every pixel q inside one of its windows is then left
    unbounded (infinite).  The count of such pixels p is returned so tests can hold it small.  entry_err = (e1, e2): per-entry error bounds of the integral
    image (measured_entry_errors); by default the depth model of entry_bound.  The window
    moments then also carry the FP64 rounding of m and var (8 * 2^-53 of S2/N + |mu2| +
    m^2 + |m mu1|).  input_err = (d1, d2): per-pixel bounds on how far the device's terms
    q = v and q = v^2 may lie from the oracle's (as in forward_bound); their window sums join
    the moments' errors, and d1(q) also enters the final 2 v(q) s2(q) through
    2 d1(q) sum_j box(|g| |R2_j|)."""
    H, W = lum.shape
    s = len(rx)
    u = 2.0 ** -24
    v = np.abs(lum.astype(np.float64))
    gabs = np.abs(np.asarray(g, dtype=np.float64))
    e1, e2 = entry_err if entry_err is not None else entry_bound(lum, prec, vec, th, mu1, mu2)
    D = Wj.sum(axis=0)
    geo, dvar, dm = [], [], []
    for j in range(s):
        xm, xp, ym, yp, N = corners(H, W, rx[j], ry[j])
        c1 = e1[ym, xm] + e1[ym, xp] + e1[yp, xm] + e1[yp, xp]
        c2 = e2[ym, xm] + e2[ym, xp] + e2[yp, xm] + e2[yp, xp]
        if input_err is not None:
            c1 = c1 + _box(input_err[0], xm, xp, ym, yp)
            c2 = c2 + _box(input_err[1], xm, xp, ym, yp)
        m = S1j[j] / N
        geo.append((xm, xp, ym, yp, N))
        r64 = 8.0 * 2.0 ** -53 * (np.abs(varj[j]) + 2.0 * m * m + abs(mu2) + np.abs(m * mu1))
        dvar.append((c2 + 2.0 * np.abs(m) * c1) / N + r64)
        dm.append(c1 / N + 8.0 * 2.0 ** -53 * (np.abs(m) + abs(mu1)))
    del e1, e2
    dD = 4.0 * u * s + sum(eps / (varj[j] + eps) ** 2 * dvar[j] for j in range(s))
    with np.errstate(divide="ignore", invalid="ignore"):
        Dd = np.where(D > 0, D, 1.0)
        bad = (dD >= 0.25 * D) & ((D > 0) | (dD > 0))
        relD = dD / Dd
        # error of the device's L: first-order variance part (margin 2) + FP32 fusion
        dLv = np.zeros((H, W))
        for j in range(s):
            dLv += np.abs(Lj[j] - Lref) / Dd * eps / (varj[j] + eps) ** 2 * dvar[j]
        dLbase = 2.0 * dLv + (2.0 * s + 6.0) * u * np.abs(Lref)
        B = np.zeros((H, W))
        Q1 = np.zeros((H + 1, W + 1))
        Q2 = np.zeros((H + 1, W + 1))
        for j in range(s):
            xm, xp, ym, yp, N = geo[j]
            a = eps / (varj[j] + eps) ** 2
            c = np.where((D > 0) & (varj[j] > 0), (Lj[j] - Lref) / Dd * a, 0.0)
            rel = 16.0 * u + 2.0 * dvar[j] / (varj[j] + eps) + relD
            dLp = dLbase + u * np.abs(Lj[j])
            dc = np.abs(c) * rel + a / Dd * dLp
            flip = dvar[j] >= varj[j]
            dc = np.where(flip, np.maximum(dc, (np.abs(Lj[j] - Lref) + dLp) / Dd / eps
                                           * (1.0 + rel)), dc)
            m = S1j[j] / N
            R2 = np.abs(c) / N
            dR2 = dc / N + 2.0 * u * R2
            dR1 = 2.0 * np.abs(m) * dR2 + 2.0 * R2 * dm[j] + 4.0 * u * np.abs(m) * R2
            B += _box(gabs * dR1, xm, xp, ym, yp) + 2.0 * v * _box(gabs * dR2, xm, xp, ym, yp)
            if input_err is not None:
                B += 2.0 * input_err[0] * _box(gabs * (R2 + dR2), xm, xp, ym, yp)
            # absolute deposits at the four corners (the -1 border never enters a suffix)
            t1 = gabs * (2.0 * np.abs(m) * R2 + dR1)
            t2 = gabs * (R2 + dR2)
            for cy, cx in ((ym, xm), (ym, xp), (yp, xm), (yp, xp)):
                idx = (cy * (W + 1) + cx).ravel()
                Q1 += np.bincount(idx, t1.ravel(), (H + 1) * (W + 1)).reshape(H + 1, W + 1)
                Q2 += np.bincount(idx, t2.ravel(), (H + 1) * (W + 1)).reshape(H + 1, W + 1)
        depth64 = sat_depth(H, W, vec, th) + H + W + 64
        Q1 = _suffix2d(Q1)[1:, 1:]
        Q2 = _suffix2d(Q2)[1:, 1:]
        B = 2.0 * B + depth64 * 2.0 ** -53 * (Q1 + 2.0 * v * Q2) + 1e-300
        if dv_ref is not None:
            B += 2.0 * u * np.abs(dv_ref)
        if bad.any():
            hit = np.zeros((H, W))
            for j in range(s):
                xm, xp, ym, yp, _ = geo[j]
                hit += _box(bad.astype(np.float64), xm, xp, ym, yp)
            B = np.where(hit > 0, np.inf, B)
    return B, int(bad.sum())
