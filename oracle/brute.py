"""Pure-Python brute force of the tone-mapping method, exact rational arithmetic.

TEST INFRASTRUCTURE ONLY.  It pins the C oracle on tiny images: every quantity is a
``fractions.Fraction``, every window statistic is taken directly over the window's pixels,
and the bin of a pixel is decided from the definition of equal-width log bins without
going through any edge table.  Nothing here shares code with ``tm_oracle.c``.
"""
from __future__ import annotations

import math
from fractions import Fraction

import numpy as np

FLT_MIN = Fraction(1, 2 ** 126)


def round_f32(q: Fraction) -> np.float32:
    """Round an exact rational to the nearest FP32 (ties to even), with subnormals."""
    if q == 0:
        return np.float32(0.0)
    sign = -1 if q < 0 else 1
    a = abs(q)
    # e = floor(log2(a))
    e = a.numerator.bit_length() - a.denominator.bit_length()
    if Fraction(2) ** e > a:
        e -= 1
    while Fraction(2) ** (e + 1) <= a:
        e += 1
    e_eff = max(e, -126)
    scale = Fraction(2) ** (23 - e_eff)
    m = a * scale
    fl = m.numerator // m.denominator
    rem = m - fl
    if rem > Fraction(1, 2) or (rem == Fraction(1, 2) and fl % 2 == 1):
        fl += 1
    val = Fraction(fl) / scale
    if val >= Fraction(2) ** 128:
        return np.float32(sign * np.inf)
    return np.float32(sign * float(val))


def luminance_px(r, g, b) -> np.float32:
    """Eq. 11 for one pixel, each fused step rounded once: fma(0.0722, B,
    fma(0.7152, G, 0.2126 * R)), with the coefficients taken as FP32."""
    cr, cg, cb = (Fraction(float(np.float32(c))) for c in (0.2126, 0.7152, 0.0722))
    t = round_f32(cr * Fraction(float(r)))
    t = round_f32(cg * Fraction(float(g)) + Fraction(float(t)))
    return round_f32(cb * Fraction(float(b)) + Fraction(float(t)))


def bin_of(v, vmin, vmax, n: int) -> int:
    """Equal-width bin of log(v) over [log vmin, log vmax] (vmin floored at FLT_MIN):
    bin >= k  iff  log v >= log vmin + k/n (log vmax - log vmin)
              iff  v^n >= vmin^(n-k) vmax^k      (exact, for positive values)."""
    a = max(Fraction(float(vmin)), FLT_MIN)
    b = Fraction(float(vmax))
    x = Fraction(float(v))
    if n == 1 or not b > a or x <= 0:
        return 0
    cnt = 0
    xn = x ** n
    for k in range(1, n):
        if xn >= a ** (n - k) * b ** k:
            cnt += 1
    return cnt


def window(x, y, W, H, rx, ry):
    """Clamped receptive field of Algorithm 1: x' in (x-(rx+1), x+rx], y' likewise."""
    x0 = max(x - rx, 0)
    x1 = min(x + rx, W - 1)
    y0 = max(y - ry, 0)
    y1 = min(y + ry, H - 1)
    return x0, x1, y0, y1


def forward(v: np.ndarray, n: int, rx, ry, eps=0.1, ldmin=0.0, ldmax=1.0,
            per_scale=False, var_domain="linear"):
    """Exact L (as Fractions, returned as float64) for a tiny float32 image v [H, W].
    var_domain="log": the window variance is taken of the FP64 natural logarithms
    math.log(max(v, 2^-126)) (exact rational arithmetic from there on)."""
    H, W = v.shape
    vmin, vmax = float(v.min()), float(v.max())
    B = [[bin_of(v[y, x], vmin, vmax, n) for x in range(W)] for y in range(H)]
    if var_domain == "log":
        V = [[Fraction(math.log(max(float(v[y, x]), float(FLT_MIN)))) for x in range(W)]
             for y in range(H)]
    else:
        V = [[Fraction(float(v[y, x])) for x in range(W)] for y in range(H)]
    e = Fraction(float(eps))
    lo, hi = Fraction(float(ldmin)), Fraction(float(ldmax))
    s = len(rx)
    L = np.empty((H, W))
    Ls = np.empty((s, H, W))
    Ws = np.empty((s, H, W))
    for y in range(H):
        for x in range(W):
            b = B[y][x]
            num = den = Fraction(0)
            lsum = Fraction(0)
            for j in range(s):
                x0, x1, y0, y1 = window(x, y, W, H, rx[j], ry[j])
                f = [0] * n
                s1 = s2 = Fraction(0)
                for yy in range(y0, y1 + 1):
                    for xx in range(x0, x1 + 1):
                        f[B[yy][xx]] += 1
                        s1 += V[yy][xx]
                        s2 += V[yy][xx] ** 2
                T = sum(f)                                   # Eq. 1
                P = Fraction(sum(f[:b]), T)
                Lj = lo + (hi - lo) * P                     # Eq. 2
                N = (x1 - x0 + 1) * (y1 - y0 + 1)
                var = s2 / N - (s1 / N) ** 2                 # Eq. 10 (population variance)
                var = max(var, Fraction(0))
                Wj = var / (var + e)                         # Eq. 4
                num += Wj * Lj
                den += Wj
                lsum += Lj
                Ls[j, y, x] = float(Lj)
                Ws[j, y, x] = float(Wj)
            L[y, x] = float(num / den) if den > 0 else float(lsum / s)   # Eq. 3
    return (L, Ls, Ws) if per_scale else L


def window_hist(bins: np.ndarray, n: int, x0, x1, y0, y1):
    """Histogram of the bin map over the inclusive window (direct count)."""
    sub = bins[y0:y1 + 1, x0:x1 + 1].ravel()
    return np.bincount(sub, minlength=n)
