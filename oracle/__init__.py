"""CPU oracle for integral-image / integral-histogram multi-receptive-field tone mapping.

TEST INFRASTRUCTURE ONLY: only the tests, the smoke check and the bench's CPU-baseline leg
may import this package.  It shares no code with the HIP library; the two meet only through
the seeded inputs drawn by ``synth``.

Contents
  * ``exact_edges``: the equal-width log-domain bin edges of Section II-A, computed exactly
    with integer arithmetic (Python's unbounded ints);
  * thin numpy wrappers around the plain C oracle (``tm_oracle.c``): luminance (Eq. 11),
    bins (Eq. 7), integral histogram (Eq. 8), integral images (Eq. 5), the forward method
    (Eq. 1-4, 6, 9, 10) with integral tables or with direct window sums -- with Eq. 10's
    variance taken of the luminance or, as a variant, of its natural logarithm -- the
    backward, colour restoration (Eq. 12);
  * ``paper_radii``: the receptive-field pyramid of Section II-C.
The pure-Python brute force used to pin the C code lives in ``oracle.brute``.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

from . import build as _build

__all__ = [
    "FLT_MIN", "paper_radii", "exact_edges", "luminance", "bins", "integral_histogram",
    "integral_image", "forward", "forward_direct", "backward", "box_filter", "lib",
    "set_threads",
]

FLT_MIN = float(np.finfo(np.float32).tiny)  # 2^-126, smallest normal FP32
_LIB = None


def lib() -> ctypes.CDLL:
    """Load the oracle's C library, compiling it first if it has not been built or is older
    than its source."""
    global _LIB
    if _LIB is None:
        if _build.stale():
            _build.build()
        L = ctypes.CDLL(_build.LIB)
        P = ctypes.c_void_p
        I64 = ctypes.c_int64
        I = ctypes.c_int
        D = ctypes.c_double
        L.orc_luminance.argtypes = [P, I64, I64, P]
        L.orc_bins.argtypes = [P, I64, P, I, P]
        L.orc_integral_histogram.argtypes = [P, I64, I64, I, I, P]
        L.orc_integral_image.argtypes = [P, I64, I64, I, P, P]
        L.orc_forward.argtypes = [P, I64, I64, P, I, I, P, P, D, D, D, I, P, P, P, P]
        L.orc_forward.restype = I
        L.orc_forward_direct.argtypes = [P, I64, I64, P, I, I, P, P, D, D, D, I, P, I64, P]
        L.orc_forward_direct.restype = I
        L.orc_backward.argtypes = [P, I64, I64, P, I, I, P, P, D, D, D, I, P, P, P]
        L.orc_backward.restype = I
        L.orc_box_filter.argtypes = [P, I64, I64, ctypes.c_int32, ctypes.c_int32, P]
        L.orc_box_filter.restype = I
        L.orc_color_restore.argtypes = [P, P, P, I64, I64, D, P]
        L.orc_color_restore.restype = None
        L.orc_set_threads.argtypes = [I]
        L.orc_set_threads.restype = None
        _LIB = L
    return _LIB


def _ptr(a: np.ndarray):
    return ctypes.c_void_p(a.ctypes.data) if a is not None else None


def _c(a, dtype):
    return np.ascontiguousarray(a, dtype=dtype)


def set_threads(n: int) -> None:
    """OpenMP threads of the oracle's per-pixel loops (results do not depend on it)."""
    lib().orc_set_threads(int(n))


# ---------------------------------------------------------------------------- pyramid
def paper_radii(H: int, W: int, s: int):
    """Receptive-field half-widths of Section II-C: the largest field spans the image and
    each next one is half as wide (w_i / w_{i+1} = 2).  Reading: scale j = 1..s has the
    per-axis radius (floor(W / 2^j), floor(H / 2^j)), i.e. a window side of about
    dim / 2^(j-1), with Algorithm 1's separate x and y radii."""
    rx = [W >> j for j in range(1, s + 1)]
    ry = [H >> j for j in range(1, s + 1)]
    return rx, ry


# ---------------------------------------------------------------------------- edges
def _ratio(f) -> tuple[int, int]:
    return float(f).as_integer_ratio()


def _pow_ge(c, n, num_t, den_t) -> bool:
    """c^n >= num_t / den_t, exactly."""
    cn, cd = _ratio(c)
    return cn ** n * den_t >= num_t * cd ** n


def exact_edges(lum_min, lum_max, n: int) -> np.ndarray:
    """Bin edges for n equal-width bins of l = log(i) over [log i_min, log i_max]
    (Section II-A: the log image is divided into n bins by value, Eq. 7).

    Readings: the range is the image's own [min, max]; i_min is floored at the smallest
    normal FP32 so the logarithm is defined; bins are half-open.  Edge k (k = 1..n-1) sits
    at log i_min + k/n (log i_max - log i_min), i.e. at the real number
    e_k = i_min^(1-k/n) i_max^(k/n), so a pixel is in a bin >= k exactly when i >= e_k.
    For FP32 pixels that test equals i >= c_k with c_k the smallest FP32 >= e_k, which is
    what is returned: c_k is the least FP32 with c_k^n >= i_min^(n-k) i_max^k, found with
    exact integer arithmetic.  If i_max <= i_min every edge is +inf (one bin)."""
    if n < 1:
        raise ValueError("n must be >= 1")
    a = np.float32(max(float(np.float32(lum_min)), FLT_MIN))
    b = np.float32(lum_max)
    out = np.full(max(n - 1, 0), np.inf, dtype=np.float32)
    if n == 1 or not (float(b) > float(a)):
        return out
    an, ad = _ratio(a)
    bn, bd = _ratio(b)
    la, lb = np.log(float(a)), np.log(float(b))
    for k in range(1, n):
        num_t = an ** (n - k) * bn ** k
        den_t = ad ** (n - k) * bd ** k
        c = np.float32(np.exp(la + (k / n) * (lb - la)))
        if not np.isfinite(c):
            c = np.float32(b)
        while not _pow_ge(c, n, num_t, den_t):
            c = np.nextafter(c, np.float32(np.inf))
        while True:
            p = np.nextafter(c, np.float32(-np.inf))
            if p > 0 and _pow_ge(p, n, num_t, den_t):
                c = p
            else:
                break
        out[k - 1] = c
    return out


# ---------------------------------------------------------------------------- C wrappers
def luminance(rgb: np.ndarray) -> np.ndarray:
    """Eq. 11 on planar float32 RGB [3, H, W] -> float32 [H, W]."""
    rgb = _c(rgb, np.float32)
    _, H, W = rgb.shape
    out = np.empty((H, W), dtype=np.float32)
    lib().orc_luminance(_ptr(rgb), H, W, _ptr(out))
    return out


def bins(lum: np.ndarray, edges: np.ndarray) -> np.ndarray:
    """Eq. 7 bin index of every pixel (int32, same shape as lum)."""
    lum = _c(lum, np.float32)
    edges = _c(edges, np.float32)
    n = edges.size + 1
    out = np.empty(lum.shape, dtype=np.int32)
    lib().orc_bins(_ptr(lum), lum.size, _ptr(edges) if edges.size else None, n, _ptr(out))
    return out


def integral_histogram(b: np.ndarray, n: int, cumulative: bool = False) -> np.ndarray:
    """Eq. 8 tables: uint64 [planes, H+1, W+1] with zero row 0 / column 0.  Per-bin planes
    H_k (k = 0..n-1) or cumulative planes G_k = sum_{j<k} H_j (k = 1..n-1)."""
    b = _c(b, np.int32)
    H, W = b.shape
    planes = n - 1 if cumulative else n
    out = np.empty((planes, H + 1, W + 1), dtype=np.uint64)
    lib().orc_integral_histogram(_ptr(b), H, W, n, int(cumulative), _ptr(out))
    return out


def integral_image(v: np.ndarray, square: bool = False):
    """Eq. 5 table of v (or v^2) in double-double: (hi, lo) float64 [H+1, W+1]."""
    v = _c(v, np.float32)
    H, W = v.shape
    hi = np.empty((H + 1, W + 1), dtype=np.float64)
    lo = np.empty((H + 1, W + 1), dtype=np.float64)
    lib().orc_integral_image(_ptr(v), H, W, int(square), _ptr(hi), _ptr(lo))
    return hi, lo


def _radii(rx, ry):
    rx = np.ascontiguousarray(rx, dtype=np.int32)
    ry = np.ascontiguousarray(ry, dtype=np.int32)
    if rx.shape != ry.shape or rx.ndim != 1 or not (1 <= rx.size <= 16):
        raise ValueError("rx, ry must be equal-length 1-D sequences of 1..16 radii")
    return rx, ry


VAR_DOMAINS = ("linear", "log")


def _var_log(var_domain: str) -> int:
    if var_domain not in VAR_DOMAINS:
        raise ValueError(f"var_domain must be one of {VAR_DOMAINS}")
    return int(var_domain == "log")


def forward(v, edges, rx, ry, eps=0.1, ldmin=0.0, ldmax=1.0, per_scale=False,
            var_domain="linear"):
    """Tone-mapped luminance L (float64 [H, W]) by Eq. 1-10 with integral tables.
    With per_scale=True also returns (L_j, W_j, var_j), each float64 [s, H, W].
    var_domain="log": Eq. 10's window variance is that of l = ln(max(v, FLT_MIN)), in FP64,
    instead of v itself (the bins still come from v)."""
    v = _c(v, np.float32)
    edges = _c(edges, np.float32)
    rx, ry = _radii(rx, ry)
    H, W = v.shape
    s = rx.size
    L = np.empty((H, W), dtype=np.float64)
    extra = [np.empty((s, H, W), dtype=np.float64) for _ in range(3)] if per_scale else None
    ptrs = [_ptr(e) for e in extra] if extra else [None, None, None]
    rc = lib().orc_forward(_ptr(v), H, W, _ptr(edges) if edges.size else None,
                           edges.size + 1, s, _ptr(rx), _ptr(ry), float(eps), float(ldmin),
                           float(ldmax), _var_log(var_domain), _ptr(L), *ptrs)
    if rc != 0:
        raise MemoryError("oracle forward: allocation failed")
    return (L, *extra) if per_scale else L


def forward_direct(v, edges, rx, ry, pix, eps=0.1, ldmin=0.0, ldmax=1.0, var_domain="linear"):
    """L at the flat pixel indices pix, with window histograms and sums taken directly."""
    v = _c(v, np.float32)
    edges = _c(edges, np.float32)
    rx, ry = _radii(rx, ry)
    pix = _c(pix, np.int64)
    H, W = v.shape
    L = np.empty(pix.size, dtype=np.float64)
    rc = lib().orc_forward_direct(_ptr(v), H, W, _ptr(edges) if edges.size else None,
                                  edges.size + 1, rx.size, _ptr(rx), _ptr(ry), float(eps),
                                  float(ldmin), float(ldmax), _var_log(var_domain), _ptr(pix),
                                  pix.size, _ptr(L))
    if rc != 0:
        raise MemoryError("oracle forward_direct: allocation failed")
    return L


def backward(v, edges, rx, ry, g, eps=0.1, ldmin=0.0, ldmax=1.0, var_domain="linear"):
    """(dv float64 [H, W], (d eps, d min L_d, d max L_d)) of sum(g * L).  var_domain="log":
    the gradient of the log-domain variant (forward's var_domain="log"), through
    l = ln(max(v, FLT_MIN)); zero where the floor is taken."""
    v = _c(v, np.float32)
    edges = _c(edges, np.float32)
    rx, ry = _radii(rx, ry)
    g = _c(g, np.float64)
    H, W = v.shape
    if g.shape != (H, W):
        raise ValueError("g must have the image's shape")
    dv = np.empty((H, W), dtype=np.float64)
    gp = np.empty(3, dtype=np.float64)
    rc = lib().orc_backward(_ptr(v), H, W, _ptr(edges) if edges.size else None,
                            edges.size + 1, rx.size, _ptr(rx), _ptr(ry), float(eps),
                            float(ldmin), float(ldmax), _var_log(var_domain), _ptr(g), _ptr(dv),
                            _ptr(gp))
    if rc != 0:
        raise MemoryError("oracle backward: allocation failed")
    return dv, tuple(float(x) for x in gp)


def box_filter(a, rx: int, ry: int):
    """Clamped box sum of a float64 plane at every pixel (window of Algorithm 1)."""
    a = _c(a, np.float64)
    H, W = a.shape
    out = np.empty((H, W), dtype=np.float64)
    if lib().orc_box_filter(_ptr(a), H, W, int(rx), int(ry), _ptr(out)) != 0:
        raise MemoryError("oracle box_filter: allocation failed")
    return out


def color_restore(rgb, lum, L, sat: float = 0.6) -> np.ndarray:
    """Eq. 12 (Section II-D): out_c = (c / v)^sat * L for c = R, G, B, in FP64 (planar
    [3, H, W]); channels below 0 count as 0 and the ratio is 1 where v == 0."""
    rgb = _c(rgb, np.float32)
    lum = _c(lum, np.float32)
    L = _c(L, np.float64)
    H, W = lum.shape
    out = np.empty((3, H, W), dtype=np.float64)
    lib().orc_color_restore(_ptr(rgb), _ptr(lum), _ptr(L), H, W, float(sat), _ptr(out))
    return out
