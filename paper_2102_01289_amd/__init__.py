"""MI355X (gfx950) multi-receptive-field local tone mapping with integral images and
integral histograms (arXiv 2102.01289), behind a C ABI (include/tm.h).

This module is the thin Python binding: it marshals torch device tensors into the C entry
points of the same names and allocates outputs.  Every step of the method runs in the HIP
kernels of libtm355.so; there is no host or PyTorch fallback, and a missing library raises.
"""
from __future__ import annotations

import ctypes
from dataclasses import dataclass

import torch

from . import _capi

__all__ = [
    "TmError", "Table", "table_geometry", "paper_radii", "make_params", "tune", "default_tune",
    "image_tune", "tm_integral_histogram_lookback", "tm_log_luminance_backward",
    "tm_luminance", "tm_image_stats", "tm_prologue", "tm_prologue_log", "tm_integral_image",
    "tm_integral_histogram", "tm_integral_tables", "tm_integral_tables_split",
    "tm_integral_tables_log",
    "tm_tonemap_forward",
    "tm_tonemap_backward", "tm_tonemap_forward_train", "tm_tonemap_backward_resid",
    "tm_tonemap_backward_resid_log", "tm_tonemap_backward_log",
    "residual_planes", "residual_pairs", "ToneMapper", "tonemap", "Batch",
    "tm_tonemap_forward_rgb", "tonemap_rgb", "tm_tonemap_forward_maps", "tm_prologue_noalloc",
]


class TmError(RuntimeError):
    def __init__(self, name: str, status: int):
        self.status = status
        msg = _capi.load().tm_status_string(status).decode()
        super().__init__(f"{name}: {_capi.STATUS.get(status, status)} ({msg})")


def _ck(name: str, status: int) -> None:
    if status != 0:
        raise TmError(name, status)


def _lib():
    return _capi.load()


def _vp(t) -> ctypes.c_void_p:
    if t is None:
        return ctypes.c_void_p(0)
    if isinstance(t, int):
        return ctypes.c_void_p(t)
    return ctypes.c_void_p(t.data_ptr())


def _stream(stream=None) -> ctypes.c_void_p:
    s = stream if stream is not None else torch.cuda.current_stream()
    return ctypes.c_void_p(s.cuda_stream)


def _img(t: torch.Tensor, name: str):
    if t.dtype != torch.float32 or t.dim() != 2 or t.stride(1) != 1 or not t.is_cuda:
        raise ValueError(f"{name} must be a CUDA float32 [H, W] tensor with unit column stride")
    return t.shape[0], t.shape[1], t.stride(0)


def _ws(nbytes: int, device) -> torch.Tensor:
    return torch.empty(max(int(nbytes), 1), dtype=torch.uint8, device=device)


# ------------------------------------------------------------------------ parameters
def table_geometry(H: int, W: int):
    ld, org, el = ctypes.c_int64(), ctypes.c_int64(), ctypes.c_int64()
    _ck("tm_table_geometry", _lib().tm_table_geometry(H, W, ctypes.byref(ld), ctypes.byref(org),
                                                       ctypes.byref(el)))
    return ld.value, org.value, el.value


def paper_radii(H: int, W: int, s: int):
    p = _capi.TmParams()
    p.n_scales = s
    _ck("tm_paper_radii", _lib().tm_paper_radii(H, W, ctypes.byref(p)))
    return list(p.rx[:s]), list(p.ry[:s])


def make_params(n_bins: int = 5, n_scales: int = 5, rx=None, ry=None, eps: float = 0.1,
                ld_min: float = 0.0, ld_max: float = 1.0, H: int | None = None,
                W: int | None = None, scalars=None) -> _capi.TmParams:
    """tm_params; radii default to the paper's pyramid for an H x W image.  scalars: a device
    float32 tensor [3] = (eps, ld_min, ld_max) the kernels read at run time instead of the
    eps, ld_min, ld_max arguments (the caller keeps it alive while launches use it)."""
    p = _capi.TmParams()
    p.n_bins = n_bins
    p.n_scales = n_scales
    if rx is None or ry is None:
        if H is None or W is None:
            raise ValueError("give rx, ry or the image size H, W")
        rx, ry = paper_radii(H, W, n_scales)
    if len(rx) != n_scales or len(ry) != n_scales:
        raise ValueError("rx, ry must have n_scales entries")
    for j in range(n_scales):
        p.rx[j] = int(rx[j])
        p.ry[j] = int(ry[j])
    p.eps = eps
    p.ld_min = ld_min
    p.ld_max = ld_max
    if scalars is not None:
        if (scalars.dtype != torch.float32 or scalars.numel() != 3 or not scalars.is_cuda
                or not scalars.is_contiguous()):
            raise ValueError("scalars must be a contiguous CUDA float32 tensor of 3 values")
        p.scalars = scalars.data_ptr()
    return p


def tune(tile_w_vec: int, tile_h: int, bin_chunk: int) -> _capi.TmTune:
    return _capi.TmTune(tile_w_vec, tile_h, bin_chunk)


def default_tune(H: int, W: int, n_bins: int = 5) -> _capi.TmTune:
    """The scan tiling an H x W image with an n_bins-bin histogram gets by default
    (tm_default_tune)."""
    t = _capi.TmTune()
    _ck("tm_default_tune", _lib().tm_default_tune(H, W, n_bins, ctypes.byref(t)))
    return t


def image_tune(t, H: int, W: int, n_bins: int = 5) -> _capi.TmTune:
    """A batch tiling as one image of shape H x W (n_bins bins) uses it: 0 fields take the
    image's default."""
    d = default_tune(H, W, n_bins)
    if t is None:
        return d
    return _capi.TmTune(t.tile_w_vec or d.tile_w_vec, t.tile_h or d.tile_h, t.bin_chunk)


# ------------------------------------------------------------------------ tables
_KIND = {"f32": (2, torch.float32), "c32x2": (4, torch.float32), "f64": (2, torch.float64),
         "u32": (1, torch.uint32)}


class Table:
    """One or more integral tables of an H x W image in the library's table layout
    (origin pointer, row pitch ld >= W+1, zero row -1 and column -1), on a CUDA device."""

    def __init__(self, H: int, W: int, kind: str, planes: int = 1, device="cuda"):
        comps, dtype = _KIND[kind]
        self.H, self.W, self.kind, self.planes, self.comps = H, W, kind, planes, comps
        self.ld, self.origin, self.elems = table_geometry(H, W)
        self.buf = torch.empty(max(planes, 1) * self.elems * comps, dtype=dtype, device=device)
        self.itemsize = self.buf.element_size() * comps
        self.plane_stride = self.elems

    @property
    def ptr(self) -> int:
        return self.buf.data_ptr() + self.origin * self.itemsize

    def padded(self) -> torch.Tensor:
        """[planes, H+1, W+1, comps] with entry [p, y+1, x+1] = T_p(x, y) and the zero
        border at index 0 -- the oracle's layout -- copied to the host."""
        b = self.buf.view(max(self.planes, 1), self.elems, self.comps)
        lo = self.origin - self.ld
        rows = b[:, lo:lo + (self.H + 1) * self.ld].reshape(-1, self.H + 1, self.ld, self.comps)
        out = torch.empty((rows.shape[0], self.H + 1, self.W + 1, self.comps), dtype=b.dtype)
        r = rows.cpu()
        out[:, :, 1:] = r[:, :, :self.W]
        out[:, 1:, 0] = r[:, :-1, self.ld - 1]          # x = -1 of row y is column ld-1 of row y-1
        out[:, 0, 0] = b[:, lo - 1].cpu()               # (x, y) = (-1, -1)
        return out

    def raw_region(self) -> torch.Tensor:
        """Everything the producing call must write: [planes, (H+1)*ld + 1, comps]."""
        b = self.buf.view(max(self.planes, 1), self.elems, self.comps)
        lo = self.origin - self.ld - 1
        return b[:, lo:self.origin + self.H * self.ld]


# ------------------------------------------------------------------------ entry points
def tm_luminance(rgb: torch.Tensor, lum: torch.Tensor | None = None, stream=None):
    """Eq. 11 on planar float32 RGB [3, H, W] (CUDA) -> luminance [H, W]."""
    if rgb.dtype != torch.float32 or rgb.dim() != 3 or rgb.shape[0] != 3 or rgb.stride(2) != 1:
        raise ValueError("rgb must be float32 [3, H, W] with unit column stride")
    _, H, W = rgb.shape
    if lum is None:
        lum = torch.empty((H, W), dtype=torch.float32, device=rgb.device)
    _ck("tm_luminance", _lib().tm_luminance(_vp(rgb), rgb.stride(0), rgb.stride(1), H, W,
                                            _vp(lum), lum.stride(0), _stream(stream)))
    return lum


def tm_image_stats(lum: torch.Tensor, n_bins: int, stream=None):
    """(edges [n_bins-1], offsets [2], minmax [2]) of a luminance image."""
    H, W, ld = _img(lum, "lum")
    dev = lum.device
    edges = torch.empty(max(n_bins - 1, 1), dtype=torch.float32, device=dev)
    offsets = torch.empty(2, dtype=torch.float32, device=dev)
    minmax = torch.empty(2, dtype=torch.float32, device=dev)
    nb = _lib().tm_image_stats_workspace_bytes(H, W)
    ws = _ws(nb, dev)
    _ck("tm_image_stats", _lib().tm_image_stats(_vp(lum), ld, H, W, n_bins, _vp(edges),
                                                _vp(offsets), _vp(minmax), _vp(ws), ws.numel(),
                                                _stream(stream)))
    return edges[:n_bins - 1], offsets, minmax


def tm_log_luminance(lum: torch.Tensor, stream=None, out=None, offsets=None, minmax=None,
                     ws=None, write_plane: bool = True):
    """Log image l = ln(max(lum, FLT_MIN)) and its statistics: (l [H, W], offsets [2] =
    FP32 means of l and l^2, minmax [2]); l is None when write_plane is False (the
    statistics only)."""
    H, W, ld = _img(lum, "lum")
    dev = lum.device
    if out is None and write_plane:
        out = torch.empty((H, W), dtype=torch.float32, device=dev)
    if offsets is None:
        offsets = torch.empty(2, dtype=torch.float32, device=dev)
    if minmax is None:
        minmax = torch.empty(2, dtype=torch.float32, device=dev)
    if ws is None:
        ws = _ws(_lib().tm_image_stats_workspace_bytes(H, W), dev)
    ldo = _img(out, "out")[2] if out is not None else 0
    _ck("tm_log_luminance", _lib().tm_log_luminance(
        _vp(lum), ld, H, W, _vp(out), ldo, _vp(offsets), _vp(minmax), _vp(ws), ws.numel(),
        _stream(stream)))
    return out, offsets, minmax


def tm_log_luminance_backward(lum: torch.Tensor, grad_l: torch.Tensor, out=None, stream=None):
    """Chain rule through l = ln(max(lum, FLT_MIN)): grad_l / lum above the floor, 0 where
    the floor is taken.  out may be grad_l itself (in place)."""
    H, W, ld = _img(lum, "lum")
    _, _, ldg = _img(grad_l, "grad_l")
    if out is None:
        out = torch.empty((H, W), dtype=torch.float32, device=lum.device)
    _, _, ldo = _img(out, "out")
    _ck("tm_log_luminance_backward", _lib().tm_log_luminance_backward(
        _vp(lum), ld, H, W, _vp(grad_l), ldg, _vp(out), ldo, _stream(stream)))
    return out


def _stack(stack: torch.Tensor):
    if (stack.dtype != torch.uint8 or stack.dim() != 4 or stack.shape[1] != 3
            or stack.stride(3) != 1 or not stack.is_cuda):
        raise ValueError("stack must be a CUDA uint8 [P, 3, H, W] tensor with unit column stride")
    P, _, H, W = stack.shape
    return P, H, W, stack.stride(0), stack.stride(1), stack.stride(2)


def _check_log_dt(log_dt, P):
    if log_dt.dtype != torch.float32 or log_dt.numel() != P or not log_dt.is_contiguous():
        raise ValueError("log_dt must be a contiguous float32 vector with one entry per exposure")


def tm_hdr_response(stack: torch.Tensor, log_dt: torch.Tensor, samples: torch.Tensor,
                    lam: float = 100.0, g=None, ws=None, stream=None) -> torch.Tensor:
    """Inverse log camera responses g [3, 256] (FP32, g[:, 128] = 0) from the pixels at the
    flat indices `samples` (int32) of an exposure stack [P, 3, H, W] with log times log_dt."""
    P, H, W, es, cs, ld = _stack(stack)
    dev = stack.device
    if samples.dtype != torch.int32 or samples.dim() != 1 or not samples.is_contiguous():
        raise ValueError("samples must be a contiguous int32 vector of flat pixel indices")
    _check_log_dt(log_dt, P)
    if g is None:
        g = torch.empty((3, 256), dtype=torch.float32, device=dev)
    if ws is None:
        ws = _ws(_lib().tm_hdr_response_workspace_bytes(), dev)
    _ck("tm_hdr_response", _lib().tm_hdr_response(
        _vp(stack), es, cs, ld, P, H, W, _vp(samples), samples.numel(), _vp(log_dt),
        float(lam), _vp(g), _vp(ws), ws.numel(), _stream(stream)))
    return g


def tm_hdr_merge(stack: torch.Tensor, log_dt: torch.Tensor, g: torch.Tensor, out=None,
                 stream=None) -> torch.Tensor:
    """Radiance map E [3, H, W] (FP32, planar) of an exposure stack [P, 3, H, W]."""
    P, H, W, es, cs, ld = _stack(stack)
    _check_log_dt(log_dt, P)
    if g.dtype != torch.float32 or tuple(g.shape) != (3, 256) or not g.is_contiguous():
        raise ValueError("g must be a contiguous float32 [3, 256] tensor")
    if out is None:
        out = torch.empty((3, H, W), dtype=torch.float32, device=stack.device)
    _ck("tm_hdr_merge", _lib().tm_hdr_merge(
        _vp(stack), es, cs, ld, P, H, W, _vp(log_dt), _vp(g), _vp(out), out.stride(0),
        out.stride(1), _stream(stream)))
    return out


def tm_prologue(rgb: torch.Tensor, n_bins: int, stream=None):
    """Eq. 11 and the image statistics in one pass: (lum, edges, offsets, minmax)."""
    _, H, W = rgb.shape
    dev = rgb.device
    lum = torch.empty((H, W), dtype=torch.float32, device=dev)
    edges = torch.empty(max(n_bins - 1, 1), dtype=torch.float32, device=dev)
    offsets = torch.empty(2, dtype=torch.float32, device=dev)
    minmax = torch.empty(2, dtype=torch.float32, device=dev)
    ws = _ws(_lib().tm_image_stats_workspace_bytes(H, W), dev)
    _ck("tm_prologue", _lib().tm_prologue(_vp(rgb), rgb.stride(0), rgb.stride(1), H, W, n_bins,
                                          _vp(lum), lum.stride(0), _vp(edges), _vp(offsets),
                                          _vp(minmax), _vp(ws), ws.numel(), _stream(stream)))
    return lum, edges[:n_bins - 1], offsets, minmax


def tm_prologue_log(rgb: torch.Tensor, n_bins: int, stream=None, write_log: bool = True):
    """Log-domain variant's prologue in one pass: (lum, logv, edges, log_offsets, minmax),
    equal to tm_prologue's lum, edges, minmax and tm_log_luminance's plane and offsets
    (logv is None when write_log is False: only its offsets are formed)."""
    _check_rgb(rgb)
    _, H, W = rgb.shape
    dev = rgb.device
    lum = torch.empty((H, W), dtype=torch.float32, device=dev)
    logv = torch.empty((H, W), dtype=torch.float32, device=dev) if write_log else None
    edges = torch.empty(max(n_bins - 1, 1), dtype=torch.float32, device=dev)
    offsets = torch.empty(2, dtype=torch.float32, device=dev)
    minmax = torch.empty(2, dtype=torch.float32, device=dev)
    ws = _ws(_lib().tm_image_stats_workspace_bytes(H, W), dev)
    _ck("tm_prologue_log", _lib().tm_prologue_log(
        _vp(rgb), rgb.stride(0), rgb.stride(1), H, W, n_bins, _vp(lum), lum.stride(0),
        _vp(logv), logv.stride(0) if write_log else 0, _vp(edges), _vp(offsets), _vp(minmax),
        _vp(ws), ws.numel(), _stream(stream)))
    return lum, logv, edges[:n_bins - 1], offsets, minmax


def tm_prologue_noalloc(rgb: torch.Tensor, n_bins: int, lum=None, edges=None, offsets=None,
                        minmax=None, stream=None):
    """tm_prologue with no workspace (its partials live in the library's static device
    array): (lum, edges, offsets, minmax).  Outputs may be passed in preallocated."""
    _check_rgb(rgb)
    _, H, W = rgb.shape
    dev = rgb.device
    if lum is None:
        lum = torch.empty((H, W), dtype=torch.float32, device=dev)
    if edges is None:
        edges = torch.empty(max(n_bins - 1, 1), dtype=torch.float32, device=dev)
    if offsets is None:
        offsets = torch.empty(2, dtype=torch.float32, device=dev)
    if minmax is None:
        minmax = torch.empty(2, dtype=torch.float32, device=dev)
    _ck("tm_prologue_noalloc", _lib().tm_prologue_noalloc(
        _vp(rgb), rgb.stride(0), rgb.stride(1), H, W, n_bins, _vp(lum), lum.stride(0),
        _vp(edges), _vp(offsets), _vp(minmax), _stream(stream)))
    return lum, edges[:n_bins - 1], offsets, minmax


def _tune_ref(t):
    return ctypes.byref(t) if t is not None else None


def tm_integral_tables(v: torch.Tensor, prec: str | None = "c32x2", offsets=None, edges=None,
                       n_bins: int = 5, layout: str | None = "cumulative", tune=None,
                       stream=None, sat: Table | None = None, hist: Table | None = None):
    """Integral image (prec, or None to skip) and integral histogram (layout, or None to
    skip) of v in one pass.  Returns (sat Table | None, hist Table | None); preallocated
    tables may be passed in."""
    H, W, ld = _img(v, "v")
    dev = v.device
    if sat is None and prec is not None:
        sat = Table(H, W, prec, 1, dev)
    if hist is None and layout is not None:
        planes = n_bins if layout == "per_bin" else n_bins - 1
        hist = Table(H, W, "u32", planes, dev) if planes > 0 else None
    if sat is None and hist is None:
        return None, None
    pcode = _capi.SAT_PREC[prec] if prec is not None else 0
    nbytes = _lib().tm_tables_workspace_bytes(H, W, n_bins, pcode, _tune_ref(tune))
    ws = _ws(nbytes, dev)
    st = _lib().tm_integral_tables(
        _vp(v), ld, H, W, pcode, _vp(offsets), _vp(sat.ptr if sat else None),
        sat.ld if sat else 0, _vp(edges), n_bins, _capi.HIST_LAYOUT[layout or "cumulative"],
        _vp(hist.ptr if hist else None), hist.ld if hist else 0,
        hist.plane_stride if hist else 0, _tune_ref(tune), _vp(ws), ws.numel(), _stream(stream))
    _ck("tm_integral_tables", st)
    return sat, hist


def tm_integral_tables_split(v_sat: torch.Tensor, v_hist: torch.Tensor, prec: str = "c32x2",
                             offsets=None, edges=None, n_bins: int = 5,
                             layout: str = "cumulative", tune=None, stream=None,
                             sat: Table | None = None, hist: Table | None = None):
    """Integral image of v_sat (prec) and integral histogram of v_hist's bins (layout) in one
    pass: the log-domain variant's tables (statistics of ln i, bins of i).  Returns (sat,
    hist); n_bins must leave at least one plane."""
    H, W, ld = _img(v_sat, "v_sat")
    Hh, Wh, ldh = _img(v_hist, "v_hist")
    if (Hh, Wh) != (H, W):
        raise ValueError("v_sat and v_hist must have the same shape")
    dev = v_sat.device
    sat = sat if sat is not None else Table(H, W, prec, 1, dev)
    planes = n_bins if layout == "per_bin" else n_bins - 1
    if hist is None:
        if planes < 1:
            raise ValueError("the histogram needs at least one plane")
        hist = Table(H, W, "u32", planes, dev)
    pcode = _capi.SAT_PREC[prec]
    ws = _ws(_lib().tm_tables_workspace_bytes(H, W, n_bins, pcode, _tune_ref(tune)), dev)
    _ck("tm_integral_tables_split", _lib().tm_integral_tables_split(
        _vp(v_sat), ld, _vp(v_hist), ldh, H, W, pcode, _vp(offsets), _vp(sat.ptr), sat.ld,
        _vp(edges), n_bins, _capi.HIST_LAYOUT[layout], _vp(hist.ptr), hist.ld,
        hist.plane_stride, _tune_ref(tune), _vp(ws), ws.numel(), _stream(stream)))
    return sat, hist


def tm_integral_tables_log(lum: torch.Tensor, prec: str = "c32x2", log_offsets=None,
                           edges=None, n_bins: int = 5, layout: str | None = "cumulative",
                           tune=None, stream=None, sat: Table | None = None,
                           hist: Table | None = None):
    """The log-domain variant's tables from lum alone: integral image of
    l = ln max(lum, FLT_MIN) (formed on load) and integral histogram of lum's bins (layout,
    or None to skip).  Returns (sat, hist | None)."""
    H, W, ld = _img(lum, "lum")
    dev = lum.device
    sat = sat if sat is not None else Table(H, W, prec, 1, dev)
    if hist is None and layout is not None:
        planes = n_bins if layout == "per_bin" else n_bins - 1
        hist = Table(H, W, "u32", planes, dev) if planes > 0 else None
    pcode = _capi.SAT_PREC[prec]
    ws = _ws(_lib().tm_tables_workspace_bytes(H, W, n_bins, pcode, _tune_ref(tune)), dev)
    _ck("tm_integral_tables_log", _lib().tm_integral_tables_log(
        _vp(lum), ld, H, W, pcode, _vp(log_offsets), _vp(sat.ptr), sat.ld, _vp(edges), n_bins,
        _capi.HIST_LAYOUT[layout or "cumulative"], _vp(hist.ptr if hist else None),
        hist.ld if hist else 0, hist.plane_stride if hist else 0, _tune_ref(tune), _vp(ws),
        ws.numel(), _stream(stream)))
    return sat, hist


def tm_integral_image(v, prec="c32x2", offsets=None, tune=None, stream=None) -> Table:
    H, W, ld = _img(v, "v")
    sat = Table(H, W, prec, 1, v.device)
    pcode = _capi.SAT_PREC[prec]
    ws = _ws(_lib().tm_tables_workspace_bytes(H, W, 1, pcode, _tune_ref(tune)), v.device)
    _ck("tm_integral_image", _lib().tm_integral_image(
        _vp(v), ld, H, W, pcode, _vp(offsets), _vp(sat.ptr), sat.ld, _tune_ref(tune), _vp(ws),
        ws.numel(), _stream(stream)))
    return sat


def tm_integral_histogram(v, edges, n_bins: int, layout="cumulative", tune=None,
                          stream=None) -> Table:
    H, W, ld = _img(v, "v")
    planes = n_bins if layout == "per_bin" else n_bins - 1
    hist = Table(H, W, "u32", planes, v.device)
    ws = _ws(_lib().tm_tables_workspace_bytes(H, W, n_bins, 0, _tune_ref(tune)), v.device)
    _ck("tm_integral_histogram", _lib().tm_integral_histogram(
        _vp(v), ld, H, W, _vp(edges), n_bins, _capi.HIST_LAYOUT[layout], _vp(hist.ptr),
        hist.ld, hist.plane_stride, _tune_ref(tune), _vp(ws), ws.numel(), _stream(stream)))
    return hist


def tm_integral_histogram_lookback(v, edges, n_bins: int, layout="cumulative", hist=None,
                                   ws=None, stream=None):
    """The integral histogram in one pass with decoupled look-back (up to 8 planes):
    (hist Table, workspace).  Word 1 of the workspace (its status) reads 0 after the pass, or
    1 if a wait for another tile's record ran out."""
    H, W, ld = _img(v, "v")
    planes = n_bins if layout == "per_bin" else n_bins - 1
    if hist is None:
        hist = Table(H, W, "u32", planes, v.device)
    if ws is None:
        ws = _ws(_lib().tm_lookback_workspace_bytes(H, W, n_bins, _capi.HIST_LAYOUT[layout]),
                 v.device)
    _ck("tm_integral_histogram_lookback", _lib().tm_integral_histogram_lookback(
        _vp(v), ld, H, W, _vp(edges), n_bins, _capi.HIST_LAYOUT[layout], _vp(hist.ptr),
        hist.ld, hist.plane_stride, _vp(ws), ws.numel(), _stream(stream)))
    return hist, ws


def tm_tonemap_forward(v, sat: Table, hist: Table | None, edges, params, offsets=None,
                       out=None, stream=None):
    """Fused per-pixel query and blend (Eq. 1-4, 6, 9, 10, fusion Eq. 3) -> L [H, W]."""
    H, W, ld = _img(v, "v")
    if out is None:
        out = torch.empty((H, W), dtype=torch.float32, device=v.device)
    _ck("tm_tonemap_forward", _lib().tm_tonemap_forward(
        _vp(v), ld, H, W, _vp(sat.ptr), sat.ld, _capi.SAT_PREC[sat.kind], _vp(offsets),
        _vp(hist.ptr if hist else None), hist.ld if hist else 0,
        hist.plane_stride if hist else 0, _vp(edges), ctypes.byref(params), _vp(out),
        out.stride(0), _stream(stream)))
    return out


def tm_tonemap_forward_maps(v, sat: Table, hist: Table | None, edges, params, offsets=None,
                            out=None, maps=None, stream=None):
    """Forward plus the per-field maps of Fig. 3: (L [H, W], maps [2s, H, W]) with the tone
    values L_j (Eq. 2) in maps[:s] and the weights W_j (Eq. 4) in maps[s:]."""
    H, W, ld = _img(v, "v")
    s = params.n_scales
    if out is None:
        out = torch.empty((H, W), dtype=torch.float32, device=v.device)
    if maps is None:
        maps = torch.empty((2 * s, H, W), dtype=torch.float32, device=v.device)
    if tuple(maps.shape) != (2 * s, H, W) or not maps.is_contiguous():
        raise ValueError(f"maps must be a contiguous [{2 * s}, {H}, {W}] tensor")
    _ck("tm_tonemap_forward_maps", _lib().tm_tonemap_forward_maps(
        _vp(v), ld, H, W, _vp(sat.ptr), sat.ld, _capi.SAT_PREC[sat.kind], _vp(offsets),
        _vp(hist.ptr if hist else None), hist.ld if hist else 0,
        hist.plane_stride if hist else 0, _vp(edges), ctypes.byref(params), _vp(out),
        out.stride(0), _vp(maps), _stream(stream)))
    return out, maps


def _check_rgb(rgb, H=None, W=None):
    if rgb.dtype != torch.float32 or rgb.dim() != 3 or rgb.shape[0] != 3 or \
            rgb.stride(2) != 1 or not rgb.is_cuda:
        raise ValueError("rgb must be a CUDA float32 planar [3, H, W] tensor with unit column "
                         "stride")
    if H is not None and tuple(rgb.shape[1:]) != (H, W):
        raise ValueError(f"rgb is {tuple(rgb.shape[1:])}, expected {(H, W)}")


def tm_tonemap_forward_rgb(v, sat: Table, hist: Table | None, edges, params, rgb,
                           saturation: float = 0.6, offsets=None, rgb_out=None, out=None,
                           stream=None):
    """Fused query and colour restoration (Eq. 12): rgb_out [3, H, W] = (rgb / v)^saturation
    * L; L is also written to `out` when given."""
    H, W, ld = _img(v, "v")
    _check_rgb(rgb, H, W)
    if rgb_out is None:
        rgb_out = torch.empty((3, H, W), dtype=torch.float32, device=v.device)
    _check_rgb(rgb_out, H, W)
    _ck("tm_tonemap_forward_rgb", _lib().tm_tonemap_forward_rgb(
        _vp(v), ld, H, W, _vp(sat.ptr), sat.ld, _capi.SAT_PREC[sat.kind], _vp(offsets),
        _vp(hist.ptr if hist else None), hist.ld if hist else 0,
        hist.plane_stride if hist else 0, _vp(edges), ctypes.byref(params), _vp(rgb),
        rgb.stride(0), rgb.stride(1), float(saturation), _vp(rgb_out), rgb_out.stride(0),
        rgb_out.stride(1), _vp(out), out.stride(0) if out is not None else 0, _stream(stream)))
    return rgb_out


def tonemap_rgb(rgb: torch.Tensor, n_bins: int = 5, n_scales: int = 5, eps: float = 0.1,
                prec: str = "c32x2", saturation: float = 0.6, ld_min: float = 0.0,
                ld_max: float = 1.0, rgb_out=None, stream=None,
                variance: str = "linear") -> torch.Tensor:
    """The whole path RGB -> RGB on one planar image (tm_tonemap_rgb): Eq. 11 luminance and
    bin edges, integral tables, fused query with colour restoration (Eq. 12).  variance="log":
    the log-domain variance variant, through ToneMapper's log prologue, tables and query."""
    _check_rgb(rgb)
    _, H, W = rgb.shape
    p = make_params(n_bins, n_scales, eps=eps, ld_min=ld_min, ld_max=ld_max, H=H, W=W)
    if variance != "linear":
        m = ToneMapper(H, W, p, prec, device=rgb.device, variance=variance)
        out = m.run_rgb(rgb, saturation, stream)
        if rgb_out is None:
            return out
        _check_rgb(rgb_out, H, W)
        rgb_out.copy_(out)
        return rgb_out
    if rgb_out is None:
        rgb_out = torch.empty((3, H, W), dtype=torch.float32, device=rgb.device)
    _check_rgb(rgb_out, H, W)
    ws = _ws(_lib().tm_tonemap_rgb_workspace_bytes(H, W, ctypes.byref(p),
                                                   _capi.SAT_PREC[prec]), rgb.device)
    _ck("tm_tonemap_rgb", _lib().tm_tonemap_rgb(
        _vp(rgb), rgb.stride(0), rgb.stride(1), H, W, ctypes.byref(p), _capi.SAT_PREC[prec],
        float(saturation), _vp(rgb_out), rgb_out.stride(0), rgb_out.stride(1), _vp(ws),
        ws.numel(), _stream(stream)))
    return rgb_out


def residual_planes(n_scales: int) -> int:
    return int(_lib().tm_residual_planes(n_scales))


def residual_pairs(resid: torch.Tensor, n_scales: int) -> torch.Tensor:
    """View of the interleaved {R1_j, R2_j} pairs of a residual buffer: [s, H, W, 2]."""
    _, H, W = resid.shape
    return resid[:2 * n_scales].reshape(n_scales, H, W, 2)


def tm_tonemap_forward_train(v, sat: Table, hist: Table | None, edges, params, offsets=None,
                             out=None, resid=None, stream=None):
    """Forward plus the residual planes of the backward: (L [H, W], resid [2s+2, H, W]).
    resid holds the s interleaved {R1_j, R2_j} pair planes (see residual_pairs) in its first
    2s planes, then E and Pbar."""
    H, W, ld = _img(v, "v")
    if out is None:
        out = torch.empty((H, W), dtype=torch.float32, device=v.device)
    if resid is None:
        resid = torch.empty((residual_planes(params.n_scales), H, W), dtype=torch.float32,
                            device=v.device)
    _ck("tm_tonemap_forward_train", _lib().tm_tonemap_forward_train(
        _vp(v), ld, H, W, _vp(sat.ptr), sat.ld, _capi.SAT_PREC[sat.kind], _vp(offsets),
        _vp(hist.ptr if hist else None), hist.ld if hist else 0,
        hist.plane_stride if hist else 0, _vp(edges), ctypes.byref(params), _vp(out),
        out.stride(0), _vp(resid), _stream(stream)))
    return out, resid


def tm_tonemap_backward_resid(v, params, resid, grad_out, stream=None, ws=None, out=None):
    """Gradient from residual planes: (grad_v [H, W] float32, grad_params [3] float64)."""
    H, W, ld = _img(v, "v")
    _, _, ldg = _img(grad_out, "grad_out")
    if out is None:
        out = (torch.empty((H, W), dtype=torch.float32, device=v.device),
               torch.empty(3, dtype=torch.float64, device=v.device))
    gv, gp = out
    if ws is None:
        ws = _ws(_lib().tm_backward_resid_workspace_bytes(H, W, ctypes.byref(params)), v.device)
    _ck("tm_tonemap_backward_resid", _lib().tm_tonemap_backward_resid(
        _vp(v), ld, H, W, ctypes.byref(params), _vp(resid), _vp(grad_out), ldg, _vp(gv),
        gv.stride(0), _vp(gp), _vp(ws), ws.numel(), _stream(stream)))
    return gv, gp


def tm_tonemap_backward_resid_log(lum, params, resid, grad_out, stream=None, ws=None,
                                  out=None):
    """Log-domain variant's gradient from residual planes, given the image i itself (the
    chain rule through l = ln max(i, FLT_MIN) is applied in the last scan pass):
    (grad_lum [H, W] float32, grad_params [3] float64)."""
    H, W, ld = _img(lum, "lum")
    _, _, ldg = _img(grad_out, "grad_out")
    if out is None:
        out = (torch.empty((H, W), dtype=torch.float32, device=lum.device),
               torch.empty(3, dtype=torch.float64, device=lum.device))
    gv, gp = out
    if ws is None:
        ws = _ws(_lib().tm_backward_resid_workspace_bytes(H, W, ctypes.byref(params)),
                 lum.device)
    _ck("tm_tonemap_backward_resid_log", _lib().tm_tonemap_backward_resid_log(
        _vp(lum), ld, H, W, ctypes.byref(params), _vp(resid), _vp(grad_out), ldg, _vp(gv),
        gv.stride(0), _vp(gp), _vp(ws), ws.numel(), _stream(stream)))
    return gv, gp


def tm_tonemap_backward_log(lum, sat: Table, hist: Table | None, edges, params, grad_out,
                            log_offsets=None, stream=None):
    """The log-domain variant's backward from its tables (integral image and offsets of l,
    histogram of lum): (grad_lum [H, W] float32, grad_params [3] float64)."""
    H, W, ld = _img(lum, "lum")
    _, _, ldg = _img(grad_out, "grad_out")
    gv = torch.empty((H, W), dtype=torch.float32, device=lum.device)
    gp = torch.empty(3, dtype=torch.float64, device=lum.device)
    ws = _ws(_lib().tm_backward_workspace_bytes(H, W, ctypes.byref(params)), lum.device)
    _ck("tm_tonemap_backward_log", _lib().tm_tonemap_backward_log(
        _vp(lum), ld, H, W, _vp(sat.ptr), sat.ld, _capi.SAT_PREC[sat.kind], _vp(log_offsets),
        _vp(hist.ptr if hist else None), hist.ld if hist else 0,
        hist.plane_stride if hist else 0, _vp(edges), ctypes.byref(params), _vp(grad_out), ldg,
        _vp(gv), gv.stride(0), _vp(gp), _vp(ws), ws.numel(), _stream(stream)))
    return gv, gp


def tm_tonemap_backward(v, sat: Table, hist: Table | None, edges, params, grad_out,
                        offsets=None, stream=None):
    """(grad_v [H, W] float32, grad_params [3] float64 = d/d(eps, ld_min, ld_max))."""
    H, W, ld = _img(v, "v")
    _, _, ldg = _img(grad_out, "grad_out")
    gv = torch.empty((H, W), dtype=torch.float32, device=v.device)
    gp = torch.empty(3, dtype=torch.float64, device=v.device)
    nb = _lib().tm_backward_workspace_bytes(H, W, ctypes.byref(params))
    ws = _ws(nb, v.device)
    _ck("tm_tonemap_backward", _lib().tm_tonemap_backward(
        _vp(v), ld, H, W, _vp(sat.ptr), sat.ld, _capi.SAT_PREC[sat.kind], _vp(offsets),
        _vp(hist.ptr if hist else None), hist.ld if hist else 0,
        hist.plane_stride if hist else 0, _vp(edges), ctypes.byref(params), _vp(grad_out), ldg,
        _vp(gv), gv.stride(0), _vp(gp), _vp(ws), ws.numel(), _stream(stream)))
    return gv, gp


# ------------------------------------------------------------------------ pipeline
@dataclass
class Stage:
    lum: torch.Tensor
    edges: torch.Tensor
    offsets: torch.Tensor
    minmax: torch.Tensor
    sat: Table
    hist: Table | None
    out: torch.Tensor


VARIANCE_DOMAINS = ("linear", "log")


class ToneMapper:
    """Preallocated forward path for one image shape: prologue (Eq. 11 + statistics),
    integral tables (Eq. 5, 8), fused query (Eq. 1-4).  All buffers and workspaces are
    allocated once so that run() only enqueues kernels (capturable in a HIP graph).
    variance="log": Eq. 10's window variance is that of the log image l = ln i (the
    prologue forms l's offsets, the tables pass scans l formed as it reads i and bins i, the
    residual backward forms l the same way); run, run_train and backward_resid (not the
    table-based backward).
    tune: a TmTune, None for the shape's default tiling, or "cached" for the tiling the
    autotuner stored for this device, shape bucket, bin count and precision
    (autotune.tune_image), falling back to the default when none is stored."""

    def __init__(self, H: int, W: int, params, prec: str = "c32x2", tune=None,
                 device="cuda", variance: str = "linear"):
        if variance not in VARIANCE_DOMAINS:
            raise ValueError(f"variance must be one of {VARIANCE_DOMAINS}")
        if isinstance(tune, str):
            if tune != "cached":
                raise ValueError('tune must be a TmTune, None or "cached"')
            from .autotune import cached_image_tune
            tune = cached_image_tune(H, W, params.n_bins, prec, torch.device(device))
        self.variance = variance
        self.H, self.W, self.params, self.prec, self.tune = H, W, params, prec, tune
        n = params.n_bins
        dev = torch.device(device)
        self.lum = torch.empty((H, W), dtype=torch.float32, device=dev)
        self.edges = torch.empty(max(n - 1, 1), dtype=torch.float32, device=dev)
        self.offsets = torch.empty(2, dtype=torch.float32, device=dev)
        self.minmax = torch.empty(2, dtype=torch.float32, device=dev)
        self.sat = Table(H, W, prec, 1, dev)
        self.hist = Table(H, W, "u32", n - 1, dev) if n > 1 else None
        self.out = torch.empty((H, W), dtype=torch.float32, device=dev)
        self.ws_stats = _ws(_lib().tm_image_stats_workspace_bytes(H, W), dev)
        self.ws_tab = _ws(_lib().tm_tables_workspace_bytes(H, W, n, _capi.SAT_PREC[prec],
                                                            _tune_ref(tune)), dev)
        self.tune_ref = _tune_ref(tune)
        # the integral image's offsets: those of the luminance, or of its log plane
        self.sat_offsets = self.offsets
        if variance == "log":
            # no log plane is kept: the prologue forms l's offsets, the tables pass and the
            # backward form l from lum as they read it
            self.log_offsets = torch.empty(2, dtype=torch.float32, device=dev)
            self.sat_offsets = self.log_offsets

    def prologue(self, rgb, stream=None):
        if self.variance == "log":
            # luminance, bin edges and l's offsets in one pass
            _ck("tm_prologue_log", _lib().tm_prologue_log(
                _vp(rgb), rgb.stride(0), rgb.stride(1), self.H, self.W, self.params.n_bins,
                _vp(self.lum), self.lum.stride(0), None, 0, _vp(self.edges),
                _vp(self.log_offsets), _vp(self.minmax), _vp(self.ws_stats),
                self.ws_stats.numel(), _stream(stream)))
            return
        _ck("tm_prologue", _lib().tm_prologue(
            _vp(rgb), rgb.stride(0), rgb.stride(1), self.H, self.W, self.params.n_bins,
            _vp(self.lum), self.lum.stride(0), _vp(self.edges), _vp(self.offsets),
            _vp(self.minmax), _vp(self.ws_stats), self.ws_stats.numel(), _stream(stream)))

    def tables(self, stream=None):
        h = self.hist
        if self.variance == "log":
            # integral image of l (formed on load) and histogram of lum in one pass
            _ck("tm_integral_tables_log", _lib().tm_integral_tables_log(
                _vp(self.lum), self.lum.stride(0), self.H, self.W, _capi.SAT_PREC[self.prec],
                _vp(self.log_offsets), _vp(self.sat.ptr), self.sat.ld, _vp(self.edges),
                self.params.n_bins, 1, _vp(h.ptr if h else None), h.ld if h else 0,
                h.plane_stride if h else 0, self.tune_ref, _vp(self.ws_tab),
                self.ws_tab.numel(), _stream(stream)))
            return
        _ck("tm_integral_tables", _lib().tm_integral_tables(
            _vp(self.lum), self.lum.stride(0), self.H, self.W, _capi.SAT_PREC[self.prec],
            _vp(self.offsets), _vp(self.sat.ptr), self.sat.ld, _vp(self.edges),
            self.params.n_bins, 1, _vp(h.ptr if h else None), h.ld if h else 0,
            h.plane_stride if h else 0, self.tune_ref, _vp(self.ws_tab), self.ws_tab.numel(),
            _stream(stream)))

    def query(self, stream=None):
        tm_tonemap_forward(self.lum, self.sat, self.hist, self.edges, self.params,
                           self.sat_offsets, self.out, stream)

    def run(self, rgb, stream=None) -> torch.Tensor:
        self.prologue(rgb, stream)
        self.tables(stream)
        self.query(stream)
        return self.out

    def query_maps(self, stream=None):
        """Fused query that also writes the per-field tone values and weights (Fig. 3):
        (L, maps [2s, H, W])."""
        return tm_tonemap_forward_maps(self.lum, self.sat, self.hist, self.edges, self.params,
                                       self.sat_offsets, self.out, None, stream)

    def query_rgb(self, rgb, saturation: float = 0.6, stream=None) -> torch.Tensor:
        """Fused query with colour restoration (Eq. 12) of rgb: returns rgb_out [3, H, W]
        (L is also left in self.out)."""
        if not hasattr(self, "rgb_out"):
            self.rgb_out = torch.empty((3, self.H, self.W), dtype=torch.float32,
                                       device=self.lum.device)
        return tm_tonemap_forward_rgb(self.lum, self.sat, self.hist, self.edges, self.params,
                                      rgb, saturation, self.sat_offsets, self.rgb_out, self.out,
                                      stream)

    def run_rgb(self, rgb, saturation: float = 0.6, stream=None) -> torch.Tensor:
        self.prologue(rgb, stream)
        self.tables(stream)
        return self.query_rgb(rgb, saturation, stream)

    def query_train(self, stream=None):
        """Fused query that also writes the backward's residual planes (those of the log
        image's window statistics for variance="log")."""
        if not hasattr(self, "resid"):
            self.resid = torch.empty((residual_planes(self.params.n_scales), self.H, self.W),
                                     dtype=torch.float32, device=self.lum.device)
        tm_tonemap_forward_train(self.lum, self.sat, self.hist, self.edges, self.params,
                                 self.sat_offsets, self.out, self.resid, stream)

    def run_train(self, rgb, stream=None) -> torch.Tensor:
        self.prologue(rgb, stream)
        self.tables(stream)
        self.query_train(stream)
        return self.out

    def _bwd_buffers(self):
        if not hasattr(self, "grad_v"):
            dev = self.lum.device
            self.grad_v = torch.empty((self.H, self.W), dtype=torch.float32, device=dev)
            self.grad_params = torch.empty(3, dtype=torch.float64, device=dev)

    def backward_resid(self, grad_out: torch.Tensor, stream=None):
        """Adjoint from the residual planes of the last run_train: (grad_lum, grad_params).
        variance="log": the residual backward forms l from lum in its last pass and applies
        the chain rule through the logarithm there, returning the gradient w.r.t. lum."""
        self._bwd_buffers()
        if not hasattr(self, "ws_bwd_resid"):
            self.ws_bwd_resid = _ws(_lib().tm_backward_resid_workspace_bytes(
                self.H, self.W, ctypes.byref(self.params)), self.lum.device)
        bwd = (tm_tonemap_backward_resid_log if self.variance == "log"
               else tm_tonemap_backward_resid)
        bwd(self.lum, self.params, self.resid, grad_out, stream, self.ws_bwd_resid,
            (self.grad_v, self.grad_params))
        return self.grad_v, self.grad_params

    def backward(self, grad_out: torch.Tensor, stream=None):
        """Adjoint of the last forward from its tables: (grad_lum, grad_params)."""
        self._bwd_buffers()
        if not hasattr(self, "ws_bwd"):
            self.ws_bwd = _ws(_lib().tm_backward_workspace_bytes(self.H, self.W,
                                                                 ctypes.byref(self.params)),
                              self.lum.device)
        h = self.hist
        _, _, ldg = _img(grad_out, "grad_out")
        log = self.variance == "log"    # the tables and offsets of l, the chain rule to lum
        name = "tm_tonemap_backward_log" if log else "tm_tonemap_backward"
        _ck(name, getattr(_lib(), name)(
            _vp(self.lum), self.lum.stride(0), self.H, self.W, _vp(self.sat.ptr), self.sat.ld,
            _capi.SAT_PREC[self.prec], _vp(self.sat_offsets), _vp(h.ptr if h else None),
            h.ld if h else 0, h.plane_stride if h else 0, _vp(self.edges),
            ctypes.byref(self.params), _vp(grad_out), ldg, _vp(self.grad_v),
            self.grad_v.stride(0), _vp(self.grad_params), _vp(self.ws_bwd), self.ws_bwd.numel(),
            _stream(stream)))
        return self.grad_v, self.grad_params


def tonemap(rgb: torch.Tensor, n_bins: int = 5, n_scales: int = 5, eps: float = 0.1,
            prec: str = "c32x2", ld_min: float = 0.0, ld_max: float = 1.0,
            variance: str = "linear") -> torch.Tensor:
    """Tone-mapped luminance of one planar RGB image with the paper's parameter set
    (variance "linear", or "log" for the log-domain variance variant)."""
    _, H, W = rgb.shape
    p = make_params(n_bins, n_scales, eps=eps, ld_min=ld_min, ld_max=ld_max, H=H, W=W)
    return ToneMapper(H, W, p, prec, device=rgb.device, variance=variance).run(rgb).clone()


# ------------------------------------------------------------------------ batches
class Batch:
    """Forward of many images of uneven size: per-image buffers laid out in one workspace,
    one launch per phase over each group of images (tm_batch_forward), optionally recorded
    once into a HIP graph and replayed (tm_batch_capture / tm_batch_replay)."""

    def __init__(self, rgbs, n_bins: int = 5, n_scales: int = 5, eps: float = 0.1,
                 ld_min: float = 0.0, ld_max: float = 1.0, prec: str = "c32x2", tune=None,
                 stream=None):
        self.count = len(rgbs)
        self.rgbs = list(rgbs)
        self.outs = []
        self.descs = (_capi.TmImageDesc * self.count)()
        for i, rgb in enumerate(self.rgbs):
            if rgb.dtype != torch.float32 or rgb.dim() != 3 or rgb.shape[0] != 3 \
                    or rgb.stride(2) != 1 or not rgb.is_cuda:
                raise ValueError("each image must be a CUDA float32 [3, H, W] tensor")
            _, H, W = rgb.shape
            out = torch.empty((H, W), dtype=torch.float32, device=rgb.device)
            self.outs.append(out)
            d = self.descs[i]
            d.rgb, d.ch_stride, d.ld_rgb = rgb.data_ptr(), rgb.stride(0), rgb.stride(1)
            d.out, d.ld_out, d.H, d.W = out.data_ptr(), out.stride(0), H, W
            rx, ry = paper_radii(H, W, n_scales)
            for j in range(n_scales):
                d.rx[j], d.ry[j] = rx[j], ry[j]
        self.params = make_params(n_bins, n_scales, [0] * n_scales, [0] * n_scales, eps,
                                  ld_min, ld_max)
        self.prec = prec
        self.tune = tune
        pc = _capi.SAT_PREC[prec]
        nbytes = _lib().tm_batch_workspace_bytes(self.descs, self.count,
                                                 ctypes.byref(self.params), pc, _tune_ref(tune))
        if nbytes == 0:
            raise TmError("tm_batch_workspace_bytes", -1)
        self.ws = _ws(nbytes, self.rgbs[0].device)
        h = ctypes.c_void_p()
        _ck("tm_batch_create", _lib().tm_batch_create(
            self.descs, self.count, ctypes.byref(self.params), pc, _tune_ref(tune), _vp(self.ws),
            self.ws.numel(), _stream(stream), ctypes.byref(h)))
        self.handle = h

    def set_concurrency(self, streams: int = 1, images_per_group: int = 0):
        """Spread forward() over `streams` internal streams (phases of different image groups
        overlap), with at most `images_per_group` images per group (0: no limit)."""
        _ck("tm_batch_set_concurrency", _lib().tm_batch_set_concurrency(
            self.handle, int(streams), int(images_per_group)))

    def set_variance(self, variance: str = "linear", stream=None):
        """Variance domain of the following forwards ("linear" or "log", as ToneMapper's);
        a graph captured before must be captured again."""
        if variance not in VARIANCE_DOMAINS:
            raise ValueError(f"variance must be one of {VARIANCE_DOMAINS}")
        _ck("tm_batch_set_variance", _lib().tm_batch_set_variance(
            self.handle, 1 if variance == "log" else 0, _stream(stream)))

    def forward(self, stream=None):
        _ck("tm_batch_forward", _lib().tm_batch_forward(self.handle, _stream(stream)))
        return self.outs

    def capture(self, stream):
        """Record forward() into a HIP graph on a non-null stream (nothing runs)."""
        _ck("tm_batch_capture", _lib().tm_batch_capture(self.handle, _stream(stream)))

    def replay(self, stream=None):
        _ck("tm_batch_replay", _lib().tm_batch_replay(self.handle, _stream(stream)))
        return self.outs

    def image_buffers(self, i: int):
        P = ctypes.c_void_p
        lum, edges, offs, sat, hist = P(), P(), P(), P(), P()
        ldl, lds, ldh, ps = (ctypes.c_int64() for _ in range(4))
        _ck("tm_batch_image_buffers", _lib().tm_batch_image_buffers(
            self.handle, i, ctypes.byref(lum), ctypes.byref(ldl), ctypes.byref(edges),
            ctypes.byref(offs), ctypes.byref(sat), ctypes.byref(lds), ctypes.byref(hist),
            ctypes.byref(ldh), ctypes.byref(ps)))
        return dict(lum=lum.value, ld_lum=ldl.value, edges=edges.value, offsets=offs.value,
                    sat=sat.value, ld_sat=lds.value, hist=hist.value, ld_hist=ldh.value,
                    plane_stride=ps.value)

    def close(self):
        if getattr(self, "handle", None):
            _lib().tm_batch_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
