"""ctypes declarations of the C ABI in include/tm.h (argument marshalling only)."""
from __future__ import annotations

import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libtm355.so")

TM_MAX_SCALES = 8
TM_MAX_BINS = 256

STATUS = {0: "TM_OK", -1: "TM_ERR_ARG", -2: "TM_ERR_SHAPE", -3: "TM_ERR_ALIGN",
          -4: "TM_ERR_WORKSPACE", -5: "TM_ERR_HIP", -6: "TM_ERR_UNSUPPORTED"}

SAT_PREC = {"f32": 0, "c32x2": 1, "f64": 2}
HIST_LAYOUT = {"per_bin": 0, "cumulative": 1}


class TmParams(ctypes.Structure):
    _fields_ = [("n_bins", ctypes.c_int32), ("n_scales", ctypes.c_int32),
                ("rx", ctypes.c_int32 * TM_MAX_SCALES), ("ry", ctypes.c_int32 * TM_MAX_SCALES),
                ("eps", ctypes.c_float), ("ld_min", ctypes.c_float), ("ld_max", ctypes.c_float),
                ("scalars", ctypes.c_void_p)]


class TmTune(ctypes.Structure):
    _fields_ = [("tile_w_vec", ctypes.c_int32), ("tile_h", ctypes.c_int32),
                ("bin_chunk", ctypes.c_int32)]


class TmImageDesc(ctypes.Structure):
    _fields_ = [("rgb", ctypes.c_void_p), ("ch_stride", ctypes.c_int64),
                ("ld_rgb", ctypes.c_int64), ("out", ctypes.c_void_p), ("ld_out", ctypes.c_int64),
                ("H", ctypes.c_int32), ("W", ctypes.c_int32),
                ("rx", ctypes.c_int32 * TM_MAX_SCALES), ("ry", ctypes.c_int32 * TM_MAX_SCALES)]


# (name, restype, argtypes) for every entry point of include/tm.h
P, I32, I64, SZ, F, D = (ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_size_t,
                         ctypes.c_float, ctypes.c_double)
PP = ctypes.POINTER(TmParams)
PT = ctypes.POINTER(TmTune)
PI64 = ctypes.POINTER(ctypes.c_int64)

SIGNATURES = {
    "tm_status_string": (ctypes.c_char_p, [ctypes.c_int]),
    "tm_paper_radii": (ctypes.c_int, [I32, I32, PP]),
    "tm_default_tune": (ctypes.c_int, [I32, I32, I32, PT]),
    "tm_table_geometry": (ctypes.c_int, [I32, I32, PI64, PI64, PI64]),
    "tm_luminance": (ctypes.c_int, [P, I64, I64, I32, I32, P, I64, P]),
    "tm_image_stats_workspace_bytes": (SZ, [I32, I32]),
    "tm_image_stats": (ctypes.c_int, [P, I64, I32, I32, I32, P, P, P, P, SZ, P]),
    "tm_prologue": (ctypes.c_int, [P, I64, I64, I32, I32, I32, P, I64, P, P, P, P, SZ, P]),
    "tm_prologue_log": (ctypes.c_int, [P, I64, I64, I32, I32, I32, P, I64, P, I64, P, P, P, P,
                                       SZ, P]),
    "tm_prologue_noalloc": (ctypes.c_int, [P, I64, I64, I32, I32, I32, P, I64, P, P, P, P]),
    "tm_log_luminance": (ctypes.c_int, [P, I64, I32, I32, P, I64, P, P, P, SZ, P]),
    "tm_lookback_set_spin_limit": (None, [ctypes.c_uint32]),
    "tm_log_luminance_backward": (ctypes.c_int, [P, I64, I32, I32, P, I64, P, I64, P]),
    "tm_hdr_response_workspace_bytes": (SZ, []),
    "tm_hdr_response": (ctypes.c_int, [P, I64, I64, I64, I32, I32, I32, P, I32, P,
                                       ctypes.c_float, P, P, SZ, P]),
    "tm_hdr_merge": (ctypes.c_int, [P, I64, I64, I64, I32, I32, I32, P, P, P, I64, I64, P]),
    "tm_integral_image": (ctypes.c_int, [P, I64, I32, I32, ctypes.c_int, P, P, I64, PT, P, SZ,
                                         P]),
    "tm_integral_histogram": (ctypes.c_int, [P, I64, I32, I32, P, I32, ctypes.c_int, P, I64,
                                             I64, PT, P, SZ, P]),
    "tm_integral_tables": (ctypes.c_int, [P, I64, I32, I32, ctypes.c_int, P, P, I64, P, I32,
                                          ctypes.c_int, P, I64, I64, PT, P, SZ, P]),
    "tm_integral_tables_split": (ctypes.c_int, [P, I64, P, I64, I32, I32, ctypes.c_int, P, P,
                                                I64, P, I32, ctypes.c_int, P, I64, I64, PT, P,
                                                SZ, P]),
    "tm_integral_tables_log": (ctypes.c_int, [P, I64, I32, I32, ctypes.c_int, P, P, I64, P,
                                              I32, ctypes.c_int, P, I64, I64, PT, P, SZ, P]),
    "tm_tables_workspace_bytes": (SZ, [I32, I32, I32, ctypes.c_int, PT]),
    "tm_lookback_workspace_bytes": (SZ, [I32, I32, I32, ctypes.c_int]),
    "tm_integral_histogram_lookback": (ctypes.c_int, [P, I64, I32, I32, P, I32, ctypes.c_int, P,
                                                      I64, I64, P, SZ, P]),
    "tm_tonemap_forward": (ctypes.c_int, [P, I64, I32, I32, P, I64, ctypes.c_int, P, P, I64,
                                          I64, P, PP, P, I64, P]),
    "tm_backward_workspace_bytes": (SZ, [I32, I32, PP]),
    "tm_tonemap_forward_maps": (ctypes.c_int, [P, I64, I32, I32, P, I64, ctypes.c_int, P, P, I64,
                                               I64, P, PP, P, I64, P, P]),
    "tm_tonemap_forward_rgb": (ctypes.c_int, [P, I64, I32, I32, P, I64, ctypes.c_int, P, P, I64,
                                              I64, P, PP, P, I64, I64, F, P, I64, I64, P, I64,
                                              P]),
    "tm_tonemap_rgb_workspace_bytes": (SZ, [I32, I32, PP, ctypes.c_int]),
    "tm_tonemap_rgb": (ctypes.c_int, [P, I64, I64, I32, I32, PP, ctypes.c_int, F, P, I64, I64, P,
                                      SZ, P]),
    "tm_residual_planes": (I32, [I32]),
    "tm_tonemap_forward_train": (ctypes.c_int, [P, I64, I32, I32, P, I64, ctypes.c_int, P, P,
                                                I64, I64, P, PP, P, I64, P, P]),
    "tm_backward_resid_workspace_bytes": (SZ, [I32, I32, PP]),
    "tm_tonemap_backward_resid": (ctypes.c_int, [P, I64, I32, I32, PP, P, P, I64, P, I64, P, P,
                                                 SZ, P]),
    "tm_tonemap_backward_resid_log": (ctypes.c_int, [P, I64, I32, I32, PP, P, P, I64, P, I64,
                                                     P, P, SZ, P]),
    "tm_batch_workspace_bytes": (SZ, [ctypes.POINTER(TmImageDesc), I32, PP, ctypes.c_int, PT]),
    "tm_batch_create": (ctypes.c_int, [ctypes.POINTER(TmImageDesc), I32, PP, ctypes.c_int, PT, P,
                                       SZ, P, ctypes.POINTER(P)]),
    "tm_batch_forward": (ctypes.c_int, [P, P]),
    "tm_batch_set_concurrency": (ctypes.c_int, [P, I32, I32]),
    "tm_batch_set_variance": (ctypes.c_int, [P, I32, P]),
    "tm_batch_capture": (ctypes.c_int, [P, P]),
    "tm_batch_replay": (ctypes.c_int, [P, P]),
    "tm_batch_destroy": (ctypes.c_int, [P]),
    "tm_batch_image_buffers": (ctypes.c_int, [P, I32] + [ctypes.POINTER(P), PI64] +
                               [ctypes.POINTER(P)] * 3 + [PI64, ctypes.POINTER(P), PI64, PI64]),
    "tm_tonemap_backward": (ctypes.c_int, [P, I64, I32, I32, P, I64, ctypes.c_int, P, P, I64,
                                           I64, P, PP, P, I64, P, I64, P, P, SZ, P]),
    "tm_tonemap_backward_log": (ctypes.c_int, [P, I64, I32, I32, P, I64, ctypes.c_int, P, P,
                                               I64, I64, P, PP, P, I64, P, I64, P, P, SZ, P]),
}

_LIB = None


def load() -> ctypes.CDLL:
    """Load the in-tree HIP library.  Raises if it has not been built: there is no
    fallback path."""
    global _LIB
    if _LIB is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(
                f"HIP library {LIB_PATH} is missing; build it with "
                "`python -c 'import __graft_entry__ as g; g.build()'` or "
                "`python paper_2102_01289_amd/build.py`")
        lib = ctypes.CDLL(LIB_PATH)
        for name, (res, args) in SIGNATURES.items():
            fn = getattr(lib, name)
            fn.restype = res
            fn.argtypes = args
        _LIB = lib
    return _LIB
