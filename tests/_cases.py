"""Shared helpers of the GPU parity tests: seeded inputs and oracle references."""
from __future__ import annotations

import numpy as np
import torch

import oracle
from synth import gen_wdr

U32 = np.uint32


def rgb_case(H, W, K=6, lo=-2.0, hi=4.0, seed=0):
    return gen_wdr(H, W, K, lo, hi, seed).rgb


def to_dev(a: np.ndarray) -> torch.Tensor:
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def lum_ref(rgb):
    return oracle.luminance(rgb)


def edges_ref(lum, n):
    return oracle.exact_edges(lum.min(), lum.max(), n)


def fill_garbage(t) -> None:
    """Overwrite a Table's whole buffer with a non-zero pattern so that the border zeros the
    producing call must write are really checked."""
    buf = t.buf
    if buf.dtype in (torch.float32, torch.float64):
        buf.fill_(float("nan"))
    else:
        buf.view(torch.int32).fill_(-559038737)


def hist_ref(lum, edges, n, layout):
    b = oracle.bins(lum, edges)
    return oracle.integral_histogram(b, n, cumulative=(layout == "cumulative"))
