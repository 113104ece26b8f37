"""tm_prologue_noalloc -- the prologue whose reduction partials live in the library's static
device array instead of a caller workspace -- against tm_prologue, bit for bit, through the C
ABI: two calls in a row on one GPU, the second on a smaller image (the array keeps the first
call's partials; every partial the second needs is rewritten), then the first image again."""
import numpy as np
import pytest
import torch

import oracle
import paper_2102_01289_amd as tm
from _cases import rgb_case, to_dev

pytestmark = pytest.mark.gpu


def _compare(rgb, n):
    a = tm.tm_prologue(rgb, n)
    b = tm.tm_prologue_noalloc(rgb, n)
    torch.cuda.synchronize()
    for name, x, y in zip(("lum", "edges", "offsets", "minmax"), a, b):
        assert torch.equal(x, y), name
    return b


def test_noalloc_prologue_matches_the_workspace_prologue():
    # 4000 x 3000 uses all 1024 partials of the array; 37 x 123 uses 37
    cases = [(3000, 4000, 5, 103), (37, 123, 64, 5), (3000, 4000, 5, 103)]
    for H, W, n, seed in cases:
        print(f"noalloc prologue {H}x{W} n={n}", flush=True)
        host = rgb_case(H, W, 6, seed=seed)
        lum, edges, _, _ = _compare(to_dev(host), n)
        # and the luminance and edges against the oracle
        ref = oracle.luminance(host)
        assert np.array_equal(lum.cpu().numpy().view(np.uint32), ref.view(np.uint32))
        assert np.array_equal(edges.cpu().numpy(), oracle.exact_edges(ref.min(), ref.max(), n))


def test_noalloc_prologue_rejects_bad_arguments():
    rgb = to_dev(rgb_case(8, 8, 2, seed=1))
    with pytest.raises(tm.TmError):
        tm.tm_prologue_noalloc(rgb, 0)
    with pytest.raises(tm.TmError):
        tm.tm_prologue_noalloc(rgb, 300)
