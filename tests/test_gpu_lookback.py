"""The single-pass integral histogram (decoupled look-back between tiles) against the oracle's
integral histogram (Eq. 7-8) and the three-stage build, bit for bit, on ragged, degenerate
and multi-tile shapes, both layouts; the status word must read 0 (no wait ran out)."""
import numpy as np
import pytest
import torch

import paper_2102_01289_amd as tm
from _cases import edges_ref, fill_garbage, hist_ref, lum_ref, rgb_case, to_dev

pytestmark = pytest.mark.gpu

# ragged and degenerate shapes, several tiles each way, and two long carry chains: 250 tile
# rows in one tile column pair (the column look-back) and 71 tiles in one tile row (the row
# and corner look-backs)
SHAPES = [(1, 1), (1, 300), (300, 1), (37, 123), (64, 256), (100, 700), (257, 1030),
          (1000, 777), (4000, 130), (8, 9000)]


def _status(ws):
    torch.cuda.synchronize()
    return int(ws[4:8].cpu().view(torch.int32)[0])


@pytest.mark.parametrize("H,W", SHAPES)
@pytest.mark.parametrize("n,layout", [(2, "cumulative"), (5, "cumulative"), (9, "cumulative"),
                                      (1, "per_bin"), (4, "per_bin"), (8, "per_bin")])
def test_lookback_histogram_bit_exact(H, W, n, layout):
    ref = lum_ref(rgb_case(H, W, 6, -2.0, 4.0, seed=5 * n + W + H))
    v = to_dev(ref)
    edges = to_dev(edges_ref(ref, n))
    planes = n if layout == "per_bin" else n - 1
    hist = tm.Table(H, W, "u32", planes)
    fill_garbage(hist)
    _, ws = tm.tm_integral_histogram_lookback(v, edges, n, layout, hist=hist)
    assert _status(ws) == 0
    got = hist.padded()[..., 0].numpy().astype(np.uint64)
    want = hist_ref(ref, edges_ref(ref, n), n, layout)
    assert np.array_equal(got, want)
    # the three-stage build gives the same planes, border included
    three = tm.tm_integral_histogram(v, edges, n, layout)
    assert torch.equal(three.raw_region(), hist.raw_region())


def test_lookback_histogram_repeats_and_reuses_its_workspace():
    H, W, n = 1080, 1920, 5
    ref = lum_ref(rgb_case(H, W, 8, -2.0, 4.0, seed=41))
    v = to_dev(ref)
    edges = to_dev(edges_ref(ref, n))
    h1, ws = tm.tm_integral_histogram_lookback(v, edges, n)
    first = h1.raw_region().clone()
    for _ in range(3):
        fill_garbage(h1)
        tm.tm_integral_histogram_lookback(v, edges, n, hist=h1, ws=ws)
        assert _status(ws) == 0
        assert torch.equal(h1.raw_region(), first)
    want = hist_ref(ref, edges_ref(ref, n), n, "cumulative")
    assert np.array_equal(h1.padded()[..., 0].numpy().astype(np.uint64), want)


def test_lookback_histogram_at_12_megapixels_equals_the_three_stage_build():
    H, W, n = 3000, 4000, 5
    ref = lum_ref(rgb_case(H, W, 64, -3.0, 5.0, seed=43))
    v = to_dev(ref)
    edges = to_dev(edges_ref(ref, n))
    h, ws = tm.tm_integral_histogram_lookback(v, edges, n)
    assert _status(ws) == 0
    three = tm.tm_integral_histogram(v, edges, n)
    assert torch.equal(three.raw_region(), h.raw_region())
    # the last entry of each plane is the pixel count of bins <= the plane's bin
    b = np.searchsorted(edges_ref(ref, n), ref.ravel(), side="right")
    last = h.padded()[:, -1, -1, 0].numpy()
    assert last.tolist() == [int((b <= p).sum()) for p in range(n - 1)]


def test_lookback_histogram_rejects_more_than_eight_planes():
    v = torch.zeros((8, 8), dtype=torch.float32, device="cuda")
    edges = torch.arange(16, dtype=torch.float32, device="cuda")
    with pytest.raises(tm.TmError) as e:
        tm.tm_integral_histogram_lookback(v, edges, 10, "cumulative",
                                          ws=torch.empty(1 << 20, dtype=torch.uint8, device="cuda"))
    assert "UNSUPPORTED" in str(e.value) or "-6" in str(e.value)


def test_lookback_bounded_waits_end_in_the_status_word():
    # one poll per window: a wait that finds a record absent gives up almost at once, counts
    # the record as an inclusive zero and raises the status word, and the pass still completes.
    # Either no wait gave up (status 0, planes exact) or one did (status 1: planes not to be
    # used).  With the default bound restored the pass is exact again.
    H, W, n = 3000, 4000, 5
    ref = lum_ref(rgb_case(H, W, 16, -3.0, 5.0, seed=47))
    v = to_dev(ref)
    edges = to_dev(edges_ref(ref, n))
    three = tm.tm_integral_histogram(v, edges, n)
    lib = tm._lib()
    try:
        lib.tm_lookback_set_spin_limit(1)
        for _ in range(3):
            h, ws = tm.tm_integral_histogram_lookback(v, edges, n)
            st = _status(ws)
            assert st in (0, 1)
            if st == 0:
                assert torch.equal(three.raw_region(), h.raw_region())
    finally:
        lib.tm_lookback_set_spin_limit(0)
    h, ws = tm.tm_integral_histogram_lookback(v, edges, n)
    assert _status(ws) == 0
    assert torch.equal(three.raw_region(), h.raw_region())
