"""Parity at the size limits of the interface: H*W just under 2^31 entries per table (the
documented limit, with the table border included), at the widest image (W = TM_MAX_WIDTH =
2^24, 126 rows) and at 510 x 2^22, each with the compensated FP32 and the FP64 tables.

No oracle finishes a 2-gigapixel image, so the input is one seeded WDR row repeated down
every row.  For such an image the window mean, variance and bin CDF of every field do not
depend on the row (the window's row count cancels from each ratio), so the tone-mapped value
of pixel (x, y) equals the oracle's on the single row at x, and the integral histogram's
entry at row y is (y + 1) times the row's own cumulative count.  Checked:
  * bin edges bit-exact;
  * three rows of every cumulative histogram plane, bit-exact (counts up to H*W);
  * six whole output rows against the FP64 oracle within the derived per-pixel bound;
  * every output pixel: the per-column max and min over all rows within the bound taken at
    its largest over the rows, and within a stated max-abs envelope.
The bound is the one of the other parity tests (quadrant sums of |q| times the summation
depth and the table's unit roundoff, carried through the variance and the fusion), with the
quadrant sums of this image written in closed form: Y times the row's prefix sum."""
import functools
import gc

import numpy as np
import pytest
import torch

import oracle
import paper_2102_01289_amd as tm
from _bounds import U, sat_depth, tiling
from _cases import edges_ref
from synth import gen_wdr_row

pytestmark = [pytest.mark.gpu, pytest.mark.slow]

EPS = 0.1
N_BINS = 5
N_SCALES = 5
# Stated max-abs envelope over every output pixel, beside the derived bound (which is loose
# for the compensated tables here: its summation depth counts the 2^16-long row carries
# as if every rounding added up).
ENVELOPE = {"c32x2": 1e-4, "f64": 2e-6}


def _row_bound(row, H, rx, ry, Lref, Lj, Wj, varj, prec, ys):
    """Per-pixel bound on |L_gpu - L_oracle| for rows ys of the row-invariant image, and
    (last entry) the bound at its largest over all rows."""
    W = row.shape[0]
    vec, th = tiling(H, W)
    du = sat_depth(H, W, vec, th) * U[prec]
    v = row.astype(np.float64)
    if prec == "c32x2":
        mu1, mu2 = float(np.float32(v.mean())), float(np.float32((v * v).mean()))
    else:
        mu1 = mu2 = 0.0
    A1 = np.concatenate([[0.0], np.cumsum(np.abs(v) + abs(mu1))])
    A2 = np.concatenate([[0.0], np.cumsum(v * v + abs(mu2))])
    P1 = np.concatenate([[0.0], np.cumsum(v)])
    xs = np.arange(W)
    yy = np.arange(H)
    D = Wj.sum(axis=0)[0]
    out = [np.zeros(W) for _ in range(len(ys) + 1)]
    for j in range(len(rx)):
        xm = np.maximum(xs - rx[j] - 1, -1) + 1
        xp = np.minimum(xs + rx[j], W - 1) + 1
        cols = (xp - xm).astype(np.float64)
        m = (P1[xp] - P1[xm]) / cols
        # per unit of (ym + yp) / rows: the corner-entry bounds through the variance
        base = du * ((A2[xm] + A2[xp]) + 2.0 * np.abs(m) * (A1[xm] + A1[xp])) / cols
        ym_all = np.maximum(yy - ry[j] - 1, -1) + 1
        yp_all = np.minimum(yy + ry[j], H - 1) + 1
        f_all = (ym_all + yp_all) / (yp_all - ym_all)
        with np.errstate(divide="ignore", invalid="ignore"):
            sens = np.abs(Lj[j][0] - Lref[0]) / D * EPS / (varj[j][0] + EPS) ** 2
        for i, f in enumerate([f_all[y] for y in ys] + [f_all.max()]):
            out[i] += np.where(D > 0, sens * base * f, 1.0)
    return [4.0 * o + 4e-6 for o in out]


def _hist_row(hist, p, y, W):
    """Row y (0-based) of cumulative plane p, columns 0..W-1, as uint64 on the host."""
    o = p * hist.plane_stride + hist.origin + y * hist.ld
    return hist.buf[o:o + W].cpu().numpy().view(np.uint32).astype(np.uint64)


@functools.lru_cache(maxsize=1)
def _reference(H, W):
    """The seeded row, its exact edges, the paper radii and the FP64 oracle on the row (the
    forward with per-field maps, and the cumulative histogram row)."""
    row = gen_wdr_row(W, K=8, lo=-2.0, hi=4.0, seed=W + H)
    lum = row[None, :]
    e = edges_ref(lum, N_BINS)
    rx, ry = oracle.paper_radii(H, W, N_SCALES)
    fwd = oracle.forward(lum, e, rx, ry, EPS, per_scale=True)
    G = oracle.integral_histogram(oracle.bins(lum, e), N_BINS, cumulative=True)[:, 1, 1:]
    return row, e, rx, ry, fwd, G


# the widest image (W = TM_MAX_WIDTH) and a taller one, each with the largest H its tables
# allow; both table precisions with 16-byte entries (the largest lane offsets)
@pytest.mark.parametrize("H,W,prec", [(126, 1 << 24, "c32x2"), (126, 1 << 24, "f64"),
                                      (510, 1 << 22, "c32x2"), (510, 1 << 22, "f64")])
def test_forward_at_the_size_limit(H, W, prec):
    ld, _, _ = tm.table_geometry(H, W)
    assert (H + 1) * ld + 1 < 2 ** 31 <= (H + 2) * ld + 1      # the largest H for this W
    row, e, rx, ry, (Lref, Lj, Wj, varj), G = _reference(H, W)
    p = tm.make_params(N_BINS, N_SCALES, eps=EPS, rx=rx, ry=ry)

    torch.cuda.empty_cache()
    v = torch.from_numpy(row).cuda().expand(H, W).contiguous()
    edges, offsets, _ = tm.tm_image_stats(v, N_BINS)
    sat, hist = tm.tm_integral_tables(v, prec, offsets, edges, N_BINS, "cumulative")
    L = tm.tm_tonemap_forward(v, sat, hist, edges, p, offsets)
    torch.cuda.synchronize()
    assert np.array_equal(edges.cpu().numpy(), e)

    # integral histogram rows: (y + 1) x the row's cumulative counts
    for pl in range(N_BINS - 1):
        for y in (0, H // 2, H - 1):
            assert np.array_equal(_hist_row(hist, pl, y, W), (y + 1) * G[pl]), (pl, y)
    del sat, hist
    gc.collect()

    # the tone-mapped output against the oracle on the row
    ys = [0, 1, ry[-1], H // 2, H - 2, H - 1]
    bounds = _row_bound(row, H, rx, ry, Lref, Lj, Wj, varj, prec, ys)
    for y, b in zip(ys, bounds[:-1]):
        got = L[y].cpu().numpy().astype(np.float64)
        err = np.abs(got - Lref[0])
        assert np.all(err <= b), (y, float(err.max()), float(b[np.argmax(err - b)]))
    hi = L.amax(dim=0).cpu().numpy().astype(np.float64)
    lo = L.amin(dim=0).cpu().numpy().astype(np.float64)
    worst = np.maximum(np.abs(hi - Lref[0]), np.abs(lo - Lref[0]))
    assert np.all(worst <= bounds[-1]), float(worst.max())
    assert worst.max() <= ENVELOPE[prec], float(worst.max())
    print(f"\n{H}x{W} {prec}: max |err| over all pixels {worst.max():.3e}, "
          f"p99.9 {np.quantile(worst, 0.999):.3e}, median bound {np.median(bounds[-1]):.2e}")
    del v, L, edges, offsets
    gc.collect()
    torch.cuda.empty_cache()
