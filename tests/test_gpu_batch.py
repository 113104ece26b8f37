"""Batched forward: equal to per-image calls bit for bit, graph replays equal to eager runs,
and the autotuner's choice valid."""
import numpy as np
import pytest
import torch

import paper_2102_01289_amd as tm
from paper_2102_01289_amd import autotune
from _bounds import tiling
from _cases import rgb_case, to_dev

pytestmark = pytest.mark.gpu

SHAPES = [(37, 123), (256, 256), (1, 1), (1, 300), (300, 1), (130, 1030), (64, 2100), (90, 91)]


def _images(seed=0, shapes=SHAPES):
    return [to_dev(rgb_case(h, w, 5, -2.0, 4.0, seed=seed + 7 * i)) for i, (h, w) in
            enumerate(shapes)]


@pytest.mark.parametrize("prec", ["c32x2", "f64", "f32"])
@pytest.mark.parametrize("t", [(4, 16, 4), (2, 5, 2), (8, 32, 8)])
def test_batch_equals_per_image(prec, t):
    imgs = _images()
    b = tm.Batch(imgs, 5, 5, prec=prec, tune=tm.tune(*t))
    outs = [o.clone() for o in b.forward()]
    torch.cuda.synchronize()
    for i, rgb in enumerate(imgs):
        _, H, W = rgb.shape
        p = tm.make_params(5, 5, eps=0.1, H=H, W=W)
        ref = tm.ToneMapper(H, W, p, prec, tune=tm.tune(*t)).run(rgb)
        torch.cuda.synchronize()
        assert torch.equal(outs[i], ref), i


@pytest.mark.parametrize("t", [(4, 0, 4), (0, 8, 2), (0, 0, 4), None])
def test_batch_per_image_tiling(t):
    # 0 fields (and the default tiling): each image scans with its own shape's default;
    # the images are processed grouped by columns per lane, outputs stay in image order
    imgs = _images(seed=11, shapes=SHAPES + [(40, 2500), (20, 4100)])
    b = tm.Batch(imgs, 5, 5, tune=tm.tune(*t) if t else None)
    outs = [o.clone() for o in b.forward()]
    torch.cuda.synchronize()
    tt = t or (0, 0, 4)
    for i, rgb in enumerate(imgs):
        _, H, W = rgb.shape
        p = tm.make_params(5, 5, eps=0.1, H=H, W=W)
        vec, th = tiling(H, W)
        ref = tm.ToneMapper(H, W, p, "c32x2",
                            tune=tm.tune(tt[0] or vec, tt[1] or th, tt[2])).run(rgb)
        torch.cuda.synchronize()
        assert torch.equal(outs[i], ref), i


def test_batch_other_parameters():
    imgs = _images(seed=5, shapes=[(50, 70), (33, 300), (200, 20)])
    b = tm.Batch(imgs, n_bins=64, n_scales=3, eps=0.05, ld_min=0.1, ld_max=0.9)
    outs = [o.clone() for o in b.forward()]
    for i, rgb in enumerate(imgs):
        _, H, W = rgb.shape
        p = tm.make_params(64, 3, eps=0.05, ld_min=0.1, ld_max=0.9, H=H, W=W)
        # the default batch tiling is each image's own default
        ref = tm.ToneMapper(H, W, p, "c32x2").run(rgb)
        assert torch.equal(outs[i], ref)


def test_batch_graph_replays_match_eager():
    imgs = _images(seed=11)
    b = tm.Batch(imgs)
    eager = [o.clone() for o in b.forward()]
    torch.cuda.synchronize()
    s = torch.cuda.Stream()
    b.capture(s)
    for rep in range(3):
        for o in b.outs:
            o.fill_(-1.0)                      # eager work between replays
        b.replay(s)
        s.synchronize()
        for i, o in enumerate(b.outs):
            assert torch.equal(o, eager[i]), (rep, i)
        _ = torch.randn(1000, device="cuda").sum().item()
    # the graph reads the inputs at replay time
    for r in imgs:
        r.mul_(2.0)
    b.replay(s)
    s.synchronize()
    scaled = [o.clone() for o in b.outs]
    fresh = [o.clone() for o in tm.Batch(imgs).forward()]
    torch.cuda.synchronize()
    for a, c in zip(scaled, fresh):
        assert torch.equal(a, c)


def test_autotune_picks_a_valid_tiling(tmp_path, monkeypatch):
    monkeypatch.setenv("TM355_TUNE_CACHE", str(tmp_path / "tune.json"))
    imgs = _images(seed=3, shapes=[(120, 500), (300, 200)])
    t, ms = autotune.tune_batch(imgs, reps=2, cands=[(2, 8, 4), (4, 16, 4), (4, 0, 4)])
    assert (t.tile_w_vec, t.tile_h, t.bin_chunk) in [(2, 8, 4), (4, 16, 4), (4, 0, 4)] and ms > 0
    t2, _ = autotune.tune_image(imgs[0], reps=2)
    assert t2.tile_w_vec in (2, 4, 8)
    t3, _ = autotune.tune_image(imgs[0], reps=2)       # second call is served by the cache
    assert (t3.tile_w_vec, t3.tile_h, t3.bin_chunk) == (t2.tile_w_vec, t2.tile_h, t2.bin_chunk)
    # the single-image path takes the stored tiling on request, and the default without one
    _, H, W = imgs[0].shape
    p = tm.make_params(5, 2, eps=0.1, H=H, W=W)
    m = tm.ToneMapper(H, W, p, "c32x2", tune="cached")
    assert (m.tune.tile_w_vec, m.tune.tile_h, m.tune.bin_chunk) == \
        (t2.tile_w_vec, t2.tile_h, t2.bin_chunk)
    assert torch.equal(m.run(imgs[0]), tm.ToneMapper(H, W, p, "c32x2", tune=t2).run(imgs[0]))
    assert tm.ToneMapper(H, W, p, "f64", tune="cached").tune is None   # nothing stored for f64


@pytest.mark.parametrize("streams,per_group", [(2, 0), (4, 1), (3, 2), (8, 1)])
def test_batch_concurrency_changes_no_output_bit(streams, per_group):
    # groups dealt to internal streams (forked from and joined back to the caller's stream):
    # eager and graph-replayed outputs equal the single-stream batch bit for bit
    imgs = _images(seed=3, shapes=SHAPES + [(40, 2500), (700, 900)])
    b = tm.Batch(imgs, 5, 5)
    ref = [o.clone() for o in b.forward()]
    torch.cuda.synchronize()
    b.set_concurrency(streams, per_group)
    for o in b.outs:
        o.fill_(float("nan"))
    outs = [o.clone() for o in b.forward()]
    torch.cuda.synchronize()
    for i in range(len(imgs)):
        assert torch.equal(outs[i], ref[i]), i
    s = torch.cuda.Stream()
    b.capture(s)
    for rep in range(3):
        for o in b.outs:
            o.fill_(float("nan"))
        torch.cuda.synchronize()
        b.replay(s)
        s.synchronize()
        for i in range(len(imgs)):
            assert torch.equal(b.outs[i], ref[i]), (rep, i)
        _ = torch.randn(1024, device="cuda").sum().item()
    # back to one stream
    b.set_concurrency(1, 0)
    outs = [o.clone() for o in b.forward()]
    torch.cuda.synchronize()
    for i in range(len(imgs)):
        assert torch.equal(outs[i], ref[i]), i


def test_batch_concurrency_arguments():
    b = tm.Batch(_images(seed=4, shapes=[(20, 30)]), 5, 5)
    for bad in ((0, 0), (9, 0), (2, -1)):
        with pytest.raises(tm.TmError):
            b.set_concurrency(*bad)


@pytest.mark.parametrize("prec", ["c32x2", "f64"])
@pytest.mark.parametrize("t", [(4, 16, 4), (2, 5, 2)])
def test_batch_log_variance_equals_per_image(prec, t):
    # the log-domain variant over a batch: every image equals ToneMapper(variance="log"),
    # eagerly and from a graph captured after the switch; switching back restores the
    # linear outputs
    imgs = _images(seed=5)
    imgs[0][:, 3, :4] = 0.0                       # black pixels take the floor constant
    b = tm.Batch(imgs, 5, 5, prec=prec, tune=tm.tune(*t))
    lin = [o.clone() for o in b.forward()]
    b.set_variance("log")
    outs = [o.clone() for o in b.forward()]
    torch.cuda.synchronize()
    for i, rgb in enumerate(imgs):
        _, H, W = rgb.shape
        p = tm.make_params(5, 5, eps=0.1, H=H, W=W)
        ref = tm.ToneMapper(H, W, p, prec, tune=tm.tune(*t), variance="log").run(rgb)
        torch.cuda.synchronize()
        assert torch.equal(outs[i], ref), i
    assert any(not torch.equal(a, c) for a, c in zip(lin, outs))
    s = torch.cuda.Stream()
    b.capture(s)
    for rep in range(3):
        for o in b.outs:
            o.zero_()
        b.replay(s)
        s.synchronize()
        assert all(torch.equal(o, r) for o, r in zip(b.outs, outs)), rep
        _ = torch.randn(4096, device="cuda").sum().item()
    b.set_variance("linear")
    with pytest.raises(tm.TmError):
        b.replay(s)                               # the earlier graph was released
    back = [o.clone() for o in b.forward()]
    torch.cuda.synchronize()
    assert all(torch.equal(a, c) for a, c in zip(lin, back))
    # switches and forwards queued back to back, no synchronisation in between: each
    # forward runs with the variant set before it
    got = []
    for v in ("log", "linear", "log", "log", "linear"):
        b.set_variance(v)
        got.append((v, [o.clone() for o in b.forward()]))
    torch.cuda.synchronize()
    for v, o in got:
        want = outs if v == "log" else lin
        assert all(torch.equal(x, y) for x, y in zip(o, want)), v
