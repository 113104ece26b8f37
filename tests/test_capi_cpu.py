"""Host-side checks of the C ABI: the library loads without a GPU, exports every entry point
declared in include/tm.h, and rejects bad arguments before launching anything."""
import ctypes
import os
import re

import pytest
import torch

import paper_2102_01289_amd as tm
from paper_2102_01289_amd import _capi

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    names = set()
    for fn in os.listdir(os.path.join(ROOT, "include")):
        if fn.endswith(".h"):
            txt = open(os.path.join(ROOT, "include", fn)).read()
            txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
            names |= set(re.findall(r"\b(tm_[a-z0-9_]+)\s*\(", txt))
    return names


def test_library_exports_every_declared_symbol():
    lib = _capi.load()
    declared = _declared()
    assert {"tm_integral_image", "tm_integral_histogram", "tm_tonemap_forward",
            "tm_tonemap_backward"} <= declared
    for name in sorted(declared):
        assert hasattr(lib, name), name
    # and the binding declares a signature for each of them
    assert declared <= set(_capi.SIGNATURES)


def test_status_strings():
    lib = _capi.load()
    for code in _capi.STATUS:
        assert lib.tm_status_string(code)


def test_geometry_and_radii():
    ld, org, el = tm.table_geometry(3000, 4000)
    assert ld >= 4001 and ld % 64 == 0 and org >= ld + 1 and org % 64 == 0
    assert el >= org + 3000 * ld and el % 64 == 0
    rx, ry = tm.paper_radii(3000, 4000, 5)
    assert rx == [2000, 1000, 500, 250, 125] and ry == [1500, 750, 375, 187, 93]
    rx, ry = tm.paper_radii(256, 256, 5)
    assert rx == ry == [128, 64, 32, 16, 8]


def test_workspace_sizes_grow_with_problem():
    lib = _capi.load()
    a = lib.tm_tables_workspace_bytes(256, 256, 5, 1, None)
    b = lib.tm_tables_workspace_bytes(1080, 1920, 5, 1, None)
    c = lib.tm_tables_workspace_bytes(1080, 1920, 64, 1, None)
    assert 0 < a < b < c
    assert lib.tm_tables_workspace_bytes(0, 10, 5, 1, None) == 0
    assert lib.tm_tables_workspace_bytes(10, 10, 5, 7, None) == 0
    assert lib.tm_image_stats_workspace_bytes(3000, 4000) > 0


def _params(**kw):
    p = tm.make_params(5, 2, [4, 2], [4, 2])
    for k, v in kw.items():
        setattr(p, k, v)
    return p


def test_argument_checks_return_before_launch():
    lib = _capi.load()
    P = ctypes.c_void_p
    fake = P(1 << 20)      # never dereferenced: every call below fails its host checks
    null = P(0)
    # bad shapes / pointers
    assert lib.tm_luminance(fake, 100, 10, 0, 10, fake, 10, null) == -2
    assert lib.tm_luminance(null, 100, 10, 10, 10, fake, 10, null) == -1
    wide = (1 << 24) + 1                                  # one column past TM_MAX_WIDTH
    assert lib.tm_luminance(fake, 2 * wide, wide, 1, wide, fake, wide, null) == -2
    assert lib.tm_luminance(fake, 10, 10, 10, 10, fake, 10, null) == -2     # ch_stride < H*ld
    assert lib.tm_image_stats(fake, 10, 10, 10, 0, fake, null, null, fake, 1 << 20, null) == -1
    assert lib.tm_image_stats(fake, 10, 10, 10, 257, fake, null, null, fake, 1 << 20, null) == -1
    assert lib.tm_image_stats(fake, 10, 10, 10, 5, fake, null, null, null, 0, null) == -4
    # integral tables: ld too small, misaligned table, missing offsets, bad layout
    assert lib.tm_integral_image(fake, 10, 10, 10, 0, null, fake, 10, None, fake, 1 << 20,
                                 null) == -2
    assert lib.tm_integral_image(fake, 10, 10, 10, 0, null, P((1 << 20) + 4), 64, None, fake,
                                 1 << 20, null) == -3
    assert lib.tm_integral_image(fake, 10, 10, 10, 1, null, fake, 64, None, fake, 1 << 20,
                                 null) == -1
    assert lib.tm_integral_image(fake, 10, 10, 10, 9, null, fake, 64, None, fake, 1 << 20,
                                 null) == -1
    assert lib.tm_integral_histogram(fake, 10, 10, 10, fake, 5, 3, fake, 64, 1 << 12, None,
                                     fake, 1 << 20, null) == -1
    assert lib.tm_integral_histogram(fake, 10, 10, 10, fake, 5, 1, fake, 64, 64, None,
                                     fake, 1 << 20, null) == -2           # planes overlap
    assert lib.tm_integral_image(fake, 10, 10, 10, 0, null, fake, 64, None, P((1 << 20) + 8),
                                 1 << 20, null) == -4                      # ws misaligned
    bad_tune = tm.tune(3, 16, 4)
    assert lib.tm_integral_image(fake, 10, 10, 10, 0, null, fake, 64, ctypes.byref(bad_tune),
                                 fake, 1 << 20, null) == -1
    # forward: parameter checks
    for kw in (dict(n_bins=0), dict(n_bins=300), dict(n_scales=0), dict(n_scales=9),
               dict(eps=0.0), dict(eps=float("nan")), dict(ld_min=1.0, ld_max=1.0)):
        p = _params(**kw)
        assert lib.tm_tonemap_forward(fake, 10, 10, 10, fake, 64, 1, fake, fake, 64, 1 << 12,
                                      fake, ctypes.byref(p), fake, 10, null) == -1, kw
    p = _params()
    p.rx[1] = -1
    assert lib.tm_tonemap_forward(fake, 10, 10, 10, fake, 64, 1, fake, fake, 64, 1 << 12, fake,
                                  ctypes.byref(p), fake, 10, null) == -1


def test_residual_planes_must_be_8_byte_aligned():
    lib = _capi.load()
    P = ctypes.c_void_p
    fake = P(1 << 20)
    odd = P((1 << 20) + 4)                          # 4-byte aligned only
    null = P(0)
    p = _params()
    assert lib.tm_tonemap_forward_train(fake, 10, 10, 10, fake, 64, 1, fake, fake, 64, 1 << 12,
                                        fake, ctypes.byref(p), fake, 10, odd, null) == -3
    assert lib.tm_tonemap_backward_resid(fake, 10, 10, 10, ctypes.byref(p), odd, fake, 10, fake,
                                         10, fake, fake, 1 << 20, null) == -3


def test_table_padded_view_layout_on_host():
    # the layout helper itself, exercised on a CPU buffer filled by hand
    H, W = 3, 5
    t = tm.Table(H, W, "u32", planes=2, device="cpu")
    t.buf.zero_()
    b = t.buf.view(2, t.elems)
    for p in range(2):
        for y in range(H):
            for x in range(W):
                b[p, t.origin + y * t.ld + x] = 100 * p + 10 * y + x + 1
    pad = t.padded()[..., 0].to(torch.int64)
    assert pad.shape == (2, H + 1, W + 1)
    assert torch.all(pad[:, 0, :] == 0) and torch.all(pad[:, :, 0] == 0)
    for p in range(2):
        for y in range(H):
            for x in range(W):
                assert pad[p, y + 1, x + 1] == 100 * p + 10 * y + x + 1


def test_default_tune_matches_the_documented_rule():
    from _bounds import tiling
    for H, W in [(3000, 4000), (1080, 1920), (256, 256), (20, 4100), (1, 1), (4000, 360)]:
        for n in (0, 5, 32, 33, 64, 256):
            t = tm.default_tune(H, W, n)
            assert (t.tile_w_vec, t.tile_h, t.bin_chunk) == (*tiling(H, W, n_bins=n), 4)
    assert tm.default_tune(3000, 4000, 64).tile_h == 32
    assert tm.default_tune(1080, 1920, 64).tile_h == 16
    assert tm.default_tune(1080, 1920, 32).tile_h == 8
    t = tm.image_tune(tm.tune(0, 8, 2), 1080, 1920)
    assert (t.tile_w_vec, t.tile_h, t.bin_chunk) == (2, 8, 2)
    t = tm.image_tune(tm.tune(0, 0, 4), 1080, 1920, 64)
    assert (t.tile_w_vec, t.tile_h, t.bin_chunk) == (2, 16, 4)
    lib = _capi.load()
    tt = _capi.TmTune()
    assert lib.tm_default_tune(100, 100, -1, ctypes.byref(tt)) == -1
    assert lib.tm_default_tune(100, 100, 257, ctypes.byref(tt)) == -1


def test_rgb_entry_argument_checks():
    lib = _capi.load()
    P = ctypes.c_void_p
    fake, null = P(1 << 20), P(0)
    p = _params()
    args = lambda sat, cs=100, rgb=fake: (fake, 10, 10, 10, fake, 64, 1, fake, fake, 64, 1 << 12,
                                          fake, ctypes.byref(p), rgb, cs, 10, sat, fake, 100, 10,
                                          null, 0, null)
    for sat in (-0.1, float("nan"), float("inf")):
        assert lib.tm_tonemap_forward_rgb(*args(sat)) == -1, sat
    assert lib.tm_tonemap_forward_rgb(*args(0.6, rgb=null)) == -1
    assert lib.tm_tonemap_forward_rgb(*args(0.6, cs=50)) == -2             # ch_stride < H*ld
    H, W = 30, 40
    pp = tm.make_params(5, 5, H=H, W=W)
    need = lib.tm_tonemap_rgb_workspace_bytes(H, W, ctypes.byref(pp), 1)
    assert need > 0 and lib.tm_tonemap_rgb_workspace_bytes(H, W, ctypes.byref(pp), 7) == 0
    assert lib.tm_tonemap_rgb(fake, H * W, W, H, W, ctypes.byref(pp), 1, 0.6, fake, H * W, W,
                              fake, need - 1, null) == -4


def test_log_and_exposure_entry_argument_checks():
    lib = _capi.load()
    P = ctypes.c_void_p
    fake, null = P(1 << 20), P(0)
    # log-luminance: null output, pitch too small, workspace missing
    assert lib.tm_log_luminance(null, 10, 10, 10, fake, 10, null, null, fake, 1 << 20, null) == -1
    assert lib.tm_log_luminance(fake, 10, 10, 10, fake, 9, null, null, fake, 1 << 20, null) == -2
    assert lib.tm_log_luminance(fake, 10, 10, 10, fake, 10, null, null, null, 0, null) == -4
    # exposure stacks: P out of range, overlapping channel/exposure strides
    ws = lib.tm_hdr_response_workspace_bytes()
    assert ws >= 3 * 255 * 256 * 8
    H, W, ld = 10, 10, 16
    cs, es = H * ld, 3 * H * ld
    f = ctypes.c_float
    resp = lambda P_, es_=es, cs_=cs, n=50, lam=100.0, w=ws: lib.tm_hdr_response(
        fake, es_, cs_, ld, P_, H, W, fake, n, fake, f(lam), fake, fake, w, null)
    assert resp(0) == -1 and resp(17) == -1
    assert resp(4, cs_=H * ld - 1) == -2 and resp(4, es_=3 * cs - 1) == -2
    assert resp(4, n=0) == -1 and resp(4, n=32768 // 4 + 1) == -1
    assert resp(4, lam=-1.0) == -1 and resp(4, lam=float("nan")) == -1
    assert resp(4, w=ws - 1) == -4
    merge = lambda P_, ldo=W, cso=H * W, out=fake: lib.tm_hdr_merge(
        fake, es, cs, ld, P_, H, W, fake, fake, out, cso, ldo, null)
    assert merge(0) == -1 and merge(4, out=null) == -1
    assert merge(4, ldo=W - 1) == -2 and merge(4, cso=H * W - 1) == -2


def test_device_scalars_checks():
    lib = _capi.load()
    P = ctypes.c_void_p
    fake = P(1 << 20)      # never dereferenced: every call below fails its host checks
    null = P(0)
    # device scalars: a misaligned pointer is refused; host eps/ld are then not checked
    p = tm.make_params(5, 2, [4, 2], [4, 2], eps=-1.0, ld_min=1.0, ld_max=0.0)
    bad = (1 << 20) + 2
    p.scalars = bad
    ld, org, el = tm.table_geometry(10, 10)
    assert lib.tm_tonemap_forward(fake, 10, 10, 10, fake, ld, 1, fake, fake, ld, el, fake,
                                  ctypes.byref(p), fake, 10, null) == -3
    p.scalars = None
    assert lib.tm_tonemap_forward(fake, 10, 10, 10, fake, ld, 1, fake, fake, ld, el, fake,
                                  ctypes.byref(p), fake, 10, null) == -1


def test_radii_beyond_the_image_are_clamped_on_the_host():
    # workspace sizing runs the comb schedule on the radii: INT32_MAX must size exactly as the
    # image size does (and not overflow)
    lib = _capi.load()
    big = 2 ** 31 - 1
    a = tm.make_params(5, 3, [big, 4000, 7], [big, 3000, big])
    b = tm.make_params(5, 3, [4000, 4000, 7], [3000, 3000, 3000])
    for f in (lib.tm_backward_workspace_bytes, lib.tm_backward_resid_workspace_bytes):
        sa, sb = f(3000, 4000, ctypes.byref(a)), f(3000, 4000, ctypes.byref(b))
        assert sa == sb > 0


def test_noalloc_prologue_checks():
    lib = _capi.load()
    P = ctypes.c_void_p
    fake = P(1 << 20)      # never dereferenced: every call below fails its host checks
    null = P(0)
    assert lib.tm_prologue_noalloc(null, 100, 10, 10, 10, 5, fake, 10, fake, fake, fake,
                                   null) == -1
    assert lib.tm_prologue_noalloc(fake, 100, 10, 0, 10, 5, fake, 10, fake, fake, fake,
                                   null) == -2
    assert lib.tm_prologue_noalloc(fake, 100, 10, 10, 10, 5, fake, 10, null, fake, fake,
                                   null) == -1          # edges missing with n > 1
    assert lib.tm_prologue_noalloc(fake, 50, 10, 10, 10, 5, fake, 10, fake, fake, fake,
                                   null) == -2          # channel stride below H * ld


def test_lookback_histogram_workspace_and_argument_checks():
    lib = _capi.load()
    P = ctypes.c_void_p
    cum, per = _capi.HIST_LAYOUT["cumulative"], _capi.HIST_LAYOUT["per_bin"]
    # header (256 bytes) + 32-bit row and column records and 64-bit corner records of every
    # tile of 128 columns x 32 rows (each area a whole number of 256-byte blocks)
    up = lambda b: (b + 255) // 256 * 256
    ws = lib.tm_lookback_workspace_bytes(3000, 4000, 5, cum)
    tiles = 32 * ((3000 + 31) // 32)
    assert ws == 256 + up(tiles * 32 * 4 * 4) + up(tiles * 4 * 128 * 4) + up(tiles * 4 * 8)
    # 16 rows per tile when 32 would give fewer than 480 tiles
    tiles = 1 * ((100 + 15) // 16)
    assert lib.tm_lookback_workspace_bytes(100, 100, 5, cum) == \
        256 + up(tiles * 16 * 4 * 4) + up(tiles * 4 * 128 * 4) + up(tiles * 4 * 8)
    # the records hold 30-bit counts: H below 2^30
    assert lib.tm_lookback_workspace_bytes((1 << 30) - 1, 1, 5, cum) > 0
    assert lib.tm_lookback_workspace_bytes(1 << 30, 1, 5, cum) == 0
    assert lib.tm_lookback_workspace_bytes(100, 100, 9, cum) > 0
    assert lib.tm_lookback_workspace_bytes(100, 100, 10, cum) == 0      # 9 planes
    assert lib.tm_lookback_workspace_bytes(100, 100, 9, per) == 0       # 9 planes
    assert lib.tm_lookback_workspace_bytes(100, 100, 0, cum) == 0
    fake = P(1 << 20)
    # no pointers, too many planes: rejected before any device work
    assert lib.tm_integral_histogram_lookback(None, 128, 8, 8, fake, 5, cum, fake, 64, 9 * 64 + 1,
                                              fake, 1 << 20, None) == -1
    assert lib.tm_integral_histogram_lookback(fake, 128, 8, 8, fake, 10, cum, fake, 64,
                                              9 * 64 + 64, fake, 1 << 20, None) == -6
    assert lib.tm_integral_histogram_lookback(fake, 1, 1 << 30, 1, fake, 5, cum, fake, 64,
                                              64 * ((1 << 30) + 1), fake, 1 << 20, None) == -6
    # one bin, cumulative: no planes, nothing to do
    assert lib.tm_integral_histogram_lookback(fake, 128, 8, 8, None, 1, cum, fake, 64, 0,
                                              None, 0, None) == 0


def test_tone_mapper_tune_argument_checked_on_the_host():
    # only a TmTune, None or "cached" is accepted; the check runs before any device work
    p = tm.make_params(5, 1, [1], [1])
    with pytest.raises(ValueError):
        tm.ToneMapper(16, 16, p, "c32x2", tune="fastest", device="cpu")


def test_log_chain_rule_argument_checks():
    # no pointers, overlapping gradient buffers, in place with another pitch: rejected on the
    # host before any device work
    lib = _capi.load()
    P = ctypes.c_void_p
    a = 1 << 20
    assert lib.tm_log_luminance_backward(None, 64, 8, 8, P(a), 64, P(a), 64, None) == -1
    assert lib.tm_log_luminance_backward(P(a), 64, 8, 8, P(a), 64, P(a + 256), 64, None) == -1
    assert lib.tm_log_luminance_backward(P(a), 64, 8, 8, P(a), 64, P(a), 128, None) == -1
    assert lib.tm_log_luminance_backward(P(a), 4, 8, 8, P(a), 64, P(a), 64, None) == -2


def test_split_tables_argument_checks():
    # both planes and both tables are required; the histogram plane's pitch is checked like
    # the other's; all before any device work
    lib = _capi.load()
    P = ctypes.c_void_p
    a = P(1 << 20)
    ok = dict(prec=0, ws=1 << 20)

    def call(vs, ldvs, vh, ldvh, sat, hist, ld_hist=64):
        return lib.tm_integral_tables_split(vs, ldvs, vh, ldvh, 10, 10, ok["prec"], None, sat,
                                            64, a, 5, 1, hist, ld_hist, 1 << 12, None, a,
                                            ok["ws"], None)
    assert call(None, 10, a, 10, a, a) == -1
    assert call(a, 10, None, 10, a, a) == -1
    assert call(a, 10, a, 10, None, a) == -1
    assert call(a, 10, a, 10, a, None) == -1
    assert call(a, 10, a, 9, a, a) == -2          # histogram plane's pitch below W
    assert call(a, 9, a, 10, a, a) == -2


def test_log_residual_backward_argument_checks():
    # the fused log-domain residual backward checks its arguments like the plain one
    lib = _capi.load()
    P = ctypes.c_void_p
    a = P(1 << 20)
    prm = tm.make_params(5, 2, [1, 2], [1, 2], 0.1)
    pr = ctypes.byref(prm)
    assert lib.tm_tonemap_backward_resid_log(None, 64, 8, 8, pr, a, a, 64, a, 64, a, a, 1 << 20,
                                             None) == -1
    assert lib.tm_tonemap_backward_resid_log(a, 64, 8, 8, pr, None, a, 64, a, 64, a, a, 1 << 20,
                                             None) == -1
    assert lib.tm_tonemap_backward_resid_log(a, 64, 8, 8, pr, P((1 << 20) + 4), a, 64, a, 64, a,
                                             a, 1 << 20, None) == -3
    assert lib.tm_tonemap_backward_resid_log(a, 4, 8, 8, pr, a, a, 64, a, 64, a, a, 1 << 20,
                                             None) == -2


def test_log_prologue_argument_checks():
    lib = _capi.load()
    P = ctypes.c_void_p
    a, b = P(1 << 20), P(1 << 24)
    W = 8

    def call(lum, logv, ld_log=64, n=5, edges=a):
        return lib.tm_prologue_log(a, 64 * 8, 64, 8, W, n, lum, 64, logv, ld_log, edges, a, a, a,
                                   1 << 20, None)
    assert call(None, a) == -1                      # no luminance plane
    assert call(b, P((1 << 24) + 64)) == -1         # log plane overlaps the luminance
    assert call(b, a, n=5, edges=None) == -1        # edges needed for more than one bin
    assert call(b, a, ld_log=4) == -2               # pitch below W


def test_log_tables_argument_checks():
    lib = _capi.load()
    P = ctypes.c_void_p
    a = P(1 << 20)
    # no integral image, missing offsets for C32X2, pitch below W
    assert lib.tm_integral_tables_log(a, 64, 8, 8, 1, a, None, 64, a, 5, 1, a, 64, 1 << 12, None,
                                      a, 1 << 20, None) == -1
    assert lib.tm_integral_tables_log(a, 64, 8, 8, 1, None, a, 64, a, 5, 1, a, 64, 1 << 12, None,
                                      a, 1 << 20, None) == -1
    assert lib.tm_integral_tables_log(a, 4, 8, 8, 1, a, a, 64, a, 5, 1, a, 64, 1 << 12, None,
                                      a, 1 << 20, None) == -2


def test_batch_set_variance_argument_checks():
    lib = _capi.load()
    assert lib.tm_batch_set_variance(None, 0, None) == -1
    assert lib.tm_batch_set_variance(None, 2, None) == -1
