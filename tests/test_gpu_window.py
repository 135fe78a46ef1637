"""Bit-exact parity of the grey-level-window kernel (2-D) with the CPU oracle,
and of the tiered kernel at the radii where the window kernel is the default.

Each case sets the tile configuration explicitly (window_rows > 0: window
kernel; 0: tiered kernel alone), so both paths are checked whatever the
defaults are.  The inputs reach every branch of the window kernel: leaves
scanned as placed, the range moved and rebuilt, rows counted again with 16-bit
fields (a clamped corner repeats one pixel (r+1)^2 times, more than a byte
holds from r = 15), rows computed in several passes (medians spread wider than
the leaves), and rows left to the tiered kernel (uniform full-range noise,
where no 128 consecutive grey levels hold a row's medians).
"""
import numpy as np
import pytest

import oracle
from gpu_util import announce, first_mismatch, to_dev, to_host
from paper_1105_3829_amd import datagen

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def hrrm():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1105_3829_amd as m
    m.lib()
    return m


@pytest.fixture(scope="module")
def ctx(hrrm):
    return hrrm.Context(0)


def _run(hrrm, ctx, img, r, variant, window_rows, rank=None):
    code = hrrm.U16 if img.dtype == np.uint16 else hrrm.U8
    ctx.set_tile(code, 2, r, variant, window_rows=window_rows)
    try:
        t = to_dev(img)
        if rank is None:
            out = ctx.median2d(t, r, variant=variant)
        else:
            out = ctx.rank2d(t, r, rank=rank, variant=variant)
        return to_host(out)
    finally:
        ctx.set_tile(code, 2, r, variant)


def _check(hrrm, ctx, name, img, r, variant="plain", window_rows=16, rank=None):
    announce("window", name, img.dtype, img.shape, "r=%d" % r, variant, "rows=%d" % window_rows,
             "rank=%s" % rank)
    got = _run(hrrm, ctx, img, r, variant, window_rows, rank)
    want = oracle.rank2d(img, r, rank) if rank is not None else oracle.median2d(img, r)
    assert np.array_equal(got, want), first_mismatch(got, want)


@pytest.mark.parametrize("variant", ["plain", "adaptive"])
@pytest.mark.parametrize("r", [6, 8, 15, 20, 31, 33, 50])
def test_u16_xray(hrrm, ctx, variant, r):
    img = datagen.xray_u16(150, 333, seed=300 + r)
    _check(hrrm, ctx, "xray", img, r, variant)


@pytest.mark.parametrize("variant", ["plain", "adaptive"])
@pytest.mark.parametrize("r", [1, 2, 3, 5, 6, 8, 12, 16, 24, 32])
def test_u8_lowkey(hrrm, ctx, variant, r):
    img = datagen.lowkey_u8(140, 290, seed=320 + r)
    _check(hrrm, ctx, "lowkey", img, r, variant)


@pytest.mark.parametrize("r", [1, 2, 3, 5])
def test_small_radii(hrrm, ctx, r):
    # small windows: 8-bit uniform noise (a row's medians spread over most of
    # the grey range: passes moved and rebuilt, rows left to the tiered
    # kernel) and the 16-bit X-ray-like image, both variants
    img8 = datagen.uniform_u8(90, 300, seed=330 + r)
    img16 = datagen.xray_u16(90, 300, seed=335 + r)
    for variant in ("plain", "adaptive"):
        _check(hrrm, ctx, "noise u8", img8, r, variant)
        _check(hrrm, ctx, "xray small r", img16, r, variant)


@pytest.mark.parametrize("r", [3, 9, 20])
def test_u8_subtree_crossings(hrrm, ctx, r):
    # 8-bit gradients whose row medians drift across the 64-level subtree
    # boundaries: the uniform tree's scan narrows to one subtree and widens
    # again on a miss; a steep ramp also spreads one row over both subtrees
    y, x = np.mgrid[0:160, 0:300]
    for slope in (0.1, 0.5):
        img = np.clip(40 + slope * x + 0.3 * y + (x * 7 + y * 13) % 5, 0, 255).astype(np.uint8)
        for variant in ("plain", "adaptive"):
            _check(hrrm, ctx, "u8 ramp %.1f" % slope, img, r, variant)


@pytest.mark.parametrize("r", [6, 15, 33])
def test_tiered_at_window_defaults(hrrm, ctx, r):
    # the tiered kernel alone at radii where the window kernel is the default
    img = datagen.xray_u16(130, 300, seed=340 + r)
    _check(hrrm, ctx, "xray tiered", img, r, "plain", window_rows=0)
    img8 = datagen.lowkey_u8(120, 280, seed=341 + r)
    _check(hrrm, ctx, "lowkey tiered", img8, r, "plain", window_rows=0)


@pytest.mark.parametrize("shape", [(1, 1), (1, 70), (70, 1), (5, 63), (9, 64), (9, 65), (33, 129),
                                   (3, 200)])
@pytest.mark.parametrize("variant", ["plain", "adaptive"])
def test_tiny_and_ragged(hrrm, ctx, shape, variant):
    h, w = shape
    img = datagen.xray_u16(h, w, seed=350 + h * 7 + w)
    for r in (6, 17):
        _check(hrrm, ctx, "tiny", img, r, variant, window_rows=4)


@pytest.mark.parametrize("window_rows", [1, 3, 7, 64, 1000])
def test_segment_heights(hrrm, ctx, window_rows):
    img = datagen.xray_u16(100, 200, seed=360)
    _check(hrrm, ctx, "segments", img, 9, "adaptive", window_rows=window_rows)
    _check(hrrm, ctx, "segments", img, 9, "plain", window_rows=window_rows)


@pytest.mark.parametrize("r", [15, 20, 40])
def test_corner_counts_past_a_byte(hrrm, ctx, r):
    # a two-level image: every clamped corner window holds (r+1)^2 > 255 copies
    # of the corner pixel, and windows inside the flat regions hold up to
    # (2r+1)^2 copies of one value: rows recounted with 16-bit fields
    g = np.random.default_rng(370 + r)
    img = np.full((90, 200), 1800, np.uint16)
    img[:, 100:] = 1830
    img[g.random(img.shape) < 0.05] = 1815
    for variant in ("plain", "adaptive"):
        _check(hrrm, ctx, "corner", img, r, variant)
    img8 = datagen.lowkey_u8(80, 190, seed=371 + r)
    _check(hrrm, ctx, "corner u8", img8, r, "adaptive")


@pytest.mark.parametrize("r", [6, 12])
def test_wide_medians_multipass(hrrm, ctx, r):
    # a diagonal sine: a row's medians sweep the grey range, so rows take
    # several passes with the range moved, and some go to the tiered kernel
    img = datagen.diagonal_sine(120, 260, period=60.0, bits=16)
    for variant in ("plain", "adaptive"):
        _check(hrrm, ctx, "sine", img, r, variant)
    img8 = datagen.diagonal_sine(120, 260, period=60.0, bits=8)
    _check(hrrm, ctx, "sine u8", img8, r, "plain")


def test_rows_left_to_the_tiered_kernel(hrrm, ctx):
    # i.i.d. full-range 16-bit noise at r = 6: a row's 64 medians spread over
    # thousands of grey levels, so most rows exceed the pass limit and their
    # tiles are recomputed by the tiered kernel
    img = datagen.uniform_u16(100, 300, seed=380)
    for variant in ("plain", "adaptive"):
        _check(hrrm, ctx, "noise", img, 6, variant)


@pytest.mark.parametrize("rank_of", [0.0, 0.1, 0.5, 0.9, 1.0])
def test_rank_filters(hrrm, ctx, rank_of):
    img = datagen.xray_u16(120, 250, seed=390)
    for r in (5, 9):  # 256 and 128 grey levels per column (uniform tree)
        n = (2 * r + 1) ** 2
        k = min(n - 1, int(rank_of * n))
        for variant in ("plain", "adaptive"):
            _check(hrrm, ctx, "rank", img, r, variant, rank=k)


@pytest.mark.parametrize("r", [4, 7])
def test_u16_wide_columns_move(hrrm, ctx, r):
    # 16-bit images at r <= 7 (256 grey levels per column, uniform tree) whose
    # row medians drift across the window of grey levels: steep ramps move it
    # by whole subtrees and rebuild it
    y, x = np.mgrid[0:150, 0:320]
    for slope in (1.0, 4.0):
        img = np.clip(900 + slope * x + 2.0 * y + (x * 7 + y * 13) % 23, 0, 65535).astype(np.uint16)
        _check(hrrm, ctx, "u16 ramp %.0f" % slope, img, r, "plain")


def test_strided_rows(hrrm, ctx):
    import torch
    img = datagen.xray_u16(100, 230, seed=395)
    big = np.zeros((100, 300), np.uint16)
    big[:, :230] = img
    src = to_dev(big)[:, :230]
    ctx.set_tile(hrrm.U16, 2, 11, "adaptive", window_rows=16)
    try:
        out = torch.zeros((100, 300), dtype=torch.uint16, device="cuda:0")
        ctx.median2d(src, 11, variant="adaptive", out=out[:, :230])
        got = to_host(out)
    finally:
        ctx.set_tile(hrrm.U16, 2, 11, "adaptive")
    want = oracle.median2d(img, 11)
    assert np.array_equal(got[:, :230], want), first_mismatch(got[:, :230], want)
    assert not got[:, 230:].any()
    ctx.set_tile(hrrm.U16, 2, 5, "plain", window_rows=16)
    try:
        out = torch.zeros((100, 300), dtype=torch.uint16, device="cuda:0")
        ctx.median2d(src, 5, variant="plain", out=out[:, :230])
        got = to_host(out)
    finally:
        ctx.set_tile(hrrm.U16, 2, 5, "plain")
    want = oracle.median2d(img, 5)
    assert np.array_equal(got[:, :230], want), first_mismatch(got[:, :230], want)
    assert not got[:, 230:].any()


def test_concurrent_streams(hrrm, ctx):
    # calls overlapping in time on two streams, each with rows left to the
    # tiered kernel, keep their own tile flags: each result equals the oracle
    import torch
    imgs = [datagen.uniform_u16(120, 260, seed=400 + i) for i in range(4)]
    want = [oracle.median2d(im, 6) for im in imgs]
    ctx.set_tile(hrrm.U16, 2, 6, "plain", window_rows=8)
    try:
        streams = [torch.cuda.Stream(), torch.cuda.Stream()]
        srcs = [to_dev(im) for im in imgs]
        outs = [torch.empty_like(s) for s in srcs]
        torch.cuda.synchronize()
        for rep in range(3):
            for i, (s, o) in enumerate(zip(srcs, outs)):
                st = streams[i % 2]
                with torch.cuda.stream(st):
                    ctx.median2d(s, 6, out=o, stream=st)
            torch.cuda.synchronize()
            for i, o in enumerate(outs):
                got = to_host(o)
                assert np.array_equal(got, want[i]), (rep, i, first_mismatch(got, want[i]))
    finally:
        ctx.set_tile(hrrm.U16, 2, 6, "plain")
