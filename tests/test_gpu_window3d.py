"""Bit-exact parity of the grey-level-window kernel on 16-bit volumes (cube
windows, every slice's tiles in turn) with the CPU oracle.

Each case sets the 3-D tile configuration explicitly (window_rows > 0: window
kernel), except the last, which takes the defaults.  The inputs reach the
kernel's branches in 3-D: leaves scanned as placed and moved (X-ray-like
volumes with 1 % impulses at 0 and 65535), rows counted again with 16-bit
fields (a clamped corner repeats one voxel (r+1)^3 times), and rows left to
the tiered kernel's 3-D pass over the flagged tiles (full-range noise, whose
medians no 128 consecutive grey levels hold).
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


def _check(hrrm, ctx, name, vol, r, variant="plain", window_rows=32):
    announce("window3d", name, vol.shape, "r=%d" % r, variant, "rows=%s" % window_rows)
    if window_rows is not None:
        ctx.set_tile(hrrm.U16, 3, r, variant, window_rows=window_rows)
    try:
        got = to_host(ctx.median3d(to_dev(vol), r, variant=variant))
    finally:
        if window_rows is not None:
            ctx.set_tile(hrrm.U16, 3, r, variant)
    want = oracle.median3d(vol, r)
    assert np.array_equal(got, want), first_mismatch(got, want)


def _noise(d, h, w, seed):
    return datagen.rng(seed).integers(0, 65536, size=(d, h, w), dtype=np.uint16)


@pytest.mark.parametrize("variant", ["plain", "adaptive"])
@pytest.mark.parametrize("r", [1, 2, 3, 5, 7])
def test_xray_volume(hrrm, ctx, r, variant):
    vol = datagen.xray_volume_u16(20, 70, 150, seed=30 + r)
    _check(hrrm, ctx, "xray", vol, r, variant)


@pytest.mark.parametrize("window_rows", [1, 8, 200])
def test_segment_heights(hrrm, ctx, window_rows):
    vol = datagen.xray_volume_u16(9, 40, 131, seed=41)
    _check(hrrm, ctx, "xray", vol, 3, "plain", window_rows)
    _check(hrrm, ctx, "xray", vol, 4, "adaptive", window_rows)


@pytest.mark.parametrize("variant", ["plain", "adaptive"])
def test_rows_left_to_the_tiered_kernel(hrrm, ctx, variant):
    # full-range noise: rows whose medians no pass holds go to the tiered
    # kernel's 3-D pass, whose flags carry the slice
    _check(hrrm, ctx, "noise", _noise(7, 50, 140, seed=42), 3, variant, 16)
    _check(hrrm, ctx, "noise", _noise(6, 40, 130, seed=48), 5, variant, 16)


@pytest.mark.parametrize("shape", [(1, 1, 1), (1, 5, 70), (3, 1, 1), (2, 9, 65), (5, 33, 129),
                                   (11, 2, 64)])
def test_tiny_and_ragged(hrrm, ctx, shape):
    vol = datagen.xray_volume_u16(*shape, seed=43)
    _check(hrrm, ctx, "xray", vol, 3, "plain", 32)
    _check(hrrm, ctx, "xray", vol, 7, "adaptive", 32)


def test_corner_counts_past_a_byte(hrrm, ctx):
    # constant background with a few distinct voxels: leaf counts pass 255
    vol = np.full((12, 40, 90), 3000, np.uint16)
    vol[0, 0, 0] = 10
    vol[5, 20, 45] = 60000
    vol[11, 39, 89] = 2999
    _check(hrrm, ctx, "flat", vol, 7, "plain")
    _check(hrrm, ctx, "flat", vol, 5, "adaptive")


def test_strided_volume(hrrm, ctx):
    import torch
    d, h, w, r = 6, 45, 100, 4
    vol = datagen.xray_volume_u16(d, h, w, seed=44)
    big = np.zeros((d, h + 3, w + 17), np.uint16)
    big[:, :h, :w] = vol
    src = to_dev(big)[:, :h, :w]
    ctx.set_tile(hrrm.U16, 3, r, "plain", window_rows=32)
    try:
        out = torch.zeros((d, h + 5, w + 30), dtype=torch.uint16, device="cuda:0")
        ctx.median3d(src, r, variant="plain", out=out[:, :h, :w])
        got = to_host(out)
    finally:
        ctx.set_tile(hrrm.U16, 3, r, "plain")
    want = oracle.median3d(vol, r)
    assert np.array_equal(got[:, :h, :w], want), first_mismatch(got[:, :h, :w], want)
    assert not got[:, h:, :].any() and not got[:, :, w:].any()


@pytest.mark.parametrize("variant", ["plain", "adaptive"])
def test_default_tiles(hrrm, ctx, variant):
    # the defaults send 16-bit volumes from r = 2 to the window kernel (256
    # grey levels per column up to r = 3)
    vol = datagen.xray_volume_u16(10, 60, 140, seed=45)
    for r in (1, 2, 3, 4):
        _check(hrrm, ctx, "xray", vol, r, variant, None)


def test_forced_tiles_outside_the_window_path(hrrm, ctx):
    # window_rows > 0 where the window kernel does not serve volumes (r = 0,
    # 8-bit data): the tiered kernel computes them, with the same results
    vol = datagen.xray_volume_u16(4, 20, 70, seed=46)
    _check(hrrm, ctx, "xray", vol, 0, "plain", 32)
    v8 = datagen.rng(47).integers(0, 256, size=(5, 20, 70), dtype=np.uint8)
    announce("window3d", "u8 forced", v8.shape)
    ctx.set_tile(hrrm.U8, 3, 2, "plain", window_rows=32)
    try:
        got = to_host(ctx.median3d(to_dev(v8), 2))
    finally:
        ctx.set_tile(hrrm.U8, 3, 2, "plain")
    want = oracle.median3d(v8, 2)
    assert np.array_equal(got, want), first_mismatch(got, want)
