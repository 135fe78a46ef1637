"""Bit-exact parity of the HIP path (through the C ABI) with the CPU oracle.

Sizes are chosen so the oracle finishes in seconds while the images still
span several 256-column strips, several row segments and a ragged tail.
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


def _check2d(hrrm, img, r, variant="plain", **kw):
    announce("2d", img.dtype, img.shape, "r=%d" % r, variant, kw)
    got = to_host(hrrm.median2d(to_dev(img), r, variant=variant, **kw))
    want = oracle.median2d(img, r)
    assert np.array_equal(got, want), first_mismatch(got, want)


def test_c0_full_image(hrrm):
    img = datagen.uniform_u8(512, 512, seed=0)
    _check2d(hrrm, img, 3)


@pytest.mark.parametrize("r", [0, 1, 2, 5, 15, 31, 32, 33, 63, 64])
def test_u8_radii_ragged(hrrm, r):
    img = datagen.uniform_u8(200, 300, seed=10 + r)
    _check2d(hrrm, img, r)


@pytest.mark.parametrize("r", [100, 127])
def test_u8_large_radius(hrrm, r):
    img = datagen.lowkey_u8(90, 270, seed=r)
    _check2d(hrrm, img, r)
    img = datagen.uniform_u8(60, 300, seed=r + 1)
    _check2d(hrrm, img, r)


@pytest.mark.parametrize("r", [0, 1, 2, 3, 4, 5, 15, 31, 32, 50])
def test_u16_xray_radii(hrrm, r):
    img = datagen.xray_u16(180, 290, seed=20 + r)
    _check2d(hrrm, img, r)


@pytest.mark.parametrize("r", [64, 100, 127])
def test_u16_xray_large_radii_default_tiles(hrrm, r):
    # the 16-bit defaults past r = 63 (whole-LDS tiered tiles, or the window
    # kernel), on an image a few strips wide
    img = datagen.xray_u16(70, 300, seed=30 + r)
    _check2d(hrrm, img, r)
    _check2d(hrrm, img, r, variant="adaptive")


@pytest.mark.parametrize("r", [1, 3, 4, 7, 15])
def test_u16_full_range_many_subtrees(hrrm, r):
    # i.i.d. full-range values: medians scatter over many deep subtrees, which
    # exercises slot eviction and the direct-count path
    img = datagen.uniform_u16(150, 300, seed=30 + r)
    _check2d(hrrm, img, r)


@pytest.mark.parametrize("r", [1, 2, 4])
def test_u16_extremes(hrrm, r):
    g = np.random.default_rng(40 + r)
    img = np.array([0, 1, 65534, 65535], dtype=np.uint16)[g.integers(0, 4, size=(70, 280))]
    _check2d(hrrm, img, r)


@pytest.mark.parametrize("shape", [(1, 1), (1, 2), (2, 1), (3, 3), (5, 1), (1, 7), (2, 257)])
def test_tiny_images(hrrm, shape):
    g = np.random.default_rng(sum(shape))
    for dt, hi in ((np.uint8, 256), (np.uint16, 65536)):
        img = g.integers(0, hi, size=shape).astype(dt)
        for r in (0, 1, 3, 9):
            _check2d(hrrm, img, r)


def test_constant_and_two_level(hrrm):
    _check2d(hrrm, np.full((40, 300), 77, np.uint8), 6)
    _check2d(hrrm, np.full((40, 300), 4095, np.uint16), 6)
    g = np.random.default_rng(3)
    two = np.where(g.random((50, 270)) < 0.5, 0, 65535).astype(np.uint16)
    _check2d(hrrm, two, 3)


@pytest.mark.parametrize("variant", ["adaptive"])
@pytest.mark.parametrize("kind,r", [("u8lowkey", 1), ("u8lowkey", 5), ("u8uniform", 3),
                                    ("u16xray", 2), ("u16xray", 8), ("u16uniform", 3),
                                    ("u8lowkey", 40)])
def test_adaptive(hrrm, kind, r, variant):
    if kind == "u8lowkey":
        img = datagen.lowkey_u8(120, 300, seed=r)
    elif kind == "u8uniform":
        img = datagen.uniform_u8(100, 290, seed=r)
    elif kind == "u16xray":
        img = datagen.xray_u16(110, 280, seed=r)
    else:
        img = datagen.uniform_u16(90, 270, seed=r)
    _check2d(hrrm, img, r, variant)


@pytest.mark.parametrize("dt,r", [(np.uint16, 0), (np.uint16, 1), (np.uint16, 2), (np.uint16, 3),
                                  (np.uint8, 1), (np.uint8, 2), (np.uint8, 5), (np.uint8, 7),
                                  (np.uint16, 7)])
def test_3d(hrrm, dt, r):
    if dt == np.uint16:
        vol = datagen.xray_volume_u16(5, 40, 270, seed=50 + r)
    else:
        vol = np.stack([datagen.lowkey_u8(30, 100, seed=60 + z) for z in range(4)])
    if r == 7:
        vol = vol[:3, :24, :]
    announce("3d", vol.dtype, vol.shape, "r=%d" % r)
    got = to_host(hrrm.median3d(to_dev(vol), r))
    want = oracle.median3d(vol, r)
    assert np.array_equal(got, want), first_mismatch(got, want)


def test_3d_adaptive(hrrm):
    vol = datagen.xray_volume_u16(4, 30, 260, seed=70)
    announce("3d adaptive", vol.shape)
    got = to_host(hrrm.median3d(to_dev(vol), 2, variant="adaptive"))
    assert np.array_equal(got, oracle.median3d(vol, 2))


def test_rank_and_reduced_precision(hrrm):
    img = datagen.xray_u16(90, 280, seed=80)
    r = 4
    n = (2 * r + 1) ** 2
    for k in (0, 1, n // 4, n - 1):
        announce("rank", k)
        got = to_host(hrrm.rank2d(to_dev(img), r, k))
        assert np.array_equal(got, oracle.rank2d(img, r, k)), k
    for drop in (1, 4, 8, 16):
        announce("drop", drop)
        got = to_host(hrrm.rank2d(to_dev(img), r, (n - 1) // 2, drop_levels=drop))
        assert np.array_equal(got, oracle.rank2d(img, r, None, drop_bits=drop)), drop
    img8 = datagen.uniform_u8(80, 270, seed=81)
    for drop in (0, 3, 8):
        got = to_host(hrrm.rank2d(to_dev(img8), r, (n - 1) // 2, drop_levels=drop))
        assert np.array_equal(got, oracle.rank2d(img8, r, None, drop_bits=drop)), drop


def test_strided_rows(hrrm):
    import torch
    img = datagen.uniform_u8(70, 300, seed=90)
    big = torch.zeros((70, 333), dtype=torch.uint8, device="cuda:0")
    big[:, :300] = to_dev(img)
    view = big[:, :300]
    out_big = torch.full((70, 320), 7, dtype=torch.uint8, device="cuda:0")
    out = out_big[:, :300]
    hrrm.median2d(view, 5, out=out)
    got = to_host(out_big)
    assert np.array_equal(got[:, :300], oracle.median2d(img, 5))
    assert (got[:, 300:] == 7).all()  # nothing written past the width


def test_repeatable(hrrm):
    img = datagen.xray_u16(200, 520, seed=91)
    d = to_dev(img)
    a = to_host(hrrm.median2d(d, 9))
    for _ in range(3):
        assert np.array_equal(to_host(hrrm.median2d(d, 9)), a)


@pytest.mark.parametrize("r", [1, 4, 5, 15, 50])
def test_c1_full_size_sampled(hrrm, r):
    # the headline workload at full size: u16 4096^2, both variants, default
    # tiles (the launch the benchmark times); the oracle checks 20000 sampled
    # pixels plus sampled pixels of the first and last rows
    img = datagen.xray_u16(4096, 4096, seed=1)
    d = to_dev(img)
    g = np.random.default_rng(1)
    ys = np.concatenate([g.integers(0, 4096, 20000), np.zeros(512, int), np.full(512, 4095)])
    xs = np.concatenate([g.integers(0, 4096, 20000), g.integers(0, 4096, 1024)])
    want = oracle.rank2d_at(img, r, xs, ys)
    for variant in ("plain", "adaptive"):
        announce("c1 full", "r=%d" % r, variant)
        got = to_host(hrrm.median2d(d, r, variant=variant))
        assert np.array_equal(got[ys, xs], want), variant


@pytest.mark.parametrize("r", [1, 16, 100])
def test_c2_full_size_sampled(hrrm, r):
    # u8 8192^2 low-key image at full size (plain and full-update forms)
    img = datagen.lowkey_u8(8192, 8192, seed=2)
    d = to_dev(img)
    g = np.random.default_rng(2)
    n = 4000 if r == 100 else 20000
    ys = np.concatenate([g.integers(0, 8192, n), np.zeros(256, int), np.full(256, 8191)])
    xs = np.concatenate([g.integers(0, 8192, n), g.integers(0, 8192, 512)])
    want = oracle.rank2d_at(img, r, xs, ys)
    for variant in ("plain", "full"):
        announce("c2 full", "r=%d" % r, variant)
        got = to_host(hrrm.median2d(d, r, variant=variant))
        assert np.array_equal(got[ys, xs], want), variant


@pytest.mark.parametrize("r", [1, 2, 7])
def test_c3_full_size_sampled(hrrm, r):
    # u16 512x512x256 volume with impulses at full size, default tiles (r = 1
    # and 2 count every deeper tier raw at six workgroups per CU)
    vol = datagen.xray_volume_u16(256, 512, 512, seed=3)
    d = to_dev(vol)
    g = np.random.default_rng(3)
    zs = np.concatenate([g.integers(0, 256, 3000), np.zeros(200, int), np.full(200, 255)])
    ys = g.integers(0, 512, zs.size)
    xs = g.integers(0, 512, zs.size)
    want = oracle.rank3d_at(vol, r, xs, ys, zs)
    announce("c3 full", "r=%d" % r)
    got = to_host(hrrm.median3d(d, r))
    assert np.array_equal(got[zs, ys, xs], want)


@pytest.mark.parametrize("r", [0, 1, 5, 31, 33, 64, 100])
def test_full_update_u8(hrrm, r):
    # the unconditional whole-window-tree update gives the same medians
    img = datagen.uniform_u8(120, 300, seed=100 + r) if r % 2 else datagen.lowkey_u8(120, 300,
                                                                                      seed=100 + r)
    _check2d(hrrm, img, r, "full")


def test_full_update_rank_3d_and_errors(hrrm):
    import torch
    img = datagen.uniform_u8(70, 280, seed=110)
    r = 3
    n = (2 * r + 1) ** 2
    for k, drop in ((0, 0), (n // 3, 0), (n - 1, 0), ((n - 1) // 2, 3)):
        announce("full rank", k, drop)
        got = to_host(hrrm.rank2d(to_dev(img), r, k, drop_levels=drop, variant="full"))
        assert np.array_equal(got, oracle.rank2d(img, r, k, drop_bits=drop)), (k, drop)
    vol = np.stack([datagen.lowkey_u8(30, 270, seed=111 + z) for z in range(5)])
    for r3 in (1, 3):
        announce("full 3d", r3)
        got = to_host(hrrm.median3d(to_dev(vol), r3, variant="full"))
        assert np.array_equal(got, oracle.median3d(vol, r3)), r3
    u16 = to_dev(datagen.xray_u16(20, 30, seed=112))
    with pytest.raises(hrrm.HrrmError):
        hrrm.median2d(u16, 2, variant="full")
    torch.cuda.synchronize()


@pytest.mark.parametrize("r", [2, 9])
def test_video_sequence_u16(hrrm, r):
    # frame t's topology comes from frame t-1's median output (left on the
    # device); frame 0 falls back to the running mean
    import torch
    frames = datagen.xray_frames_u16(4, 110, 300, seed=140 + r)
    prev = None
    for t in range(frames.shape[0]):
        announce("video", "r=%d" % r, "frame", t)
        cur = hrrm.median2d_video(to_dev(frames[t]), r, estimate=prev)
        want = oracle.median2d(frames[t], r)
        assert np.array_equal(to_host(cur), want), first_mismatch(to_host(cur), want)
        prev = cur
    # output written over the estimate buffer itself
    est = to_dev(oracle.median2d(frames[2], r))
    got = hrrm.median2d_video(to_dev(frames[3]), r, estimate=est, out=est)
    torch.cuda.synchronize()
    assert np.array_equal(to_host(got), oracle.median2d(frames[3], r))


def test_video_u8_and_degenerate_estimates(hrrm):
    frames = [datagen.lowkey_u8(90, 280, seed=150 + t) for t in range(3)]
    prev = None
    for t, f in enumerate(frames):
        cur = hrrm.median2d_video(to_dev(f), 5, estimate=prev)
        assert np.array_equal(to_host(cur), oracle.median2d(f, 5)), t
        prev = cur
    # estimates unrelated to the frame (constant, all-maximum) change speed, never results
    img = datagen.xray_u16(100, 270, seed=151)
    for fill in (0, 4095, 65535):
        est = to_dev(np.full(img.shape, fill, np.uint16))
        got = to_host(hrrm.median2d_video(to_dev(img), 6, estimate=est))
        assert np.array_equal(got, oracle.median2d(img, 6)), fill


@pytest.mark.parametrize("r", [3, 12, 40])
def test_u16_diagonal_sine(hrrm, r):
    # the paper's worst case: medians change fast along every row, so a wave's
    # pixels want many different deep subtrees (raw counting and wave-local
    # subtree builds instead of slots)
    img = datagen.diagonal_sine(96, 700, period=100.0, bits=16)
    _check2d(hrrm, img, r)
    _check2d(hrrm, datagen.diagonal_sine(80, 300, period=25.0, bits=16), r)


@pytest.mark.parametrize("r", [4, 15, 50])
def test_u16_sharp_edge(hrrm, r):
    # a disc 600 grey levels darker than the X-ray-like background: along rows
    # that cross its rim the medians sweep through many deep subtrees
    img = datagen.xray_u16(200, 600, seed=160 + r).astype(np.int32)
    yy, xx = np.mgrid[0:200, 0:600]
    img[(xx - 300) ** 2 + (yy - 100) ** 2 < 80 ** 2] -= 600
    img = np.clip(img, 0, 4095).astype(np.uint16)
    _check2d(hrrm, img, r)
    _check2d(hrrm, img, r, "adaptive")


@pytest.mark.parametrize("bits_free", [0, 1, 3, 5, 9])
def test_u16_common_prefix(hrrm, bits_free):
    # 16-bit values confined to an aligned or unaligned band: the tile's common
    # prefix fixes many top levels (all of them for a constant image)
    g = np.random.default_rng(120 + bits_free)
    for base in (0x1230, 0xFFFF - (1 << bits_free) + 1, 0x7FF0):
        img = (base + g.integers(0, 1 << bits_free, size=(90, 300))).astype(np.uint16)
        for r in (1, 4, 12):
            _check2d(hrrm, img, r)
        n = 81
        for drop in (2, 13, 16):
            announce("prefix drop", bits_free, hex(base), drop)
            got = to_host(hrrm.rank2d(to_dev(img), 4, (n - 1) // 2, drop_levels=drop))
            assert np.array_equal(got, oracle.rank2d(img, 4, None, drop_bits=drop)), drop


def test_u16_mixed_prefix_tiles(hrrm):
    # tiles with different common prefixes side by side (constant, narrow band,
    # full range), and a band crossing a power-of-two boundary
    g = np.random.default_rng(130)
    img = np.empty((140, 800), np.uint16)
    img[:, :260] = 4000
    img[:, 260:520] = 0x8000 + g.integers(0, 8, size=(140, 260))
    img[:, 520:] = g.integers(0, 65536, size=(140, 280))
    img[100:, :] = (0x7FFC + g.integers(0, 8, size=(40, 800))).astype(np.uint16)
    for r in (2, 7, 20):
        _check2d(hrrm, img, r)


def test_validation_errors(hrrm):
    import torch
    L = hrrm.lib()
    ctx = hrrm.context(0).handle
    d = torch.zeros((10, 10), dtype=torch.uint8, device="cuda:0")
    o = torch.zeros((10, 10), dtype=torch.uint8, device="cuda:0")
    s, t = d.data_ptr(), o.data_ptr()
    assert L.hrrm_median2d(ctx, s, t, 1, 10, 10, 10, 10, -1, 0, None) == hrrm.EINVAL
    assert L.hrrm_median2d(ctx, s, t, 1, 10, 10, 10, 10, 128, 0, None) == hrrm.EUNSUPPORTED
    assert L.hrrm_median2d(ctx, s, t, 3, 10, 10, 10, 10, 1, 0, None) == hrrm.EINVAL
    assert L.hrrm_median2d(ctx, s, t, 1, 10, 10, 9, 10, 1, 0, None) == hrrm.EINVAL
    assert L.hrrm_median2d(ctx, None, t, 1, 10, 10, 10, 10, 1, 0, None) == hrrm.EINVAL
    assert L.hrrm_median2d(ctx, s, s + 5, 1, 10, 10, 10, 10, 1, 0, None) == hrrm.EINVAL
    assert L.hrrm_median2d(ctx, s, t, 1, 10, 10, 10, 10, 1, 7, None) == hrrm.EINVAL
    assert L.hrrm_median2d(ctx, s, t, 1, 0, 10, 10, 10, 1, 0, None) == hrrm.OK
    assert L.hrrm_median2d(None, s, t, 1, 10, 10, 10, 10, 1, 0, None) == hrrm.EINVAL
    assert L.hrrm_median3d(ctx, s, t, 1, 10, 5, 2, 10, 40, 10, 50, 1, 0, None) == hrrm.EINVAL
    assert L.hrrm_median3d(ctx, s, t, 1, 5, 2, 2, 5, 10, 5, 10, 8, 0, None) == hrrm.EUNSUPPORTED
    assert L.hrrm_rank2d(ctx, s, t, 1, 10, 10, 10, 10, 1, 9, 0, 0, None) == hrrm.EINVAL
    assert L.hrrm_rank2d(ctx, s, t, 1, 10, 10, 10, 10, 1, 4, 9, 0, None) == hrrm.EINVAL
    assert L.hrrm_rank2d(ctx, s, t, 1, 10, 10, 10, 10, 1, 4, 2, 1, None) == hrrm.EINVAL
    odd = torch.zeros(21, dtype=torch.uint8, device="cuda:0").data_ptr() + 1
    assert L.hrrm_median2d(ctx, odd, t, 2, 5, 2, 5, 5, 1, 0, None) == hrrm.EINVAL
    torch.cuda.synchronize()
    assert (o == 0).all()  # rejected calls enqueue nothing
