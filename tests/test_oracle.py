"""Pins of the brute-force oracle against what the paper and mathematics fix.

The oracle (oracle/hrrm_oracle.cpp) selects with std::nth_element.  Every pin
here reaches the expected value another way: hand-worked fixtures, counting
instead of selection, numpy's own edge padding instead of the oracle's clamp,
the threshold-decomposition (stacking) property, closed-form special cases and
invariances that hold only for the true middle element of an odd window.
"""
import ctypes
import os
import shutil
import subprocess

import numpy as np
import pytest

import brute
from golden_io import load_cases
from paper_1105_3829_amd import datagen


def test_worked_examples(oracle_mod):
    cases = load_cases()
    assert len(cases) >= 3
    for c in cases:
        if c["dims"] == 2:
            got = oracle_mod.median2d(c["input"], c["r"], threads=1)
        else:
            got = oracle_mod.median3d(c["input"], c["r"], threads=1)
        np.testing.assert_array_equal(got, c["output"], err_msg=c["name"])


TINY_SHAPES = [(1, 1), (1, 2), (2, 1), (2, 2), (1, 3), (3, 1), (1, 4), (1, 5), (1, 6),
               (2, 3), (3, 2)]


@pytest.mark.parametrize("shape", TINY_SHAPES)
def test_exhaustive_tiny_u8(oracle_mod, shape):
    imgs = datagen.enumerate_images(shape[0], shape[1], [0, 1, 2]).astype(np.uint8)
    for r in (0, 1, 2, 3, 5):
        want = brute.median_by_counting(imgs, r, 2)
        for i in range(imgs.shape[0]):
            got = oracle_mod.median2d(imgs[i], r, threads=1)
            if not np.array_equal(got, want[i]):
                raise AssertionError("shape %s r=%d image %s: %s vs %s"
                                     % (shape, r, imgs[i].tolist(), got.tolist(), want[i].tolist()))


def test_exhaustive_3x3_u8(oracle_mod):
    imgs = datagen.enumerate_images(3, 3, [0, 1, 2]).astype(np.uint8)
    for r in (1, 2):
        want = brute.median_by_counting(imgs, r, 2)
        got = np.stack([oracle_mod.median2d(im, r, threads=1) for im in imgs])
        np.testing.assert_array_equal(got, want)


@pytest.mark.parametrize("shape", [(1, 1), (2, 2), (1, 4), (4, 1), (2, 3)])
def test_exhaustive_tiny_u16_extremes(oracle_mod, shape):
    imgs = datagen.enumerate_images(shape[0], shape[1], [0, 1, 65534, 65535]).astype(np.uint16)
    for r in (0, 1, 2, 4):
        want = brute.median_by_counting(imgs, r, 2)
        got = np.stack([oracle_mod.median2d(im, r, threads=1) for im in imgs])
        np.testing.assert_array_equal(got, want)


def test_exhaustive_cube_2x2x2(oracle_mod):
    flat = datagen.enumerate_images(1, 8, [0, 1]).astype(np.uint8)
    vols = flat.reshape(-1, 2, 2, 2)
    for r in (0, 1, 2):
        want = brute.median_by_counting(vols, r, 3)
        got = np.stack([oracle_mod.median3d(v, r, threads=1) for v in vols])
        np.testing.assert_array_equal(got, want)


@pytest.mark.parametrize("dtype,hw,r", [(np.uint8, (7, 11), 1), (np.uint8, (13, 5), 3),
                                        (np.uint16, (9, 10), 2), (np.uint16, (6, 17), 7),
                                        (np.uint8, (4, 4), 9)])
def test_certificate_random(oracle_mod, dtype, hw, r):
    g = np.random.default_rng(hash((hw, r)) % 2**32)
    hi = 256 if dtype == np.uint8 else 65536
    for trial in range(3):
        img = g.integers(0, hi if trial != 1 else 4, size=hw).astype(dtype)
        out = oracle_mod.median2d(img, r)
        k = ((2 * r + 1) ** 2 - 1) // 2
        assert brute.certificate_ok(img, out, r, 2, k)
        np.testing.assert_array_equal(out, brute.median_by_counting(img, r, 2))


def test_certificate_3d(oracle_mod):
    g = np.random.default_rng(5)
    vol = g.integers(0, 65536, size=(5, 6, 7)).astype(np.uint16)
    for r in (1, 2):
        out = oracle_mod.median3d(vol, r)
        k = ((2 * r + 1) ** 3 - 1) // 2
        assert brute.certificate_ok(vol, out, r, 3, k)


@pytest.mark.parametrize("dtype,top", [(np.uint8, 255), (np.uint16, 65535)])
def test_complement_invariance(oracle_mod, dtype, top):
    # med(M - I) = M - med(I) holds only for the middle element of an odd window;
    # an off-by-one rank breaks it.
    g = np.random.default_rng(7)
    img = g.integers(0, top + 1, size=(37, 29)).astype(dtype)
    for r in (1, 2, 5, 16):
        a = oracle_mod.median2d(img, r)
        b = oracle_mod.median2d((top - img.astype(np.int64)).astype(dtype), r)
        np.testing.assert_array_equal(b.astype(np.int64), top - a.astype(np.int64))
    vol = g.integers(0, top + 1, size=(6, 7, 8)).astype(dtype)
    a = oracle_mod.median3d(vol, 1)
    b = oracle_mod.median3d((top - vol.astype(np.int64)).astype(dtype), 1)
    np.testing.assert_array_equal(b.astype(np.int64), top - a.astype(np.int64))


def test_monotone_remap_invariance(oracle_mod):
    g = np.random.default_rng(11)
    img = g.integers(0, 256, size=(31, 23)).astype(np.uint8)
    lut8 = np.sort(g.integers(0, 256, size=256)).astype(np.uint8)       # non-decreasing
    lut16 = np.sort(g.integers(0, 65536, size=256)).astype(np.uint16)
    for r in (1, 3, 6):
        m = oracle_mod.median2d(img, r)
        np.testing.assert_array_equal(oracle_mod.median2d(lut8[img], r), lut8[m])
        np.testing.assert_array_equal(oracle_mod.median2d(lut16[img], r), lut16[m])
        widened = img.astype(np.uint16) * 257
        np.testing.assert_array_equal(oracle_mod.median2d(widened, r), m.astype(np.uint16) * 257)
        shifted = (img.astype(np.uint16) << 8) | 0x5A
        np.testing.assert_array_equal(oracle_mod.median2d(shifted, r),
                                      (m.astype(np.uint16) << 8) | 0x5A)


def test_trivial_cases(oracle_mod):
    g = np.random.default_rng(3)
    img = g.integers(0, 65536, size=(19, 33)).astype(np.uint16)
    np.testing.assert_array_equal(oracle_mod.median2d(img, 0), img)          # r = 0
    c = np.full((9, 14), 123, dtype=np.uint8)
    for r in (1, 4, 20):
        np.testing.assert_array_equal(oracle_mod.median2d(c, r), c)          # constant
    for r in (0, 1, 7, 40):
        one = np.array([[201]], dtype=np.uint8)
        np.testing.assert_array_equal(oracle_mod.median2d(one, r), one)      # 1x1
        two = np.array([[5, 250]], dtype=np.uint8)                          # own pixel: r+1 vs r
        np.testing.assert_array_equal(oracle_mod.median2d(two, r), two)
        np.testing.assert_array_equal(oracle_mod.median2d(two.T.copy(), r), two.T)
    vol = g.integers(0, 65536, size=(4, 5, 6)).astype(np.uint16)
    np.testing.assert_array_equal(oracle_mod.median3d(vol, 0), vol)


def test_flip_transpose_equivariance(oracle_mod):
    g = np.random.default_rng(13)
    img = g.integers(0, 256, size=(21, 34)).astype(np.uint8)
    for r in (1, 4, 11):
        m = oracle_mod.median2d(img, r)
        np.testing.assert_array_equal(oracle_mod.median2d(img[:, ::-1].copy(), r), m[:, ::-1])
        np.testing.assert_array_equal(oracle_mod.median2d(img[::-1, :].copy(), r), m[::-1, :])
        np.testing.assert_array_equal(oracle_mod.median2d(img.T.copy(), r), m.T)
    vol = g.integers(0, 65536, size=(5, 7, 9)).astype(np.uint16)
    m3 = oracle_mod.median3d(vol, 1)
    for perm in [(0, 2, 1), (1, 0, 2), (2, 1, 0)]:
        np.testing.assert_array_equal(
            oracle_mod.median3d(np.ascontiguousarray(vol.transpose(perm)), 1), m3.transpose(perm))
    np.testing.assert_array_equal(oracle_mod.median3d(vol[::-1].copy(), 1), m3[::-1])


def test_dimension_reductions(oracle_mod):
    g = np.random.default_rng(17)
    img = g.integers(0, 65536, size=(12, 15)).astype(np.uint16)
    for r in (1, 2, 3):
        m2 = oracle_mod.median2d(img, r)
        # depth 1: the z-axis clamps onto the single slice; each 2-D window
        # multiset is repeated 2r+1 times, which keeps its median
        np.testing.assert_array_equal(oracle_mod.median3d(img[None], r)[0], m2)
        # identical slices give the per-slice 2-D median
        stack = np.repeat(img[None], 4, axis=0)
        np.testing.assert_array_equal(oracle_mod.median3d(stack, r), np.repeat(m2[None], 4, 0))
    # identical rows: each window is 2r+1 copies of a 1-D clamped window
    row = g.integers(0, 256, size=(1, 40)).astype(np.uint8)
    rows = np.repeat(row, 6, axis=0)
    for r in (1, 3, 8):
        one_d = np.median(brute.windows(row[0], r, 1).astype(np.int64), axis=-1).astype(np.uint8)
        np.testing.assert_array_equal(oracle_mod.median2d(rows, r), np.repeat(one_d[None], 6, 0))


@pytest.mark.parametrize("r", [1, 3, 8, 20])
def test_threshold_decomposition_u8(oracle_mod, r):
    g = np.random.default_rng(100 + r)
    img = g.integers(0, 256, size=(96, 77)).astype(np.uint8)
    np.testing.assert_array_equal(oracle_mod.median2d(img, r), brute.median_by_thresholds_u8(img, r))
    low = datagen.lowkey_u8(64, 90, seed=r)
    np.testing.assert_array_equal(oracle_mod.median2d(low, r), brute.median_by_thresholds_u8(low, r))


@pytest.mark.parametrize("r", [0, 1, 2, 5, 17, 40])
def test_threshold_path_equals_selection(oracle_mod, r):
    # the oracle's two routes to the 8-bit rank filter (nth_element per window,
    # threshold decomposition with box counts) must agree everywhere
    g = np.random.default_rng(300 + r)
    shapes = [(1, 1), (1, 7), (5, 1), (33, 47), (70, 130)]
    for h, w in shapes:
        img = g.integers(0, 256, size=(h, w)).astype(np.uint8)
        n = (2 * r + 1) ** 2
        for k in sorted({0, (n - 1) // 2, n - 1, n // 3}):
            np.testing.assert_array_equal(oracle_mod.rank2d_u8_thresholds(img, r, k),
                                          oracle_mod.rank2d(img, r, k))
    ext = np.where(g.random((40, 50)) < 0.5, 0, 255).astype(np.uint8)  # only the extremes
    np.testing.assert_array_equal(oracle_mod.rank2d_u8_thresholds(ext, r),
                                  oracle_mod.median2d(ext, r))
    low = datagen.lowkey_u8(90, 61, seed=r)
    np.testing.assert_array_equal(oracle_mod.rank2d_u8_thresholds(low, r),
                                  brute.median_by_thresholds_u8(low, r))


def test_rank_extremes_and_general(oracle_mod):
    g = np.random.default_rng(19)
    img = g.integers(0, 65536, size=(17, 23)).astype(np.uint16)
    for r in (1, 3):
        w = brute.windows(img, r, 2)
        n = w.shape[-1]
        np.testing.assert_array_equal(oracle_mod.rank2d(img, r, 0), w.min(-1))       # min filter
        np.testing.assert_array_equal(oracle_mod.rank2d(img, r, n - 1), w.max(-1))   # max filter
        for k in (1, n // 4, n - 2):
            np.testing.assert_array_equal(oracle_mod.rank2d(img, r, k),
                                          brute.rank_by_counting(img, r, 2, k))


def test_reduced_precision_from_counts(oracle_mod):
    # independent pin of the drop_bits branch: the early-stopped descent's
    # lower bound computed from coarse threshold counts (tests/brute.py), with
    # no selection and no bit mask
    g = np.random.default_rng(41)
    img16 = (g.integers(0, 64, size=(9, 11)) * 1031 % 65536).astype(np.uint16)
    img8 = g.integers(0, 256, size=(10, 9)).astype(np.uint8)
    for img, bits in ((img16, (0, 3, 9, 12, 16)), (img8, (0, 1, 4, 7, 8))):
        for r in (1, 2):
            n = (2 * r + 1) ** 2
            for k in (0, (n - 1) // 2, n - 1):
                for b in bits:
                    np.testing.assert_array_equal(
                        oracle_mod.rank2d(img, r, k, drop_bits=b),
                        brute.rank_dropped_by_coarse_counts(img, r, 2, k, b))


def test_reduced_precision(oracle_mod):
    g = np.random.default_rng(23)
    img = datagen.xray_u16(40, 50, seed=23)
    exact = oracle_mod.median2d(img, 3)
    for b in (0, 1, 4, 8, 16):
        got = oracle_mod.rank2d(img, 3, None, drop_bits=b)
        np.testing.assert_array_equal(got, exact & np.uint16((0xFFFF << b) & 0xFFFF))
        # error bound of Sec. III-D: at most the width of the last node
        assert np.all(exact.astype(np.int64) - got.astype(np.int64) < (1 << b))


def test_sampled_points_match_full(oracle_mod):
    img = datagen.xray_u16(60, 70, seed=29)
    full = oracle_mod.median2d(img, 5)
    g = np.random.default_rng(29)
    ys = g.integers(0, 60, 500)
    xs = g.integers(0, 70, 500)
    np.testing.assert_array_equal(oracle_mod.rank2d_at(img, 5, xs, ys), full[ys, xs])
    vol = datagen.xray_volume_u16(6, 9, 11, seed=31)
    full3 = oracle_mod.median3d(vol, 2)
    zs = g.integers(0, 6, 200)
    ys = g.integers(0, 9, 200)
    xs = g.integers(0, 11, 200)
    np.testing.assert_array_equal(oracle_mod.rank3d_at(vol, 2, xs, ys, zs), full3[zs, ys, xs])


def test_strided_buffers(oracle_mod):
    # the C entry points take element strides; a padded layout must give the
    # same result as the packed one
    lib = oracle_mod._load()
    img = datagen.uniform_u8(13, 21, seed=37)
    pad = np.zeros((13, 32), dtype=np.uint8)
    pad[:, :21] = img
    out = np.zeros((13, 40), dtype=np.uint8)
    rc = lib.oracle_rank2d(1, pad.ctypes.data, out.ctypes.data, 21, 13, 32, 40, 2, 12, 0, 1)
    assert rc == 0
    np.testing.assert_array_equal(out[:, :21], oracle_mod.median2d(img, 2))
    assert not out[:, 21:].any()
    assert lib.oracle_rank2d(1, pad.ctypes.data, out.ctypes.data, 21, 13, 20, 40, 2, 12, 0, 1) == -1


# A plausible mistake anywhere in the oracle must fail at least one pin.  Each
# mutant below is a copy of the oracle source with one planted mistake, built
# on the CPU; the pins are re-run against it and must not all pass.
MUTANTS = {
    "rank_off_by_one": ("buf.begin() + k, buf.begin() + n);\n  return buf[k];",
                        "buf.begin() + k + 1, buf.begin() + n);\n  return buf[k + 1];"),
    "clamp_short": ("const int64_t xx = clampi(x + dx, 0, w - 1);\n      buf[n++] = src[yy * stride + xx];",
                    "const int64_t xx = clampi(x + dx, 0, w - 2 < 0 ? 0 : w - 2);\n      buf[n++] = src[yy * stride + xx];"),
    "dropped_column": ("for (int64_t dx = -r; dx <= r; ++dx) {\n      const int64_t xx = clampi(x + dx, 0, w - 1);\n      buf[n++] = src[yy * stride + xx];",
                       "for (int64_t dx = -r; dx <= r; ++dx) {\n      const int64_t xx = clampi(x + (dx == r ? -r : dx), 0, w - 1);\n      buf[n++] = src[yy * stride + xx];"),
    "transposed_window": ("const int64_t yy = clampi(y + dy, 0, h - 1);\n    for (int64_t dx = -r; dx <= r; ++dx) {\n      const int64_t xx = clampi(x + dx, 0, w - 1);",
                          "const int64_t yy = clampi(y + dy / 2, 0, h - 1);\n    for (int64_t dx = -r; dx <= r; ++dx) {\n      const int64_t xx = clampi(x + dx, 0, w - 1);"),
    "wrap_border": ("const int64_t xx = clampi(x + dx, 0, w - 1);\n      buf[n++] = src[yy * stride + xx];",
                    "const int64_t xx = ((x + dx) % w + w) % w;\n      buf[n++] = src[yy * stride + xx];"),
}


import contextlib


@contextlib.contextmanager
def _oracle_from(lib_path):
    """Point the oracle loader at another shared library for the duration."""
    import oracle as orc
    saved = (orc._lib, orc._LIB, orc.build)
    orc._lib, orc._LIB = None, lib_path
    orc.build = lambda force=False: lib_path
    try:
        yield orc
    finally:
        orc._lib, orc._LIB, orc.build = saved


def _pins_pass(lib_path):
    with _oracle_from(lib_path) as orc:
        for fn in (test_worked_examples, test_complement_invariance_u8_only,
                   test_threshold_small, test_trivial_cases):
            try:
                fn(orc)
            except AssertionError:
                return False
        return True


def test_complement_invariance_u8_only(oracle_mod):
    g = np.random.default_rng(8)
    img = g.integers(0, 256, size=(9, 12)).astype(np.uint8)
    for r in (1, 2):
        a = oracle_mod.median2d(img, r)
        b = oracle_mod.median2d((255 - img).astype(np.uint8), r)
        np.testing.assert_array_equal(b.astype(np.int64), 255 - a.astype(np.int64))


def test_threshold_small(oracle_mod):
    g = np.random.default_rng(9)
    img = g.integers(0, 256, size=(11, 14)).astype(np.uint8)
    for r in (1, 2):
        np.testing.assert_array_equal(oracle_mod.median2d(img, r), brute.median_by_thresholds_u8(img, r))


@pytest.mark.skipif(shutil.which("g++") is None, reason="needs g++")
@pytest.mark.parametrize("name", sorted(MUTANTS))
def test_pins_catch_planted_mistakes(tmp_path, oracle_mod, name):
    import oracle as orc
    src = open(orc._SRC).read()
    old, new = MUTANTS[name]
    assert old in src, "mutant anchor not found: " + name
    mutated = src.replace(old, new)
    cpp = tmp_path / "mutant.cpp"
    cpp.write_text(mutated)
    so = tmp_path / "libmutant.so"
    subprocess.check_call(["g++", "-O1", "-std=c++17", "-fPIC", "-shared", "-pthread", str(cpp),
                           "-o", str(so)])
    # the unmutated oracle passes the same pins; the mutant must not
    assert _pins_pass(orc._LIB)
    assert not _pins_pass(str(so)), "planted mistake %s went unnoticed" % name
