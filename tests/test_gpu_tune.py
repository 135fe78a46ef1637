"""Autotuner and tile table: every tile configuration gives the same output."""
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


CONFIGS = [dict(seg_rows=1), dict(seg_rows=7), dict(seg_rows=300), dict(lds_budget=16 * 1024),
           dict(lds_budget=160 * 1024), dict(nslots=1), dict(nslots=2), dict(max_groups=0),
           dict(max_groups=64), dict(min_group=1), dict(min_group=65), dict(tiered_u8=1),
           dict(tiered_u8=1, max_groups=0), dict(tiered_u8=1, nslots=1), dict(tiered_u8=0),
           dict(raw_window=0), dict(raw_window=100000), dict(raw_window=100000, nslots=1),
           dict(wave_slots=1), dict(wave_slots=1, nslots=1), dict(wave_slots=1, max_groups=0),
           dict(wave_slots=1, lds_budget=160 * 1024), dict(wave_slots=1, raw_window=0)]


@pytest.mark.parametrize("kind,r", [("u8", 3), ("u16", 5), ("u16", 40), ("u8", 70)])
def test_every_tile_config_same_output(hrrm, kind, r):
    ctx = hrrm.Context(0)
    img = datagen.uniform_u8(130, 530, seed=r) if kind == "u8" else datagen.xray_u16(120, 520, seed=r)
    dt = hrrm.U8 if kind == "u8" else hrrm.U16
    want = oracle.median2d(img, r)
    d = to_dev(img)
    for cfg in CONFIGS:
        for variant in ("plain", "adaptive"):
            c = ctx.get_tile(dt, 2, r, variant)
            for k, v in cfg.items():
                setattr(c, k, v)
            ctx.set_tile(dt, 2, r, variant, c)
            announce(kind, r, variant, cfg)
            got = to_host(ctx.median2d(d, r, variant=variant))
            assert np.array_equal(got, want), (cfg, variant, first_mismatch(got, want))
            ctx.set_tile(dt, 2, r, variant, None)


@pytest.mark.parametrize("kind,r", [("u16", 9), ("u16", 15), ("u16", 31), ("u16", 33), ("u16", 64),
                                    ("u16", 127), ("u8", 16), ("u8", 100)])
def test_wave_private_slots(hrrm, kind, r):
    # deeper subtrees in per-wave slots: every wave builds, evicts and updates
    # its own, including windows wider than 64 columns (several update passes)
    ctx = hrrm.Context(0)
    if kind == "u8":
        img, dt = datagen.uniform_u8(110, 600, seed=80 + r), hrrm.U8
    else:
        img, dt = datagen.uniform_u16(100, 560, seed=80 + r), hrrm.U16
    want = oracle.median2d(img, r)
    d = to_dev(img)
    for budget in (24 * 1024, 80 * 1024):
        c = ctx.get_tile(dt, 2, r)
        c.wave_slots, c.lds_budget, c.seg_rows = 1, budget, 37
        ctx.set_tile(dt, 2, r, "plain", c)
        announce("wave slots", kind, r, budget)
        got = to_host(ctx.median2d(d, r))
        assert np.array_equal(got, want), (budget, first_mismatch(got, want))
    ctx.set_tile(dt, 2, r, "plain", None)


def test_autotune_cache_roundtrip(hrrm, tmp_path):
    ctx = hrrm.Context(0)
    path = str(tmp_path / "tune.json")
    tried = ctx.autotune(hrrm.U16, 15, "plain", 1024, 1024, cache_path=path)
    assert tried > 5
    tuned = ctx.get_tile(hrrm.U16, 2, 15).as_dict()
    img = datagen.xray_u16(300, 600, seed=3)
    got = to_host(ctx.median2d(to_dev(img), 15))
    assert np.array_equal(got, oracle.median2d(img, 15))
    # tune on the caller's own data too
    sample = to_dev(datagen.uniform_u8(512, 700, seed=4))
    assert ctx.autotune(hrrm.U8, 3, "plain", sample=sample, cache_path=path) > 3
    ctx2 = hrrm.Context(0)
    ctx2.load_tuning(path)
    assert ctx2.get_tile(hrrm.U16, 2, 15).as_dict() == tuned
    assert "\"r\": 3" in open(path).read()


@pytest.mark.parametrize("kind,r", [("u16", 9), ("u16", 20), ("u8", 12)])
def test_wave_private_slots_rank_and_precision(hrrm, kind, r):
    # other ranks and early stops with per-wave slots (deeper subtrees end at
    # the stop depth; the descent is the median's with another K)
    ctx = hrrm.Context(0)
    if kind == "u8":
        img, dt = datagen.uniform_u8(90, 520, seed=90 + r), hrrm.U8
    else:
        img, dt = datagen.xray_u16(90, 520, seed=90 + r), hrrm.U16
    n = (2 * r + 1) ** 2
    c = ctx.get_tile(dt, 2, r)
    c.wave_slots, c.lds_budget = 1, 40 * 1024
    ctx.set_tile(dt, 2, r, "plain", c)
    d = to_dev(img)
    for k in (0, n // 3, n - 1):
        announce("wave slots rank", kind, r, k)
        got = to_host(ctx.rank2d(d, r, k))
        assert np.array_equal(got, oracle.rank2d(img, r, k)), k
    for drop in (3, 6):
        announce("wave slots drop", kind, r, drop)
        got = to_host(ctx.rank2d(d, r, (n - 1) // 2, drop_levels=drop))
        assert np.array_equal(got, oracle.rank2d(img, r, None, drop_bits=drop)), drop
    ctx.set_tile(dt, 2, r, "plain", None)
