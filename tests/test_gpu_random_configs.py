"""Seeded random sweep: element type, dimensions, radius, image shape, variant
and tile configuration (LDS budget across one to six workgroups per CU,
segment height, wave-wide count threshold, raw-count window, wave-private
slots) drawn together; every output compared bit for bit with the oracle."""
import numpy as np
import pytest

import oracle
from gpu_util import announce, first_mismatch, to_dev, to_host
from paper_1105_3829_amd import datagen

pytestmark = pytest.mark.gpu

BUDGETS = [26880, 40960, 53760, 80 * 1024, 112 * 1024, 160 * 1024]


@pytest.fixture(scope="module")
def hrrm():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1105_3829_amd as m
    m.lib()
    return m


def _case(g):
    dims = 3 if g.random() < 0.25 else 2
    u8 = g.random() < 0.4
    r = int(g.integers(0, 8 if dims == 3 else 80))
    variant = "adaptive" if g.random() < 0.2 else "plain"
    if dims == 3:
        d, h, w = int(g.integers(1, 6)), int(g.integers(1, 40)), int(g.integers(1, 300))
        vol = (np.stack([datagen.lowkey_u8(h, w, seed=int(g.integers(1 << 30))) for _ in range(d)])
               if u8 else datagen.xray_volume_u16(d, h, w, seed=int(g.integers(1 << 30))))
        img = vol
    else:
        h, w = int(g.integers(1, 90)), int(g.integers(1, 600))
        kind = g.integers(0, 3)
        seed = int(g.integers(1 << 30))
        if u8:
            img = datagen.uniform_u8(h, w, seed=seed) if kind == 0 else datagen.lowkey_u8(h, w, seed=seed)
        else:
            img = (datagen.uniform_u16(h, w, seed=seed) if kind == 0 else
                   datagen.diagonal_sine(h, w, period=float(g.integers(5, 60)), bits=16) if kind == 1
                   else datagen.xray_u16(h, w, seed=seed))
    cfg = dict(lds_budget=int(g.choice(BUDGETS)), seg_rows=int(g.choice([1, 3, 8, 17, 48, 200])),
               max_groups=int(g.choice([0, 1, 2, 64])), raw_window=int(g.choice([0, 49, 121, 100000])),
               wave_slots=int(dims == 2 and g.random() < 0.3))
    return dims, u8, r, variant, img, cfg


@pytest.mark.parametrize("seed", range(10))
def test_random_configs(hrrm, seed):
    g = np.random.default_rng(1000 + seed)
    ctx = hrrm.Context(0)
    for i in range(12):
        dims, u8, r, variant, img, cfg = _case(g)
        dt = hrrm.U8 if u8 else hrrm.U16
        c = ctx.get_tile(dt, dims, r, variant)
        for k, v in cfg.items():
            setattr(c, k, v)
        ctx.set_tile(dt, dims, r, variant, c)
        announce("random", seed, i, img.dtype, img.shape, "r=%d" % r, variant, cfg)
        d = to_dev(img)
        if dims == 3:
            got = to_host(ctx.median3d(d, r, variant=variant))
            want = oracle.median3d(img, r)
        else:
            got = to_host(ctx.median2d(d, r, variant=variant))
            want = oracle.median2d(img, r)
        ctx.set_tile(dt, dims, r, variant, None)
        assert np.array_equal(got, want), (seed, i, r, variant, cfg, first_mismatch(got, want))
