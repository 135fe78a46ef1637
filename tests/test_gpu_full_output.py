"""Whole-output parity at the benchmark workloads' full sizes.

tests/golden/full_output_sha256.json holds, for every workload and radius,
the SHA-256 of the oracle's output (written by make_full_output_hashes.py,
which calls only the oracle) and of the seeded input it was computed from.
Each test regenerates the input, checks its hash (a change of the generators
fails here, not as a filter error), runs the filter on the GPU with the
default tile configuration (the launches the benchmark times) and compares
the SHA-256 of the whole output: every pixel, both tree variants.
"""
import hashlib
import json
import os

import numpy as np
import pytest

from gpu_util import announce, to_dev, to_host
from paper_1105_3829_amd import datagen

pytestmark = pytest.mark.gpu

HERE = os.path.dirname(os.path.abspath(__file__))
TABLE = os.path.join(HERE, "golden", "full_output_sha256.json")

GEN = {
    "c0_u8_512x512_uniform": lambda: datagen.uniform_u8(512, 512, seed=0),
    "c1_u16_4096x4096_xray": lambda: datagen.xray_u16(4096, 4096, seed=1),
    "c2_u8_8192x8192_lowkey": lambda: datagen.lowkey_u8(8192, 8192, seed=2),
    "c3_u16_512x512x256_xray_impulses": lambda: datagen.xray_volume_u16(256, 512, 512, seed=3),
}
# variants checked per workload (the 8-bit sweep also with the full update
# where its window fits the dense build quickly)
VARIANTS = {
    "c0_u8_512x512_uniform": ("plain", "adaptive", "full"),
    "c1_u16_4096x4096_xray": ("plain", "adaptive"),
    "c2_u8_8192x8192_lowkey": ("plain", "adaptive"),
    "c3_u16_512x512x256_xray_impulses": ("plain", "adaptive"),
}


def sha(a: np.ndarray) -> str:
    return hashlib.sha256(np.ascontiguousarray(a).tobytes()).hexdigest()


def table():
    with open(TABLE) as f:
        return json.load(f)


def cases():
    if not os.path.exists(TABLE):
        return []
    out = []
    for name, entry in sorted(table().items()):
        for r in sorted(int(k) for k in entry["output_sha256"]):
            out.append((name, r))
    return out


@pytest.fixture(scope="module")
def hrrm():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1105_3829_amd as m
    m.lib()
    return m


_inputs = {}


def _input(name):
    if name not in _inputs:
        _inputs.clear()
        img = GEN[name]()
        assert sha(img) == table()[name]["input_sha256"], "seeded generator changed: %s" % name
        _inputs[name] = (img, to_dev(img))
    return _inputs[name]


def test_fixture_present():
    assert os.path.exists(TABLE), "run tests/golden/make_full_output_hashes.py"
    t = table()
    assert set(t) == set(GEN)
    assert sorted(int(r) for r in t["c1_u16_4096x4096_xray"]["output_sha256"]) == [1, 5, 15, 50]
    assert len(t["c2_u8_8192x8192_lowkey"]["output_sha256"]) == 8
    assert len(t["c3_u16_512x512x256_xray_impulses"]["output_sha256"]) == 5


@pytest.mark.parametrize("name,r", cases())
def test_whole_output_matches_oracle_hash(hrrm, name, r):
    want = table()[name]["output_sha256"][str(r)]
    img, d = _input(name)
    for variant in VARIANTS[name]:
        announce("full output", name, "r=%d" % r, variant)
        if img.ndim == 3:
            got = to_host(hrrm.median3d(d, r, variant=variant))
        else:
            got = to_host(hrrm.median2d(d, r, variant=variant))
        assert sha(got) == want, (name, r, variant)
