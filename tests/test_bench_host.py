"""Host-side parts of bench.py's contract: one GPU only, the LDS work figure
of the roofline, and no silent CPU path."""
import json
import os
import subprocess
import sys

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)


def run_bench(*args, env=None):
    e = dict(os.environ)
    e.update(env or {})
    return subprocess.run([sys.executable, os.path.join(ROOT, "bench.py")] + list(args),
                          capture_output=True, text=True, timeout=300, env=e)


def json_lines(text):
    out = []
    for ln in text.splitlines():
        ln = ln.strip()
        if ln.startswith("{"):
            try:
                out.append(json.loads(ln))
            except ValueError:
                pass
    return out


def test_more_than_one_gpu_is_refused():
    p = run_bench("--gpus", "2")
    assert p.returncode == 2
    assert "one GPU" in p.stderr
    assert not json_lines(p.stdout)


def test_world_size_above_one_is_refused():
    p = run_bench(env={"WORLD_SIZE": "4"})
    assert p.returncode == 2
    assert not json_lines(p.stdout)


def test_lds_work_closed_forms():
    from bench import lds_work_per_pixel
    # every value 0: each of the d levels takes the update (bit 0 -> left node)
    a, zbar, d = lds_work_per_pixel(np.zeros((4, 4), np.uint8))
    assert (zbar, d) == (8.0, 8) and a == 2 * 8 + 2 * 8
    # every value all-ones: no level takes the update, only the descent reads
    a, zbar, d = lds_work_per_pixel(np.full((4, 4), 0xFFFF, np.uint16))
    assert (zbar, d) == (0.0, 16) and a == 2 * 16
    # half 0x0F, half 0xF0 in 8 bits: four zero bits either way
    img = np.array([[0x0F, 0xF0]], np.uint8)
    a, zbar, _ = lds_work_per_pixel(img, "full")
    assert zbar == 4.0 and a == 2 * 4 + 2 * 255
    # a volume's column takes 2r + 1 removals and insertions per row step
    a, zbar, _ = lds_work_per_pixel(np.zeros((2, 2, 2), np.uint16), "plain", r=3)
    assert zbar == 16.0 and a == 2 * 16 * 7 + 2 * 16


@pytest.mark.skipif(__import__("torch").cuda.is_available(), reason="needs a host without a GPU")
def test_no_gpu_fails_loudly():
    p = run_bench("--workload", "c0", "--r", "1", "--steps", "1", "--warmup", "0",
                  "--serving-seconds", "0", "--no-cpu-baseline")
    assert p.returncode != 0
    assert not json_lines(p.stdout)
