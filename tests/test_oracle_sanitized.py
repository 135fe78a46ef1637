"""The oracle's C++ built with AddressSanitizer and UBSan (host code only) and
driven over tiny, ragged and degenerate inputs on buffers of exact extent: no
access outside them, no undefined behaviour, no rejected valid call."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_oracle_is_clean_under_sanitizers(tmp_path):
    gxx = shutil.which("g++")
    if not gxx:
        pytest.skip("g++ not available")
    exe = str(tmp_path / "oracle_sanitize")
    cmd = [gxx, "-std=c++17", "-O1", "-g", "-pthread", "-fsanitize=address,undefined",
           "-fno-sanitize-recover=undefined", os.path.join(ROOT, "oracle", "hrrm_oracle.cpp"),
           os.path.join(ROOT, "tests", "native", "oracle_sanitize_drv.cpp"), "-o", exe]
    b = subprocess.run(cmd, capture_output=True, text=True)
    if b.returncode != 0 and "asan" in b.stderr.lower():
        pytest.skip("sanitizer runtime not available: " + b.stderr[-200:])
    assert b.returncode == 0, b.stderr
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:verify_asan_link_order=0")
    p = subprocess.run([exe], capture_output=True, text=True, timeout=300, env=env)
    assert p.returncode == 0, p.stdout + p.stderr[-2000:]
    assert "errors 0" in p.stdout
