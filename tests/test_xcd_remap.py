"""Host check of the median kernels' workgroup-to-tile map: a permutation of
the tiles for every grid size, with each XCD's workgroups on one contiguous
band (built from the kernel header with hipcc for the host)."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_xcd_remap_is_a_banded_permutation(tmp_path):
    from paper_1105_3829_amd import build as B
    hipcc = B.hipcc()
    if not (os.path.exists(hipcc) or shutil.which(hipcc)):
        pytest.skip("hipcc not available")
    exe = str(tmp_path / "xcd_remap_check")
    src = os.path.join(ROOT, "tests", "native", "xcd_remap_check.cpp")
    subprocess.run([hipcc] + B.DEVICE + B.COMMON + [src, "-o", exe], check=True,
                   capture_output=True, text=True)
    out = subprocess.run([exe], capture_output=True, text=True, timeout=300)
    assert out.returncode == 0, out.stdout + out.stderr
    assert "bad map: 0" in out.stdout
