"""Host check of the clamped-row walk of the window builds (clamp-to-edge
borders): built from the kernel header
with hipcc for the host and compared against the clamp written out directly,
exhaustively over small images and near the ends of very tall ones."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_rowwalk_matches_clamped_rows(tmp_path):
    from paper_1105_3829_amd import build as B
    hipcc = B.hipcc()
    if not (os.path.exists(hipcc) or shutil.which(hipcc)):
        pytest.skip("hipcc not available")
    exe = str(tmp_path / "rowwalk_check")
    src = os.path.join(ROOT, "tests", "native", "rowwalk_check.cpp")
    subprocess.run([hipcc] + B.DEVICE + B.COMMON + [src, "-o", exe], check=True,
                   capture_output=True, text=True)
    out = subprocess.run([exe], capture_output=True, text=True, timeout=120)
    assert out.returncode == 0, out.stdout + out.stderr
    assert "mismatches 0" in out.stdout
