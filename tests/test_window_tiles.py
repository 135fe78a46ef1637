"""Host check of the grey-level-window kernel's tile layout: the header the
kernel and its launch set-up use (csrc/window_geom.hpp), built with hipcc for
the host; every (strip, row) of an image is covered by exactly one tile, over
many image sizes, segment heights, GPU sizes and radii."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_window_tiles_cover_every_row_once(tmp_path):
    from paper_1105_3829_amd import build as B
    hipcc = B.hipcc()
    if not (os.path.exists(hipcc) or shutil.which(hipcc)):
        pytest.skip("hipcc not available")
    exe = str(tmp_path / "window_tiles_check")
    src = os.path.join(ROOT, "tests", "native", "window_tiles_check.cpp")
    subprocess.run([hipcc] + B.DEVICE + B.COMMON + ["-I", B.CSRC, src, "-o", exe], check=True,
                   capture_output=True, text=True)
    out = subprocess.run([exe], capture_output=True, text=True, timeout=300)
    assert out.returncode == 0, out.stdout[-2000:] + out.stderr[-2000:]
    assert "mismatches 0" in out.stdout
