"""Host check of the adaptive tree's register-held subtree masks against the
topology walk they replace (Sec. III-C's adaptive topology, one 4-level tier
subtree per lane), over random topologies: built from the kernel header with
hipcc for the host."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_register_subtree_mask_matches_topology_walk(tmp_path):
    from paper_1105_3829_amd import build as B
    hipcc = B.hipcc()
    if not (os.path.exists(hipcc) or shutil.which(hipcc)):
        pytest.skip("hipcc not available")
    exe = str(tmp_path / "amask_check")
    src = os.path.join(ROOT, "tests", "native", "amask_check.cpp")
    subprocess.run([hipcc] + B.DEVICE + B.COMMON + [src, "-o", exe], check=True,
                   capture_output=True, text=True)
    out = subprocess.run([exe], capture_output=True, text=True, timeout=120)
    assert out.returncode == 0, out.stdout + out.stderr
    assert "mismatches 0" in out.stdout
