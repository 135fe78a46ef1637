"""Builds libhrrm.so (HIP kernels + C ABI) for gfx950, in-tree.

    python -m paper_1105_3829_amd.build          # build (always recompiles)

Every translation unit is compiled by hipcc for gfx950 and linked into one
shared library next to this file.  Packed-FP32 instruction selection is
disabled for all device code.
"""
from __future__ import annotations

import concurrent.futures
import os
import shutil
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
INCLUDE = os.path.join(ROOT, "include")
LIB = os.path.join(HERE, "libhrrm.so")
BUILD_DIR = os.path.join(ROOT, "_build")
ARCH = os.environ.get("HRRM_OFFLOAD_ARCH", "gfx950")

SOURCES = [
    "median_kernels.hip",
    "median_tiered.hip",
    "median_window.hip",
    "topology.hip",
    "batched.hip",
    "hrrm_api.cpp",
    "tune.cpp",
    "server.cpp",
]

COMMON = ["-std=c++17", "-O3", "-fPIC", "-I" + INCLUDE, "-I" + CSRC,
          "-Wall", "-Wno-unused-function", "-Wno-unused-command-line-argument"]
DEVICE = ["--offload-arch=" + ARCH, "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
          "-x", "hip"]
# Per-source flags.  The grey-level-window kernel's LDS atomics from many lanes
# to one address (the running lo/hi counts) are left to the LDS unit: the
# compiler's default rewrite of such atomics into a loop over the active
# lanes costs more instructions than the hardware takes to serialise them.
EXTRA = {"median_window.hip": ["-mllvm", "-amdgpu-atomic-optimizer-strategy=None"]}


def hipcc() -> str:
    p = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"
    return p


def _compile(src: str) -> str:
    os.makedirs(BUILD_DIR, exist_ok=True)
    obj = os.path.join(BUILD_DIR, os.path.splitext(src)[0] + ".o")
    cmd = [hipcc()] + DEVICE + COMMON + EXTRA.get(src, []) + ["-c", os.path.join(CSRC, src), "-o", obj]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError("compile failed: %s\n%s\n%s" % (" ".join(cmd), r.stdout, r.stderr))
    warn = "\n".join(ln for ln in r.stderr.splitlines() if "packed-fp32-ops" not in ln and ln.strip())
    if warn:
        sys.stderr.write(warn + "\n")
    return obj


MEASURE_SRC = os.path.join(HERE, "measure", "peaks.hip")
MEASURE_LIB = os.path.join(HERE, "libhrrm_measure.so")


def build_measure(verbose: bool = True) -> str:
    """libhrrm_measure.so: the benchmark's peak-bandwidth kernels (not the filter)."""
    tmp = MEASURE_LIB + ".tmp%d" % os.getpid()
    cmd = [hipcc()] + DEVICE + COMMON + ["-shared", MEASURE_SRC, "-o", tmp]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError("compile failed: %s\n%s\n%s" % (" ".join(cmd), r.stdout, r.stderr))
    os.replace(tmp, MEASURE_LIB)
    if verbose:
        print("built", MEASURE_LIB)
    return MEASURE_LIB


def build(verbose: bool = True) -> str:
    """Compile every source for gfx950 and link libhrrm.so.  Returns its path."""
    srcs = [s for s in SOURCES if os.path.exists(os.path.join(CSRC, s))]
    with concurrent.futures.ThreadPoolExecutor(max_workers=min(8, len(srcs))) as ex:
        objs = list(ex.map(_compile, srcs))
    tmp = LIB + ".tmp%d" % os.getpid()
    cmd = [hipcc(), "--offload-arch=" + ARCH, "-shared", "-fPIC", "-o", tmp] + objs + ["-lpthread"]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError("link failed: %s\n%s\n%s" % (" ".join(cmd), r.stdout, r.stderr))
    os.replace(tmp, LIB)
    if verbose:
        print("built", LIB)
    return LIB


if __name__ == "__main__":
    build()
