"""Python front of the brute-force CPU oracle (``hrrm_oracle.cpp``).

Test infrastructure only: the test-suite, the smoke check and the benchmark's
CPU-baseline leg may call it; the product package never imports it.

Every function takes numpy arrays (x fastest) and returns numpy arrays.  The
result is the plain definition of the running order statistic (median
definition, Sec. II): for each pixel, the k-th smallest (0-based) of the
(2r+1)^D values in its clamp-to-edge window, k = (N-1)/2 for the median.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
import threading

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "hrrm_oracle.cpp")
_LIB = os.path.join(_HERE, "liboracle.so")
_lock = threading.Lock()
_lib = None


def build(force: bool = False) -> str:
    """Compile the oracle with the host compiler (g++), in-tree."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp%d" % os.getpid()
        subprocess.check_call(["g++", "-O2", "-std=c++17", "-fPIC", "-shared", "-pthread",
                               _SRC, "-o", tmp])
        os.replace(tmp, _LIB)
    return _LIB


def _load():
    global _lib
    with _lock:
        if _lib is None:
            build()
            lib = ctypes.CDLL(_LIB)
            i64, i32, vp = ctypes.c_int64, ctypes.c_int, ctypes.c_void_p
            lib.oracle_rank2d.argtypes = [i32, vp, vp, i64, i64, i64, i64, i32, i64, i32, i32]
            lib.oracle_rank2d_u8_thresholds.argtypes = [vp, vp, i64, i64, i64, i64, i32, i64,
                                                        i32]
            lib.oracle_rank3d.argtypes = [i32, vp, vp, i64, i64, i64, i64, i64, i64, i64, i32,
                                          i64, i32]
            lib.oracle_rank2d_at.argtypes = [i32, vp, i64, i64, i64, i32, i64, vp, vp, i64, vp,
                                             i32]
            lib.oracle_rank3d_at.argtypes = [i32, vp, i64, i64, i64, i64, i64, i32, i64, vp, vp,
                                             vp, i64, vp, i32]
            for f in (lib.oracle_rank2d, lib.oracle_rank2d_u8_thresholds, lib.oracle_rank3d, lib.oracle_rank2d_at,
                      lib.oracle_rank3d_at, lib.oracle_default_threads):
                f.restype = ctypes.c_int
            _lib = lib
    return _lib


def default_threads() -> int:
    return int(_load().oracle_default_threads())


def _bytes(a: np.ndarray) -> int:
    if a.dtype == np.uint8:
        return 1
    if a.dtype == np.uint16:
        return 2
    raise TypeError("oracle takes uint8 or uint16 images, got %s" % a.dtype)


def window_size(r: int, dims: int) -> int:
    return (2 * r + 1) ** dims


def median_rank(r: int, dims: int) -> int:
    """0-based rank of the median of an odd window of (2r+1)^dims values."""
    return (window_size(r, dims) - 1) // 2


def rank2d(img: np.ndarray, r: int, k: int | None = None, drop_bits: int = 0,
           threads: int = 0) -> np.ndarray:
    img = np.ascontiguousarray(img)
    assert img.ndim == 2
    h, w = img.shape
    if k is None:
        k = median_rank(r, 2)
    out = np.empty_like(img)
    if h == 0 or w == 0:
        return out
    rc = _load().oracle_rank2d(_bytes(img), img.ctypes.data, out.ctypes.data, w, h, w, w, r, k,
                               drop_bits, threads)
    if rc != 0:
        raise ValueError("oracle_rank2d rejected its arguments")
    return out


def median2d(img: np.ndarray, r: int, threads: int = 0) -> np.ndarray:
    return rank2d(img, r, None, 0, threads)


def rank2d_u8_thresholds(img: np.ndarray, r: int, k: int | None = None,
                         threads: int = 0) -> np.ndarray:
    """Same filter as rank2d for uint8 images, computed by threshold
    decomposition (stacking property): out >= t iff at least N - k window
    values are >= t.  Its cost does not depend on r."""
    img = np.ascontiguousarray(img)
    assert img.ndim == 2 and img.dtype == np.uint8
    h, w = img.shape
    if k is None:
        k = median_rank(r, 2)
    out = np.empty_like(img)
    if h == 0 or w == 0:
        return out
    rc = _load().oracle_rank2d_u8_thresholds(img.ctypes.data, out.ctypes.data, w, h, w, w, r, k,
                                             threads)
    if rc != 0:
        raise ValueError("oracle_rank2d_u8_thresholds rejected its arguments")
    return out


def rank3d(vol: np.ndarray, r: int, k: int | None = None, threads: int = 0) -> np.ndarray:
    vol = np.ascontiguousarray(vol)
    assert vol.ndim == 3
    d, h, w = vol.shape
    if k is None:
        k = median_rank(r, 3)
    out = np.empty_like(vol)
    if vol.size == 0:
        return out
    rc = _load().oracle_rank3d(_bytes(vol), vol.ctypes.data, out.ctypes.data, w, h, d, w, w * h,
                               w, w * h, r, k, threads)
    if rc != 0:
        raise ValueError("oracle_rank3d rejected its arguments")
    return out


def median3d(vol: np.ndarray, r: int, threads: int = 0) -> np.ndarray:
    return rank3d(vol, r, None, threads)


def rank2d_at(img: np.ndarray, r: int, xs, ys, k: int | None = None, threads: int = 0) -> np.ndarray:
    img = np.ascontiguousarray(img)
    h, w = img.shape
    xs = np.ascontiguousarray(xs, dtype=np.int64)
    ys = np.ascontiguousarray(ys, dtype=np.int64)
    if k is None:
        k = median_rank(r, 2)
    out = np.empty(xs.shape[0], dtype=img.dtype)
    rc = _load().oracle_rank2d_at(_bytes(img), img.ctypes.data, w, h, w, r, k, xs.ctypes.data,
                                  ys.ctypes.data, xs.shape[0], out.ctypes.data, threads)
    if rc != 0:
        raise ValueError("oracle_rank2d_at rejected its arguments")
    return out


def rank3d_at(vol: np.ndarray, r: int, xs, ys, zs, k: int | None = None,
              threads: int = 0) -> np.ndarray:
    vol = np.ascontiguousarray(vol)
    d, h, w = vol.shape
    xs = np.ascontiguousarray(xs, dtype=np.int64)
    ys = np.ascontiguousarray(ys, dtype=np.int64)
    zs = np.ascontiguousarray(zs, dtype=np.int64)
    if k is None:
        k = median_rank(r, 3)
    out = np.empty(xs.shape[0], dtype=vol.dtype)
    rc = _load().oracle_rank3d_at(_bytes(vol), vol.ctypes.data, w, h, d, w, w * h, r, k,
                                  xs.ctypes.data, ys.ctypes.data, zs.ctypes.data, xs.shape[0],
                                  out.ctypes.data, threads)
    if rc != 0:
        raise ValueError("oracle_rank3d_at rejected its arguments")
    return out
