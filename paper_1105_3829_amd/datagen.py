"""Seeded synthetic inputs for the running-median workloads.

This module only draws pixels; it holds none of the filter's arithmetic, so
both the oracle-side tests and the GPU path may use it.

The paper's own test images (an up-scaled "airfield" target, a low-key
photograph, an industrial X-ray of a weld; Sec. IV, Fig. "test images") are not
available, so seeded stand-ins with the same kind of value distribution are
drawn here.  Every generator takes an explicit seed and returns a C-contiguous
numpy array, x fastest.

Recipes (all from numpy's PCG64 via ``default_rng(seed)``):

* ``uniform_u8(h, w)`` - i.i.d. uniform 0..255.
* ``xray_u16(h, w)`` - 12-bit "X-ray-like" values: per pixel a component is
  drawn with weights 0.3/0.5/0.2, then a normal value with mean 800/2000/3100
  and standard deviation 60/150/200; a smooth ramp
  R = 150 * (x/(W-1) + y/(H-1)) - 150 (range -150..+150) is added; the result
  is rounded to nearest and clipped to 0..4095.
* ``lowkey_u8(h, w)`` - low-key image: floor(Exponential(mean 20)) plus an
  independent integer uniform in -3..3, clipped to 0..255 (median near 14).
* ``xray_volume_u16(d, h, w)`` - the 12-bit mixture above without the ramp,
  then every voxel independently with probability 0.01 replaced by 0 or 65535
  (each with probability 1/2): salt-and-pepper impulses.
* ``serving_trace(...)`` - Poisson arrivals of mixed-size u8/u16 requests.
* ``diagonal_sine(h, w, period, bits)`` - the paper's worst-case pattern
  (diagonal sine, Sec. IV), amplitude filling the type's range; supplementary.
"""
from __future__ import annotations

import dataclasses
import itertools
from typing import Iterator, List, Optional

import numpy as np

MIX_WEIGHTS = (0.3, 0.5, 0.2)
MIX_MEANS = (800.0, 2000.0, 3100.0)
MIX_SDS = (60.0, 150.0, 200.0)


def rng(seed: int) -> np.random.Generator:
    return np.random.default_rng(np.random.PCG64(seed))


def uniform_u8(h: int, w: int, seed: int = 0) -> np.ndarray:
    return rng(seed).integers(0, 256, size=(h, w), dtype=np.uint8)


def uniform_u16(h: int, w: int, seed: int = 0, hi: int = 65536) -> np.ndarray:
    return rng(seed).integers(0, hi, size=(h, w), dtype=np.uint16)


def _mixture(g: np.random.Generator, shape) -> np.ndarray:
    comp = g.choice(3, size=shape, p=MIX_WEIGHTS).astype(np.int8)
    means = np.asarray(MIX_MEANS, dtype=np.float32)[comp]
    sds = np.asarray(MIX_SDS, dtype=np.float32)[comp]
    return means + sds * g.standard_normal(size=shape, dtype=np.float32)


def xray_u16(h: int, w: int, seed: int = 1, ramp: bool = True) -> np.ndarray:
    g = rng(seed)
    v = _mixture(g, (h, w))
    if ramp:
        xs = np.arange(w, dtype=np.float32) / np.float32(max(w - 1, 1))
        ys = np.arange(h, dtype=np.float32) / np.float32(max(h - 1, 1))
        v += 150.0 * (xs[None, :] + ys[:, None]) - 150.0
    return np.clip(np.rint(v), 0, 4095).astype(np.uint16)


def xray_frames_u16(n: int, h: int, w: int, seed: int = 5) -> np.ndarray:
    """A seeded sequence of n X-ray-like frames (n, h, w): fresh mixture noise
    per frame (as xray_u16), the ramp, a global brightness drift of +30 grey
    levels per frame and a disc-shaped absorber (-600) of radius min(h, w)/8
    moving from 20 % to 80 % of the width along the middle row."""
    g = rng(seed)
    xs = np.arange(w, dtype=np.float32)
    ys = np.arange(h, dtype=np.float32)
    ramp = 150.0 * (xs[None, :] / np.float32(max(w - 1, 1)) +
                    ys[:, None] / np.float32(max(h - 1, 1))) - 150.0
    out = np.empty((n, h, w), dtype=np.uint16)
    rad2 = (min(h, w) / 8.0) ** 2
    for t in range(n):
        v = _mixture(g, (h, w)) + ramp + np.float32(30.0 * t)
        cx = (0.2 + 0.6 * t / max(n - 1, 1)) * (w - 1)
        cy = 0.5 * (h - 1)
        disc = (xs[None, :] - cx) ** 2 + (ys[:, None] - cy) ** 2 < rad2
        v[disc] -= 600.0
        out[t] = np.clip(np.rint(v), 0, 4095).astype(np.uint16)
    return out


def lowkey_u8(h: int, w: int, seed: int = 2) -> np.ndarray:
    g = rng(seed)
    e = np.floor(g.exponential(20.0, size=(h, w)).astype(np.float32))
    n = g.integers(-3, 4, size=(h, w), dtype=np.int16)
    return np.clip(e.astype(np.int32) + n, 0, 255).astype(np.uint8)


def xray_volume_u16(d: int, h: int, w: int, seed: int = 3, p_impulse: float = 0.01) -> np.ndarray:
    g = rng(seed)
    out = np.empty((d, h, w), dtype=np.uint16)
    for z in range(d):  # slice by slice keeps peak memory small
        v = _mixture(g, (h, w))
        out[z] = np.clip(np.rint(v), 0, 4095).astype(np.uint16)
    hit = g.random(size=(d, h, w), dtype=np.float32) < p_impulse
    hi = g.random(size=(d, h, w), dtype=np.float32) < 0.5
    out[hit & hi] = 65535
    out[hit & ~hi] = 0
    return out


def diagonal_sine(h: int, w: int, period: float = 100.0, bits: int = 8) -> np.ndarray:
    top = (1 << bits) - 1
    ys, xs = np.mgrid[0:h, 0:w].astype(np.float64)
    v = 0.5 * top * (1.0 + np.sin(2.0 * np.pi * (xs + ys) / (period * np.sqrt(2.0))))
    return np.rint(v).astype(np.uint8 if bits == 8 else np.uint16)


def enumerate_images(h: int, w: int, alphabet) -> np.ndarray:
    """All len(alphabet)**(h*w) images over the alphabet, shape (n, h, w)."""
    a = np.asarray(alphabet)
    idx = np.array(list(itertools.product(range(len(a)), repeat=h * w)), dtype=np.int64)
    if idx.size == 0:
        idx = np.zeros((1, 0), dtype=np.int64)
    return a[idx].reshape(-1, h, w)


@dataclasses.dataclass
class Request:
    arrival_s: float
    width: int
    height: int
    dtype: str  # "u8" or "u16"
    radius: int
    seed: int
    pool_index: int = 0  # which pre-drawn pool image the pixels come from
    offset_x: int = 0    # crop origin in the pool image
    offset_y: int = 0
    offset_flat: int = 0  # start of a packed w*h run of the flattened pool image


SERVING_RADII = (1, 2, 3, 7, 15, 31)


def serving_trace(duration_s: float = 5.0, rate_hz: float = 2000.0, seed: int = 4,
                  min_side: int = 256, max_side: int = 4096, pool_images: int = 4,
                  pool_side: int = 4096, max_requests: Optional[int] = None) -> List[Request]:
    """Poisson arrivals; W, H ~ U{min_side..max_side}; half u8, half u16;
    radius uniform over SERVING_RADII.  Requests are crops, at seeded offsets,
    of pre-drawn pool images (uniform u8 pool images for u8 requests, X-ray-like
    u16 pool images for u16 requests), so host memory stays bounded."""
    g = rng(seed)
    out: List[Request] = []
    t = 0.0
    i = 0
    while True:
        t += float(g.exponential(1.0 / rate_hz))
        if t >= duration_s or (max_requests is not None and i >= max_requests):
            break
        w = int(g.integers(min_side, max_side + 1))
        h = int(g.integers(min_side, max_side + 1))
        is16 = bool(g.integers(0, 2))
        rad = int(SERVING_RADII[int(g.integers(0, len(SERVING_RADII)))])
        req = Request(t, w, h, "u16" if is16 else "u8", rad, seed=1000 + i)
        req.pool_index = int(g.integers(0, pool_images))
        req.offset_x = int(g.integers(0, pool_side - w + 1))
        req.offset_y = int(g.integers(0, pool_side - h + 1))
        req.offset_flat = int(g.integers(0, pool_side * pool_side - w * h + 1))
        out.append(req)
        i += 1
    return out


def serving_pool(pool_images: int = 4, pool_side: int = 4096, seed: int = 4,
                 dtype: str = "u16") -> Iterator[np.ndarray]:
    for k in range(pool_images):
        if dtype == "u16":
            yield xray_u16(pool_side, pool_side, seed=10_000 + seed * 100 + k)
        else:
            yield uniform_u8(pool_side, pool_side, seed=20_000 + seed * 100 + k)


def request_pixels(req: Request, pool: Optional[List[np.ndarray]] = None,
                   packed: bool = False) -> np.ndarray:
    """The request's pixels: a crop of its pool image, or with packed=True the
    w*h consecutive pool pixels from offset_flat laid out as rows of width w
    (same value distribution, contiguous in host memory); without a pool, a
    fresh image of the same kind."""
    if pool is None:
        if req.dtype == "u8":
            return uniform_u8(req.height, req.width, seed=req.seed)
        return xray_u16(req.height, req.width, seed=req.seed)
    src = pool[req.pool_index % len(pool)]
    if packed:
        flat = src.reshape(-1)
        return flat[req.offset_flat:req.offset_flat + req.width * req.height].reshape(
            req.height, req.width)
    return np.ascontiguousarray(
        src[req.offset_y:req.offset_y + req.height, req.offset_x:req.offset_x + req.width])
