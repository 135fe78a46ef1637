"""MI355X (gfx950) hierarchical recursive running median.

Thin ctypes binding over ``libhrrm.so`` (the C ABI in ``include/hrrm.h``):
argument marshalling only, every step of the filter runs in the library's HIP
kernels.  PyTorch supplies device memory and streams.

    import torch, paper_1105_3829_amd as hrrm
    img = torch.randint(0, 4096, (4096, 4096), dtype=torch.uint16, device="cuda")
    out = hrrm.median2d(img, r=15)                   # plain (uniform tree)
    out = hrrm.median2d(img, r=15, variant="adaptive")

The binding raises if the shared library has not been built
(``python -m paper_1105_3829_amd.build``); there is no fallback path.
"""
from __future__ import annotations

import ctypes
import os
import threading
from typing import List, Optional, Sequence

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libhrrm.so")

OK, EINVAL, ENOMEM, EUNSUPPORTED, EDEVICE, EAGAIN = 0, -1, -2, -3, -4, -5
U8, U16 = 1, 2
PLAIN, ADAPTIVE, FULL_UPDATE = 0, 1, 2
MAX_R_2D, MAX_R_3D = 127, 7

_lib = None
_lock = threading.Lock()


class HrrmError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__("hrrm error %d: %s" % (code, msg))
        self.code = code


class _Image(ctypes.Structure):
    _fields_ = [("src", ctypes.c_void_p), ("dst", ctypes.c_void_p), ("width", ctypes.c_int64),
                ("height", ctypes.c_int64), ("src_row_stride", ctypes.c_int64),
                ("dst_row_stride", ctypes.c_int64), ("dtype", ctypes.c_int32),
                ("r", ctypes.c_int32)]


class TileConfig(ctypes.Structure):
    _fields_ = [("seg_rows", ctypes.c_int32), ("nslots", ctypes.c_int32),
                ("min_group", ctypes.c_int32), ("max_groups", ctypes.c_int32),
                ("lds_budget", ctypes.c_int32), ("tiered_u8", ctypes.c_int32),
                ("raw_window", ctypes.c_int32), ("wave_slots", ctypes.c_int32),
                ("window_rows", ctypes.c_int32)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


class _Request(ctypes.Structure):
    _fields_ = [("src", ctypes.c_void_p), ("width", ctypes.c_int64), ("height", ctypes.c_int64),
                ("src_row_stride", ctypes.c_int64), ("dtype", ctypes.c_int32),
                ("r", ctypes.c_int32)]


class _Result(ctypes.Structure):
    _fields_ = [("d_dst", ctypes.c_void_p), ("width", ctypes.c_int64), ("height", ctypes.c_int64),
                ("dtype", ctypes.c_int32), ("status", ctypes.c_int32), ("t_submit", ctypes.c_double),
                ("t_admit", ctypes.c_double), ("t_done", ctypes.c_double)]


def lib():
    """Load libhrrm.so (raises if it is missing: no fallback exists)."""
    global _lib
    with _lock:
        if _lib is None:
            if not os.path.exists(LIB_PATH):
                raise ImportError("libhrrm.so is not built; run `python -m paper_1105_3829_amd.build`")
            L = ctypes.CDLL(LIB_PATH)
            i32, i64, vp, cp = ctypes.c_int32, ctypes.c_int64, ctypes.c_void_p, ctypes.c_char_p
            sig = {
                "hrrm_last_error": ([], cp),
                "hrrm_version": ([], cp),
                "hrrm_ctx_create": ([i32, ctypes.POINTER(vp)], i32),
                "hrrm_ctx_destroy": ([vp], i32),
                "hrrm_ctx_reserve": ([vp, i32, i64, i32, i32], i32),
                "hrrm_median2d": ([vp, vp, vp, i32, i64, i64, i64, i64, i32, i32, vp], i32),
                "hrrm_median3d": ([vp, vp, vp, i32, i64, i64, i64, i64, i64, i64, i64, i32, i32, vp],
                                  i32),
                "hrrm_rank2d": ([vp, vp, vp, i32, i64, i64, i64, i64, i32, i64, i32, i32, vp], i32),
                "hrrm_rank2d_noalloc": ([vp, vp, vp, i32, i64, i64, i64, i64, i32, i64, i32, vp],
                                        i32),
                "hrrm_median2d_video": ([vp, vp, vp, vp, i32, i64, i64, i64, i64, i64, i32, vp],
                                        i32),
                "hrrm_median2d_batched": ([vp, ctypes.POINTER(_Image), i32, vp], i32),
                "hrrm_batch_capacity": ([], i32),
                "hrrm_autotune": ([vp, vp, i32, i32, i32, i64, i64, i64, cp, ctypes.POINTER(i32)],
                                  i32),
                "hrrm_load_tuning": ([vp, cp], i32),
                "hrrm_save_tuning": ([vp, cp], i32),
                "hrrm_set_tile_config": ([vp, i32, i32, i32, i32, ctypes.POINTER(TileConfig)], i32),
                "hrrm_get_tile_config": ([vp, i32, i32, i32, i32, i64, i64, i64,
                                          ctypes.POINTER(TileConfig)], i32),
                "hrrm_server_create": ([vp, ctypes.c_size_t, i32, i32, ctypes.c_uint32,
                                        ctypes.POINTER(vp)], i32),
                "hrrm_server_submit": ([vp, ctypes.POINTER(_Request), ctypes.POINTER(ctypes.c_uint64)],
                                       i32),
                "hrrm_server_poll": ([vp, ctypes.c_uint64, ctypes.POINTER(_Result)], i32),
                "hrrm_server_release": ([vp, ctypes.c_uint64], i32),
                "hrrm_server_drain": ([vp, ctypes.POINTER(ctypes.c_uint64), ctypes.POINTER(_Result),
                                       i32], i32),
                "hrrm_server_cancel": ([vp, ctypes.c_uint64], i32),
                "hrrm_server_now": ([vp], ctypes.c_double),
                "hrrm_server_destroy": ([vp], i32),
            }
            for name, (args, res) in sig.items():
                f = getattr(L, name)
                f.argtypes = args
                f.restype = res
            _lib = L
    return _lib


def last_error() -> str:
    return lib().hrrm_last_error().decode()


def check(rc: int) -> int:
    if rc < 0:
        raise HrrmError(rc, last_error())
    return rc


def _torch():
    import torch
    return torch


def _dtype_code(t) -> int:
    torch = _torch()
    if t.dtype == torch.uint8:
        return U8
    if t.dtype == torch.uint16:
        return U16
    raise TypeError("hrrm filters uint8 or uint16 images, got %s" % t.dtype)


def _variant_code(v) -> int:
    if v in (PLAIN, "plain", "uniform"):
        return PLAIN
    if v in (ADAPTIVE, "adaptive"):
        return ADAPTIVE
    if v in (FULL_UPDATE, "full", "full_update"):
        return FULL_UPDATE
    raise ValueError("variant must be 'plain', 'adaptive' or 'full'")


def _stream_ptr(t, stream) -> int:
    torch = _torch()
    s = stream if stream is not None else torch.cuda.current_stream(t.device)
    return int(s.cuda_stream)


class Context:
    """One library context per device (owns adaptive workspaces and the tile table)."""

    def __init__(self, device: int = 0):
        self._h = ctypes.c_void_p()
        check(lib().hrrm_ctx_create(device, ctypes.byref(self._h)))
        self.device = device

    @property
    def handle(self):
        return self._h

    def close(self):
        if self._h:
            lib().hrrm_ctx_destroy(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def reserve(self, dtype: int, max_pixels: int, max_r: int, variant="plain"):
        check(lib().hrrm_ctx_reserve(self._h, dtype, max_pixels, max_r, _variant_code(variant)))

    def _out(self, src, out):
        torch = _torch()
        if out is None:
            out = torch.empty_like(src, memory_format=torch.contiguous_format)
        if out.dtype != src.dtype or out.shape != src.shape or out.device != src.device:
            raise ValueError("out must match src in dtype, shape and device")
        return out

    def median2d(self, src, r: int, variant="plain", out=None, stream=None):
        return self.rank2d(src, r, None, 0, variant, out, stream)

    def rank2d(self, src, r: int, rank: Optional[int] = None, drop_levels: int = 0,
               variant="plain", out=None, stream=None):
        if src.dim() != 2:
            raise ValueError("median2d takes a (H, W) tensor")
        if src.stride(1) != 1:
            raise ValueError("rows must be contiguous (stride 1 along x)")
        out = self._out(src, out)
        if out.stride(1) != 1:
            raise ValueError("out rows must be contiguous")
        h, w = src.shape
        n = (2 * r + 1) ** 2
        k = (n - 1) // 2 if rank is None else int(rank)
        check(lib().hrrm_rank2d(self._h, src.data_ptr(), out.data_ptr(), _dtype_code(src), w, h,
                                src.stride(0), out.stride(0), r, k, drop_levels,
                                _variant_code(variant), _stream_ptr(src, stream)))
        return out

    def rank2d_noalloc(self, src, r: int, rank: Optional[int] = None, variant="plain", out=None,
                       stream=None):
        """hrrm_rank2d_noalloc: as rank2d (full precision), with no device allocation."""
        if src.dim() != 2 or src.stride(1) != 1:
            raise ValueError("rank2d_noalloc takes a (H, W) tensor with contiguous rows")
        out = self._out(src, out)
        if out.stride(1) != 1:
            raise ValueError("out rows must be contiguous")
        h, w = src.shape
        n = (2 * r + 1) ** 2
        k = (n - 1) // 2 if rank is None else int(rank)
        check(lib().hrrm_rank2d_noalloc(self._h, src.data_ptr(), out.data_ptr(), _dtype_code(src),
                                        w, h, src.stride(0), out.stride(0), r, k,
                                        _variant_code(variant), _stream_ptr(src, stream)))
        return out

    def median2d_video(self, src, r: int, estimate=None, out=None, stream=None):
        """Adaptive-tree median of one frame; `estimate` (same shape and dtype,
        e.g. the previous frame's output) replaces the running-mean histogram
        in the topology; None = running mean.  `out` may be `estimate`."""
        if src.dim() != 2 or src.stride(1) != 1:
            raise ValueError("median2d_video takes a (H, W) tensor with contiguous rows")
        out = self._out(src, out)
        h, w = src.shape
        ep, es = None, 0
        if estimate is not None:
            if estimate.shape != src.shape or estimate.dtype != src.dtype or estimate.stride(1) != 1:
                raise ValueError("estimate must match src in shape and dtype, rows contiguous")
            ep, es = estimate.data_ptr(), estimate.stride(0)
        check(lib().hrrm_median2d_video(self._h, src.data_ptr(), out.data_ptr(), ep,
                                        _dtype_code(src), w, h, src.stride(0), out.stride(0), es,
                                        r, _stream_ptr(src, stream)))
        return out

    def median3d(self, src, r: int, variant="plain", out=None, stream=None):
        if src.dim() != 3:
            raise ValueError("median3d takes a (D, H, W) tensor")
        if src.stride(2) != 1:
            raise ValueError("rows must be contiguous (stride 1 along x)")
        out = self._out(src, out)
        d, h, w = src.shape
        check(lib().hrrm_median3d(self._h, src.data_ptr(), out.data_ptr(), _dtype_code(src), w, h,
                                  d, src.stride(1), src.stride(0), out.stride(1), out.stride(0),
                                  r, _variant_code(variant), _stream_ptr(src, stream)))
        return out

    def median2d_batched(self, srcs: Sequence, radii: Sequence[int], outs=None, stream=None):
        if outs is None:
            outs = [_torch().empty_like(s) for s in srcs]
        arr = (_Image * max(1, len(srcs)))()
        for i, (s, o, r) in enumerate(zip(srcs, outs, radii)):
            arr[i] = _Image(s.data_ptr(), o.data_ptr(), s.shape[1], s.shape[0], s.stride(0),
                            o.stride(0), _dtype_code(s), int(r))
        st = _stream_ptr(srcs[0], stream) if len(srcs) else 0
        check(lib().hrrm_median2d_batched(self._h, arr, len(srcs), st))
        return outs

    def autotune(self, dtype: int, r: int, variant="plain", width: int = 4096, height: int = 4096,
                 sample=None, cache_path: Optional[str] = None) -> int:
        """Tune the tile configuration for (dtype, r, variant); `sample` is an
        optional (H, W) device tensor to tune on.  Returns candidates timed."""
        tried = ctypes.c_int32(-1)
        if sample is not None:
            height, width = sample.shape
            ptr, stride = sample.data_ptr(), sample.stride(0)
        else:
            ptr, stride = None, width
        check(lib().hrrm_autotune(self._h, ptr, dtype, r, _variant_code(variant), width, height,
                                  stride, cache_path.encode() if cache_path else None,
                                  ctypes.byref(tried)))
        return tried.value

    def save_tuning(self, path: str):
        check(lib().hrrm_save_tuning(self._h, path.encode()))

    def set_tile(self, dtype: int, dims: int, r: int, variant="plain", cfg=None, **fields):
        """Set the tile configuration for one key (cfg=None and no fields: reset)."""
        if cfg is None and fields:
            cfg = self.get_tile(dtype, dims, r, variant)
        if cfg is not None:
            for k, v in fields.items():
                setattr(cfg, k, int(v))
        check(lib().hrrm_set_tile_config(self._h, dtype, dims, r, _variant_code(variant),
                                         ctypes.byref(cfg) if cfg is not None else None))

    def get_tile(self, dtype: int, dims: int, r: int, variant="plain", width: int = 4096,
                 height: int = 4096, depth: int = 1) -> TileConfig:
        cfg = TileConfig()
        check(lib().hrrm_get_tile_config(self._h, dtype, dims, r, _variant_code(variant), width,
                                         height, depth, ctypes.byref(cfg)))
        return cfg

    def load_tuning(self, path: str):
        check(lib().hrrm_load_tuning(self._h, path.encode()))


def _hip():
    """The HIP runtime library the process already uses (for raw copies only)."""
    global _hiplib
    if _hiplib is None:
        _hiplib = ctypes.CDLL("libamdhip64.so")
        _hiplib.hipMemcpy.argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_size_t,
                                      ctypes.c_int]
        _hiplib.hipMemcpy.restype = ctypes.c_int
    return _hiplib


_hiplib = None


class Server:
    """Continuous-batching request loop on one device (hrrm_server_*).

    submit() takes a HOST image (numpy array or CPU tensor, ideally pinned) and
    returns a ticket; the image must stay alive until the ticket is done, so the
    wrapper keeps a reference.  poll() returns None until done, then a dict with
    the device output pointer and the server-clock timestamps."""

    PER_IMAGE = 1

    def __init__(self, ctx: "Context", budget_bytes: int, max_inflight: int = 1024,
                 max_queue: int = 1 << 20, per_image: bool = False):
        self._h = ctypes.c_void_p()
        check(lib().hrrm_server_create(ctx.handle, budget_bytes, max_inflight, max_queue,
                                       self.PER_IMAGE if per_image else 0, ctypes.byref(self._h)))
        self._keep = {}
        # per calling thread: (max_n, tickets, results), reused by drain()
        self._drain_tls = threading.local()

    def submit(self, img, r: int) -> int:
        torch = _torch()
        t = img if isinstance(img, torch.Tensor) else torch.from_numpy(img)
        if t.dim() != 2 or t.stride(1) != 1:
            raise ValueError("submit takes a (H, W) image with contiguous rows")
        req = _Request(t.data_ptr(), t.shape[1], t.shape[0], t.stride(0), _dtype_code(t), int(r))
        tk = ctypes.c_uint64()
        check(lib().hrrm_server_submit(self._h, ctypes.byref(req), ctypes.byref(tk)))
        self._keep[tk.value] = t
        return tk.value

    def poll(self, ticket: int):
        res = _Result()
        rc = lib().hrrm_server_poll(self._h, ticket, ctypes.byref(res))
        if rc == EAGAIN:
            return None
        check(rc)
        self._keep.pop(ticket, None)
        return {"d_dst": res.d_dst, "width": res.width, "height": res.height, "dtype": res.dtype,
                "status": res.status, "t_submit": res.t_submit, "t_admit": res.t_admit,
                "t_done": res.t_done}

    def fetch(self, res) -> "object":
        """Copy a done ticket's output to a new host tensor (marshalling only)."""
        torch = _torch()
        dt = torch.uint8 if res["dtype"] == U8 else torch.int16
        out = torch.empty((res["height"], res["width"]), dtype=dt)
        rc = _hip().hipMemcpy(out.data_ptr(), res["d_dst"], out.numel() * out.element_size(), 2)
        if rc != 0:
            raise HrrmError(EDEVICE, "hipMemcpy device to host failed (%d)" % rc)
        return out if res["dtype"] == U8 else out.view(torch.uint16)

    def drain(self, max_n: int = 4096):
        """Done tickets not reported before: list of (ticket, result dict)."""
        bufs = getattr(self._drain_tls, "bufs", None)
        if bufs is None or bufs[0] != max_n:
            bufs = (max_n, (ctypes.c_uint64 * max_n)(), (_Result * max_n)())
            self._drain_tls.bufs = bufs
        _, tk, rs = bufs
        n = check(lib().hrrm_server_drain(self._h, tk, rs, max_n))
        out = []
        for i in range(n):
            r = rs[i]
            self._keep.pop(tk[i], None)
            out.append((tk[i], {"d_dst": r.d_dst, "width": r.width, "height": r.height,
                                "dtype": r.dtype, "status": r.status, "t_submit": r.t_submit,
                                "t_admit": r.t_admit, "t_done": r.t_done}))
        return out

    def release(self, ticket: int):
        check(lib().hrrm_server_release(self._h, ticket))

    def cancel(self, ticket: int) -> bool:
        rc = lib().hrrm_server_cancel(self._h, ticket)
        if rc == EAGAIN:
            return False
        check(rc)
        self._keep.pop(ticket, None)
        return True

    def now(self) -> float:
        return lib().hrrm_server_now(self._h)

    def close(self):
        if self._h:
            lib().hrrm_server_destroy(self._h)
            self._h = ctypes.c_void_p()
            self._keep.clear()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


_contexts = {}


def context(device: Optional[int] = None) -> Context:
    if device is None:
        device = _torch().cuda.current_device()
    with _lock:
        c = _contexts.get(device)
    if c is None:
        c = Context(device)
        with _lock:
            _contexts[device] = c
    return c


def _dev(t) -> int:
    return t.device.index if t.device.index is not None else _torch().cuda.current_device()


def median2d(src, r: int, variant="plain", out=None, stream=None):
    return context(_dev(src)).median2d(src, r, variant, out, stream)


def rank2d(src, r: int, rank: int, drop_levels: int = 0, variant="plain", out=None, stream=None):
    return context(_dev(src)).rank2d(src, r, rank, drop_levels, variant, out, stream)


def median3d(src, r: int, variant="plain", out=None, stream=None):
    return context(_dev(src)).median3d(src, r, variant, out, stream)


def median2d_video(src, r: int, estimate=None, out=None, stream=None):
    return context(_dev(src)).median2d_video(src, r, estimate, out, stream)


def median2d_batched(srcs, radii, outs=None, stream=None):
    return context(_dev(srcs[0])).median2d_batched(srcs, radii, outs, stream)


EXPORTED_SYMBOLS: List[str] = [
    "hrrm_last_error", "hrrm_version", "hrrm_ctx_create", "hrrm_ctx_destroy", "hrrm_ctx_reserve",
    "hrrm_median2d", "hrrm_median3d", "hrrm_rank2d", "hrrm_rank2d_noalloc", "hrrm_median2d_video",
    "hrrm_median2d_batched",
    "hrrm_batch_capacity", "hrrm_autotune", "hrrm_load_tuning", "hrrm_save_tuning",
    "hrrm_set_tile_config",
    "hrrm_get_tile_config", "hrrm_server_create",
    "hrrm_server_submit", "hrrm_server_poll", "hrrm_server_drain", "hrrm_server_release",
    "hrrm_server_cancel",
    "hrrm_server_now", "hrrm_server_destroy",
]
