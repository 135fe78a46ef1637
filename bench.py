#!/usr/bin/env python
"""Benchmark of the running-median hot path on one MI355X.

Default workload: 16-bit 4096 x 4096 X-ray-like image (12-bit Gaussian mixture
plus a smooth ramp), radius 15 (31 x 31 window), clamp-to-edge, plain
(uniform-tree) variant, default tile configuration.  One step = one full
filter pass over one image that is already resident in HBM; the timed region
rotates over input/output copies larger than the 256 MB last-level cache so
every step reads from HBM.

Prints ONE JSON line.  Besides the throughput it carries
  * roofline: the LDS bound of the filter (algorithmic LDS work per pixel from
    the input histogram) against the LDS read bandwidth measured in this run
    by a peak kernel (the nominal 256 CUs x 128 B x 2.4 GHz beside it), the
    step's kernel time taken from HIP events on the launch stream, and the HBM
    view against the published 8 TB/s, with a streaming copy measured in this
    run beside it;
  * variants: the adaptive tree on the same image;
  * sweeps: radius sweeps of the other workloads (8-bit 8192^2 low-key image,
    r = 1..100; 16-bit 512 x 512 x 256 volume, r = 1..7; the 16-bit image at
    r = 5 and 50), one pass each after a warm-up;
  * serving: the Poisson request trace at 2000 req/s, and a ladder of
    offered rates giving each mode's highest rate served within the latency
    bound;
  * cpu_baseline: the brute-force CPU oracle timed on a band of full rows of
    the same image on this host's cores.

    python bench.py [--gpus 1] [--steps 20] [--warmup 3] [--workload c0/c1/c2/c3] [--r 15]

(c0, c1, c2: 2-D images; c3: the 16-bit 512 x 512 x 256 volume, 3-D windows.)
"""
from __future__ import annotations

import argparse
import ctypes
import gc
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "output Mpix/s (u16 4096², r=15) + % HBM/LDS roofline; serving p50/p99 ms"
HBM_PEAK_GBS = 8000.0  # MI355X published HBM3E bandwidth
# LDS, nominal: 256 CUs x 128 bytes per clock x 2.4 GHz
LDS_NOMINAL_GBS = 256 * 128 * 2.4
SERVING_SLO_MS = 20.0  # p99 latency bound of the serving ladder


def workload(name: str, r: int):
    from paper_1105_3829_amd import datagen
    if name == "c1":
        return datagen.xray_u16(4096, 4096, seed=1), "u16 4096x4096 X-ray-like mixture + ramp"
    if name == "c0":
        return datagen.uniform_u8(512, 512, seed=0), "u8 512x512 uniform"
    if name == "c2":
        return datagen.lowkey_u8(8192, 8192, seed=2), "u8 8192x8192 low-key"
    if name == "c3":
        return (datagen.xray_volume_u16(256, 512, 512, seed=3),
                "u16 512x512x256 X-ray-like volume with 1% impulses")
    raise SystemExit("unknown workload %s" % name)


def lds_work_per_pixel(img, variant: str = "plain", r: int = 0) -> tuple:
    """Algorithmic LDS dword-operations per output pixel of the uniform method:
    2*zbar counter updates (one removal, one insertion per column per row; an
    update touches the levels where the value's bit is 0; a volume's column
    takes 2r + 1 of each per row step) plus two column-counter reads (entering
    and leaving column) per window-tree node brought up to date: the d nodes
    the descent visits for the on-demand update, all 2^d - 1 nodes for the
    full update.  zbar is exact for this input (from its histogram)."""
    import numpy as np
    d = 8 * img.dtype.itemsize
    hist = np.bincount(img.ravel(), minlength=1 << d).astype(np.float64)
    ones = np.array([bin(v).count("1") for v in range(1 << d)], dtype=np.float64)
    zbar = d - float((hist * ones).sum() / hist.sum())
    nodes = (1 << d) - 1 if variant == "full" else d
    per_step = 2 * r + 1 if img.ndim == 3 else 1
    return 2.0 * zbar * per_step + 2.0 * nodes, zbar, d


def cpu_model() -> str:
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def host_threads() -> int:
    try:
        return len(os.sched_getaffinity(0))
    except AttributeError:
        return os.cpu_count() or 1


def cpu_baseline(img, r: int, seconds_target: float = 10.0):
    import numpy as np
    import oracle
    threads = host_threads()
    model = cpu_model()
    if img.ndim == 3:
        # a slab of whole slices, clamped at the slab's own bottom slice
        d, h, w = img.shape
        probe = np.ascontiguousarray(img[:1])
        t = time.perf_counter()
        oracle.median3d(probe, r, threads=threads)
        rate = probe.size / max(time.perf_counter() - t, 1e-6)
        n = int(max(1, min(d, seconds_target * rate / (h * w))))
        slab = np.ascontiguousarray(img[:n])
        t = time.perf_counter()
        oracle.median3d(slab, r, threads=threads)
        dt = time.perf_counter() - t
        return {"value": round(slab.size / dt / 1e6, 4), "unit": "Mvox/s", "cores": threads,
                "kind": "oracle", "cpu": model,
                "sample": "slices 0..%d of the same volume (%d x %d x %d voxels, clamp at the "
                          "slab's own last slice), brute-force nth_element per window, %.1f s" % (
                              n - 1, w, h, n, dt)}
    h, w = img.shape
    # calibrate on a thin band, then time a band sized for ~seconds_target
    probe = np.ascontiguousarray(img[: min(h, 16 + 2 * r)])
    t = time.perf_counter()
    oracle.median2d(probe, r, threads=threads)
    rate = probe.size / max(time.perf_counter() - t, 1e-6)
    rows = int(max(32, min(h, seconds_target * rate / w)))
    band = np.ascontiguousarray(img[:rows])
    t = time.perf_counter()
    oracle.median2d(band, r, threads=threads)
    dt = time.perf_counter() - t
    return {"value": round(band.size / dt / 1e6, 4), "unit": "Mpix/s", "cores": threads,
            "kind": "oracle", "cpu": model,
            "sample": "rows 0..%d of the same image (%d x %d pixels, clamp at the image's own "
                      "top border), brute-force nth_element per window, %.1f s" % (rows - 1, w, rows,
                                                                                  dt)}


def measure_peaks():
    """LDS read and HBM streaming-copy bandwidth measured now, on this GPU."""
    from paper_1105_3829_amd import build as b
    if not os.path.exists(b.MEASURE_LIB):
        return None
    L = ctypes.CDLL(b.MEASURE_LIB)
    L.hrrm_measure_lds_read.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.POINTER(ctypes.c_double)]
    L.hrrm_measure_hbm_copy.argtypes = [ctypes.c_int, ctypes.c_int64, ctypes.c_int,
                                        ctypes.POINTER(ctypes.c_double)]
    lds = ctypes.c_double(0)
    hbm = ctypes.c_double(0)
    nbytes = 1 << 30  # 1 GiB each way: far above the 256 MB last-level cache
    if L.hrrm_measure_lds_read(0, 5, ctypes.byref(lds)) != 0:
        return None
    if L.hrrm_measure_hbm_copy(0, nbytes, 5, ctypes.byref(hbm)) != 0:
        return None
    return {"lds_read_gbs": round(lds.value / 1e9, 1), "hbm_copy_gbs": round(hbm.value / 1e9, 1),
            "hbm_copy_bytes": nbytes,
            "how": "best of 5: conflict-free ds_read_b128 from two 64 KB workgroups per CU; "
                   "a streaming uint4 copy of 1 GiB between two buffers (read + write bytes)"}


def serving(seconds: float, warmup_s: float = 0.5, rate: float = 2000.0, per_image: bool = False,
            pools=None, sides=(256, 4096)):
    """Replay the seeded Poisson request trace against the continuous-batching
    server; latency = completion - scheduled arrival (upload included, output
    left on the device), throughput = output Mpix completed per second inside
    the measurement window (arrivals after the warm-up)."""
    import numpy as np
    import paper_1105_3829_amd as hrrm
    from paper_1105_3829_amd import datagen
    trace = datagen.serving_trace(duration_s=warmup_s + seconds, rate_hz=rate, seed=4,
                                  min_side=sides[0], max_side=sides[1])
    ctx = hrrm.context(0)
    srv = hrrm.Server(ctx, 48 << 30, max_inflight=1 << 14, max_queue=1 << 20, per_image=per_image)
    # each request's packed run of pinned pool pixels (one linear upload per
    # request), cut before the clock starts
    imgs = []
    for q in trace:
        pool = pools[q.dtype][q.pool_index % len(pools[q.dtype])]
        imgs.append(pool.view(-1)[q.offset_flat:q.offset_flat + q.width * q.height].view(
            q.height, q.width))
    t0 = srv.now() + 0.05
    lat, done_pairs, late = [], [], []
    submitted = {}
    i = 0
    n = len(trace)
    ndone = 0
    last_note = time.time()
    # the client loop allocates many small objects: a cyclic-garbage pass
    # inside the window would stall submissions for tens of milliseconds
    gc.collect()
    gc.disable()
    try:
        while ndone < n:
            now = srv.now()
            if time.time() - last_note > 5.0:
                print("serving %s %.0f/s: t=%.1fs submitted %d/%d done %d" % (
                    "per-image" if per_image else "batched", rate, now - t0, i, n, ndone),
                    file=sys.stderr, flush=True)
                last_note = time.time()
            while i < n and t0 + trace[i].arrival_s <= now:
                q = trace[i]
                submitted[srv.submit(imgs[i], q.radius)] = i
                if q.arrival_s >= warmup_s:
                    late.append(srv.now() - (t0 + q.arrival_s))
                i += 1
            for tk, res in srv.drain():
                q = trace[submitted.pop(tk)]
                srv.release(tk)
                ndone += 1
                if res["status"] != 0:
                    raise RuntimeError("request failed with %d" % res["status"])
                if q.arrival_s >= warmup_s:
                    lat.append(res["t_done"] - (t0 + q.arrival_s))
                    done_pairs.append((res["t_done"] - t0, q.width * q.height))
            if i < n:
                wait = t0 + trace[i].arrival_s - srv.now()
                if wait > 0:
                    time.sleep(min(wait, 0.0005))
            else:
                time.sleep(0.0005)
    finally:
        gc.enable()
    srv.close()
    lat = np.array(lat) * 1e3
    window = warmup_s + seconds
    measured = [q for q in trace if q.arrival_s >= warmup_s]
    offered = sum(q.width * q.height for q in measured) / seconds / 1e6
    done_win = sum(p for t, p in done_pairs if t <= window)
    last = max(t for t, _ in done_pairs)
    pix_all = sum(p for _, p in done_pairs)
    return {
        "mode": "per_image" if per_image else "batched",
        "rate_hz": rate,
        "requests": len(measured),
        "p50_ms": round(float(np.percentile(lat, 50)), 3),
        "p99_ms": round(float(np.percentile(lat, 99)), 3),
        # how late the client loop submitted (part of every latency above)
        "submit_late_p99_ms": round(float(np.percentile(late, 99)) * 1e3, 3),
        "completed_mpix_s_in_window": round(done_win / seconds / 1e6, 1),
        "drain_mpix_s": round(pix_all / max(last - warmup_s, 1e-9) / 1e6, 1),
        "offered_mpix_s": round(offered, 1),
        # stable: the server keeps up with the offered load inside the window
        "queue_stable": bool(done_win / seconds >= 0.97 * offered * 1e6),
    }


def serving_pools():
    import torch
    from paper_1105_3829_amd import datagen
    u16 = [torch.from_numpy(p).pin_memory() for p in datagen.serving_pool(4, dtype="u16")]
    u8 = [torch.from_numpy(p).pin_memory() for p in datagen.serving_pool(4, dtype="u8")]
    return {"u16": u16, "u8": u8}


def serving_ladder(pools, rates, seconds, sides=(256, 4096)):
    """Each mode at increasing offered rates: the highest rate whose queue is
    stable with p99 latency within SERVING_SLO_MS is the mode's capacity."""
    out = {"slo_p99_ms": SERVING_SLO_MS, "seconds_per_rate": seconds, "rates": list(rates),
           "sides": list(sides)}
    for per_image in (False, True):
        mode = "per_image" if per_image else "batched"
        runs = []
        best = None
        for rate in rates:
            r = serving(seconds, rate=rate, per_image=per_image, pools=pools, sides=sides)
            runs.append(r)
            if r["queue_stable"] and r["p99_ms"] <= SERVING_SLO_MS:
                best = r
            elif best is not None:
                break  # past capacity
        out[mode] = {"runs": runs,
                     "max_rate_hz_within_slo": best["rate_hz"] if best else None,
                     "mpix_s_within_slo": best["completed_mpix_s_in_window"] if best else None}
    b, p = out["batched"]["mpix_s_within_slo"], out["per_image"]["mpix_s_within_slo"]
    out["throughput_gain_at_slo"] = round(b / p, 3) if b and p else None
    return out


def timed_steps(ctx, srcs, outs, r, variant, steps, warmup, stream, vol):
    """ms per step (wall clock) and the mean step time from HIP events on the
    launch stream, rotating over the given input/output copies."""
    import numpy as np
    import torch
    copies = len(srcs)

    def step(i):
        if vol:
            ctx.median3d(srcs[i % copies], r, variant=variant, out=outs[i % copies], stream=stream)
        else:
            ctx.median2d(srcs[i % copies], r, variant=variant, out=outs[i % copies], stream=stream)

    for i in range(warmup):
        step(i)
    torch.cuda.synchronize()
    evs = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
           for _ in range(steps)]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i in range(steps):
        evs[i][0].record(stream)
        step(i)
        evs[i][1].record(stream)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    return (t1 - t0) * 1e3 / steps, float(np.mean([a.elapsed_time(b) for a, b in evs]))


def roofline(img, variant, r, kernel_ms, pixels, peaks):
    a_ops, zbar, d = lds_work_per_pixel(img, variant, r)
    lds_bytes = a_ops * 4.0 * pixels
    hbm_bytes = 2.0 * img.dtype.itemsize * pixels
    lds_gbs = lds_bytes / (kernel_ms * 1e-3) / 1e9
    hbm_gbs = hbm_bytes / (kernel_ms * 1e-3) / 1e9
    lds_peak = peaks["lds_read_gbs"] if peaks else LDS_NOMINAL_GBS
    return {"bound": "lds", "achieved": round(lds_gbs, 2), "peak": lds_peak, "unit": "GB/s",
            "frac": round(lds_gbs / lds_peak, 5),
            "peak_source": "measured in this run (LDS read kernel)" if peaks else "nominal",
            "peak_nominal": LDS_NOMINAL_GBS, "frac_nominal": round(lds_gbs / LDS_NOMINAL_GBS, 5),
            "kernel_ms": round(kernel_ms, 4), "lds_dword_ops_per_pixel": round(a_ops, 3),
            "zbar": round(zbar, 4),
            "hbm": {"achieved": round(hbm_gbs, 2), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                    "frac": round(hbm_gbs / HBM_PEAK_GBS, 6), "bytes_per_launch": hbm_bytes,
                    "copy_measured_gbs": peaks["hbm_copy_gbs"] if peaks else None}}


def stored_traffic(workload, r, variant):
    """HBM traffic per launch from rocprofv3 counters (FETCH_SIZE, WRITE_SIZE,
    scaled by the same counters of a plain copy), taken for the kernel source
    as it was; null once that source has changed."""
    tfile = os.path.join(ROOT, "profiles", "hbm_traffic_%s_r%d_%s.json" % (workload, r, variant))
    if not os.path.exists(tfile):
        return None, None
    try:
        t = json.load(open(tfile))
    except Exception:
        return None, None
    name = t.get("kernel_source")
    src = os.path.join(ROOT, "paper_1105_3829_amd", "csrc", name) if name else ""
    if not name or not os.path.isfile(src):
        return None, "no counters for the current kernel"
    digest = hashlib.sha256(open(src, "rb").read()).hexdigest()
    if digest != t.get("kernel_source_sha256"):
        return None, "stale: %s changed since the counters were taken" % t.get("kernel_source")
    return t.get("bytes_per_launch"), t.get("source")


def sweeps(ctx, stream, steps=5, warmup=2):
    """Radius sweeps: one image on the device, `steps` timed passes per radius."""
    import numpy as np
    import torch
    from paper_1105_3829_amd import datagen
    out = {}

    def dev(a):
        t = torch.from_numpy(a)
        if t.dtype == torch.uint16:
            return t.view(torch.int16).to("cuda:0").view(torch.uint16)
        return t.to("cuda:0")

    def run(key, img, radii, variants, vol=False):
        d = dev(img)
        o = torch.empty_like(d)
        res = {}
        for variant in variants:
            row = {}
            for r in radii:
                _, k_ms = timed_steps(ctx, [d], [o], r, variant, steps, warmup, stream, vol)
                row[str(r)] = {"kernel_ms": round(k_ms, 4), "mpix_s": round(img.size / k_ms / 1e3, 1)}
            rates = [v["mpix_s"] for v in row.values()]
            row["min_over_max"] = round(min(rates) / max(rates), 3)
            res[variant] = row
        out[key] = res
        del d, o
        torch.cuda.synchronize()

    print("sweeps: 8-bit 8192^2 low-key", file=sys.stderr, flush=True)
    run("c2_u8_8192x8192_lowkey", datagen.lowkey_u8(8192, 8192, seed=2),
        (1, 2, 4, 8, 16, 32, 64, 100), ("plain", "adaptive"))
    print("sweeps: 16-bit 512x512x256 volume", file=sys.stderr, flush=True)
    run("c3_u16_512x512x256_volume", datagen.xray_volume_u16(256, 512, 512, seed=3),
        (1, 2, 3, 5, 7), ("plain", "adaptive"), vol=True)
    print("sweeps: 16-bit 4096^2 x-ray", file=sys.stderr, flush=True)
    run("c1_u16_4096x4096_xray", datagen.xray_u16(4096, 4096, seed=1), (5, 15, 50),
        ("plain", "adaptive"))
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="c1")
    ap.add_argument("--r", type=int, default=15)
    ap.add_argument("--variant", default="plain")
    ap.add_argument("--copies", type=int, default=0, help="input/output copies rotated over")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-sweeps", action="store_true")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="also run a plain device copy of one image (counter calibration)")
    ap.add_argument("--serving-seconds", type=float, default=5.0,
                    help="length of the replayed serving trace (0 = skip serving)")
    ap.add_argument("--ladder-rates", default="2000,2500,3000,3500,4000,4500,5000",
                    help="offered rates of the serving ladder (empty = skip it)")
    ap.add_argument("--ladder-seconds", type=float, default=2.0)
    ap.add_argument("--small-ladder-rates", default="4000,8000,12000,16000,24000,32000,48000",
                    help="offered rates of the small-image serving ladder (empty = skip it)")
    args = ap.parse_args()

    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print("bench.py measures one GPU: the library has no multi-GPU path (the filter "
              "would shard into row bands with r halo rows, one per GPU)", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    import paper_1105_3829_amd as hrrm

    peaks = measure_peaks()
    img, desc = workload(args.workload, args.r)
    vol = img.ndim == 3
    depth = img.shape[0] if vol else 1
    h, w = img.shape[-2:]
    dev = torch.device("cuda:0")
    host = torch.from_numpy(img)
    if host.dtype == torch.uint16:
        base = host.view(torch.int16).to(dev).view(torch.uint16)
    else:
        base = host.to(dev)
    nbytes = img.nbytes
    copies = args.copies or max(2, int(np.ceil(2 * 256 * 2**20 / (2 * nbytes))) + 1)
    srcs = [base.clone() for _ in range(copies)]
    outs = [torch.empty_like(base) for _ in range(copies)]
    ctx = hrrm.context(0)
    stream = torch.cuda.current_stream(dev)
    if args.copy_calibration:
        tmp = torch.empty_like(base)
        tmp.copy_(srcs[0])
        torch.cuda.synchronize()

    ms_per_step, kernel_ms = timed_steps(ctx, srcs, outs, args.r, args.variant, args.steps,
                                         args.warmup, stream, vol)
    pixels = h * w * depth
    value = pixels / (ms_per_step * 1e-3) / 1e6
    roof = roofline(img, args.variant, args.r, kernel_ms, pixels, peaks)
    roof["traffic"], roof["traffic_source"] = stored_traffic(args.workload, args.r, args.variant)
    roof["kernel_ms_covers"] = ("every launch of a step: for the 2-D window kernel, that kernel "
                                "plus the tiered kernel's pass over the tiles it flags")
    other = "adaptive" if args.variant == "plain" else "plain"
    o_ms, o_kms = timed_steps(ctx, srcs, outs, args.r, other, args.steps, args.warmup, stream,
                              vol)

    res = {
        "metric": METRIC,
        "value": round(value, 2),
        "unit": "Mvox/s" if vol else "Mpix/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_per_step, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "u%d" % (8 * img.dtype.itemsize),
        "data": "synthetic",
        "config": {"workload": "%s, r=%d (%s window), clamp-to-edge, %s tree" % (
            desc, args.r, "x".join([str(2 * args.r + 1)] * (3 if vol else 2)), args.variant),
            "width": w, "height": h, **({"depth": depth} if vol else {}), "r": args.r,
            "variant": args.variant, "input_copies": copies},
        "roofline": roof,
        "peaks": peaks,
        "variants": {other: {"value": round(pixels / (o_ms * 1e-3) / 1e6, 2),
                             "ms_per_step": round(o_ms, 4),
                             "roofline": roofline(img, other, args.r, o_kms, pixels, peaks)}},
    }
    del srcs, outs
    torch.cuda.synchronize()
    if not args.no_sweeps and args.workload == "c1":
        res["sweeps"] = sweeps(ctx, stream)
    if args.serving_seconds > 0:
        print("serving: drawing request pools", file=sys.stderr, flush=True)
        pools = serving_pools()
        b = serving(args.serving_seconds, per_image=False, pools=pools)
        p = serving(args.serving_seconds, per_image=True, pools=pools)
        res["serving"] = {
            "workload": "Poisson 2000 req/s (seed 4), W,H ~ U{256..4096}, half u8 uniform / half "
                        "u16 X-ray-like pool pixels (packed pinned host rows), "
                        "r in {1,2,3,7,15,31}; 0.5 s warm-up; upload included",
            "batched": b, "per_image": p,
            "p50_ms": b["p50_ms"], "p99_ms": b["p99_ms"],
            "throughput_gain": round(b["completed_mpix_s_in_window"] /
                                     max(p["completed_mpix_s_in_window"], 1e-9), 3)}
        rates = [float(x) for x in args.ladder_rates.split(",") if x.strip()]
        if rates:
            res["serving"]["ladder"] = serving_ladder(pools, rates, args.ladder_seconds)
        rates = [float(x) for x in args.small_ladder_rates.split(",") if x.strip()]
        if rates:
            # the same mix of types and radii with small images (W, H ~
            # U{64..512}), where one launch per image cannot fill the GPU
            res["serving"]["ladder_small"] = serving_ladder(pools, rates, args.ladder_seconds,
                                                            sides=(64, 512))
    if not args.no_cpu_baseline:
        print("cpu baseline: timing the oracle", file=sys.stderr, flush=True)
        res["cpu_baseline"] = cpu_baseline(img, args.r)
    print(json.dumps(res), flush=True)


if __name__ == "__main__":
    main()
