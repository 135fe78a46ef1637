#!/usr/bin/env python
"""Benchmark of the running-median hot path on one MI355X.

Default workload: 16-bit 4096 x 4096 X-ray-like image (12-bit Gaussian mixture
plus a smooth ramp), radius 15 (31 x 31 window), clamp-to-edge, plain
(uniform-tree) variant.  One step = one full filter pass over one image that is
already resident in HBM; the timed region rotates over input/output copies
larger than the 256 MB last-level cache so every step reads from HBM.

Prints ONE JSON line.  Besides the throughput it carries
  * roofline: the LDS bound of the kernel (algorithmic LDS work per pixel from
    the input histogram) against the LDS peak, the kernel time
    taken from HIP events on the launch stream, with the HBM view alongside;
  * cpu_baseline: the brute-force CPU oracle timed on a band of full rows of
    the same image on this host's cores.

    python bench.py [--gpus 1] [--steps 20] [--warmup 3] [--workload c0/c1/c2/c3] [--r 15]

(c0, c1, c2: 2-D images; c3: the 16-bit 512 x 512 x 256 volume, 3-D windows.)
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "output Mpix/s (u16 4096², r=15) + % HBM/LDS roofline; serving p50/p99 ms"
HBM_PEAK_GBS = 8000.0
# LDS: 256 CUs x 32 banks x 4 B per clock x 2.4 GHz
LDS_PEAK_GBS = 256 * 32 * 4 * 2.4


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


def cpu_baseline(img, r: int, seconds_target: float = 10.0):
    import numpy as np
    import oracle
    threads = int(os.environ.get("OMP_NUM_THREADS", "0") or 0) or min(16, os.cpu_count() or 1)
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
                "kind": "oracle",
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
            "kind": "oracle",
            "sample": "rows 0..%d of the same image (%d x %d pixels, clamp at the image's own "
                      "top border), brute-force nth_element per window, %.1f s" % (rows - 1, w, rows,
                                                                                  dt)}


def serving(seconds: float, warmup_s: float = 0.5, rate: float = 2000.0, per_image: bool = False,
            pools=None):
    """Replay the seeded Poisson request trace against the continuous-batching
    server; latency = completion - scheduled arrival (upload included, output
    left on the device), throughput = output Mpix completed per second inside
    the measurement window (arrivals after the warm-up)."""
    import numpy as np
    import paper_1105_3829_amd as hrrm
    from paper_1105_3829_amd import datagen
    trace = datagen.serving_trace(duration_s=warmup_s + seconds, rate_hz=rate, seed=4)
    ctx = hrrm.context(0)
    srv = hrrm.Server(ctx, 48 << 30, max_inflight=1 << 14, max_queue=1 << 20, per_image=per_image)
    t0 = srv.now() + 0.05
    lat, done_pairs = [], []
    submitted = {}
    i = 0
    n = len(trace)
    ndone = 0
    last_note = time.time()
    while ndone < n:
        now = srv.now()
        if time.time() - last_note > 5.0:
            print("serving %s: t=%.1fs submitted %d/%d done %d" % (
                "per-image" if per_image else "batched", now - t0, i, n, ndone),
                file=sys.stderr, flush=True)
            last_note = time.time()
        while i < n and t0 + trace[i].arrival_s <= now:
            q = trace[i]
            pool = pools[q.dtype][q.pool_index % len(pools[q.dtype])]
            # packed run of pinned pool pixels (one linear upload per request)
            img = pool.view(-1)[q.offset_flat:q.offset_flat + q.width * q.height].view(
                q.height, q.width)
            submitted[srv.submit(img, q.radius)] = i
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
        "requests": len(measured),
        "p50_ms": round(float(np.percentile(lat, 50)), 3),
        "p99_ms": round(float(np.percentile(lat, 99)), 3),
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
    ap.add_argument("--copy-calibration", action="store_true",
                    help="also run a plain device copy of one image (counter calibration)")
    ap.add_argument("--serving-seconds", type=float, default=5.0,
                    help="length of the replayed serving trace (0 = skip serving)")
    ap.add_argument("--saturation-rate", type=float, default=4000.0,
                    help="request rate of the overload trace (0 = skip it)")
    ap.add_argument("--saturation-seconds", type=float, default=2.5)
    args = ap.parse_args()

    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print("bench.py measures one GPU: the library has no multi-GPU path (the filter "
              "would shard into row bands with r halo rows, one per GPU)", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    import paper_1105_3829_amd as hrrm

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

    def step(i):
        if vol:
            ctx.median3d(srcs[i % copies], args.r, variant=args.variant, out=outs[i % copies],
                         stream=stream)
        else:
            ctx.median2d(srcs[i % copies], args.r, variant=args.variant, out=outs[i % copies],
                         stream=stream)

    for i in range(args.warmup):
        step(i)
    torch.cuda.synchronize()
    if args.copy_calibration:
        tmp = torch.empty_like(base)
        tmp.copy_(srcs[0])
        torch.cuda.synchronize()

    evs = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
           for _ in range(args.steps)]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i in range(args.steps):
        evs[i][0].record(stream)
        step(i)
        evs[i][1].record(stream)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    ms_per_step = (t1 - t0) * 1e3 / args.steps
    kernel_ms = float(np.mean([a.elapsed_time(b) for a, b in evs]))
    pixels = h * w * depth
    value = pixels / (ms_per_step * 1e-3) / 1e6

    a_ops, zbar, d = lds_work_per_pixel(img, args.variant, args.r)
    lds_bytes_launch = a_ops * 4.0 * pixels
    hbm_bytes_launch = 2.0 * img.dtype.itemsize * pixels
    lds_gbs = lds_bytes_launch / (kernel_ms * 1e-3) / 1e9
    hbm_gbs = hbm_bytes_launch / (kernel_ms * 1e-3) / 1e9
    traffic = None
    tfile = os.path.join(ROOT, "profiles", "hbm_traffic_%s_r%d_%s.json" % (args.workload, args.r,
                                                                           args.variant))
    if os.path.exists(tfile):
        try:
            traffic = json.load(open(tfile)).get("bytes_per_launch")
        except Exception:
            traffic = None

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
        "roofline": {"bound": "lds", "achieved": round(lds_gbs, 2), "peak": LDS_PEAK_GBS,
                     "unit": "GB/s", "frac": round(lds_gbs / LDS_PEAK_GBS, 5),
                     "traffic": traffic, "kernel_ms": round(kernel_ms, 4),
                     "lds_dword_ops_per_pixel": round(a_ops, 3), "zbar": round(zbar, 4),
                     "hbm": {"achieved": round(hbm_gbs, 2), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                             "frac": round(hbm_gbs / HBM_PEAK_GBS, 6),
                             "bytes_per_launch": hbm_bytes_launch}},
    }
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
        if args.saturation_rate > 0:
            # the same trace recipe at a rate neither mode can sustain: the
            # completed throughput inside the window is each mode's capacity
            sb = serving(args.saturation_seconds, rate=args.saturation_rate, per_image=False,
                         pools=pools)
            sp = serving(args.saturation_seconds, rate=args.saturation_rate, per_image=True,
                         pools=pools)
            res["serving"]["saturated"] = {
                "rate_hz": args.saturation_rate, "seconds": args.saturation_seconds,
                "batched": sb, "per_image": sp,
                "throughput_gain": round(sb["completed_mpix_s_in_window"] /
                                         max(sp["completed_mpix_s_in_window"], 1e-9), 3)}
    if not args.no_cpu_baseline:
        print("cpu baseline: timing the oracle", file=sys.stderr, flush=True)
        res["cpu_baseline"] = cpu_baseline(img, args.r)
    print(json.dumps(res), flush=True)


if __name__ == "__main__":
    main()
