"""Writes full_output_sha256.json: SHA-256 of the oracle's output for every
full-size workload and radius the GPU tests check whole, next to the SHA-256
of the seeded input it was computed from (so a change of the generators shows
up as a fixture mismatch, not as a filter bug).

Calls only oracle/ (and the seeded generators, which hold no filter
arithmetic).  The 8-bit 8192 x 8192 sweep uses the oracle's threshold-
decomposition route (its cost does not grow with r); everything else uses the
oracle's per-window selection.  Run from the repository root:

    python tests/golden/make_full_output_hashes.py [--threads N]
"""
import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import numpy as np  # noqa: E402

import oracle  # noqa: E402
from paper_1105_3829_amd import datagen  # noqa: E402

OUT = os.path.join(os.path.dirname(os.path.abspath(__file__)), "full_output_sha256.json")

# (name, generator call, radii, route)
CASES = [
    ("c0_u8_512x512_uniform", lambda: datagen.uniform_u8(512, 512, seed=0), (3,), "select2d"),
    ("c1_u16_4096x4096_xray", lambda: datagen.xray_u16(4096, 4096, seed=1), (1, 5, 15, 50),
     "select2d"),
    ("c2_u8_8192x8192_lowkey", lambda: datagen.lowkey_u8(8192, 8192, seed=2),
     (1, 2, 4, 8, 16, 32, 64, 100), "thresholds"),
    ("c3_u16_512x512x256_xray_impulses", lambda: datagen.xray_volume_u16(256, 512, 512, seed=3),
     (1, 2, 3, 5, 7), "select3d"),
]


def sha(a: np.ndarray) -> str:
    return hashlib.sha256(np.ascontiguousarray(a).tobytes()).hexdigest()


def main() -> None:
    ap = argparse.ArgumentParser()
    ap.add_argument("--threads", type=int, default=0)
    ap.add_argument("--only", default="")
    args = ap.parse_args()
    table = {}
    if os.path.exists(OUT):
        with open(OUT) as f:
            table = json.load(f)
    for name, gen, radii, route in CASES:
        if args.only and args.only not in name:
            continue
        img = gen()
        entry = table.get(name, {})
        entry.update({"shape": list(img.shape), "dtype": str(img.dtype), "input_sha256": sha(img),
                      "route": route})
        outs = entry.setdefault("output_sha256", {})
        for r in radii:
            t0 = time.time()
            if route == "thresholds":
                out = oracle.rank2d_u8_thresholds(img, r, threads=args.threads)
            elif route == "select3d":
                out = oracle.median3d(img, r, threads=args.threads)
            else:
                out = oracle.median2d(img, r, threads=args.threads)
            outs[str(r)] = sha(out)
            print("%s r=%d %.1f s" % (name, r, time.time() - t0), flush=True)
            table[name] = entry
            with open(OUT, "w") as f:
                json.dump(table, f, indent=1, sort_keys=True)
                f.write("\n")


if __name__ == "__main__":
    main()
