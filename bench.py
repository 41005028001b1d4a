"""Benchmark: exact 3D distance + intersects between two 512 x 512-cell TINs.

Workload (one geometry pair): two heightfield TINs of 524,288 triangles each
over a 1000 x 1000 extent, seeded 6-octave value-noise heights of amplitude
50, the second surface lifted to a minimum vertical clearance of 0.01 (the
two-surface "nearly touching" configuration).  The paper measures on mining
data that is not distributed; these synthetic surfaces stand in for it.

A step is one pass of the whole path over the input already resident in HBM:
sd3_distance (validation, Morton sort + tiling, tile-pair bounds and queue,
FP32 triangle-pair pass with error bounds, FP64 rescue, exact fallback, final
reduction) followed by sd3_intersects (same stages, any-hit).

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--no-cpu-baseline]

Prints one JSON line.  value = all-pairs-equivalent triangle-pair tests per
second (Na * Nb pairs settled per step / step time); geometry-pairs/s, the
triangle-pair tests actually executed, and the plain-FP64 comparison are
reported beside it.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "tri-pair tests/s + geometry-pairs/s, FP32+learned vs plain FP64, exact match"

# Algorithmic work per unit (counted from the kernel source, FMA = 2 flops,
# reciprocal / reciprocal square root = 1, min/max/select = 0):
FLOPS_FP32_PAIR = 711   # full FP32 triangle-pair test: 9 edge/edge, 6 vertex/face,
                        # separating-axis bound
FLOPS_BOX = 12          # triangle bounding-box lower bound per boxed pair
FLOPS_TRI_PREP = 64     # per staged triangle (edges, reciprocals, dual basis, box)
PEAK_FP32_TFLOPS = 157.3
HBM_PEAK_GBS = 8000.0


def parse():
    p = argparse.ArgumentParser()
    p.add_argument("--gpus", type=int, default=1)
    p.add_argument("--steps", type=int, default=20)
    p.add_argument("--warmup", type=int, default=3)
    p.add_argument("--no-cpu-baseline", action="store_true")
    p.add_argument("--no-fp64", action="store_true", help="skip the plain FP64 comparison")
    return p.parse_args()


def cpu_baseline(A, B):
    """The FP64 oracle (exact pruned mode) on the same workload, all host cores."""
    import oracle
    threads = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
    t0 = time.perf_counter()
    d, h, tests = oracle.mesh(A, B, mode="pruned", threads=threads)
    dt = time.perf_counter() - t0
    pairs = len(A[1]) * len(B[1])
    return {"value": pairs / dt, "unit": "tri-pairs/s (all-pairs-equivalent)", "cores": threads,
            "kind": "oracle",
            "sample": f"full workload once, exact pruned mode ({tests} pair tests, {dt:.2f} s)",
            "distance": d, "intersects": h}


def main():
    args = parse()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (got --gpus {args.gpus}); multi-GPU is not part "
              "of this build", file=sys.stderr)
        sys.exit(2)
    import numpy as np
    import torch

    from paper_1808_09571_amd import sd3, synth

    A, B = synth.config_tin_pair()
    na, nb = len(A[1]), len(B[1])
    dev = "cuda:0"
    ba = sd3.Batch.from_packed(synth.pack([A]), dev)
    bb = sd3.Batch.from_packed(synth.pack([B]), dev)
    ctx = sd3.Context(0)

    def step(prec, timing=False):
        d, h, sd = ctx.distance(ba, bb, precision=prec, stats=True, timing=timing)
        hi, si = ctx.intersects(ba, bb, precision=prec, stats=True, timing=timing)
        return d, h, hi, sd, si

    def timed(prec):
        for _ in range(args.warmup):
            step(prec)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(args.steps):
            out = step(prec)
        torch.cuda.synchronize()
        return (time.perf_counter() - t0) / args.steps, out

    # FP32 + FP64 rescue (the method), then the plain FP64 path on the same input
    t32, (d32, h32, hi32, sd32, si32) = timed("fp32")
    res = {"dist": float(d32.cpu()[0]), "hit": bool(h32.cpu()[0]), "hit_any": bool(hi32.cpu()[0])}
    fp64 = None
    if not args.no_fp64:
        t64, (d64, h64, hi64, sd64, si64) = timed("fp64")
        exact = (d32.cpu().numpy().view(np.int64)[0] == d64.cpu().numpy().view(np.int64)[0]
                 and bool(h32.cpu()[0]) == bool(h64.cpu()[0])
                 and bool(hi32.cpu()[0]) == bool(hi64.cpu()[0]))
        fp64 = {"ms_per_step": t64 * 1e3, "geometry_pairs_per_s": 1.0 / t64,
                "tri_pairs_fp64_per_step": sd64["tri_pairs_fp64"] + si64["tri_pairs_fp64"],
                "exact_match_fp32_vs_fp64": bool(exact), "speedup_fp32_over_fp64": t64 / t32}

    # phase timing (HIP events on the call's stream) for the roofline of the
    # dominant kernel; separate steps so the throughput above carries no events
    n_t = max(3, min(args.steps, 10))
    acc = {}
    for _ in range(n_t):
        _, _, _, sd, si = step("fp32", timing=True)
        for tag, s in (("dist", sd), ("isect", si)):
            for k, v in s["ms_phase"].items():
                acc[(tag, k)] = acc.get((tag, k), 0.0) + v / n_t
    ms_pairs = acc[("dist", "pairs")]
    flops = (sd["tri_pairs_fp32"] * FLOPS_FP32_PAIR + sd["tri_pairs_boxed"] * FLOPS_BOX +
             sd["tile_pairs_evaluated"] * 2 * sd3_K() * FLOPS_TRI_PREP)
    achieved = flops / (ms_pairs * 1e-3) / 1e12 if ms_pairs > 0 else 0.0
    roofline = {"kernel": "k_pairs<fp32,distance>", "bound": "alu",
                "achieved": achieved, "peak": PEAK_FP32_TFLOPS, "unit": "TFLOP/s",
                "frac": achieved / PEAK_FP32_TFLOPS, "traffic": None,
                "avg_launch_ms": ms_pairs, "flops_per_launch": flops}

    tri_exec = (sd32["tri_pairs_fp32"] + sd32["tri_pairs_fp64"] + si32["tri_pairs_fp32"] +
                si32["tri_pairs_fp64"])
    line = {
        "metric": METRIC,
        "value": na * nb / t32,
        "unit": "tri-pairs/s (all-pairs-equivalent: Na*Nb settled per second)",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": t32 * 1e3, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f32 (bulk) + f64 (rescue, result)", "data": "synthetic",
        "config": {"workload": "two 512x512-cell TINs, 524288 triangles each, clearance 0.01, "
                               "distance + intersects", "triangles_a": na, "triangles_b": nb,
                   "geometry_pairs": 1, "order": "bound"},
        "geometry_pairs_per_s": 1.0 / t32,
        "tri_pairs_executed_per_step": tri_exec,
        "tri_pairs_executed_per_s": tri_exec / t32,
        "result": res,
        "stats_distance": {k: v for k, v in sd32.items() if k != "ms_phase"},
        "phase_ms": {f"{t}.{k}": round(v, 4) for (t, k), v in acc.items()},
        "plain_fp64": fp64,
        "roofline": roofline,
    }
    if not args.no_cpu_baseline:
        cb = cpu_baseline(A, B)
        ok = (cb["intersects"] == res["hit"] and
              abs(cb["distance"] - res["dist"]) <= 1e-12 * cb["distance"])
        cb["matches_gpu"] = bool(ok)
        line["cpu_baseline"] = {k: v for k, v in cb.items() if k not in ("distance", "intersects")}
    print(json.dumps(line), flush=True)


def sd3_K():
    return 64


if __name__ == "__main__":
    main()
