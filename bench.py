"""Benchmark: exact 3D distance + intersects between two 512 x 512-cell TINs.

Workload (one geometry pair): two heightfield TINs of 524,288 triangles each
over a 1000 x 1000 extent, seeded 6-octave value-noise heights of amplitude
50, the second surface lifted to a minimum vertical clearance of 0.01 (the
two-surface "nearly touching" configuration).  The paper measures on mining
data that is not distributed; these synthetic surfaces stand in for it.

A step is one pass of the whole path over the input already resident in HBM:
sd3_distance (validation, Morton sort + tiling, tile-pair bounds and queue,
learned seed round, FP32 triangle-pair pass with error bounds, FP64 rescue,
exact fallback, final reduction) followed by sd3_intersects (same stages,
any-hit).  The plain-FP64 path (box-bound seed order) runs the same step for
comparison; the results must match bit for bit.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--no-cpu-baseline]
    python bench.py --copy-calibration     # device copy of known size, for PMC scaling

Prints one JSON line.  value = all-pairs-equivalent triangle-pair tests per
second (Na * Nb pairs settled per step / step time).
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "tri-pair tests/s + geometry-pairs/s, FP32+learned vs plain FP64, exact match"

# Algorithmic work per unit, counted from the kernel source (FMA = 2 flops,
# reciprocal / reciprocal square root = 1, min/max/select = 0):
FLOPS_FP32_PAIR = 711   # full FP32 triangle-pair test: 9 edge/edge, 6 vertex/face, bound
FLOPS_BOX = 12          # triangle bounding-box lower bound per boxed pair
FLOPS_TRI_PREP = 64     # per staged triangle (edges, reciprocals, dual basis, box)
# Algorithmic bytes of tile building per triangle: sorted index 4, triangle
# indices 12, three FP64 vertices 72 (read); FP64 copy 72, FP32 copy 36 (write)
BYTES_TILE_TRI = 4 + 12 + 72 + 72 + 36
PEAK_FP32_TFLOPS = 157.3
PEAK_FP64_TFLOPS = 78.6
HBM_PEAK_GBS = 8000.0
COPY_BYTES = 1 << 30    # --copy-calibration: 1 GiB read + 1 GiB written

TRAFFIC_FILE = os.path.join(ROOT, "profiles", "traffic_tin512_pair.json")
KERNEL_SRC = os.path.join(ROOT, "paper_1808_09571_amd", "csrc", "sd3_kernels.hip")


def parse():
    p = argparse.ArgumentParser()
    p.add_argument("--gpus", type=int, default=1)
    p.add_argument("--steps", type=int, default=20)
    p.add_argument("--warmup", type=int, default=3)
    p.add_argument("--no-cpu-baseline", action="store_true")
    p.add_argument("--no-fp64", action="store_true", help="skip the plain FP64 comparison")
    p.add_argument("--copy-calibration", action="store_true")
    return p.parse_args()


def kernel_source_hash():
    with open(KERNEL_SRC, "rb") as f:
        return hashlib.sha256(f.read()).hexdigest()[:16]


def measured_traffic(kernel):
    """HBM bytes per launch from committed PMC counters, or None when the
    kernel source changed since they were taken."""
    try:
        with open(TRAFFIC_FILE) as f:
            t = json.load(f)
    except (OSError, ValueError):
        return None
    if t.get("kernel_source_sha256_16") != kernel_source_hash():
        return None
    k = t.get("kernels", {}).get(kernel)
    return None if k is None else k.get("bytes_per_launch")


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


def copy_calibration():
    import torch
    a = torch.empty(COPY_BYTES // 4, dtype=torch.float32, device="cuda:0").fill_(1.0)
    b = torch.empty_like(a)
    torch.cuda.synchronize()
    for _ in range(3):
        b.copy_(a)
    torch.cuda.synchronize()
    print(json.dumps({"copy_bytes_read": COPY_BYTES, "copy_bytes_written": COPY_BYTES,
                      "launches": 3}))


def roofline_for(kernel, st_list, ms, n):
    """Roofline object of one instrumented kernel class over a step.
    st_list: stats of the step's calls; ms / n: its summed time / launches."""
    avg = ms / max(n, 1)
    if kernel == "scatter":
        items = st_list[0]["sort_items"]
        kb = st_list[0]["sort_key_bytes"]
        per = items * (kb + 4) * 2
        ach = per / (avg * 1e-3) / 1e9
        return {"kernel": "k_scatter (radix sort pass)", "bound": "hbm", "achieved": ach,
                "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": ach / HBM_PEAK_GBS,
                "traffic": measured_traffic("k_scatter"), "avg_launch_ms": avg,
                "algorithmic_bytes_per_launch": per,
                "per_unit": f"{2 * (kb + 4)} B per key ({kb} B key + 4 B value, read + write)"}
    if kernel == "tiles":
        tris = st_list[0]["sort_items"] / 2.0
        per = tris * BYTES_TILE_TRI
        ach = per / (avg * 1e-3) / 1e9
        return {"kernel": "k_tiles", "bound": "hbm", "achieved": ach, "peak": HBM_PEAK_GBS,
                "unit": "GB/s", "frac": ach / HBM_PEAK_GBS, "traffic": measured_traffic("k_tiles"),
                "avg_launch_ms": avg, "algorithmic_bytes_per_launch": per,
                "per_unit": f"{BYTES_TILE_TRI} B per triangle"}
    raise KeyError(kernel)


def pairs_roofline(st, ms, n):
    avg = ms / max(n, 1)
    flops = (st["tri_pairs_fp32"] * FLOPS_FP32_PAIR + st["tri_pairs_boxed"] * FLOPS_BOX +
             st["tile_pairs_evaluated"] * 128 * FLOPS_TRI_PREP)
    ach = flops / (avg * 1e-3) / 1e12 if avg > 0 else 0.0
    return {"kernel": "k_pairs<fp32,distance>", "bound": "alu", "achieved": ach,
            "peak": PEAK_FP32_TFLOPS, "unit": "TFLOP/s", "frac": ach / PEAK_FP32_TFLOPS,
            "avg_launch_ms": avg, "flops_per_launch": flops,
            "per_unit": f"{FLOPS_FP32_PAIR} flops per FP32 pair test, {FLOPS_BOX} per box test"}


def main():
    args = parse()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (got --gpus {args.gpus}); multi-GPU is not part "
              "of this build", file=sys.stderr)
        sys.exit(2)
    if args.copy_calibration:
        copy_calibration()
        return
    import numpy as np
    import torch

    from paper_1808_09571_amd import ranker, sd3, synth

    A, B = synth.config_tin_pair()
    na, nb = len(A[1]), len(B[1])
    dev = "cuda:0"
    ba = sd3.Batch.from_packed(synth.pack([A]), dev)
    bb = sd3.Batch.from_packed(synth.pack([B]), dev)
    ctx = sd3.Context(0)
    weights = ranker.load(device=dev)

    def step(prec, order, timing=False):
        w = weights if order == "learned" else None
        d, h, sd = ctx.distance(ba, bb, precision=prec, order=order, stats=True, timing=timing,
                                ranker=w)
        hi, si = ctx.intersects(ba, bb, precision=prec, stats=True, timing=timing)
        return d, h, hi, sd, si

    def timed(prec, order):
        for _ in range(args.warmup):
            step(prec, order)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(args.steps):
            out = step(prec, order)
        torch.cuda.synchronize()
        return (time.perf_counter() - t0) / args.steps, out

    # the method: FP32 + FP64 rescue with the learned seed round
    t32, (d32, h32, hi32, sd32, si32) = timed("fp32", "learned")
    res = {"dist": float(d32.cpu()[0]), "hit": bool(h32.cpu()[0]), "hit_any": bool(hi32.cpu()[0])}
    tiles = {"learned": sd32["tile_pairs_evaluated"]}
    for order in ("bound", "none"):
        tiles[order] = ctx.distance(ba, bb, order=order, stats=True)[2]["tile_pairs_evaluated"]
    fp64 = None
    if not args.no_fp64:
        t64, (d64, h64, hi64, sd64, si64) = timed("fp64", "bound")
        exact = (d32.cpu().numpy().view(np.int64)[0] == d64.cpu().numpy().view(np.int64)[0]
                 and bool(h32.cpu()[0]) == bool(h64.cpu()[0])
                 and bool(hi32.cpu()[0]) == bool(hi64.cpu()[0]))
        fp64 = {"ms_per_step": t64 * 1e3, "geometry_pairs_per_s": 1.0 / t64,
                "value": na * nb / t64, "order": "bound",
                "tile_pairs_evaluated": sd64["tile_pairs_evaluated"],
                "tri_pairs_fp64_per_step": sd64["tri_pairs_fp64"] + si64["tri_pairs_fp64"],
                "exact_match_fp32_vs_fp64": bool(exact), "speedup_fp32_over_fp64": t64 / t32}

    # live per-kernel timing (HIP events on the call's stream), separate steps
    n_t = max(3, min(args.steps, 10))
    phase, kms, kn = {}, {}, {}
    for _ in range(n_t):
        _, _, _, sd, si = step("fp32", "learned", timing=True)
        for tag, s in (("dist", sd), ("isect", si)):
            for k, v in s["ms_phase"].items():
                phase[(tag, k)] = phase.get((tag, k), 0.0) + v / n_t
            for k, v in s["ms_kernel"].items():
                kms[k] = kms.get(k, 0.0) + v / n_t
                kn[k] = kn.get(k, 0) + s["n_kernel"][k] / n_t
    # the dominant kernel by device time per step
    hbm_classes = [k for k in ("scatter", "tiles") if kn.get(k)]
    dom = max(kms, key=lambda k: kms[k])
    if dom in hbm_classes:
        roof = roofline_for(dom, [sd, si], kms[dom], kn[dom])
    else:
        roof = pairs_roofline(sd, kms["pairs"] / 2, max(kn["pairs"] / 2, 1))
    roof["dominant_by_time"] = dom
    roof["kernel_ms_per_step"] = {k: round(v, 4) for k, v in kms.items()}
    secondary = pairs_roofline(sd, sd["ms_kernel"]["pairs"], sd["n_kernel"]["pairs"])

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
                   "geometry_pairs": 1, "order": "learned", "ranker": "ranker_weights.npy"},
        "geometry_pairs_per_s": 1.0 / t32,
        "tri_pairs_executed_per_step": tri_exec,
        "tri_pairs_executed_per_s": tri_exec / t32,
        "tile_pairs_evaluated": tiles,
        "result": res,
        "stats_distance": {k: v for k, v in sd32.items()
                           if k not in ("ms_phase", "ms_kernel", "n_kernel")},
        "phase_ms": {f"{t}.{k}": round(v, 4) for (t, k), v in phase.items()},
        "plain_fp64": fp64,
        "roofline": roof,
        "roofline_pairs_fp32": secondary,
    }
    if not args.no_cpu_baseline:
        cb = cpu_baseline(A, B)
        ok = (cb["intersects"] == res["hit"] and
              abs(cb["distance"] - res["dist"]) <= 1e-12 * cb["distance"])
        cb["matches_gpu"] = bool(ok)
        line["cpu_baseline"] = {k: v for k, v in cb.items() if k not in ("distance", "intersects")}
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
