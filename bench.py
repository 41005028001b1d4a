"""Benchmark: exact 3D distance + intersects between triangulated surfaces.

Default workload (one geometry pair, the configuration the headline metric
is quoted on): two heightfield TINs of 524,288 triangles each over a
1000 x 1000 extent, seeded 6-octave value-noise heights of amplitude 50, the
second surface lifted to a minimum vertical clearance of 0.01 (the
two-surface "nearly touching" configuration).  --workload batch4096 runs the
4096-row drill-hole / ore-body batch, --workload scale the 4M-triangle TIN vs
1M-triangle blob.  The paper measures on mining data that is not
distributed; these synthetic inputs stand in for it.

A step is one pass of the whole path over the input already resident in HBM:
sd3_distance (validation, Morton sort + tiling, tile-pair bounds and queue,
learned seed round, FP32 triangle-pair pass with error bounds, FP64 rescue,
exact fallback, final reduction) and sd3_intersects (same stages, any-hit),
each replayed from a HIP graph with the tile size chosen by the autotuner;
the two queries are independent and run on two streams (the one-stream time
is reported beside).  The plain-FP64 path (box-bound seed order, its own
graphs and tuned tiles) runs the same step for comparison; the results must
match bit for bit.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--no-cpu-baseline]
                    [--workload tin512|batch4096|scale] [--orders]
    python bench.py --copy-calibration     # device copy of known size, for PMC scaling

--orders adds, per seed order (learned, box bound, none) and precision, the
sd3_distance graph time, the tile pairs it evaluated and whether its bits
equal the others'.

Prints one JSON line.  value = all-pairs-equivalent triangle-pair tests per
second (sum over rows of Na * Nb pairs settled per step / step time).
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
# Algorithmic bytes of tile building per triangle on the FP32 path: sorted
# index 4, triangle indices 12, three FP64 vertices 72 (read); FP32 copy 36,
# slot triangle id 4 (write)
BYTES_TILE_TRI = 4 + 12 + 72 + 36 + 4
PEAK_FP32_TFLOPS = 157.3
PEAK_FP64_TFLOPS = 78.6
HBM_PEAK_GBS = 8000.0
COPY_BYTES = 1 << 30    # --copy-calibration: 1 GiB read + 1 GiB written
TUNE_REPS = 8           # autotuner rounds (each times every tile size once)

TRAFFIC_FILES = {"tin512": "traffic_tin512_pair.json", "batch4096": "traffic_batch4096.json",
                 "scale": "traffic_scale_tin_blob.json"}
KERNEL_SRC = os.path.join(ROOT, "paper_1808_09571_amd", "csrc", "sd3_kernels.hip")


def parse():
    p = argparse.ArgumentParser()
    p.add_argument("--gpus", type=int, default=1)
    p.add_argument("--steps", type=int, default=20)
    p.add_argument("--warmup", type=int, default=3)
    p.add_argument("--no-cpu-baseline", action="store_true")
    p.add_argument("--no-fp64", action="store_true", help="skip the plain FP64 comparison")
    p.add_argument("--copy-calibration", action="store_true")
    p.add_argument("--orders", action="store_true",
                   help="also time sd3_distance per seed order and precision")
    p.add_argument("--workload", default="tin512", choices=["tin512", "batch4096", "scale"],
                   help="tin512 (default): the two-TIN pair; batch4096: the 4096-row tube/blob "
                        "batch; scale: the 4M-triangle TIN vs 1M-triangle blob")
    return p.parse_args()


def kernel_source_hash():
    with open(KERNEL_SRC, "rb") as f:
        return hashlib.sha256(f.read()).hexdigest()[:16]


def measured_traffic(kernel, workload):
    """HBM bytes per launch from committed PMC counters of this workload, or
    None when the kernel source changed since they were taken."""
    try:
        with open(os.path.join(ROOT, "profiles", TRAFFIC_FILES[workload])) as f:
            t = json.load(f)
    except (OSError, ValueError):
        return None
    if t.get("kernel_source_sha256_16") != kernel_source_hash():
        return None
    k = t.get("kernels", {}).get(kernel)
    return None if k is None else k.get("bytes_per_launch")


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


def roofline_for(kernel, st_list, ms, n, workload):
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
                "traffic": measured_traffic("k_scatter", workload), "avg_launch_ms": avg,
                "algorithmic_bytes_per_launch": per,
                "per_unit": f"{2 * (kb + 4)} B per key ({kb} B key + 4 B value, read + write)"}
    if kernel == "tiles":
        # one launch builds the tiles of both sides: every sorted item
        tris = float(st_list[0]["sort_items"])
        per = tris * BYTES_TILE_TRI
        ach = per / (avg * 1e-3) / 1e9
        return {"kernel": "k_tiles", "bound": "hbm", "achieved": ach, "peak": HBM_PEAK_GBS,
                "unit": "GB/s", "frac": ach / HBM_PEAK_GBS, "traffic": measured_traffic("k_tiles", workload),
                "avg_launch_ms": avg, "algorithmic_bytes_per_launch": per,
                "per_unit": f"{BYTES_TILE_TRI} B per triangle"}
    raise KeyError(kernel)


def pairs_roofline(st, ms, n, workload):
    """st: the call's stats (every queue pass); ms / n: the call's summed
    main-pass time / launches (one per queue pass)."""
    n = max(n, 1)
    avg = ms / n
    flops = (st["tri_pairs_fp32"] * FLOPS_FP32_PAIR + st["tri_pairs_boxed"] * FLOPS_BOX +
             st["tile_pairs_evaluated"] * 128 * FLOPS_TRI_PREP) / n
    ach = flops / (avg * 1e-3) / 1e12 if avg > 0 else 0.0
    return {"kernel": "k_pairs<fp32,distance>", "bound": "alu", "achieved": ach,
            "peak": PEAK_FP32_TFLOPS, "unit": "TFLOP/s", "frac": ach / PEAK_FP32_TFLOPS,
            "traffic": measured_traffic(f"k_pairs<fp32,distance,{st['tile']}> main pass", workload),
            "avg_launch_ms": avg, "flops_per_launch": flops,
            "per_unit": f"{FLOPS_FP32_PAIR} flops per FP32 pair test, {FLOPS_BOX} per box test"}


WORKLOADS = {
    "tin512": "two 512x512-cell TINs, 524288 triangles each, clearance 0.01, distance + intersects",
    "batch4096": "4096 rows: drill-hole tube (200-20k triangles) vs ore-body blob (1k-200k "
                 "triangles), log-uniform sizes, distance + intersects",
    "scale": "2000x1000-cell TIN (4,000,000 triangles) vs 1,003,520-triangle blob 0.001 above "
             "it, distance + intersects",
}


def time_orders(ctx, ba, bb, weights, args):
    """sd3_distance graph replays per seed order and precision: ms per call,
    tile pairs evaluated, and whether the bits equal the first variant's."""
    import numpy as np
    import torch
    out, ref = {}, None
    for prec in ("fp32", "fp64"):
        for order in ("learned", "bound", "none"):
            g = ctx.graph("distance", ba, bb, precision=prec, order=order,
                          ranker=weights if order == "learned" else None)
            for _ in range(max(args.warmup, 1)):
                g.launch()
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            for _ in range(args.steps):
                g.launch()
            torch.cuda.synchronize()
            ms = (time.perf_counter() - t0) / args.steps * 1e3
            st = g.result(stats=True)
            bits = g.dist.cpu().numpy().view(np.int64).copy()
            ref = bits if ref is None else ref
            out[f"{prec}.{order}"] = {"ms_per_call": round(ms, 4),
                                      "tile_pairs_evaluated": st["tile_pairs_evaluated"],
                                      "same_bits": bool(np.array_equal(bits, ref))}
            g.close()
    return out


def make_workload(name):
    from paper_1808_09571_amd import synth
    if name == "tin512":
        A, B = synth.config_tin_pair()
        return [A], [B]
    if name == "batch4096":
        return synth.config_tube_blob_batch(rows=4096, seed=3)
    if name == "scale":
        A, B = synth.config_tin_blob()
        return [A], [B]
    raise KeyError(name)


def cpu_baseline_rows(A, B, budget_s=12.0):
    """The FP64 oracle (exact pruned mode, all host cores) on whole rows taken
    in order until about ``budget_s`` of work; for a single-row workload the
    row is repeated until the budget is spent.  Returns the rate over the
    sample and the sampled rows' results."""
    import oracle
    threads = oracle.default_threads()
    t_all, pairs, runs, rows = 0.0, 0, 0, []
    while t_all < budget_s and runs < 50:
        g = runs % len(A)
        t0 = time.perf_counter()
        d, h, tests = oracle.mesh(A[g], B[g], mode="pruned", threads=threads)
        t_all += time.perf_counter() - t0
        pairs += len(A[g][1]) * len(B[g][1])
        runs += 1
        if len(rows) < len(A) and (not rows or rows[-1][0] != g):
            rows.append((g, d, h))
    sample = (f"{runs} oracle run(s) over rows 0..{min(runs, len(A)) - 1} of the same workload, "
              f"exact pruned mode, {t_all:.1f} s")
    return {"value": pairs / t_all, "unit": "tri-pairs/s (all-pairs-equivalent)", "cores": threads,
            "kind": "oracle", "sample": sample}, rows


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

    A, B = make_workload(args.workload)
    G = len(A)
    na = sum(len(a[1]) for a in A)
    nb = sum(len(b[1]) for b in B)
    allpairs = sum(len(a[1]) * len(b[1]) for a, b in zip(A, B))
    dev = "cuda:0"
    ba = sd3.Batch.from_packed(synth.pack(A), dev)
    bb = sd3.Batch.from_packed(synth.pack(B), dev)
    ctx = sd3.Context(0)
    weights = ranker.load(device=dev)

    # tile sizes picked by the autotuner on this workload (the choice is kept
    # in the context for tile=0 calls and graphs)
    tune = {"distance": ctx.autotune("distance", ba, bb, order="learned", ranker=weights, reps=TUNE_REPS),
            "intersects": ctx.autotune("intersects", ba, bb, reps=TUNE_REPS)}
    tune64 = {"distance": ctx.autotune("distance", ba, bb, precision="fp64", reps=TUNE_REPS),
              "intersects": ctx.autotune("intersects", ba, bb, precision="fp64", reps=TUNE_REPS)}

    def graphs(prec, order):
        w = weights if order == "learned" else None
        return (ctx.graph("distance", ba, bb, precision=prec, order=order, ranker=w),
                ctx.graph("intersects", ba, bb, precision=prec))

    # the step's two queries are independent and each graph has its own
    # workspace: distance replays on the current stream, intersects on a
    # second one (default priority), so the two overlap; replays of one graph
    # stay in order on its own stream
    side = torch.cuda.Stream()

    def timed_graphs(gd, gi):
        """K steps of (distance replay, intersects replay): concurrent on two
        streams (the step time) and serial on one stream (reported beside)."""
        def step(concurrent):
            gd.launch()
            if concurrent:
                with torch.cuda.stream(side):
                    gi.launch()
            else:
                gi.launch()

        out = {}
        for concurrent in (False, True):
            for _ in range(args.warmup):
                step(concurrent)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            for _ in range(args.steps):
                step(concurrent)
            torch.cuda.synchronize()
            out[concurrent] = (time.perf_counter() - t0) / args.steps
        return out[True], out[False], gd.result(stats=True), gi.result(stats=True)

    # the method: FP32 + FP64 rescue with the learned seed round, HIP graphs
    gd32, gi32 = graphs("fp32", "learned")
    t32, t32_serial, sd32, si32 = timed_graphs(gd32, gi32)
    d32 = gd32.dist.cpu().numpy()
    h32 = gd32.hit.cpu().numpy().astype(bool)
    hi32 = gi32.hit.cpu().numpy().astype(bool)
    tiles = {"learned": sd32["tile_pairs_evaluated"]}
    for order in ("bound", "none"):
        tiles[order] = ctx.distance(ba, bb, order=order, stats=True)[2]["tile_pairs_evaluated"]
    # the same step as eager calls (one host synchronisation per call)
    for _ in range(args.warmup):
        ctx.distance(ba, bb, order="learned", ranker=weights)
        ctx.intersects(ba, bb)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        ctx.distance(ba, bb, order="learned", ranker=weights)
        ctx.intersects(ba, bb)
    t_eager = (time.perf_counter() - t0) / args.steps
    fp64 = None
    if not args.no_fp64:
        gd64, gi64 = graphs("fp64", "bound")
        t64, t64_serial, sd64, si64 = timed_graphs(gd64, gi64)
        exact = (np.array_equal(d32.view(np.int64), gd64.dist.cpu().numpy().view(np.int64))
                 and np.array_equal(h32, gd64.hit.cpu().numpy().astype(bool))
                 and np.array_equal(hi32, gi64.hit.cpu().numpy().astype(bool)))
        fp64 = {"ms_per_step": t64 * 1e3, "serial_ms_per_step": t64_serial * 1e3,
                "geometry_pairs_per_s": G / t64,
                "value": allpairs / t64, "order": "bound",
                "tiles": {"distance": tune64["distance"]["best"],
                          "intersects": tune64["intersects"]["best"]},
                "tile_pairs_evaluated": sd64["tile_pairs_evaluated"],
                "tri_pairs_fp64_per_step": sd64["tri_pairs_fp64"] + si64["tri_pairs_fp64"],
                "exact_match_fp32_vs_fp64": bool(exact), "speedup_fp32_over_fp64": t64 / t32}
        gd64.close()
        gi64.close()

    # live per-kernel timing (HIP events on the call's stream), eager steps
    n_t = max(3, min(args.steps, 10))
    phase, kms, kn = {}, {}, {}
    for _ in range(n_t):
        _, _, sd = ctx.distance(ba, bb, order="learned", ranker=weights, stats=True, timing=True)
        _, si = ctx.intersects(ba, bb, stats=True, timing=True)
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
        roof = roofline_for(dom, [sd, si], kms[dom], kn[dom], args.workload)
    else:
        roof = pairs_roofline(sd, sd["ms_kernel"]["pairs"], max(sd["n_kernel"]["pairs"], 1), args.workload)
    roof["dominant_by_time"] = dom
    roof["kernel_ms_per_step"] = {k: round(v, 4) for k, v in kms.items()}
    secondary = pairs_roofline(sd, sd["ms_kernel"]["pairs"], sd["n_kernel"]["pairs"], args.workload)

    tri_exec = (sd32["tri_pairs_fp32"] + sd32["tri_pairs_fp64"] + si32["tri_pairs_fp32"] +
                si32["tri_pairs_fp64"])
    line = {
        "metric": METRIC,
        "value": allpairs / t32,
        "unit": "tri-pairs/s (all-pairs-equivalent: Na*Nb settled per second)",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": t32 * 1e3, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f32 (bulk) + f64 (rescue, result)", "data": "synthetic",
        "config": {"workload": WORKLOADS[args.workload], "triangles_a": na, "triangles_b": nb,
                   "geometry_pairs": G, "order": "learned", "ranker": "ranker_weights.npy",
                   "launch": "HIP graph per operator; distance and intersects on two streams",
                   "tiles": {"distance": tune["distance"]["best"],
                             "intersects": tune["intersects"]["best"]}},
        "geometry_pairs_per_s": G / t32,
        "tri_pairs_executed_per_step": tri_exec,
        "tri_pairs_executed_per_s": tri_exec / t32,
        "serial_ms_per_step": t32_serial * 1e3,
        "eager_ms_per_step": t_eager * 1e3,
        "autotune_ms": {k: {str(t): round(v, 4) for t, v in r["ms"].items()} for k, r in tune.items()},
        "tile_pairs_evaluated": tiles,
        "result": {"rows": G, "hits_distance": int(h32.sum()), "hits_intersects": int(hi32.sum()),
                   "dist_row0": float(d32[0]), "hit_row0": bool(h32[0])},
        "stats_distance": {k: v for k, v in sd32.items()
                           if k not in ("ms_phase", "ms_kernel", "n_kernel", "ms_total")},
        "phase_ms": {f"{t}.{k}": round(v, 4) for (t, k), v in phase.items()},
        "plain_fp64": fp64,
        "roofline": roof,
        "roofline_pairs_fp32": secondary,
    }
    gd32.close()
    gi32.close()
    if args.orders:
        line["orders_distance"] = time_orders(ctx, ba, bb, weights, args)
    if not args.no_cpu_baseline:
        cb, rows = cpu_baseline_rows(A, B)
        ok = all(h == bool(h32[g]) and (h or abs(d - d32[g]) <= 1e-12 * d) for g, d, h in rows)
        cb["matches_gpu"] = bool(ok)
        # largest relative error of the method's distances against the oracle
        # over the sampled rows (intersecting rows: both must be exactly 0)
        def rel_err(d, x):
            if d == 0.0 or d == float("inf"):
                return 0.0 if x == d else float("inf")
            return abs(d - x) / d

        errs = [rel_err(d, float(d32[g])) for g, d, h in rows]
        cb["max_rel_err_vs_oracle"] = max(errs) if errs else None
        cb["rows_checked"] = len(rows)
        line["cpu_baseline"] = cb
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
