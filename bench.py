"""Benchmark: exact 3D distance + intersects between triangulated surfaces.

Headline workload (the configuration the metric is quoted on: a batch of
geometry pairs, one per table row, FP32 + learned seed order): 4096 rows of
a drill-hole tube (16-gon cross-section along a random 3D polyline, 200-20k
triangles) against an ore-body blob (icosphere with seeded radial noise,
1k-200k triangles, log-uniform sizes), about a third of the rows touching;
1.7e8 triangles in all.  Two more workloads ride along as sub-objects of the
same line: the 4M-triangle TIN vs 1M-triangle blob scale case and the pair
of 512 x 512-cell TINs nearly touching.  The paper measures on mining data
that is not distributed; these synthetic inputs stand in for it, with its
shapes (drill holes, ore bodies, terrain surfaces).

A step is one pass of the whole path over the batch already resident in HBM:
sd3_distance (validation, Morton sort + tiling, tile-pair bounds and queue,
learned seed round, FP32 triangle-pair pass with error bounds, FP64 rescue,
exact fallback, final reduction) and sd3_intersects (same stages, any-hit),
each replayed from a HIP graph with the tile size the autotuner chose; the
two queries are independent and run on two streams, each on a hardware queue
of its own (the one-stream time is reported beside).  The plain-FP64 path
(box-bound seed order, its own graphs and tuned tiles) runs the same step for
comparison, and the line records whether the bits match.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--no-cpu-baseline]
                    [--workload batch4096|scale|tin512] [--extras scale,tin512]
                    [--no-fp64] [--orders]
    python bench.py --copy-calibration      # device copy of known size, for PMC scaling
    python bench.py --summarize DIR --kind stats|pmc|sq [--workload W]
                                            # profile summaries from rocprofv3 output

value = geometry pairs per second of the headline workload (rows / step
time, a step being both queries).  Executed triangle-pair tests per second
(FP32 pass and FP64 re-evaluations separately) and the all-pairs-equivalent
rate (sum over rows of Na * Nb / step time) are labelled extras.
"""
from __future__ import annotations

import argparse
import csv
import glob
import hashlib
import json
import os
import platform
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
# Algorithmic bytes of tile building on the FP32 path: per triangle the sorted
# item 4 and the triangle indices 12 (read) and the slot triangle id 4
# (written), plus the FP32 copy 36 (written) in calls of fewer than
# LAZY_COPY_MIN_TILES tiles (larger calls write the copies of queued tiles
# only, in a later kernel); per vertex its FP64 coordinates 24, read once (a
# vertex is shared by the triangles around it); per tile its 112-byte metadata
BYTES_TILE_TRI = 4 + 12 + 4
BYTES_TILE_COPY = 36
BYTES_TILE_VTX = 24
BYTES_TILE_META = 112
LAZY_COPY_MIN_TILES = 16384
TILE_META_PER_WAVE = {32: 4, 64: 4, 128: 2}  # metadata-only build: tiles per wave
VOL_BYTES_TRI = 12 + 72  # volume: triangle indices and three FP64 vertices
PEAK_FP32_TFLOPS = 157.3
PEAK_FP64_TFLOPS = 78.6
HBM_PEAK_GBS = 8000.0
COPY_BYTES = 1 << 30    # --copy-calibration: 1 GiB read + 1 GiB written
TUNE_REPS = 8           # autotuner rounds (each times every tile size once)
CPU_BUDGET_S = 12.0     # oracle time per CPU-baseline leg (all cores, then one core)

TRAFFIC_FILES = {"tin512": "traffic_tin512_pair.json", "batch4096": "traffic_batch4096.json",
                 "scale": "traffic_scale_tin_blob.json"}
KERNEL_SRC = os.path.join(ROOT, "paper_1808_09571_amd", "csrc", "sd3_kernels.hip")

WORKLOADS = {
    "batch4096": "4096 rows: drill-hole tube (200-20k triangles) vs ore-body blob (1k-200k "
                 "triangles), log-uniform sizes, distance + intersects",
    "scale": "2000x1000-cell TIN (4,000,000 triangles) vs 1,003,520-triangle blob 0.001 above "
             "it, distance + intersects",
    "tin512": "two 512x512-cell TINs, 524288 triangles each, clearance 0.01, distance + intersects",
}


def parse():
    p = argparse.ArgumentParser()
    p.add_argument("--gpus", type=int, default=1)
    p.add_argument("--steps", type=int, default=20)
    p.add_argument("--warmup", type=int, default=3)
    p.add_argument("--no-cpu-baseline", action="store_true")
    p.add_argument("--no-fp64", action="store_true", help="skip the plain FP64 comparison")
    p.add_argument("--copy-calibration", action="store_true")
    p.add_argument("--orders", action="store_true",
                   help="also time sd3_distance per seed order in FP64 (FP32 is always timed)")
    p.add_argument("--workload", default="batch4096", choices=list(WORKLOADS))
    p.add_argument("--extras", default="scale,tin512,segments,volume",
                   help="comma-separated sub-objects: scale, tin512 (mesh workloads), segments "
                        "(5 M drill-hole segments vs a 500-face body), volume (every mesh of the "
                        "headline workload); '' for none")
    p.add_argument("--summarize", default=None, metavar="DIR",
                   help="summarise rocprofv3 output under DIR (see --kind) and exit")
    p.add_argument("--kind", default="stats", choices=["stats", "pmc", "sq"])
    p.add_argument("--cmd", action="append", default=[], metavar="COMMAND",
                   help="with --summarize: a command that produced the profiled output (recorded "
                        "in the summary; repeatable)")
    p.add_argument("--calib", default=None, metavar="DIR",
                   help="with --kind pmc: rocprofv3 output of --copy-calibration (FETCH, WRITE dirs "
                        "as DIR_FETCH_SIZE, DIR_WRITE_SIZE)")
    return p.parse_args()


def kernel_source_hash():
    with open(KERNEL_SRC, "rb") as f:
        return hashlib.sha256(f.read()).hexdigest()[:16]


def cpu_model():
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return platform.processor() or "unknown"


def measured_traffic(kernel, workload):
    """HBM bytes per launch from committed PMC counters of this workload, or
    None when the kernel source changed since they were taken."""
    if workload not in TRAFFIC_FILES:
        return None
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


# ---------------------------------------------------------------------------
# roofline objects
# ---------------------------------------------------------------------------
def roofline_for(kernel, st_list, ms, n, workload, nverts):
    """Roofline object of one instrumented HBM-bound kernel class over a
    step.  st_list: stats of the step's calls; ms / n: summed time / launches;
    nverts: vertices of both sides."""
    avg = ms / max(n, 1)
    if kernel == "scatter":
        items = st_list[0]["sort_items"]
        ib, npass = st_list[0]["sort_item_bytes"], st_list[0]["sort_passes"]
        # bytes an item moves, read and written, averaged over the passes
        # (key + value passes move 16 B, the narrowing pass and a last
        # key + value pass 12 B, the last pass of a narrow sort 8 B)
        per_item = ib / npass
        what = f"{per_item:g} B per item ({ib} B over {npass} passes, read + write)"
        per = items * per_item
        ach = per / (avg * 1e-3) / 1e9
        return {"kernel": "k_scatter (radix sort pass)", "bound": "hbm", "achieved": ach,
                "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": ach / HBM_PEAK_GBS,
                "traffic": measured_traffic("k_scatter", workload), "avg_launch_ms": avg,
                "algorithmic_bytes_per_launch": per, "per_unit": what}
    if kernel == "tiles":
        # one launch builds the tiles of both sides: every sorted item; the
        # step's launches use the two queries' tile sizes
        tris = float(st_list[0]["sort_items"])
        ntiles = tris / st_list[0]["tile"]
        per_tri = BYTES_TILE_TRI + (BYTES_TILE_COPY if ntiles < LAZY_COPY_MIN_TILES else 0)
        per = tris * per_tri + float(nverts) * BYTES_TILE_VTX + ntiles * BYTES_TILE_META
        ach = per / (avg * 1e-3) / 1e9
        # kernel names: large calls build metadata only (k_tiles_meta<tile
        # size, tiles per wave>), small ones copies too (k_tiles<two slots
        # per lane>)
        def tile_kernel(x):
            tk = x["tile"]
            if x["sort_items"] / tk >= LAZY_COPY_MIN_TILES:
                return f"k_tiles_meta<{tk}, {TILE_META_PER_WAVE[tk]}>"
            return f"k_tiles<{'true' if tk == 128 else 'false'}>"
        tr = [measured_traffic(tile_kernel(x), workload) for x in st_list]
        return {"kernel": "k_tiles", "bound": "hbm", "achieved": ach, "peak": HBM_PEAK_GBS,
                "unit": "GB/s", "frac": ach / HBM_PEAK_GBS,
                "traffic": None if None in tr else sum(tr) / len(tr),
                "avg_launch_ms": avg, "algorithmic_bytes_per_launch": per,
                "per_unit": f"{per_tri} B per triangle + {BYTES_TILE_VTX} B per vertex + "
                            f"{BYTES_TILE_META} B per tile"}
    raise KeyError(kernel)


def pairs_roofline(st, ms, n, workload):
    """st: the call's stats (every queue pass); ms / n: the call's summed
    main-pass time / launches (one per queue pass)."""
    n = max(n, 1)
    avg = ms / n
    flops = (st["tri_pairs_fp32"] * FLOPS_FP32_PAIR + st["tri_pairs_boxed"] * FLOPS_BOX +
             st["tile_pairs_evaluated"] * 2 * st["tile"] * FLOPS_TRI_PREP) / n
    ach = flops / (avg * 1e-3) / 1e12 if avg > 0 else 0.0
    return {"kernel": "k_pairs<fp32,distance>", "bound": "alu", "achieved": ach,
            "peak": PEAK_FP32_TFLOPS, "unit": "TFLOP/s", "frac": ach / PEAK_FP32_TFLOPS,
            "traffic": measured_traffic(f"k_pairs<fp32,distance,{st['tile']}> main pass", workload),
            "avg_launch_ms": avg, "flops_per_launch": flops,
            "per_unit": f"{FLOPS_FP32_PAIR} flops per FP32 pair test, {FLOPS_BOX} per box test, "
                        f"{FLOPS_TRI_PREP} per staged triangle"}


# ---------------------------------------------------------------------------
# workloads
# ---------------------------------------------------------------------------
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


def graph_time(g, steps, warmup):
    import torch
    for _ in range(max(warmup, 1)):
        g.launch()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        g.launch()
    torch.cuda.synchronize()
    return (time.perf_counter() - t0) / steps


def time_orders(ctx, ba, bb, weights, args, precisions=("fp32",)):
    """sd3_distance graph replays per seed order: ms per call, tile pairs
    evaluated, and whether the bits equal the first variant's."""
    import numpy as np
    out, ref = {}, None
    for prec in precisions:
        for order in ("learned", "bound", "none"):
            g = ctx.graph("distance", ba, bb, precision=prec, order=order,
                          ranker=weights if order == "learned" else None)
            ms = graph_time(g, args.steps, args.warmup) * 1e3
            st = g.result(stats=True)
            bits = g.dist.cpu().numpy().view(np.int64).copy()
            ref = bits if ref is None else ref
            out[f"{prec}.{order}"] = {"ms_per_call": round(ms, 4),
                                      "tile_pairs_evaluated": st["tile_pairs_evaluated"],
                                      "tri_pairs_fp32": st["tri_pairs_fp32"],
                                      "same_bits": bool(np.array_equal(bits, ref))}
            g.close()
    return out


class QueueStreams:
    """Streams that each own a hardware queue.  HIP maps ordinary streams onto
    a few hardware queues (four by default), shared in turn, so two ordinary
    streams can land on one queue and run one after the other; whether they
    do depends on how many streams the process created before.  A stream made
    with a CU mask (here every CU) gets a queue of its own.  Such a stream
    orders itself against the null stream, so the timed steps launch on these
    streams only.  The handles come from torch's own HIP runtime (loaded
    under the same name)."""

    def __init__(self, n):
        import ctypes
        import torch
        self._hip = ctypes.CDLL("libamdhip64.so")
        ncu = torch.cuda.get_device_properties(0).multi_processor_count
        words = (ncu + 31) // 32
        mask = (ctypes.c_uint32 * words)(*([0xFFFFFFFF] * words))
        self._raw, self.streams = [], []
        for _ in range(n):
            h = ctypes.c_void_p()
            st = self._hip.hipExtStreamCreateWithCUMask(ctypes.byref(h), ctypes.c_uint32(words), mask)
            if st != 0:
                self.close()
                raise RuntimeError(f"hipExtStreamCreateWithCUMask failed ({st})")
            self._raw.append(h)
            self.streams.append(torch.cuda.ExternalStream(h.value))

    def close(self):
        import torch
        torch.cuda.synchronize()
        for h in self._raw:
            self._hip.hipStreamDestroy(h)
        self._raw, self.streams = [], []


def measure(name, A, B, ctx, weights, args, headline):
    """Time one workload: the method (FP32 + rescue, learned seed round) and
    the plain FP64 path, graph-replayed, both queries per step.  The headline
    workload also gets per-kernel timing (roofline) and the seed-order table."""
    import numpy as np
    import torch
    from paper_1808_09571_amd import sd3, synth

    G = len(A)
    na = sum(len(a[1]) for a in A)
    nb = sum(len(b[1]) for b in B)
    allpairs = sum(len(a[1]) * len(b[1]) for a, b in zip(A, B))
    dev = "cuda:0"
    ba = sd3.Batch.from_packed(synth.pack(A), dev)
    bb = sd3.Batch.from_packed(synth.pack(B), dev)

    # tile sizes picked by the autotuner on this workload (the choice is kept
    # in the context for tile=0 calls and graphs)
    tune = {"distance": ctx.autotune("distance", ba, bb, order="learned", ranker=weights, reps=TUNE_REPS),
            "intersects": ctx.autotune("intersects", ba, bb, reps=TUNE_REPS)}
    tune64 = None
    if not args.no_fp64:
        tune64 = {"distance": ctx.autotune("distance", ba, bb, precision="fp64", reps=TUNE_REPS),
                  "intersects": ctx.autotune("intersects", ba, bb, precision="fp64", reps=TUNE_REPS)}

    def graphs(prec, order):
        w = weights if order == "learned" else None
        return (ctx.graph("distance", ba, bb, precision=prec, order=order, ranker=w),
                ctx.graph("intersects", ba, bb, precision=prec))

    # the step's two queries are independent and each graph has its own
    # workspace: distance replays on one stream, intersects on a second one
    # (default priority, each stream on a hardware queue of its own), so the
    # two overlap; replays of one graph stay in order on its own stream
    qs = QueueStreams(2)
    main, side = qs.streams

    def timed_graphs(gd, gi):
        """K steps of (distance replay, intersects replay): concurrent on two
        streams (the step time) and serial on one stream (reported beside)."""
        def step(concurrent):
            with torch.cuda.stream(main):
                gd.launch()
            with torch.cuda.stream(side if concurrent else main):
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
    gd32.close()
    gi32.close()
    fp64 = None
    if not args.no_fp64:
        gd64, gi64 = graphs("fp64", "bound")
        t64, t64_serial, sd64, si64 = timed_graphs(gd64, gi64)
        exact = (np.array_equal(d32.view(np.int64), gd64.dist.cpu().numpy().view(np.int64))
                 and np.array_equal(h32, gd64.hit.cpu().numpy().astype(bool))
                 and np.array_equal(hi32, gi64.hit.cpu().numpy().astype(bool)))
        fp64 = {"ms_per_step": t64 * 1e3, "serial_ms_per_step": t64_serial * 1e3,
                "geometry_pairs_per_s": G / t64, "order": "bound",
                "tiles": {"distance": tune64["distance"]["best"],
                          "intersects": tune64["intersects"]["best"]},
                "tile_pairs_evaluated": sd64["tile_pairs_evaluated"],
                "tri_pairs_fp64_per_step": sd64["tri_pairs_fp64"] + si64["tri_pairs_fp64"],
                "exact_match_fp32_vs_fp64": bool(exact), "speedup_fp32_over_fp64": t64 / t32}
        gd64.close()
        gi64.close()
    qs.close()

    fp32_tests =sd32["tri_pairs_fp32"] + si32["tri_pairs_fp32"]
    fp64_tests = sd32["tri_pairs_fp64"] + si32["tri_pairs_fp64"]
    res = {
        "workload": WORKLOADS[name], "rows": G, "triangles_a": na, "triangles_b": nb,
        "ms_per_step": t32 * 1e3, "serial_ms_per_step": t32_serial * 1e3,
        "geometry_pairs_per_s": G / t32,
        "tri_pairs_executed_per_step": {"fp32": fp32_tests, "fp64": fp64_tests},
        "tri_pairs_executed_per_s": {"fp32": fp32_tests / t32, "fp64": fp64_tests / t32},
        "all_pairs_equivalent_per_s": allpairs / t32,
        "tiles": {"distance": tune["distance"]["best"], "intersects": tune["intersects"]["best"]},
        "autotune_ms": {k: {str(t): round(v, 4) for t, v in r["ms"].items()} for k, r in tune.items()},
        "result": {"hits_distance": int(h32.sum()), "hits_intersects": int(hi32.sum()),
                   "flags_equal": bool(np.array_equal(h32, hi32)),
                   "dist_row0": float(d32[0]), "hit_row0": bool(h32[0])},
        "stats_distance": {k: v for k, v in sd32.items()
                           if k not in ("ms_phase", "ms_kernel", "n_kernel", "ms_total")},
        "plain_fp64": fp64,
    }
    if headline:
        # the same step as eager calls (one host synchronisation per call)
        for _ in range(args.warmup):
            ctx.distance(ba, bb, order="learned", ranker=weights)
            ctx.intersects(ba, bb)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(args.steps):
            ctx.distance(ba, bb, order="learned", ranker=weights)
            ctx.intersects(ba, bb)
        res["eager_ms_per_step"] = (time.perf_counter() - t0) / args.steps * 1e3
        # learned vs box-bound vs no seed order: time per distance call and
        # tile pairs evaluated (the ranking comparison; identical bits)
        res["orders_distance"] = time_orders(ctx, ba, bb, weights, args,
                                             ("fp32", "fp64") if args.orders else ("fp32",))
        # live per-kernel timing (HIP events on the call's stream), eager calls
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
            roof = roofline_for(dom, [sd, si], kms[dom], kn[dom], name,
                                sum(len(a[0]) for a in A) + sum(len(b[0]) for b in B))
        else:
            roof = pairs_roofline(sd, sd["ms_kernel"]["pairs"], max(sd["n_kernel"]["pairs"], 1), name)
        roof["dominant_by_time"] = dom
        roof["kernel_ms_per_step"] = {k: round(v, 4) for k, v in kms.items()}
        res["roofline"] = roof
        res["roofline_pairs_fp32"] = pairs_roofline(sd, sd["ms_kernel"]["pairs"],
                                                    sd["n_kernel"]["pairs"], name)
        res["phase_ms"] = {f"{t}.{k}": round(v, 4) for (t, k), v in phase.items()}
    res["_d32"], res["_h32"] = d32, h32
    return res


def measure_segments(ctx, args):
    """The paper's segment workload: 5 M drill-hole segments against one
    500-face ore body; a step is sd3_segments distance, intersects and the
    distance-threshold filter (r = 2) over every segment."""
    import numpy as np
    import torch
    from paper_1808_09571_amd import sd3, synth
    seg, body = synth.config_drillholes()
    sg = torch.from_numpy(seg).to("cuda:0")
    mb = sd3.Batch.from_packed(synth.pack([body]), "cuda:0")
    r = 2.0

    def step():
        ctx.segments("distance", sg, mb)
        ctx.segments("intersects", sg, mb)
        ctx.segments("within", sg, mb, r=r)

    for _ in range(max(args.warmup, 1)):
        step()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        step()
    torch.cuda.synchronize()
    t = (time.perf_counter() - t0) / args.steps
    (d, h), sd = ctx.segments("distance", sg, mb, stats=True)
    w = ctx.segments("within", sg, mb, r=r)
    per_op = {}
    for op in ("distance", "intersects", "within"):
        for _ in range(2):
            ctx.segments(op, sg, mb, r=r)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(args.steps):
            ctx.segments(op, sg, mb, r=r)
        torch.cuda.synchronize()
        per_op[op] = (time.perf_counter() - t0) / args.steps * 1e3
    d, h, w = d.cpu().numpy(), h.cpu().numpy().astype(bool), w.cpu().numpy().astype(bool)
    n = seg.shape[0]
    return {"workload": f"{n} drill-hole segments (100,000 holes x 50) vs one 500-face ore body",
            "segments": n, "faces": int(body[1].shape[0]), "ms_per_step": t * 1e3,
            "ms_per_operator": per_op, "segments_per_s": 3 * n / t,
            "distance_segments_per_s": n / (per_op["distance"] * 1e-3),
            "segment_triangle_tests_per_step": {"box": sd["tri_pairs_boxed"], "fp64": sd["tri_pairs_fp64"]},
            "hits": int(h.sum()), "within_r": int(w.sum()), "r": r,
            "consistent": bool(np.array_equal(w, d <= r) and np.array_equal(h, d == 0.0)),
            "paper_context": "3D distance of 5 M segments vs a 500-face solid: 0.685 s end to end "
                             "on a V100 inside PostgreSQL (Sec. 4); a different system, not a target"}


def measure_volume(ctx, A, B, args):
    """sd3_volume over every mesh of the workload (both sides' rows)."""
    import torch
    from paper_1808_09571_amd import sd3, synth
    meshes = list(A) + list(B)
    bt = sd3.Batch.from_packed(synth.pack(meshes), "cuda:0")
    for _ in range(max(args.warmup, 1)):
        ctx.volume(bt)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        v = ctx.volume(bt)
    torch.cuda.synchronize()
    t = (time.perf_counter() - t0) / args.steps
    ntri = sum(len(m[1]) for m in meshes)
    per = ntri * VOL_BYTES_TRI
    ach = per / t / 1e9
    return {"workload": f"volume of {len(meshes)} meshes ({ntri} triangles)", "ms_per_call": t * 1e3,
            "meshes_per_s": len(meshes) / t, "triangles_per_s": ntri / t,
            "roofline": {"bound": "hbm", "achieved": ach, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                         "frac": ach / HBM_PEAK_GBS, "traffic": None,
                         "per_unit": f"{VOL_BYTES_TRI} B per triangle (indices 12, three vertices 72), "
                                     "wall time of the call (validation included)"},
            "sum_volume": float(v.sum().item()),
            "paper_context": "3D volume of a 500-face solid: 0.91 s end to end on a V100 (Sec. 4)"}


def cpu_baseline_rows(A, B, threads, budget_s):
    """The FP64 oracle (exact pruned mode, distance and intersects of a row in
    one run) on whole rows taken in order until about ``budget_s`` of work;
    a single-row workload repeats its row.  Returns the rate in rows per
    second and the sampled rows' results."""
    import oracle
    t_all, runs, rows = 0.0, 0, []
    while t_all < budget_s and runs < 400:
        g = runs % len(A)
        t0 = time.perf_counter()
        d, h, _ = oracle.mesh(A[g], B[g], mode="pruned", threads=threads)
        t_all += time.perf_counter() - t0
        runs += 1
        if len(rows) < len(A) and (not rows or rows[-1][0] != g):
            rows.append((g, d, h))
    sample = (f"{runs} oracle run(s) over rows 0..{min(runs, len(A)) - 1} of the same workload, "
              f"exact pruned mode, {t_all:.1f} s")
    return runs / t_all, sample, rows


def cpu_baseline(A, B, d32, h32):
    import oracle
    threads = oracle.default_threads()
    v_all, s_all, rows = cpu_baseline_rows(A, B, threads, CPU_BUDGET_S)
    v_one, s_one, rows1 = cpu_baseline_rows(A, B, 1, CPU_BUDGET_S)
    ok = all(h == bool(h32[g]) and (h or abs(d - d32[g]) <= 1e-12 * d) for g, d, h in rows + rows1)

    def rel_err(d, x):
        if d == 0.0 or d == float("inf"):
            return 0.0 if x == d else float("inf")
        return abs(d - x) / d

    errs = [rel_err(d, float(d32[g])) for g, d, h in rows]
    return {"value": v_all, "unit": "geometry-pairs/s (distance + intersects per row)",
            "cores": threads, "kind": "oracle", "sample": s_all, "cpu_model": cpu_model(),
            "one_core": {"value": v_one, "cores": 1, "sample": s_one},
            "matches_gpu": bool(ok), "max_rel_err_vs_oracle": max(errs) if errs else None,
            "rows_checked": len({g for g, _, _ in rows + rows1})}


# ---------------------------------------------------------------------------
# profile summaries (rocprofv3 output -> profiles/)
# ---------------------------------------------------------------------------
def _csv_rows(pattern):
    out = []
    for f in sorted(glob.glob(pattern, recursive=True)):
        with open(f, newline="") as fh:
            out.extend(csv.DictReader(fh))
    return out


def _short(name):
    n = name.split("(")[0]
    return n.replace("void ", "").strip()


def summarize(args):
    """Print a Markdown (stats, sq) or JSON (pmc) summary of rocprofv3 CSV
    output found under args.summarize."""
    d = args.summarize
    if args.kind == "stats":
        rows = _csv_rows(os.path.join(d, "**", "*kernel_stats.csv"))
        rows.sort(key=lambda r: -float(r["TotalDurationNs"]))
        print("| Kernel | Calls | Total ms | Avg us | % |\n|---|---:|---:|---:|---:|")
        for r in rows:
            print(f"| `{_short(r['Name'])}` | {r['Calls']} | {float(r['TotalDurationNs']) / 1e6:.3f} | "
                  f"{float(r['AverageNs']) / 1e3:.2f} | {float(r['Percentage']):.2f} |")
        return
    if args.kind == "sq":
        rows = _csv_rows(os.path.join(d, "**", "*counter_collection.csv"))
        acc = {}
        for r in rows:
            k = _short(r["Kernel_Name"])
            e = acc.setdefault(k, {"dispatches": set()})
            e["dispatches"].add(r["Dispatch_Id"])
            e[r["Counter_Name"]] = e.get(r["Counter_Name"], 0.0) + float(r["Counter_Value"])
        names = sorted({c for e in acc.values() for c in e if c != "dispatches"})
        print("| Kernel | Dispatches | " + " | ".join(names) + " (per dispatch) |")
        print("|---|---:|" + "---:|" * len(names))
        for k, e in sorted(acc.items(), key=lambda kv: -kv[1].get("SQ_WAVE_CYCLES", 0.0)):
            n = len(e["dispatches"])
            print(f"| `{k}` | {n} | " + " | ".join(f"{e.get(c, 0.0) / n:.3g}" for c in names) + " |")
        return
    # pmc: FETCH_SIZE and WRITE_SIZE runs of the workload and of the copy.
    # Keys: "k_scatter" (every radix pass), "k_tiles<TK>", "k_pairs<fp32|fp64,
    # distance|intersects,TK> main pass" (dispatches above a tenth of the
    # kernel's largest count: the seed passes, which evaluate at most one tile
    # pair per row, fall below), other kernels by name.
    def traffic_key(name):
        n = _short(name).replace("sd3::", "")
        if n.startswith("k_scatter"):
            return "k_scatter"
        if n.startswith("k_pairs<"):
            p, m, t = [x.strip() for x in n[len("k_pairs<"):-1].split(",")]
            return (f"k_pairs<{'fp32' if p == '0' else 'fp64'},{'distance' if m == '0' else 'intersects'},"
                    f"{t}> main pass")
        return n

    def per_kernel(counter, base):
        rows = _csv_rows(os.path.join(base + "_" + counter, "**", "*counter_collection.csv"))
        disp = {}
        for r in rows:
            if r["Counter_Name"] != counter:
                continue
            k = traffic_key(r["Kernel_Name"])
            e = disp.setdefault(k, {})
            e[r["Dispatch_Id"]] = e.get(r["Dispatch_Id"], 0.0) + float(r["Counter_Value"])
        out = {}
        for k, e in disp.items():
            vals = list(e.values())
            if k.endswith("main pass"):
                top = max(vals)
                vals = [v for v in vals if v >= 0.1 * top]
            out[k] = (sum(vals) / len(vals), len(vals))
        return out

    fetch, write = per_kernel("FETCH_SIZE", d), per_kernel("WRITE_SIZE", d)
    calib = {"copy_bytes": COPY_BYTES, "fetch_factor": 1.0, "write_factor": 1.0}
    if args.calib:
        cf, cw = per_kernel("FETCH_SIZE", args.calib), per_kernel("WRITE_SIZE", args.calib)
        fk = max(cf.values(), key=lambda x: x[0])[0] if cf else 0.0
        wk = max(cw.values(), key=lambda x: x[0])[0] if cw else 0.0
        calib.update({"fetch_size_kib": fk, "write_size_kib": wk,
                      "fetch_factor": COPY_BYTES / (fk * 1024) if fk else 1.0,
                      "write_factor": COPY_BYTES / (wk * 1024) if wk else 1.0})
    kernels = {}
    for k in sorted(set(fetch) | set(write)):
        fb = fetch.get(k, (0.0, 0))[0] * 1024 * calib["fetch_factor"]
        wb = write.get(k, (0.0, 0))[0] * 1024 * calib["write_factor"]
        kernels[k] = {"fetch_bytes_per_launch": fb, "write_bytes_per_launch": wb,
                      "bytes_per_launch": fb + wb,
                      "launches_sampled": max(fetch.get(k, (0, 0))[1], write.get(k, (0, 0))[1])}
    print(json.dumps({"kernel_source_sha256_16": kernel_source_hash(), "calibration": calib,
                      "workload": args.workload, "commands": args.cmd, "kernels": kernels}, indent=1))


def main():
    args = parse()
    if args.summarize:
        summarize(args)
        return
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (got --gpus {args.gpus}); multi-GPU is not part "
              "of this build", file=sys.stderr)
        sys.exit(2)
    if args.copy_calibration:
        copy_calibration()
        return
    from paper_1808_09571_amd import ranker, sd3

    ctx = sd3.Context(0)
    weights = ranker.load(device="cuda:0")
    print(f"[bench] generating {args.workload}", file=sys.stderr, flush=True)
    A, B = make_workload(args.workload)
    print(f"[bench] measuring {args.workload}", file=sys.stderr, flush=True)
    head = measure(args.workload, A, B, ctx, weights, args, headline=True)
    d32, h32 = head.pop("_d32"), head.pop("_h32")
    extras = {}
    for name in [x for x in args.extras.split(",") if x and x != args.workload]:
        print(f"[bench] generating and measuring {name}", file=sys.stderr, flush=True)
        if name == "segments":
            extras[name] = measure_segments(ctx, args)
            continue
        if name == "volume":
            extras[name] = measure_volume(ctx, A, B, args)
            continue
        Ae, Be = make_workload(name)
        r = measure(name, Ae, Be, ctx, weights, args, headline=False)
        r.pop("_d32"), r.pop("_h32")
        extras[name] = r
        del Ae, Be
    t32 = head["ms_per_step"] * 1e-3
    line = {
        "metric": METRIC,
        "value": head["geometry_pairs_per_s"],
        "unit": "geometry-pairs/s (distance + intersects per row, inputs resident in HBM)",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": head["ms_per_step"], "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f32 (bulk) + f64 (rescue, result)", "data": "synthetic",
        "config": {"workload": WORKLOADS[args.workload], "rows": head["rows"],
                   "triangles_a": head["triangles_a"], "triangles_b": head["triangles_b"],
                   "order": "learned", "ranker": "ranker_weights.npy",
                   "launch": "HIP graph per operator; distance and intersects on two streams with hardware queues of their own",
                   "tiles": head["tiles"]},
    }
    for k in ("tri_pairs_executed_per_step", "tri_pairs_executed_per_s", "all_pairs_equivalent_per_s",
              "serial_ms_per_step", "eager_ms_per_step", "plain_fp64", "orders_distance",
              "roofline", "roofline_pairs_fp32", "result", "stats_distance", "phase_ms",
              "autotune_ms"):
        line[k] = head.get(k)
    line["extras"] = extras
    if not args.no_cpu_baseline:
        print("[bench] CPU oracle", file=sys.stderr, flush=True)
        line["cpu_baseline"] = cpu_baseline(A, B, d32, h32)
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
