"""Learned tile-pair ranking for the seed round of sd3_distance.

The ranker is a 10 -> 64 -> 64 -> 64 -> 1 ReLU MLP (FP32) that predicts, from
a candidate tile pair's box features, the log of the smallest distance between
its triangles.  sd3_distance (order="learned") evaluates each row's
best-ranked tile pair first, so that a tight upper bound prunes the remaining
candidates; the plain box-bound order is the fallback, and results never
depend on the order.

Training data are logged from the method's own runs (one record per dequeued
tile pair: features and outcome); training runs on the GPU through the
library's forward / backward / Adam kernels (sd3_mlp_loss_grad, sd3_adam_step).

    python -m paper_1808_09571_amd.ranker --out paper_1808_09571_amd/ranker_weights.npy
"""
from __future__ import annotations

import argparse
import json
import os
import time

import numpy as np

from . import sd3, synth

HERE = os.path.dirname(os.path.abspath(__file__))
WEIGHTS = os.path.join(HERE, "ranker_weights.npy")


def init_params(seed: int = 0) -> np.ndarray:
    """He-normal weights, zero biases, in the packed layout of include/sd3.h."""
    g = np.random.Generator(np.random.PCG64(seed))
    H, N = sd3.MLP_NPARAM, 64
    parts = [g.normal(0, np.sqrt(2.0 / 10), (64, 10)), np.zeros(64),
             g.normal(0, np.sqrt(2.0 / 64), (64, 64)), np.zeros(64),
             g.normal(0, np.sqrt(2.0 / 64), (64, 64)), np.zeros(64),
             g.normal(0, np.sqrt(1.0 / 64), 64), np.zeros(1)]
    p = np.concatenate([x.reshape(-1) for x in parts]).astype(np.float32)
    assert p.size == H and N == 64
    return p


def to_batches(pairs, device="cuda:0"):
    """[(A_meshes, B_meshes), ...] -> [(Batch, Batch)] on the device."""
    out = []
    for A, B in pairs:
        out.append((sd3.Batch.from_packed(synth.pack(A), device),
                    sd3.Batch.from_packed(synth.pack(B), device)))
    return out


def collect(ctx, batches, cap=1 << 20, precision="fp32"):
    """Run sd3_distance without a seed round and gather the logged records.
    Returns (features [n, 10], targets [n]) as device float32 tensors."""
    import torch
    xs, ts = [], []
    for ba, bb in batches:
        buf = torch.zeros((cap, sd3.LOG_STRIDE), dtype=torch.float32, device=ba.xyz.device)
        _, _, st = ctx.distance(ba, bb, precision=precision, order="none", stats=True, log=buf)
        n = min(int(st["logged"]), cap)
        xs.append(buf[:n, :sd3.MLP_NIN].clone())
        ts.append(buf[:n, sd3.MLP_NIN].clone())
    return torch.cat(xs), torch.cat(ts)


def train(ctx, X, t, steps=1500, batch=4096, lr=2e-3, seed=0, verbose=False):
    """Minibatch Adam on the MSE of the predicted log distance.  Returns the
    parameters (device float32) and the loss history."""
    import torch
    r = sd3.Ranker(ctx)
    dev = X.device
    p = torch.from_numpy(init_params(seed)).to(dev)
    m = torch.zeros_like(p)
    v = torch.zeros_like(p)
    gen = torch.Generator(device=dev)
    gen.manual_seed(seed)
    hist = []
    n = X.shape[0]
    for step in range(1, steps + 1):
        idx = torch.randint(0, n, (min(batch, n),), device=dev, generator=gen)
        loss, grad = r.loss_grad(p, X[idx].contiguous(), t[idx].contiguous())
        r.adam(p, grad, m, v, step, lr=lr)
        if step % 100 == 0 or step == 1:
            hist.append((step, float(loss.item())))
            if verbose:
                print(f"step {step} loss {hist[-1][1]:.4f}", flush=True)
    return p, hist


def save(params, path=WEIGHTS):
    np.save(path, params.detach().cpu().numpy().astype(np.float32), allow_pickle=False)


def load(path=WEIGHTS, device="cuda:0"):
    import torch
    p = np.load(path, allow_pickle=False).astype(np.float32)
    assert p.shape == (sd3.MLP_NPARAM,)
    return torch.from_numpy(p).to(device)


def training_pairs():
    """TIN training workloads, disjoint from the benchmark's seeds: TIN pairs
    with other noise seeds and clearances."""
    pairs = []
    for k, (gap, n) in enumerate([(0.01, 256), (0.05, 256), (0.002, 256), (0.01, 384)]):
        A, B = synth.config_tin_pair(n=n, extent=1000.0 * n / 512, gap=gap,
                                     seeds=(31 + 2 * k, 32 + 2 * k))
        pairs.append(([A], [B]))
    return pairs


def batch_training_pairs(seed):
    """One chunk of 128 rows of the drill-hole / ore-body batch distribution
    (the benchmark's batch uses seed 3; training seeds start at 1000)."""
    return synth.config_tube_blob_batch(rows=128, seed=seed)


def collect_records(ctx, records, verbose=False):
    """Logged (features, target) records from the TIN training pairs and from
    batch-distribution chunks of seeds 1000, 1001, ... until ``records``
    records are gathered.  Returns device tensors and the seeds used."""
    import torch
    xs, ts = [], []
    X, t = collect(ctx, to_batches(training_pairs()))
    xs.append(X)
    ts.append(t)
    n, seed = X.shape[0], 1000
    while n < records:
        A, B = batch_training_pairs(seed)
        X, t = collect(ctx, to_batches([(A, B)]))
        xs.append(X)
        ts.append(t)
        n += X.shape[0]
        if verbose:
            print(f"seed {seed}: {n} records", flush=True)
        seed += 1
    return torch.cat(xs), torch.cat(ts), list(range(1000, seed))


def evaluate(ctx, ba, bb, params, precision="fp32"):
    """Tile pairs evaluated and results under box-bound and learned seeding."""
    res = {}
    for order in ("none", "bound", "learned"):
        d, h, st = ctx.distance(ba, bb, precision=precision, order=order, stats=True,
                                ranker=params if order == "learned" else None)
        res[order] = {"tile_pairs_evaluated": st["tile_pairs_evaluated"],
                      "tri_pairs_fp32": st["tri_pairs_fp32"],
                      "dist": d.cpu().numpy(), "hit": h.cpu().numpy()}
    return res


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--out", default=WEIGHTS)
    ap.add_argument("--steps", type=int, default=4000)
    ap.add_argument("--records", type=int, default=1_000_000,
                    help="logged tile-pair outcomes to train on (TIN pairs + batch chunks)")
    ap.add_argument("--report", default=None, help="write a JSON summary here")
    args = ap.parse_args()
    ctx = sd3.Context(0)
    t0 = time.time()
    X, t, seeds = collect_records(ctx, args.records, verbose=True)
    t1 = time.time()
    params, hist = train(ctx, X, t, steps=args.steps, verbose=True)
    t2 = time.time()
    save(params, args.out)
    heldout = {}
    same = True
    A, B = synth.config_tin_pair()
    held = [("tin512_seeds_1_2", [A], [B]),
            ("batch_seed3_rows_0_511",) + tuple(synth.config_tube_blob_batch(rows=512, seed=3))]
    for name, HA, HB in held:
        ba, bb = to_batches([(HA, HB)])[0]
        ev = evaluate(ctx, ba, bb, params)
        same = same and all(np.array_equal(ev[o]["dist"].view(np.int64), ev["none"]["dist"].view(np.int64))
                            for o in ev)
        heldout[name] = {o: ev[o]["tile_pairs_evaluated"] for o in ev}
    summary = {"records": int(X.shape[0]), "batch_training_seeds": [seeds[0], seeds[-1]] if seeds else [],
               "collect_s": t1 - t0, "train_s": t2 - t1, "steps": args.steps,
               "loss_first": hist[0][1], "loss_last": hist[-1][1],
               "heldout_tile_pairs_evaluated": heldout, "identical_results": bool(same)}
    print(json.dumps(summary), flush=True)
    if args.report:
        with open(args.report, "w") as f:
            json.dump(summary, f)


if __name__ == "__main__":
    main()
