"""GPU tests of batched execution: tile sizes, queue passes, HIP-graph replay
and the tile-size autotuner (one launch over all rows' tile pairs).

Every configuration must return what the FP64 oracle returns (flags exact,
distances within 1e-12 relative) and the same bits as every other
configuration: tile size, queue capacity and graph replay change how the work
is scheduled, never which FP64 pair values reach the minimum.
"""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu

from paper_1808_09571_amd import sd3, synth
from test_gpu_parity import _check, _oracle_rows


@pytest.fixture(scope="module")
def ctx():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return sd3.Context(0)


def _dev(A, B):
    return (sd3.Batch.from_packed(synth.pack(A), "cuda:0"),
            sd3.Batch.from_packed(synth.pack(B), "cuda:0"))


def _bits(d):
    return d.cpu().numpy().view(np.int64).copy()


def _workloads():
    out = {}
    A, B = [], []
    for seed in range(8):
        a, b = synth.config_icospheres(seed)
        A.append(a)
        B.append(b)
    out["icospheres"] = (A, B)
    sizes = [(1, 1), (31, 33), (32, 32), (63, 65), (64, 64), (127, 129), (128, 128), (200, 7),
             (0, 5), (5, 0), (0, 0), (257, 1)]
    A, B = [], []
    for k, (na, nb) in enumerate(sizes):
        A.append(synth.random_triangle_soup(na, 10 + k, scale=2.0))
        B.append(synth.random_triangle_soup(nb, 50 + k, scale=2.0, center=(1.5, 0.5, 0)))
    out["ragged"] = (A, B)
    out["tube_blob"] = synth.config_tube_blob_batch(rows=12, seed=21, tube_tri=(200, 1500),
                                                    blob_tri=(1000, 5000), aim_range=1.5)
    return out


WORK = None


def _work():
    global WORK
    if WORK is None:
        WORK = _workloads()
    return WORK


@pytest.mark.parametrize("name", ["icospheres", "ragged", "tube_blob"])
def test_tile_sizes_agree_with_oracle_and_each_other(ctx, name):
    A, B = _work()[name]
    d_o, h_o = _oracle_rows(A, B)
    ba, bb = _dev(A, B)
    ref = None
    for prec in ("fp32", "fp64"):
        for tile in sd3.TILES:
            d, h, st = ctx.distance(ba, bb, precision=prec, tile=tile, stats=True)
            hi = ctx.intersects(ba, bb, precision=prec, tile=tile)
            assert st["tile"] == tile
            _check(A, B, d.cpu().numpy(), h.cpu().numpy(), d_o, h_o)
            assert np.array_equal(hi.cpu().numpy().astype(bool), h_o)
            got = (_bits(d), h.cpu().numpy().copy())
            if ref is None:
                ref = got
            assert np.array_equal(got[0], ref[0]) and np.array_equal(got[1], ref[1])


def test_queue_passes_agree_with_single_pass(ctx):
    """A queue too small for all candidate tile pairs: the work items run in
    several passes (each with its own seed round) and give the same bits."""
    A, B = synth.config_tin_pair(n=96, extent=187.5, amplitude=20.0, gap=0.01, seeds=(61, 62))
    ba, bb = _dev([A], [B])
    for order in ("bound", "none"):
        d1, h1, s1 = ctx.distance(ba, bb, order=order, stats=True)
        dm, hm, sm = ctx.distance(ba, bb, order=order, stats=True, queue_cap=1)
        assert s1["queue_passes"] == 1 and sm["queue_passes"] > 2
        assert np.array_equal(_bits(d1), _bits(dm)) and np.array_equal(h1.cpu(), hm.cpu())
    hi1 = ctx.intersects(ba, bb)
    him, st = ctx.intersects(ba, bb, queue_cap=1, stats=True)
    assert st["queue_passes"] > 2 and np.array_equal(hi1.cpu(), him.cpu())
    # the tiles of one pass-split call agree with the oracle's pruned search
    import oracle
    d_o, h_o, _ = oracle.mesh(A, B, mode="pruned")
    assert not h_o and abs(float(dm.cpu()[0]) - d_o) <= 1e-12 * d_o


def test_graph_replays_match_eager_calls(ctx):
    import torch
    A, B = _work()["tube_blob"]
    d_o, h_o = _oracle_rows(A, B)
    ba, bb = _dev(A, B)
    d_e, h_e = ctx.distance(ba, bb)
    hi_e = ctx.intersects(ba, bb)
    _check(A, B, d_e.cpu().numpy(), h_e.cpu().numpy(), d_o, h_o)
    gd = ctx.graph("distance", ba, bb)
    gi = ctx.graph("intersects", ba, bb, precision="fp64")
    for r in range(3):
        gd.launch()
        gi.launch()
        st = gd.result(stats=True)
        gi.result()
        assert np.array_equal(_bits(gd.dist), _bits(d_e)), r
        assert np.array_equal(gd.hit.cpu(), h_e.cpu()) and np.array_equal(gi.hit.cpu(), hi_e.cpu())
        assert st["tile_pairs_evaluated"] > 0
        # eager work of the program between replays
        d64, _ = ctx.distance(ba, bb, precision="fp64")
        torch.cuda.synchronize()
        assert np.array_equal(_bits(d64), _bits(d_e))
    # the contents may change between replays: move B by a power of two
    with torch.no_grad():
        bb.xyz += 0.25
    gd.launch()
    gd.result()
    d_m, h_m = ctx.distance(ba, bb)
    assert np.array_equal(_bits(gd.dist), _bits(d_m)) and np.array_equal(gd.hit.cpu(), h_m.cpu())
    assert not np.array_equal(_bits(d_m), _bits(d_e))
    gd.close()
    gi.close()


def test_graphs_replayed_concurrently_on_two_streams(ctx):
    """Each graph has its own workspace: a distance graph and an intersects
    graph replayed on two streams at once give the eager results, step after
    step (replays of one graph stay in order on its stream)."""
    import torch
    A, B = _work()["tube_blob"]
    ba, bb = _dev(A, B)
    d_e, h_e = ctx.distance(ba, bb, precision="fp64")
    hi_e = ctx.intersects(ba, bb)
    gd = ctx.graph("distance", ba, bb)
    gi = ctx.graph("intersects", ba, bb)
    side = torch.cuda.Stream()
    for step in range(4):
        for _ in range(3):
            gd.launch()
            with torch.cuda.stream(side):
                gi.launch()
        torch.cuda.synchronize()
        gd.result()
        gi.result()
        assert np.array_equal(_bits(gd.dist), _bits(d_e)), step
        assert np.array_equal(gd.hit.cpu(), h_e.cpu()) and np.array_equal(gi.hit.cpu(), hi_e.cpu())
        # eager work of the program between the steps
        d2, _ = ctx.distance(ba, bb)
        torch.cuda.synchronize()
        assert np.array_equal(_bits(d2), _bits(d_e))
    gd.close()
    gi.close()


def test_graph_replay_reports_invalid_contents(ctx):
    """A replay over contents that no longer validate leaves the outputs
    untouched and reports the error; after repair it runs again.  (Indices
    are clamped into their row before use, so the kernels stay in bounds.)"""
    A, B = _work()["icospheres"]
    ba, bb = _dev(A, B)
    g = ctx.graph("distance", ba, bb)
    g.launch()
    g.result()
    before = _bits(g.dist)
    saved = int(bb.tri[5].item())
    bb.tri[5] = 1 << 20
    g.launch()
    with pytest.raises(sd3.SD3Error) as e:
        g.result()
    assert e.value.name == "SD3_E_INDEX_RANGE"
    assert np.array_equal(_bits(g.dist), before)
    bb.tri[5] = saved
    g.launch()
    g.result()
    assert np.array_equal(_bits(g.dist), before)
    g.close()


def test_graph_rejects_host_batches(ctx):
    A, B = _work()["icospheres"]
    ha, hb = sd3.Batch.from_packed(synth.pack(A)), sd3.Batch.from_packed(synth.pack(B))
    with pytest.raises(AssertionError):
        ctx.graph("distance", ha, hb)


def test_autotune_choice_is_used_and_changes_nothing(ctx):
    A, B = _work()["tube_blob"]
    ba, bb = _dev(A, B)
    d0, h0 = ctx.distance(ba, bb, tile=64)
    r = ctx.autotune("distance", ba, bb, reps=2)
    assert r["best"] in sd3.TILES and set(r["ms"]) == set(sd3.TILES)
    assert all(v > 0 for v in r["ms"].values())
    d1, h1, st = ctx.distance(ba, bb, stats=True)
    assert st["tile"] == r["best"]
    assert np.array_equal(_bits(d0), _bits(d1)) and np.array_equal(h0.cpu(), h1.cpu())
    # another kind of workload still uses the default
    a2, b2 = synth.config_icospheres(3)
    ba2, bb2 = _dev([a2], [b2])
    _, _, st2 = ctx.distance(ba2, bb2, stats=True)
    assert st2["tile"] == 64
    ri = ctx.autotune("intersects", ba, bb, reps=1)
    hi, sti = ctx.intersects(ba, bb, stats=True)
    assert sti["tile"] == ri["best"] and np.array_equal(hi.cpu(), h0.cpu())
