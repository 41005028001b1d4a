"""GPU tests of the pre-cull of large calls.

On a large sort (more than 2^22 triangles) of more than 64 rows, tiles hold
only the triangles that can matter: for intersects those whose boxes meet the
other side's row box (a triangle whose three vertices lie beyond one plane of
that box cannot meet the other side), for distance those within the row's
cull distance of it (an upper bound of the row distance from sampled corners,
plus a margin).  A triangle can cross the box with every vertex outside it,
on different sides; it must be kept.  Flags and distance bits must equal
those of calls of at most 64 rows (which cull nothing), and the oracle's.
"""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu

import oracle
from paper_1808_09571_amd import sd3, synth


@pytest.fixture(scope="module")
def ctx():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return sd3.Context(0)


def _tri(*verts):
    return np.array(verts, dtype=np.float64), np.array([[0, 1, 2]], dtype=np.int32)


def _flat_grid(n, size, z):
    xs = np.linspace(0.0, size, n + 1)
    X, Y = np.meshgrid(xs, xs, indexing="ij")
    xyz = np.stack([X.reshape(-1), Y.reshape(-1), np.full(X.size, z)], axis=1)
    return xyz, synth.grid_triangles(n, n)


def _rows():
    unit = synth.icosphere(3)  # box [-1, 1]^3
    small = [
        # every vertex outside the box, on different sides; crosses the sphere
        (_tri((-10.0, -10.0, 0.0), (10.0, -10.0, 0.0), (0.0, 10.0, 0.0)), unit, True),
        (_tri((-10.0, 0.0, -10.0), (10.0, 0.0, -10.0), (0.0, 0.0, 10.0)), unit, True),
        # the same triangles beyond one plane of the box: no contact
        (_tri((-10.0, -10.0, 5.0), (10.0, -10.0, 5.0), (0.0, 10.0, 5.0)), unit, False),
        (_tri((-10.0, 3.0, -10.0), (10.0, 3.0, -10.0), (0.0, 3.0, 10.0)), unit, False),
        # crosses the box but passes beside the sphere (box corner region)
        (_tri((0.9, 0.9, -5.0), (0.9, 0.9, 5.0), (5.0, 5.0, 0.0)), unit, False),
    ]
    rows = small * 13
    rows += [
        # a 4.5M-triangle grid makes the call a large sort; a sphere dips
        # through it
        (_flat_grid(1500, 100.0, 0.0), synth.icosphere(3, center=(50.0, 50.0, 0.5)), True),
        # spheres above grids: most grid triangles lie beyond the cull distance
        (_flat_grid(200, 100.0, 0.0), synth.icosphere(3, center=(50.0, 50.0, 3.0)), False),
        (_flat_grid(8, 100.0, 0.0), synth.icosphere(3, center=(20.0, 70.0, 3.0)), False),
    ]
    return rows


def test_pre_cull_keeps_what_matters(ctx):
    rows = _rows()
    A = [r[0] for r in rows]
    B = [r[1] for r in rows]
    G = len(rows)
    assert G > 64 and sum(len(a[1]) + len(b[1]) for a, b in zip(A, B)) > (1 << 22)
    want = np.array([r[2] for r in rows])
    ba = sd3.Batch.from_packed(synth.pack(A), "cuda:0")
    bb = sd3.Batch.from_packed(synth.pack(B), "cuda:0")
    # calls of at most 64 rows cull nothing: the reference bits
    ref_d, ref_h = [], []
    for r0 in range(0, G, 64):
        ca = sd3.Batch.from_packed(synth.pack(A[r0:r0 + 64]), "cuda:0")
        cb = sd3.Batch.from_packed(synth.pack(B[r0:r0 + 64]), "cuda:0")
        d, h = ctx.distance(ca, cb)
        ref_d.append(d.cpu().numpy().view(np.int64).copy())
        ref_h.append(h.cpu().numpy().astype(bool))
    ref_d, ref_h = np.concatenate(ref_d), np.concatenate(ref_h)
    assert np.array_equal(ref_h, want), ref_h
    for prec in ("fp32", "fp64"):
        for tile in sd3.TILES:
            d, h = ctx.distance(ba, bb, precision=prec, tile=tile)
            assert np.array_equal(d.cpu().numpy().view(np.int64), ref_d), (prec, tile)
            assert np.array_equal(h.cpu().numpy().astype(bool), want), (prec, tile)
            hi = ctx.intersects(ba, bb, precision=prec, tile=tile).cpu().numpy().astype(bool)
            assert np.array_equal(hi, want), (prec, tile, hi)
    # the small rows and the small grid row against the oracle
    dist = ref_d.view(np.float64)
    for r in (0, 1, 2, 3, 4, G - 1):
        d_o, h_o, _ = oracle.mesh(A[r], B[r], mode="pruned")
        assert bool(h_o) == bool(want[r]), r
        if not h_o:
            assert abs(dist[r] - d_o) <= 1e-12 * d_o, (r, dist[r], d_o)
