"""GPU parity of solid semantics (opts.semantics = "solid"): rows are the
solids their closed meshes bound (the paper's ore bodies, Sec. 4), so nested
meshes meet at distance 0.  Checked against the oracle's solid reading
(surface test plus the winding number of one vertex per side), with the
surface results unchanged wherever the surfaces meet or the solids are
disjoint.  Integer-coordinate cubes make the first ray direction (+z) pass
through edges, so the retry with the next direction runs."""
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


def _rows():
    g = np.random.default_rng(4)
    A, B = [], []
    outer = synth.icosphere(3)
    for k in range(12):
        r = g.uniform(0.2, 0.6)
        c = g.uniform(-0.25, 0.25, size=3) if k % 3 else g.uniform(1.5, 2.5, size=3)
        A.append(synth.icosphere(2, radius=r, center=tuple(c)))
        B.append(outer)
    # cubes on the integer grid: nested, disjoint, touching, overlapping
    for lo, size in (((1.0, 1.0, 1.0), 1.0), ((5.0, 0.0, 0.0), 1.0), ((4.0, 1.0, 1.0), 1.0),
                     ((2.0, 2.0, 2.0), 2.0)):
        A.append(synth.cube(lo, size))
        B.append(synth.cube((0.0, 0.0, 0.0), 4.0))
    # blobs with short drill-hole tubes, some inside
    for k in range(8):
        bl = synth.blob(3000, 5.0, (0.0, 0.0, 0.0), 40 + k)
        path = synth.polyline(6, g, (0.0, 0.0, -1.0 if k % 2 else 9.0), (0.0, 0.0, 1.0))
        A.append(synth.tube(path, radius=0.05))
        B.append(bl)
    return A, B


@pytest.mark.parametrize("device", [True, False])
def test_solid_rows_against_oracle(ctx, device):
    A, B = _rows()
    want = [oracle.mesh_solid(a, b, mode="all") for a, b in zip(A, B)]
    d_w = np.array([w[0] for w in want])
    h_w = np.array([w[1] for w in want])
    assert h_w.sum() >= 8 and (~h_w).sum() >= 6  # both kinds present
    dev = "cuda:0" if device else None
    ba = sd3.Batch.from_packed(synth.pack(A), dev)
    bb = sd3.Batch.from_packed(synth.pack(B), dev)
    for prec in ("fp32", "fp64"):
        d, h = ctx.distance(ba, bb, precision=prec, semantics="solid")
        hi = ctx.intersects(ba, bb, precision=prec, semantics="solid")
        d, h, hi = [x.cpu().numpy() if device else x for x in (d, h, hi)]
        assert np.array_equal(h.astype(bool), h_w) and np.array_equal(hi.astype(bool), h_w)
        assert np.all(d[h_w] == 0.0)
        nz = ~h_w
        assert np.all(np.abs(d[nz] - d_w[nz]) <= 1e-12 * d_w[nz])
        # surface semantics on the same rows: nested rows are apart again
        ds, hs = ctx.distance(ba, bb, precision=prec)
        ds, hs = (ds.cpu().numpy(), hs.cpu().numpy()) if device else (ds, hs)
        assert np.array_equal(ds[nz].view(np.int64), d[nz].view(np.int64))
        assert hs.sum() < h.sum()


def test_solid_semantics_not_in_graphs(ctx):
    A, B = _rows()
    ba = sd3.Batch.from_packed(synth.pack(A[:2]), "cuda:0")
    bb = sd3.Batch.from_packed(synth.pack(B[:2]), "cuda:0")
    import ctypes
    g = ba.geoms(), bb.geoms()
    o = sd3.Context._opts("fp32", "bound", semantics="solid")
    h = ctypes.c_void_p()
    import torch
    d = torch.empty(2, dtype=torch.float64, device="cuda:0")
    st = ctx.lib.sd3_graph_create(ctx.handle, 0, ctypes.byref(g[0]), ctypes.byref(g[1]), d.data_ptr(), None,
                                  ctypes.byref(o), ctypes.byref(h))
    assert sd3.STATUS[st] == "SD3_E_INVALID_ARG"
