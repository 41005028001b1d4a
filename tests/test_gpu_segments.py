"""GPU parity of the segment / point path (sd3_segments): drill-hole segments
against one ore-body mesh, the workload the paper measures (Sec. 4), with the
distance of Sec. 3.2.2 (items (i)-(iii)), the intersection of Sec. 3.2.3
(Eq. 4, closed constraints) and the distance-threshold filter.

Bar: flags bit-exact against the oracle (which takes a segment as the
degenerate triangle (P0, P1, P1)); distances within 1e-12 relative, or within
the FP64 error model 1e-12 d + 64 u S (S the extent of the segment and the
mesh) when the gap is below 1e-6 S, where FP64 resolves the extent but not
the gap to 12 digits (the same bar as the mesh path); the segment path bit-identical to sd3_distance on the same degenerate triangles;
the threshold filter exactly (distance <= r) of the distance the library
returns.
"""
import json
import math
import os

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

import oracle
from paper_1808_09571_amd import sd3, synth

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "segment_forms.json")
TRI1 = np.array([[0, 1, 2]], np.int32)


@pytest.fixture(scope="module")
def ctx():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return sd3.Context(0)


def _mesh_batch(mesh, device):
    return sd3.Batch.from_packed(synth.pack([mesh]), "cuda:0" if device else None)


def _seg_dev(seg, device):
    if not device:
        return np.ascontiguousarray(seg, dtype=np.float64)
    import torch
    return torch.from_numpy(np.ascontiguousarray(seg, dtype=np.float64)).to("cuda:0")


def _np(x):
    return x.cpu().numpy() if hasattr(x, "cpu") else np.asarray(x)


U = 2.0 ** -53


def _tol(seg_i, mesh, d_o):
    """Distance tolerance of one segment: 1e-12 relative, plus 64 u S below
    1e-6 S (S = largest extent of the segment's and the mesh's joint box)."""
    pts = np.vstack([np.asarray(seg_i, np.float64).reshape(-1, 3), mesh[0]])
    S = float(np.max(pts.max(axis=0) - pts.min(axis=0)))
    return 1e-12 * d_o + 64 * U * S if d_o < 1e-6 * S else 1e-12 * d_o


def _oracle_segments(seg, mesh, idx):
    d, h = [], []
    for i in idx:
        p, q = seg[i]
        dd, hh, _ = oracle.mesh((np.array([p, q, q]), TRI1), mesh)
        d.append(dd)
        h.append(hh)
    return np.array(d), np.array(h)


def _all_ops(ctx, seg, mesh, device, r):
    mb = _mesh_batch(mesh, device)
    sg = _seg_dev(seg, device)
    d, h = ctx.segments("distance", sg, mb)
    hi = ctx.segments("intersects", sg, mb)
    w = ctx.segments("within", sg, mb, r=r)
    return _np(d), _np(h).astype(bool), _np(hi).astype(bool), _np(w).astype(bool)


@pytest.mark.parametrize("device", [True, False])
def test_segment_closed_forms(ctx, device):
    with open(GOLDEN) as f:
        g = json.load(f)
    mesh = (np.asarray(g["triangle"], float), TRI1)
    seg = np.array([c["segment"] for c in g["cases"]], dtype=np.float64)
    want = np.array([c["distance"] for c in g["cases"]])
    hits = np.array([c["intersects"] for c in g["cases"]])
    d, h, hi, w = _all_ops(ctx, seg, mesh, device, r=0.5)
    assert np.array_equal(h, hits) and np.array_equal(hi, hits)
    assert np.all(np.abs(d - want) <= 1e-15 * np.maximum(1.0, want)), (d, want)
    assert np.array_equal(w, d <= 0.5)


def _random_case(seed, n=3000):
    g = np.random.default_rng(seed)
    meshes = [synth.icosphere(2, radius=1.0), synth.random_triangle_soup(40, seed, scale=1.0, size=0.4),
              synth.cube((-0.5, -0.5, -0.5), 1.0)]
    mesh = meshes[seed % len(meshes)]
    p = g.uniform(-1.6, 1.6, size=(n, 3))
    q = p + g.normal(size=(n, 3)) * g.uniform(0.0, 1.0, size=(n, 1))
    q[: n // 10] = p[: n // 10]                   # points
    ints = g.integers(-2, 3, size=(n // 10, 2, 3)).astype(float) * 0.5  # exact degeneracies
    seg = np.stack([p, q], axis=1)
    seg[n // 10: n // 10 + ints.shape[0]] = ints
    return seg, mesh


@pytest.mark.parametrize("seed", [0, 1, 2])
@pytest.mark.parametrize("device", [True, False])
def test_random_segments_against_oracle(ctx, seed, device):
    seg, mesh = _random_case(seed)
    d, h, hi, w = _all_ops(ctx, seg, mesh, device, r=0.3)
    d_o, h_o = _oracle_segments(seg, mesh, range(len(seg)))
    assert np.array_equal(h, h_o) and np.array_equal(hi, h_o)
    nz = ~h_o
    assert np.all(d[h_o] == 0.0)
    assert np.all(np.abs(d[nz] - d_o[nz]) <= 1e-12 * d_o[nz]), np.max(np.abs(d[nz] - d_o[nz]) / d_o[nz])
    assert np.array_equal(w, d <= 0.3)


def test_segments_equal_mesh_path_bits(ctx):
    # the segment path and sd3_distance on the same degenerate triangles give
    # the same bits (same FP64 pair routine, same exact test)
    seg, mesh = _random_case(4, n=400)
    d, h, _, _ = _all_ops(ctx, seg, mesh, True, r=0.0)
    A = [(np.array([p, q, q]), TRI1) for p, q in seg]
    B = [mesh] * len(A)
    ba = sd3.Batch.from_packed(synth.pack(A), "cuda:0")
    bb = sd3.Batch.from_packed(synth.pack(B), "cuda:0")
    for prec in ("fp32", "fp64"):
        dm, hm = ctx.distance(ba, bb, precision=prec)
        assert np.array_equal(_np(dm).view(np.int64), d.view(np.int64))
        assert np.array_equal(_np(hm).astype(bool), h)


def test_million_drillhole_segments_vs_500_face_body(ctx):
    # the paper's workload shape at 1e6 segments: 20,000 drill holes of 50
    # segments against a 500-face ore body
    seg, body = synth.config_drillholes(holes=20_000, segs=50, seed=21)
    assert seg.shape[0] == 1_000_000 and body[1].shape[0] == 500
    print("segments: GPU", flush=True)
    d, h, hi, w = _all_ops(ctx, seg, body, True, r=2.0)
    assert np.array_equal(h, hi)
    assert np.all((d == 0.0) == h)
    assert np.array_equal(w, d <= 2.0)
    frac = h.mean()
    assert 0.005 < frac < 0.5, frac
    # a sample against the oracle, with the extremes
    g = np.random.default_rng(3)
    pos = np.nonzero(~h)[0]
    idx = set(g.choice(len(seg), 300, replace=False).tolist())
    idx |= set(np.nonzero(h)[0][:20].tolist())
    idx |= {int(pos[np.argmin(d[pos])]), int(pos[np.argmax(d[pos])])}
    near = pos[np.argsort(np.abs(d[pos] - 2.0))[:20]]  # around the threshold
    idx |= set(near.tolist())
    idx = sorted(idx)
    print(f"segments: oracle on {len(idx)}", flush=True)
    d_o, h_o = _oracle_segments(seg, body, idx)
    assert np.array_equal(h[idx], h_o)
    for k, i in enumerate(idx):
        if h_o[k]:
            assert d[i] == 0.0
        else:
            assert abs(d[i] - d_o[k]) <= _tol(seg[i], body, d_o[k]), (i, d[i], d_o[k])


def test_segment_errors(ctx):
    mesh = synth.icosphere(1)
    seg = np.zeros((4, 2, 3))
    two = sd3.Batch.from_packed(synth.pack([mesh, mesh]))
    with pytest.raises(ValueError):
        ctx.segments("distance", seg, two)
    bad = seg.copy()
    bad[2, 1, 0] = np.nan
    with pytest.raises(sd3.SD3Error) as e:
        ctx.segments("distance", bad, _mesh_batch(mesh, False))
    assert e.value.name == "SD3_E_NONFINITE"
    with pytest.raises(sd3.SD3Error) as e:
        ctx.segments("distance", _seg_dev(bad, True), _mesh_batch(mesh, True))
    assert e.value.name == "SD3_E_NONFINITE"
    broken = (mesh[0], mesh[1].copy())
    broken[1][3, 1] = 10_000
    with pytest.raises(sd3.SD3Error) as e:
        ctx.segments("intersects", _seg_dev(seg, True), _mesh_batch(broken, True))
    assert e.value.name == "SD3_E_INDEX_RANGE"
    with pytest.raises(sd3.SD3Error) as e:
        ctx.segments("within", seg, _mesh_batch(mesh, False), r=-1.0)
    assert e.value.name == "SD3_E_INVALID_ARG"
    # empty inputs
    d, h = ctx.segments("distance", np.zeros((0, 2, 3)), _mesh_batch(mesh, False))
    assert d.shape == (0,)
    empty = (np.zeros((0, 3)), np.zeros((0, 3), np.int32))
    d, h = ctx.segments("distance", seg, _mesh_batch(empty, False))
    assert np.all(np.isinf(d)) and not h.any()
