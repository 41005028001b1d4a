"""Seeded synthetic inputs: triangle meshes shaped like the paper's mining workloads.

The paper evaluates on a synthetic mining data set (drill holes, closed ore-body
meshes, block models; Sec. 4 "Use case") that is not distributed with it.  The
generators here make inputs of the same kinds and sizes from fixed seeds:

* icospheres (closed polyhedral surfaces),
* heightfield TINs with fractal value noise (terrain),
* drill-hole tubes (16-gon cross-section along a gently curving polyline),
* ore-body blobs (geodesic spheres with smooth radial noise).

This module is shared by the oracle-side tests and by the GPU path's tests and
benchmark, so it deliberately contains no part of the distance/intersection
arithmetic: it only places vertices and lists triangles.  All randomness comes
from numpy's PCG64 generator seeded explicitly.

A mesh is ``(xyz, tri)``: ``xyz`` float64 ``[nv, 3]``, ``tri`` int32 ``[nt, 3]``
(vertex indices into ``xyz``).  A batch is a list of meshes, packed into CSR
form by :func:`pack`.
"""
from __future__ import annotations

import math
from dataclasses import dataclass

import numpy as np

__all__ = [
    "Packed", "pack", "rng", "icosahedron", "icosphere", "geodesic_sphere",
    "fractal_noise_2d", "value_noise_3d", "heightfield", "cube", "tube", "blob",
    "config_icospheres", "config_tin_pair", "config_tube_blob_batch",
    "config_tin_blob", "random_triangle_soup",
]


def rng(seed: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(seed))


# ----------------------------------------------------------------------------
# CSR packing of a batch of meshes (one mesh per table row)
# ----------------------------------------------------------------------------
@dataclass
class Packed:
    xyz: np.ndarray     # float64 [nv_total*3]
    tri: np.ndarray     # int32   [nt_total*3], indices local to the row
    v_off: np.ndarray   # int64   [G+1]
    t_off: np.ndarray   # int64   [G+1]

    @property
    def count(self) -> int:
        return int(self.v_off.shape[0] - 1)

    def row(self, g: int):
        v0, v1 = int(self.v_off[g]), int(self.v_off[g + 1])
        t0, t1 = int(self.t_off[g]), int(self.t_off[g + 1])
        return (self.xyz[3 * v0:3 * v1].reshape(-1, 3),
                self.tri[3 * t0:3 * t1].reshape(-1, 3))


def pack(meshes) -> Packed:
    nv = np.array([m[0].shape[0] for m in meshes], dtype=np.int64)
    nt = np.array([m[1].shape[0] for m in meshes], dtype=np.int64)
    v_off = np.zeros(len(meshes) + 1, dtype=np.int64)
    t_off = np.zeros(len(meshes) + 1, dtype=np.int64)
    np.cumsum(nv, out=v_off[1:])
    np.cumsum(nt, out=t_off[1:])
    xyz = np.empty(int(v_off[-1]) * 3, dtype=np.float64)
    tri = np.empty(int(t_off[-1]) * 3, dtype=np.int32)
    for g, (x, t) in enumerate(meshes):
        xyz[3 * v_off[g]:3 * v_off[g + 1]] = np.asarray(x, dtype=np.float64).reshape(-1)
        tri[3 * t_off[g]:3 * t_off[g + 1]] = np.asarray(t, dtype=np.int32).reshape(-1)
    return Packed(xyz, tri, v_off, t_off)


# ----------------------------------------------------------------------------
# Spheres
# ----------------------------------------------------------------------------
def icosahedron():
    p = (1.0 + math.sqrt(5.0)) / 2.0
    v = np.array([[-1, p, 0], [1, p, 0], [-1, -p, 0], [1, -p, 0],
                  [0, -1, p], [0, 1, p], [0, -1, -p], [0, 1, -p],
                  [p, 0, -1], [p, 0, 1], [-p, 0, -1], [-p, 0, 1]], dtype=np.float64)
    v /= np.linalg.norm(v, axis=1, keepdims=True)
    f = np.array([[0, 11, 5], [0, 5, 1], [0, 1, 7], [0, 7, 10], [0, 10, 11],
                  [1, 5, 9], [5, 11, 4], [11, 10, 2], [10, 7, 6], [7, 1, 8],
                  [3, 9, 4], [3, 4, 2], [3, 2, 6], [3, 6, 8], [3, 8, 9],
                  [4, 9, 5], [2, 4, 11], [6, 2, 10], [8, 6, 7], [9, 8, 1]], dtype=np.int32)
    return v, f


def icosphere(levels: int, radius: float = 1.0, center=(0.0, 0.0, 0.0)):
    """Icosahedron refined ``levels`` times by edge-midpoint subdivision, each new
    vertex pushed back to the unit sphere at every level (levels=3: 642 vertices,
    1280 triangles)."""
    v, f = icosahedron()
    verts = [tuple(x) for x in v]
    for _ in range(levels):
        cache = {}
        nf = []

        def mid(a, b):
            key = (a, b) if a < b else (b, a)
            if key not in cache:
                m = np.asarray(verts[a]) + np.asarray(verts[b])
                m /= np.linalg.norm(m)
                cache[key] = len(verts)
                verts.append(tuple(m))
            return cache[key]

        for a, b, c in f:
            ab, bc, ca = mid(a, b), mid(b, c), mid(c, a)
            nf += [(a, ab, ca), (b, bc, ab), (c, ca, bc), (ab, bc, ca)]
        f = np.array(nf, dtype=np.int32)
    xyz = np.asarray(verts, dtype=np.float64) * radius + np.asarray(center, dtype=np.float64)
    return xyz, f


_GEO_CACHE: dict = {}


def geodesic_sphere(freq: int):
    """Unit geodesic sphere of frequency ``freq``: every icosahedron face split into
    freq^2 triangles, vertices projected to the sphere (20*freq^2 triangles,
    10*freq^2+2 vertices).  Cached per frequency; callers must copy before editing."""
    if freq in _GEO_CACHE:
        return _GEO_CACHE[freq]
    n = int(freq)
    v, f = icosahedron()
    # lattice (i, j), i + j <= n, on each face
    ii, jj = np.meshgrid(np.arange(n + 1), np.arange(n + 1), indexing="ij")
    keep = (ii + jj) <= n
    ii, jj = ii[keep], jj[keep]
    loc = -np.ones((n + 1, n + 1), dtype=np.int64)
    loc[ii, jj] = np.arange(ii.size)
    # local triangles on the lattice
    ui, uj = np.nonzero(np.add.outer(np.arange(n), np.arange(n)) < n)         # i + j < n
    di, dj = np.nonzero(np.add.outer(np.arange(n), np.arange(n)) + 1 < n)     # i + j + 1 < n
    up = np.stack([loc[ui, uj], loc[ui + 1, uj], loc[ui, uj + 1]], axis=1)
    down = np.stack([loc[di + 1, dj], loc[di + 1, dj + 1], loc[di, dj + 1]], axis=1)
    tl = np.concatenate([up, down])
    pts = []
    tris = []
    base = 0
    for a, b, c in f:
        A, B, C = v[a], v[b], v[c]
        p = A[None, :] + (B - A)[None, :] * (ii[:, None] / n) + (C - A)[None, :] * (jj[:, None] / n)
        p /= np.linalg.norm(p, axis=1, keepdims=True)
        pts.append(p)
        tris.append(tl + base)
        base += p.shape[0]
    pts = np.concatenate(pts)
    tris = np.concatenate(tris)
    # merge the copies of points shared by neighbouring faces
    key = np.round(pts * 1e9).astype(np.int64)
    _, first, inv = np.unique(key, axis=0, return_index=True, return_inverse=True)
    xyz = pts[first]
    tri = inv.reshape(-1)[tris].astype(np.int32)
    _GEO_CACHE[freq] = (xyz, tri)
    return xyz, tri


# ----------------------------------------------------------------------------
# Value noise
# ----------------------------------------------------------------------------
def _fade(t):
    return t * t * t * (t * (t * 6.0 - 15.0) + 10.0)


def _value_noise_2d(u, v, table):
    i = np.floor(u).astype(np.int64)
    j = np.floor(v).astype(np.int64)
    fu, fv = _fade(u - i), _fade(v - j)
    i = np.clip(i, 0, table.shape[0] - 2)
    j = np.clip(j, 0, table.shape[1] - 2)
    a = table[i, j] + (table[i + 1, j] - table[i, j]) * fu
    b = table[i, j + 1] + (table[i + 1, j + 1] - table[i, j + 1]) * fu
    return a + (b - a) * fv


def fractal_noise_2d(x, y, extent, seed, octaves=6, base_freq=4.0, lacunarity=2.0,
                     gain=0.5):
    """Sum of ``octaves`` value-noise octaves at positions (x, y) in [0, extent_x] x
    [0, extent_y]; octave ``o`` has ``base_freq*lacunarity**o`` lattice cells along
    the longer extent and weight ``gain**o``.  Normalised to [-1, 1]."""
    ex, ey = float(extent[0]), float(extent[1])
    L = max(ex, ey)
    total = np.zeros(np.broadcast(x, y).shape, dtype=np.float64)
    wsum = 0.0
    for o in range(octaves):
        fq = base_freq * lacunarity ** o
        nx = int(math.ceil(fq * ex / L)) + 2
        ny = int(math.ceil(fq * ey / L)) + 2
        table = rng(seed * 1009 + o).uniform(-1.0, 1.0, size=(nx, ny))
        w = gain ** o
        total += w * _value_noise_2d(x / L * fq, y / L * fq, table)
        wsum += w
    return total / wsum


def value_noise_3d(p, seed, freq=2.0, octaves=2, gain=0.5):
    """Smooth value noise in [-1, 1] at points ``p`` [n, 3] inside [-1, 1]^3."""
    total = np.zeros(p.shape[0], dtype=np.float64)
    wsum = 0.0
    for o in range(octaves):
        fq = freq * 2.0 ** o
        n = int(math.ceil(2.0 * fq)) + 2
        table = rng(seed * 7919 + o).uniform(-1.0, 1.0, size=(n, n, n))
        q = (p + 1.0) * fq
        i = np.clip(np.floor(q).astype(np.int64), 0, n - 2)
        f = _fade(q - i)
        acc = np.zeros(p.shape[0])
        for dx in (0, 1):
            wx = f[:, 0] if dx else 1.0 - f[:, 0]
            for dy in (0, 1):
                wy = f[:, 1] if dy else 1.0 - f[:, 1]
                for dz in (0, 1):
                    wz = f[:, 2] if dz else 1.0 - f[:, 2]
                    acc += wx * wy * wz * table[i[:, 0] + dx, i[:, 1] + dy, i[:, 2] + dz]
        w = gain ** o
        total += w * acc
        wsum += w
    return total / wsum


# ----------------------------------------------------------------------------
# Terrain, tubes, blobs, cubes
# ----------------------------------------------------------------------------
def grid_triangles(nx: int, ny: int) -> np.ndarray:
    """Triangles of an (nx x ny)-cell grid whose (nx+1)*(ny+1) vertices are stored
    x-major (index = i*(ny+1) + j); every cell is cut along the same diagonal."""
    i, j = np.meshgrid(np.arange(nx), np.arange(ny), indexing="ij")
    v00 = (i * (ny + 1) + j).reshape(-1)
    v10 = v00 + (ny + 1)
    v01 = v00 + 1
    v11 = v10 + 1
    t = np.empty((2 * v00.size, 3), dtype=np.int32)
    t[0::2] = np.stack([v00, v10, v11], axis=1)
    t[1::2] = np.stack([v00, v11, v01], axis=1)
    return t


def heightfield(nx, ny, sx, sy, seed, amplitude=50.0, octaves=6, base_freq=4.0):
    """TIN over [0, sx] x [0, sy] with nx x ny cells and fractal value-noise heights
    of the given amplitude.  Returns (xyz, tri)."""
    xs = np.linspace(0.0, sx, nx + 1)
    ys = np.linspace(0.0, sy, ny + 1)
    X, Y = np.meshgrid(xs, ys, indexing="ij")
    Z = amplitude * fractal_noise_2d(X, Y, (sx, sy), seed, octaves=octaves,
                                     base_freq=base_freq)
    xyz = np.stack([X.reshape(-1), Y.reshape(-1), Z.reshape(-1)], axis=1)
    return xyz, grid_triangles(nx, ny)


def cube(lo=(0.0, 0.0, 0.0), size=1.0):
    """Closed axis-aligned cube surface (8 vertices, 12 triangles)."""
    lo = np.asarray(lo, dtype=np.float64)
    s = np.asarray(size, dtype=np.float64) * np.ones(3)
    corners = np.array([[i, j, k] for i in (0, 1) for j in (0, 1) for k in (0, 1)],
                       dtype=np.float64)
    xyz = lo + corners * s
    # vertex id = 4*i + 2*j + k
    quads = [(0, 1, 3, 2), (4, 6, 7, 5),    # x = 0, x = 1
             (0, 4, 5, 1), (2, 3, 7, 6),    # y = 0, y = 1
             (0, 2, 6, 4), (1, 5, 7, 3)]    # z = 0, z = 1
    tri = []
    for a, b, c, d in quads:
        tri += [(a, b, c), (a, c, d)]
    return xyz, np.asarray(tri, dtype=np.int32)


def _unit(v):
    return v / np.linalg.norm(v)


def _perp(d):
    a = np.array([1.0, 0.0, 0.0]) if abs(d[0]) < 0.9 else np.array([0.0, 1.0, 0.0])
    return _unit(np.cross(d, a))


def _cross3(a, b):
    return (a[1] * b[2] - a[2] * b[1], a[2] * b[0] - a[0] * b[2], a[0] * b[1] - a[1] * b[0])


def _unit3(v):
    n = math.sqrt(v[0] * v[0] + v[1] * v[1] + v[2] * v[2])
    return (v[0] / n, v[1] / n, v[2] / n)


def polyline(n_seg, g: np.random.Generator, start, direction, step=(0.2, 0.4),
             max_turn_deg=5.0):
    """Gently curving 3D polyline: ``n_seg`` steps of length U[step], each turning by
    at most ``max_turn_deg`` about a random axis (plain float arithmetic per
    step; the random draws are made in bulk)."""
    ang = np.radians(g.uniform(0.0, max_turn_deg, size=n_seg)).tolist()
    phi = g.uniform(0.0, 2 * math.pi, size=n_seg).tolist()
    stp = g.uniform(step[0], step[1], size=n_seg).tolist()
    pts = [tuple(float(x) for x in start)]
    d = _unit3(tuple(float(x) for x in direction))
    for s in range(n_seg):
        ref = (1.0, 0.0, 0.0) if abs(d[0]) < 0.9 else (0.0, 1.0, 0.0)
        ax = _unit3(_cross3(d, ref))
        b = _cross3(d, ax)
        c, sn = math.cos(phi[s]), math.sin(phi[s])
        ax = (c * ax[0] + sn * b[0], c * ax[1] + sn * b[1], c * ax[2] + sn * b[2])
        ca, sa = math.cos(ang[s]), math.sin(ang[s])
        d = _unit3((ca * d[0] + sa * ax[0], ca * d[1] + sa * ax[1], ca * d[2] + sa * ax[2]))
        p = pts[-1]
        pts.append((p[0] + stp[s] * d[0], p[1] + stp[s] * d[1], p[2] + stp[s] * d[2]))
    return np.asarray(pts, dtype=np.float64)


def tube(path, radius=0.05, sides=16):
    """Closed tube of a 16-gon cross-section swept along ``path`` [k+1, 3] with
    parallel-transport frames: 2*sides triangles per segment plus two fan caps of
    sides-2 triangles each (32k + 28 triangles for 16 sides)."""
    path = np.asarray(path, dtype=np.float64)
    m = path.shape[0]
    tang = np.empty_like(path)
    tang[1:-1] = path[2:] - path[:-2]
    tang[0] = path[1] - path[0]
    tang[-1] = path[-1] - path[-2]
    tang /= np.linalg.norm(tang, axis=1, keepdims=True)
    nrm = np.empty_like(path)
    nrm[0] = _perp(tang[0])
    for i in range(1, m):
        v = nrm[i - 1] - np.dot(nrm[i - 1], tang[i]) * tang[i]
        nrm[i] = _unit(v)
    bin_ = np.cross(tang, nrm)
    th = 2 * math.pi * np.arange(sides) / sides
    ring = (np.cos(th)[None, :, None] * nrm[:, None, :] +
            np.sin(th)[None, :, None] * bin_[:, None, :]) * radius
    xyz = (path[:, None, :] + ring).reshape(-1, 3)
    i, k = np.meshgrid(np.arange(m - 1), np.arange(sides), indexing="ij")
    a = (i * sides + k).reshape(-1)
    b = (i * sides + (k + 1) % sides).reshape(-1)
    c, d = a + sides, b + sides
    side_tri = np.empty((2 * a.size, 3), dtype=np.int64)
    side_tri[0::2] = np.stack([a, b, d], axis=1)
    side_tri[1::2] = np.stack([a, d, c], axis=1)
    last = (m - 1) * sides
    kk = np.arange(1, sides - 1)
    caps = np.empty((2 * kk.size, 3), dtype=np.int64)
    caps[0::2] = np.stack([np.zeros_like(kk), kk + 1, kk], axis=1)
    caps[1::2] = np.stack([np.full_like(kk, last), last + kk, last + kk + 1], axis=1)
    return xyz, np.concatenate([side_tri, caps]).astype(np.int32)


def blob(n_tri_target, radius, center, seed, noise=0.3):
    """Ore-body blob: geodesic sphere with about ``n_tri_target`` triangles
    (frequency round(sqrt(T/20))), radius scaled by 1 + noise*N(direction) with N a
    smooth 3D value noise in [-1, 1]."""
    freq = max(1, int(round(math.sqrt(n_tri_target / 20.0))))
    u, tri = geodesic_sphere(freq)
    r = radius * (1.0 + noise * value_noise_3d(u, seed))
    xyz = u * r[:, None] + np.asarray(center, dtype=np.float64)
    return xyz, tri.copy()


def random_triangle_soup(n, seed, scale=1.0, center=(0.0, 0.0, 0.0), size=0.5):
    """``n`` independent random triangles (3n vertices) with vertices uniform in a
    cube of side ``2*scale`` around ``center``, each triangle of extent ~``size``."""
    g = rng(seed)
    c = g.uniform(-scale, scale, size=(n, 1, 3)) + np.asarray(center)
    v = c + g.uniform(-size, size, size=(n, 3, 3))
    return v.reshape(-1, 3), np.arange(3 * n, dtype=np.int32).reshape(n, 3)


# ----------------------------------------------------------------------------
# Benchmark configurations
# ----------------------------------------------------------------------------
def config_icospheres(seed: int):
    """Two level-3 icospheres of radius 1 (1280 triangles each); the second centred
    at (2.5, 0, 0) plus uniform jitter in [-0.6, 0.6]^3 drawn from ``seed``."""
    g = rng(seed)
    c2 = np.array([2.5, 0.0, 0.0]) + g.uniform(-0.6, 0.6, size=3)
    return icosphere(3), icosphere(3, center=c2)


def config_tin_pair(n=512, extent=1000.0, amplitude=50.0, gap=0.01, seeds=(1, 2)):
    """Two n x n-cell TINs over the same [0, extent]^2 grid and diagonal, heights
    from seeded 6-octave value noise of the given amplitude.  The second surface
    is lifted so that its lowest vertical clearance over the first, taken over the
    shared vertices, equals ``gap``; because both surfaces are linear on the same
    cells the clearance is at least ``gap`` everywhere, so the surfaces do not
    meet and their distance is at most ``gap``."""
    a = heightfield(n, n, extent, extent, seeds[0], amplitude=amplitude)
    b = heightfield(n, n, extent, extent, seeds[1], amplitude=amplitude)
    lift = gap - np.min(b[0][:, 2] - a[0][:, 2])
    xyz_b = b[0].copy()
    xyz_b[:, 2] += lift
    return a, (xyz_b, b[1])


def config_tin_blob(nx=2000, ny=1000, amplitude=50.0, blob_freq=224, blob_radius=50.0,
                    gap=0.001, seed=5):
    """Scale case: an nx x ny-cell TIN (spacing 1, fractal noise) and a noisy closed
    blob (20*blob_freq^2 triangles) hovering over a terrain peak.  The peak is the
    highest vertex within a (2*r_max)-wide window in every direction; the blob is
    moved so that its lowest vertex sits ``gap`` straight above the peak.  Every
    blob point is then higher than every terrain vertex under the blob's footprint,
    so the two never meet, and their distance is at most ``gap``."""
    tin = heightfield(nx, ny, float(nx), float(ny), seed, amplitude=amplitude)
    H = tin[0][:, 2].reshape(nx + 1, ny + 1)
    rmax = blob_radius * 1.3
    w = int(math.ceil(2 * rmax)) + 2
    from scipy.ndimage import maximum_filter
    M = maximum_filter(H, size=2 * w + 1, mode="constant", cval=-np.inf)
    cand = (H == M)
    cand[:w, :] = False
    cand[-w:, :] = False
    cand[:, :w] = False
    cand[:, -w:] = False
    ci, cj = np.nonzero(cand)
    if ci.size == 0:
        raise ValueError("no isolated terrain peak found")
    k = int(np.argmax(H[ci, cj]))
    pi, pj = int(ci[k]), int(cj[k])
    peak = tin[0][pi * (ny + 1) + pj]
    bx, bt = blob(20 * blob_freq ** 2, blob_radius, (0.0, 0.0, 0.0), seed + 17)
    low = bx[int(np.argmin(bx[:, 2]))].copy()
    shift = np.array([peak[0] - low[0], peak[1] - low[1], peak[2] + gap - low[2]])
    bx = bx + shift
    return tin, (bx, bt)


def config_tube_blob_batch(rows=4096, seed=3, tube_tri=(200, 20000),
                           blob_tri=(1000, 200000), blob_radius=5.0,
                           aim_range=3.3, tube_radius=0.05):
    """Batch of drill-hole tube vs ore-body blob pairs, one per table row.  Tube
    and blob triangle counts are log-uniform in the given ranges; each tube's
    polyline passes through an aim point at distance U[0, aim_range*R] from the
    blob centre, so roughly a third of the rows touch or cross the blob surface."""
    g = rng(seed)
    A, B = [], []
    for r in range(rows):
        tt = math.exp(g.uniform(math.log(tube_tri[0]), math.log(tube_tri[1])))
        bt = math.exp(g.uniform(math.log(blob_tri[0]), math.log(blob_tri[1])))
        nseg = max(1, int(round((tt - 28) / 32)))
        center = g.uniform(-100.0, 100.0, size=3)
        B.append(blob(bt, blob_radius, center, seed * 100003 + r))
        dirn = _unit(g.normal(size=3))
        off = _perp(dirn)
        phi = g.uniform(0, 2 * math.pi)
        off = math.cos(phi) * off + math.sin(phi) * np.cross(dirn, off)
        aim = center + g.uniform(0.0, aim_range * blob_radius) * off
        half = nseg // 2
        fwd = polyline(nseg - half, g, aim, dirn)
        bwd = polyline(half, g, aim, -dirn)
        path = np.concatenate([bwd[::-1], fwd[1:]], axis=0)
        A.append(tube(path, radius=tube_radius))
    return A, B


def drill_holes(n_holes, segs, seed, extent, top, step=(1.0, 3.0), turn=0.05):
    """Drill holes as polylines of ``segs`` segments each (the segment workload
    of Sec. 4): collars uniform over [-extent, extent]^2 at height top + U[0, 10],
    initial direction downward with a dip of U[60, 90] degrees from the
    horizontal and a uniform azimuth, each step of length U[step] after a small
    random change of direction (Gaussian of deviation ``turn``, renormalised).
    Returns the segments as a float64 array [n_holes * segs, 2, 3], hole by hole
    (consecutive segments of a hole are adjacent)."""
    g = rng(seed)
    collar = np.c_[g.uniform(-extent, extent, size=(n_holes, 2)), top + g.uniform(0.0, 10.0, n_holes)]
    dip = np.radians(g.uniform(60.0, 90.0, n_holes))
    az = g.uniform(0.0, 2.0 * math.pi, n_holes)
    d = np.c_[np.cos(dip) * np.cos(az), np.cos(dip) * np.sin(az), -np.sin(dip)]
    pts = np.empty((n_holes, segs + 1, 3), dtype=np.float64)
    pts[:, 0] = collar
    for s in range(segs):
        d = d + g.normal(0.0, turn, size=(n_holes, 3))
        d /= np.linalg.norm(d, axis=1, keepdims=True)
        pts[:, s + 1] = pts[:, s] + g.uniform(step[0], step[1], size=(n_holes, 1)) * d
    return np.ascontiguousarray(np.stack([pts[:, :-1], pts[:, 1:]], axis=2).reshape(-1, 2, 3))


def config_drillholes(holes=100_000, segs=50, seed=11, faces=500, radius=50.0):
    """Segment workload of Sec. 4: ``holes`` x ``segs`` drill-hole segments (5 M by
    default) against one ore body, a noisy closed blob of ``faces`` triangles
    (frequency-5 geodesic sphere: 500 faces) of radius ``radius`` at the origin.
    Collars cover [-1.5 R, 1.5 R]^2 above the body; holes reach about 100 units
    down, so a part of them pass through or near it."""
    body = blob(faces, radius, (0.0, 0.0, 0.0), seed + 1)
    seg = drill_holes(holes, segs, seed, 1.5 * radius, 1.3 * radius + 5.0)
    return seg, body
