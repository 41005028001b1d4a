"""ctypes wrapper of the FP64 CPU oracle -- TEST INFRASTRUCTURE ONLY.

Only ``tests/``, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may import this package.  The GPU library neither links nor calls
it.  See ``sd3_oracle.c`` for what is computed and the passages of the paper it
follows (Sec. 3.2.2 distance, Sec. 3.2.3 intersection, Eq. 3, Eq. 4).
"""
from __future__ import annotations

import ctypes
import math
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(_HERE, "sd3_oracle.c")
LIB = os.path.join(_HERE, "libsd3oracle.so")

_lib = None

_D = ctypes.POINTER(ctypes.c_double)
_I32 = ctypes.POINTER(ctypes.c_int32)


def build(src: str = SRC, out: str = LIB) -> str:
    """Compile the oracle with gcc (portable x86-64, FP64, no contraction)."""
    cmd = ["gcc", "-O2", "-std=c11", "-fopenmp", "-ffp-contract=off", "-fno-fast-math",
           "-fPIC", "-shared", src, "-o", out + ".tmp", "-lm"]
    subprocess.run(cmd, check=True)
    os.replace(out + ".tmp", out)
    return out


def load(path: str | None = None):
    """Load the oracle library (building it if it is missing)."""
    global _lib
    if path is None and _lib is not None:
        return _lib
    p = path or LIB
    if not os.path.exists(p):
        build(out=p)
    lib = ctypes.CDLL(p)
    for name in ("sd3o_orient3d", "sd3o_orient3d_exact"):
        f = getattr(lib, name)
        f.argtypes = [_D] * 4
        f.restype = ctypes.c_int
    for name in ("sd3o_orient2d", "sd3o_orient2d_exact"):
        f = getattr(lib, name)
        f.argtypes = [_D] * 3
        f.restype = ctypes.c_int
    lib.sd3o_exact_calls.restype = ctypes.c_longlong
    lib.sd3o_tri_tri_intersect.argtypes = [_D, _D]
    lib.sd3o_tri_tri_intersect.restype = ctypes.c_int
    for name in ("sd3o_pair_d2", "sd3o_disjoint_pair_d2"):
        f = getattr(lib, name)
        f.argtypes = [_D, _D]
        f.restype = ctypes.c_double
    lib.sd3o_seg_seg_d2.argtypes = [_D] * 4
    lib.sd3o_seg_seg_d2.restype = ctypes.c_double
    lib.sd3o_point_seg_d2.argtypes = [_D] * 3
    lib.sd3o_point_seg_d2.restype = ctypes.c_double
    lib.sd3o_vertex_face_d2.argtypes = [_D] * 4
    lib.sd3o_vertex_face_d2.restype = ctypes.c_double
    lib.sd3o_mesh.argtypes = [_D, _I32, ctypes.c_int64, _D, _I32, ctypes.c_int64, ctypes.c_int,
                              ctypes.c_int, ctypes.c_int, _D, ctypes.POINTER(ctypes.c_int)]
    lib.sd3o_mesh.restype = ctypes.c_int64
    lib.sd3o_volume6_exact.argtypes = [_D, ctypes.c_int64, _I32, ctypes.c_int64, ctypes.c_int,
                                       ctypes.POINTER(ctypes.c_uint32), ctypes.POINTER(ctypes.c_int),
                                       ctypes.POINTER(ctypes.c_int)]
    lib.sd3o_volume6_exact.restype = ctypes.c_int
    lib.sd3o_winding.argtypes = [_D, _I32, ctypes.c_int64, _D]
    lib.sd3o_winding.restype = ctypes.c_double
    if path is None:
        _lib = lib
    return lib


def _vec(a, n):
    a = np.ascontiguousarray(np.asarray(a, dtype=np.float64).reshape(-1))
    assert a.size == n
    return a, a.ctypes.data_as(_D)


def check_range(xyz) -> bool:
    """Coordinates the exact predicates support: finite, each 0 or with
    magnitude in [2^-256, 2^256]."""
    x = np.abs(np.asarray(xyz, dtype=np.float64))
    if not np.all(np.isfinite(x)):
        return False
    nz = x[x != 0]
    return bool(np.all((nz >= 2.0 ** -256) & (nz <= 2.0 ** 256)))


def orient3d(a, b, c, d, lib=None) -> int:
    lib = lib or load()
    ps = [_vec(p, 3) for p in (a, b, c, d)]
    return lib.sd3o_orient3d(*[p[1] for p in ps])


def orient3d_exact(a, b, c, d, lib=None) -> int:
    lib = lib or load()
    ps = [_vec(p, 3) for p in (a, b, c, d)]
    return lib.sd3o_orient3d_exact(*[p[1] for p in ps])


def orient2d(a, b, c, lib=None) -> int:
    lib = lib or load()
    ps = [_vec(p, 2) for p in (a, b, c)]
    return lib.sd3o_orient2d(*[p[1] for p in ps])


def exact_calls(lib=None) -> int:
    return int((lib or load()).sd3o_exact_calls())


def tri_tri_intersect(A, B, lib=None) -> bool:
    lib = lib or load()
    a, pa = _vec(A, 9)
    b, pb = _vec(B, 9)
    return bool(lib.sd3o_tri_tri_intersect(pa, pb))


def pair_d2(A, B, lib=None) -> float:
    lib = lib or load()
    a, pa = _vec(A, 9)
    b, pb = _vec(B, 9)
    return float(lib.sd3o_pair_d2(pa, pb))


def seg_seg_d2(p0, p1, q0, q1, lib=None) -> float:
    lib = lib or load()
    ps = [_vec(p, 3) for p in (p0, p1, q0, q1)]
    return float(lib.sd3o_seg_seg_d2(*[p[1] for p in ps]))


def vertex_face_d2(p, x, y, z, lib=None) -> float:
    lib = lib or load()
    ps = [_vec(q, 3) for q in (p, x, y, z)]
    return float(lib.sd3o_vertex_face_d2(*[q[1] for q in ps]))


def default_threads():
    """OMP_NUM_THREADS when set (the host's CPU share), else every core."""
    env = os.environ.get("OMP_NUM_THREADS", "")
    return int(env) if env.isdigit() and int(env) > 0 else (os.cpu_count() or 1)


def mesh(A, B, mode="all", want="distance", threads=None, lib=None):
    """Distance and intersects between meshes A=(xyz, tri) and B.

    mode: "all" (all pairs) or "pruned" (exact chunk pruning).
    want: "distance" (returns (dist, hit)) or "intersects" (returns (None, hit)).
    Returns (dist, hit, pair_tests)."""
    lib = lib or load()
    xa = np.ascontiguousarray(A[0], dtype=np.float64).reshape(-1)
    ta = np.ascontiguousarray(A[1], dtype=np.int32).reshape(-1)
    xb = np.ascontiguousarray(B[0], dtype=np.float64).reshape(-1)
    tb = np.ascontiguousarray(B[1], dtype=np.int32).reshape(-1)
    if not (check_range(xa) and check_range(xb)):
        raise ValueError("coordinates outside the supported range")
    for x, t in ((xa, ta), (xb, tb)):
        if t.size and (t.min() < 0 or t.max() >= x.size // 3):
            raise ValueError("triangle index out of range")
    if threads is None:
        threads = default_threads()
    d = ctypes.c_double(math.nan)
    h = ctypes.c_int(0)
    tests = lib.sd3o_mesh(xa.ctypes.data_as(_D), ta.ctypes.data_as(_I32), ta.size // 3,
                          xb.ctypes.data_as(_D), tb.ctypes.data_as(_I32), tb.size // 3,
                          0 if mode == "all" else 1, 2 if want == "intersects" else 1,
                          int(threads), ctypes.byref(d), ctypes.byref(h))
    dist = None if want == "intersects" else float(d.value)
    return dist, bool(h.value), int(tests)


def batch(packed_a, packed_b, mode="all", want="distance", threads=None, rows=None, lib=None):
    """Row-by-row oracle over two CSR batches (row g of A with row g of B)."""
    G = packed_a.count
    rows = range(G) if rows is None else rows
    dist = np.full(len(rows), np.nan)
    hit = np.zeros(len(rows), dtype=bool)
    for k, g in enumerate(rows):
        d, h, _ = mesh(packed_a.row(g), packed_b.row(g), mode=mode, want=want, threads=threads,
                       lib=lib)
        dist[k] = np.nan if d is None else d
        hit[k] = h
    return dist, hit


def volume_exact(mesh, threads=None, lib=None):
    """Volume of a mesh by the divergence theorem (Sec. 3.2.1, Eq. 2:
    1/6 of the sum over faces of u . ((v - u) x (w - u))), evaluated exactly:
    returned as a fractions.Fraction."""
    from fractions import Fraction
    lib = lib or load()
    x = np.ascontiguousarray(mesh[0], dtype=np.float64).reshape(-1)
    t = np.ascontiguousarray(mesh[1], dtype=np.int32).reshape(-1)
    if not check_range(x):
        raise ValueError("coordinates outside the supported range")
    limbs = (ctypes.c_uint32 * 72)()
    neg, e0 = ctypes.c_int(0), ctypes.c_int(0)
    n = lib.sd3o_volume6_exact(x.ctypes.data_as(_D), x.size // 3, t.ctypes.data_as(_I32), t.size // 3,
                               int(threads or default_threads()), limbs, ctypes.byref(neg),
                               ctypes.byref(e0))
    if n < 0:
        raise ValueError("triangle index out of range")
    mag = sum(int(limbs[i]) << (32 * i) for i in range(n))
    v6 = Fraction(-mag if neg.value else mag) * Fraction(2) ** (3 * e0.value)
    return v6 / 6


def volume(mesh, threads=None, lib=None):
    """The exact volume rounded to the nearest double."""
    return float(volume_exact(mesh, threads, lib))


def winding(mesh, p, lib=None):
    """Generalised winding number of a closed mesh around point p (FP64)."""
    lib = lib or load()
    x = np.ascontiguousarray(mesh[0], dtype=np.float64).reshape(-1)
    t = np.ascontiguousarray(mesh[1], dtype=np.int32).reshape(-1)
    q = np.ascontiguousarray(p, dtype=np.float64).reshape(3)
    return float(lib.sd3o_winding(x.ctypes.data_as(_D), t.ctypes.data_as(_I32), t.size // 3,
                                  q.ctypes.data_as(_D)))


def mesh_solid(A, B, mode="pruned", threads=None, lib=None):
    """Distance and intersects under solid semantics: each row is the closed
    region a closed, outward-oriented (connected) mesh bounds.  The solids meet
    iff the surfaces meet or a vertex of one lies inside the other (winding
    number above 1/2); the distance is then 0, else the surface distance.
    Returns (dist, hit)."""
    d, h, _ = mesh(A, B, mode=mode, threads=threads, lib=lib)
    if h:
        return 0.0, True
    inside = ((len(A[1]) and len(B[1]) and winding(B, np.asarray(A[0])[int(np.asarray(A[1])[0][0])], lib) > 0.5)
              or (len(A[1]) and len(B[1]) and winding(A, np.asarray(B[0])[int(np.asarray(B[1])[0][0])], lib) > 0.5))
    return (0.0, True) if inside else (d, False)
