"""Exact rational brute force for the distance between two closed triangles.

Independent of the oracle's decomposition: every point of a triangle lies in
the relative interior of one of its 7 faces (3 vertices, 3 edges, the
interior).  The global minimiser of |p - q|^2 over the pair lies in the
relative interior of some face pair, where it is a stationary point of the
quadratic restricted to the two affine hulls.  When that restricted problem is
non-singular its stationary point is unique; when it is singular the minimum
is also attained on a smaller face.  So the exact squared distance is the
minimum over all 49 face pairs of the non-singular stationary points that lie
in their closed faces.  All arithmetic uses fractions.Fraction (exact for
binary64 inputs).  The squared distance is 0 exactly iff the triangles meet.
"""
from __future__ import annotations

from fractions import Fraction


def _fr(v):
    return tuple(Fraction(float(c)) for c in v)


def _sub(a, b):
    return tuple(x - y for x, y in zip(a, b))


def _dot(a, b):
    return sum(x * y for x, y in zip(a, b))


def _faces(T):
    v0, v1, v2 = T
    return [
        (v0, [], "pt"), (v1, [], "pt"), (v2, [], "pt"),
        (v0, [_sub(v1, v0)], "seg"), (v1, [_sub(v2, v1)], "seg"), (v2, [_sub(v0, v2)], "seg"),
        (v0, [_sub(v1, v0), _sub(v2, v0)], "tri"),
    ]


def _solve(M, rhs):
    """Gaussian elimination over fractions; None if singular."""
    n = len(rhs)
    A = [list(M[i]) + [rhs[i]] for i in range(n)]
    for c in range(n):
        p = next((r for r in range(c, n) if A[r][c] != 0), None)
        if p is None:
            return None
        A[c], A[p] = A[p], A[c]
        for r in range(n):
            if r != c and A[r][c] != 0:
                f = A[r][c] / A[c][c]
                A[r] = [x - f * y for x, y in zip(A[r], A[c])]
    return [A[i][n] / A[i][i] for i in range(n)]


def _feasible(x, kind):
    if kind == "pt":
        return True
    if kind == "seg":
        return 0 <= x[0] <= 1
    return x[0] >= 0 and x[1] >= 0 and x[0] + x[1] <= 1


def tri_tri_d2(A, B) -> Fraction:
    """Exact squared distance between closed triangles A, B (3x3 coordinates)."""
    TA = [_fr(A[i]) for i in range(3)]
    TB = [_fr(B[i]) for i in range(3)]
    best = None
    for oa, da, ka in _faces(TA):
        for ob, db, kb in _faces(TB):
            r0 = _sub(oa, ob)
            cols = list(da) + [tuple(-c for c in d) for d in db]
            n = len(cols)
            if n == 0:
                x = []
            else:
                G = [[_dot(cols[i], cols[j]) for j in range(n)] for i in range(n)]
                x = _solve(G, [-_dot(cols[i], r0) for i in range(n)])
                if x is None:
                    continue
            if not (_feasible(x[:len(da)], ka) and _feasible(x[len(da):], kb)):
                continue
            w = tuple(r0[k] + sum(x[i] * cols[i][k] for i in range(n)) for k in range(3))
            d2 = _dot(w, w)
            if best is None or d2 < best:
                best = d2
    return best


def orient3d_sign(a, b, c, d) -> int:
    a, b, c, d = _fr(a), _fr(b), _fr(c), _fr(d)
    u, v, w = _sub(b, a), _sub(c, a), _sub(d, a)
    det = (u[1] * v[2] - u[2] * v[1]) * w[0] + (u[2] * v[0] - u[0] * v[2]) * w[1] + \
        (u[0] * v[1] - u[1] * v[0]) * w[2]
    return (det > 0) - (det < 0)


def orient2d_sign(a, b, c) -> int:
    a = tuple(Fraction(float(x)) for x in a)
    b = tuple(Fraction(float(x)) for x in b)
    c = tuple(Fraction(float(x)) for x in c)
    det = (b[0] - a[0]) * (c[1] - a[1]) - (b[1] - a[1]) * (c[0] - a[0])
    return (det > 0) - (det < 0)
