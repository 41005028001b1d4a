"""Pins of the oracle's exact volume (Sec. 3.2.1, Eq. 1-2: 1/6 of the sum of
u . ((v - u) x (w - u)) over counter-clockwise faces) against closed forms and
exact invariants that do not come from the formula itself:

* boxes a x b x c (abc), the unit right tetrahedron (1/6), the regular
  octahedron of radius r (4 r^3 / 3), prisms over convex polygons (shoelace
  area times height, computed with fractions);
* orientation reversal negates, translations by dyadic vectors keep and
  scaling by 2 multiplies by 8, all exactly;
* a planted mistake (a dropped 1/6, a reversed cross product, the origin taken
  from the wrong vertex of an open mesh) fails at least one of the above.
"""
import math
from fractions import Fraction

import numpy as np
import pytest

import oracle
from paper_1808_09571_amd import synth


def _box(a, b, c, lo=(0.0, 0.0, 0.0)):
    x, t = synth.cube((0.0, 0.0, 0.0), 1.0)
    x = x * np.array([a, b, c]) + np.asarray(lo)
    return x, t


def _tet():
    x = np.array([[0, 0, 0], [1, 0, 0], [0, 1, 0], [0, 0, 1]], float)
    t = np.array([[0, 2, 1], [0, 1, 3], [0, 3, 2], [1, 2, 3]], np.int32)
    return x, t


def _octahedron(r):
    x = np.array([[r, 0, 0], [-r, 0, 0], [0, r, 0], [0, -r, 0], [0, 0, r], [0, 0, -r]], float)
    t = []
    for sx, i in ((1, 0), (-1, 1)):
        for sy, j in ((1, 2), (-1, 3)):
            for sz, k in ((1, 4), (-1, 5)):
                tri = [i, j, k]
                if sx * sy * sz < 0:
                    tri = [i, k, j]
                t.append(tri)
    return x, np.array(t, np.int32)


def _prism(n, h, rad, center=(0.0, 0.0)):
    """Convex n-gon (vertices on a circle, rounded to doubles) extruded by h."""
    ang = 2 * math.pi * np.arange(n) / n
    xy = np.c_[rad * np.cos(ang) + center[0], rad * np.sin(ang) + center[1]]
    bot = np.c_[xy, np.zeros(n)]
    top = np.c_[xy, np.full(n, h)]
    x = np.vstack([bot, top])
    t = []
    for k in range(1, n - 1):
        t.append([0, k + 1, k])              # bottom, seen from below
        t.append([n, n + k, n + k + 1])      # top
    for k in range(n):
        a, b = k, (k + 1) % n
        t.append([a, b, n + b])
        t.append([a, n + b, n + a])
    area2 = sum(Fraction(xy[k][0]) * Fraction(xy[(k + 1) % n][1]) -
                Fraction(xy[(k + 1) % n][0]) * Fraction(xy[k][1]) for k in range(n))
    return (x, np.array(t, np.int32)), area2 / 2 * Fraction(h)


@pytest.mark.parametrize("abc", [(1.0, 1.0, 1.0), (2.0, 3.0, 0.5), (0.1, 7.25, 1e3)])
def test_box_volume(abc, olib):
    a, b, c = abc
    x, t = _box(a, b, c, lo=(-3.5, 2.0, 100.0))
    # the box the rounded corner coordinates span: product of its side lengths
    side = [Fraction(float(x[:, k].max())) - Fraction(float(x[:, k].min())) for k in range(3)]
    assert oracle.volume_exact((x, t), lib=olib) == side[0] * side[1] * side[2]


def test_tetrahedron_and_octahedron(olib):
    assert oracle.volume_exact(_tet(), lib=olib) == Fraction(1, 6)
    for r in (1.0, 0.5, 3.0):
        assert oracle.volume_exact(_octahedron(r), lib=olib) == Fraction(4, 3) * Fraction(r) ** 3


@pytest.mark.parametrize("n", [3, 5, 17, 64])
def test_prism_is_shoelace_area_times_height(n, olib):
    m, want = _prism(n, 2.5, 1.3, center=(0.75, -2.0))
    assert oracle.volume_exact(m, lib=olib) == want


def _integer_mesh(m, scale=2.0 ** 20):
    # the same closed mesh with its vertices rounded to integers (translations
    # by integer vectors are then exact in binary64)
    return np.round(m[0] * scale), m[1]


def test_exact_invariants(olib):
    for m in (_integer_mesh(synth.icosphere(2)), _integer_mesh(synth.blob(2000, 3.0, (1.0, -2.0, 0.5), 7)),
              _tet(), _octahedron(3.0)):
        v = oracle.volume_exact(m, lib=olib)
        x, t = m
        assert oracle.volume_exact((x, t[:, ::-1].copy()), lib=olib) == -v
        assert oracle.volume_exact((x + np.array([5.0, -1024.0, 3.0]), t), lib=olib) == v
        assert oracle.volume_exact((x * 2.0, t), lib=olib) == 8 * v
        # shuffled triangle order and rotated corner order
        p = np.random.default_rng(0).permutation(len(t))
        assert oracle.volume_exact((x, np.roll(t[p], 1, axis=1).copy()), lib=olib) == v


def test_icosphere_approaches_the_ball(olib):
    for lv in (2, 3, 4):
        v = oracle.volume(synth.icosphere(lv), lib=olib)
        assert v < 4 / 3 * math.pi
        assert 4 / 3 * math.pi - v < 3.0 / 4 ** lv


def test_planted_mistakes_fail_a_pin():
    box, want = _box(2.0, 3.0, 0.5), Fraction(3)

    def exact(m, term):
        x, t = m
        return sum(term(*[[Fraction(c) for c in x[i]] for i in tri]) for tri in t)

    def cross(a, b):
        return [a[1] * b[2] - a[2] * b[1], a[2] * b[0] - a[0] * b[2], a[0] * b[1] - a[1] * b[0]]

    def sub(a, b):
        return [p - q for p, q in zip(a, b)]

    def dot(a, b):
        return sum(p * q for p, q in zip(a, b))

    good = lambda u, v, w: dot(u, cross(sub(v, u), sub(w, u))) / 6
    assert exact(box, good) == want
    mutants = [lambda u, v, w: dot(u, cross(sub(v, u), sub(w, u))),          # no 1/6
               lambda u, v, w: dot(u, cross(sub(w, u), sub(v, u))) / 6,      # reversed cross
               lambda u, v, w: dot(v, cross(sub(v, u), sub(w, u))) / 6 - 1]  # shifted
    for mt in mutants:
        assert exact(box, mt) != want


# --- point in solid (solid semantics): the oracle's winding number ---------
def test_winding_number_inside_outside(olib):
    # a closed outward mesh winds once around interior points and not at all
    # around exterior ones, whatever the mesh (a topological invariant)
    cube = synth.cube((0.0, 0.0, 0.0), 1.0)
    for p, w in (((0.5, 0.5, 0.5), 1.0), ((0.01, 0.99, 0.5), 1.0), ((1.5, 0.5, 0.5), 0.0),
                 ((-3.0, 2.0, 1.0), 0.0)):
        assert abs(oracle.winding(cube, p, lib=olib) - w) < 1e-12, p
    for m in (synth.icosphere(3), synth.blob(5000, 2.0, (0.0, 0.0, 0.0), 9), _octahedron(1.0)):
        assert abs(oracle.winding(m, (0.1, -0.05, 0.2), lib=olib) - 1.0) < 1e-12
        assert abs(oracle.winding(m, (4.0, 1.0, -2.0), lib=olib)) < 1e-12
        flipped = (m[0], m[1][:, ::-1].copy())
        assert abs(oracle.winding(flipped, (0.1, -0.05, 0.2), lib=olib) + 1.0) < 1e-12


def test_solid_semantics_of_nested_meshes(olib):
    outer = synth.icosphere(3)
    inner = synth.icosphere(2, radius=0.5, center=(0.1, 0.0, -0.05))
    d_s, h_s, _ = oracle.mesh(inner, outer, lib=olib)
    assert not h_s and d_s > 0.3
    assert oracle.mesh_solid(inner, outer, lib=olib) == (0.0, True)
    assert oracle.mesh_solid(outer, inner, lib=olib) == (0.0, True)
    far = synth.icosphere(2, radius=0.5, center=(3.0, 0.0, 0.0))
    d, h, _ = oracle.mesh(far, outer, lib=olib)
    assert oracle.mesh_solid(far, outer, lib=olib) == (d, False)
    # a planted mistake (the solid angle without its factor 2) puts interior
    # points at winding 1/2, which the 1/2 threshold no longer separates
    x, t = outer
    p = np.array([0.1, 0.0, 0.0])
    tot = 0.0
    for tri in t:
        a, b, c = (x[i] - p for i in tri)
        la, lb, lc = (np.linalg.norm(v) for v in (a, b, c))
        tot += math.atan2(np.dot(a, np.cross(b, c)),
                          la * lb * lc + np.dot(a, b) * lc + np.dot(a, c) * lb + np.dot(b, c) * la)
    assert abs(tot / (4 * math.pi) - 0.5) < 1e-9
