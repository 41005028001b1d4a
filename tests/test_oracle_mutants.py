"""The pins must catch plausible mistakes in the oracle.

Each case copies the oracle source, plants one mistake (a dropped term, a
flipped sign, a transposed operand, an open instead of a closed constraint, a
missing exact fallback, an unsafe pruning rule), builds it into a temporary
library and runs a reduced battery of the pins of test_oracle.py against it.
At least one pin must fail for every mutant, while the unmodified source passes
the same battery.  Everything runs on the CPU.
"""
import math
import os

import numpy as np
import pytest

import bruteforce as bf
import oracle
import test_oracle as pins
from paper_1808_09571_amd import synth

MUTANTS = {
    "drop_vertex_face": (
        "x = sd3o_vertex_face_d2(A + 3 * i, B, B + 3, B + 6);", "x = INFINITY;"),
    "orient3d_sign_flip": (
        "double bound = 9.0 * U64 * perm;\n    if (det > bound) return 1;",
        "double bound = 9.0 * U64 * perm;\n    if (det > bound) return -1;"),
    "segseg_transposed": (
        "double s = (b * e - c * d) / D", "double s = (b * d - c * e) / D"),
    "drop_side_t1": (
        "x = sd3o_point_seg_d2(q1, p0, p1);               /* side t = 1 */", "x = INFINITY;"),
    "drop_interior_edge_edge": ("if (D > 0.0) {", "if (D < 0.0) {"),
    "no_exact_fallback": (
        "return sd3o_orient3d_exact(a, b, c, d);", "return det > 0 ? 1 : (det < 0 ? -1 : 0);"),
    "open_plane_test": ("if (op * oq > 0) return 0;", "if (op * oq >= 0) return 0;"),
    "inside_test_sign": ("if (dot3(m, n) < 0.0) return INFINITY;\n    sub3(z, y, ek);",
                         "if (dot3(m, n) > 0.0) return INFINITY;\n    sub3(z, y, ek);"),
    "coplanar_any_projection": ("if (!seg_tri_2d(P, Q, A, B, C)) return 0;",
                                "if (seg_tri_2d(P, Q, A, B, C)) return 1;"),
    "unsafe_pruning": ("cp[k].lb * (1.0 - 1e-9) > bd + 1e-9 * (bd + 2.0 * ext)",
                       "cp[k].lb > 0.5 * bd"),
    "intersect_skips_B_edges": (
        "if (seg_tri_3d(B + 3 * i, B + 3 * ((i + 1) % 3), A, A + 3, A + 6)) return 1;", ";"),
}


def _battery(lib):
    """Reduced pin battery; returns the names of the pins that failed."""
    failed = []

    def run(name, fn):
        try:
            fn()
        except AssertionError:
            failed.append(name)

    def pairs():
        for dist in pins.DISTS:
            g = np.random.default_rng(2000 + pins.DISTS.index(dist))
            for _ in range(40):
                A, B = pins._sample(dist, g)
                pins._check_pair(A, B, lib)

    def orients():
        g = np.random.default_rng(9)
        for _ in range(300):
            P = pins._onplane(g, 4, scale=10.0 ** g.uniform(-2, 3))
            assert oracle.orient3d(*P, lib=lib) == bf.orient3d_sign(*P)
            P = g.normal(size=(4, 3))
            assert oracle.orient3d(*P, lib=lib) == bf.orient3d_sign(*P)

    def closed():
        for case in pins._golden_cases():
            pins.test_closed_forms(case, lib)

    def spheres():
        for seed in (0, 2):
            A, B = synth.config_icospheres(seed)
            d, h, _ = oracle.mesh(A, B, lib=lib)
            assert oracle.mesh(A, B, mode="pruned", lib=lib)[:2] == (d, h)

    def tins():
        pins.test_tin_pair_construction(lib)

    def primitives():
        pins.test_segment_and_point_primitives(lib)

    def adversarial():
        pins.test_pruning_adversarial(lib)

    run("pairs", pairs)
    run("orient3d", orients)
    run("closed_forms", closed)
    run("icospheres_pruned", spheres)
    run("tin_pair", tins)
    run("primitives", primitives)
    run("pruning_adversarial", adversarial)
    return failed


def _build_variant(tmp_path, name, repl):
    src = open(oracle.SRC).read()
    if repl is not None:
        old, new = repl
        assert src.count(old) == 1, f"mutation site for {name} not unique/found"
        src = src.replace(old, new)
    path = os.path.join(str(tmp_path), f"sd3o_{name}.c")
    with open(path, "w") as f:
        f.write(src)
    so = os.path.join(str(tmp_path), f"libsd3o_{name}.so")
    oracle.build(src=path, out=so)
    return oracle.load(so)


def test_unmutated_passes_battery(tmp_path):
    lib = _build_variant(tmp_path, "clean", None)
    assert _battery(lib) == []


@pytest.mark.parametrize("name", sorted(MUTANTS))
def test_mutant_is_caught(name, tmp_path):
    lib = _build_variant(tmp_path, name, MUTANTS[name])
    failed = _battery(lib)
    assert failed, f"no pin caught mutant {name}"
