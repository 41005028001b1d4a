"""Pins of the FP64 ranker-MLP reference (oracle/mlp.py): analytic gradients
against central finite differences, the packed layout against include/sd3.h,
and the first Adam step against its closed form."""
import re
import os

import numpy as np

from oracle import mlp

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _random(seed, n=37):
    g = np.random.default_rng(seed)
    p = g.normal(size=mlp.NPARAM) * 0.3
    X = g.normal(size=(n, mlp.NIN))
    t = g.normal(size=n)
    return p, X, t


def test_layout_matches_header():
    h = open(os.path.join(ROOT, "include", "sd3.h")).read()
    assert int(re.search(r"#define SD3_MLP_NPARAM (\d+)", h).group(1)) == mlp.NPARAM == 9089
    assert int(re.search(r"#define SD3_MLP_NIN (\d+)", h).group(1)) == mlp.NIN
    assert int(re.search(r"#define SD3_MLP_NHID (\d+)", h).group(1)) == mlp.NH
    p = np.arange(mlp.NPARAM, dtype=float)
    assert np.array_equal(mlp.pack(mlp.unpack(p)), p)


def test_gradient_matches_central_differences():
    p, X, t = _random(0)
    _, g = mlp.loss_grad(p, X, t)
    rng = np.random.default_rng(1)
    idx = np.concatenate([rng.choice(mlp.NPARAM, 300, replace=False),
                          [0, 639, 640, 703, 704, 9088]])
    h = 1e-6
    for i in idx:
        e = np.zeros(mlp.NPARAM)
        e[i] = h
        fd = (mlp.loss_grad(p + e, X, t)[0] - mlp.loss_grad(p - e, X, t)[0]) / (2 * h)
        assert abs(fd - g[i]) <= 1e-6 * max(1.0, abs(g[i])), (i, fd, g[i])


def test_forward_matches_explicit_loops():
    p, X, _ = _random(2, n=3)
    q = mlp.unpack(p)
    y, _ = mlp.forward(p, X)
    for i in range(3):
        h = [max(0.0, q["b1"][j] + sum(q["W1"][j][k] * X[i][k] for k in range(10))) for j in range(64)]
        h2 = [max(0.0, q["b2"][j] + sum(q["W2"][j][k] * h[k] for k in range(64))) for j in range(64)]
        h3 = [max(0.0, q["b3"][j] + sum(q["W3"][j][k] * h2[k] for k in range(64))) for j in range(64)]
        yy = q["b4"][0] + sum(q["w4"][j] * h3[j] for j in range(64))
        assert abs(yy - y[i]) <= 1e-12 * max(1.0, abs(yy))


def test_first_adam_step_closed_form():
    g = np.array([0.5, -2.0, 1e-3, 0.0])
    p = np.zeros(4)
    p1, m, v = mlp.adam(p, g, np.zeros(4), np.zeros(4), 1, lr=0.1, eps=1e-8)
    # step 1: bias-corrected m = g, v = g^2, so the update is lr * g / (|g| + eps)
    assert np.allclose(p1, -0.1 * g / (np.abs(g) + 1e-8), rtol=1e-12, atol=0)
