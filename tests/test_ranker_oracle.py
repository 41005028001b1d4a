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


def test_adam_constant_gradient_closed_form():
    # with a constant gradient g the moments after k steps are (1 - beta1^k) g
    # and (1 - beta2^k) g^2, so each bias-corrected step moves every parameter
    # by exactly lr * g / (|g| + eps): after k steps p_k = p_0 - k lr g / (|g| + eps).
    # A bias correction with a wrong exponent (say beta ** 1 instead of
    # beta ** step) agrees at step 1 and fails here from step 2 on.
    g = np.array([0.5, -2.0, 1e-3, 3.0, -1e-2])
    p = np.array([1.0, -1.0, 0.25, 0.0, 2.0])
    m = np.zeros(5)
    v = np.zeros(5)
    lr, b1, b2, eps = 0.01, 0.9, 0.999, 1e-8
    step_size = lr * g / (np.abs(g) + eps)
    p0 = p.copy()
    for k in range(1, 9):
        p, m, v = mlp.adam(p, g, m, v, k, lr=lr, beta1=b1, beta2=b2, eps=eps)
        assert np.allclose(m, (1.0 - b1 ** k) * g, rtol=1e-12, atol=0)
        assert np.allclose(v, (1.0 - b2 ** k) * g * g, rtol=1e-12, atol=0)
        assert np.allclose(p, p0 - k * step_size, rtol=1e-12, atol=1e-15)


def test_adam_mutant_bias_exponent_fails_the_pin():
    # a planted slip in the bias correction (exponent fixed at 1) passes the
    # step-1 pin but not the constant-gradient pin above
    def adam_bad(p, g, m, v, step, lr, beta1=0.9, beta2=0.999, eps=1e-8):
        m = beta1 * m + (1.0 - beta1) * g
        v = beta2 * v + (1.0 - beta2) * g * g
        return p - lr * (m / (1.0 - beta1)) / (np.sqrt(v / (1.0 - beta2)) + eps), m, v

    g = np.array([0.5, -2.0])
    p, m, v = np.zeros(2), np.zeros(2), np.zeros(2)
    p1, _, _ = adam_bad(p, g, m, v, 1, lr=0.1)
    assert np.allclose(p1, -0.1 * g / (np.abs(g) + 1e-8), rtol=1e-12)
    for k in range(1, 4):
        p, m, v = adam_bad(p, g, m, v, k, lr=0.1)
    assert not np.allclose(p, -3 * 0.1 * g / (np.abs(g) + 1e-8), rtol=1e-6)
