"""FP64 reference of the tile-pair ranker MLP -- TEST INFRASTRUCTURE ONLY.

Plain numpy forward / backward / Adam for the 10 -> 64 -> 64 -> 64 -> 1 ReLU
network whose parameters are packed as W1[64][10] b1[64] W2[64][64] b2[64]
W3[64][64] b3[64] w4[64] b4 (the layout of include/sd3.h).  Loss: mean squared
error.  Used to check the GPU training kernels; itself pinned by central finite
differences and the closed-form first Adam step (tests/test_ranker_oracle.py).
"""
from __future__ import annotations

import numpy as np

NIN, NH = 10, 64
SIZES = [("W1", (NH, NIN)), ("b1", (NH,)), ("W2", (NH, NH)), ("b2", (NH,)),
         ("W3", (NH, NH)), ("b3", (NH,)), ("w4", (NH,)), ("b4", (1,))]
NPARAM = sum(int(np.prod(s)) for _, s in SIZES)  # 9089


def unpack(p):
    p = np.asarray(p, dtype=np.float64)
    out, i = {}, 0
    for name, shape in SIZES:
        n = int(np.prod(shape))
        out[name] = p[i:i + n].reshape(shape)
        i += n
    return out


def pack(d):
    return np.concatenate([np.asarray(d[name], dtype=np.float64).reshape(-1) for name, _ in SIZES])


def forward(p, X):
    q = unpack(p)
    X = np.asarray(X, dtype=np.float64)
    z1 = X @ q["W1"].T + q["b1"]
    h1 = np.maximum(z1, 0.0)
    z2 = h1 @ q["W2"].T + q["b2"]
    h2 = np.maximum(z2, 0.0)
    z3 = h2 @ q["W3"].T + q["b3"]
    h3 = np.maximum(z3, 0.0)
    y = h3 @ q["w4"] + q["b4"][0]
    return y, (X, z1, h1, z2, h2, z3, h3)


def loss_grad(p, X, t):
    """MSE loss and its gradient with respect to the packed parameters."""
    q = unpack(p)
    y, (X, z1, h1, z2, h2, z3, h3) = forward(p, X)
    t = np.asarray(t, dtype=np.float64)
    n = X.shape[0]
    e = y - t
    loss = float(np.mean(e * e))
    dy = 2.0 * e / n
    g = {}
    g["w4"] = h3.T @ dy
    g["b4"] = np.array([dy.sum()])
    d3 = np.outer(dy, q["w4"]) * (z3 > 0)
    g["W3"] = d3.T @ h2
    g["b3"] = d3.sum(0)
    d2 = (d3 @ q["W3"]) * (z2 > 0)
    g["W2"] = d2.T @ h1
    g["b2"] = d2.sum(0)
    d1 = (d2 @ q["W2"]) * (z1 > 0)
    g["W1"] = d1.T @ X
    g["b1"] = d1.sum(0)
    return loss, pack(g)


def adam(p, g, m, v, step, lr=1e-3, beta1=0.9, beta2=0.999, eps=1e-8):
    """One bias-corrected Adam update (Kingma & Ba 2015); returns (p, m, v)."""
    m = beta1 * m + (1.0 - beta1) * g
    v = beta2 * v + (1.0 - beta2) * g * g
    mh = m / (1.0 - beta1 ** step)
    vh = v / (1.0 - beta2 ** step)
    return p - lr * mh / (np.sqrt(vh) + eps), m, v
