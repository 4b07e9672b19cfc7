"""FP64 reference of the width cost model -- TEST INFRASTRUCTURE ONLY.

A 5-64-64-1 perceptron with ReLU, y = W3 relu(W2 relu(W1 x + b1) + b2) + b3,
its mean-squared-error gradient by back-propagation, and one Adam step
(Kingma & Ba 2015, with bias correction), in plain numpy FP64.  The flat
parameter layout is W1[64][5] b1[64] W2[64][64] b2[64] W3[64] b3.  Pinned by
central finite differences in tests/test_mlp_oracle.py; shares no code with
the HIP kernels.
"""
from __future__ import annotations

import numpy as np

IN, H = 5, 64
SIZES = {"W1": (H, IN), "b1": (H,), "W2": (H, H), "b2": (H,), "W3": (H,), "b3": (1,)}
NPARAM = sum(int(np.prod(s)) for s in SIZES.values())


def unpack(p):
    p = np.asarray(p, dtype=np.float64)
    out, o = {}, 0
    for k, s in SIZES.items():
        n = int(np.prod(s))
        out[k] = p[o:o + n].reshape(s)
        o += n
    return out


def pack(d):
    return np.concatenate([np.asarray(d[k], dtype=np.float64).ravel() for k in SIZES])


def forward(p, x):
    """Returns (y[rows], h1[rows, 64], h2[rows, 64])."""
    w = unpack(p)
    x = np.asarray(x, dtype=np.float64)
    h1 = np.maximum(x @ w["W1"].T + w["b1"], 0.0)
    h2 = np.maximum(h1 @ w["W2"].T + w["b2"], 0.0)
    y = h2 @ w["W3"] + w["b3"][0]
    return y, h1, h2


def mse(y, t):
    y = np.asarray(y, dtype=np.float64)
    t = np.asarray(t, dtype=np.float64)
    return float(np.mean((y - t) ** 2)), 2.0 * (y - t) / y.shape[0]


def backward(p, x, dy):
    """Gradient of sum_r dy_r y_r with respect to the flat parameters."""
    w = unpack(p)
    x = np.asarray(x, dtype=np.float64)
    dy = np.asarray(dy, dtype=np.float64)
    _, h1, h2 = forward(p, x)
    g = {}
    g["W3"] = dy @ h2
    g["b3"] = np.array([dy.sum()])
    dz2 = np.outer(dy, w["W3"]) * (h2 > 0)
    g["W2"] = dz2.T @ h1
    g["b2"] = dz2.sum(axis=0)
    dz1 = (dz2 @ w["W2"]) * (h1 > 0)
    g["W1"] = dz1.T @ x
    g["b1"] = dz1.sum(axis=0)
    return pack(g)


def loss_and_grad(p, x, t):
    y, _, _ = forward(p, x)
    loss, dy = mse(y, t)
    return loss, backward(p, x, dy)


def adam(p, g, m, v, step, lr=1e-3, b1=0.9, b2=0.999, eps=1e-8):
    """One bias-corrected Adam step; returns new (p, m, v)."""
    m = b1 * m + (1.0 - b1) * g
    v = b2 * v + (1.0 - b2) * g * g
    mh = m / (1.0 - b1 ** step)
    vh = v / (1.0 - b2 ** step)
    return p - lr * mh / (np.sqrt(vh) + eps), m, v


def init(seed=0):
    """He-uniform weights, zero biases (the initial point used for training)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    d = {}
    for k, s in SIZES.items():
        if k.startswith("W"):
            fan_in = s[-1] if len(s) == 2 else H
            lim = np.sqrt(6.0 / fan_in)
            d[k] = rng.uniform(-lim, lim, size=s)
        else:
            d[k] = np.zeros(s)
    return pack(d)
