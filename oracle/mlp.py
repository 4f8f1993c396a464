"""Float64 reference of the tail-closure network: 16 -> 64 -> 64 -> 1.

TEST INFRASTRUCTURE: CPU oracle of the network the GPU trains and runs with
its own kernels.  Layers: h1 = silu(W1 x + b1), h2 = silu(W2 h1 + b2),
y = W3 h2 + b3, with silu(a) = a * sigmoid(a).  Loss: mean squared error.
Optimiser: Adam (Kingma & Ba, 2015) with bias correction.

Parameter layout (one flat float vector, the same order the GPU uses):
W1 [64,16] row-major, b1 [64], W2 [64,64], b2 [64], W3 [1,64], b3 [1]:
5,313 values.
"""
from __future__ import annotations

import numpy as np

D_IN, D_H = 16, 64
SHAPES = [("W1", (D_H, D_IN)), ("b1", (D_H,)), ("W2", (D_H, D_H)), ("b2", (D_H,)),
          ("W3", (1, D_H)), ("b3", (1,))]
NPARAM = sum(int(np.prod(s)) for _, s in SHAPES)


def unpack(theta):
    out, o = {}, 0
    for name, shp in SHAPES:
        k = int(np.prod(shp))
        out[name] = np.asarray(theta[o:o + k], dtype=np.float64).reshape(shp)
        o += k
    return out


def pack(p):
    return np.concatenate([np.asarray(p[name], np.float64).ravel() for name, _ in SHAPES])


def sigmoid(a):
    return 1.0 / (1.0 + np.exp(-a))


def silu(a):
    return a * sigmoid(a)


def silu_grad(a):
    s = sigmoid(a)
    return s * (1.0 + a * (1.0 - s))


def forward(theta, X):
    p = unpack(theta)
    a1 = X @ p["W1"].T + p["b1"]
    h1 = silu(a1)
    a2 = h1 @ p["W2"].T + p["b2"]
    h2 = silu(a2)
    y = h2 @ p["W3"].T + p["b3"]
    return y[:, 0], (X, a1, h1, a2, h2)


def loss_and_grad(theta, X, z):
    """Mean squared error 1/N sum (y - z)^2 and its gradient."""
    p = unpack(theta)
    y, (X, a1, h1, a2, h2) = forward(theta, X)
    N = len(z)
    r = y - z
    loss = float(np.mean(r ** 2))
    dy = (2.0 / N) * r[:, None]                  # [N,1]
    g = {}
    g["W3"] = dy.T @ h2
    g["b3"] = dy.sum(0)
    dh2 = dy @ p["W3"]
    da2 = dh2 * silu_grad(a2)
    g["W2"] = da2.T @ h1
    g["b2"] = da2.sum(0)
    dh1 = da2 @ p["W2"]
    da1 = dh1 * silu_grad(a1)
    g["W1"] = da1.T @ X
    g["b1"] = da1.sum(0)
    return loss, pack(g)


def init(seed):
    """Scaled uniform initialisation (fan-in), biases zero."""
    rng = np.random.default_rng(seed)
    p = {}
    for name, shp in SHAPES:
        if name.startswith("W"):
            lim = np.sqrt(3.0 / shp[1])
            p[name] = rng.uniform(-lim, lim, size=shp)
        else:
            p[name] = np.zeros(shp)
    return pack(p)


def adam_step(theta, grad, m1, m2, t, lr=1e-3, b1=0.9, b2=0.999, eps=1e-8):
    """One Adam update (t is the 1-based step count); returns new (theta, m1, m2)."""
    m1 = b1 * m1 + (1 - b1) * grad
    m2 = b2 * m2 + (1 - b2) * grad * grad
    mh = m1 / (1 - b1 ** t)
    vh = m2 / (1 - b2 ** t)
    return theta - lr * mh / (np.sqrt(vh) + eps), m1, m2
