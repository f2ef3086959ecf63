"""FP64 reference of the warm-start network (TEST INFRASTRUCTURE ONLY).

    h1 = GELU(W1 u + b1), h2 = GELU(W2 h1 + b2), y = W3 h2 + b3,
    GELU(z) = z (1 + erf(z / sqrt 2)) / 2,  loss = mean((y - target)^2),

with the flat parameter layout W1 (H x I, row-major), b1, W2 (H x H), b2,
W3 (O x H), b3, and the Adam update (beta1 0.9, beta2 0.999, eps 1e-8).
Backpropagation is written out by hand and pinned against central finite
differences of the forward pass in the tests.
"""
from __future__ import annotations

import math

import numpy as np
from scipy.special import erf


def sizes(I, H, O):
    return [("W1", (H, I)), ("b1", (H,)), ("W2", (H, H)), ("b2", (H,)), ("W3", (O, H)), ("b3", (O,))]


def unflatten(p, I, H, O):
    out, off = {}, 0
    for name, shp in sizes(I, H, O):
        cnt = int(np.prod(shp))
        out[name] = np.asarray(p[off:off + cnt], dtype=np.float64).reshape(shp)
        off += cnt
    return out


def flatten(d, I, H, O):
    return np.concatenate([d[name].reshape(-1) for name, _ in sizes(I, H, O)])


def gelu(z):
    return 0.5 * z * (1.0 + erf(z / math.sqrt(2.0)))


def gelu_grad(z):
    return 0.5 * (1.0 + erf(z / math.sqrt(2.0))) + z * np.exp(-0.5 * z * z) / math.sqrt(2.0 * math.pi)


def forward(p, u, I, H, O):
    w = unflatten(p, I, H, O)
    z1 = u @ w["W1"].T + w["b1"]
    h1 = gelu(z1)
    z2 = h1 @ w["W2"].T + w["b2"]
    h2 = gelu(z2)
    y = h2 @ w["W3"].T + w["b3"]
    return y, (z1, h1, z2, h2)


def loss(p, u, target, I, H, O):
    y, _ = forward(p, u, I, H, O)
    return float(np.mean((y - target) ** 2))


def grad(p, u, target, I, H, O):
    """(loss, flat gradient) by backpropagation."""
    w = unflatten(p, I, H, O)
    y, (z1, h1, z2, h2) = forward(p, u, I, H, O)
    dy = 2.0 * (y - target) / y.size
    g = {"W3": dy.T @ h2, "b3": dy.sum(0)}
    dh2 = (dy @ w["W3"]) * gelu_grad(z2)
    g["W2"] = dh2.T @ h1
    g["b2"] = dh2.sum(0)
    dh1 = (dh2 @ w["W2"]) * gelu_grad(z1)
    g["W1"] = dh1.T @ u
    g["b1"] = dh1.sum(0)
    return float(np.mean((y - target) ** 2)), flatten(g, I, H, O)


def adam(p, g, m, v, step, lr, b1=0.9, b2=0.999, eps=1e-8):
    """One Adam step (step counts from 1); returns (p, m, v)."""
    m = b1 * m + (1 - b1) * g
    v = b2 * v + (1 - b2) * g * g
    mhat = m / (1 - b1 ** step)
    vhat = v / (1 - b2 ** step)
    return p - lr * mhat / (np.sqrt(vhat) + eps), m, v
