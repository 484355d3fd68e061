"""Placement-MLP oracle -- TEST INFRASTRUCTURE ONLY.

Float64 NumPy forward pass and backpropagation of the 12 -> 64 -> 64 -> 2 ReLU
network, written from the definition of the masked squared error

    L = (1/n) * sum_s sum_o mask[s,o] * (y[s,o] - t[s,o])^2,

with the parameter layout W1[64][12], b1[64], W2[64][64], b2[64], W3[2][64],
b3[2] flattened in that order.  Pinned in tests by central finite
differences of `loss`, and against torch's CPU linear layers, autograd and
Adam optimizer in float64 (forward pass, gradient, update), with planted
mistakes that the pins must reject.
"""
from __future__ import annotations

import numpy as np

IN, HID, OUT = 12, 64, 2
SIZES = [("W1", (HID, IN)), ("b1", (HID,)), ("W2", (HID, HID)), ("b2", (HID,)), ("W3", (OUT, HID)), ("b3", (OUT,))]
NPARAMS = sum(int(np.prod(s)) for _, s in SIZES)


def unpack(p):
    p = np.asarray(p, dtype=np.float64)
    out, o = {}, 0
    for name, shape in SIZES:
        k = int(np.prod(shape))
        out[name] = p[o:o + k].reshape(shape)
        o += k
    return out


def pack(d):
    return np.concatenate([np.asarray(d[name], np.float64).ravel() for name, _ in SIZES])


def forward(p, x):
    w = unpack(p)
    x = np.asarray(x, np.float64)
    z1 = x @ w["W1"].T + w["b1"]
    h1 = np.maximum(z1, 0.0)
    z2 = h1 @ w["W2"].T + w["b2"]
    h2 = np.maximum(z2, 0.0)
    y = h2 @ w["W3"].T + w["b3"]
    return y, (x, z1, h1, z2, h2)


def loss(p, x, t, mask):
    y, _ = forward(p, x)
    n = len(x)
    return float(np.sum(np.asarray(mask, np.float64) * (y - np.asarray(t, np.float64)) ** 2) / n)


def loss_grad(p, x, t, mask):
    w = unpack(p)
    y, (x, z1, h1, z2, h2) = forward(p, x)
    n = len(x)
    m = np.asarray(mask, np.float64)
    d = y - np.asarray(t, np.float64)
    L = float(np.sum(m * d * d) / n)
    dy = 2.0 * m * d / n                      # dL/dy
    g = {"W3": dy.T @ h2, "b3": dy.sum(0)}
    dz2 = (dy @ w["W3"]) * (z2 > 0)           # through ReLU
    g["W2"] = dz2.T @ h1
    g["b2"] = dz2.sum(0)
    dz1 = (dz2 @ w["W2"]) * (z1 > 0)
    g["W1"] = dz1.T @ x
    g["b1"] = dz1.sum(0)
    return L, pack(g)


def adam(p, grad, m, v, step, lr, b1=0.9, b2=0.999, eps=1e-8):
    """One Adam update (Kingma & Ba) with bias correction; returns (p, m, v)."""
    m = b1 * m + (1 - b1) * grad
    v = b2 * v + (1 - b2) * grad * grad
    mh = m / (1 - b1 ** step)
    vh = v / (1 - b2 ** step)
    return p - lr * mh / (np.sqrt(vh) + eps), m, v
