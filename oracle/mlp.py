"""Plain NumPy reference of the learned initial guess's network.

Test infrastructure only (see the package docstring).

Architecture: 16 inputs -> 64 -> 64 -> 3 outputs, GELU after each hidden
layer (GELU(x) = x Phi(x) = x (1 + erf(x / sqrt 2)) / 2), mean squared error
against the targets, Adam updates. Parameter vector layout (float32 on the
GPU, float64 here): W1 (64 x 16, row-major), b1 (64), W2 (64 x 64), b2 (64),
W3 (3 x 64), b3 (3).
"""
from __future__ import annotations

import numpy as np
from scipy.special import erf

SIZES = (16, 64, 64, 3)


def n_params(sizes=SIZES) -> int:
    return sum(sizes[i + 1] * sizes[i] + sizes[i + 1] for i in range(len(sizes) - 1))


def unpack(theta: np.ndarray, sizes=SIZES):
    out, o = [], 0
    for i in range(len(sizes) - 1):
        fi, fo = sizes[i], sizes[i + 1]
        w = theta[o:o + fo * fi].reshape(fo, fi); o += fo * fi
        b = theta[o:o + fo]; o += fo
        out.append((w, b))
    return out


def gelu(x):
    return 0.5 * x * (1.0 + erf(x / np.sqrt(2.0)))


def gelu_grad(x):
    return 0.5 * (1.0 + erf(x / np.sqrt(2.0))) + x * np.exp(-0.5 * x * x) / np.sqrt(2.0 * np.pi)


def forward(theta, x, sizes=SIZES):
    """x: batch x 16. Returns (y, cache)."""
    layers = unpack(theta, sizes)
    acts, pre = [x], []
    h = x
    for li, (w, b) in enumerate(layers):
        z = h @ w.T + b
        pre.append(z)
        h = gelu(z) if li < len(layers) - 1 else z
        acts.append(h)
    return h, (acts, pre)


def loss(y, t):
    """Mean squared error over the batch and the outputs."""
    return float(np.mean((y - t) ** 2))


def backward(theta, x, t, sizes=SIZES):
    """Gradient of ``loss(forward(theta, x), t)`` with respect to theta."""
    layers = unpack(theta, sizes)
    y, (acts, pre) = forward(theta, x, sizes)
    g = 2.0 * (y - t) / y.size
    grads = []
    for li in range(len(layers) - 1, -1, -1):
        w, _ = layers[li]
        if li < len(layers) - 1:
            g = g * gelu_grad(pre[li])
        gw = g.T @ acts[li]
        gb = g.sum(axis=0)
        grads.append((gw, gb))
        g = g @ w
    flat = []
    for gw, gb in reversed(grads):
        flat.append(gw.ravel()); flat.append(gb)
    return np.concatenate(flat), loss(y, t)


def adam(theta, grad, m, v, step, lr=1e-3, b1=0.9, b2=0.999, eps=1e-8):
    """One Adam update (bias-corrected moments); ``step`` counts from 1."""
    m = b1 * m + (1 - b1) * grad
    v = b2 * v + (1 - b2) * grad * grad
    mh = m / (1 - b1 ** step)
    vh = v / (1 - b2 ** step)
    return theta - lr * mh / (np.sqrt(vh) + eps), m, v
