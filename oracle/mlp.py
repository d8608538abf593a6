"""FP64 multilayer perceptron of the learned warm start (oracle).

The warm start maps a flow condition and a cell position to the steady
flow's primitive variables.  Network: features f (5) -> n_hidden layers of
width d_hidden with SiLU activation -> linear output (5):
    h_0 = f,  h_{l+1} = silu(W_l h_l + b_l),  y = W_out h_L + b_out,
silu(z) = z / (1 + exp(-z)).  Loss: mean squared error over points and
outputs.  Optimiser: Adam with bias correction.

Features of a cell (i, j, k) of an ni x nj x nk channel block at inflow Mach
M and bump height h: [(M - 0.675)/0.175, (h - 0.06)/0.04, 2 xi - 1,
2 eta - 1, 2 zeta - 1] with xi = (i + 1/2)/ni etc.  Targets: deviations of
the primitives from the inflow stream, (rho - 1, u - M sqrt(gamma), v, w, p - 1).

Parameters are a list of (W [out, in], b [out]) per layer, FP64.
"""
from __future__ import annotations

import math

import numpy as np


def silu(z):
    return z / (1.0 + np.exp(-z))


def silu_grad(z):
    s = 1.0 / (1.0 + np.exp(-z))
    return s * (1.0 + z * (1.0 - s))


def features(mach, hb, ni, nj, nk):
    """Features of every cell of one block, [nk, nj, ni, 5]."""
    k, j, i = np.meshgrid(np.arange(nk), np.arange(nj), np.arange(ni), indexing="ij")
    f = np.empty((nk, nj, ni, 5))
    f[..., 0] = (mach - 0.675) / 0.175
    f[..., 1] = (hb - 0.06) / 0.04
    f[..., 2] = 2.0 * (i + 0.5) / ni - 1.0
    f[..., 3] = 2.0 * (j + 0.5) / nj - 1.0
    f[..., 4] = 2.0 * (k + 0.5) / nk - 1.0
    return f


def targets(q, mach, gamma=1.4):
    """Primitive deviations from the inflow stream for conserved states q [5, ...] -> [..., 5]."""
    rho = q[0]
    u = q[1] / rho
    v = q[2] / rho
    w = q[3] / rho
    p = (gamma - 1.0) * (q[4] - 0.5 * rho * (u * u + v * v + w * w))
    return np.stack([rho - 1.0, u - mach * math.sqrt(gamma), v, w, p - 1.0], axis=-1)


def conserved_from_output(y, mach, gamma=1.4):
    """Conserved state [5, ...] from network outputs [..., 5]."""
    rho = 1.0 + y[..., 0]
    u = mach * math.sqrt(gamma) + y[..., 1]
    v = y[..., 2]
    w = y[..., 3]
    p = 1.0 + y[..., 4]
    e = p / (gamma - 1.0) + 0.5 * rho * (u * u + v * v + w * w)
    return np.stack([rho, rho * u, rho * v, rho * w, e])


def forward(params, X):
    """Outputs [P, d_out] and the cache (layer inputs, pre-activations)."""
    h = X
    cache = []
    for l, (W, b) in enumerate(params):
        z = h @ W.T + b
        cache.append((h, z))
        h = silu(z) if l < len(params) - 1 else z
    return h, cache


def mse(Y, T):
    d = Y - T
    return float(np.mean(d * d)), 2.0 * d / d.size


def backward(params, cache, dY):
    """Gradients [(dW, db)] of the loss whose output gradient is dY."""
    grads = [None] * len(params)
    g = dY
    for l in range(len(params) - 1, -1, -1):
        h, z = cache[l]
        if l < len(params) - 1:
            g = g * silu_grad(z)
        W, _ = params[l]
        grads[l] = (g.T @ h, g.sum(axis=0))
        g = g @ W
    return grads


def adam(theta, m, v, g, lr, b1, b2, eps, t):
    """One Adam step (bias-corrected); returns new (theta, m, v)."""
    m = b1 * m + (1.0 - b1) * g
    v = b2 * v + (1.0 - b2) * g * g
    mh = m / (1.0 - b1 ** t)
    vh = v / (1.0 - b2 ** t)
    return theta - lr * mh / (np.sqrt(vh) + eps), m, v
