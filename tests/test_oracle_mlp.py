"""Pins for the oracle MLP (CPU only): central finite differences of the
loss, the closed form of a purely linear network, SiLU's derivative, Adam's
first step and the feature/target round trip."""
import math

import numpy as np

from oracle import mlp
from paper_1710_09995_amd import cases


def _loss(params, X, T):
    Y, _ = mlp.forward(params, X)
    return mlp.mse(Y, T)[0]


def test_gradcheck_central_differences():
    rng = np.random.default_rng(0)
    params = cases.mlp_init(5, 12, 2, 5, seed=1, out_scale=1.0)
    params = [(W, b + 0.1 * rng.normal(size=b.shape)) for W, b in params]
    X = rng.normal(size=(7, 5))
    T = rng.normal(size=(7, 5))
    Y, cache = mlp.forward(params, X)
    _, dY = mlp.mse(Y, T)
    grads = mlp.backward(params, cache, dY)
    h = 1e-6
    for l, (W, b) in enumerate(params):
        for arr, g in ((W, grads[l][0]), (b, grads[l][1])):
            idx = list(np.ndindex(arr.shape))
            for n in rng.choice(len(idx), size=min(12, len(idx)), replace=False):
                ix = idx[n]
                old = arr[ix]
                arr[ix] = old + h
                lp = _loss(params, X, T)
                arr[ix] = old - h
                lm = _loss(params, X, T)
                arr[ix] = old
                fd = (lp - lm) / (2 * h)
                assert abs(fd - g[ix]) <= 1e-7 * max(1.0, abs(fd)), (l, ix, fd, g[ix])


def test_linear_network_closed_form():
    rng = np.random.default_rng(2)
    W = rng.normal(size=(5, 4))
    b = rng.normal(size=5)
    X = rng.normal(size=(9, 4))
    T = rng.normal(size=(9, 5))
    Y, cache = mlp.forward([(W, b)], X)
    assert np.allclose(Y, X @ W.T + b, rtol=0, atol=1e-14)
    loss, dY = mlp.mse(Y, T)
    assert abs(loss - np.mean((X @ W.T + b - T) ** 2)) < 1e-14
    (dW, db), = mlp.backward([(W, b)], cache, dY)
    R = 2.0 * (X @ W.T + b - T) / (9 * 5)
    assert np.allclose(dW, R.T @ X, rtol=0, atol=1e-14)
    assert np.allclose(db, R.sum(0), rtol=0, atol=1e-14)


def test_silu_and_derivative():
    z = np.linspace(-6, 6, 41)
    assert np.allclose(mlp.silu(z), z * (1 / (1 + np.exp(-z))), atol=1e-15)
    h = 1e-6
    fd = (mlp.silu(z + h) - mlp.silu(z - h)) / (2 * h)
    assert np.max(np.abs(fd - mlp.silu_grad(z))) < 1e-9
    assert mlp.silu(0.0) == 0.0 and abs(mlp.silu_grad(0.0) - 0.5) < 1e-16


def test_adam_first_step_closed_form():
    g = np.array([0.3, -2.0, 1e-9, 0.0])
    th, m, v = mlp.adam(np.zeros(4), np.zeros(4), np.zeros(4), g, lr=1e-3, b1=0.9, b2=0.999, eps=1e-8, t=1)
    want = -1e-3 * g / (np.abs(g) + 1e-8)
    assert np.allclose(th, want, rtol=1e-12, atol=0)
    assert np.allclose(m, 0.1 * g) and np.allclose(v, 0.001 * g * g)


def test_features_targets_round_trip():
    f = mlp.features(0.5, 0.1, 4, 3, 2)
    assert f.shape == (2, 3, 4, 5)
    assert f[0, 0, 0, 0] == (0.5 - 0.675) / 0.175 and abs(f[0, 0, 0, 1] - 1.0) < 1e-15
    assert abs(f[1, 2, 3, 2] - (2 * 3.5 / 4 - 1)) < 1e-15 and abs(f[1, 2, 3, 4] - 0.5) < 1e-15
    rng = np.random.default_rng(3)
    rho = rng.uniform(0.8, 1.2, 10)
    u, v, w = rng.uniform(-0.3, 0.9, (3, 10))
    p = rng.uniform(0.8, 1.2, 10)
    q = cases.conserved_from(rho, u, v, w, p, 1.4)
    t = mlp.targets(q, 0.7)
    assert np.allclose(t[:, 1], u - 0.7 * math.sqrt(1.4), atol=1e-14)
    assert np.allclose(mlp.conserved_from_output(t, 0.7), q, rtol=1e-14, atol=1e-14)
