"""GPU checks of the warm-start network kernels against the FP64 oracle.

The GPU evaluates in BF16 (MFMA, FP32 accumulate), so the oracle is run on
the same BF16-rounded weights and inputs (rounded here, independently of the
library) and the outputs agree to the BF16 rounding of the hidden
activations: 2e-2 relative L2 for the forward pass, 3e-2 for gradients.
Adam and the state <-> feature conversions are FP32 / FP64 and agree to
float rounding."""
import math

import numpy as np
import pytest

from oracle import mlp as omlp
from paper_1710_09995_amd import cases

pytestmark = pytest.mark.gpu


def round_bf16(a):
    """Round to the nearest BF16 value (ties to even), returned as float64."""
    a = np.ascontiguousarray(np.asarray(a, dtype=np.float32))
    u = a.view(np.uint32).astype(np.uint64)
    u = (u + 0x7FFF + ((u >> 16) & 1)) >> 16
    return (u.astype(np.uint32) << 16).view(np.float32).astype(np.float64)


def _rel(a, b):
    return float(np.linalg.norm(np.ravel(a) - np.ravel(b)) / np.linalg.norm(np.ravel(b)))


def _net(seed=0, hidden=128, layers=4):
    return cases.mlp_init(5, hidden, layers, 5, seed=seed, out_scale=1.0)


def test_forward_matches_oracle():
    import torch
    from paper_1710_09995_amd.binding import Mlp
    params = _net()
    m = Mlp(params)
    rng = np.random.default_rng(1)
    X = rng.uniform(-1, 1, (1003, 5)).astype(np.float32)      # ragged: not a multiple of 16 or 64
    y = m.forward(torch.from_numpy(X).cuda()).cpu().numpy()
    pb = [(round_bf16(W), round_bf16(b)) for W, b in params]
    want, _ = omlp.forward(pb, round_bf16(X))
    err = _rel(y, want)
    print("forward rel L2", err)
    assert err <= 2e-2
    # gathered rows through an index array give the same outputs
    idx = rng.integers(0, 1003, 77).astype(np.int32)
    yi = m.forward(torch.from_numpy(X).cuda(), idx=torch.from_numpy(idx).cuda()).cpu().numpy()
    assert np.array_equal(yi, y[idx])


def test_backward_matches_oracle():
    import torch
    from paper_1710_09995_amd.binding import Mlp, unpack_params
    params = _net(seed=2)
    m = Mlp(params)
    rng = np.random.default_rng(3)
    X = rng.uniform(-1, 1, (517, 5)).astype(np.float32)
    T = rng.normal(0, 0.3, (517, 5)).astype(np.float32)
    xt, tt = torch.from_numpy(X).cuda(), torch.from_numpy(T).cuda()
    y, cache = m.forward(xt, cache=True)
    loss, dy = m.mse(y, tt)
    g = unpack_params(m.backward(cache, dy).cpu().numpy(), 5, 128, 4, 5)
    pb = [(round_bf16(W), round_bf16(b)) for W, b in params]
    Y, oc = omlp.forward(pb, round_bf16(X))
    l_ora, dY = omlp.mse(Y, T.astype(np.float64))
    assert abs(float(loss.item()) - l_ora) <= 2e-2 * l_ora
    want = omlp.backward(pb, oc, dY)
    for l, ((gw, gb), (ww, wb)) in enumerate(zip(g, want)):
        ew, eb = _rel(gw, ww), _rel(gb, wb)
        print("layer", l, "dW rel", ew, "db rel", eb)
        assert ew <= 3e-2 and eb <= 3e-2


def test_adam_matches_formula():
    import torch
    from paper_1710_09995_amd.binding import Mlp, pack_params
    params = _net(seed=4, hidden=16, layers=1)
    m = Mlp(params, d_hidden=16, n_hidden=1)
    rng = np.random.default_rng(5)
    theta = m.master.cpu().numpy().astype(np.float64)
    mom = np.zeros_like(theta)
    vel = np.zeros_like(theta)
    for t in range(1, 4):
        g = rng.normal(size=theta.size).astype(np.float32)
        m.grad.copy_(torch.from_numpy(g))
        m.adam(lr=1e-2)
        theta, mom, vel = omlp.adam(theta, mom, vel, g.astype(np.float64), 1e-2, 0.9, 0.999, 1e-8, t)
    got = m.master.cpu().numpy()
    assert np.max(np.abs(got - theta)) <= 1e-5 * max(1.0, np.max(np.abs(theta)))
    assert np.array_equal(m.bf16.cpu().numpy().view(np.uint16),
                          (round_bf16(got).astype(np.float32).view(np.uint32) >> 16).astype(np.uint16))
    del pack_params


def test_features_targets_state_round_trip():
    from paper_1710_09995_amd.binding import Solver
    conds = [(0.6, 0.05), (0.82, 0.09)]
    case = cases.channel_batch_case(conds, 20, 8, 6)
    s = Solver(case)
    x = s.mlp_features(conds).cpu().numpy()
    t = s.mlp_targets(conds).cpu().numpy()
    off = 0
    for b, (mch, hb) in enumerate(conds):
        n = 20 * 8 * 6
        f = omlp.features(mch, hb, 20, 8, 6).reshape(-1, 5)
        assert np.max(np.abs(x[off:off + n] - f)) <= 1e-6
        tw = omlp.targets(case.q0[b], mch).reshape(-1, 5)
        assert np.max(np.abs(t[off:off + n] - tw)) <= 1e-6
        off += n
    # outputs -> state: feeding the targets back reproduces the state to float rounding
    import torch
    arena = s.new_arena()
    s.mlp_to_state(torch.from_numpy(t).cuda(), conds, arena=arena)
    got = s.state(arena)
    for b in range(2):
        assert np.max(np.abs(got[b] - case.q0[b]) / np.abs(case.q0[b]).max()) <= 1e-6
    s.close()


def test_training_reduces_loss():
    import torch
    from paper_1710_09995_amd.binding import Mlp
    rng = np.random.default_rng(6)
    X = rng.uniform(-1, 1, (4096, 5)).astype(np.float32)
    T = np.stack([0.3 * np.sin(2 * X[:, 0] + X[:, 2]), 0.2 * X[:, 1] * X[:, 3], 0.1 * np.cos(3 * X[:, 4]),
                  0.05 * X[:, 0], 0.25 * np.tanh(X[:, 2] - X[:, 3])], axis=1).astype(np.float32)
    m = Mlp(cases.mlp_init(seed=7))
    xt, tt = torch.from_numpy(X).cuda(), torch.from_numpy(T).cuda()
    gen = torch.Generator(device="cuda").manual_seed(0)
    losses = []
    for it in range(300):
        idx = torch.randint(0, 4096, (512,), device="cuda", generator=gen, dtype=torch.int32)
        losses.append(float(m.train_step(xt, tt, idx, lr=2e-3).item()))
    print("loss", losses[0], "->", losses[-1])
    assert math.isfinite(losses[-1]) and np.mean(losses[-20:]) < 0.1 * np.mean(losses[:5])
