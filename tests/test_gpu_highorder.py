"""GPU parity of the sixth-order staggered flux difference (Section 2.2,
Eq. 2) through the C ABI, against the FP64 oracle on the same seeded face
fields: every direction, ragged extents, one cell along the direction, one
variable; at a full block size by sampled cells; and the exactness on
polynomials up to degree 6 that pins the oracle, on the GPU's own output.

Tolerance: the kernel may fuse the three products into FMAs, the oracle
rounds each; the terms reach about 2.7 max|F| / h and a few roundings
differ, so the bar is 4e-15 * max|F| / h (a few ulps of the largest term)."""
import numpy as np
import pytest

from gpu_util import say
from oracle import highorder as ho

pytestmark = pytest.mark.gpu


def _field(n, d, nvar, seed):
    rng = np.random.default_rng(seed)
    shape = [nvar, n[2], n[1], n[0]]
    shape[3 - d] += 5
    return rng.uniform(-1.0, 1.0, shape)


def _run(f, n, d, h):
    import torch
    from paper_1710_09995_amd.binding import staggered_diff6
    ft = torch.from_numpy(f).cuda()
    out = staggered_diff6(ft, n, d, h)
    torch.cuda.synchronize()
    return out.cpu().numpy()


@pytest.mark.parametrize("d", [0, 1, 2])
@pytest.mark.parametrize("n,nvar", [((37, 11, 9), 5), ((64, 8, 4), 5), ((130, 3, 2), 1), ((5, 7, 1), 3),
                                    ((1, 1, 1), 5)])
def test_parity_with_oracle(n, nvar, d):
    h = 0.037
    f = _field(n, d, nvar, seed=hash((n, d, nvar)) % 1000)
    say("diff6", n, d, nvar)
    got = _run(f, n, d, h)
    want = ho.staggered_diff6(f, d, h)
    assert got.shape == want.shape
    assert np.max(np.abs(got - want)) <= 4e-15 * np.max(np.abs(f)) / h


@pytest.mark.parametrize("d", [0, 1, 2])
def test_full_block_sampled(d):
    """A 256 x 128 x 128 block, 5 variables (the size the benchmark times):
    sampled cells against the oracle's formula evaluated at those cells only."""
    import torch
    from paper_1710_09995_amd.binding import staggered_diff6
    n = (256, 128, 128)
    shape = [5, n[2], n[1], n[0]]
    shape[3 - d] += 5
    g = torch.Generator(device="cuda").manual_seed(7 + d)
    ft = torch.rand(shape, dtype=torch.float64, device="cuda", generator=g) * 2 - 1
    h = 0.01
    out = staggered_diff6(ft, n, d, h).cpu().numpy()
    f = ft.cpu().numpy()
    rng = np.random.default_rng(d)
    idx = [rng.integers(0, m, 2000) for m in (5, n[2], n[1], n[0])]
    ax = 3 - d
    vals = []
    for s in range(6):
        ii = list(idx)
        ii[ax] = ii[ax] + s
        vals.append(f[tuple(ii)])
    want = (ho.C1 / h) * (vals[3] - vals[2]) + (ho.C2 / h) * (vals[4] - vals[1]) + (ho.C3 / h) * (vals[5] - vals[0])
    got = out[tuple(idx)]
    assert np.max(np.abs(got - want)) <= 4e-15 / h


@pytest.mark.parametrize("d", [0, 1, 2])
def test_exact_on_polynomials_gpu(d):
    n = (12, 10, 9)
    h = 0.1
    for p in range(7):
        xf = 0.35 + (np.arange(-2, n[d] + 3) - 0.5) * h
        shape = [2, n[2], n[1], n[0]]
        shape[3 - d] += 5
        sh = [1, 1, 1, 1]
        sh[3 - d] = n[d] + 5
        f = np.ascontiguousarray(np.broadcast_to((xf ** p).reshape(sh), shape))
        got = _run(f, n, d, h)
        xc = 0.35 + np.arange(n[d]) * h
        want = (p * xc ** (p - 1) if p else 0 * xc)
        sh[3 - d] = n[d]
        assert np.max(np.abs(got - want.reshape(sh))) <= 1e-12 * max(1.0, p * np.max(np.abs(xc)) ** max(p - 1, 0))
