"""GPU parity of split cases (Section 3.2.1): the library's split plan and
tables, run through the stage kernels, give bitwise the state of the unsplit
blocks, and both agree with the FP64 oracle on the unsplit case.  Covers
viscous walls and far field (bump), partial patches (uneven chain), and
periodic seams (curvilinear vortex), on the default and plane-ring kernels."""
import numpy as np
import pytest

from gpu_util import oracle_steps, rel_l2, say
from paper_1710_09995_amd import cases
from paper_1710_09995_amd import partition as part

pytestmark = pytest.mark.gpu

SPLITS = {
    "bump_ns": (lambda: cases.bump_ns_case(70, 20, 12, seed=3, noise=1e-3, reynolds=5e3), 2500, 4),
    "batched": (lambda: cases.batched_euler_case(nblk=5, seed=4, lo=6, hi=23, flux_fp32=0), 900, 4),
    "vortex_curv": (lambda: cases.vortex_case(20, nz=12, seed=2, curvilinear=True), 700, 6),
}
TUNINGS = {"default": None, "ring": {"kernel": 2, "tile_j": 8, "tile_k": 3}}


@pytest.mark.parametrize("tun", list(TUNINGS))
@pytest.mark.parametrize("name", list(SPLITS))
def test_split_case_bitwise_and_oracle(name, tun):
    from paper_1710_09995_amd.binding import Solver
    make, max_cells, nsteps = SPLITS[name]
    case = make()
    split, pieces = part.split_case(case, max_cells)
    say("split", name, tun, "pieces", len(pieces), "of", case.nblk, "blocks")
    assert len(pieces) > case.nblk
    s0 = Solver(case, tuning=TUNINGS[tun])
    h0 = s0.step(nsteps).cpu().numpy()
    q0 = s0.state()
    s0.close()
    s1 = Solver(split, tuning=TUNINGS[tun])
    h1 = s1.step(nsteps).cpu().numpy()
    q1 = part.assemble(case, pieces, s1.state())
    s1.close()
    for a, b in zip(q1, q0):
        assert np.array_equal(a, b)
    assert np.array_equal(h1[:, 0], h0[:, 0])                      # dt: a minimum, order-free
    l2 = np.abs(h0[:, 1:6]).max(axis=1, keepdims=True)              # sums in another order: rounding
    assert np.max(np.abs(h1[:, 1:6] - h0[:, 1:6]) / l2) <= 1e-13
    tot = np.abs(h0[:, 6:11]).max(axis=0) + np.abs(h0[:, 6:11]).max()
    assert np.max(np.abs(h1[:, 6:11] - h0[:, 6:11]) / tot) <= 1e-13
    assert np.array_equal(h1[:, 11], h0[:, 11])                    # max |R_rho|: order-free
    want, _ = oracle_steps(case, nsteps)
    err = rel_l2(q1, want)
    say("  rel L2 vs oracle", err)
    assert err <= 1e-12
