"""GPU parity on the edge cases of the method, against the FP64 oracle.

- thinnest blocks: a periodic curvilinear box split into 32 blocks two cells
  thick (the ghost depth) in every direction, so every ghost layer of every
  block comes from a neighbour's full extent;
- supersonic far field (M = 1.6): both supersonic branches of the
  characteristic boundary state (inflow takes the freestream, outflow the
  interior);
- a strong shock tube (pressure and density ratios 1e3) along j, which
  drives the limiter far from smooth data;
- a walled box: slip walls on the i-faces and no-slip walls on the j-faces of
  a curvilinear grid, periodic in k, with a pressure pulse (wall ghosts on
  the i-faces, where each ghost layer has its own lane).

Every case runs on the default kernel, on the tiled kernel with two-row tiles
and on the plane-ring kernel, at the FP64 parity bar of the other step tests.
"""
import numpy as np
import pytest

from gpu_util import max_rel, oracle_steps, rel_l2, say
from paper_1710_09995_amd import cases

pytestmark = pytest.mark.gpu

TUNINGS = {"default": None, "tiled2": {"kernel": 0, "tile_j": 2, "tile_k": 3},
           "ring": {"kernel": 2, "tile_j": 8, "tile_k": 3}}


def thin_blocks():
    base = cases.vortex_case(8, nz=4, seed=7, curvilinear=True)
    return cases.split_periodic_box(base, parts=(4, 4, 2))      # 32 blocks of 2 x 2 x 2


def supersonic():
    return cases.bump_ns_case(40, 12, 8, seed=8, mach=1.6, reynolds=5e3)


def shock_tube():
    dims = (6, 40, 4)
    X = cases.cartesian_nodes(dims, h=(1.0 / 6, 1.0 / 40, 1.0 / 4))
    C = cases.centroids(X)
    left = C[1] < 0.5
    rho = np.where(left, 1.0, 1e-3)
    p = np.where(left, 1.0, 1e-3)
    zero = np.zeros_like(rho)
    q = cases.conserved_from(rho, zero, zero, zero, p, 1.4)
    conns = cases.periodic_pair(0, dims, 0, 1.0) + cases.periodic_pair(0, dims, 2, 1.0)
    bcs = [cases.full_bc(0, dims, 2, cases.EXTRAP), cases.full_bc(0, dims, 3, cases.EXTRAP)]
    par = cases.Params(cfl=0.4, mach=0.0)
    return cases.Case("shock_tube", par, [dims], [X], conns, bcs, [q])


def walled_box():
    dims = (20, 14, 6)
    X = cases.cartesian_nodes(dims, h=(1.0 / 20, 1.0 / 14, 1.0 / 6))
    X[0] = X[0] + 0.01 * np.sin(2 * np.pi * X[1]) * np.sin(2 * np.pi * X[2])
    X[1] = X[1] + 0.01 * np.sin(2 * np.pi * X[0]) * np.sin(2 * np.pi * X[2])
    par = cases.Params(cfl=0.5, mach=0.3, viscous=1, reynolds=2e3, alpha=0.3)
    q = cases.pressure_pulses(cases.centroids(X), [(0.4, 0.5, 0.5)], 0.05, 0.12, par)
    conns = cases.periodic_pair(0, dims, 2, 1.0)
    bcs = [cases.full_bc(0, dims, 0, cases.SLIPWALL), cases.full_bc(0, dims, 1, cases.SLIPWALL),
           cases.full_bc(0, dims, 2, cases.NOSLIP_ADIABATIC), cases.full_bc(0, dims, 3, cases.NOSLIP_ADIABATIC)]
    return cases.Case("walled_box", par, [dims], [X], conns, bcs, [q])


CASES = {"thin_blocks": thin_blocks, "supersonic": supersonic, "shock_tube": shock_tube, "walled_box": walled_box}


@pytest.mark.parametrize("tun", list(TUNINGS))
@pytest.mark.parametrize("name,nsteps", [("thin_blocks", 6), ("supersonic", 5), ("shock_tube", 12),
                                         ("walled_box", 8)])
def test_edge_case_step_parity(name, nsteps, tun):
    from paper_1710_09995_amd.binding import Solver
    case = CASES[name]()
    say("edge", name, tun, "blocks", case.nblk, "dims", case.dims[0])
    s = Solver(case, tuning=TUNINGS[tun])
    h = s.step(nsteps).cpu().numpy()
    got = s.state()
    want, rows = oracle_steps(case, nsteps)
    err, emax = rel_l2(got, want), max_rel(got, want)
    say("  rel L2", err, "max element", emax)
    assert err <= 1e-12
    assert emax <= 1e-12        # an error confined to a few cells, which the L2 would dilute
    rows = np.array(rows)
    assert np.max(np.abs(h[:, 0] - rows[:, 0]) / rows[:, 0]) <= 1e-13
    assert np.all(np.isfinite(h))
    s.close()


def test_thin_blocks_metrics_and_ghosts():
    """Metrics and one ghost fill of the 2 x 2 x 2 blocks: the ghost copies
    across connections are bitwise; metrics agree to rounding."""
    from oracle import geometry as ogeo
    from oracle import solver as osol
    from paper_1710_09995_amd.binding import Solver
    case = thin_blocks()
    s = Solver(case)
    _, Ss, Vs = ogeo.build_metrics(case, 2)
    for b in range(case.nblk):
        m = s.metrics(b)
        S = Ss[b].reshape(9, *Ss[b].shape[2:])
        assert np.max(np.abs(m[:9] - S)) <= 4e-15 * np.max(np.abs(S)), b
        assert np.max(np.abs(m[9] - Vs[b]) / np.abs(Vs[b])) <= 1e-13, b
    s.fill_ghosts()
    got = [v.cpu().numpy() for v in s.views()]
    st = osol.setup(case)
    osol.fill(st)
    for b in range(case.nblk):
        assert np.array_equal(got[b], st.Qs[b]), b
    s.close()


@pytest.mark.parametrize("which", ["channel", "chain", "thin"])
@pytest.mark.parametrize("tuning", list(TUNINGS))
def test_inviscid_steps_never_read_edge_or_corner_ghosts(which, tuning):
    """Inviscid steps fill each face's ghost layers over the face's own cells
    only, so the edge and corner ghost cells keep whatever they held.  Poison
    test: from a state arena whose every ghost cell is NaN, and from one whose
    ghosts (edges and corners included) were filled by cfd_fill_ghosts' sweeps,
    5 steps give bitwise the same history rows and interior states, all
    finite: no inviscid stencil, time step or norm reads those cells."""
    import torch
    from paper_1710_09995_amd.binding import Solver
    case = {"channel": lambda: cases.channel_case(24, 12, 12, mach=0.6, hb=0.05),
            "chain": lambda: cases.batched_euler_case(nblk=5, seed=3, lo=8, hi=20, flux_fp32=0),
            "thin": lambda: cases.split_periodic_box(cases.vortex_case(8, nz=4, seed=7, curvilinear=True),
                                                     parts=(4, 4, 2))}[which]()
    assert not case.params.viscous
    say("edge/corner ghost poison", which, tuning)
    s = Solver(case)
    if TUNINGS[tuning]:
        s.set_tuning(**TUNINGS[tuning])
    runs = []
    for prefill in (False, True):
        a = s.new_arena()                       # every entry NaN
        s.set_state(case.q0, a)
        if prefill:
            s.fill_ghosts(a)
        h = s.step(5, hist=True, arena=a)
        q = [v.clone() for v in s.interior_views(a)]
        runs.append((h, q))
    (h0, q0), (h1, q1) = runs
    assert bool(torch.isfinite(h0).all()) and all(bool(torch.isfinite(v).all()) for v in q0)
    assert torch.equal(h0, h1)
    assert all(torch.equal(x, y) for x, y in zip(q0, q1))
