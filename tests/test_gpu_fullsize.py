"""GPU parity at the benchmark's full size and launch configuration.

The NS bump block of 256 x 128 x 128 cells (the bench workload) takes one
RK3 step on the GPU with the autotuned tiling.  The oracle cannot run the
whole block for a step in seconds, so it checks sampled outputs exactly:
the block is periodic in k, and after one step (three stages, MUSCL stencil
of two cells, one more for the viscous transverse stencil) a cell depends
only on cells within 7 planes in k.  A slab of the same grid and state with
7 extra planes on each side and extrapolated k faces therefore reproduces
the full block's result on its middle planes.  The global time step comes
from the oracle's per-cell steps over the whole block.
"""
import numpy as np
import pytest

from gpu_util import rel_l2, say
from oracle import solver as osol
from paper_1710_09995_amd import cases

pytestmark = pytest.mark.gpu

MARGIN = 7


def _slab(case, k0, width):
    ni, nj, nk = case.dims[0]
    ka, kb = k0 - MARGIN, k0 + width + MARGIN
    dims = (ni, nj, kb - ka)
    X = case.nodes[0][:, ka:kb + 1].copy()
    q = case.q0[0][:, ka:kb].copy()
    conns = cases.periodic_pair(0, dims, 0, 2.0)
    bcs = [cases.full_bc(0, dims, 2, cases.NOSLIP_ADIABATIC), cases.full_bc(0, dims, 3, cases.FARFIELD),
           cases.full_bc(0, dims, 4, cases.EXTRAP), cases.full_bc(0, dims, 5, cases.EXTRAP)]
    return cases.Case("slab", case.params, [dims], [X], conns, bcs, [q])


@pytest.mark.parametrize("flux", ["fp64", "fp32"])
def test_bump_ns_full_size_one_step(flux, tmp_path, monkeypatch):
    from paper_1710_09995_amd.autotune import autotune
    from paper_1710_09995_amd.binding import Solver
    monkeypatch.setenv("CFD_TUNE_CACHE", str(tmp_path / "tune.json"))
    case = cases.bump_ns_case(256, 128, 128, seed=0).with_params(flux_fp32=1 if flux == "fp32" else 0)
    say("full-size NS step", flux)
    s = Solver(case)
    res = autotune(s)
    say("  tuning", res["tuning"])
    h = s.step(1).cpu().numpy()[0]
    got = s.state()[0]
    s.close()
    full = osol.setup(case.with_params(flux_fp32=0))
    dt = osol.time_step(full)
    assert abs(h[0] - dt) <= 1e-14 * dt
    del full
    for k0, width in ((0 + MARGIN, 3), (61, 4), (128 - MARGIN - 3, 3)):
        slab = _slab(case.with_params(flux_fp32=0), k0, width)
        st = osol.setup(slab)
        osol.step(st, dt=dt)
        want = osol.interior_state(st, 0)[:, MARGIN:MARGIN + width]
        err = rel_l2([got[:, k0:k0 + width]], [want])
        say(f"  k0={k0} rel L2 {err:.3e}")
        assert err <= (1e-12 if flux == "fp64" else 1e-5)
