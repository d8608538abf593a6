"""GPU parity of the multigrid cycles (cfd_mg_cycles: full approximation
storage, RK3 smoothing, volume-weighted restriction, injected corrections)
against the oracle's cycles (oracle/multigrid.py) through the C ABI: a
subsonic channel on three levels (far field, slip walls, local steps), the
wall-bump Navier-Stokes block on two (no-slip wall, global step) and a
periodic box cut into 8 blocks on two.  The state after the cycles is held to
the FP64 gate (relative L2 and element-wise max within 1e-12 of max |Q|) and
the history rows as the RK3 tests hold them; then on a 48 x 24 x 24 channel
the cycles reach a 1e-8 drop in less wall time than the RK3 march.
"""
import time

import numpy as np
import pytest

from gpu_util import max_rel, rel_l2, say
from oracle import multigrid as omg
from oracle import solver as osol
from paper_1710_09995_amd import cases

pytestmark = pytest.mark.gpu


def _cases():
    return {
        "channel": (cases.channel_case(32, 16, 8, mach=0.58, hb=0.08), 3, 1, 2, 4),
        "bump_ns": (cases.bump_ns_case(16, 16, 8, seed=3, noise=1e-3, reynolds=5e3), 2, 1, 2, 3),
        "split_box": (cases.split_periodic_box(cases.vortex_case(16, nz=8, seed=2, curvilinear=True), (2, 2, 2))
                      .with_params(local_dt=1), 2, 1, 2, 3),
    }


@pytest.mark.parametrize("name", ["channel", "bump_ns", "split_box"])
def test_cycles_match_the_oracle(name):
    from paper_1710_09995_amd.binding import Multigrid, Solver
    case, L, pre, coarse, n = _cases()[name]
    say("multigrid", name, "levels", L, "cycles", n)
    s = Solver(case)
    mg = Multigrid(s, L, pre, coarse)
    h = mg.cycles(n).cpu().numpy()
    got = s.state()
    mg.close()
    s.close()
    lv = omg.setup_levels(cases.hierarchy(case, L))
    rows = np.array([omg.v_cycle(lv, pre, coarse) for _ in range(n)])
    want = osol.interior_state(lv[0])
    err, emax = rel_l2(got, want), max_rel(got, want)
    say(f"  rel L2 {err:.3e}, max element {emax:.3e}")
    assert err <= 1e-12 and emax <= 1e-12
    assert np.max(np.abs(h[:, 0] - rows[:, 0]) / rows[:, 0]) <= 1e-13
    l2_scale = np.abs(rows[:, 1:6]).max(axis=1, keepdims=True)
    assert np.max(np.abs(h[:, 1:6] - rows[:, 1:6]) / l2_scale) <= 1e-11
    tot_scale = np.abs(rows[:, 6:11]).max(axis=0) + np.abs(rows[:, 6:11]).max()
    assert np.max(np.abs(h[:, 6:11] - rows[:, 6:11]) / tot_scale) <= 1e-13


def test_cycles_reach_the_target_before_the_rk3_march():
    import torch
    from paper_1710_09995_amd.binding import Multigrid, Solver
    case = cases.channel_case(48, 24, 24, mach=0.58, hb=0.08)
    s = Solver(case)
    r0 = s.step(1, hist=True)[0, 1].item()
    s.set_state(case.q0)
    mg = Multigrid(s, 4, 1, 2)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    n_mg = None
    for k in range(40):
        r = mg.cycles(250)[:, 1].cpu().numpy()
        hit = np.nonzero(r < 1e-8 * r0)[0]
        if hit.size:
            n_mg = 250 * k + int(hit[0])
            break
    t_mg = time.perf_counter() - t0
    say(f"  multigrid: 1e-8 at cycle {n_mg}, {t_mg:.2f} s")
    mg.close()
    assert n_mg is not None
    s.set_state(case.q0)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    done = 0
    while done < 60000 and time.perf_counter() - t0 < t_mg:
        r = s.step(1000, hist=True)[:, 1].cpu().numpy()
        done += 1000
        if np.any(r < 1e-8 * r0):
            break
    say(f"  RK3 in the same wall time: {done} steps, drop {r[-1] / r0:.2e}")
    s.close()
    assert r[-1] > 1e-8 * r0


def test_captured_cycles_are_bitwise_the_eager_cycles():
    """The cycle replayed from its captured graph (the default) against the same
    cycles launched one by one (graphs off on the finest level): bitwise the
    same states and history rows after every call, with the program's own
    eager work (a residual evaluation) and synchronisations between the
    replays; a retuned coarse level makes the next call capture again."""
    import torch
    from paper_1710_09995_amd.binding import Multigrid, Solver
    case = cases.channel_case(32, 16, 8, mach=0.7, hb=0.06)
    sa, sb = Solver(case), Solver(case)
    sb.set_tuning(use_graph=0)
    ma, mb = Multigrid(sa, 3, 1, 2), Multigrid(sb, 3, 1, 2)
    for n in (3, 1, 4):
        ha, hb = ma.cycles(n), mb.cycles(n)
        torch.cuda.synchronize()
        assert torch.equal(ha, hb)
        for x, y in zip(sa.state(), sb.state()):
            assert np.array_equal(x, y)
        sa.residual()
        torch.cuda.synchronize()
    ma.levels[1].set_tuning(tile_k=16)
    mb.levels[1].set_tuning(tile_k=16)
    ha, hb = ma.cycles(2), mb.cycles(2)
    assert torch.equal(ha, hb)
    for x, y in zip(sa.state(), sb.state()):
        assert np.array_equal(x, y)
    for m in (ma, mb):
        m.close()
    sa.close()
    sb.close()


def test_coarse_levels_give_bitwise_the_same_cycles_on_every_stage_kernel():
    """A coarse level's forcing is applied inside the tiled and simple stage
    kernels and by a pass of its own after the plane-ring kernel, rounded the
    same way, and the states do not depend on the stage kernel or its tiles:
    cycles with the coarse levels on each of the three stage kernels give
    bitwise the same states and history rows, on the channel (local steps)
    and on the wall-bump Navier-Stokes block (global step)."""
    from paper_1710_09995_amd.binding import Multigrid, Solver
    tunings = ({"kernel": 0, "tile_j": 4, "tile_k": 1}, {"kernel": 1, "tile_j": 4, "tile_k": 8},
               {"kernel": 2, "tile_j": 8, "tile_k": 4})
    for name in ("channel", "bump_ns"):
        case, L, pre, coarse, n = _cases()[name]
        ref = None
        for tun in tunings:
            say("multigrid coarse levels", name, tun)
            s = Solver(case)
            mg = Multigrid(s, L, pre, coarse)
            for lv in mg.levels[1:]:
                lv.set_tuning(**tun)
            h = mg.cycles(n).cpu().numpy()
            q = s.state()
            mg.close()
            s.close()
            if ref is None:
                ref = (h, q)
                continue
            assert np.array_equal(h, ref[0]), (name, tun)
            for x, y in zip(q, ref[1]):
                assert np.array_equal(x, y), (name, tun)


def test_hierarchy_is_checked():
    """A level that is not the coarsening of the one above (same extents, or
    other flow parameters) is refused before anything runs."""
    import ctypes as C
    from paper_1710_09995_amd import binding as B
    from paper_1710_09995_amd.binding import Solver
    case = cases.channel_case(16, 8, 4, mach=0.6, hb=0.05)
    coarse = cases.coarsen_case(case)
    a, b, c = Solver(case), Solver(case), Solver(coarse.with_params(mach=0.61))
    nb = C.c_size_t()
    for pair, what in (((a, b), "twice"), ((a, c), "flow parameters")):
        lv = (C.c_void_p * 2)(*[s.ctx.value for s in pair])
        with pytest.raises(B.CfdError) as e:
            B._check(B.lib().cfd_mg_work_size(lv, 2, C.byref(nb)))
        assert e.value.status == -1 and what in str(e.value)
    for s in (a, b, c):
        s.close()
