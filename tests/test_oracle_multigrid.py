"""Pins of the oracle's multigrid cycle (full approximation storage with RK3
smoothing; oracle/multigrid.py):

* one level is the plain RK3 march of Eqs. 4-6: bitwise the solver's steps,
  history rows included;
* the restriction keeps sum V Q where the coarse volumes are the sums of the
  fine ones (a Cartesian box);
* on a periodic box a whole cycle keeps the conserved totals (the forcing
  sums to zero over the coarse grid, the injected correction adds what the
  coarse steps changed);
* the cycles converge to the state the explicit RK3 march converges to
  (R = 0 does not depend on the solver; a wrong forcing on any level
  converges elsewhere or not at all), in fewer fine-grid steps.
The scale of the injected correction and the volume weights of the
restricted residual change how fast the cycles converge, not where they
converge; nothing independent fixes them (a halved correction or unweighted
restriction passes these pins): parity unpinned for those two choices.
"""
import numpy as np

from oracle import multigrid as omg
from oracle import solver as osol
from paper_1710_09995_amd import cases


def _channel():
    return cases.channel_case(16, 8, 4, mach=0.58, hb=0.08, cfl=1.0)


def _box():
    return cases.vortex_case(16, seed=2, nz=8, cfl=0.5)


def test_one_level_is_plain_rk3():
    for case in (_channel(), cases.bump_ns_case(12, 8, 4, seed=2, noise=1e-3, reynolds=5e3)):
        a = osol.setup(case)
        b = omg.setup_levels([case])
        rows_a = [osol.step(a, record=True)] + [osol.step(a) for _ in range(2)]
        row_b = omg.v_cycle(b, pre=1, coarse=3)
        assert rows_a[0] == row_b
        for qa, qb in zip(a.Qs, b[0].Qs):
            assert np.array_equal(osol.interior(qa, case.dims[0], a.g), osol.interior(qb, case.dims[0], a.g))


def test_restriction_keeps_the_totals():
    case = _box()
    lv = omg.setup_levels(cases.hierarchy(case, 2))
    st, cn = lv
    rng = np.random.default_rng(1)
    for Q in st.Qs:
        Q *= 1.0 + 0.01 * rng.standard_normal(Q.shape)
    omg.restrict(st, cn, None)
    tot_f = osol.norms_from(st, st.Qs, None)[5:10]
    tot_c = osol.norms_from(cn, cn.Qs, None)[5:10]
    assert np.allclose(tot_c, tot_f, rtol=1e-13, atol=0.0)


def test_cycle_keeps_the_totals_on_a_periodic_box():
    case = _box()
    lv = omg.setup_levels(cases.hierarchy(case, 2))
    before = osol.norms_from(lv[0], lv[0].Qs, None)[5:10]
    for _ in range(3):
        omg.v_cycle(lv, pre=1, coarse=2)
    after = osol.norms_from(lv[0], lv[0].Qs, None)[5:10]
    scale = max(abs(x) for x in before)
    assert max(abs(a - b) for a, b in zip(after, before)) <= 1e-12 * scale


def test_cycles_reach_the_rk3_steady_state():
    """Subsonic channel 16 x 8 x 4 (local steps, CFL 1): three-level cycles
    bring L2(R_rho) below 1e-10 of its initial value (measured: 551 cycles;
    at most 600 allowed), the RK3 march below 1e-8 (about 2,750 steps), and
    the two states agree to 1e-7 of max |Q|."""
    case = _channel()
    lv = omg.setup_levels(cases.hierarchy(case, 3))
    r0 = None
    for n in range(1, 1201):
        row = omg.v_cycle(lv, pre=1, coarse=2)
        r0 = row[1] if r0 is None else r0
        if row[1] < 1e-10 * r0:
            break
    assert row[1] < 1e-10 * r0, row[1] / r0
    n_mg = n
    assert n_mg <= 600, n_mg
    q_mg = osol.interior_state(lv[0], 0)
    se = osol.setup(case)
    n_rk = None
    for m in range(1, 20001):
        rec = m % 50 == 1
        row = osol.step(se, record=rec)
        if rec and row[1] < 1e-8 * r0:
            n_rk = m
            break
    assert n_rk is not None and n_rk > 2 * n_mg, (n_rk, n_mg)
    q_rk = osol.interior_state(se, 0)
    assert np.max(np.abs(q_mg - q_rk)) <= 1e-7 * np.max(np.abs(q_rk))
