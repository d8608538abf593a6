"""Pins of the oracle's implicit step on the finite-volume residual (the
reading of the linear solve that Section 2.3's flowchart names without a
method; oracle/implicit.py):

* backward Euler's first-order limit, dQ = -dt R + O(dt^2);
* a uniform stream on a curvilinear periodic grid stays uniform;
* the point-Jacobi sweeps reach their fixed point;
* the operator read off the sweeps as a black box equals V/dt plus the
  Jacobian of a first-order local Lax-Friedrichs residual with frozen
  dissipation, written here from its definition and differentiated by central
  differences (inviscid and viscous);
* a periodic box cut into 8 blocks gives bitwise the unsplit box's steps;
* the steady state of a channel reached by implicit steps is the one the
  explicit RK3 march of Eqs. 4-6 reaches (R = 0 does not depend on the
  solver), in far fewer steps.
"""
import math

import numpy as np
import pytest

from oracle import implicit as oim
from oracle import solver as osol
from paper_1710_09995_amd import cases


def _vortex(viscous=False, n=10, nz=6):
    c = cases.vortex_case(n, seed=3, nz=nz, curvilinear=True)
    if viscous:
        c = c.with_params(viscous=1, reynolds=50.0)
    return c


def _channel(n=(16, 8, 4), cfl=1.0):
    return cases.channel_case(*n, mach=0.58, hb=0.08, cfl=cfl).with_params(limiter_eps=1e-4)


def _rhs_and_dts(st):
    c = st.case
    R = osol.residual(st)
    dts = [osol.local_dt_block(st.Qs[b], st.Ss[b], st.Vs[b], c.dims[b], c.params, st.g) for b in range(c.nblk)]
    if not c.params.local_dt:
        dts = min(float(x.min()) for x in dts)
    rhs = [-osol.interior(st.Vs[b], c.dims[b], st.g) * R[b] for b in range(c.nblk)]
    return R, rhs, dts


@pytest.mark.parametrize("name", ["vortex", "vortex_ns", "channel"])
def test_explicit_euler_limit(name):
    """|dQ + dt R| / (dt max|R|) falls tenfold per tenfold smaller step."""
    rel = []
    for cfl in (1e-2, 1e-3, 1e-4):
        base = {"vortex": _vortex(), "vortex_ns": _vortex(True), "channel": _channel()}[name]
        st = osol.setup(base.with_params(cfl=cfl))
        R, rhs, dts = _rhs_and_dts(st)
        dQ, _ = oim.implicit_sweeps(st, st.Qs, rhs, dts, 3)
        num = max(float(np.max(np.abs(d + (t if not isinstance(dts, float) else dts) * r)))
                  for d, r, t in zip(dQ, R, dts if isinstance(dts, list) else [dts] * len(R)))
        den = max(float(np.max(np.abs((t if not isinstance(dts, float) else dts) * r)))
                  for r, t in zip(R, dts if isinstance(dts, list) else [dts] * len(R)))
        rel.append(num / den)
    assert rel[0] < 0.05 and 8.0 < rel[0] / rel[1] < 12.0 and 8.0 < rel[1] / rel[2] < 12.0, rel


def test_uniform_stream_stays_uniform():
    c = _vortex().with_params(cfl=50.0)
    q = cases.uniform_state(c.dims[0], c.params)
    c = cases.Case(c.name, c.params, c.dims, c.nodes, c.conns, c.bcs, [q])
    st = osol.setup(c)
    for _ in range(3):
        oim.implicit_step(st, 4)
    got = osol.interior_state(st, 0)
    assert np.max(np.abs(got - q)) <= 1e-12 * np.max(np.abs(q))


def test_sweeps_reach_their_fixed_point():
    """At CFL 2 (local steps) 80 sweeps reach the relaxation's fixed point: one
    more changes nothing at 1e-13 of max |dQ|.  (The contraction slows as the
    step grows, as point relaxation does, but stays below 1: measured per
    sweep about 0.63 at CFL 2 and 0.9 at CFL 10^4.)"""
    st = osol.setup(_channel(cfl=2.0).with_params(local_dt=1))
    _, rhs, dts = _rhs_and_dts(st)
    a, _ = oim.implicit_sweeps(st, st.Qs, rhs, dts, 80)
    b, _ = oim.implicit_sweeps(st, st.Qs, rhs, dts, 81)
    assert np.max(np.abs(a[0] - b[0])) <= 1e-13 * np.max(np.abs(a[0]))


def _llf_times_volume(st, Qpad_list, mu_frozen):
    """V R1: the first-order local Lax-Friedrichs residual, face flux
    (F(Q_L) + F(Q_R)) . S / 2 - mu (Q_R - Q_L), summed over each cell's faces
    with the outward sign; ghost cells as filled (periodic copies here)."""
    c = st.case
    g = st.g
    gam = c.params.gamma
    out = []
    for b in range(c.nblk):
        n = c.dims[b]
        acc = 0.0
        for d in range(3):
            Sf = osol.window(st.Ss[b][d], n, d, (0, 0, 0), g)
            QL = osol.window(Qpad_list[b], n, d, osol.unit(d, -1), g)
            QR = osol.window(Qpad_list[b], n, d, (0, 0, 0), g)

            def fdot(Q):
                rho = Q[0]
                u, v, w = Q[1] / rho, Q[2] / rho, Q[3] / rho
                p = (gam - 1.0) * (Q[4] - 0.5 * rho * (u * u + v * v + w * w))
                U = u * Sf[0] + v * Sf[1] + w * Sf[2]
                return np.stack([rho * U, Q[1] * U + p * Sf[0], Q[2] * U + p * Sf[1], Q[3] * U + p * Sf[2],
                                 (Q[4] + p) * U])
            Fh = 0.5 * (fdot(QL) + fdot(QR)) - mu_frozen[b][d] * (QR - QL)
            ax = Fh.ndim - 1 - d
            acc = acc + (np.take(Fh, np.arange(1, n[d] + 1), axis=ax) - np.take(Fh, np.arange(0, n[d]), axis=ax))
        out.append(acc)
    return out


def _mu_from_definition(st):
    """The frozen dissipation coefficient, from its definition: half the
    spectral radius |u . S| + c |S| of the mean primitive state of the face's
    two cells, plus for viscous flow max(4/3, gamma/Pr) (mean mu/rho) |S|^2 /
    (mean V)."""
    c = st.case
    p = c.params
    out = []
    for b in range(c.nblk):
        n = c.dims[b]
        Q = st.Qs[b]
        rho = Q[0]
        u, v, w = Q[1] / rho, Q[2] / rho, Q[3] / rho
        pr = (p.gamma - 1.0) * (Q[4] - 0.5 * rho * (u * u + v * v + w * w))
        mus = []
        for d in range(3):
            def side(a, off):
                return osol.window(a, n, d, off, st.g)
            L, R = osol.unit(d, -1), (0, 0, 0)
            um = [0.5 * (side(x, L) + side(x, R)) for x in (u, v, w)]
            rm, pm = 0.5 * (side(rho, L) + side(rho, R)), 0.5 * (side(pr, L) + side(pr, R))
            Sf = side(st.Ss[b][d], R)
            area = np.sqrt(Sf[0] ** 2 + Sf[1] ** 2 + Sf[2] ** 2)
            mu = 0.5 * (np.abs(um[0] * Sf[0] + um[1] * Sf[1] + um[2] * Sf[2]) + np.sqrt(p.gamma * pm / rm) * area)
            if p.viscous:
                mu_inf = p.mach * math.sqrt(p.gamma) / p.reynolds

                def nu(a):
                    T = side(pr, a) / side(rho, a)
                    return mu_inf * T ** 1.5 * (1.0 + p.sutherland) / (T + p.sutherland) / side(rho, a)
                vm = 0.5 * (side(st.Vs[b], L) + side(st.Vs[b], R))
                mu = mu + max(4.0 / 3.0, p.gamma / p.prandtl) * 0.5 * (nu(L) + nu(R)) * area ** 2 / vm
            mus.append(mu)
        out.append(mus)
    return out


@pytest.mark.parametrize("viscous", [False, True])
@pytest.mark.parametrize("split", [False, True])
def test_operator_is_the_frozen_llf_jacobian(viscous, split):
    """The operator L(dQ) = D dQ + O(dQ) read off the sweeps (zero sweeps from
    dQ = rhs / D give D; one sweep from rhs = D dQ gives D (2 dQ - dQ_1))
    equals V/dt + d(V R1)/dQ, R1 the frozen-dissipation local Lax-Friedrichs
    residual; its central difference agrees to O(|dQ|^2) (1e-8 at 1e-4 |Q|),
    also with the box cut into 8 blocks joined face to face."""
    c = _vortex(viscous).with_params(cfl=5.0)
    if split:
        c = cases.split_periodic_box(c, (2, 2, 2))
    st = osol.setup(c)
    osol.fill(st)
    _, _, dts = _rhs_and_dts(st)
    ones = [np.ones_like(osol.interior(Q, c.dims[b], st.g)) for b, Q in enumerate(st.Qs)]
    dq0, _ = oim.implicit_sweeps(st, st.Qs, ones, dts, 0)
    D = [o / x for o, x in zip(ones, dq0)]
    vol = [osol.interior(st.Vs[b], c.dims[b], st.g) for b in range(c.nblk)]
    assert all(np.all(d > v / t) for d, v, t in zip(D, vol, dts if isinstance(dts, list) else [dts] * c.nblk))

    def L_oracle(dq):
        dq1, _ = oim.implicit_sweeps(st, st.Qs, [d * x for d, x in zip(D, dq)], dts, 1)
        return [d * (2.0 * x - y) for d, x, y in zip(D, dq, dq1)]

    rng = np.random.default_rng(5)
    vdir = [rng.uniform(-1.0, 1.0, x.shape) * np.abs(osol.interior(Q, c.dims[b], st.g)).max(axis=(1, 2, 3),
                                                                                          keepdims=True)
            for b, (x, Q) in enumerate(zip(ones, st.Qs))]
    mu_def = _mu_from_definition(st)

    def VR1(sign, h):
        Qp = [Q.copy() for Q in st.Qs]
        for b in range(c.nblk):
            osol.interior(Qp[b], c.dims[b], st.g)[...] += sign * h * vdir[b]
        osol.fill(st, Qp)
        return _llf_times_volume(st, Qp, mu_def)
    h = 1e-5
    plus, minus = VR1(1.0, h), VR1(-1.0, h)
    dt_list = dts if isinstance(dts, list) else [dts] * c.nblk
    L_ref = [v / t * x + (p - m) / (2.0 * h) for v, t, x, p, m in zip(vol, dt_list, vdir, plus, minus)]
    scale = max(float(np.abs(x).max()) for x in L_ref)
    eta = 1e-4
    lp, lm = L_oracle([eta * x for x in vdir]), L_oracle([-eta * x for x in vdir])
    err = max(float(np.abs((a - b) / (2.0 * eta) - r).max()) for a, b, r in zip(lp, lm, L_ref)) / scale
    assert err <= 1e-8, err


def test_split_box_steps_bitwise_equal_the_unsplit_box():
    c = _vortex(n=12, nz=8).with_params(cfl=5.0, local_dt=1)
    whole = osol.setup(c)
    split = cases.split_periodic_box(c, (2, 2, 2))
    parts = osol.setup(split)
    for _ in range(2):
        oim.implicit_step(whole, 4)
        oim.implicit_step(parts, 4)
    W = osol.interior_state(whole, 0)
    for b, m in enumerate(split.dims):          # blocks numbered i fastest, then j, then k
        o = ((b % 2) * m[0], (b // 2 % 2) * m[1], (b // 4) * m[2])
        got = osol.interior_state(parts, b)
        assert np.array_equal(got, W[:, o[2]:o[2] + m[2], o[1]:o[1] + m[1], o[0]:o[0] + m[0]]), b


def test_channel_steady_state_matches_the_rk3_march():
    """A subsonic channel (16 x 8 x 4, limiter eps 1e-4, local steps):
    implicit steps at CFL 50 with 10 sweeps bring L2(R_rho) below 1e-10 of the
    initial value; the explicit RK3 march at CFL 1 needs more than five times
    as many steps to reach 1e-8 (measured: about 250 against 2,750), and its
    state there equals the implicit steady state to 1e-7 of max |Q| (R = 0
    does not depend on the solver)."""
    st = osol.setup(_channel(cfl=50.0).with_params(local_dt=1))
    r0, n8_impl = None, None
    for n in range(1, 500):
        row = oim.implicit_step(st, 10, record=True)
        r0 = row[1] if r0 is None else r0
        if n8_impl is None and row[1] < 1e-8 * r0:
            n8_impl = n
        if row[1] < 1e-10 * r0:
            break
    assert row[1] < 1e-10 * r0 and n8_impl is not None
    q_impl = osol.interior_state(st, 0)
    se = osol.setup(_channel(cfl=1.0).with_params(local_dt=1))
    n_rk = None
    for m in range(1, 20001):
        rec = m % 50 == 1
        row = osol.step(se, record=rec)
        if rec and row[1] < 1e-8 * r0:
            n_rk = m
            break
    assert n_rk is not None and n_rk > 5 * n8_impl, (n_rk, n8_impl)
    q_rk = osol.interior_state(se, 0)
    assert np.max(np.abs(q_impl - q_rk)) <= 1e-7 * np.max(np.abs(q_rk))
