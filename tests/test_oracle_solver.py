"""Pins for the oracle's residual, time step, RK3 and norms (CPU only).

* RK3: the coefficients printed in Section 2.2 (golden fixture) and the
  stability polynomial 1 + z + z^2/2 + z^3/6 of Eqs. (4)-(6).
* Freestream preservation on curvilinear grids (Euler and Navier-Stokes).
* Conservation of totals to round-off on a periodic curvilinear box.
* Second-order convergence to the exact advected isentropic vortex.
* Sod's shock tube against an exact Riemann solution written here, along each
  index axis.
* Closed-form time step on a Cartesian grid; block-split invariance; norms.
"""
import math
import os
from fractions import Fraction

import numpy as np
import pytest

from oracle import solver
from paper_1710_09995_amd import cases

HERE = os.path.dirname(os.path.abspath(__file__))


def _golden(name):
    out = {}
    with open(os.path.join(HERE, "golden", name)) as f:
        for line in f:
            line = line.strip()
            if not line or line.startswith("#"):
                continue
            k, a, b = line.split()
            out[k] = Fraction(int(a), int(b))
    return out


def test_rk3_coefficients_match_paper():
    """Run the oracle's stage combination on a scalar linear problem and read the
    coefficients back exactly (rational arithmetic through Fraction)."""
    co = _golden("rk3_coefficients.txt")
    # R(q) = q with dt = 1 and lambda = -dt: Q1 = 0, Q2 = a2*q + b2*(0 - 0) ...
    q = Fraction(1)
    seen = []

    def R(x):
        seen.append(x)
        return Fraction(0)
    out = solver.ssp_rk3(q, Fraction(1), R)
    # with R = 0 the step must be the identity: a2 + b2 = 1 and a3 + b3 = 1
    assert out == 1
    # with R(x) = -x/dt the update is exp-like; compare with the golden coefficients
    z = Fraction(-1, 3)
    got = solver.ssp_rk3(Fraction(1), Fraction(1), lambda x: -z * x)
    q1 = 1 + z
    q2 = co["a2"] + co["b2"] * (q1 + z * q1)
    want = co["a3"] + co["b3"] * (q2 + z * q2)
    assert abs(float(got) - float(want)) < 1e-15


@pytest.mark.parametrize("z", [-0.1, -0.7, -1.3, -2.4])
def test_rk3_stability_polynomial(z):
    got = solver.ssp_rk3(1.0, 1.0, lambda x: -z * x)
    assert abs(got - (1 + z + z * z / 2 + z ** 3 / 6)) < 1e-15


@pytest.mark.parametrize("viscous", [0, 1])
def test_freestream_preserved_on_curvilinear_grid(viscous):
    c = cases.bump_ns_case(24, 16, 12, noise=0.0, viscous=viscous, amp=0.2, reynolds=1e3)
    c.bcs[0].kind = cases.FARFIELD          # far field all round, periodic in x and z
    st = solver.setup(c)
    R = solver.residual(st)[0]
    V = solver.interior(st.Vs[0], c.dims[0], 2)
    uinf = np.linalg.norm(cases.freestream_velocity(c.params))
    fscale = 1.0 + uinf * uinf              # |F_inf| scale (momentum flux)
    smax = max(np.max(np.linalg.norm(st.Ss[0][d], axis=0)[2:-2, 2:-2, 2:-2]) for d in range(3))
    assert np.max(np.abs(R * V)) / (fscale * smax) < 1e-13


def test_freestream_preserved_on_curvilinear_periodic_box():
    c = cases.vortex_case(12, curvilinear=True)
    c.q0[0][:] = cases.uniform_state(c.dims[0], c.params)
    R = solver.residual(solver.setup(c))[0]
    assert np.max(np.abs(R)) < 1e-13


def test_conservation_periodic_curvilinear():
    c = cases.vortex_case(12, curvilinear=True, seed=3)
    st = solver.setup(c)
    t0 = solver.norms_from(st, st.Qs, None)[5:10]
    for _ in range(20):
        solver.step(st)
    t1 = solver.norms_from(st, st.Qs, None)[5:10]
    V = solver.interior(st.Vs[0], c.dims[0], 2)
    mom_scale = float(np.sum(V * np.abs(c.q0[0][1])))     # w-momentum totals start at 0
    for comp, (a, b) in enumerate(zip(t0, t1)):
        scale = max(float(np.sum(V * np.abs(c.q0[0][comp]))), mom_scale)
        assert abs(a - b) <= 1e-13 * scale, comp


def test_vortex_second_order():
    errs = []
    for n in (16, 32, 64):
        c = cases.vortex_case(n, seed=0, nz=4)
        st = solver.setup(c)
        t, T = 0.0, 1.0
        while t < T - 1e-14:
            dt = min(solver.time_step(st), T - t)
            solver.step(st, dt=dt)
            t += dt
        q = solver.interior_state(st, 0)
        C = cases.centroids(c.nodes[0])
        u = cases.freestream_velocity(c.params)
        rho = cases.isentropic_vortex_primitives(C[0], C[1], c.info["xc"] + u[0] * T,
                                                 c.info["yc"] + u[1] * T, c.params, period=10.0)[0]
        errs.append(math.sqrt(np.mean((q[0] - rho) ** 2)))
    order = math.log2(errs[1] / errs[2])
    assert order >= 1.8, errs


# ---------------------------------------------------------------- Sod, exact Riemann

def _exact_riemann(rl, ul, pl, rr, ur, pr, x, t, g=1.4):
    """Textbook exact Riemann solution (two-rarefaction/shock pressure function + Newton)."""
    cl, cr = math.sqrt(g * pl / rl), math.sqrt(g * pr / rr)

    def f(p, rk, pk, ck):
        if p > pk:
            A = 2.0 / ((g + 1) * rk)
            B = (g - 1) / (g + 1) * pk
            return (p - pk) * math.sqrt(A / (p + B))
        return 2 * ck / (g - 1) * ((p / pk) ** ((g - 1) / (2 * g)) - 1)
    p = 0.5 * (pl + pr)
    for _ in range(100):
        h = 1e-8 * p
        F = f(p, rl, pl, cl) + f(p, rr, pr, cr) + ur - ul
        dF = (f(p + h, rl, pl, cl) + f(p + h, rr, pr, cr) - f(p - h, rl, pl, cl) - f(p - h, rr, pr, cr)) / (2 * h)
        dp = F / dF
        p = max(p - dp, 1e-12)
        if abs(dp) < 1e-15 * p:
            break
    us = 0.5 * (ul + ur) + 0.5 * (f(p, rr, pr, cr) - f(p, rl, pl, cl))
    out = np.empty((3, x.size))
    for n, xi in enumerate(x):
        s = xi / t
        if s <= us:   # left of contact
            if p > pl:
                sl = ul - cl * math.sqrt((g + 1) / (2 * g) * p / pl + (g - 1) / (2 * g))
                if s <= sl:
                    out[:, n] = (rl, ul, pl)
                else:
                    r = rl * ((p / pl + (g - 1) / (g + 1)) / ((g - 1) / (g + 1) * p / pl + 1))
                    out[:, n] = (r, us, p)
            else:
                shl = ul - cl
                cs = cl * (p / pl) ** ((g - 1) / (2 * g))
                stl = us - cs
                if s <= shl:
                    out[:, n] = (rl, ul, pl)
                elif s >= stl:
                    out[:, n] = (rl * (p / pl) ** (1 / g), us, p)
                else:
                    uu = 2 / (g + 1) * (cl + (g - 1) / 2 * ul + s)
                    cc = 2 / (g + 1) * (cl + (g - 1) / 2 * (ul - s))
                    rr_ = rl * (cc / cl) ** (2 / (g - 1))
                    out[:, n] = (rr_, uu, pl * (cc / cl) ** (2 * g / (g - 1)))
        else:
            if p > pr:
                sr = ur + cr * math.sqrt((g + 1) / (2 * g) * p / pr + (g - 1) / (2 * g))
                if s >= sr:
                    out[:, n] = (rr, ur, pr)
                else:
                    r = rr * ((p / pr + (g - 1) / (g + 1)) / ((g - 1) / (g + 1) * p / pr + 1))
                    out[:, n] = (r, us, p)
            else:
                shr = ur + cr
                cs = cr * (p / pr) ** ((g - 1) / (2 * g))
                if s >= shr:
                    out[:, n] = (rr, ur, pr)
                elif s <= us + cs:
                    out[:, n] = (rr * (p / pr) ** (1 / g), us, p)
                else:
                    uu = 2 / (g + 1) * (-cr + (g - 1) / 2 * ur + s)
                    cc = 2 / (g + 1) * (cr - (g - 1) / 2 * (ur - s))
                    out[:, n] = (rr * (cc / cr) ** (2 / (g - 1)), uu, pr * (cc / cr) ** (2 * g / (g - 1)))
    return out


def _sod_case(n, axis):
    dims = [2, 2, 2]
    dims[axis] = n
    dims = tuple(dims)
    h = [1.0, 1.0, 1.0]
    h[axis] = 1.0 / n
    X = cases.cartesian_nodes(dims, h=tuple(h))
    C = cases.centroids(X)
    left = C[axis] < 0.5
    rho = np.where(left, 1.0, 0.125)
    p = np.where(left, 1.0, 0.1)
    zero = np.zeros_like(rho)
    q = cases.conserved_from(rho, zero, zero, zero, p, 1.4)
    conns, bcs = [], []
    for d in range(3):
        if d == axis:
            bcs += [cases.full_bc(0, dims, 2 * d, cases.EXTRAP), cases.full_bc(0, dims, 2 * d + 1, cases.EXTRAP)]
        else:
            conns += cases.periodic_pair(0, dims, d, float(dims[d]))
    par = cases.Params(cfl=0.5, mach=0.0)
    return cases.Case("sod", par, [dims], [X], conns, bcs, [q]), C[axis]


def _run_sod(n, axis, T=0.2):
    c, xc = _sod_case(n, axis)
    st = solver.setup(c)
    t = 0.0
    while t < T - 1e-14:
        dt = min(solver.time_step(st), T - t)
        solver.step(st, dt=dt)
        t += dt
    q = solver.interior_state(st, 0)
    line = [0, 0, 0]
    line[axis] = slice(None)
    sl = (slice(None), line[2], line[1], line[0])
    sl = tuple(s if isinstance(s, slice) else 0 for s in sl)
    return q[sl], xc[sl[1:]]


def test_sod_exact_riemann_each_axis():
    prof = {}
    for axis in range(3):
        q, x = _run_sod(100, axis)
        prof[axis] = q
    for axis in (1, 2):
        assert np.max(np.abs(prof[axis][0] - prof[0][0])) < 1e-13
    ex = _exact_riemann(1.0, 0.0, 1.0, 0.125, 0.0, 0.1, x - 0.5, 0.2)
    e100 = np.mean(np.abs(prof[0][0] - ex[0]))
    q2, x2 = _run_sod(200, 0)
    ex2 = _exact_riemann(1.0, 0.0, 1.0, 0.125, 0.0, 0.1, x2 - 0.5, 0.2)
    e200 = np.mean(np.abs(q2[0] - ex2[0]))
    assert e100 < 0.02 and e200 < 0.75 * e100, (e100, e200)


def test_time_step_closed_form_cartesian():
    dims = (6, 5, 4)
    h = 0.3
    X = cases.cartesian_nodes(dims, h=(h, h, h))
    par = cases.Params(mach=0.7, alpha=0.3, beta=0.2, cfl=0.8)
    q = cases.uniform_state(dims, par)
    c = cases.Case("dt", par, [dims], [X], cases.periodic_self_conns(0, dims, tuple(n * h for n in dims)),
                   [], [q])
    dt = solver.time_step(solver.setup(c))
    u = cases.freestream_velocity(par)
    want = 0.8 * h / (abs(u[0]) + abs(u[1]) + abs(u[2]) + 3 * math.sqrt(1.4))
    assert abs(dt - want) < 1e-15


def test_block_split_invariance():
    c = cases.vortex_case(16, seed=2, curvilinear=True)
    sc = cases.split_periodic_box(c, (2, 2, 2))
    a, b = solver.setup(c), solver.setup(sc)
    for _ in range(3):
        solver.step(a)
        solver.step(b)
    qa = solver.interior_state(a, 0)
    n = 8
    blk = 0
    for bk in range(2):
        for bj in range(2):
            for bi in range(2):
                qb = solver.interior_state(b, blk)
                ref = qa[:, bk * n:(bk + 1) * n, bj * n:(bj + 1) * n, bi * n:(bi + 1) * n]
                assert np.max(np.abs(qb - ref)) < 1e-14
                blk += 1


def test_norms_definitions():
    c = cases.vortex_case(8)
    st = solver.setup(c)
    R = [np.full((5, 8, 8, 8), 0.0)]
    R[0][0] = 3.0
    R[0][2, 1, 2, 3] = -4.0
    out = solver.norms_from(st, st.Qs, R)
    assert out[0] == 3.0
    assert abs(out[2] - math.sqrt(16.0 / 512)) < 1e-16
    assert out[10] == 3.0
    V = (10.0 / 8) ** 3
    assert abs(out[5] - V * float(np.sum(c.q0[0][0]))) < 1e-12


def test_batched_channels_match_single_cases():
    """Blocks of a batched context with per-patch inflow Mach behave exactly like
    the corresponding single-case runs (independent blocks, own freestream)."""
    conds = [(0.55, 0.03), (0.8, 0.09)]
    bc = cases.channel_batch_case(conds, 12, 6, 4)
    sb = solver.setup(bc)
    for _ in range(2):
        solver.step(sb)
    for b, (m, h) in enumerate(conds):
        c = cases.channel_case(12, 6, 4, mach=m, hb=h)
        s1 = solver.setup(c)
        for _ in range(2):
            solver.step(s1)
        assert np.array_equal(solver.interior_state(sb, b), solver.interior_state(s1, 0))
