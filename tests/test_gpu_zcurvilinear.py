"""GPU parity of the WCNS-E-5 scheme on curvilinear blocks (Section 2.2)
through the C ABI, against the FP64 oracle on the same seeded grids and
states: the metrics (periodic, and from a block's own vertices), the inviscid
residual, RK3 steps, the fourth-order viscous terms, the CFL time step and
blocks joined face to face; with the properties that pin the oracle (a kept
uniform stream, the Cartesian reduction, convergence orders) checked on the
GPU's own output, at 256 x 128 x 128 where the oracle is too slow.

Tolerances: metrics within 1e-13 of their largest entry (a few ulps: the
kernels sum in another order and fuse products), residuals and steps within
1e-12 of the largest entry, the time step within 1e-14 (a minimum of cell
values)."""
import numpy as np
import pytest

from gpu_util import say
from oracle import highorder as ho
from test_gpu_highorder import _smooth_state

pytestmark = pytest.mark.gpu


def _dev(a):
    """An oracle array on the device, C-contiguous as the library requires."""
    import torch
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


# ------------------------------------------- curvilinear metrics and residual

def _curv_grid(n, kind):
    """Vertices and periods of a periodic curvilinear block: a wavy grid (every
    coordinate displaced by sines of the other two) or a sheared, stretched
    affine grid."""
    from test_oracle_highorder import _positions, _wavy_grid
    if kind == "wavy":
        Xv, P, _ = _wavy_grid(n, (3.0, 2.0, 1.5), 0.08)
        return np.ascontiguousarray(Xv), P
    A = np.array([[0.3, 0.05, 0.0], [0.02, 0.25, 0.04], [0.0, -0.03, 0.2]])     # columns: one index step
    pos = np.stack(_positions(n, (0.5, 0.5, 0.5)))
    Xv = np.einsum("ab,bkji->akji", A, pos) + np.array([0.1, -0.2, 0.3])[:, None, None, None]
    return np.ascontiguousarray(Xv), np.stack([n[d] * A[:, d] for d in range(3)])


@pytest.mark.parametrize("n,kind", [((37, 21, 13), "wavy"), ((16, 16, 16), "wavy"), ((9, 7, 5), "affine"),
                                    ((70, 3, 2), "wavy"), ((2, 9, 7), "wavy")])
def test_curvilinear_metrics_and_residual_parity(n, kind):
    """Metrics and residual against the oracle on the same grid and state:
    S and J^{-1} within 1e-13 of their largest entry (a few ulps; the kernel
    sums the outer derivative in another order), R within 1e-12 of max |R|."""
    import torch
    from paper_1710_09995_amd.binding import wcns5_euler_residual_curv_periodic, wcns5_metrics_periodic
    Xv, P = _curv_grid(n, kind)
    say("curvilinear metrics + residual", n, kind)
    S, J = wcns5_metrics_periodic(torch.from_numpy(Xv).cuda(), P)
    So, Jo = ho.metrics6(ho.periodic_vertices(Xv, P))
    assert np.max(np.abs(S.cpu().numpy() - So)) <= 1e-13 * np.max(np.abs(So))
    assert np.max(np.abs(J.cpu().numpy() - Jo)) <= 1e-13 * np.max(np.abs(Jo))
    q = _smooth_state(n, seed=sum(n) + 1)
    got = wcns5_euler_residual_curv_periodic(torch.from_numpy(q).cuda(), S, J).cpu().numpy()
    want = ho.wcns5_euler_residual_curv_periodic(q, So, Jo, 1.4, 0.1)
    assert np.max(np.abs(got - want)) <= 1e-12 * np.max(np.abs(want))


def test_curvilinear_full_size_freestream_and_cartesian_reduction():
    """At 256 x 128 x 128: a uniform stream on the wavy grid stays uniform
    (the geometric conservation law, any size), and on a uniform Cartesian
    grid the curvilinear residual equals the Cartesian one to rounding.  That
    rounding grows with resolution: the symmetric metrics difference products
    of coordinates (size 1) and their derivatives (size h), so S carries a
    relative error of about eps / h (3e-14 at h = 1/256), and Eq. (2)'s
    difference of nearly equal face fluxes amplifies it by about 1 / (h k)
    (400 for this flow's wave number k = 2 pi): some 1e-11 of max |R|
    (8.4e-12 measured); the bar is 1e-10."""
    import torch
    from paper_1710_09995_amd import cases
    from paper_1710_09995_amd.binding import (wcns5_euler_residual_curv_periodic, wcns5_euler_residual_periodic,
                                              wcns5_metrics_periodic)
    from test_oracle_highorder import _positions
    n = (256, 128, 128)
    say("curvilinear full size", n)
    Xv, P = _curv_grid(n, "wavy")
    S, J = wcns5_metrics_periodic(torch.from_numpy(Xv).cuda(), P)
    assert float(J.min()) > 0
    q = cases.conserved_from(np.full((n[2], n[1], n[0]), 1.2), 0.5, -0.3, 0.2, 1.0 / 1.4, 1.4)
    R = wcns5_euler_residual_curv_periodic(torch.from_numpy(np.ascontiguousarray(q)).cuda(), S, J)
    assert float(R.abs().max()) <= 1e-10
    del S, J, R
    h = (1.0 / n[0], 1.0 / n[1], 1.0 / n[2])
    Xc = np.ascontiguousarray(np.stack([(x + 0.5) * h[d] for d, x in enumerate(_positions(n, (0.5, 0.5, 0.5)))]))
    S, J = wcns5_metrics_periodic(torch.from_numpy(Xc).cuda(), np.eye(3))
    qs = torch.from_numpy(_smooth_state(n, seed=5)).cuda()
    got = wcns5_euler_residual_curv_periodic(qs, S, J)
    want = wcns5_euler_residual_periodic(qs, h)
    assert float((got - want).abs().max()) <= 1e-10 * float(want.abs().max())


def test_curvilinear_vortex_order_gpu():
    """The isentropic vortex on the wavy grid of the oracle's pin, on the GPU:
    -R approaches the exact dQ/dt at fourth order or better."""
    import torch
    from paper_1710_09995_amd import cases
    from paper_1710_09995_amd.binding import wcns5_euler_residual_curv_periodic, wcns5_metrics_periodic
    from test_oracle_highorder import _positions, _wavy_grid
    par = cases.Params(mach=0.5)
    xc, yc = 0.3, -0.4
    uinf = cases.freestream_velocity(par)
    errs = []
    for m in (32, 64, 128):
        n = (m, m, 4)
        Xv, P, fmap = _wavy_grid(n, (10.0, 10.0, 1.0), 0.03, planar=True)
        sh = 5.0 * np.array([1.0, 1.0, 0.0])[:, None, None, None]
        S, J = wcns5_metrics_periodic(torch.from_numpy(np.ascontiguousarray(Xv - sh)).cuda(), P)
        X = fmap(_positions(n, (0.0, 0.0, 0.0))) - sh

        def Q(xx, yy):
            return cases.conserved_from(*cases.isentropic_vortex_primitives(xx, yy, xc, yc, par, period=10.0),
                                        par.gamma)
        e = 1e-5
        rate = -(uinf[0] * (Q(X[0] + e, X[1]) - Q(X[0] - e, X[1])) +
                 uinf[1] * (Q(X[0], X[1] + e) - Q(X[0], X[1] - e))) / (2 * e)
        R = wcns5_euler_residual_curv_periodic(torch.from_numpy(np.ascontiguousarray(Q(X[0], X[1]))).cuda(), S,
                                               J).cpu().numpy()
        near = ((np.abs(X[0] - xc) < 3) & (np.abs(X[1] - yc) < 3))[None]
        errs.append(np.max(np.abs(-R - rate) * near))
    assert min(np.log2(errs[i] / errs[i + 1]) for i in range(2)) >= 4.0, errs


def test_curvilinear_steps_parity_and_freestream():
    """RK3 steps on the curvilinear residual against the oracle's (5 steps, the
    smooth periodic flow on the wavy grid, oracle metrics on both sides), and
    a uniform stream kept uniform with the device's own metrics."""
    import torch
    from paper_1710_09995_amd import cases
    from paper_1710_09995_amd.binding import wcns5_euler_steps_curv_periodic, wcns5_metrics_periodic
    n = (20, 12, 8)
    Xv, P = _curv_grid(n, "wavy")
    So, Jo = ho.metrics6(ho.periodic_vertices(Xv, P))
    q = _smooth_state(n, seed=3)
    say("curvilinear steps", n)
    got = wcns5_euler_steps_curv_periodic(torch.from_numpy(q.copy()).cuda(), _dev(So),
                                          _dev(Jo), 0.01, 5).cpu().numpy()
    want = ho.wcns5_euler_steps_curv_periodic(q, So, Jo, 1.4, 0.1, 0.01, 5)
    assert np.max(np.abs(got - want)) <= 1e-12 * np.max(np.abs(want))
    S, J = wcns5_metrics_periodic(torch.from_numpy(Xv).cuda(), P)
    qu = np.ascontiguousarray(cases.conserved_from(np.full((n[2], n[1], n[0]), 1.2), 0.5, -0.3, 0.2, 1.0 / 1.4, 1.4))
    got = wcns5_euler_steps_curv_periodic(torch.from_numpy(qu.copy()).cuda(), S, J, 0.02, 4).cpu().numpy()
    assert np.max(np.abs(got - qu)) <= 1e-12


@pytest.mark.parametrize("n,kind", [((20, 12, 10), "wavy"), ((9, 7, 11), "affine")])
def test_curvilinear_viscous_parity(n, kind):
    """The curvilinear viscous terms added to a zero residual, against the
    oracle's on the same metrics (the oracle's), within 1e-12 of max |R_v|."""
    import torch
    from paper_1710_09995_amd.binding import c4_viscous_add_curv_periodic
    Xv, P = _curv_grid(n, kind)
    So, Jo = ho.metrics6(ho.periodic_vertices(Xv, P))
    q = _smooth_state(n, seed=sum(n) + 2)
    say("curvilinear viscous", n, kind)
    r = torch.zeros((5, n[2], n[1], n[0]), dtype=torch.float64, device="cuda")
    got = c4_viscous_add_curv_periodic(torch.from_numpy(q).cuda(), r, _dev(So),
                                       _dev(Jo), 1.4, 0.72, 0.02, 0.38).cpu().numpy()
    want = ho.viscous_residual_curv_periodic(q, So, Jo, 1.4, 0.72, 0.02, 0.38)
    assert np.max(np.abs(got - want)) <= 1e-12 * np.max(np.abs(want))


def test_curvilinear_viscous_fourth_order_gpu():
    """The shear field of the oracle's pin on the wavy grid, metrics and
    viscous terms both from the device: fourth order to the closed form."""
    import torch
    from paper_1710_09995_amd.binding import c4_viscous_add_curv_periodic, wcns5_metrics_periodic
    from test_oracle_highorder import _positions, _wavy_grid
    g, mu0 = 1.4, 0.01
    L = 2 * np.pi
    errs = []
    for m in (16, 32, 64):
        n = (m, m, m)
        Xv, P, fmap = _wavy_grid(n, (L, L, L), 0.02)
        S, J = wcns5_metrics_periodic(torch.from_numpy(np.ascontiguousarray(Xv)).cuda(), P)
        X, Y, Z = fmap(_positions(n, (0.0, 0.0, 0.0)))
        u, v, w = np.sin(Y), np.sin(Z), np.sin(X)
        Q = np.ascontiguousarray(np.stack([np.ones_like(X), u, v, w, 1.0 / (g - 1.0) + 0.5 * (u * u + v * v + w * w)]))
        exact = np.stack([0 * X, mu0 * np.sin(Y), mu0 * np.sin(Z), mu0 * np.sin(X),
                          -mu0 * (np.cos(2 * X) + np.cos(2 * Y) + np.cos(2 * Z))])
        r = torch.zeros((5, m, m, m), dtype=torch.float64, device="cuda")
        Rv = c4_viscous_add_curv_periodic(torch.from_numpy(Q).cuda(), r, S, J, g, 0.72, mu0, 0.38).cpu().numpy()
        errs.append(np.max(np.abs(Rv - exact)))
    assert min(np.log2(errs[i] / errs[i + 1]) for i in range(2)) > 3.7, errs


@pytest.mark.parametrize("viscous", [False, True])
def test_curvilinear_time_step_parity(viscous):
    """The global CFL step on the wavy grid (ragged extents, the smooth flow)
    against the oracle's, within 1e-14 relative: a minimum over cells, where
    only the cell values' roundings differ."""
    import torch
    from paper_1710_09995_amd.binding import wcns5_time_step_curv_periodic
    n = (37, 21, 13)
    Xv, P = _curv_grid(n, "wavy")
    So, Jo = ho.metrics6(ho.periodic_vertices(Xv, P))
    q = _smooth_state(n, seed=9)
    say("curvilinear time step", n, viscous)
    got = float(wcns5_time_step_curv_periodic(torch.from_numpy(q).cuda(), _dev(So),
                                              _dev(Jo), 0.7, 1.4, viscous, 0.72, 0.05,
                                              0.38).cpu()[0])
    want = ho.cfl_time_step_curv_periodic(q, So, Jo, 1.4, 0.7, viscous, 0.72, 0.05, 0.38)
    assert abs(got - want) <= 1e-14 * want


@pytest.mark.parametrize("n,cuts", [((40, 30, 24), ([17], [8, 20], [11])), ((30, 15, 10), ([5, 25], [5], [5]))])
def test_block_seams_match_the_unsplit_block(n, cuts):
    """A periodic wavy block cut into 2 x 3 x 2 blocks joined face to face:
    each block's metrics from its own vertices (cfd_wcns5_metrics_ext) match
    the unsplit block's within 1e-13 (the wrapped coordinates are formed on
    the host here and on the device there); with the unsplit block's metrics
    sliced, the blocks' residuals are bitwise the unsplit residual's slices;
    and the residuals match the oracle's blocks within 1e-12.  The second
    split has blocks exactly five cells deep, the least a seam allows."""
    import torch
    from paper_1710_09995_amd.binding import (wcns5_euler_residual_blocks, wcns5_euler_residual_curv_periodic,
                                              wcns5_metrics_ext, wcns5_metrics_periodic)
    from test_oracle_highorder import _split_box
    Xv, P = _curv_grid(n, "wavy")
    say("block seams", n, cuts)
    S, J = wcns5_metrics_periodic(torch.from_numpy(Xv).cuda(), P)
    q = _smooth_state(n, seed=4)
    qt = torch.from_numpy(q).cuda()
    R = wcns5_euler_residual_curv_periodic(qt, S, J)
    lo, m, nbr = _split_box(n, cuts)
    qs, Ss, Js, Sx, Jx = [], [], [], [], []
    for o, e in zip(lo, m):
        sl = (slice(o[2], o[2] + e[2]), slice(o[1], o[1] + e[1]), slice(o[0], o[0] + e[0]))
        qs.append(qt[(slice(None),) + sl].contiguous())
        Ss.append(S[(slice(None), slice(None)) + sl].contiguous())
        Js.append(J[sl].contiguous())
        Sb, Jb = wcns5_metrics_ext(torch.from_numpy(np.ascontiguousarray(ho.block_vertices(Xv, P, o, e))).cuda())
        assert float((Sb - Ss[-1]).abs().max()) <= 1e-13 * float(S.abs().max())
        assert float((Jb - Js[-1]).abs().max()) <= 1e-13 * float(J.abs().max())
        Sx.append(Sb)
        Jx.append(Jb)
    Rs = wcns5_euler_residual_blocks(qs, Ss, Js, nbr)
    for (o, e), Rb in zip(zip(lo, m), Rs):
        assert torch.equal(Rb, R[:, o[2]:o[2] + e[2], o[1]:o[1] + e[1], o[0]:o[0] + e[0]])
    Rx = wcns5_euler_residual_blocks(qs, Sx, Jx, nbr)
    want = ho.wcns5_euler_residual_blocks([t.cpu().numpy() for t in qs], [t.cpu().numpy() for t in Sx],
                                          [t.cpu().numpy() for t in Jx], nbr, 1.4, 0.1)
    top = max(float(np.max(np.abs(w))) for w in want)
    for got, w in zip(Rx, want):
        assert np.max(np.abs(got.cpu().numpy() - w)) <= 1e-12 * top


def test_viscous_seams_match_the_unsplit_block():
    """The 2 x 3 x 2 split of a periodic wavy block: the viscous terms across
    the seams are bitwise the unsplit block's (the kernels repeat the
    periodic kernels' arithmetic) and match the oracle's blocks within 1e-12."""
    import torch
    from paper_1710_09995_amd.binding import c4_viscous_add_blocks, c4_viscous_add_curv_periodic, wcns5_metrics_periodic
    from test_oracle_highorder import _split_box
    n = (40, 30, 24)
    Xv, P = _curv_grid(n, "wavy")
    say("viscous seams", n)
    S, J = wcns5_metrics_periodic(torch.from_numpy(Xv).cuda(), P)
    q = _smooth_state(n, seed=6)
    qt = torch.from_numpy(q).cuda()
    Rv = c4_viscous_add_curv_periodic(qt, torch.zeros_like(qt), S, J, 1.4, 0.72, 0.02, 0.38)
    lo, m, nbr = _split_box(n, ([17], [8, 20], [11]))
    sls = [(slice(o[2], o[2] + e[2]), slice(o[1], o[1] + e[1]), slice(o[0], o[0] + e[0])) for o, e in zip(lo, m)]
    qs = [qt[(slice(None),) + sl].contiguous() for sl in sls]
    Ss = [S[(slice(None), slice(None)) + sl].contiguous() for sl in sls]
    Js = [J[sl].contiguous() for sl in sls]
    rs = c4_viscous_add_blocks(qs, [torch.zeros_like(t) for t in qs], Ss, Js, nbr, 1.4, 0.72, 0.02, 0.38)
    for sl, rb in zip(sls, rs):
        assert torch.equal(rb, Rv[(slice(None),) + sl])
    want = ho.viscous_residual_blocks([t.cpu().numpy() for t in qs], [t.cpu().numpy() for t in Ss],
                                      [t.cpu().numpy() for t in Js], nbr, 1.4, 0.72, 0.02, 0.38)
    top = max(float(np.max(np.abs(w))) for w in want)
    for got, w in zip(rs, want):
        assert np.max(np.abs(got.cpu().numpy() - w)) <= 1e-12 * top


def test_ns_steps_parity_and_shear_wave():
    """RK3 Navier-Stokes steps on the device: 4 steps of the smooth flow on
    the wavy grid against the oracle's (oracle metrics on both sides, within
    1e-12 of max |q|), and the shear wave of the oracle's pin on a wavy grid
    with the device's own metrics: fourth-order decay at exp(-nu t)."""
    import torch
    from paper_1710_09995_amd.binding import wcns5_metrics_periodic, wcns5_ns_steps_curv_periodic
    from test_oracle_highorder import _shear_wave
    n = (20, 12, 8)
    Xv, P = _curv_grid(n, "wavy")
    So, Jo = ho.metrics6(ho.periodic_vertices(Xv, P))
    q = _smooth_state(n, seed=12)
    say("ns steps", n)
    got = wcns5_ns_steps_curv_periodic(torch.from_numpy(q.copy()).cuda(), _dev(So), _dev(Jo), 0.01, 4, 1.4, 0.1,
                                       1e-6, 0.72, 0.02, 0.38).cpu().numpy()
    want = ho.ns_steps_curv_periodic(q, So, Jo, 1.4, 0.1, 0.72, 0.02, 0.38, 0.01, 4)
    assert np.max(np.abs(got - want)) <= 1e-12 * np.max(np.abs(want))
    nu, eps_a = 0.05, 1e-3
    errs = []
    for m in (8, 16, 32):
        qw, _, _, Y, Xw, Pw = _shear_wave(m, True, eps_a)
        S, J = wcns5_metrics_periodic(_dev(Xw), Pw)
        qe = wcns5_ns_steps_curv_periodic(_dev(qw), S, J, 0.05, 20, 1.4, 0.1, 1e-6, 0.72, nu, 0.38).cpu().numpy()
        errs.append(np.max(np.abs(qe[1] / qe[0] - 0.3 - eps_a * np.exp(-nu) * np.sin(Y))) / eps_a)
    assert min(np.log2(errs[i] / errs[i + 1]) for i in range(2)) > 3.8 and errs[-1] < 2e-6, errs


def _implicit_gate(got, want, q0, tag):
    """The implicit steps' parity bar: the state within 1e-12 of max |q|, and
    the accumulated update Q - Q0 within 1e-10 of its own largest entry (the
    sweeps form flux differences F(Q + dQ) - F(Q), whose rounding is relative
    to |F|, not to the difference, and the kernels' operation order differs
    from the oracle's)."""
    got, want, q0 = ([np.asarray(x) for x in v] for v in (got, want, q0))
    err = max(float(np.max(np.abs(g - w))) for g, w in zip(got, want))
    top = max(float(np.max(np.abs(w))) for w in want)
    dtop = max(float(np.max(np.abs(w - z))) for w, z in zip(want, q0))
    say(f"  {tag}: max error / max|q| {err / top:.2e}, / max|Q - Q0| {err / dtop:.2e}")
    assert err <= 1e-12 * top
    assert err <= 1e-10 * dtop


def test_implicit_steps_parity_and_stability():
    """Implicit steps on the device against the oracle's (3 steps, 4 sweeps,
    the smooth flow on the wavy grid, oracle metrics on both sides) to the
    implicit bar (_implicit_gate); and at 20 times the CFL-1 step, with the
    device's own metrics, the steps stay bounded."""
    import torch
    from paper_1710_09995_amd.binding import wcns5_implicit_steps_curv_periodic, wcns5_metrics_periodic
    n = (20, 12, 8)
    Xv, P = _curv_grid(n, "wavy")
    So, Jo = ho.metrics6(ho.periodic_vertices(Xv, P))
    q = _smooth_state(n, seed=14)
    say("implicit steps", n)
    got = wcns5_implicit_steps_curv_periodic(torch.from_numpy(q.copy()).cuda(), _dev(So), _dev(Jo), 0.02, 3,
                                             4).cpu().numpy()
    want = ho.implicit_steps_curv_periodic(q, So, Jo, 1.4, 0.1, 0.02, 3, 4)
    _implicit_gate([got], [want], [q], "inviscid")
    S, J = wcns5_metrics_periodic(_dev(Xv), P)
    dt = 20.0 * ho.cfl_time_step_curv_periodic(q, So, Jo, 1.4, 1.0)
    qi = wcns5_implicit_steps_curv_periodic(torch.from_numpy(q.copy()).cuda(), S, J, dt, 20, 4).cpu().numpy()
    assert np.all(np.isfinite(qi)) and qi[0].min() > 0.5 and np.max(np.abs(qi - q)) < 1.5


def test_viscous_implicit_steps_parity():
    """Implicit Navier-Stokes steps on the device against the oracle's (3 steps,
    4 sweeps, the smooth flow on the wavy grid, oracle metrics on both sides),
    to the implicit bar (_implicit_gate)."""
    import torch
    from paper_1710_09995_amd.binding import wcns5_implicit_steps_curv_periodic
    n = (20, 12, 8)
    Xv, P = _curv_grid(n, "wavy")
    So, Jo = ho.metrics6(ho.periodic_vertices(Xv, P))
    q = _smooth_state(n, seed=15)
    say("viscous implicit steps", n)
    got = wcns5_implicit_steps_curv_periodic(torch.from_numpy(q.copy()).cuda(), _dev(So), _dev(Jo), 0.02, 3, 4,
                                             viscous=True, prandtl=0.72, mu_inf=0.02, s_star=0.38).cpu().numpy()
    want = ho.implicit_steps_curv_periodic(q, So, Jo, 1.4, 0.1, 0.02, 3, 4, viscous=True, prandtl=0.72, mu_inf=0.02,
                                           s_star=0.38)
    _implicit_gate([got], [want], [q], "viscous")


def test_implicit_steps_on_split_blocks_match_the_unsplit_block():
    """The 12-block split of a periodic wavy block: 2 implicit steps with 4
    sweeps on the blocks are bitwise the unsplit block's on the device (the
    kernels repeat the periodic kernels' arithmetic, and point-Jacobi reads
    only the previous iterate), and match the oracle's blocks to the implicit
    bar (_implicit_gate)."""
    import torch
    from paper_1710_09995_amd.binding import (wcns5_implicit_steps_blocks, wcns5_implicit_steps_curv_periodic,
                                              wcns5_metrics_periodic)
    from test_oracle_highorder import _split_box
    n = (40, 30, 24)
    Xv, P = _curv_grid(n, "wavy")
    say("implicit blocks", n)
    S, J = wcns5_metrics_periodic(torch.from_numpy(Xv).cuda(), P)
    q = _smooth_state(n, seed=16)
    qt = torch.from_numpy(q).cuda()
    lo, m, nbr = _split_box(n, ([17], [8, 20], [11]))
    sls = [(slice(o[2], o[2] + e[2]), slice(o[1], o[1] + e[1]), slice(o[0], o[0] + e[0])) for o, e in zip(lo, m)]
    qs = [qt[(slice(None),) + sl].contiguous() for sl in sls]
    Ss = [S[(slice(None), slice(None)) + sl].contiguous() for sl in sls]
    Js = [J[sl].contiguous() for sl in sls]
    q0s = [t.cpu().numpy() for t in qs]
    whole = wcns5_implicit_steps_curv_periodic(qt.clone(), S, J, 0.05, 2, 4)
    got = wcns5_implicit_steps_blocks(qs, Ss, Js, nbr, 0.05, 2, 4)
    for sl, g in zip(sls, got):
        assert torch.equal(g, whole[(slice(None),) + sl])
    want = ho.implicit_steps_blocks(q0s, [t.cpu().numpy() for t in Ss], [t.cpu().numpy() for t in Js], nbr, 1.4, 0.1,
                                    0.05, 2, 4)
    _implicit_gate([g.cpu().numpy() for g in got], want, q0s, "blocks")


@pytest.mark.parametrize("n,cuts", [((40, 30, 24), ([17], [8, 20], [11])), ((30, 15, 10), ([5, 25], [5], [5]))])
def test_ns_steps_on_split_blocks_match_the_unsplit_block(n, cuts):
    """The paper's explicit method on a multi-block grid on the device: 2 RK3
    Navier-Stokes steps on the 12-block split of a periodic wavy block are
    bitwise the unsplit block's, and match the oracle's blocks within 1e-12."""
    import torch
    from paper_1710_09995_amd.binding import wcns5_metrics_periodic, wcns5_ns_steps_blocks, wcns5_ns_steps_curv_periodic
    from test_oracle_highorder import _split_box
    Xv, P = _curv_grid(n, "wavy")
    say("ns blocks", n, cuts)
    S, J = wcns5_metrics_periodic(torch.from_numpy(Xv).cuda(), P)
    q = _smooth_state(n, seed=17)
    qt = torch.from_numpy(q).cuda()
    lo, m, nbr = _split_box(n, cuts)
    sls = [(slice(o[2], o[2] + e[2]), slice(o[1], o[1] + e[1]), slice(o[0], o[0] + e[0])) for o, e in zip(lo, m)]
    qs = [qt[(slice(None),) + sl].contiguous() for sl in sls]
    Ss = [S[(slice(None), slice(None)) + sl].contiguous() for sl in sls]
    Js = [J[sl].contiguous() for sl in sls]
    q0s = [t.cpu().numpy() for t in qs]
    whole = wcns5_ns_steps_curv_periodic(qt.clone(), S, J, 0.005, 2, 1.4, 0.1, 1e-6, 0.72, 0.02, 0.38)
    got = wcns5_ns_steps_blocks(qs, Ss, Js, nbr, 0.005, 2, 1.4, 0.1, 1e-6, 0.72, 0.02, 0.38)
    for sl, g in zip(sls, got):
        assert torch.equal(g, whole[(slice(None),) + sl])
    want = ho.ns_steps_blocks(q0s, [t.cpu().numpy() for t in Ss], [t.cpu().numpy() for t in Js], nbr, 1.4, 0.1, 0.72,
                              0.02, 0.38, 0.005, 2)
    top = max(float(np.max(np.abs(w))) for w in want)
    for g, w in zip(got, want):
        assert np.max(np.abs(g.cpu().numpy() - w)) <= 1e-12 * top


@pytest.mark.parametrize("n", [(512, 128, 8), (512, 8, 128)])
def test_row_and_marching_passes_match_the_oracle(n):
    """The inviscid residual on blocks whose long rows take the i row pass and
    whose lines along the thin direction (8 cells, one chunk) take a marching
    pass, on the oracle's own metrics (at 512 cells per row, the few-ulp
    differences between the two metric computations alone move R by some
    1e-11 of max |R|), against the oracle within 1e-12 of max |R|."""
    import torch
    from paper_1710_09995_amd.binding import wcns5_euler_residual_curv_periodic
    Xv, P = _curv_grid(n, "wavy")
    say("row and marching passes", n)
    So, Jo = ho.metrics6(ho.periodic_vertices(Xv, P))
    q = _smooth_state(n, seed=sum(n) + 5)
    got = wcns5_euler_residual_curv_periodic(torch.from_numpy(q).cuda(), _dev(So), _dev(Jo)).cpu().numpy()
    want = ho.wcns5_euler_residual_curv_periodic(q, So, Jo, 1.4, 0.1)
    err = np.max(np.abs(got - want)) / np.max(np.abs(want))
    say(f"  max error / max|R| {err:.2e}")
    assert err <= 1e-12


def test_marching_passes_match_the_three_pass_path_at_full_size():
    """At 256 x 128 x 128 the unsplit block's inviscid residual runs its j and
    k directions as one marching pass each (primitives, WCNS-E-5 face states,
    Roe's flux and Eq. 2 in registers); its 2 x 2 x 2 split into 128 x 64 x 64
    blocks has too few lines for the march and runs the padded-primitive, face
    and Eq. 2 passes.  The residuals, the residuals with the viscous terms and
    two RK3 Navier-Stokes steps are bitwise the same on both, and a uniform
    stream keeps R within 1e-10 of its flux scale."""
    import torch
    from paper_1710_09995_amd.binding import (c4_viscous_add_blocks, c4_viscous_add_curv_periodic,
                                              wcns5_euler_residual_blocks, wcns5_euler_residual_curv_periodic,
                                              wcns5_metrics_periodic, wcns5_ns_steps_blocks,
                                              wcns5_ns_steps_curv_periodic)
    from test_oracle_highorder import _split_box
    n = (256, 128, 128)
    say("marching passes vs three-pass blocks", n)
    Xv, P = _curv_grid(n, "wavy")
    S, J = wcns5_metrics_periodic(torch.from_numpy(Xv).cuda(), P)
    del Xv
    qt = torch.from_numpy(_smooth_state(n, seed=23)).cuda()
    lo, m, nbr = _split_box(n, ([128], [64], [64]))
    sls = [(slice(o[2], o[2] + e[2]), slice(o[1], o[1] + e[1]), slice(o[0], o[0] + e[0])) for o, e in zip(lo, m)]
    qs = [qt[(slice(None),) + sl].contiguous() for sl in sls]
    Ss = [S[(slice(None), slice(None)) + sl].contiguous() for sl in sls]
    Js = [J[sl].contiguous() for sl in sls]
    whole = wcns5_euler_residual_curv_periodic(qt, S, J)
    parts = wcns5_euler_residual_blocks(qs, Ss, Js, nbr)
    assert all(torch.equal(p, whole[(slice(None),) + sl]) for sl, p in zip(sls, parts))
    whole = c4_viscous_add_curv_periodic(qt, whole, S, J, 1.4, 0.72, 0.02, 0.38)
    parts = c4_viscous_add_blocks(qs, parts, Ss, Js, nbr, 1.4, 0.72, 0.02, 0.38)
    assert all(torch.equal(p, whole[(slice(None),) + sl]) for sl, p in zip(sls, parts))
    del whole, parts
    steps_whole = wcns5_ns_steps_curv_periodic(qt.clone(), S, J, 1e-4, 2, 1.4, 0.1, 1e-6, 0.72, 0.02, 0.38)
    steps_parts = wcns5_ns_steps_blocks([t.clone() for t in qs], Ss, Js, nbr, 1e-4, 2, 1.4, 0.1, 1e-6, 0.72, 0.02,
                                        0.38)
    assert all(torch.equal(p, steps_whole[(slice(None),) + sl]) for sl, p in zip(sls, steps_parts))
    del steps_whole, steps_parts
    u = torch.empty_like(qt)
    u[0], u[1], u[2], u[3] = 1.0, 0.5, -0.2, 0.3
    u[4] = 1.0 / 0.4 + 0.5 * (0.25 + 0.04 + 0.09)
    R = wcns5_euler_residual_curv_periodic(u, S, J)
    scale = float(torch.max(torch.abs(S))) * 3.0 / float(torch.min(torch.abs(J)))
    assert float(torch.max(torch.abs(R))) <= 1e-10 * scale


def test_viscous_implicit_steps_on_split_blocks_match_the_unsplit_block():
    """The 12-block split with viscous terms: 2 implicit Navier-Stokes steps
    with 4 sweeps on the blocks are bitwise the unsplit block's on the device,
    and match the oracle's blocks to the implicit bar (_implicit_gate)."""
    import torch
    from paper_1710_09995_amd.binding import (wcns5_implicit_steps_blocks, wcns5_implicit_steps_curv_periodic,
                                              wcns5_metrics_periodic)
    from test_oracle_highorder import _split_box
    n = (40, 30, 24)
    Xv, P = _curv_grid(n, "wavy")
    say("viscous implicit blocks", n)
    S, J = wcns5_metrics_periodic(torch.from_numpy(Xv).cuda(), P)
    q = _smooth_state(n, seed=18)
    qt = torch.from_numpy(q).cuda()
    lo, m, nbr = _split_box(n, ([17], [8, 20], [11]))
    sls = [(slice(o[2], o[2] + e[2]), slice(o[1], o[1] + e[1]), slice(o[0], o[0] + e[0])) for o, e in zip(lo, m)]
    qs = [qt[(slice(None),) + sl].contiguous() for sl in sls]
    Ss = [S[(slice(None), slice(None)) + sl].contiguous() for sl in sls]
    Js = [J[sl].contiguous() for sl in sls]
    q0s = [t.cpu().numpy() for t in qs]
    kw = dict(viscous=True, prandtl=0.72, mu_inf=0.02, s_star=0.38)
    whole = wcns5_implicit_steps_curv_periodic(qt.clone(), S, J, 0.05, 2, 4, **kw)
    got = wcns5_implicit_steps_blocks(qs, Ss, Js, nbr, 0.05, 2, 4, **kw)
    for sl, g in zip(sls, got):
        assert torch.equal(g, whole[(slice(None),) + sl])
    want = ho.implicit_steps_blocks(q0s, [t.cpu().numpy() for t in Ss], [t.cpu().numpy() for t in Js], nbr, 1.4, 0.1,
                                    0.05, 2, 4, **kw)
    _implicit_gate([g.cpu().numpy() for g in got], want, q0s, "viscous blocks")
