"""Pins for the oracle's ghost-cell fill (CPU only).

* A periodic box split into blocks must see, in every ghost cell (edges and
  corners included), the value of the cell at the same place of the unsplit
  periodic field: an index-free physical check of the connection sweeps.
* Partial patches: brute-force enumeration of which neighbour cell each ghost
  cell must hold.
* Wall conditions reduce to textbook mirror states on flat walls.
* Far field: Riemann-invariant and entropy identities of the boundary state.
"""
import math

import numpy as np
import pytest

from oracle import geometry, ghosts, solver
from paper_1710_09995_amd import cases

G = 2


def _fill(case):
    st = solver.setup(case, G)
    solver.fill(st)
    return st


@pytest.mark.parametrize("parts", [(1, 1, 1), (2, 1, 1), (2, 2, 2), (1, 2, 3)])
def test_periodic_split_ghosts_equal_global_field(parts):
    n = (6, 6, 6)
    rng = np.random.default_rng(0)
    f = rng.uniform(1.0, 2.0, (5, n[2], n[1], n[0]))
    c = cases.vortex_case(6)
    c.q0[0][:] = f
    sc = cases.split_periodic_box(c, parts)
    st = _fill(sc)
    si, sj, sk = n[0] // parts[0], n[1] // parts[1], n[2] // parts[2]
    b = 0
    for bk in range(parts[2]):
        for bj in range(parts[1]):
            for bi in range(parts[0]):
                Q = st.Qs[b]
                for k in range(-G, sk + G):
                    for j in range(-G, sj + G):
                        for i in range(-G, si + G):
                            want = f[:, (bk * sk + k) % n[2], (bj * sj + j) % n[1], (bi * si + i) % n[0]]
                            assert np.array_equal(Q[:, k + G, j + G, i + G], want), (b, i, j, k)
                b += 1


def test_partial_patch_bruteforce():
    """Block A (+i face) joined to block B (-i face) over a sub-rectangle."""
    dA, dB = (3, 5, 4), (2, 3, 6)
    mj, mk = 3, 4
    XA = cases.cartesian_nodes(dA)
    XB = cases.cartesian_nodes(dB, origin=(3.0, 0.0, 0.0))
    conns = [cases.Conn(0, 1, 1, 0, (0, 0), (mj, mk), (0, 0)),
             cases.Conn(1, 0, 0, 1, (0, 0), (mj, mk), (0, 0))]
    bcs = []
    for b, dims in enumerate((dA, dB)):
        for face in range(6):
            e1, e2 = cases.face_extent(dims, face)
            if (b, face) in ((0, 1), (1, 0)):
                if e1 > mj:
                    bcs.append(cases.BC(b, face, cases.EXTRAP, (mj, 0), (e1, e2)))
                if e2 > mk:
                    bcs.append(cases.BC(b, face, cases.EXTRAP, (0, mk), (mj, e2)))
            else:
                bcs.append(cases.BC(b, face, cases.EXTRAP, (0, 0), (e1, e2)))
    rng = np.random.default_rng(2)
    qA = rng.uniform(1, 2, (5,) + dA[::-1])
    qB = rng.uniform(1, 2, (5,) + dB[::-1])
    case = cases.Case("pair", cases.Params(), [dA, dB], [XA, XB], conns, bcs, [qA, qB])
    st = _fill(case)
    QA, QB = st.Qs
    # A's +i ghosts (i = 3, 4) inside the patch come from B's cells i = 0, 1
    for m in (1, 2):
        for k in range(mk):
            for j in range(mj):
                assert np.array_equal(QA[:, k + G, j + G, dA[0] - 1 + m + G], qB[:, k, j, m - 1])
    # outside the patch they extrapolate A's last cell
    for m in (1, 2):
        for k in range(dA[2]):
            for j in range(dA[1]):
                if j < mj and k < mk:
                    continue
                assert np.array_equal(QA[:, k + G, j + G, dA[0] - 1 + m + G], qA[:, k, j, dA[0] - 1])
    # B's -i ghosts inside the patch come from A's cells i = 2, 1; outside they extrapolate
    for m in (1, 2):
        for k in range(dB[2]):
            for j in range(dB[1]):
                want = qA[:, k, j, dA[0] - m] if (j < mj and k < mk) else qB[:, k, j, 0]
                assert np.array_equal(QB[:, k + G, j + G, G - m], want)


def _flat_wall_case(kind, face):
    dims = (3, 4, 3)
    X = cases.cartesian_nodes(dims, h=(0.5, 0.25, 0.5))
    rng = np.random.default_rng(4)
    rho = rng.uniform(0.8, 1.2, dims[::-1])
    u, v, w = (rng.uniform(-0.5, 0.5, dims[::-1]) for _ in range(3))
    p = rng.uniform(0.8, 1.2, dims[::-1])
    q = cases.conserved_from(rho, u, v, w, p, 1.4)
    bcs = [cases.full_bc(0, dims, f, kind if f == face else cases.EXTRAP) for f in range(6)]
    return cases.Case("wall", cases.Params(), [dims], [X], [], bcs, [q]), q


@pytest.mark.parametrize("face", [2, 3])
def test_slip_wall_mirror(face):
    case, q = _flat_wall_case(cases.SLIPWALL, face)
    Q = _fill(case).Qs[0]
    nj = case.dims[0][1]
    for m in (1, 2):
        gj = -m if face == 2 else nj - 1 + m
        ij = m - 1 if face == 2 else nj - m
        got = Q[:, G:-G, gj + G, G:-G]
        src = q[:, :, ij, :]
        assert np.array_equal(got[[0, 1, 3, 4]], src[[0, 1, 3, 4]])
        assert np.array_equal(got[2], -src[2])


def test_noslip_wall_mirror():
    case, q = _flat_wall_case(cases.NOSLIP_ADIABATIC, 2)
    Q = _fill(case).Qs[0]
    for m in (1, 2):
        got = Q[:, G:-G, G - m, G:-G]
        src = q[:, :, m - 1, :]
        assert np.array_equal(got[[0, 4]], src[[0, 4]])
        assert np.array_equal(got[1:4], -src[1:4])


def _prim(Q, g=1.4):
    rho = Q[0]
    u = Q[1:4] / rho
    p = (g - 1) * (Q[4] - 0.5 * rho * np.sum(u * u, axis=0))
    return rho, u, p


@pytest.mark.parametrize("mach,scale", [(0.5, 1.0), (0.8, 1.05), (0.3, 0.93)])
def test_farfield_invariants(mach, scale):
    """Subsonic far field: outgoing invariant from the interior, incoming from the stream,
    entropy from the upwind side; a freestream interior is returned unchanged."""
    par = cases.Params(mach=mach)
    rng = np.random.default_rng(5)
    n_out = rng.normal(size=(3, 50))
    n_out /= np.linalg.norm(n_out, axis=0)
    rho = scale * rng.uniform(0.9, 1.1, 50)
    u = cases.freestream_velocity(par)[:, None] * rng.uniform(0.8, 1.2, (3, 50))
    p = rng.uniform(0.9, 1.1, 50)
    Qi = cases.conserved_from(rho, u[0], u[1], u[2], p, 1.4)
    Qb = ghosts._farfield_state(Qi, n_out, par)
    g = 1.4
    rb, ub, pb = _prim(Qb)
    ri, ui, pi = _prim(Qi)
    cb, ci = np.sqrt(g * pb / rb), np.sqrt(g * pi / ri)
    Ub, Ui = np.sum(ub * n_out, 0), np.sum(ui * n_out, 0)
    uinf = cases.freestream_velocity(par)[:, None]
    Uinf = np.sum(uinf * n_out, 0)
    cinf = math.sqrt(g)
    sub = np.abs(Ui) < ci
    assert sub.all()
    assert np.allclose((Ub + 2 * cb / (g - 1)), Ui + 2 * ci / (g - 1), rtol=0, atol=1e-13)
    assert np.allclose((Ub - 2 * cb / (g - 1)), Uinf - 2 * cinf / (g - 1), rtol=0, atol=1e-13)
    s_b = pb / rb ** g
    out = Ub >= 0
    assert np.allclose(s_b[out], (pi / ri ** g)[out], rtol=1e-13)
    assert np.allclose(s_b[~out], 1.0, rtol=1e-13)
    ut_b = ub - Ub * n_out
    ut_src = np.where(out, ui - Ui * n_out, uinf - Uinf * n_out)
    assert np.max(np.abs(ut_b - ut_src)) < 1e-13
    # freestream in, freestream out
    one = np.ones(50)
    Qf = cases.conserved_from(one, uinf[0] * one, uinf[1] * one, uinf[2] * one, one, g)
    assert np.max(np.abs(ghosts._farfield_state(Qf, n_out, par) - Qf)) < 1e-14


def test_farfield_supersonic_limits():
    par = cases.Params(mach=0.5)
    n_out = np.array([[1.0, -1.0], [0.0, 0.0], [0.0, 0.0]])
    rho = np.array([1.3, 0.7])
    p = np.array([0.9, 1.2])
    c = np.sqrt(1.4 * p / rho)
    u = np.array([[2.5 * c[0], 3.0 * c[1]], [0.1, 0.2], [0.0, -0.1]])   # out via +x, in via -x
    Qi = cases.conserved_from(rho, u[0], u[1], u[2], p, 1.4)
    Qb = ghosts._farfield_state(Qi, n_out, par)
    assert np.array_equal(Qb[:, 0], Qi[:, 0])           # supersonic outflow: interior
    uinf = cases.freestream_velocity(par)
    Qf = cases.conserved_from(np.ones(1), uinf[0:1], uinf[1:2], uinf[2:3], np.ones(1), 1.4)
    assert np.max(np.abs(Qb[:, 1] - Qf[:, 0])) < 1e-15   # supersonic inflow: freestream


def test_metric_ghosts_copied_across_connections():
    """The seam face vector seen by the lower block is the upper block's own."""
    c = cases.batched_euler_case(nblk=3, seed=1, lo=4, hi=9)
    Xs, Ss, Vs = geometry.build_metrics(c, G)
    for cn in c.conns:
        if cn.face != 1:
            continue
        a, b = cn.blk, cn.nbr
        ni = c.dims[a][0]
        for k in range(cn.hi[1]):
            for j in range(cn.hi[0]):
                assert np.array_equal(Ss[a][0][:, k + G, j + G, ni + G], Ss[b][0][:, k + G, j + G, G])
                assert Vs[a][k + G, j + G, ni + G] == Vs[b][k + G, j + G, G]
