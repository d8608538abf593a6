"""Pins of the oracle's WCNS-E-5 closures at walls and the far field (the
ghost-block reading of the block-boundary treatment that Section 2.2 leaves to
its references; oracle/closures.py):

* a uniform stream on the curved wall-bump grid (tanh-stretched, the one-GPU
  share's geometry) with the far field on both bounded faces stays uniform,
  inviscid and with the viscous terms;
* on a grid straight and uniform across two flat walls (wavy along the
  walls), a state and its mirror images form a field periodic over twice the
  height; the closed residual equals the periodic residual of that field
  (slip and no-slip walls, inviscid and viscous), which pins the ghost
  ordering, the mirrored momentum, the extrapolated metrics and the ring of
  ghost blocks in one comparison;
* the vertex extension continues a grid linear along the bounded direction
  exactly;
* cells more than the stencils' reach from both faces do not see the closure;
* owners tiling the periodic directions (each with ghost blocks joined to
  its neighbours' ghost blocks) give bitwise the single closed block;
* closed across two directions (corner ghost blocks): a uniform stream on the
  warm-start channel grid stays uniform, and walls on all four faces of a
  flat duct give the periodic residual of the doubly mirrored field.
"""
import numpy as np
import pytest

from oracle import closures as cl
from oracle import highorder as ho
from oracle.ghosts import FARFIELD, NOSLIP_ADIABATIC, SLIPWALL
from paper_1710_09995_amd import cases

GAMMA = 1.4
VISC = (0.72, 0.02, 0.38)          # Pr, mu_inf, Sutherland constant


def _bump(n=(24, 16, 8)):
    c = cases.bump_ns_case(*n, seed=1)
    return c.nodes[0][:, 1:, :, 1:], [(2.0, 0.0, 0.0), (0.0, 0.0, 0.0), (0.0, 0.0, 1.0)]


def _flat(n=(16, 10, 6), h=0.1, amp=0.3):
    """Vertices straight and uniform in y (planes y = -h .. (n_j - 1) h, i.e.
    walls at y = -h... shifted so that plane -1 is y = 0), wavy in x and z."""
    ni, nj, nk = n
    i = np.arange(1, ni + 1)
    k = np.arange(1, nk + 1)
    K, I = np.meshgrid(k, i, indexing="ij")
    x = I * h + amp * h * np.sin(2 * np.pi * K / nk)
    z = K * h + amp * h * np.sin(2 * np.pi * I / ni)
    y = np.arange(nj + 1) * h
    X = np.empty((3, nk, nj + 1, ni))
    X[0] = x[:, None, :]
    X[1] = y[None, :, None]
    X[2] = z[:, None, :]
    return X, [(ni * h, 0.0, 0.0), (0.0, 0.0, 0.0), (0.0, 0.0, nk * h)], h


def _smooth_state(n, seed):
    rng = np.random.default_rng(seed)
    ni, nj, nk = n
    k, j, i = np.meshgrid(np.arange(nk), np.arange(nj), np.arange(ni), indexing="ij")
    ph = rng.uniform(0, 2 * np.pi, 5)
    rho = 1.0 + 0.1 * np.sin(2 * np.pi * i / ni + ph[0]) * np.cos(np.pi * (j + 0.5) / nj + ph[1])
    u = 0.5 + 0.1 * np.cos(2 * np.pi * k / nk + ph[2])
    v = 0.08 * np.sin(2 * np.pi * i / ni + ph[3]) * np.sin(np.pi * (j + 0.5) / nj)
    w = 0.05 * np.cos(2 * np.pi * (i / ni + k / nk) + ph[4])
    p = 1.0 / GAMMA + 0.05 * np.sin(2 * np.pi * k / nk) * np.cos(np.pi * (j + 0.5) / nj)
    E = p / (GAMMA - 1.0) + 0.5 * rho * (u * u + v * v + w * w)
    return np.stack([rho, rho * u, rho * v, rho * w, E])


def _freestream(n, mach):
    c = cases.uniform_state(n, cases.Params(mach=mach))
    return c


@pytest.mark.parametrize("viscous", [False, True])
def test_uniform_stream_on_the_bump_grid_stays_uniform(viscous):
    Xv, P = _bump()
    c = cl.Closed(Xv, P, 1, (FARFIELD, FARFIELD), GAMMA, freestream=(0.8, 0.0, 0.0))
    q = _freestream(c.n, 0.8)
    R = c.residual(q, viscous=VISC if viscous else None)
    assert np.max(np.abs(R)) <= 1e-12
    # the ghost blocks really are curved and stretched: metrics vary cell to cell
    assert np.ptp(c.Jinv[1]) > 1e-3 * np.max(c.Jinv[1])


def _mirror_cell(q, kind):
    """Mirror image of conserved states q about a y = const wall."""
    out = q.copy()
    if kind == SLIPWALL:
        out[2] = -q[2]
    else:
        out[1:4] = -q[1:4]
    return out


@pytest.mark.parametrize("kind", [SLIPWALL, NOSLIP_ADIABATIC])
@pytest.mark.parametrize("viscous", [False, True])
def test_walls_equal_the_mirrored_periodic_field(kind, viscous):
    n = (16, 10, 6)
    Xv, P, h = _flat(n)
    c = cl.Closed(Xv, P, 1, (kind, kind), GAMMA)
    q = _smooth_state(n, seed=3)
    R = c.residual(q, viscous=VISC if viscous else None)
    # the doubled field: cells 0 .. n_j - 1 the state, n_j .. 2 n_j - 1 its mirror image
    nj = n[1]
    qd = np.concatenate([q, _mirror_cell(q[:, :, ::-1], kind)], axis=2)
    Xd = np.concatenate([Xv[:, :, 1:], Xv[:, :, 1:].copy()], axis=2)
    Xd[1, :, nj:] = (np.arange(nj + 1, 2 * nj + 1) * h)[None, :, None]
    Pd = [P[0], (0.0, 2 * nj * h, 0.0), P[2]]
    Sd, Jd = ho.metrics6(ho.periodic_vertices(Xd, Pd))
    Rd = ho.wcns5_euler_residual_curv_periodic(qd, Sd, Jd, GAMMA, 0.1)
    if viscous:
        Rd = Rd + ho.viscous_residual_curv_periodic(qd, Sd, Jd, GAMMA, *VISC)
    ref = Rd[:, :, :nj]
    assert np.max(np.abs(R - ref)) <= 1e-12 * np.max(np.abs(ref)), np.max(np.abs(R - ref))


def test_vertex_extension_continues_a_linear_grid():
    n = (8, 6, 4)
    ni, nj, nk = n
    k, j, i = np.meshgrid(np.arange(1, nk + 1), np.arange(-1, nj), np.arange(1, ni + 1), indexing="ij")
    A = np.array([[0.3, 0.1, -0.2], [0.05, 0.4, 0.1], [0.0, -0.1, 0.25]])
    Xv = np.einsum("ab,bkji->akji", A, np.stack([i, j, k]).astype(float))
    P = [tuple(A[:, 0] * ni), (0.0, 0.0, 0.0), tuple(A[:, 2] * nk)]
    E, origin = cl.extended_vertices(Xv, P, 1)
    idx = [np.arange(E.shape[3]) - origin[0], np.arange(E.shape[2]) - origin[1], np.arange(E.shape[1]) - origin[2]]
    kk, jj, ii = np.meshgrid(idx[2], idx[1], idx[0], indexing="ij")
    want = np.einsum("ab,bkji->akji", A, np.stack([ii + 1, jj, kk + 1]).astype(float))
    assert E.shape[2] == nj + 1 + 2 * cl.XLAYERS and np.max(np.abs(E - want)) <= 1e-13


def test_cells_far_from_both_faces_do_not_see_the_closure():
    n = (12, 24, 6)
    Xv, P, h = _flat(n)
    q = _smooth_state(n, seed=4)
    a = cl.Closed(Xv, P, 1, (SLIPWALL, FARFIELD), GAMMA).residual(q, viscous=VISC)
    b = cl.Closed(Xv, P, 1, (NOSLIP_ADIABATIC, SLIPWALL), GAMMA).residual(q, viscous=VISC)
    assert np.array_equal(a[:, :, 8:-8], b[:, :, 8:-8])
    assert np.max(np.abs(a[:, :, :3] - b[:, :, :3])) > 1e-6


@pytest.mark.parametrize("viscous", [False, True])
def test_tiled_owners_give_the_single_block(viscous):
    """The wall-bump grid cut unevenly into 2 x 2 owners along its periodic
    directions, each with its own ghost blocks joined to its neighbours'
    ghost blocks: every owner's closed residual is bitwise the single closed
    block's residual there (the stencils and ghost layers are the same)."""
    n = (24, 16, 12)
    Xv, P = _bump(n)
    q = _smooth_state(n, seed=6)
    kinds = (NOSLIP_ADIABATIC, FARFIELD)
    one = cl.Closed(Xv, P, 1, kinds, GAMMA, freestream=(0.8, 0.0, 0.0))
    R1 = one.residual(q, viscous=VISC if viscous else None)
    tl = cl.ClosedBlocks(Xv, P, 1, kinds, {0: [0, 10, 24], 2: [0, 5, 12]}, GAMMA, freestream=(0.8, 0.0, 0.0))
    Rs = tl.residual(tl.split(q), viscous=VISC if viscous else None)
    assert len(Rs) == 4
    for (lo, ext), R in zip(tl.owners, Rs):
        sl = (slice(None), slice(lo[2], lo[2] + ext[2]), slice(lo[1], lo[1] + ext[1]), slice(lo[0], lo[0] + ext[0]))
        assert np.array_equal(R, R1[sl]), (lo, ext)


def _channel_vertices(n=(24, 12, 8)):
    c = cases.channel_case(*n, mach=0.6, hb=0.06)
    return np.ascontiguousarray(c.nodes[0][:, 1:, :, :]), [(0.0, 0.0, 0.0), (0.0, 0.0, 0.0), (0.0, 0.0, 1.0)]


@pytest.mark.parametrize("viscous", [False, True])
def test_duct_keeps_a_uniform_stream(viscous):
    """The warm-start channel grid (bump on the lower wall), closed across x
    and y with the far field on all four faces, corners included: a uniform
    stream stays uniform."""
    Xv, P = _channel_vertices()
    kinds = {0: (FARFIELD, FARFIELD), 1: (FARFIELD, FARFIELD)}
    d = cl.ClosedDuct(Xv, P, (0, 1), kinds, GAMMA, freestream=(0.6, 0.0, 0.0))
    q = _freestream(d.n, 0.6)
    assert np.max(np.abs(d.residual(q, viscous=VISC if viscous else None))) <= 1e-12


@pytest.mark.parametrize("kind", [SLIPWALL, NOSLIP_ADIABATIC])
@pytest.mark.parametrize("viscous", [False, True])
def test_duct_walls_equal_the_mirrored_periodic_field(kind, viscous):
    """A flat duct (uniform in x and y, stretched along the periodic z) with
    walls on all four faces: the state, its mirror images across x and y and
    across both form a field periodic over twice the width and height; the
    closed residual (corner ghost blocks included: the viscous terms read
    them) equals the periodic residual of that field."""
    ni, nj, nk = 10, 8, 6
    hx, hy = 0.1, 0.12
    k = np.arange(1, nk + 1)
    z = k / nk + 0.03 * np.sin(2 * np.pi * k / nk)
    X = np.empty((3, nk, nj + 1, ni + 1))
    X[0] = (np.arange(ni + 1) * hx)[None, None, :]
    X[1] = (np.arange(nj + 1) * hy)[None, :, None]
    X[2] = z[:, None, None]
    P = [(0.0, 0.0, 0.0), (0.0, 0.0, 0.0), (0.0, 0.0, 1.0)]
    d = cl.ClosedDuct(X, P, (0, 1), {0: (kind, kind), 1: (kind, kind)}, GAMMA)
    q = _smooth_state((ni, nj, nk), seed=11)
    R = d.residual(q, viscous=VISC if viscous else None)

    def mirror(a, axis_vel):
        out = a.copy()
        if kind == SLIPWALL:
            out[axis_vel] = -a[axis_vel]
        else:
            out[1:4] = -a[1:4]
        return out
    qx = mirror(q[:, :, :, ::-1], 1)
    top = np.concatenate([q, qx], axis=3)
    qd = np.concatenate([top, mirror(top[:, :, ::-1, :], 2)], axis=2)
    Xd = np.empty((3, nk, 2 * nj, 2 * ni))
    Xd[0] = (np.arange(1, 2 * ni + 1) * hx)[None, None, :]
    Xd[1] = (np.arange(1, 2 * nj + 1) * hy)[None, :, None]
    Xd[2] = z[:, None, None]
    Pd = [(2 * ni * hx, 0.0, 0.0), (0.0, 2 * nj * hy, 0.0), (0.0, 0.0, 1.0)]
    Sd, Jd = ho.metrics6(ho.periodic_vertices(Xd, Pd))
    Rd = ho.wcns5_euler_residual_curv_periodic(qd, Sd, Jd, GAMMA, 0.1)
    if viscous:
        Rd = Rd + ho.viscous_residual_curv_periodic(qd, Sd, Jd, GAMMA, *VISC)
    ref = Rd[:, :, :nj, :ni]
    assert np.max(np.abs(R - ref)) <= 1e-12 * np.max(np.abs(ref)), np.max(np.abs(R - ref))
