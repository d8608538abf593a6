"""GPU parity of the WCNS-E-5 closures at walls and the far field (ghost
blocks; cfd_wcns5_extend_vertices, cfd_wcns5_fill_ghost_blocks and the
joined-block residual, viscous terms and RK3 steps through the C ABI) against
the oracle (oracle/closures.py) on the wall-bump geometry of the one-GPU share
and of the 256 x 128 x 128 workload (periodic x and z, tanh-stretched y, a
no-slip wall below and the far field above), reduced to sizes the oracle
finishes in seconds; then the full 256 x 128 x 128 grid keeps a uniform stream
(far field on both faces) to rounding.
"""
import math

import numpy as np
import pytest

from gpu_util import say
from oracle import closures as ocl
from oracle.ghosts import FARFIELD, NOSLIP_ADIABATIC, SLIPWALL
from paper_1710_09995_amd import cases

pytestmark = pytest.mark.gpu

GAMMA = 1.4
MACH = 0.8
UINF = (MACH * math.sqrt(GAMMA), 0.0, 0.0)
VISC = (0.72, 0.02, 0.38)
PERIOD = [(2.0, 0.0, 0.0), (0.0, 0.0, 0.0), (0.0, 0.0, 1.0)]


def _bump_vertices(n):
    c = cases.bump_ns_case(*n, seed=1)
    return np.ascontiguousarray(c.nodes[0][:, 1:, :, 1:])


def _smooth_state(n, seed):
    rng = np.random.default_rng(seed)
    ni, nj, nk = n
    k, j, i = np.meshgrid(np.arange(nk), np.arange(nj), np.arange(ni), indexing="ij")
    ph = rng.uniform(0, 2 * np.pi, 5)
    rho = 1.0 + 0.1 * np.sin(2 * np.pi * i / ni + ph[0]) * np.cos(np.pi * (j + 0.5) / nj + ph[1])
    u = UINF[0] * (1.0 + 0.1 * np.cos(2 * np.pi * k / nk + ph[2]))
    v = 0.08 * np.sin(2 * np.pi * i / ni + ph[3]) * np.sin(np.pi * (j + 0.5) / nj)
    w = 0.05 * np.cos(2 * np.pi * (i / ni + k / nk) + ph[4])
    p = 1.0 + 0.05 * np.sin(2 * np.pi * k / nk) * np.cos(np.pi * (j + 0.5) / nj)
    E = p / (GAMMA - 1.0) + 0.5 * rho * (u * u + v * v + w * w)
    return np.stack([rho, rho * u, rho * v, rho * w, E])


def _dev(a):
    import torch
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def _pair(n, kinds):
    from paper_1710_09995_amd.binding import WcnsClosedBlock
    Xv = _bump_vertices(n)
    o = ocl.Closed(Xv, PERIOD, 1, kinds, GAMMA, freestream=(MACH, 0.0, 0.0))
    g = WcnsClosedBlock(_dev(Xv), PERIOD, 1, kinds, UINF, GAMMA)
    return o, g


def _rel(a, b):
    return float(np.max(np.abs(a - b)) / np.max(np.abs(b)))


def test_extended_vertices_and_metrics_match_the_oracle():
    from paper_1710_09995_amd.binding import wcns5_extend_vertices
    n = (24, 16, 8)
    say("closure geometry", n)
    Xv = _bump_vertices(n)
    E, _ = ocl.extended_vertices(Xv, PERIOD, 1)
    Eg = wcns5_extend_vertices(_dev(Xv), 1, PERIOD).cpu().numpy()
    assert Eg.shape == E.shape and _rel(Eg, E) <= 1e-15
    o, g = _pair(n, (NOSLIP_ADIABATIC, FARFIELD))
    for b in range(3):
        assert _rel(g.S[b].cpu().numpy(), o.S[b]) <= 1e-13, b
        assert _rel(g.jinv[b].cpu().numpy(), o.Jinv[b]) <= 1e-13, b


@pytest.mark.parametrize("kinds", [(NOSLIP_ADIABATIC, FARFIELD), (SLIPWALL, SLIPWALL), (FARFIELD, NOSLIP_ADIABATIC)])
def test_ghost_states_match_the_oracle(kinds):
    n = (24, 16, 8)
    say("ghost fill", kinds)
    o, g = _pair(n, kinds)
    q = _smooth_state(n, seed=5)
    want = o.blocks(q)
    qd = _dev(q)
    g.fill(qd)
    for b in (1, 2):
        got = g.ghosts[b - 1].cpu().numpy()
        assert _rel(got, want[b]) <= 1e-14, (b, _rel(got, want[b]))


@pytest.mark.parametrize("viscous", [False, True])
def test_closed_residual_matches_the_oracle(viscous):
    n = (32, 24, 12)
    say("closed residual", n, "viscous", viscous)
    o, g = _pair(n, (NOSLIP_ADIABATIC, FARFIELD))
    q = _smooth_state(n, seed=6)
    want = o.residual(q, viscous=VISC if viscous else None)
    got = g.residual(_dev(q), viscous=VISC if viscous else None).cpu().numpy()
    err = _rel(got, want)
    l2 = float(np.linalg.norm(got - want) / np.linalg.norm(want))
    say(f"  max error / max|R| {err:.2e}, rel L2 {l2:.2e}")
    assert err <= 1e-12 and l2 <= 1e-12


def test_closed_ns_steps_match_the_oracle():
    n = (24, 16, 8)
    say("closed NS steps", n)
    o, g = _pair(n, (NOSLIP_ADIABATIC, FARFIELD))
    q = _smooth_state(n, seed=7)
    visc = (0.72, 0.002, 0.38)          # within the explicit viscous limit of the wall cells at this step
    want = o.ns_steps(q, 5e-4, 3, viscous=visc)
    got = g.steps(_dev(q), 5e-4, 3, viscous=visc).cpu().numpy()
    dq = float(np.max(np.abs(got - want)) / np.max(np.abs(want - q)))
    say(f"  max error / max|Q| {_rel(got, want):.2e}, / max|Q - Q0| {dq:.2e}")
    assert _rel(got, want) <= 1e-12 and dq <= 1e-10


def test_inviscid_closed_steps_match_the_oracle():
    n = (24, 16, 8)
    o, g = _pair(n, (SLIPWALL, FARFIELD))
    q = _smooth_state(n, seed=8)
    want = o.ns_steps(q, 2e-3, 2)
    got = g.steps(_dev(q), 2e-3, 2).cpu().numpy()
    assert _rel(got, want) <= 1e-12


def test_full_size_bump_grid_keeps_a_uniform_stream():
    """The 256 x 128 x 128 wall-bump grid, far field on both faces: a uniform
    stream's residual (inviscid and viscous) stays at rounding level of its
    face terms (1e-13 of them; a metric that broke the identity would leave
    terms of order h^6 or more), and the no-slip/far-field Navier-Stokes steps
    from it stay finite."""
    import torch
    from paper_1710_09995_amd.binding import WcnsClosedBlock
    n = (256, 128, 128)
    say("full-size closed bump grid", n)
    xv = _dev(_bump_vertices(n))
    g = WcnsClosedBlock(xv, PERIOD, 1, (FARFIELD, FARFIELD), UINF, GAMMA)
    q = _dev(cases.uniform_state(n, cases.Params(mach=MACH)))
    # the size of one face term of R = J sum_d D_d (F . S_d): |F| |S| / J^-1,
    # about 2,400 here (wall cells some 1e-3 high); rounding is relative to it
    S, jinv = g.S[0], g.jinv[0]
    area = sum(torch.sqrt((S[d] ** 2).sum(0)) for d in range(3))
    scale = float((area / jinv).max()) * (1.0 + UINF[0] ** 2)
    for visc in (None, VISC):
        R = g.residual(q, viscous=visc)
        top = float(R.abs().max())
        say(f"  viscous {visc is not None}: max |R| {top:.2e} = {top / scale:.1e} of the face-term scale {scale:.0f}")
        assert top <= 1e-13 * scale
    w = WcnsClosedBlock(xv, PERIOD, 1, (NOSLIP_ADIABATIC, FARFIELD), UINF, GAMMA)
    w.steps(q, 1e-4, 2, viscous=(0.72, UINF[0] / 1e6, 0.38))
    assert bool(torch.isfinite(q).all())


def test_tiled_owners_on_the_one_gpu_share_geometry():
    """The one-GPU share's geometry at reduced size: 4 x 4 blocks of 16 x 16 x
    12 cells tiling z and x, no-slip wall below and far field above the
    wall-normal direction, each block closed by its own ghost blocks.  On the
    device the tiled residual (viscous terms included) and two RK3
    Navier-Stokes steps are bitwise the single closed block's, and the
    residual matches the oracle's tiling."""
    import torch
    from paper_1710_09995_amd.binding import WcnsClosedBlock, WcnsClosedTiling
    Xv, P = cases.paper_share_vertices(4, 4, 16, 16, 12)
    n = (64, 64, 12)
    say("closed tiling 4 x 4 of 16 x 16 x 12")
    kinds = (NOSLIP_ADIABATIC, FARFIELD)
    cuts = {0: [0, 16, 32, 48, 64], 1: [0, 16, 32, 48, 64]}
    xv = _dev(Xv)
    one = WcnsClosedBlock(xv, P, 2, kinds, UINF, GAMMA)
    tl = WcnsClosedTiling(xv, P, 2, kinds, UINF, GAMMA, cuts=cuts)
    q = _smooth_state(n, seed=9)
    qd = _dev(q)
    R1 = one.residual(qd, viscous=VISC)
    Rs = tl.residual(tl.split(qd), viscous=VISC)
    o = ocl.ClosedBlocks(Xv, P, 2, kinds, cuts, GAMMA, freestream=(MACH, 0.0, 0.0))
    want = o.residual(o.split(q), viscous=VISC)
    for (lo, ext), R, W in zip(tl.owners, Rs, want):
        sl = (slice(None), slice(lo[2], lo[2] + ext[2]), slice(lo[1], lo[1] + ext[1]), slice(lo[0], lo[0] + ext[0]))
        assert torch.equal(R, R1[sl]), (lo, ext)
        assert _rel(R.cpu().numpy(), W) <= 1e-12, (lo, ext, _rel(R.cpu().numpy(), W))
    visc = (0.72, 0.002, 0.38)
    qs = tl.split(qd)
    one.steps(qd, 2e-4, 2, viscous=visc)
    tl.steps(qs, 2e-4, 2, viscous=visc)
    for (lo, ext), x in zip(tl.owners, qs):
        sl = (slice(None), slice(lo[2], lo[2] + ext[2]), slice(lo[1], lo[1] + ext[1]), slice(lo[0], lo[0] + ext[0]))
        assert torch.equal(x, qd[sl]), (lo, ext)


def _channel(n):
    c = cases.channel_case(*n, mach=0.6, hb=0.06)
    return np.ascontiguousarray(c.nodes[0][:, 1:, :, :]), [(0.0, 0.0, 0.0), (0.0, 0.0, 0.0), (0.0, 0.0, 1.0)]


C4_KINDS = {0: (FARFIELD, FARFIELD), 1: (SLIPWALL, SLIPWALL)}
UINF_C4 = (0.6 * math.sqrt(GAMMA), 0.0, 0.0)


def _duct_pair(n, kinds=C4_KINDS):
    from paper_1710_09995_amd.binding import WcnsClosedDuct
    Xv, P = _channel(n)
    o = ocl.ClosedDuct(Xv, P, (0, 1), kinds, GAMMA, freestream=(0.6, 0.0, 0.0))
    g = WcnsClosedDuct(_dev(Xv), P, (0, 1), kinds, UINF_C4, GAMMA)
    return Xv, P, o, g


def test_duct_geometry_and_ghost_states_match_the_oracle():
    """The warm-start channel geometry (far field across x, slip walls across
    y, periodic z), closed by four face and four corner ghost blocks: the
    vertices continued in two directions, every block's metrics and every
    ghost state (corners included) against the oracle."""
    from paper_1710_09995_amd.binding import wcns5_extend_vertices
    import ctypes as C
    from paper_1710_09995_amd import binding as B
    n = (24, 12, 8)
    say("duct geometry", n)
    Xv, P, o, g = _duct_pair(n)
    assert len(g.S) == 9
    for b in range(9):
        assert _rel(g.S[b].cpu().numpy(), o.S[b]) <= 1e-13, b
        assert _rel(g.jinv[b].cpu().numpy(), o.Jinv[b]) <= 1e-13, b
    q = _smooth_state(n, seed=12)
    want = o.blocks(q)
    qd = _dev(q)
    g.fill(qd)
    for b in range(1, 9):
        assert _rel(g.ghosts[b - 1].cpu().numpy(), want[b]) <= 1e-14, b


@pytest.mark.parametrize("viscous", [False, True])
def test_duct_residual_matches_the_oracle(viscous):
    n = (24, 16, 8)
    say("duct residual", n, "viscous", viscous)
    _, _, o, g = _duct_pair(n, {0: (FARFIELD, FARFIELD), 1: (NOSLIP_ADIABATIC, SLIPWALL)})
    q = _smooth_state(n, seed=13)
    want = o.residual(q, viscous=VISC if viscous else None)
    got = g.residual(_dev(q), viscous=VISC if viscous else None).cpu().numpy()
    err = _rel(got, want)
    say(f"  max error / max|R| {err:.2e}")
    assert err <= 1e-12 and float(np.linalg.norm(got - want) / np.linalg.norm(want)) <= 1e-12


def test_duct_steps_match_the_oracle():
    n = (24, 12, 8)
    _, _, o, g = _duct_pair(n)
    q = _smooth_state(n, seed=14)
    visc = (0.72, 0.002, 0.38)
    want = o.ns_steps(q, 5e-4, 2, viscous=visc)
    got = g.steps(_dev(q), 5e-4, 2, viscous=visc).cpu().numpy()
    dq = float(np.max(np.abs(got - want)) / np.max(np.abs(want - q)))
    say(f"  duct NS steps: max error / max|Q| {_rel(got, want):.2e}, / max|Q - Q0| {dq:.2e}")
    assert _rel(got, want) <= 1e-12 and dq <= 1e-10


def test_full_size_channel_duct_keeps_a_uniform_stream():
    """The warm-start fine grid (192 x 96 x 96 channel with its bump), closed
    across x and y with the far field on all four faces: a uniform stream's
    residual stays at 1e-13 of its face terms; with the warm-start conditions
    (far field across x, slip walls across y) RK3 steps from it stay finite."""
    import torch
    from paper_1710_09995_amd.binding import WcnsClosedDuct
    n = (192, 96, 96)
    say("full-size channel duct", n)
    Xv, P = _channel(n)
    xv = _dev(Xv)
    g = WcnsClosedDuct(xv, P, (0, 1), {0: (FARFIELD, FARFIELD), 1: (FARFIELD, FARFIELD)}, UINF_C4, GAMMA)
    q = _dev(cases.uniform_state(n, cases.Params(mach=0.6)))
    S, jinv = g.S[0], g.jinv[0]
    area = sum(torch.sqrt((S[d] ** 2).sum(0)) for d in range(3))
    scale = float((area / jinv).max()) * (1.0 + UINF_C4[0] ** 2)
    top = float(g.residual(q).abs().max())
    say(f"  max |R| {top:.2e} = {top / scale:.1e} of the face-term scale {scale:.0f}")
    assert top <= 1e-13 * scale
    w = WcnsClosedDuct(xv, P, (0, 1), C4_KINDS, UINF_C4, GAMMA)
    w.steps(q, 1e-4, 2)
    assert bool(torch.isfinite(q).all())
