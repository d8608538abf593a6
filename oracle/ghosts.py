"""Ghost-cell fill of the conserved state (oracle; plain FP64 NumPy).

Boundary data of neighbouring blocks are exchanged after every update
(Sections 2.3 and 3.2.5); on one device that exchange is a copy into the g = 2
ghost layers of each block.  Physical boundaries are not specified by the
paper; the conditions below are the ones this solver defines:

* connection: ghost layer m of face -d at transverse (p, q) takes the
  neighbour's cell at d-index n_d' - m (m - 1 for face +d), at transverse
  (p, q) - lo + nbr_lo; bitwise copy;
* slip wall: ghost m mirrors interior cell m - 1 with the momentum reflected
  about the boundary face's unit normal; density and energy are copied;
* no-slip adiabatic wall: ghost m mirrors interior m - 1 with the momentum
  negated;
* far field: both layers take a characteristic boundary state built from the
  first interior cell and the freestream (Riemann invariants along the
  outward normal; entropy and tangential velocity from the upwind side);
* extrapolation: both layers copy the first interior cell.

Sweeps run i, then j, then k; a sweep extends into the ghost layers of the
directions already swept where a patch reaches its face edge (edges and
corners, the paper's singular points, Section 3.2.3).
"""
from __future__ import annotations

import math

import numpy as np

from .geometry import index_grid, patch_ranges, transverse

FARFIELD, SLIPWALL, NOSLIP_ADIABATIC, EXTRAP = 1, 2, 3, 4


def freestream_primitives(params, mach=0.0):
    """rho, velocity, p of the freestream; mach > 0 overrides the case's Mach number."""
    g = params.gamma
    speed = (mach if mach > 0.0 else params.mach) * math.sqrt(g)
    u = speed * np.array([math.cos(params.alpha) * math.cos(params.beta),
                          math.sin(params.alpha) * math.cos(params.beta),
                          math.sin(params.beta)])
    return 1.0, u, 1.0


def _farfield_state(Qi, n_out, params, mach=0.0):
    """Characteristic far-field state for interior states Qi [5,...], outward normals n [3,...]."""
    g = params.gamma
    rho = Qi[0]
    u = Qi[1:4] / rho
    p = (g - 1.0) * (Qi[4] - 0.5 * rho * np.sum(u * u, axis=0))
    ci = np.sqrt(g * p / rho)
    Ui = np.sum(u * n_out, axis=0)
    rinf, uinf, pinf = freestream_primitives(params, mach)
    uinf = uinf.reshape(3, *([1] * (Qi.ndim - 1)))
    cinf = math.sqrt(g * pinf / rinf)
    Uinf = np.sum(uinf * n_out, axis=0)
    Rp = Ui + 2.0 * ci / (g - 1.0)
    Rm = Uinf - 2.0 * cinf / (g - 1.0)
    Ub = 0.5 * (Rp + Rm)
    cb = 0.25 * (g - 1.0) * (Rp - Rm)
    outflow = Ub >= 0.0
    s = np.where(outflow, p / rho ** g, pinf / rinf ** g)
    usrc = np.where(outflow[None], u, uinf * np.ones_like(u))
    Usrc = np.sum(usrc * n_out, axis=0)
    ut = usrc - Usrc[None] * n_out
    rb = (cb * cb / (g * s)) ** (1.0 / (g - 1.0))
    pb = rb * cb * cb / g
    ub = ut + Ub[None] * n_out
    # supersonic limits
    sup_out = Ui >= ci
    sup_in = Ui <= -ci
    rb = np.where(sup_out, rho, np.where(sup_in, rinf, rb))
    pb = np.where(sup_out, p, np.where(sup_in, pinf, pb))
    ub = np.where(sup_out[None], u, np.where(sup_in[None], uinf * np.ones_like(u), ub))
    Qb = np.empty_like(Qi)
    Qb[0] = rb
    Qb[1:4] = rb * ub
    Qb[4] = pb / (g - 1.0) + 0.5 * rb * np.sum(ub * ub, axis=0)
    return Qb


def fill_ghosts(Qs, Ss, dims, conns, bcs, params, g=2):
    """Fill the ghost cells of every block's padded state [5, nk+2g, nj+2g, ni+2g] in place."""
    for d in range(3):
        for bc in bcs:
            if bc.face // 2 != d:
                continue
            _fill_bc(Qs[bc.blk], Ss[bc.blk], dims[bc.blk], bc, params, g)
        for c in conns:
            if c.face // 2 != d:
                continue
            _fill_conn(Qs, dims, c, g)


def _fill_conn(Qs, dims, c, g):
    d = c.face // 2
    b, nb = c.blk, c.nbr
    n = dims[b][d]
    nn = dims[nb][d]
    _, rg = patch_ranges(dims[b], c.face, c.lo, c.hi, g)
    side = c.face % 2
    t1, t2 = transverse(d)
    for m in range(1, g + 1):
        gm = -m if side == 0 else n - 1 + m
        sm = nn - m if side == 0 else m - 1
        rd = dict(rg)
        rd[d] = (gm, gm + 1)
        rs = {d: (sm, sm + 1),
              t1: (rg[t1][0] - c.lo[0] + c.nbr_lo[0], rg[t1][1] - c.lo[0] + c.nbr_lo[0]),
              t2: (rg[t2][0] - c.lo[1] + c.nbr_lo[1], rg[t2][1] - c.lo[1] + c.nbr_lo[1])}
        Qs[b][(slice(None),) + index_grid(rd, g)] = Qs[nb][(slice(None),) + index_grid(rs, g)]


def _fill_bc(Q, S, dims, bc, params, g):
    d = bc.face // 2
    n = dims[d]
    side = bc.face % 2
    _, rg = patch_ranges(dims, bc.face, bc.lo, bc.hi, g)
    # boundary face vector at each transverse position (lower face of cell 0,
    # or lower face of ghost cell n for the upper side)
    fidx = 0 if side == 0 else n
    rf = dict(rg)
    rf[d] = (fidx, fidx + 1)
    Sb = S[d][(slice(None),) + index_grid(rf, g)]
    nrm = np.sqrt(np.sum(Sb * Sb, axis=0))
    nhat = Sb / nrm
    for m in range(1, g + 1):
        gm = -m if side == 0 else n - 1 + m
        im = m - 1 if side == 0 else n - m
        rd = dict(rg)
        rd[d] = (gm, gm + 1)
        ri = dict(rg)
        ri[d] = (im, im + 1)
        Qi = Q[(slice(None),) + index_grid(ri, g)]
        if bc.kind == SLIPWALL:
            mom = Qi[1:4]
            mn = np.sum(mom * nhat, axis=0)
            Qg = Qi.copy()
            Qg[1:4] = mom - 2.0 * mn[None] * nhat
        elif bc.kind == NOSLIP_ADIABATIC:
            Qg = Qi.copy()
            Qg[1:4] = -Qi[1:4]
        elif bc.kind == EXTRAP:
            r0 = dict(rg)
            i0 = 0 if side == 0 else n - 1
            r0[d] = (i0, i0 + 1)
            Qg = Q[(slice(None),) + index_grid(r0, g)].copy()
        elif bc.kind == FARFIELD:
            r0 = dict(rg)
            i0 = 0 if side == 0 else n - 1
            r0[d] = (i0, i0 + 1)
            Q0 = Q[(slice(None),) + index_grid(r0, g)]
            n_out = -nhat if side == 0 else nhat
            Qg = _farfield_state(Q0, n_out, params, getattr(bc, "mach", 0.0))
        else:
            raise ValueError(f"unknown boundary kind {bc.kind}")
        Q[(slice(None),) + index_grid(rd, g)] = Qg
