"""Closures of the WCNS-E-5 scheme at physical block faces (oracle; plain FP64
NumPy; test infrastructure, imported only by the tests).

Section 2.2 leaves the conditions at block boundaries to its references and
does not print them.  The reading taken here ("ghost blocks") keeps every
interior stencil unchanged up to the boundary:

* a block face on a wall or the far field gets a ghost block GHOST = 5 cells
  deep across that face (the reach of the interpolation and of Eq. 2's
  stencil), with the face's transverse extents, joined to the owner face to
  face; the residual of the owner is then the joined-block residual of
  highorder.py (R19) over the owner and its ghost blocks;
* geometry: the owner's vertex lines are extended past each bounded face by
  linear extrapolation, x_(b - m) = x_b + m (x_b - x_(b+1)) for the boundary
  plane b and the plane next to it inside; each block (owner or ghost) takes
  its metrics from its own window of the extended vertices (vertices -3 ..
  n + 1), so both sides of a boundary face compute it from the same
  coordinates and a uniform stream stays uniform (the metrics' identity holds
  on any vertex set);
* state of a ghost block, refilled from the owner before every residual: the
  ghost cell m = 1 .. 5 cells beyond the face mirrors the owner cell m - 1
  cells inside it:
    - slip wall: momentum reflected about the unit normal of the boundary
      face (its area vector S_d of the sixth-order metrics), rho and energy
      copied;
    - no-slip adiabatic wall: momentum negated, rho and energy copied;
    - far field: every layer the characteristic state of the finite-volume
      path's far field (Riemann invariants along the outward normal, from
      the first owner cell and the freestream);
* restriction: one bounded direction, both of whose faces carry a condition,
  and periodic transverse directions (no corner ghost blocks are needed
  then); the two ghost blocks close the bounded direction into a ring so that
  every link of the joined-block table is mutual.  The wall-bump geometry
  (periodic x and z, wall and far field across y) has this form, and so has
  the one-GPU share (blocks tiling x and z, wall and far field across the
  third direction): ClosedBlocks cuts the periodic directions into owners,
  each with its ghost blocks joined to its neighbours' ghost blocks.

Pins (tests/test_oracle_closures.py): a uniform stream on the curved wall-bump
grid with the far field on both bounded faces stays uniform; a state mirrored
about a flat slip wall gives, with the closures, the residual of the
periodic domain of twice the height that holds the state and its mirror image
(inviscid and viscous); the vertex extension reproduces a grid that is linear
along the bounded direction; away from the boundary the closed residual does
not see the closure; owners tiling the periodic directions give bitwise
the single closed block's residual; and a block closed across two
directions (ClosedDuct: corner ghost blocks filled in sweep order) keeps a
uniform stream on the warm-start channel grid and, with walls on all four
faces of a flat duct, gives the periodic residual of the field mirrored
across both directions (a skipped corner fill fails it).
"""
from __future__ import annotations

from types import SimpleNamespace

import numpy as np

from . import highorder as ho
from .ghosts import FARFIELD, NOSLIP_ADIABATIC, SLIPWALL, _farfield_state

GHOST = 5
XLAYERS = 7          # extrapolated vertex planes beyond a bounded face (a ghost block's vertices -3 .. 6)


def _axis(d):
    return 3 - d     # array axis of direction d in [3, k, j, i]


def extended_vertices(Xv: np.ndarray, period, bounded: int):
    """Xv [3, ...]: the owner's vertices; along periodic directions the n
    upper corners 0 .. n - 1 (period[d] is the grid's displacement over one
    period), along the bounded direction the n + 1 planes -1 .. n - 1.
    Returns (E, origin): E spans vertices -3 .. n + 1 along periodic
    directions and -1 - XLAYERS .. n - 1 + XLAYERS along the bounded one;
    origin[d] is the array index of vertex 0 along d."""
    shape = Xv.shape[1:]
    n = [shape[2], shape[1], shape[0]]
    if bounded in range(3):
        n[bounded] -= 1
    X = Xv
    origin = [0, 0, 0]
    for d in range(3):
        ax = _axis(d)
        if d == bounded:
            continue
        idx = np.arange(-3, n[d] + 2)
        wrap, q = idx % n[d], idx // n[d]
        X = np.take(X, wrap, axis=ax)
        shp = [1, 1, 1, 1]
        shp[ax] = idx.size
        X = X + q.reshape(shp) * np.asarray(period[d], dtype=np.float64).reshape(3, 1, 1, 1)
        origin[d] = 3
    if bounded in range(3):
        ax = _axis(bounded)
        L = XLAYERS                                             # planes -1 - L .. -2 below plane -1
        lo0, lo1 = ho._win(X, ax, 0, 1), ho._win(X, ax, 1, 1)
        hi0, hi1 = ho._win(X, ax, n[bounded], 1), ho._win(X, ax, n[bounded] - 1, 1)
        below = [lo0 + m * (lo0 - lo1) for m in range(L, 0, -1)]
        above = [hi0 + m * (hi0 - hi1) for m in range(1, XLAYERS + 1)]
        X = np.concatenate(below + [X] + above, axis=ax)
        origin[bounded] = L + 1                                 # plane -1 sits at index L
    return X, origin


def layout(n, bounded: int, kinds):
    """Blocks and neighbour table of an owner of n cells with a ghost block on
    each face of the bounded direction.  kinds = (kind of the low face, kind
    of the high face), each ghosts.FARFIELD, SLIPWALL or NOSLIP_ADIABATIC.
    Returns (dims, nbr, ghosts) with ghosts = [(block, side, kind)]; block 0
    is the owner, 1 the low ghost block, 2 the high one.  Along the bounded
    direction the three close into a ring (the low ghost's far face joins
    the high ghost's), so every link is mutual; the owner's residual never
    reads past its ghost blocks' first five cells."""
    if len(kinds) != 2 or any(k not in (FARFIELD, SLIPWALL, NOSLIP_ADIABATIC) for k in kinds):
        raise ValueError("both faces of the bounded direction need a wall or far-field condition")
    m = list(n)
    m[bounded] = GHOST
    dims = [tuple(n), tuple(m), tuple(m)]
    nbr = [[b] * 6 for b in range(3)]
    lo, hi = 2 * bounded, 2 * bounded + 1
    nbr[0][lo], nbr[1][hi] = 1, 0
    nbr[0][hi], nbr[2][lo] = 2, 0
    nbr[1][lo], nbr[2][hi] = 2, 1
    return dims, nbr, [(1, 0, kinds[0]), (2, 1, kinds[1])]


def block_metrics(E, origin, n, bounded, ghosts):
    """(S, Jinv) of the owner and of every ghost block from their windows of
    the extended vertices."""
    def window(lo):
        Xw = E
        for d in range(3):
            ext = (n[d] if d != bounded or lo is None else GHOST) + 5
            start = origin[d] - 3 + (0 if d != bounded or lo is None else lo)
            Xw = ho._win(Xw, _axis(d), start, ext)
        return Xw
    out = [ho.metrics6(window(None))]
    for _, side, _ in ghosts:
        lo = -GHOST if side == 0 else n[bounded]
        out.append(ho.metrics6(window(lo)))
    return out


def fill_ghosts(Qs, Ss, bounded, ghosts, gamma, freestream):
    """Refill the ghost blocks' states (Qs[g], in place) from the owner Qs[0].
    freestream: (mach, alpha, beta) of the far field."""
    d = bounded
    ax = _axis(d)
    Q = Qs[0]
    n = Q.shape[ax]
    params = SimpleNamespace(gamma=gamma, mach=freestream[0], alpha=freestream[1], beta=freestream[2])
    for g, side, kind in ghosts:
        # unit normal of the boundary face (+d direction): the ghost block's
        # last face below the owner, the owner's last face above it
        Sb = ho._win(Ss[g][d], ax, GHOST - 1, 1) if side == 0 else ho._win(Ss[0][d], ax, n - 1, 1)
        nhat = Sb / np.sqrt(np.sum(Sb * Sb, axis=0))
        for m in range(1, GHOST + 1):
            own = m - 1 if side == 0 else n - m
            loc = GHOST - m if side == 0 else m - 1
            Qi = ho._win(Q, ax, own, 1)
            if kind == SLIPWALL:
                Qg = Qi.copy()
                mn = np.sum(Qi[1:4] * nhat, axis=0)
                Qg[1:4] = Qi[1:4] - 2.0 * mn[None] * nhat
            elif kind == NOSLIP_ADIABATIC:
                Qg = Qi.copy()
                Qg[1:4] = -Qi[1:4]
            elif kind == FARFIELD:
                Q0 = ho._win(Q, ax, 0 if side == 0 else n - 1, 1)
                Qg = _farfield_state(Q0, -nhat if side == 0 else nhat, params)
            else:
                raise ValueError(f"unknown boundary kind {kind}")
            sl = [slice(None)] * 4
            sl[ax] = slice(loc, loc + 1)
            Qs[g][tuple(sl)] = Qg


class Closed:
    """An owner block with ghost blocks: geometry set up once."""

    def __init__(self, Xv, period, bounded, kinds, gamma=1.4, freestream=(0.5, 0.0, 0.0)):
        self.bounded = bounded
        shape = Xv.shape[1:]
        n = [shape[2], shape[1], shape[0]]
        n[bounded] -= 1
        self.n = tuple(n)
        self.E, self.origin = extended_vertices(Xv, period, bounded)
        self.dims, self.nbr, self.ghosts = layout(self.n, bounded, kinds)
        mets = block_metrics(self.E, self.origin, self.n, bounded, self.ghosts)
        self.S = [m[0] for m in mets]
        self.Jinv = [m[1] for m in mets]
        self.gamma = gamma
        self.freestream = freestream

    def blocks(self, Q):
        """[owner, ghost blocks] with the ghost states filled from Q."""
        Qs = [Q] + [np.zeros((5,) + tuple(reversed(m))) for m in self.dims[1:]]
        fill_ghosts(Qs, self.S, self.bounded, self.ghosts, self.gamma, self.freestream)
        return Qs

    def residual(self, Q, eps_h=0.1, eps=1e-6, viscous=None):
        """R (dQ/dt = -R) of the owner; viscous = (prandtl, mu_inf, s_star) adds
        the fourth-order viscous terms."""
        Qs = self.blocks(Q)
        R = ho.wcns5_euler_residual_blocks(Qs, self.S, self.Jinv, self.nbr, self.gamma, eps_h, eps)[0]
        if viscous is not None:
            R = R + ho.viscous_residual_blocks(Qs, self.S, self.Jinv, self.nbr, self.gamma, *viscous)[0]
        return R

    def ns_steps(self, Q, dt, nsteps, eps_h=0.1, eps=1e-6, viscous=None):
        """nsteps SSP-RK3 steps (Eqs. 4-6, lambda = -dt) with the ghost blocks
        refilled before every stage's residual."""
        from .solver import ssp_rk3
        q = Q
        for _ in range(nsteps):
            q = ssp_rk3(q, dt, lambda x: self.residual(x, eps_h, eps, viscous))
        return q


class ClosedBlocks:
    """Owner blocks tiling a grid that is periodic along the two directions
    other than `bounded`, each owner with its two ghost blocks.  Xv: the whole
    grid's vertices as for extended_vertices; cuts[d] (d != bounded): the
    block boundaries along d, a list 0 = c_0 < c_1 < ... < c_m = n_d.  Owners
    are numbered along the first periodic direction fastest; block 3 o is
    owner o, 3 o + 1 its low ghost block, 3 o + 2 its high one.  Owners join
    their neighbours across the cuts (wrapping around the periodic
    directions); a ghost block joins the same-side ghost block of its owner's
    neighbour, so the ghost layers of a tiling are the ghost layers of the
    untiled block cut the same way."""

    def __init__(self, Xv, period, bounded, kinds, cuts, gamma=1.4, freestream=(0.5, 0.0, 0.0)):
        if len(kinds) != 2 or any(k not in (FARFIELD, SLIPWALL, NOSLIP_ADIABATIC) for k in kinds):
            raise ValueError("both faces of the bounded direction need a wall or far-field condition")
        self.bounded, self.kinds, self.gamma, self.freestream = bounded, tuple(kinds), gamma, freestream
        shape = Xv.shape[1:]
        N = [shape[2], shape[1], shape[0]]
        N[bounded] -= 1
        self.N = tuple(N)
        self.E, self.origin = extended_vertices(Xv, period, bounded)
        per = [d for d in range(3) if d != bounded]
        self.per = per
        self.cuts = {d: list(cuts[d]) for d in per}
        for d in per:
            c = self.cuts[d]
            if c[0] != 0 or c[-1] != N[d] or any(b <= a for a, b in zip(c, c[1:])):
                raise ValueError(f"bad cuts along {d}: {c}")
        m0, m1 = len(self.cuts[per[0]]) - 1, len(self.cuts[per[1]]) - 1
        self.tiles = (m0, m1)
        self.owners = []           # (lo index per direction, extents)
        for b1 in range(m1):
            for b0 in range(m0):
                lo, ext = [0, 0, 0], list(N)
                for d, b in ((per[0], b0), (per[1], b1)):
                    lo[d] = self.cuts[d][b]
                    ext[d] = self.cuts[d][b + 1] - self.cuts[d][b]
                self.owners.append((tuple(lo), tuple(ext)))
        no = len(self.owners)
        self.dims, self.nbr = [], []
        for o, (lo, ext) in enumerate(self.owners):
            g = list(ext)
            g[bounded] = GHOST
            self.dims += [tuple(ext), tuple(g), tuple(g)]
        self.nbr = [[0] * 6 for _ in range(3 * no)]
        B = 2 * bounded
        for o in range(no):
            b0, b1 = o % m0, o // m0
            for d, (t, m) in zip(per, ((b0, m0), (b1, m1))):
                for side in (0, 1):
                    step = -1 if side == 0 else 1
                    tn = (t + step) % m
                    on = (tn + b1 * m0) if d == per[0] else (b0 + tn * m0)
                    for r in range(3):                      # owner, low ghost, high ghost
                        self.nbr[3 * o + r][2 * d + side] = 3 * on + r
            self.nbr[3 * o][B], self.nbr[3 * o + 1][B + 1] = 3 * o + 1, 3 * o
            self.nbr[3 * o][B + 1], self.nbr[3 * o + 2][B] = 3 * o + 2, 3 * o
            self.nbr[3 * o + 1][B], self.nbr[3 * o + 2][B + 1] = 3 * o + 2, 3 * o + 1
        self.S, self.Jinv = [], []
        for lo, ext in self.owners:
            for start, cnt in ((0, N[bounded]), (-GHOST, GHOST), (N[bounded], GHOST)):
                Xw = self.E
                for d in range(3):
                    if d == bounded:
                        s0, c0 = self.origin[d] - 3 + start, cnt + 5
                    else:
                        s0, c0 = self.origin[d] - 3 + lo[d], ext[d] + 5
                    Xw = ho._win(Xw, _axis(d), s0, c0)
                S, J = ho.metrics6(Xw)
                self.S.append(S)
                self.Jinv.append(J)

    def split(self, Q):
        """The owners' states cut from a whole-grid state [5, Nk, Nj, Ni]."""
        out = []
        for lo, ext in self.owners:
            sl = [slice(None)] + [slice(lo[d], lo[d] + ext[d]) for d in (2, 1, 0)]
            out.append(Q[tuple(sl)].copy())
        return out

    def blocks(self, Qo):
        """All blocks' states (owners Qo, ghost blocks filled from them)."""
        Qs = []
        for o, Q in enumerate(Qo):
            g = [np.zeros((5,) + tuple(reversed(self.dims[3 * o + r]))) for r in (1, 2)]
            trio = [Q] + g
            fill_ghosts(trio, [self.S[3 * o], self.S[3 * o + 1], self.S[3 * o + 2]], self.bounded,
                        [(1, 0, self.kinds[0]), (2, 1, self.kinds[1])], self.gamma, self.freestream)
            Qs += trio
        return Qs

    def residual(self, Qo, eps_h=0.1, eps=1e-6, viscous=None):
        """R of every owner (list)."""
        Qs = self.blocks(Qo)
        R = ho.wcns5_euler_residual_blocks(Qs, self.S, self.Jinv, self.nbr, self.gamma, eps_h, eps)
        if viscous is not None:
            V = ho.viscous_residual_blocks(Qs, self.S, self.Jinv, self.nbr, self.gamma, *viscous)
            R = [a + b for a, b in zip(R, V)]
        return [R[3 * o] for o in range(len(self.owners))]


def extended_vertices_multi(Xv: np.ndarray, period, bounded):
    """extended_vertices for one or two bounded directions (ascending tuple):
    the periodic directions wrapped first, then each bounded direction in
    ascending order continued linearly past both ends (the corner vertices
    past two ends come from continuing the already continued planes)."""
    bounded = tuple(sorted(bounded))
    shape = Xv.shape[1:]
    n = [shape[2], shape[1], shape[0]]
    for d in bounded:
        n[d] -= 1
    X = Xv
    origin = [0, 0, 0]
    for d in range(3):
        if d in bounded:
            continue
        ax = _axis(d)
        idx = np.arange(-3, n[d] + 2)
        wrap, q = idx % n[d], idx // n[d]
        X = np.take(X, wrap, axis=ax)
        shp = [1, 1, 1, 1]
        shp[ax] = idx.size
        X = X + q.reshape(shp) * np.asarray(period[d], dtype=np.float64).reshape(3, 1, 1, 1)
        origin[d] = 3
    for d in bounded:
        ax = _axis(d)
        lo0, lo1 = ho._win(X, ax, 0, 1), ho._win(X, ax, 1, 1)
        hi0, hi1 = ho._win(X, ax, n[d], 1), ho._win(X, ax, n[d] - 1, 1)
        below = [lo0 + m * (lo0 - lo1) for m in range(XLAYERS, 0, -1)]
        above = [hi0 + m * (hi0 - hi1) for m in range(1, XLAYERS + 1)]
        X = np.concatenate(below + [X] + above, axis=ax)
        origin[d] = XLAYERS + 1
    return X, origin


class ClosedDuct:
    """One owner block periodic along one direction and closed across the
    other two (bounded = (d1, d2), d1 < d2; kinds[d] = (low kind, high kind)):
    ghost blocks on its four bounded faces and corner ghost blocks where two
    of them meet.  Blocks: 0 owner; 1, 2 the low and high ghost blocks across
    d1; 3, 4 across d2; 5 .. 8 the corners (d1 side, d2 side) = (lo, lo),
    (lo, hi), (hi, lo), (hi, hi).  Along each bounded direction the ghost
    blocks close into rings, so every link is mutual.  Fill order (the sweep
    order of the finite-volume ghost fill): across d1 from the owner, then
    across d2 from the owner and, for the corners, from the d1 ghost blocks
    (the d2 condition applied to their cells)."""

    def __init__(self, Xv, period, bounded, kinds, gamma=1.4, freestream=(0.5, 0.0, 0.0)):
        d1, d2 = sorted(bounded)
        self.d1, self.d2, self.kinds, self.gamma, self.freestream = d1, d2, kinds, gamma, freestream
        for d in (d1, d2):
            if len(kinds[d]) != 2 or any(k not in (FARFIELD, SLIPWALL, NOSLIP_ADIABATIC) for k in kinds[d]):
                raise ValueError("every bounded face needs a wall or far-field condition")
        shape = Xv.shape[1:]
        n = [shape[2], shape[1], shape[0]]
        n[d1] -= 1
        n[d2] -= 1
        self.n = tuple(n)
        self.E, self.origin = extended_vertices_multi(Xv, period, (d1, d2))
        # (start, count) along d1 and d2 for each block, in block order
        G = GHOST
        spans = {d: {"own": (0, n[d]), "lo": (-G, G), "hi": (n[d], G)} for d in (d1, d2)}
        order = [("own", "own"), ("lo", "own"), ("hi", "own"), ("own", "lo"), ("own", "hi"),
                 ("lo", "lo"), ("lo", "hi"), ("hi", "lo"), ("hi", "hi")]
        self.where = order
        self.dims = []
        self.S, self.Jinv = [], []
        for w1, w2 in order:
            ext = list(n)
            ext[d1] = spans[d1][w1][1]
            ext[d2] = spans[d2][w2][1]
            self.dims.append(tuple(ext))
            Xw = self.E
            for d in range(3):
                if d == d1:
                    st, c = spans[d1][w1]
                elif d == d2:
                    st, c = spans[d2][w2]
                else:
                    st, c = 0, n[d]
                Xw = ho._win(Xw, _axis(d), self.origin[d] - 3 + st, c + 5)
            S, J = ho.metrics6(Xw)
            self.S.append(S)
            self.Jinv.append(J)
        idx = {w: b for b, w in enumerate(order)}
        nxt = {"lo": "own", "own": "hi", "hi": "lo"}          # the block above along a bounded direction (ring)
        self.nbr = [[b] * 6 for b in range(9)]
        for b, (w1, w2) in enumerate(order):
            up1, up2 = idx[(nxt[w1], w2)], idx[(w1, nxt[w2])]
            self.nbr[b][2 * d1 + 1] = up1
            self.nbr[up1][2 * d1] = b
            self.nbr[b][2 * d2 + 1] = up2
            self.nbr[up2][2 * d2] = b
        # fills: (source block, low ghost, high ghost, direction, kinds), in order
        self.fills = [(0, 1, 2, d1, kinds[d1]), (0, 3, 4, d2, kinds[d2]),
                      (1, 5, 6, d2, kinds[d2]), (2, 7, 8, d2, kinds[d2])]

    def blocks(self, Q):
        Qs = [Q] + [np.zeros((5,) + tuple(reversed(m))) for m in self.dims[1:]]
        for src, lo, hi, d, k in self.fills:
            trio = [Qs[src], Qs[lo], Qs[hi]]
            fill_ghosts(trio, [self.S[src], self.S[lo], self.S[hi]], d, [(1, 0, k[0]), (2, 1, k[1])], self.gamma,
                        self.freestream)
        return Qs

    def residual(self, Q, eps_h=0.1, eps=1e-6, viscous=None):
        Qs = self.blocks(Q)
        R = ho.wcns5_euler_residual_blocks(Qs, self.S, self.Jinv, self.nbr, self.gamma, eps_h, eps)[0]
        if viscous is not None:
            R = R + ho.viscous_residual_blocks(Qs, self.S, self.Jinv, self.nbr, self.gamma, *viscous)[0]
        return R

    def ns_steps(self, Q, dt, nsteps, eps_h=0.1, eps=1e-6, viscous=None):
        from .solver import ssp_rk3
        q = Q
        for _ in range(nsteps):
            q = ssp_rk3(q, dt, lambda x: self.residual(x, eps_h, eps, viscous))
        return q
