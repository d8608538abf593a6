"""Multigrid cycle for steady marches (oracle; plain FP64 NumPy; test
infrastructure, imported only by the tests).

A steady solve drives the residual of Eq. (3) to zero, and the convergence
test of Section 2.3 asks for a given residual drop.  The explicit stage update
of Eqs. (4)-(6) with local steps damps the smooth error modes of a fine grid
slowly (measured on the channel family: the steps per decade grow about with
the square of the cell count along the channel).  The paper names no
convergence accelerator; this library's is the full-approximation-storage
(FAS) scheme on nested grids with the RK3 step as the smoother:

* levels 0 (the given grid) .. L-1, each coarse cell the union of 2 x 2 x 2
  cells of the level above (cases.coarsen_case), the same boundary and
  connection tables;
* one V-cycle: going down, on each level l, `pre` RK3 steps (Eqs. 4-6, the
  level's own CFL steps, local or global as the case says) of
  dQ/dt = -(R_l(Q) + F_l), F_0 = 0 (the coarsest level takes `coarse`
  steps); then the next level's state and forcing,
      Q_{l+1}^0 = sum_children V Q / sum_children V          (volume-weighted mean)
      F_{l+1}   = sum_children V (R_l(Q_l) + F_l) / V_{l+1} - R_{l+1}(Q_{l+1}^0),
  so that a level whose own residual vanishes sees none on the coarse grid;
  going up, Q_l += Q_{l+1} - Q_{l+1}^0 on each of the parent's 8 children
  (the coarse correction injected);
* the history row of a cycle is that of the finest level's first step (about
  the state at the start of the cycle; the norms of R_0 without forcing).

Pins (tests/test_oracle_multigrid.py): one level is plain RK3 (bitwise the
solver's step); restriction keeps sum V Q where the coarse volumes are the
sums of the fine ones; on a periodic box a cycle keeps the conserved totals;
and three-level cycles converge to the RK3 march's steady state (a wrong
forcing on any level does not).  Parity unpinned: the unit scale of the
injected correction and the volume weights of the restricted residual, which
set how fast the cycles converge but not the state they converge to.
"""
from __future__ import annotations

from typing import List

from . import solver as osol
from .solver import interior


def _children(a):
    """The 8 children views (every second cell from each corner offset, dk
    slowest, di fastest) of an interior array a [..., 2nk, 2nj, 2ni], one
    entry per cell of the coarse grid."""
    out = []
    for dk in (0, 1):
        for dj in (0, 1):
            for di in (0, 1):
                out.append(a[..., dk::2, dj::2, di::2])
    return out


def smooth(st, F, nsteps, record=False):
    """nsteps RK3 steps of dQ/dt = -(R(Q) + F) in place on the oracle state st
    (F: interior arrays per block, or None).  Returns the first step's history
    row (about the state at its start, R without F) when record is set."""
    c = st.case
    g = st.g
    first = None
    ints = [(slice(None), slice(g, g + nk), slice(g, g + nj), slice(g, g + ni)) for (ni, nj, nk) in c.dims]
    for n in range(nsteps):
        osol.fill(st)
        dt = osol.time_step(st)
        Qn = [Q.copy() for Q in st.Qs]

        def dtb(b):
            return dt[b] if isinstance(dt, list) else dt

        def RF(Qs, fill):
            R = osol.residual(st, Qs, fill_first=fill)
            return R if F is None else [r + f for r, f in zip(R, F)]
        R0 = RF(Qn, False)
        if record and n == 0:
            R0_plain = osol.residual(st, Qn, fill_first=False)
            dtv = dt if not isinstance(dt, list) else min(float(x.min()) for x in dt)
            first = [dtv] + osol.norms_from(st, Qn, R0_plain)
        Q1 = [Q.copy() for Q in Qn]
        for b in range(c.nblk):
            Q1[b][ints[b]] = Qn[b][ints[b]] - dtb(b) * R0[b]
        R1 = RF(Q1, True)
        Q2 = [Q.copy() for Q in Qn]
        for b in range(c.nblk):
            Q2[b][ints[b]] = 0.75 * Qn[b][ints[b]] + 0.25 * (Q1[b][ints[b]] - dtb(b) * R1[b])
        R2 = RF(Q2, True)
        for b in range(c.nblk):
            st.Qs[b][ints[b]] = (1.0 / 3.0) * Qn[b][ints[b]] + (2.0 / 3.0) * (Q2[b][ints[b]] - dtb(b) * R2[b])
    return first


def restrict(st, cn, F):
    """The coarse level's initial state (written into cn) and forcing from the
    fine level st with forcing F (None on the finest level).  Returns
    (Q0 per block, F_coarse per block)."""
    c = st.case
    g = st.g
    R = osol.residual(st)
    Rtot = R if F is None else [a + f for a, f in zip(R, F)]
    Fn, Q0 = [], []
    for b in range(c.nblk):
        vf = interior(st.Vs[b], c.dims[b], g)
        qf = interior(st.Qs[b], c.dims[b], g)
        num = sum(v * q for v, q in zip(_children(vf), _children(qf)))
        den = sum(_children(vf))
        interior(cn.Qs[b], cn.case.dims[b], g)[...] = num / den
        Q0.append(num / den)
        Fn.append(sum(_children(vf * Rtot[b])) / interior(cn.Vs[b], cn.case.dims[b], g))
    Rc = osol.residual(cn)
    return Q0, [f - rc for f, rc in zip(Fn, Rc)]


def v_cycle(levels: List[osol.OracleState], pre: int = 1, coarse: int = 2):
    """One V-cycle in place on levels[0] (the other levels are working grids).
    Returns the finest level's history row of the cycle."""
    L = len(levels)
    F: List = [None] * L
    Q0: List = [None] * L
    row = None
    for l in range(L):
        r = smooth(levels[l], F[l], coarse if l == L - 1 else pre, record=(l == 0))
        if l == 0:
            row = r
        if l == L - 1:
            break
        Q0[l + 1], F[l + 1] = restrict(levels[l], levels[l + 1], F[l])
    for l in range(L - 2, -1, -1):
        st, cn = levels[l], levels[l + 1]
        g = st.g
        for b in range(st.case.nblk):
            corr = interior(cn.Qs[b], cn.case.dims[b], g) - Q0[l + 1][b]
            qf = interior(st.Qs[b], st.case.dims[b], g)
            for dk in (0, 1):
                for dj in (0, 1):
                    for di in (0, 1):
                        qf[..., dk::2, dj::2, di::2] += corr
    return row


def setup_levels(level_cases) -> List[osol.OracleState]:
    """Oracle states of a hierarchy: level_cases[0] is the grid, each next one
    its coarsening (cases.hierarchy)."""
    return [osol.setup(c) for c in level_cases]
