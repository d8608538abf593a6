"""Block split and regroup for load balance (oracle; plain Python).

Test infrastructure, like the rest of this package.

Section 3.2.1: the original mesh zones are cut into many small blocks, and the
blocks are then regrouped into the final groups that the processes own.  The
paper leaves the algorithm to a separate pre-processing tool and prints none
of it; these are the readings this solver takes:

* split plan: a block of more than ``max_cells`` cells is cut in two across
  its longest index direction (equal extents: the higher direction, k before
  j before i); both parts are split again by the same rule.  A part whose
  every extent is below 2 * ``min_width`` is kept whole, however large.  The
  lower part takes the multiple of ``align[d]`` nearest n/2 (equal distance:
  the lower one) when that lies in [n/4, 3n/4] and leaves both parts at
  least ``min_width`` cells, else floor(n/2); with align 1 always floor(n/2).
  Aligned cuts keep the pieces on the kernels' tile grid (64 cells in i, 8 in
  j).  Pieces are listed block by block, depth first, lower part first.
* split tables: a piece face inside its parent becomes a connection to every
  sibling piece across it (no shift); a piece face on its parent's face takes
  the parent's boundary patches and connections on that face, cut to the
  piece, and a connection is cut again to every piece of the neighbour block
  that it reaches.  The split case is the same discrete problem as the
  parent case.
* regroup: longest processing time first (Graham, 1969).  Pieces in
  decreasing load (equal loads: lower index first) each go to the group whose
  load after taking the piece, divided by the group's capacity, is least
  (equal: lower group).  Capacities carry the paper's load ratio between
  unlike devices (Section 3.2.1); equal capacities give Graham's bound
  max load <= (4/3 - 1/(3m)) x optimum for m groups.

Pins: the plan tiles every block exactly once (brute force), closed-form
plans of cubes, the LPT bound against a brute-force optimum, a hand-worked
regroup, and the oracle solver giving bitwise the same states on a split case
as on its parent.
"""
from __future__ import annotations

import itertools
from dataclasses import dataclass, replace
from typing import List, Sequence, Tuple


@dataclass(frozen=True)
class Piece:
    parent: int
    lo: Tuple[int, int, int]
    n: Tuple[int, int, int]

    @property
    def cells(self) -> int:
        return self.n[0] * self.n[1] * self.n[2]


@dataclass(frozen=True)
class SplitConn:
    blk: int
    face: int
    nbr: int
    nbr_face: int
    lo: Tuple[int, int]
    hi: Tuple[int, int]
    nbr_lo: Tuple[int, int]
    shift: Tuple[float, float, float] = (0.0, 0.0, 0.0)


@dataclass(frozen=True)
class SplitBC:
    blk: int
    face: int
    kind: int
    lo: Tuple[int, int]
    hi: Tuple[int, int]
    mach: float = 0.0


def _transverse(d):
    return tuple(t for t in range(3) if t != d)


def cut_position(n: int, align: int, min_width: int) -> int:
    """Cells of the lower part when n cells are cut in two (the reading above)."""
    below = (n // (2 * align)) * align          # the multiple of align at or below n/2
    above = below + align
    c = below if n - 2 * below <= 2 * above - n else above
    if c > 0 and n <= 4 * c <= 3 * n and min_width <= c <= n - min_width:
        return c
    return n // 2


def split_plan(dims: Sequence[Sequence[int]], max_cells: int, min_width: int = 2,
               align: Sequence[int] = (1, 1, 1)) -> List[Piece]:
    """Recursive bisection of every block (the reading above)."""
    out: List[Piece] = []

    def visit(b, lo, n):
        if n[0] * n[1] * n[2] > max_cells:
            d = max(range(3), key=lambda t: (n[t], t))
            if n[d] >= 2 * min_width:
                h = cut_position(n[d], align[d], min_width)
                n_lo = list(n)
                n_lo[d] = h
                n_hi = list(n)
                n_hi[d] = n[d] - h
                lo_hi = list(lo)
                lo_hi[d] = lo[d] + h
                visit(b, tuple(lo), tuple(n_lo))
                visit(b, tuple(lo_hi), tuple(n_hi))
                return
        out.append(Piece(b, tuple(lo), tuple(n)))

    for b, dm in enumerate(dims):
        visit(b, (0, 0, 0), tuple(int(v) for v in dm))
    return out


def _on_face(p: Piece, dims, face) -> bool:
    d, side = face // 2, face % 2
    if side == 0:
        return p.lo[d] == 0
    return p.lo[d] + p.n[d] == dims[p.parent][d]


def _span(p: Piece, d):
    """Transverse half-open range of piece p on a d-face, in parent indices."""
    t1, t2 = _transverse(d)
    return (p.lo[t1], p.lo[t2]), (p.lo[t1] + p.n[t1], p.lo[t2] + p.n[t2])


def _cut(lo_a, hi_a, lo_b, hi_b):
    lo = (max(lo_a[0], lo_b[0]), max(lo_a[1], lo_b[1]))
    hi = (min(hi_a[0], hi_b[0]), min(hi_a[1], hi_b[1]))
    if lo[0] >= hi[0] or lo[1] >= hi[1]:
        return None
    return lo, hi


def split_tables(dims, conns, bcs, pieces: Sequence[Piece]):
    """Connection and boundary tables of the pieces (the reading above)."""
    by_parent = {}
    for q, p in enumerate(pieces):
        by_parent.setdefault(p.parent, []).append(q)
    out_c: List[SplitConn] = []
    out_b: List[SplitBC] = []
    for bc in bcs:
        d = bc.face // 2
        for q in by_parent[bc.blk]:
            p = pieces[q]
            if not _on_face(p, dims, bc.face):
                continue
            plo, phi = _span(p, d)
            r = _cut(tuple(bc.lo), tuple(bc.hi), plo, phi)
            if r is None:
                continue
            lo, hi = r
            out_b.append(SplitBC(q, bc.face, bc.kind, (lo[0] - plo[0], lo[1] - plo[1]),
                                 (hi[0] - plo[0], hi[1] - plo[1]), getattr(bc, "mach", 0.0)))
    for c in conns:
        d = c.face // 2
        off = (c.nbr_lo[0] - c.lo[0], c.nbr_lo[1] - c.lo[1])    # this side -> neighbour's transverse index
        for q in by_parent[c.blk]:
            p = pieces[q]
            if not _on_face(p, dims, c.face):
                continue
            plo, phi = _span(p, d)
            r = _cut(tuple(c.lo), tuple(c.hi), plo, phi)
            if r is None:
                continue
            for s in by_parent[c.nbr]:
                ps = pieces[s]
                if not _on_face(ps, dims, c.nbr_face):
                    continue
                slo, shi = _span(ps, d)
                rn = _cut((r[0][0] + off[0], r[0][1] + off[1]), (r[1][0] + off[0], r[1][1] + off[1]), slo, shi)
                if rn is None:
                    continue
                lo_n, hi_n = rn
                lo = (lo_n[0] - off[0] - plo[0], lo_n[1] - off[1] - plo[1])
                hi = (hi_n[0] - off[0] - plo[0], hi_n[1] - off[1] - plo[1])
                out_c.append(SplitConn(q, c.face, s, c.nbr_face, lo, hi,
                                       (lo_n[0] - slo[0], lo_n[1] - slo[1]), tuple(c.shift)))
    for qs in by_parent.values():
        for a in qs:
            for b in qs:
                pa, pb = pieces[a], pieces[b]
                for d in range(3):
                    if pa.lo[d] + pa.n[d] != pb.lo[d]:
                        continue
                    alo, ahi = _span(pa, d)
                    blo, bhi = _span(pb, d)
                    r = _cut(alo, ahi, blo, bhi)
                    if r is None:
                        continue
                    lo, hi = r
                    out_c.append(SplitConn(a, 2 * d + 1, b, 2 * d, (lo[0] - alo[0], lo[1] - alo[1]),
                                           (hi[0] - alo[0], hi[1] - alo[1]), (lo[0] - blo[0], lo[1] - blo[1])))
                    out_c.append(SplitConn(b, 2 * d, a, 2 * d + 1, (lo[0] - blo[0], lo[1] - blo[1]),
                                           (hi[0] - blo[0], hi[1] - blo[1]), (lo[0] - alo[0], lo[1] - alo[1])))
    return out_c, out_b


def split_case(case, max_cells: int, min_width: int = 2, align: Sequence[int] = (1, 1, 1)):
    """The case cut into pieces: same object type, sliced nodes and states."""
    pieces = split_plan(case.dims, max_cells, min_width, align)
    conns, bcs = split_tables(case.dims, case.conns, case.bcs, pieces)
    nodes, q0, dims = [], [], []
    for p in pieces:
        (i0, j0, k0), (ni, nj, nk) = p.lo, p.n
        dims.append((ni, nj, nk))
        nodes.append(case.nodes[p.parent][:, k0:k0 + nk + 1, j0:j0 + nj + 1, i0:i0 + ni + 1].copy())
        q0.append(case.q0[p.parent][:, k0:k0 + nk, j0:j0 + nj, i0:i0 + ni].copy())
    return replace(case, dims=dims, nodes=nodes, conns=conns, bcs=bcs, q0=q0), pieces


def regroup(loads: Sequence[int], ngroups: int, capacity: Sequence[float] | None = None):
    """LPT assignment (the reading above): (group of each item, load per group)."""
    cap = [1.0] * ngroups if capacity is None else [float(c) for c in capacity]
    order = sorted(range(len(loads)), key=lambda i: (-loads[i], i))
    total = [0] * ngroups
    group = [-1] * len(loads)
    for i in order:
        g = min(range(ngroups), key=lambda h: ((total[h] + loads[i]) / cap[h], h))
        group[i] = g
        total[g] += loads[i]
    return group, total


def optimal_max_load(loads: Sequence[int], ngroups: int) -> int:
    """Least possible largest group load, by trying every assignment (tiny inputs only)."""
    best = None
    for assign in itertools.product(range(ngroups), repeat=len(loads)):
        tot = [0] * ngroups
        for w, g in zip(loads, assign):
            tot[g] += w
        m = max(tot)
        best = m if best is None else min(best, m)
    return best
