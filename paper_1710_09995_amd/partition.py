"""Block split and regroup for load balance (Section 3.2.1).

The grid's blocks are cut into smaller pieces and the pieces dealt into
balanced groups, one per device.  The plan, the rewritten connection and
boundary tables and the grouping come from the library's host calls
(cfd_split_plan, cfd_split_tables, cfd_regroup in include/cfd.h, where their
rules are stated); this module marshals their arguments and slices each
piece's nodes and initial state from its parent.
"""
from __future__ import annotations

import ctypes as C
from dataclasses import dataclass, replace
from typing import List, Optional, Sequence, Tuple

import numpy as np

from . import binding as B
from . import cases


@dataclass(frozen=True)
class Piece:
    parent: int
    lo: Tuple[int, int, int]
    n: Tuple[int, int, int]

    @property
    def cells(self) -> int:
        return self.n[0] * self.n[1] * self.n[2]


# cuts on the stage kernels' tile grid: 64 cells in i (one wavefront), 8 rows in j
TILE_ALIGN = (64, 8, 1)


def split_plan(dims: Sequence[Sequence[int]], max_cells: int, min_width: int = 2,
               align: Sequence[int] = TILE_ALIGN) -> List[Piece]:
    L = B.lib()
    d = B.to_dims(dims)
    al = (C.c_int32 * 3)(*[int(v) for v in align])
    count = C.c_int32()
    B._check(L.cfd_split_plan(len(dims), d, int(max_cells), int(min_width), al, None, 0, C.byref(count)))
    arr = (B.PieceS * max(count.value, 1))()
    B._check(L.cfd_split_plan(len(dims), d, int(max_cells), int(min_width), al, arr, count.value,
                              C.byref(count)))
    return [Piece(a.parent, tuple(a.lo), tuple(a.n)) for a in arr[:count.value]]


def _to_pieces(pieces: Sequence[Piece]):
    arr = (B.PieceS * max(len(pieces), 1))()
    for q, p in enumerate(pieces):
        arr[q].parent = p.parent
        arr[q].lo[:] = list(p.lo)
        arr[q].n[:] = list(p.n)
    return arr


def split_tables(case: cases.Case, pieces: Sequence[Piece]):
    """(connections, boundary patches) of the pieces, as cases.Conn / cases.BC."""
    L = B.lib()
    args = (case.nblk, B.to_dims(case.dims), B.to_conns(case.conns), len(case.conns), B.to_bcs(case.bcs),
            len(case.bcs), _to_pieces(pieces), len(pieces))
    nc, nb = C.c_int32(), C.c_int32()
    B._check(L.cfd_split_tables(*args, None, 0, C.byref(nc), None, 0, C.byref(nb)))
    oc = (B.ConnS * max(nc.value, 1))()
    ob = (B.BCS * max(nb.value, 1))()
    B._check(L.cfd_split_tables(*args, oc, nc.value, C.byref(nc), ob, nb.value, C.byref(nb)))
    conns = [cases.Conn(c.blk, c.face, c.nbr, c.nbr_face, tuple(c.lo), tuple(c.hi), tuple(c.nbr_lo),
                        tuple(c.shift)) for c in oc[:nc.value]]
    bcs = [cases.BC(b.blk, b.face, b.kind, tuple(b.lo), tuple(b.hi), b.mach) for b in ob[:nb.value]]
    return conns, bcs


def split_case(case: cases.Case, max_cells: int, min_width: int = 2, align: Sequence[int] = TILE_ALIGN):
    """(the case cut into pieces, the pieces): same parameters, sliced nodes and states."""
    pieces = split_plan(case.dims, max_cells, min_width, align)
    conns, bcs = split_tables(case, pieces)
    dims, nodes, q0 = [], [], []
    for p in pieces:
        (i0, j0, k0), (ni, nj, nk) = p.lo, p.n
        dims.append((ni, nj, nk))
        nodes.append(case.nodes[p.parent][:, k0:k0 + nk + 1, j0:j0 + nj + 1, i0:i0 + ni + 1].copy())
        q0.append(case.q0[p.parent][:, k0:k0 + nk, j0:j0 + nj, i0:i0 + ni].copy())
    split = replace(case, name=case.name + "_split", dims=dims, nodes=nodes, conns=conns, bcs=bcs, q0=q0,
                    info=dict(case.info, split_from=case.name, max_cells=int(max_cells)))
    return split, pieces


def regroup(loads: Sequence[int], ngroups: int, capacity: Optional[Sequence[float]] = None):
    """(group of each item, total load of each group) by longest processing time first."""
    L = B.lib()
    n = len(loads)
    ld = (C.c_int64 * max(n, 1))(*[int(v) for v in loads])
    cap = None if capacity is None else (C.c_double * ngroups)(*[float(v) for v in capacity])
    grp = (C.c_int32 * max(n, 1))()
    tot = (C.c_int64 * ngroups)()
    B._check(L.cfd_regroup(n, ld, int(ngroups), cap, grp, tot))
    return list(grp[:n]), list(tot)


def assemble(case: cases.Case, pieces: Sequence[Piece], states) -> list:
    """Parent-block arrays [5, nk, nj, ni] from per-piece interior states."""
    out = [np.empty((5, nk, nj, ni)) for ni, nj, nk in case.dims]
    for p, s in zip(pieces, states):
        (i0, j0, k0), (ni, nj, nk) = p.lo, p.n
        out[p.parent][:, k0:k0 + nk, j0:j0 + nj, i0:i0 + ni] = s
    return out


def balance_report(dims: Sequence[Sequence[int]], groups: Sequence[int] = (8, 16, 32, 64, 128),
                   pieces_per_group: int = 4, min_width: int = 2, align: Sequence[int] = TILE_ALIGN) -> list:
    """For each group count G: the largest group load over the mean when the
    blocks are regrouped as they are, and when they are first split to at most
    total / (pieces_per_group * G) cells (loads in cells)."""
    loads = [int(a) * int(b) * int(c) for a, b, c in dims]
    total = sum(loads)
    rows = []
    for G in groups:
        _, t_blocks = regroup(loads, G)
        max_cells = max(1, total // (pieces_per_group * G))
        pieces = split_plan(dims, max_cells, min_width, align)
        _, t_pieces = regroup([p.cells for p in pieces], G)
        rows.append({"groups": G, "blocks": len(loads), "max_over_mean_blocks": max(t_blocks) * G / total,
                     "max_cells": max_cells, "pieces": len(pieces),
                     "max_over_mean_pieces": max(t_pieces) * G / total})
    return rows
