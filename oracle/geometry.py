"""Ghost nodes and curvilinear metrics (oracle; plain FP64 NumPy).

The paper solves Eq. (1) in curvilinear coordinates and requires a geometric
conservation law (Section 2.2) without printing the metric scheme.  The
reading used here is the closed-cell finite-volume one:

* each cell stores the area vectors of its three lower faces, S_i, S_j, S_k,
  and its volume V;
* a face vector is half the cross product of the two face diagonals,
  S_d = 1/2 (x[+t1+t2] - x[0]) x (x[+t2] - x[+t1]) with (t1, t2) the two
  other directions in cyclic order after d; on a unit cube S_d = e_d;
* the volume follows from the divergence theorem,
  V = 1/3 sum over the 6 faces of (mean of the face's 4 nodes) . S_out.

Because the 6 outward face vectors of a cell sum to zero exactly in exact
arithmetic, a uniform stream gives a zero residual (freestream preservation).

Arrays are padded with g ghost layers: nodes ``[3, nk+1+2g, nj+1+2g, ni+1+2g]``
(node n at index n+g), cell arrays ``[..., nk+2g, nj+2g, ni+2g]``.

Ghost nodes are filled in three sweeps, i then j then k.  Across a
connection they are the neighbour's nodes plus the periodic shift; on a
physical face they are linear extrapolations x_{-m} = x_0 + m (x_0 - x_1).
A sweep in direction d also covers the ghost layers of the directions swept
before it wherever a patch reaches the edge of its face; this defines the
edge and corner ("singular point", Section 3.2.3) values.

After metrics are computed from the ghost-filled nodes, the metrics of ghost
cells across a connection are replaced by the neighbour's interior metrics
(same sweeps as the state).  In particular the face vector on a block seam is
the one computed by the block on the + side of the seam, so both blocks see
the same bits for the shared face.
"""
from __future__ import annotations

import numpy as np

CYCLIC = {0: (1, 2), 1: (2, 0), 2: (0, 1)}


def transverse(d):
    return tuple(t for t in range(3) if t != d)


def axis(d, lead=1):
    """Array axis of index direction d for arrays [lead..., k, j, i]."""
    return lead + 2 - d


def patch_ranges(dims, face, lo, hi, g, nodes=False):
    """Transverse index ranges (half-open) that a patch covers in its sweep.

    Node patches additionally own the last node line of the face when the
    patch reaches the face's upper edge.  Directions swept before this one are
    extended into their ghost layers where the patch reaches the face edge.
    """
    d = face // 2
    out = {}
    for a, t in enumerate(transverse(d)):
        n = dims[t]
        start, end = lo[a], hi[a]
        if nodes and hi[a] == n:
            end = n + 1
        if t < d:
            if lo[a] == 0:
                start = -g
            if hi[a] == n:
                end = (n + 1 + g) if nodes else (n + g)
        out[t] = (start, end)
    return d, out


def index_grid(ranges3, g):
    """np.ix_ index for logical ranges {0:(a,b),1:(..),2:(..)} on a [k,j,i] array."""
    ii = np.arange(ranges3[0][0], ranges3[0][1]) + g
    jj = np.arange(ranges3[1][0], ranges3[1][1]) + g
    kk = np.arange(ranges3[2][0], ranges3[2][1]) + g
    return np.ix_(kk, jj, ii)


def pad_nodes(nodes, g):
    c, a, b, e = nodes.shape
    X = np.full((3, a + 2 * g, b + 2 * g, e + 2 * g), np.nan)
    X[:, g:g + a, g:g + b, g:g + e] = nodes
    return X


def fill_ghost_nodes(Xs, dims, conns, bcs, g):
    """Fill ghost nodes of every block in place (three sweeps)."""
    for d in range(3):
        # physical faces: linear extrapolation
        for bc in bcs:
            if bc.face // 2 != d:
                continue
            b = bc.blk
            n = dims[b][d]
            _, rg = patch_ranges(dims[b], bc.face, bc.lo, bc.hi, g, nodes=True)
            side = bc.face % 2
            x0 = 0 if side == 0 else n
            x1 = 1 if side == 0 else n - 1
            r0 = dict(rg)
            r0[d] = (x0, x0 + 1)
            r1 = dict(rg)
            r1[d] = (x1, x1 + 1)
            A0 = Xs[b][(slice(None),) + index_grid(r0, g)]
            A1 = Xs[b][(slice(None),) + index_grid(r1, g)]
            for m in range(1, g + 1):
                gm = -m if side == 0 else n + m
                rm = dict(rg)
                rm[d] = (gm, gm + 1)
                Xs[b][(slice(None),) + index_grid(rm, g)] = A0 + m * (A0 - A1)
        # connections: neighbour nodes plus shift
        for c in conns:
            if c.face // 2 != d:
                continue
            b, nb = c.blk, c.nbr
            n = dims[b][d]
            nn = dims[nb][d]
            _, rg = patch_ranges(dims[b], c.face, c.lo, c.hi, g, nodes=True)
            side = c.face % 2
            t1, t2 = transverse(d)
            shift = np.asarray(c.shift, dtype=np.float64).reshape(3, 1, 1, 1)
            for m in range(1, g + 1):
                gm = -m if side == 0 else n + m
                sm = nn - m if side == 0 else m
                rd = dict(rg)
                rd[d] = (gm, gm + 1)
                rs = {d: (sm, sm + 1),
                      t1: (rg[t1][0] - c.lo[0] + c.nbr_lo[0], rg[t1][1] - c.lo[0] + c.nbr_lo[0]),
                      t2: (rg[t2][0] - c.lo[1] + c.nbr_lo[1], rg[t2][1] - c.lo[1] + c.nbr_lo[1])}
                Xs[b][(slice(None),) + index_grid(rd, g)] = \
                    Xs[nb][(slice(None),) + index_grid(rs, g)] + shift


def _node(X, d_off):
    """View of padded nodes shifted by a node offset (oi, oj, ok)."""
    oi, oj, ok = d_off
    _, a, b, c = X.shape
    # cell-sized output: nk+2g x nj+2g x ni+2g = (a-1) x (b-1) x (c-1)
    return X[:, ok:ok + a - 1, oj:oj + b - 1, oi:oi + c - 1]


def face_vectors(X):
    """Lower-face area vectors of every padded cell: [3 (d), 3 (xyz), nk+2g, nj+2g, ni+2g]."""
    S = []
    for d in range(3):
        t1, t2 = CYCLIC[d]
        e1 = [0, 0, 0]
        e1[t1] = 1
        e2 = [0, 0, 0]
        e2[t2] = 1
        e12 = [a + b for a, b in zip(e1, e2)]
        a = _node(X, e12) - _node(X, (0, 0, 0))
        b = _node(X, e2) - _node(X, e1)
        S.append(0.5 * np.cross(a, b, axis=0))
    return np.stack(S)


def face_centres(X):
    """Mean of the 4 nodes of every lower face: [3 (d), 3, nk+2g, nj+2g, ni+2g]."""
    out = []
    for d in range(3):
        t1, t2 = CYCLIC[d]
        e1 = [0, 0, 0]
        e1[t1] = 1
        e2 = [0, 0, 0]
        e2[t2] = 1
        e12 = [a + b for a, b in zip(e1, e2)]
        out.append(0.25 * (_node(X, (0, 0, 0)) + _node(X, e1) + _node(X, e2) + _node(X, e12)))
    return np.stack(out)


def upper_face_vectors(X):
    """Face vectors at the +d face of every padded cell (from the nodes)."""
    out = []
    outc = []
    for d in range(3):
        t1, t2 = CYCLIC[d]
        ed = [0, 0, 0]
        ed[d] = 1
        e1 = [0, 0, 0]
        e1[t1] = 1
        e2 = [0, 0, 0]
        e2[t2] = 1
        p0 = ed
        p1 = [a + b for a, b in zip(ed, e1)]
        p2 = [a + b for a, b in zip(ed, e2)]
        p12 = [a + b + c for a, b, c in zip(ed, e1, e2)]
        a = _node(X, p12) - _node(X, p0)
        b = _node(X, p2) - _node(X, p1)
        out.append(0.5 * np.cross(a, b, axis=0))
        outc.append(0.25 * (_node(X, p0) + _node(X, p1) + _node(X, p2) + _node(X, p12)))
    return np.stack(out), np.stack(outc)


def volumes(X):
    """Cell volumes by the divergence theorem over the 6 faces.

    Face centres are measured from each cell's lowest node: the closed-surface
    formula does not depend on the origin, and a local one keeps the sum free
    of cancellation when coordinates are large compared with the cell.
    """
    S = face_vectors(X)
    C = face_centres(X)
    Su, Cu = upper_face_vectors(X)
    x0 = _node(X, (0, 0, 0))
    acc = np.zeros(S.shape[2:])
    for d in range(3):
        acc = acc + np.sum((Cu[d] - x0) * Su[d], axis=0) - np.sum((C[d] - x0) * S[d], axis=0)
    return acc / 3.0


def copy_metric_ghosts(S, V, dims, conns, g):
    """Replace metrics of ghost cells across connections by the neighbour's."""
    for d in range(3):
        for c in conns:
            if c.face // 2 != d:
                continue
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
                ixd = index_grid(rd, g)
                ixs = index_grid(rs, g)
                S[b][(slice(None), slice(None)) + ixd] = S[nb][(slice(None), slice(None)) + ixs]
                V[b][ixd] = V[nb][ixs]


def build_metrics(case, g=2):
    """Ghost nodes + metrics for every block of a case.

    Returns (Xs, Ss, Vs): padded nodes, lower-face vectors [3,3,...] and
    volumes, one entry per block.
    """
    Xs = [pad_nodes(x, g) for x in case.nodes]
    fill_ghost_nodes(Xs, case.dims, case.conns, case.bcs, g)
    Ss = [face_vectors(X) for X in Xs]
    Vs = [volumes(X) for X in Xs]
    copy_metric_ghosts(Ss, Vs, case.dims, case.conns, g)
    return Xs, Ss, Vs
