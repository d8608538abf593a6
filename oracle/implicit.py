"""Implicit step on the finite-volume residual (oracle; plain FP64 NumPy).

The paper's flowchart solves a large sparse linear system at every step
(Section 2.3) and does not give the method.  The reading taken here is the
data-parallel one the WCNS-E-5 path uses (the implicit reading in
highorder.py), put on the finite-volume residual of solver.py (Eq. 3,
dQ/dt = -R):

* backward Euler:  (V_c / dt_c + d(V R)_c / dQ) dQ = -V_c R_c, with the CFL
  step of solver.local_dt_block per cell (local stepping) or its minimum
  (global), at the case's CFL number (large for an implicit march);
* the approximate Jacobian is the first-order flux-split one: the flux
  through a face f between cells L and R (area vector S_f pointing from L to
  R) is replaced by (F(Q_L) + F(Q_R)) . S_f / 2 - mu_f (Q_R - Q_L), with the
  dissipation coefficient mu_f = lambda_f / 2 + lv_f frozen at the step's
  start: lambda_f = |u_m . S_f| + c_m |S_f| of the mean primitive state m of
  the face's two cells, and for viscous flow lv_f = max(4/3, gamma/Pr)
  nu_m |S_f|^2 / V_m (nu = mu / rho by Sutherland's law; nu and V means of the
  two cells), the viscous radius of the time-step reading;
* point-Jacobi sweeps (every cell from the previous iterate only), from
  dQ = -V R / D with D_c = V_c / dt_c + sum of mu_f over the cell's 6 faces:
      dQ_c <- (-V_c R_c - sum_{faces f with c = L} [dF(R; S_f) / 2 - mu_f dQ_R]
                        - sum_{faces f with c = R} [-dF(L; S_f) / 2 - mu_f dQ_L]) / D_c,
  dF(m; S) = F(Q_m + dQ_m) . S - F(Q_m) . S (the physical inviscid flux);
  the cell's own term A_c . (sum of its outward face vectors) / 2 vanishes
  with the closed-cell metric identity and is left out;
* ghost cells: Q as the ordinary ghost fill leaves it; dQ is copied across
  block connections (the same sweeps as the state) and is zero in the ghost
  cells of physical boundaries (the boundary conditions act through the
  residual, explicitly);
* the step is Q + dQ on the interior cells.

Pins (tests/test_oracle_implicit.py): the explicit Euler limit
dQ = -dt R + O(dt^2); a uniform stream stays uniform; the sweeps' fixed
point; the operator read off the sweeps equals V/dt plus the Jacobian of a
first-order local Lax-Friedrichs residual with frozen dissipation (written in
the test, differentiated by central differences); a split periodic box gives
bitwise the unsplit box's steps; and a steady channel reached by implicit
steps is the steady state the RK3 march reaches.
"""
from __future__ import annotations

import numpy as np

from . import flux as fx
from .ghosts import _fill_conn
from .solver import interior, local_dt_block, norms_from, residual, unit, window


def physical_flux_dot(Q, S, gamma):
    """F(Q) . S of the inviscid flux of Eq. (1) for conserved states Q [5, ...]
    and (not necessarily unit) vectors S [3, ...]."""
    rho = Q[0]
    u, v, w = Q[1] / rho, Q[2] / rho, Q[3] / rho
    p = (gamma - 1.0) * (Q[4] - 0.5 * rho * (u * u + v * v + w * w))
    U = u * S[0] + v * S[1] + w * S[2]
    return np.stack([Q[0] * U, Q[1] * U + p * S[0], Q[2] * U + p * S[1], Q[3] * U + p * S[2],
                     (Q[4] + p) * U])


def face_mu(Q, S, V, dims, params, g):
    """mu_f = lambda_f / 2 + lv_f on the faces of every direction of one block:
    list over d of arrays with n_d + 1 faces along d (face f between cells f - 1
    and f), the interior range across."""
    gam = params.gamma
    W = fx.primitives(Q, gam)
    out = []
    for d in range(3):
        WL = window(W, dims, d, unit(d, -1), g)
        WR = window(W, dims, d, (0, 0, 0), g)
        Sf = window(S[d], dims, d, (0, 0, 0), g)
        Wm = 0.5 * (WL + WR)
        lam = (np.abs(Wm[1] * Sf[0] + Wm[2] * Sf[1] + Wm[3] * Sf[2])
               + np.sqrt(gam * Wm[4] / Wm[0]) * np.sqrt(np.sum(Sf * Sf, axis=0)))
        mu = 0.5 * lam
        if params.viscous:
            nu_l = fx.sutherland(WL[4] / WL[0], fx.mu_inf(params), params.sutherland) / WL[0]
            nu_r = fx.sutherland(WR[4] / WR[0], fx.mu_inf(params), params.sutherland) / WR[0]
            vm = 0.5 * (window(V, dims, d, unit(d, -1), g) + window(V, dims, d, (0, 0, 0), g))
            mu = mu + max(4.0 / 3.0, gam / params.prandtl) * (0.5 * (nu_l + nu_r)) * np.sum(Sf * Sf, axis=0) / vm
        out.append(mu)
    return out


def _slice_d(a, d, start, stop):
    """a[..., start:stop along index direction d] for arrays [..., k, j, i]."""
    idx = [slice(None)] * a.ndim
    idx[a.ndim - 1 - d] = slice(start, stop)
    return a[tuple(idx)]


def fill_delta_ghosts(st, dQs):
    """Ghost cells of the update: zero, then copies across the connections in
    the state's sweep order (i, j, k)."""
    c = st.case
    g = st.g
    for b in range(c.nblk):
        full = dQs[b].copy()
        dQs[b][...] = 0.0
        dQs[b][(slice(None),) + (slice(g, -g),) * 3] = full[(slice(None),) + (slice(g, -g),) * 3]
    for d in range(3):
        for cn in c.conns:
            if cn.face // 2 == d:
                _fill_conn(dQs, c.dims, cn, g)


def implicit_sweeps(st, Qs, rhs, dts, sweeps, mus=None):
    """The update dQ (interior arrays, one per block) after `sweeps`
    point-Jacobi sweeps for the right-hand side rhs = -V R (interior arrays),
    with Qs the ghost-filled padded states and dts the per-cell (arrays) or
    global (float) steps.  Returns (dQs, D)."""
    c = st.case
    g = st.g
    gam = c.params.gamma
    if mus is None:
        mus = [face_mu(Qs[b], st.Ss[b], st.Vs[b], c.dims[b], c.params, g) for b in range(c.nblk)]
    D = []
    for b in range(c.nblk):
        n = c.dims[b]
        Vc = interior(st.Vs[b], n, g)
        dtb = dts[b] if isinstance(dts, list) else dts
        Db = Vc / dtb
        for d in range(3):
            Db = Db + _slice_d(mus[b][d], d, 0, n[d]) + _slice_d(mus[b][d], d, 1, n[d] + 1)
        D.append(Db)
    dQs = []
    for b in range(c.nblk):
        pad = np.zeros_like(Qs[b])
        interior(pad, c.dims[b], g)[...] = rhs[b] / D[b]
        dQs.append(pad)
    for _ in range(sweeps):
        fill_delta_ghosts(st, dQs)
        new = []
        for b in range(c.nblk):
            n = c.dims[b]
            O = np.zeros_like(rhs[b])
            for d in range(3):
                Sf = window(st.Ss[b][d], n, d, (0, 0, 0), g)
                QL = window(Qs[b], n, d, unit(d, -1), g)
                QR = window(Qs[b], n, d, (0, 0, 0), g)
                dL = window(dQs[b], n, d, unit(d, -1), g)
                dR = window(dQs[b], n, d, (0, 0, 0), g)
                dFR = physical_flux_dot(QR + dR, Sf, gam) - physical_flux_dot(QR, Sf, gam)
                dFL = physical_flux_dot(QL + dL, Sf, gam) - physical_flux_dot(QL, Sf, gam)
                mu = mus[b][d]
                t_up = 0.5 * dFR - mu * dR          # into cell L = f - 1 (its upper face)
                t_lo = -0.5 * dFL - mu * dL         # into cell R = f (its lower face)
                O = O + _slice_d(t_up, d, 1, n[d] + 1) + _slice_d(t_lo, d, 0, n[d])
            pad = np.zeros_like(Qs[b])
            interior(pad, n, g)[...] = (rhs[b] - O) / D[b]
            new.append(pad)
        dQs = new
    return [interior(x, c.dims[b], g).copy() for b, x in enumerate(dQs)], D


def implicit_step(st, sweeps, record=False):
    """One implicit step in place on the oracle state.  Returns the history row
    [dt, L2(R(Qn)) x5, sum V Qn x5, max|R_rho(Qn)|] when record is set (dt is
    the least per-cell step under local stepping), else the step."""
    c = st.case
    g = st.g
    Rs = residual(st)                               # ghost fill of Q^n first
    dts = [local_dt_block(st.Qs[b], st.Ss[b], st.Vs[b], c.dims[b], c.params, g) for b in range(c.nblk)]
    if not c.params.local_dt:
        dts = min(float(x.min()) for x in dts)
    rhs = [-interior(st.Vs[b], c.dims[b], g) * Rs[b] for b in range(c.nblk)]
    dQs, _ = implicit_sweeps(st, st.Qs, rhs, dts, sweeps)
    Qn = [Q.copy() for Q in st.Qs]
    for b in range(c.nblk):
        interior(st.Qs[b], c.dims[b], g)[...] += dQs[b]
    if record:
        dtv = dts if not isinstance(dts, list) else min(float(x.min()) for x in dts)
        return [dtv] + norms_from(st, Qn, Rs)
    return dts
