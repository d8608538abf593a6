"""Residual, time step, SSP Runge-Kutta and norms (oracle; plain FP64 NumPy).

* Residual, Eq. (3): dQ/dt = -R(Q) with
  R_c = ((F_i+ - F_i-) + (F_j+ - F_j-) + (F_k+ - F_k-)) / V_c,
  F = (F_inv - F_vis) . S on each lower/upper face (cell-centred finite volume
  on the curvilinear metrics of the geometry module).
* Time step (the paper's lambda is not defined): per interior cell
  dt_c = CFL V / (sum_d L_d + 4 sum_d Lv_d) with S_d averaged over the cell's
  two d-faces, L_d = |u . S_d| + c |S_d| and, for viscous flow,
  Lv_d = max(4/3, gamma/Pr) (mu/rho) |S_d|^2 / V; the global step is the
  minimum over all interior cells of all blocks (or per cell when local time
  stepping is asked for).
* Time stage, Eqs. (4)-(6), with lambda = -dt so that they integrate
  dQ/dt = -R:
      Q1 = Qn - dt R(Qn)
      Q2 = 3/4 Qn + 1/4 (Q1 - dt R(Q1))
      Qn+1 = 1/3 Qn + 2/3 (Q2 - dt R(Q2)),
  with a ghost fill before every residual.
* Norms (convergence test, Section 2.3): L2(R_c) = sqrt(sum R_c^2 / N) over
  interior cells of all blocks, totals sum V Q_c, max |R_rho|, all summed
  with math.fsum.
"""
from __future__ import annotations

import math
from dataclasses import dataclass
from typing import List

import numpy as np

from . import flux as fx
from .geometry import build_metrics
from .ghosts import fill_ghosts


def window(A, dims, d, off, g):
    """View of a padded cell array [..., k, j, i] at cells R + off for every face
    of direction d (R runs over d-index 0..n_d, transverse over the interior)."""
    sl = []
    for dd in (2, 1, 0):
        n = dims[dd]
        o = off[dd]
        stop = g + o + n + (1 if dd == d else 0)
        sl.append(slice(g + o, stop))
    return A[(Ellipsis,) + tuple(sl)]


def interior(A, dims, g):
    ni, nj, nk = dims
    return A[..., g:g + nk, g:g + nj, g:g + ni]


def unit(d, s=1):
    e = [0, 0, 0]
    e[d] = s
    return e


def add(*vs):
    return [sum(t) for t in zip(*vs)]


def face_fluxes(Q, S, V, dims, params, g):
    """F = (F_inv - F_vis) . S on every face of every direction: list of [5, ...]."""
    gam = params.gamma
    W = fx.primitives(Q, gam)
    out = []
    for d in range(3):
        ed = unit(d)
        W_m2 = window(W, dims, d, unit(d, -2), g)
        W_m1 = window(W, dims, d, unit(d, -1), g)
        W_0 = window(W, dims, d, (0, 0, 0), g)
        W_p1 = window(W, dims, d, ed, g)
        WL, WR = fx.muscl(W_m2, W_m1, W_0, W_p1, params.limiter_eps)
        Sd = window(S[d], dims, d, (0, 0, 0), g)
        F = fx.roe_flux(WL, WR, Sd, gam, params.entropy_fix)
        if params.viscous:
            F = F - _viscous(W, S, V, dims, d, params, g)
        out.append(F)
    return out


def _viscous(W, S, V, dims, d, params, g):
    # phi = (u, v, w, T)
    phi = np.concatenate([W[1:4], (W[4] / W[0])[None]])
    L = unit(d, -1)
    Rr = (0, 0, 0)
    phiL = window(phi, dims, d, L, g)
    phiR = window(phi, dims, d, Rr, g)
    dts, Sts = [], []
    for t in [t for t in range(3) if t != d]:
        et = unit(t)
        emt = unit(t, -1)
        dphi = 0.25 * (window(phi, dims, d, add(L, et), g) + window(phi, dims, d, add(Rr, et), g)
                       - window(phi, dims, d, add(L, emt), g) - window(phi, dims, d, add(Rr, emt), g))
        St = 0.25 * (window(S[t], dims, d, L, g) + window(S[t], dims, d, add(L, et), g)
                     + window(S[t], dims, d, Rr, g) + window(S[t], dims, d, add(Rr, et), g))
        dts.append(dphi)
        Sts.append(St)
    Sd = window(S[d], dims, d, Rr, g)
    Vf = 0.5 * (window(V, dims, d, L, g) + window(V, dims, d, Rr, g))
    return fx.viscous_flux(phiL, phiR, dts[0], dts[1], Sd, Sts[0], Sts[1], Vf,
                           fx.mu_inf(params), params)


def residual_block(Q, S, V, dims, params, g):
    """R over the interior cells of one block, [5, nk, nj, ni]."""
    F = face_fluxes(Q, S, V, dims, params, g)
    diffs = []
    for d in range(3):
        ax = 3 - d
        n = dims[d]
        hi = np.take(F[d], np.arange(1, n + 1), axis=ax)
        lo = np.take(F[d], np.arange(0, n), axis=ax)
        diffs.append(hi - lo)
    return ((diffs[0] + diffs[1]) + diffs[2]) / interior(V, dims, g)


def local_dt_block(Q, S, V, dims, params, g):
    """Per-interior-cell admissible time step, [nk, nj, ni]."""
    gam = params.gamma
    Wc = interior(fx.primitives(Q, gam), dims, g)
    Vc = interior(V, dims, g)
    c = np.sqrt(gam * Wc[4] / Wc[0])
    lam = np.zeros_like(Vc)
    lamv = np.zeros_like(Vc)
    for d in range(3):
        Sl = interior(S[d], dims, g)
        ed = unit(d)
        ni, nj, nk = dims
        Su = S[d][:, g + ed[2]:g + ed[2] + nk, g + ed[1]:g + ed[1] + nj, g + ed[0]:g + ed[0] + ni]
        Sb = 0.5 * (Sl + Su)
        mag = np.sqrt(np.sum(Sb * Sb, axis=0))
        lam = lam + (np.abs(np.sum(Wc[1:4] * Sb, axis=0)) + c * mag)
        if params.viscous:
            T = Wc[4] / Wc[0]
            mu = fx.sutherland(T, fx.mu_inf(params), params.sutherland)
            coef = max(4.0 / 3.0, gam / params.prandtl)
            lamv = lamv + coef * (mu / Wc[0]) * mag * mag / Vc
    return params.cfl * Vc / (lam + 4.0 * lamv)


@dataclass
class OracleState:
    """Padded per-block state plus the static geometry of a case."""
    case: object
    g: int
    Xs: list
    Ss: list
    Vs: list
    Qs: list


def setup(case, g=2) -> OracleState:
    Xs, Ss, Vs = build_metrics(case, g)
    Qs = []
    for b, q in enumerate(case.q0):
        ni, nj, nk = case.dims[b]
        Q = np.full((5, nk + 2 * g, nj + 2 * g, ni + 2 * g), np.nan)
        Q[:, g:g + nk, g:g + nj, g:g + ni] = q
        Qs.append(Q)
    return OracleState(case, g, Xs, Ss, Vs, Qs)


def fill(st: OracleState, Qs=None):
    Qs = st.Qs if Qs is None else Qs
    c = st.case
    fill_ghosts(Qs, st.Ss, c.dims, c.conns, c.bcs, c.params, st.g)


def residual(st: OracleState, Qs=None, fill_first=True) -> List[np.ndarray]:
    Qs = st.Qs if Qs is None else Qs
    if fill_first:
        fill(st, Qs)
    c = st.case
    return [residual_block(Qs[b], st.Ss[b], st.Vs[b], c.dims[b], c.params, st.g)
            for b in range(c.nblk)]


def time_step(st: OracleState, Qs=None):
    """Global dt (float) or per-block local dt arrays when local_dt is set."""
    Qs = st.Qs if Qs is None else Qs
    c = st.case
    dts = [local_dt_block(Qs[b], st.Ss[b], st.Vs[b], c.dims[b], c.params, st.g)
           for b in range(c.nblk)]
    if c.params.local_dt:
        return dts
    return min(float(x.min()) for x in dts)


def ssp_rk3(q, dt, R):
    """One SSP-RK3 step of dQ/dt = -R(Q) for array-like q (Eqs. 4-6, lambda = -dt)."""
    q1 = q - dt * R(q)
    q2 = 0.75 * q + 0.25 * (q1 - dt * R(q1))
    return (1.0 / 3.0) * q + (2.0 / 3.0) * (q2 - dt * R(q2))


def norms_from(st: OracleState, Qs, Rs):
    """[L2(R_c) x5, sum V Q_c x5, max|R_rho|] with math.fsum."""
    c = st.case
    g = st.g
    N = c.ncells
    out = []
    for comp in range(5):
        if Rs is None:
            out.append(0.0)
        else:
            out.append(math.sqrt(math.fsum(float(v) for R in Rs for v in (R[comp] ** 2).ravel()) / N))
    for comp in range(5):
        out.append(math.fsum(float(v) for b in range(c.nblk)
                             for v in (interior(st.Vs[b], c.dims[b], g)
                                       * interior(Qs[b][comp], c.dims[b], g)).ravel()))
    out.append(max(float(np.abs(R[0]).max()) for R in Rs) if Rs is not None else 0.0)
    return out


def step(st: OracleState, record=False, dt=None):
    """Advance the oracle state by one RK3 step in place.

    Returns the step's history row [dt, L2(R(Qn)) x5, sum V Qn x5,
    max|R_rho(Qn)|] when ``record`` is set (all about the state at the start
    of the step), else the time step.  ``dt`` overrides the CFL step (used to
    land on a fixed final time).
    """
    c = st.case
    g = st.g
    fill(st)
    if dt is None:
        dt = time_step(st)
    st_dt = dt
    Qn = [Q.copy() for Q in st.Qs]
    ints = [(slice(None), slice(g, g + nk), slice(g, g + nj), slice(g, g + ni))
            for (ni, nj, nk) in c.dims]

    def dtb(b):
        return dt[b] if isinstance(dt, list) else dt

    R0 = residual(st, Qn, fill_first=False)
    Q1 = [Q.copy() for Q in Qn]
    for b in range(c.nblk):
        Q1[b][ints[b]] = Qn[b][ints[b]] - dtb(b) * R0[b]
    R1 = residual(st, Q1)
    Q2 = [Q.copy() for Q in Qn]
    for b in range(c.nblk):
        Q2[b][ints[b]] = 0.75 * Qn[b][ints[b]] + 0.25 * (Q1[b][ints[b]] - dtb(b) * R1[b])
    R2 = residual(st, Q2)
    for b in range(c.nblk):
        st.Qs[b][ints[b]] = ((1.0 / 3.0) * Qn[b][ints[b]]
                             + (2.0 / 3.0) * (Q2[b][ints[b]] - dtb(b) * R2[b]))
    if record:
        dtv = st_dt if not isinstance(st_dt, list) else min(float(x.min()) for x in st_dt)
        return [dtv] + norms_from(st, Qn, R0)
    return dt


def interior_state(st: OracleState, b=None):
    c = st.case
    if b is not None:
        return interior(st.Qs[b], c.dims[b], st.g).copy()
    return [interior(st.Qs[i], c.dims[i], st.g).copy() for i in range(c.nblk)]
