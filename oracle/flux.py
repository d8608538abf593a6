"""Face fluxes (oracle; plain FP64 NumPy, vectorised over faces).

Section 2.2 forms the inviscid flux at a cell edge from left- and right-hand
cell-edge states by a flux-splitting method, and discretises viscous terms
centrally; the interpolation and the splitting are left unspecified.  The
choices made here:

* primitives W = (rho, u, v, w, p), p = (gamma - 1)(rho E - rho |u|^2 / 2);
* kappa = 1/3 MUSCL in index space with the smooth limiter
  s(a, b) = (2ab + eps)/(a^2 + b^2 + eps):
      W_L = W_{c-1} + s/4 [(1 - kappa s) D- + (1 + kappa s) D+]
      W_R = W_c    - s'/4 [(1 - kappa s') D'+ + (1 + kappa s') D'-]
  with D- = W_{c-1} - W_{c-2}, D+ = W_c - W_{c-1} (and the same shifted by one
  cell for the right state); a face whose reconstructed density or pressure is
  not positive falls back to W_L = W_{c-1}, W_R = W_c;
* Roe's approximate Riemann solver (Roe 1981) with Harten's entropy fix on the
  two acoustic waves, lambda <- (lambda^2 + delta^2)/(2 delta) when
  lambda < delta, delta = eps_H (|U| + c);
* viscous flux from face gradients over the auxiliary cell straddling the
  face (finite-volume chain rule), Stokes' hypothesis, Sutherland's law and
  constant Prandtl number.

Units: rho_inf = p_inf = 1, T = p/rho, c^2 = gamma T,
mu_inf = rho_inf |u_inf| / Re (unit reference length),
mu(T) = mu_inf T^(3/2) (1 + S*) / (T + S*),  k = mu gamma / ((gamma - 1) Pr).
"""
from __future__ import annotations

import math

import numpy as np


def primitives(Q, gamma):
    rho = Q[0]
    u = Q[1] / rho
    v = Q[2] / rho
    w = Q[3] / rho
    p = (gamma - 1.0) * (Q[4] - 0.5 * rho * (u * u + v * v + w * w))
    return np.stack([rho, u, v, w, p])


def limiter(a, b, eps):
    return (2.0 * a * b + eps) / (a * a + b * b + eps)


def muscl(Wm2, Wm1, W0, Wp1, eps, kappa=1.0 / 3.0):
    """Left/right states at the face between cells c-1 and c."""
    dm = Wm1 - Wm2
    dp = W0 - Wm1
    s = limiter(dm, dp, eps)
    WL = Wm1 + 0.25 * s * ((1.0 - kappa * s) * dm + (1.0 + kappa * s) * dp)
    dm2 = W0 - Wm1
    dp2 = Wp1 - W0
    s2 = limiter(dm2, dp2, eps)
    WR = W0 - 0.25 * s2 * ((1.0 - kappa * s2) * dp2 + (1.0 + kappa * s2) * dm2)
    bad = (WL[0] <= 0.0) | (WL[4] <= 0.0) | (WR[0] <= 0.0) | (WR[4] <= 0.0)
    WL = np.where(bad[None], Wm1, WL)
    WR = np.where(bad[None], W0, WR)
    return WL, WR


def physical_flux(W, n, gamma):
    """F(W) . n for unit normal n: [rho U, rho u U + p n, rho H U]."""
    rho, u, p = W[0], W[1:4], W[4]
    U = np.sum(u * n, axis=0)
    H = gamma / (gamma - 1.0) * p / rho + 0.5 * np.sum(u * u, axis=0)
    F = np.empty_like(W)
    F[0] = rho * U
    F[1:4] = rho * u * U + p * n
    F[4] = rho * H * U
    return F


def roe_flux(WL, WR, S, gamma, eps_h, harten=True):
    """Roe flux through a face with area vector S (returns flux times |S|)."""
    area = np.sqrt(np.sum(S * S, axis=0))
    n = S / area
    rl, ul, pl = WL[0], WL[1:4], WL[4]
    rr, ur, pr = WR[0], WR[1:4], WR[4]
    Hl = gamma / (gamma - 1.0) * pl / rl + 0.5 * np.sum(ul * ul, axis=0)
    Hr = gamma / (gamma - 1.0) * pr / rr + 0.5 * np.sum(ur * ur, axis=0)
    r = np.sqrt(rr / rl)
    rhat = r * rl
    uhat = (ul + r * ur) / (1.0 + r)
    Hhat = (Hl + r * Hr) / (1.0 + r)
    q2 = np.sum(uhat * uhat, axis=0)
    c2 = (gamma - 1.0) * (Hhat - 0.5 * q2)
    chat = np.sqrt(c2)
    Uhat = np.sum(uhat * n, axis=0)
    drho = rr - rl
    du = ur - ul
    dp = pr - pl
    dU = np.sum(du * n, axis=0)
    l1 = np.abs(Uhat - chat)
    l2 = np.abs(Uhat)
    l3 = np.abs(Uhat + chat)
    if harten:
        delta = eps_h * (np.abs(Uhat) + chat)
        l1 = np.where(l1 < delta, (l1 * l1 + delta * delta) / (2.0 * delta), l1)
        l3 = np.where(l3 < delta, (l3 * l3 + delta * delta) / (2.0 * delta), l3)
    a1 = (dp - rhat * chat * dU) / (2.0 * c2)
    a5 = (dp + rhat * chat * dU) / (2.0 * c2)
    a2 = drho - dp / c2
    D = np.empty_like(WL)
    D[0] = l1 * a1 + l2 * a2 + l3 * a5
    D[1:4] = (l1 * a1 * (uhat - chat * n) + l2 * (a2 * uhat + rhat * (du - dU * n))
              + l3 * a5 * (uhat + chat * n))
    D[4] = (l1 * a1 * (Hhat - chat * Uhat)
            + l2 * (a2 * 0.5 * q2 + rhat * (np.sum(uhat * du, axis=0) - Uhat * dU))
            + l3 * a5 * (Hhat + chat * Uhat))
    FL = physical_flux(WL, n, gamma)
    FR = physical_flux(WR, n, gamma)
    return area * 0.5 * (FL + FR - D)


def sutherland(T, mu_inf, s_star):
    return mu_inf * T * np.sqrt(T) * (1.0 + s_star) / (T + s_star)


def viscous_flux(phiL, phiR, dt1, dt2, Sd, St1, St2, Vf, mu_inf, params):
    """Viscous flux F_v . S_d through a face.

    phiL, phiR: (u, v, w, T) at the two cells [4, ...]; dt1, dt2: transverse
    differences of (u, v, w, T) [4, ...]; Sd: face vector; St1, St2: averaged
    transverse face vectors of the auxiliary cell; Vf: its volume.
    """
    g = params.gamma
    grad = ((phiR - phiL)[:, None] * Sd[None] + dt1[:, None] * St1[None]
            + dt2[:, None] * St2[None]) / Vf          # [4 (u,v,w,T), 3 (x,y,z), ...]
    uf = 0.5 * (phiL[0:3] + phiR[0:3])
    Tf = 0.5 * (phiL[3] + phiR[3])
    mu = sutherland(Tf, mu_inf, params.sutherland)
    kc = mu * g / ((g - 1.0) * params.prandtl)
    div = grad[0, 0] + grad[1, 1] + grad[2, 2]
    tau = np.empty((3, 3) + Tf.shape)
    for a in range(3):
        for b in range(3):
            tau[a, b] = mu * (grad[a, b] + grad[b, a])
        tau[a, a] = tau[a, a] - (2.0 / 3.0) * mu * div
    F = np.zeros((5,) + Tf.shape)
    for a in range(3):
        F[1 + a] = tau[a, 0] * Sd[0] + tau[a, 1] * Sd[1] + tau[a, 2] * Sd[2]
    F[4] = (uf[0] * F[1] + uf[1] * F[2] + uf[2] * F[3]
            + kc * (grad[3, 0] * Sd[0] + grad[3, 1] * Sd[1] + grad[3, 2] * Sd[2]))
    return F


def mu_inf(params):
    return params.mach * math.sqrt(params.gamma) / params.reynolds
