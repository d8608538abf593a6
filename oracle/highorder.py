"""High-order pieces of the paper's WCNS-E-5 scheme (oracle; plain FP64 NumPy).

Test infrastructure, like the rest of this package.  Two operators:

1. the sixth-order staggered flux difference of Eq. (2) (below);
2. the fifth-order weighted cell-edge interpolation of WCNS-E-5 (wcns5_edge),
   which Section 2.2 names and leaves to its reference; it is written here
   from the published construction of that scheme (Deng and Zhang), so its
   nonlinear weights are "parity unpinned" with respect to the paper;
3. their composition into the inviscid residual of a periodic Cartesian block
   (wcns5_euler_residual_periodic): primitive face states by (2), Roe's flux
   through each face (the flux splitting of the finite-volume path), Eq. (2)
   along each direction, summed.  Curvilinear metrics and block closures of
   the scheme are in references the paper does not reproduce;
4. the third-order Runge-Kutta steps of Eqs. (4)-(6) on that residual
   (wcns5_euler_steps_periodic), with the oracle solver's ssp_rk3.

Section 2.2, Eq. (2): the cell-centred derivative of a face-centred flux F
along one index direction with grid size h,

    dF/dxi |_i = [ 75/64  (F_{i+1/2} - F_{i-1/2})
                 - 25/384 (F_{i+3/2} - F_{i-3/2})
                 +  3/640 (F_{i+5/2} - F_{i-5/2}) ] / h.

The face field holds n + 5 faces along the direction (faces i - 1/2 for
i = -2 .. n + 2), so every one of the n cells has its six faces.  How the
faces beyond a block are obtained (ghost cells, boundary closures) is in
references the paper does not reproduce; the operator takes them as given.

Pins: the printed weights' moment sums (exact rationals), exactness on
polynomials up to degree 6, the closed-form degree-7 error 225/64 h^6, and
sixth-order convergence on a sine.
"""
from __future__ import annotations

import numpy as np

C1, C2, C3 = 75.0 / 64.0, -25.0 / 384.0, 3.0 / 640.0


def staggered_diff6(f: np.ndarray, d: int, h: float) -> np.ndarray:
    """f: [nvar, Nk, Nj, Ni] face values with n_d + 5 entries along axis d
    (d = 0, 1, 2 for i, j, k); returns [nvar, nk, nj, ni] cell derivatives."""
    ax = 3 - d                       # array axis of direction d
    n = f.shape[ax] - 5

    def face(s):                     # faces i - 5/2 + s for the n cells
        sl = [slice(None)] * 4
        sl[ax] = slice(s, s + n)
        return f[tuple(sl)]
    c1, c2, c3 = C1 / h, C2 / h, C3 / h
    return c1 * (face(3) - face(2)) + c2 * (face(4) - face(1)) + c3 * (face(5) - face(0))


# ------------------------------------------------------------------ WCNS-E-5
# Left state at face i+1/2 from the three 3-cell stencils ending, centred and
# starting at cell i: each candidate is a second-order Taylor value
# u_i + (h/2) g_k + (h^2/8) s_k with one-sided / central first (g) and second
# (s) differences; smoothness beta_k = (h g_k)^2 + (h^2 s_k)^2; linear weights
# 1/16, 10/16, 5/16 (together the 5-cell interpolation at the face, exact to
# degree 4); nonlinear weights alpha_k = d_k / (eps + beta_k)^2, normalised.
# The right state at the same face is the mirror image built around cell i+1.
D_LIN = (1.0 / 16.0, 10.0 / 16.0, 5.0 / 16.0)


def _edge_left(um2, um1, u0, up1, up2, eps, linear):
    """Left value at the face between u0 and up1 (all arrays of one shape)."""
    hg = ((um2 - 4.0 * um1 + 3.0 * u0) / 2.0, (up1 - um1) / 2.0, (-3.0 * u0 + 4.0 * up1 - up2) / 2.0)
    hs = (um2 - 2.0 * um1 + u0, um1 - 2.0 * u0 + up1, u0 - 2.0 * up1 + up2)
    cand = [u0 + 0.5 * hg[k] + 0.125 * hs[k] for k in range(3)]
    if linear:
        w = D_LIN
    else:
        a = [D_LIN[k] / (eps + hg[k] * hg[k] + hs[k] * hs[k]) ** 2 for k in range(3)]
        tot = a[0] + a[1] + a[2]
        w = [a[k] / tot for k in range(3)]
    return w[0] * cand[0] + w[1] * cand[1] + w[2] * cand[2]


def wcns5_edge(u: np.ndarray, d: int, eps: float = 1e-6, linear: bool = False):
    """u: [nvar, ...] cell values with m + 5 entries along axis d (cells
    p - 3 .. for faces p); returns (uL, uR), each with m entries along d: the
    left and right states at face p, which lies between padded cells p + 2 and
    p + 3 (uL from cells p .. p + 4, uR from p + 1 .. p + 5)."""
    ax = 3 - d
    m = u.shape[ax] - 5

    def cell(s):
        sl = [slice(None)] * 4
        sl[ax] = slice(s, s + m)
        return u[tuple(sl)]
    c = [cell(s) for s in range(6)]
    uL = _edge_left(c[0], c[1], c[2], c[3], c[4], eps, linear)
    uR = _edge_left(c[5], c[4], c[3], c[2], c[1], eps, linear)
    return uL, uR


def wcns5_euler_residual_periodic(Q: np.ndarray, h, gamma: float, eps_h: float, eps: float = 1e-6) -> np.ndarray:
    """Q: [5, nk, nj, ni] conserved point values of a block periodic in every
    direction, uniform spacings h = (hx, hy, hz) along i, j, k.  Returns
    R = sum_d dF_d/dx_d at the cells (dQ/dt = -R)."""
    from .flux import primitives, roe_flux
    W = primitives(Q, gamma)
    R = np.zeros_like(Q)
    for d in range(3):
        ax = 1 + (2 - d)                            # array axis of direction d in [5, k, j, i]
        n = W.shape[ax]
        Wp = np.take(W, np.arange(-5, n + 5) % n, axis=ax)   # five periodic cells beyond each side
        WL, WR = wcns5_edge(Wp, d, eps)             # faces i - 1/2, i = -2 .. n + 2
        S = np.zeros((3,) + WL.shape[1:])
        S[d] = 1.0                                  # unit area along +d: flux per unit area
        F = roe_flux(WL, WR, S, gamma, eps_h)
        R = R + staggered_diff6(F, d, h[d])
    return R


def wcns5_euler_steps_periodic(Q: np.ndarray, h, gamma: float, eps_h: float, dt: float, nsteps: int,
                               eps: float = 1e-6) -> np.ndarray:
    """nsteps SSP-RK3 steps (Eqs. 4-6, lambda = -dt) of dQ/dt = -R(Q) with the
    periodic WCNS-E-5 residual and a fixed dt."""
    from .solver import ssp_rk3
    q = Q
    for _ in range(nsteps):
        q = ssp_rk3(q, dt, lambda x: wcns5_euler_residual_periodic(x, h, gamma, eps_h, eps))
    return q
