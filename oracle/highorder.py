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
   (wcns5_euler_steps_periodic), with the oracle solver's ssp_rk3;
5. the viscous terms by fourth-order central differencing, which the paper
   chooses for the viscous flux derivatives without printing the formulas
   (viscous_residual_periodic): the textbook fourth-order cell derivative,
   face value, face derivative and staggered flux difference on a periodic
   Cartesian block, with the stress tensor, Sutherland viscosity and
   conduction of the finite-volume path;
6. curvilinear periodic blocks (metrics6, wcns5_euler_residual_curv_periodic):
   face metrics in the symmetric conservative form built from Eq. (2) and a
   sixth-order mid-point interpolation, so that the discrete metric
   identities hold and a uniform stream is preserved (the geometric
   conservation law the paper requires, whose formulas are in its reference;
   the reading is stated at the section below), and RK3 steps on that
   residual (wcns5_euler_steps_curv_periodic);
7. the fourth-order viscous terms on such blocks
   (viscous_residual_curv_periodic): the chain rule with those metrics, the
   viscous flux through each face's area vector (reading stated below);
8. the CFL time step on such blocks (cfl_time_step_curv_periodic), and
   blocks joined face to face (wcns5_euler_residual_blocks, block_vertices):
   the stencils run across seams with a five-cell exchange, and the viscous
   terms across the same seams (viscous_residual_blocks);
9. RK3 Navier-Stokes steps on periodic curvilinear blocks
   (ns_steps_curv_periodic) and on blocks joined face to face
   (ns_steps_blocks);
10. an implicit step (implicit_steps_curv_periodic, and implicit_steps_blocks
   for blocks joined face to face): backward Euler with a
   flux-split approximate Jacobian relaxed by point-Jacobi sweeps, the
   reading of the sparse linear solve the paper's flowchart names (stated
   below), with the viscous terms and a central diffusion split optional.  Pinned by the explicit Euler limit, a kept uniform stream, the
   sweeps' fixed point, stability past the explicit limit, and its linear
   operator against central differences of an independently written
   first-order local Lax-Friedrichs residual with frozen dissipation
   (inviscid and viscous) to O(|dQ|^2); how well that approximate
   Jacobian solves the exact linear system is not a claim ("parity
   unpinned" for that accuracy, not for the operator).

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


# ----------------------------------------- fourth-order central viscous terms
# On a uniform periodic grid (f[i + s] by np.roll), all exact for cubics:
#   cell derivative   (f_{i-2} - 8 f_{i-1} + 8 f_{i+1} - f_{i+2}) / (12 h)
#   face value        (-f_{i-1} + 9 f_i + 9 f_{i+1} - f_{i+2}) / 16             at i + 1/2
#   face derivative   (f_{i-1} - 27 f_i + 27 f_{i+1} - f_{i+2}) / (24 h)        at i + 1/2
#   flux difference   (F_{i-3/2} - 27 F_{i-1/2} + 27 F_{i+1/2} - F_{i+3/2}) / (24 h)   at i
# (a face array holds face i + 1/2 at index i).

def _at(f, ax, s):
    """f[i + s] along axis ax, periodic."""
    return np.roll(f, -s, axis=ax)


def c4_cell_deriv(f, ax, h):
    return (_at(f, ax, -2) - 8.0 * _at(f, ax, -1) + 8.0 * _at(f, ax, 1) - _at(f, ax, 2)) / (12.0 * h)


def c4_face_value(f, ax):
    return (-_at(f, ax, -1) + 9.0 * f + 9.0 * _at(f, ax, 1) - _at(f, ax, 2)) / 16.0


def c4_face_deriv(f, ax, h):
    return (_at(f, ax, -1) - 27.0 * f + 27.0 * _at(f, ax, 1) - _at(f, ax, 2)) / (24.0 * h)


def c4_flux_diff(F, ax, h):
    return (_at(F, ax, -2) - 27.0 * _at(F, ax, -1) + 27.0 * F - _at(F, ax, 1)) / (24.0 * h)


def viscous_residual_periodic(Q: np.ndarray, h, gamma: float, prandtl: float, mu_inf: float,
                              s_star: float) -> np.ndarray:
    """-div F_v on a periodic Cartesian block (Q: [5, nk, nj, ni]); add it to
    the inviscid residual for the Navier-Stokes residual (dQ/dt = -R)."""
    from .flux import primitives, sutherland
    W = primitives(Q, gamma)
    phi = [W[1], W[2], W[3], W[4] / W[0]]                     # u, v, w, T
    axis = [3, 2, 1]                                          # array axis of x, y, z in [k, j, i]
    G = [[c4_cell_deriv(phi[a], axis[t] - 1, h[t]) for t in range(3)] for a in range(4)]
    Rv = np.zeros_like(Q)
    for d in range(3):
        ax = axis[d] - 1                                      # axis within a [k, j, i] field
        pf = [c4_face_value(phi[a], ax) for a in range(4)]
        grad = [[c4_face_deriv(phi[a], ax, h[d]) if t == d else c4_face_value(G[a][t], ax) for t in range(3)]
                for a in range(4)]
        mu = sutherland(pf[3], mu_inf, s_star)
        kc = mu * gamma / ((gamma - 1.0) * prandtl)
        div = grad[0][0] + grad[1][1] + grad[2][2]
        tau = [mu * (grad[d][b] + grad[b][d]) for b in range(3)]
        tau[d] = tau[d] - (2.0 / 3.0) * mu * div
        Fv = [tau[0], tau[1], tau[2], pf[0] * tau[0] + pf[1] * tau[1] + pf[2] * tau[2] + kc * grad[3][d]]
        for c in range(4):
            Rv[1 + c] = Rv[1 + c] - c4_flux_diff(Fv[c], ax, h[d])
    return Rv


# ------------------------------------------------------- curvilinear blocks
# Section 2.2 requires, for curvilinear multi-block grids, the geometric
# conservation law of the scheme's reference, without printing its metrics.
# The reading taken here.  Vertex v along a direction sits at index position
# v + 1/2 (the upper corner of cell v); cell centres and solution points sit
# at integer positions.  Every derivative is Eq. (2) with h = 1 (index units)
# and every mid-point value the sixth-order interpolation
#     I f = [150 (f_{+1/2} + f_{-1/2}) - 25 (f_{+3/2} + f_{-3/2})
#            + 3 (f_{+5/2} + f_{-5/2})] / 256,
# both taken from vertex positions to the centre position along one axis.
# The face metrics (grad xi_d / J at the faces of direction d, one area vector
# per face) take the symmetric conservative form
#     S_d = 1/2 [ D_b (D_a X x I_a X) - D_a (D_b X x I_b X) ],
# (a, b) = (d + 1, d + 2) mod 3, which is X_a x X_b of the continuous map.
# Because D and I along different axes commute, sum_d D_d S_d = 0 holds at
# every cell to rounding, so a uniform stream stays uniform on any grid.  The
# cell Jacobian J^{-1} is det[X_xi, X_eta, X_zeta] at the centre, each column
# D along its axis of the coordinates interpolated (I) along the other two; it
# plays no part in freestream preservation.  The residual is
#     R = J sum_d D_d( Roe(W_L, W_R; S_d) ),
# Roe's flux through the face's area vector (flux times |S_d|) from the
# WCNS-E-5 edge states, dQ/dt = -R.  On a uniform Cartesian grid S_d and
# J^{-1} reduce to the face areas and the cell volume, and R to the
# Cartesian residual above.

I1, I2, I3 = 150.0 / 256.0, -25.0 / 256.0, 3.0 / 256.0


def _win(f, ax, s, m):
    sl = [slice(None)] * f.ndim
    sl[ax] = slice(s, s + m)
    return f[tuple(sl)]


def d6(f, ax):
    """Eq. (2) with h = 1 along array axis ax: m + 5 vertex values -> m centres."""
    m = f.shape[ax] - 5
    w = [_win(f, ax, s, m) for s in range(6)]
    return C1 * (w[3] - w[2]) + C2 * (w[4] - w[1]) + C3 * (w[5] - w[0])


def i6(f, ax):
    """Sixth-order mid-point interpolation along axis ax: m + 5 vertex values -> m centres."""
    m = f.shape[ax] - 5
    w = [_win(f, ax, s, m) for s in range(6)]
    return I1 * (w[3] + w[2]) + I2 * (w[4] + w[1]) + I3 * (w[5] + w[0])


def _ax(d):
    return 3 - d                       # array axis of direction d in [3, k, j, i]


def metrics6(Xe: np.ndarray):
    """Xe: [3, nk + 5, nj + 5, ni + 5] vertex coordinates, vertices -3 .. n + 1
    along each direction.  Returns (S, Jinv): S [3 (direction d), 3 (x, y, z),
    nk, nj, ni], the area vector of face v + 1/2 of direction d at index v
    along d; Jinv [nk, nj, ni] at the cell centres."""
    n = [Xe.shape[3] - 5, Xe.shape[2] - 5, Xe.shape[1] - 5]
    A = [np.cross(d6(Xe, _ax(a)), i6(Xe, _ax(a)), axis=0) for a in range(3)]
    S = []
    for d in range(3):
        a, b = (d + 1) % 3, (d + 2) % 3
        s = 0.5 * (d6(A[a], _ax(b)) - d6(A[b], _ax(a)))
        S.append(_win(s, _ax(d), 3, n[d]))                # vertices 0 .. n - 1 along d
    cols = []
    for d in range(3):
        a, b = (d + 1) % 3, (d + 2) % 3
        cols.append(d6(i6(i6(Xe, _ax(a)), _ax(b)), _ax(d)))
    Jinv = np.sum(cols[0] * np.cross(cols[1], cols[2], axis=0), axis=0)
    return np.stack(S), Jinv


def periodic_vertices(Xv: np.ndarray, P: np.ndarray) -> np.ndarray:
    """Xv: [3, nk, nj, ni] vertex coordinates of a block periodic along every
    direction (vertex (i, j, k) is the upper corner of cell (i, j, k)); P[d]:
    the displacement of the grid over one period along direction d.  Returns
    the vertices -3 .. n + 1 along each direction (metrics6's input)."""
    nk, nj, ni = Xv.shape[1:]
    idx = [np.arange(-3, m + 2) for m in (ni, nj, nk)]
    wi, wj, wk = (idx[0] % ni, idx[1] % nj, idx[2] % nk)
    qi, qj, qk = (idx[0] // ni, idx[1] // nj, idx[2] // nk)
    X = Xv[:, wk][:, :, wj][:, :, :, wi]
    P = np.asarray(P, dtype=np.float64)
    return (X + qi[None, None, None, :] * P[0][:, None, None, None]
            + qj[None, None, :, None] * P[1][:, None, None, None]
            + qk[None, :, None, None] * P[2][:, None, None, None])


def wcns5_euler_residual_curv_periodic(Q: np.ndarray, S: np.ndarray, Jinv: np.ndarray, gamma: float,
                                       eps_h: float, eps: float = 1e-6) -> np.ndarray:
    """Q: [5, nk, nj, ni] conserved point values of a periodic curvilinear
    block; S, Jinv from metrics6.  Returns R (dQ/dt = -R)."""
    from .flux import primitives, roe_flux
    W = primitives(Q, gamma)
    R = np.zeros_like(Q)
    for d in range(3):
        ax = _ax(d)
        n = W.shape[ax]
        Wp = np.take(W, np.arange(-5, n + 5) % n, axis=ax)
        WL, WR = wcns5_edge(Wp, d, eps)                      # faces of vertices -3 .. n + 1
        Sd = np.take(S[d], np.arange(-3, n + 2) % n, axis=ax)
        F = roe_flux(WL, WR, Sd, gamma, eps_h)
        R = R + staggered_diff6(F, d, 1.0)
    return R / Jinv


def wcns5_euler_steps_curv_periodic(Q: np.ndarray, S: np.ndarray, Jinv: np.ndarray, gamma: float, eps_h: float,
                                    dt: float, nsteps: int, eps: float = 1e-6) -> np.ndarray:
    """nsteps SSP-RK3 steps (Eqs. 4-6, lambda = -dt) of dQ/dt = -R(Q) with the
    curvilinear periodic residual and a fixed dt."""
    from .solver import ssp_rk3
    q = Q
    for _ in range(nsteps):
        q = ssp_rk3(q, dt, lambda x: wcns5_euler_residual_curv_periodic(x, S, Jinv, gamma, eps_h, eps))
    return q


# ------------------------------- fourth-order viscous terms, curvilinear
# The viscous terms of the fourth-order central scheme above on a periodic
# curvilinear block with the metrics of metrics6 (reading of the paper's
# choice of fourth-order central differencing on curvilinear grids):
#   - index derivatives of u, v, w, T at the cells (cell derivative, h = 1);
#   - metrics at the cells: each S_t interpolated from its faces along t
#     (the four-point mid-point formula, from faces to the centre);
#   - at a face of direction d: the face value of u, v, w, T; the index
#     derivative along d by the compact face derivative, along t != d the
#     face value of the cell derivative; S_t (t != d) the face value of the
#     cell metrics; J^{-1} the face value of the cell J^{-1}; the physical
#     gradient J sum_t S_t d/dxi_t (the chain rule with grad xi_t = J S_t);
#   - the stress tensor, Sutherland viscosity and conduction as in the
#     Cartesian terms, the viscous flux through the face's area vector S_d;
#   - -J times the staggered flux difference, summed over directions.
# On a uniform Cartesian grid this is the Cartesian viscous residual.

def c4_face_to_cell(f, ax):
    """Value at cell i from faces i -/+ 1/2, i -/+ 3/2 (face i + 1/2 at index i)."""
    return (-_at(f, ax, -2) + 9.0 * _at(f, ax, -1) + 9.0 * f - _at(f, ax, 1)) / 16.0


def viscous_residual_curv_periodic(Q: np.ndarray, S: np.ndarray, Jinv: np.ndarray, gamma: float, prandtl: float,
                                   mu_inf: float, s_star: float) -> np.ndarray:
    """-div F_v on a periodic curvilinear block (Q: [5, nk, nj, ni]; S, Jinv
    from metrics6); add it to the inviscid residual (dQ/dt = -R)."""
    from .flux import primitives, sutherland
    W = primitives(Q, gamma)
    phi = [W[1], W[2], W[3], W[4] / W[0]]                     # u, v, w, T
    axis = [2, 1, 0]                                          # axis of direction d within a [k, j, i] field
    G = [[c4_cell_deriv(phi[a], axis[t], 1.0) for t in range(3)] for a in range(4)]
    Sc = [c4_face_to_cell(S[t], 1 + axis[t]) for t in range(3)]          # [3, k, j, i] each
    Rv = np.zeros_like(Q)
    for d in range(3):
        ax = axis[d]
        pf = [c4_face_value(phi[a], ax) for a in range(4)]
        dxi = [[c4_face_deriv(phi[a], ax, 1.0) if t == d else c4_face_value(G[a][t], ax) for t in range(3)]
               for a in range(4)]
        Sf = [S[d] if t == d else c4_face_value(Sc[t], 1 + ax) for t in range(3)]
        Jf = 1.0 / c4_face_value(Jinv, ax)
        grad = [[Jf * (Sf[0][x] * dxi[a][0] + Sf[1][x] * dxi[a][1] + Sf[2][x] * dxi[a][2]) for x in range(3)]
                for a in range(4)]                            # grad[a][x] = d phi_a / d x
        mu = sutherland(pf[3], mu_inf, s_star)
        kc = mu * gamma / ((gamma - 1.0) * prandtl)
        div = grad[0][0] + grad[1][1] + grad[2][2]
        tau = [[mu * (grad[x][y] + grad[y][x]) for y in range(3)] for x in range(3)]
        for x in range(3):
            tau[x][x] = tau[x][x] - (2.0 / 3.0) * mu * div
        e = [pf[0] * tau[x][0] + pf[1] * tau[x][1] + pf[2] * tau[x][2] + kc * grad[3][x] for x in range(3)]
        Fv = [S[d][0] * tau[0][m] + S[d][1] * tau[1][m] + S[d][2] * tau[2][m] for m in range(3)]
        Fv.append(S[d][0] * e[0] + S[d][1] * e[1] + S[d][2] * e[2])
        for c in range(4):
            Rv[1 + c] = Rv[1 + c] - c4_flux_diff(Fv[c], ax, 1.0) / Jinv
    return Rv


# ------------------------------------------------------------ time step
# The paper leaves the step size of Eqs. (4)-(6) open; the reading of the
# finite-volume path applied to these blocks: per cell
#   dt_c = CFL J^{-1} / (sum_d L_d + 4 sum_d Lv_d),  L_d = |u . Sb_d| + c |Sb_d|,
#   Lv_d = max(4/3, gamma/Pr) (mu/rho) |Sb_d|^2 / J^{-1} (viscous flow only),
# Sb_d the mean of the cell's two d-face area vectors; the step is the least
# dt_c over the block.

def cfl_time_step_curv_periodic(Q: np.ndarray, S: np.ndarray, Jinv: np.ndarray, gamma: float, cfl: float,
                                viscous: bool = False, prandtl: float = 0.72, mu_inf: float = 0.0,
                                s_star: float = 110.4 / 288.15) -> float:
    from .flux import primitives, sutherland
    W = primitives(Q, gamma)
    c = np.sqrt(gamma * W[4] / W[0])
    lam = np.zeros_like(Jinv)
    lamv = np.zeros_like(Jinv)
    axis = [2, 1, 0]
    for d in range(3):
        Sb = 0.5 * (_at(S[d], 1 + axis[d], -1) + S[d])
        mag = np.sqrt(np.sum(Sb * Sb, axis=0))
        lam = lam + (np.abs(np.sum(W[1:4] * Sb, axis=0)) + c * mag)
        if viscous:
            mu = sutherland(W[4] / W[0], mu_inf, s_star)
            lamv = lamv + max(4.0 / 3.0, gamma / prandtl) * (mu / W[0]) * mag * mag / Jinv
    return float(np.min(cfl * Jinv / (lam + 4.0 * lamv)))


# ------------------------------------------------------------ block seams
# Section 2.2 asks that the points adjacent blocks share be treated with care
# on multi-block grids.  The reading taken here for blocks that meet face to
# face (a whole face against a whole face, same transverse extents, same index
# orientation): the scheme's stencils run across the seam unchanged.  Each
# direction's padded cells (five beyond each side) come from the neighbour
# across that face, as do the area vectors of the three faces below and two
# above the block; the metrics of every block come from its own vertices
# -3 .. n + 1, taken from the global grid, so the two sides of a seam compute
# the seam's metrics from the same coordinates.  A periodic block is its own
# neighbour.  Closures at physical boundaries are not covered.

def block_vertices(Xv: np.ndarray, P: np.ndarray, lo, m) -> np.ndarray:
    """Vertices -3 .. m + 1 (metrics6's input) of the sub-block at index
    origin lo with extents m of a periodic grid (Xv, P as periodic_vertices)."""
    nk, nj, ni = Xv.shape[1:]
    idx = [np.arange(lo[d] - 3, lo[d] + m[d] + 2) for d in range(3)]
    n = (ni, nj, nk)
    w = [idx[d] % n[d] for d in range(3)]
    q = [idx[d] // n[d] for d in range(3)]
    X = Xv[:, w[2]][:, :, w[1]][:, :, :, w[0]]
    P = np.asarray(P, dtype=np.float64)
    return (X + q[0][None, None, None, :] * P[0][:, None, None, None]
            + q[1][None, None, :, None] * P[1][:, None, None, None]
            + q[2][None, :, None, None] * P[2][:, None, None, None])


def wcns5_euler_residual_blocks(Qs, Ss, Jinvs, nbr, gamma: float, eps_h: float, eps: float = 1e-6):
    """Qs, Ss, Jinvs: per block as for the periodic residual; nbr[b][2d + side]
    = the block across face (d, side) of block b (side 0: the low face).
    Returns the residual of every block (dQ/dt = -R)."""
    from .flux import primitives, roe_flux
    Ws = [primitives(Q, gamma) for Q in Qs]
    out = []
    for b, (W, S, Jinv) in enumerate(zip(Ws, Ss, Jinvs)):
        R = np.zeros_like(W)
        for d in range(3):
            ax = _ax(d)
            lo, hi = nbr[b][2 * d], nbr[b][2 * d + 1]
            nlo, nhi = Ws[lo].shape[ax], Ws[hi].shape[ax]
            assert nlo >= 5 and nhi >= 5, "a neighbour must be at least 5 cells deep across the seam"
            Wp = np.concatenate([_win(Ws[lo], ax, nlo - 5, 5), W, _win(Ws[hi], ax, 0, 5)], axis=ax)
            WL, WR = wcns5_edge(Wp, d, eps)
            Sd = np.concatenate([_win(Ss[lo][d], ax, nlo - 3, 3), S[d], _win(Ss[hi][d], ax, 0, 2)], axis=ax)
            F = roe_flux(WL, WR, Sd, gamma, eps_h)
            R = R + staggered_diff6(F, d, 1.0)
        out.append(R / Jinv)
    return out


def viscous_residual_blocks(Qs, Ss, Jinvs, nbr, gamma: float, prandtl: float, mu_inf: float, s_star: float):
    """-div F_v of curvilinear blocks joined face to face (nbr as for
    wcns5_euler_residual_blocks): the terms of viscous_residual_curv_periodic
    with every four-point stencil running across the seams.  Each field is
    padded along the stencil's direction with the neighbours' values (their
    cell derivatives and cell metrics are their own), the periodic operator
    applied and the padding cropped, so a block that is its own neighbour is
    the periodic block."""
    from .flux import primitives, sutherland
    nb = len(Qs)
    axis = [2, 1, 0]                                          # axis of direction d within a [k, j, i] field

    def pad(fields, b, d, below, above, lead=0):
        """fields[b]: array whose axis lead + axis[d] runs along d."""
        ax = lead + axis[d]
        lo, hi = nbr[b][2 * d], nbr[b][2 * d + 1]
        nlo = fields[lo].shape[ax]
        return np.concatenate([_win(fields[lo], ax, nlo - below, below), fields[b],
                               _win(fields[hi], ax, 0, above)], axis=ax)

    def crop(f, d, below, n, lead=0):
        return _win(f, lead + axis[d], below, n)

    Ws = [primitives(Q, gamma) for Q in Qs]
    phis = [np.stack([W[1], W[2], W[3], W[4] / W[0]]) for W in Ws]            # [4, k, j, i]
    dims = [(Q.shape[3], Q.shape[2], Q.shape[1]) for Q in Qs]
    Gs = []
    for b in range(nb):                                                         # G[a][t] at the cells
        G = [[None] * 3 for _ in range(4)]
        for t in range(3):
            p = pad(phis, b, t, 2, 2, lead=1)
            for a in range(4):
                G[a][t] = crop(c4_cell_deriv(p[a], axis[t], 1.0), t, 2, dims[b][t])
        Gs.append(np.stack([np.stack(G[a]) for a in range(4)]))                 # [4, 3, k, j, i]
    Scs = []
    for b in range(nb):                                                         # metrics at the cells
        Scs.append(np.stack([crop(c4_face_to_cell(pad([S[t] for S in Ss], b, t, 2, 1, lead=1), 1 + axis[t]),
                                  t, 2, dims[b][t], lead=1) for t in range(3)]))
    Rvs = [np.zeros_like(Q) for Q in Qs]
    for d in range(3):
        ax = axis[d]
        Fvs = []
        for b in range(nb):
            n = dims[b][d]
            ph = pad(phis, b, d, 1, 2, lead=1)
            G = pad(Gs, b, d, 1, 2, lead=2)
            Sc = pad(Scs, b, d, 1, 2, lead=2)
            Jp = pad(Jinvs, b, d, 1, 2)
            fv = lambda f, lead=0: crop(c4_face_value(f, lead + ax), d, 1, n, lead)         # noqa: E731
            pf = [fv(ph[a]) for a in range(4)]
            dxi = [[crop(c4_face_deriv(ph[a], ax, 1.0), d, 1, n) if t == d else fv(G[a][t]) for t in range(3)]
                   for a in range(4)]
            Sf = [Ss[b][d] if t == d else fv(Sc[t], 1) for t in range(3)]
            Jf = 1.0 / fv(Jp)
            grad = [[Jf * (Sf[0][x] * dxi[a][0] + Sf[1][x] * dxi[a][1] + Sf[2][x] * dxi[a][2]) for x in range(3)]
                    for a in range(4)]
            mu = sutherland(pf[3], mu_inf, s_star)
            kc = mu * gamma / ((gamma - 1.0) * prandtl)
            div = grad[0][0] + grad[1][1] + grad[2][2]
            tau = [[mu * (grad[x][y] + grad[y][x]) for y in range(3)] for x in range(3)]
            for x in range(3):
                tau[x][x] = tau[x][x] - (2.0 / 3.0) * mu * div
            e = [pf[0] * tau[x][0] + pf[1] * tau[x][1] + pf[2] * tau[x][2] + kc * grad[3][x] for x in range(3)]
            S = Ss[b][d]
            F = [S[0] * tau[0][m] + S[1] * tau[1][m] + S[2] * tau[2][m] for m in range(3)]
            F.append(S[0] * e[0] + S[1] * e[1] + S[2] * e[2])
            Fvs.append(np.stack(F))
        for b in range(nb):
            Fp = pad(Fvs, b, d, 2, 1, lead=1)
            for c in range(4):
                Rvs[b][1 + c] = Rvs[b][1 + c] - crop(c4_flux_diff(Fp[c], ax, 1.0), d, 2, dims[b][d]) / Jinvs[b]
    return Rvs


def ns_steps_curv_periodic(Q: np.ndarray, S: np.ndarray, Jinv: np.ndarray, gamma: float, eps_h: float,
                           prandtl: float, mu_inf: float, s_star: float, dt: float, nsteps: int,
                           eps: float = 1e-6) -> np.ndarray:
    """nsteps SSP-RK3 steps (Eqs. 4-6, lambda = -dt) of the Navier-Stokes
    equations on a periodic curvilinear block: R = the inviscid WCNS-E-5
    residual plus the fourth-order viscous terms, a fixed dt."""
    from .solver import ssp_rk3

    def R(x):
        return (wcns5_euler_residual_curv_periodic(x, S, Jinv, gamma, eps_h, eps)
                + viscous_residual_curv_periodic(x, S, Jinv, gamma, prandtl, mu_inf, s_star))
    q = Q
    for _ in range(nsteps):
        q = ssp_rk3(q, dt, R)
    return q


# ------------------------------------------------------------ implicit step
# The paper's flowchart solves a large sparse linear system each step and
# notes that its convergence degrades when the domain is decomposed; it does
# not give the method.  The reading taken here, chosen to be data parallel:
# backward Euler (I/dt + dR/dQ) dQ = -R with the first-order flux-split
# approximation of dR/dQ, A+- = (A +- lambda I)/2 at every face, lambda the
# spectral radius |u . S| + c |S| of the mean of the two cells' primitive
# states, and point-Jacobi sweeps (data-parallel lower-upper relaxation).
# With J = 1 / J^{-1} and, along each direction, the faces f+ = i + 1/2 and
# f- = i - 1/2 of cell i:
#   D_i  = 1/dt + J_i sum_d (lambda_f+ + lambda_f-) / 2
#   O_i  = sum_d [ (dF(i+1; S_f+) - lambda_f+ dQ_{i+1}) - (dF(i-1; S_f-) + lambda_f- dQ_{i-1}) ] / 2
#   dQ_i <- (-R_i - J_i O_i) / D_i,   dF(m; S) = F(Q_m + dQ_m) . S - F(Q_m) . S,
# starting from dQ = -R / D; the step is Q + dQ.  (The difference of A_f+ and
# A_f- on the diagonal vanishes with the metric identities and is dropped.)

def euler_flux_through(Q: np.ndarray, S: np.ndarray, gamma: float) -> np.ndarray:
    """The physical inviscid flux of states Q ([5, ...]) through area vectors S ([3, ...])."""
    from .flux import primitives
    W = primitives(Q, gamma)
    U = W[1] * S[0] + W[2] * S[1] + W[3] * S[2]
    return np.stack([Q[0] * U, Q[1] * U + W[4] * S[0], Q[2] * U + W[4] * S[1], Q[3] * U + W[4] * S[2],
                     (Q[4] + W[4]) * U])


def _lambda_of(W, Wn, Sf, gamma):
    """Spectral radius through Sf of the mean of primitive states W and Wn."""
    Wm = 0.5 * (W + Wn)
    c = np.sqrt(gamma * Wm[4] / Wm[0])
    return np.abs(Wm[1] * Sf[0] + Wm[2] * Sf[1] + Wm[3] * Sf[2]) + c * np.sqrt(np.sum(Sf * Sf, axis=0))


def _face_lambda(W, Sf, d, gamma):
    """Spectral radius at faces i + 1/2 along d from the mean primitive state of cells i, i + 1."""
    return _lambda_of(W, np.roll(W, -1, axis=1 + [2, 1, 0][d]), Sf, gamma)


# For viscous flow the residual adds the fourth-order viscous terms and the
# operator a central diffusion split: with the viscous spectral radius
#   lv_f = max(4/3, gamma/Pr) (mu/rho)_f |S_f|^2 / J^{-1}_f
# at each face (mu/rho and J^{-1} the means of the face's two cells),
# D_i gains J_i sum_d (lv_f+ + lv_f-) and O_i gains -(lv_f+ dQ_{i+1} + lv_f- dQ_{i-1}).

def _face_lambda_visc(W, Sf, Jinv, d, gamma, prandtl, mu_inf, s_star):
    from .flux import sutherland
    ax = [2, 1, 0][d]
    nu = sutherland(W[4] / W[0], mu_inf, s_star) / W[0]
    num = 0.5 * (nu + np.roll(nu, -1, axis=ax))
    jm = 0.5 * (Jinv + np.roll(Jinv, -1, axis=ax))
    return max(4.0 / 3.0, gamma / prandtl) * num * np.sum(Sf * Sf, axis=0) / jm


def implicit_sweeps_curv_periodic(Q, R, S, Jinv, gamma: float, dt: float, sweeps: int, viscous: bool = False,
                                  prandtl: float = 0.72, mu_inf: float = 0.0, s_star: float = 110.4 / 288.15):
    """dQ of the reading above (R: the residual at Q), after `sweeps` Jacobi sweeps."""
    from .flux import primitives
    W = primitives(Q, gamma)
    Jc = 1.0 / Jinv
    lam = [_face_lambda(W, S[d], d, gamma) for d in range(3)]       # faces i + 1/2
    lv = [(_face_lambda_visc(W, S[d], Jinv, d, gamma, prandtl, mu_inf, s_star) if viscous else 0.0 * Jinv)
          for d in range(3)]
    axis = [3, 2, 1]                                                # axis of d in [5, k, j, i]
    D = 1.0 / dt + Jc * sum(0.5 * (lam[d] + np.roll(lam[d], 1, axis=axis[d] - 1))
                            + (lv[d] + np.roll(lv[d], 1, axis=axis[d] - 1)) for d in range(3))
    dQ = -R / D
    for _ in range(sweeps):
        O = np.zeros_like(Q)
        for d in range(3):
            ax = axis[d]
            Sp, Sm = S[d], np.roll(S[d], 1, axis=ax)               # faces i + 1/2, i - 1/2
            lp, lm = lam[d], np.roll(lam[d], 1, axis=ax - 1)
            vp, vm = lv[d], np.roll(lv[d], 1, axis=ax - 1)
            Qp, dQp = np.roll(Q, -1, axis=ax), np.roll(dQ, -1, axis=ax)
            Qm, dQm = np.roll(Q, 1, axis=ax), np.roll(dQ, 1, axis=ax)
            dFp = euler_flux_through(Qp + dQp, Sp, gamma) - euler_flux_through(Qp, Sp, gamma)
            dFm = euler_flux_through(Qm + dQm, Sm, gamma) - euler_flux_through(Qm, Sm, gamma)
            O = O + 0.5 * ((dFp - lp * dQp) - (dFm + lm * dQm)) - (vp * dQp + vm * dQm)
        dQ = (-R - Jc * O) / D
    return dQ


def implicit_steps_curv_periodic(Q, S, Jinv, gamma: float, eps_h: float, dt: float, nsteps: int, sweeps: int,
                                 eps: float = 1e-6, viscous: bool = False, prandtl: float = 0.72,
                                 mu_inf: float = 0.0, s_star: float = 110.4 / 288.15):
    """nsteps implicit steps (the reading above) of the curvilinear periodic
    WCNS-E-5 residual, with the fourth-order viscous terms when viscous."""
    q = Q
    for _ in range(nsteps):
        R = wcns5_euler_residual_curv_periodic(q, S, Jinv, gamma, eps_h, eps)
        if viscous:
            R = R + viscous_residual_curv_periodic(q, S, Jinv, gamma, prandtl, mu_inf, s_star)
        q = q + implicit_sweeps_curv_periodic(q, R, S, Jinv, gamma, dt, sweeps, viscous, prandtl, mu_inf, s_star)
    return q


def implicit_steps_blocks(Qs, Ss, Jinvs, nbr, gamma: float, eps_h: float, dt: float, nsteps: int, sweeps: int,
                          eps: float = 1e-6, viscous: bool = False, prandtl: float = 0.72, mu_inf: float = 0.0,
                          s_star: float = 110.4 / 288.15):
    """Implicit steps (the reading above, viscous optional) on blocks joined face to face
    (nbr as for wcns5_euler_residual_blocks).  A cell's neighbours across a
    seam are the neighbour block's cells and every sweep reads only the
    previous iterate, so point-Jacobi is the same iteration however the domain
    is cut: a split block gives bitwise the unsplit block's steps."""
    from .flux import primitives
    nb = len(Qs)

    def shift(fields, b, d, s, lead):
        """fields[b] seen from cell i + s (s = +1 or -1) along d, across the seams."""
        ax = lead + [2, 1, 0][d]
        f = fields[b]
        n = f.shape[ax]
        if s == 1:
            hi = fields[nbr[b][2 * d + 1]]
            return np.concatenate([_win(f, ax, 1, n - 1), _win(hi, ax, 0, 1)], axis=ax)
        lo = fields[nbr[b][2 * d]]
        return np.concatenate([_win(lo, ax, lo.shape[ax] - 1, 1), _win(f, ax, 0, n - 1)], axis=ax)

    from .flux import sutherland
    coef = max(4.0 / 3.0, gamma / prandtl)
    qs = list(Qs)
    for _ in range(nsteps):
        Rs = wcns5_euler_residual_blocks(qs, Ss, Jinvs, nbr, gamma, eps_h, eps)
        if viscous:
            Rv = viscous_residual_blocks(qs, Ss, Jinvs, nbr, gamma, prandtl, mu_inf, s_star)
            Rs = [a + v for a, v in zip(Rs, Rv)]
        Ws = [primitives(q, gamma) for q in qs]
        lams = [[_lambda_of(Ws[b], shift(Ws, b, d, 1, 1), Ss[b][d], gamma) for d in range(3)] for b in range(nb)]
        nus = [sutherland(W[4] / W[0], mu_inf, s_star) / W[0] for W in Ws]
        lvs = [[(coef * (0.5 * (nus[b] + shift(nus, b, d, 1, 0))) * np.sum(Ss[b][d] * Ss[b][d], axis=0)
                 / (0.5 * (Jinvs[b] + shift(Jinvs, b, d, 1, 0))) if viscous else 0.0 * Jinvs[b]) for d in range(3)]
               for b in range(nb)]
        Ds, dQs = [], []
        for b in range(nb):
            Jc = 1.0 / Jinvs[b]
            L = [[lams[c][d] for c in range(nb)] for d in range(3)]
            V = [[lvs[c][d] for c in range(nb)] for d in range(3)]
            D = 1.0 / dt + Jc * sum(0.5 * (lams[b][d] + shift(L[d], b, d, -1, 0))
                                    + (lvs[b][d] + shift(V[d], b, d, -1, 0)) for d in range(3))
            Ds.append(D)
            dQs.append(-Rs[b] / D)
        for _ in range(sweeps):
            new = []
            for b in range(nb):
                Jc = 1.0 / Jinvs[b]
                O = np.zeros_like(qs[b])
                for d in range(3):
                    Sd = [S[d] for S in Ss]
                    Ld = [lams[c][d] for c in range(nb)]
                    Sp, Sm = Ss[b][d], shift(Sd, b, d, -1, 1)
                    lp, lm = lams[b][d], shift(Ld, b, d, -1, 0)
                    Qp, dQp = shift(qs, b, d, 1, 1), shift(dQs, b, d, 1, 1)
                    Qm, dQm = shift(qs, b, d, -1, 1), shift(dQs, b, d, -1, 1)
                    dFp = euler_flux_through(Qp + dQp, Sp, gamma) - euler_flux_through(Qp, Sp, gamma)
                    dFm = euler_flux_through(Qm + dQm, Sm, gamma) - euler_flux_through(Qm, Sm, gamma)
                    vp, vm = lvs[b][d], shift([lvs[c][d] for c in range(nb)], b, d, -1, 0)
                    O = O + 0.5 * ((dFp - lp * dQp) - (dFm + lm * dQm)) - (vp * dQp + vm * dQm)
                new.append((-Rs[b] - Jc * O) / Ds[b])
            dQs = new
        qs = [q + dq for q, dq in zip(qs, dQs)]
    return qs


def ns_steps_blocks(Qs, Ss, Jinvs, nbr, gamma: float, eps_h: float, prandtl: float, mu_inf: float, s_star: float,
                    dt: float, nsteps: int, eps: float = 1e-6):
    """nsteps SSP-RK3 steps (Eqs. 4-6, lambda = -dt) of the Navier-Stokes
    equations on blocks joined face to face: every stage's residual is
    wcns5_euler_residual_blocks plus viscous_residual_blocks over all blocks
    at that stage (the oracle solver's ssp_rk3, stage by stage)."""
    def R(xs):
        inv = wcns5_euler_residual_blocks(xs, Ss, Jinvs, nbr, gamma, eps_h, eps)
        vis = viscous_residual_blocks(xs, Ss, Jinvs, nbr, gamma, prandtl, mu_inf, s_star)
        return [a + b for a, b in zip(inv, vis)]
    qs = list(Qs)
    for _ in range(nsteps):
        r0 = R(qs)
        q1 = [q - dt * r for q, r in zip(qs, r0)]
        r1 = R(q1)
        q2 = [0.75 * q + 0.25 * (a - dt * r) for q, a, r in zip(qs, q1, r1)]
        r2 = R(q2)
        qs = [(1.0 / 3.0) * q + (2.0 / 3.0) * (a - dt * r) for q, a, r in zip(qs, q2, r2)]
    return qs
