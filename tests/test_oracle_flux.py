"""Pins for the oracle's reconstruction and fluxes (CPU only).

Textbook special cases: MUSCL exactness on linear data, Roe consistency,
pure upwinding for supersonic normal flow (the Roe property in both
directions), conservation (swap symmetry), rotational invariance, Harten fix
continuity, and exact viscous fluxes for linear fields on an affine grid.
"""
import math

import numpy as np
import pytest

from oracle import flux as fx
from oracle import solver
from paper_1710_09995_amd import cases

GAM = 1.4


def _rand_prims(rng, n, mach=0.5):
    rho = rng.uniform(0.6, 1.4, n)
    p = rng.uniform(0.6, 1.4, n)
    u = rng.uniform(-1, 1, (3, n)) * mach
    return np.vstack([rho, u, p])


def test_muscl_linear_and_constant():
    rng = np.random.default_rng(0)
    base = _rand_prims(rng, 40)
    delta = 0.01 * rng.uniform(-1, 1, (5, 40))
    W = [base + m * delta for m in (-2, -1, 0, 1)]
    WL, WR = fx.muscl(*W, eps=1e-12)
    assert np.max(np.abs(WL - (W[1] + 0.5 * delta))) < 1e-15
    assert np.max(np.abs(WR - (W[2] - 0.5 * delta))) < 1e-15
    WL, WR = fx.muscl(base, base, base, base, eps=1e-12)
    assert np.array_equal(WL, base) and np.array_equal(WR, base)


def test_muscl_discontinuity_is_first_order():
    lo = np.array([1.0, 0.1, 0.0, 0.0, 1.0])[:, None]
    hi = np.array([0.125, 0.0, 0.0, 0.0, 0.1])[:, None]
    WL, WR = fx.muscl(lo, lo, hi, hi, eps=1e-12)
    assert np.max(np.abs(WL - lo)) < 1e-10
    assert np.max(np.abs(WR - hi)) < 1e-10


def test_limiter_values():
    assert fx.limiter(0.3, 0.3, 1e-12) == 1.0
    assert abs(fx.limiter(1.0, 0.0, 1e-12)) < 1e-11
    assert abs(fx.limiter(1.0, -1.0, 0.0) + 1.0) < 1e-16


def _unit_normals(rng, n):
    v = rng.normal(size=(3, n))
    return v / np.linalg.norm(v, axis=0)


def test_roe_consistency():
    rng = np.random.default_rng(1)
    W = _rand_prims(rng, 64)
    S = rng.normal(size=(3, 64))
    F = fx.roe_flux(W, W, S, GAM, 0.1)
    area = np.linalg.norm(S, axis=0)
    Fp = fx.physical_flux(W, S / area, GAM) * area
    assert np.max(np.abs(F - Fp)) < 1e-14 * max(1.0, np.max(np.abs(Fp)))


def test_roe_physical_flux_closed_form():
    W = np.array([[1.2], [0.3], [-0.2], [0.1], [0.9]])
    n = np.array([[0.0], [1.0], [0.0]])
    F = fx.physical_flux(W, n, GAM)
    rho, u, v, w, p = W[:, 0]
    E = p / (GAM - 1) + 0.5 * rho * (u * u + v * v + w * w)
    want = [rho * v, rho * u * v, rho * v * v + p, rho * w * v, (E + p) * v]
    assert np.max(np.abs(F[:, 0] - want)) < 1e-15


@pytest.mark.parametrize("sign", [1.0, -1.0])
def test_roe_supersonic_upwinding(sign):
    """Normal Mach >= 2 on both sides: every wave runs one way, so Roe returns the
    upwind physical flux (Harten inactive since |U|-c > delta)."""
    rng = np.random.default_rng(2)
    n = _unit_normals(rng, 32)
    S = 0.7 * n
    WL = _rand_prims(rng, 32, mach=0.05)
    WR = _rand_prims(rng, 32, mach=0.05)
    for W in (WL, WR):
        c = np.sqrt(GAM * W[4] / W[0])
        W[1:4] = W[1:4] + sign * (2.2 * c) * n
    F = fx.roe_flux(WL, WR, S, GAM, 0.1)
    up = WL if sign > 0 else WR
    Fp = fx.physical_flux(up, n, GAM) * 0.7
    assert np.max(np.abs(F - Fp)) < 1e-13


def test_roe_swap_symmetry_and_rotation():
    rng = np.random.default_rng(3)
    WL = _rand_prims(rng, 50)
    WR = _rand_prims(rng, 50)
    S = rng.normal(size=(3, 50))
    F1 = fx.roe_flux(WL, WR, S, GAM, 0.1)
    F2 = fx.roe_flux(WR, WL, -S, GAM, 0.1)
    assert np.max(np.abs(F1 + F2)) < 1e-13
    # rotation
    A = np.linalg.qr(rng.normal(size=(3, 3)))[0]
    if np.linalg.det(A) < 0:
        A[:, 0] = -A[:, 0]
    rot = lambda W: np.vstack([W[0:1], A @ W[1:4], W[4:5]])
    F3 = fx.roe_flux(rot(WL), rot(WR), A @ S, GAM, 0.1)
    assert np.max(np.abs(F3[0] - F1[0])) < 1e-13
    assert np.max(np.abs(F3[4] - F1[4])) < 1e-13
    assert np.max(np.abs(F3[1:4] - A @ F1[1:4])) < 1e-13


def test_harten_fix_continuous_at_delta():
    lam = np.array([0.1 - 1e-12, 0.1, 0.1 + 1e-12])
    delta = 0.1
    fixed = np.where(lam < delta, (lam * lam + delta * delta) / (2 * delta), lam)
    assert np.max(np.abs(np.diff(fixed))) < 3e-12


def test_roe_contact_exact():
    """A stationary contact (equal p, zero normal velocity) gives zero mass flux and
    the pressure force only."""
    WL = np.array([[1.0], [0.0], [0.3], [0.0], [1.0]])
    WR = np.array([[0.5], [0.0], [0.3], [0.0], [1.0]])
    S = np.array([[2.0], [0.0], [0.0]])
    F = fx.roe_flux(WL, WR, S, GAM, 0.1)
    assert abs(F[0, 0]) < 1e-15 and abs(F[4, 0]) < 1e-15
    assert abs(F[1, 0] - 2.0) < 1e-15


def test_viscous_flux_exact_for_linear_fields():
    """u = A x + u0, T = b.x + T0 on a sheared affine grid: every face gradient is
    exact, so the oracle's viscous face flux equals the closed form."""
    rng = np.random.default_rng(4)
    E = np.eye(3) * 0.2 + 0.05 * rng.uniform(-1, 1, (3, 3))
    dims = (4, 3, 3)
    ni, nj, nk = dims
    K, J, I = np.meshgrid(np.arange(nk + 1), np.arange(nj + 1), np.arange(ni + 1), indexing="ij")
    X = (E[:, 0, None, None, None] * I + E[:, 1, None, None, None] * J + E[:, 2, None, None, None] * K)
    Am = 0.3 * rng.uniform(-1, 1, (3, 3))
    u0 = np.array([0.5, 0.1, -0.2])
    bT = 0.2 * rng.uniform(-1, 1, 3)
    T0 = 1.0
    par = cases.Params(viscous=1, reynolds=100.0, mach=0.5)
    case = cases.Case("lin", par, [dims], [X], [], [cases.full_bc(0, dims, f, cases.EXTRAP) for f in range(6)],
                      [np.ones((5, nk, nj, ni))])
    st = solver.setup(case)
    # set a linear field on all padded cells (ghosts included) at their centroids
    Xp = st.Xs[0]
    C = 0.125 * sum(Xp[:, a:a + Xp.shape[1] - 1, b:b + Xp.shape[2] - 1, c:c + Xp.shape[3] - 1]
                    for a in (0, 1) for b in (0, 1) for c in (0, 1))
    u = np.einsum("ab,b...->a...", Am, C) + u0[:, None, None, None]
    T = np.einsum("b,b...->...", bT, C) + T0
    rho = np.ones_like(T)
    p = rho * T
    st.Qs[0] = cases.conserved_from(rho, u[0], u[1], u[2], p, GAM)
    W = fx.primitives(st.Qs[0], GAM)
    mu_inf = fx.mu_inf(par)
    for d in range(3):
        Fv = solver._viscous(W, st.Ss[0], st.Vs[0], dims, d, par, 2)
        Sd = solver.window(st.Ss[0][d], dims, d, (0, 0, 0), 2)
        L = solver.unit(d, -1)
        Tf = 0.5 * (solver.window(T, dims, d, L, 2) + solver.window(T, dims, d, (0, 0, 0), 2))
        uf = 0.5 * (solver.window(u, dims, d, L, 2) + solver.window(u, dims, d, (0, 0, 0), 2))
        mu = mu_inf * Tf ** 1.5 * (1 + par.sutherland) / (Tf + par.sutherland)
        kc = mu * GAM / ((GAM - 1) * par.prandtl)
        tau = Am + Am.T - 2.0 / 3.0 * np.trace(Am) * np.eye(3)
        want_mom = mu * np.einsum("ab,b...->a...", tau, Sd)
        assert np.max(np.abs(Fv[1:4] - want_mom)) < 1e-14
        want_e = np.sum(uf * want_mom, axis=0) + kc * np.einsum("b,b...->...", bT, Sd)
        assert np.max(np.abs(Fv[4] - want_e)) < 1e-14
        assert np.all(Fv[0] == 0.0)


def test_sutherland_closed_form():
    s = 110.4 / 288.15
    assert fx.sutherland(1.0, 2.0, s) == 2.0
    T = 1.7
    assert abs(fx.sutherland(T, 1.0, s) - T ** 1.5 * (1 + s) / (T + s)) < 1e-15
    assert abs(fx.mu_inf(cases.Params(mach=0.8, reynolds=1e6)) - 0.8 * math.sqrt(1.4) / 1e6) < 1e-22
