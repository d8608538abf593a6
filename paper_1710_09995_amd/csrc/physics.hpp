// Device physics: primitives, MUSCL reconstruction, Roe flux, viscous flux,
// far-field state.  Templated on the flux precision T (double, or float for
// the FP32-flux variant); the state, metrics and all sums stay FP64.
//
// Governing equations: Section 2.1, Eq. (1); the cell-edge reconstruction and
// flux splitting of Section 2.2 are left open by the paper and are defined
// here as kappa = 1/3 MUSCL with the smooth limiter
// s(a,b) = (2ab + eps)/(a^2 + b^2 + eps) and Roe's solver with Harten's fix on
// the acoustic waves.  Units: rho_inf = p_inf = 1, T = p/rho, c^2 = gamma T.
#pragma once
#include <hip/hip_runtime.h>
#include "cfd_internal.hpp"

namespace cfd {

template <typename T>
struct Prim {
  T r, u, v, w, p;
};

template <typename T>
__device__ __forceinline__ Prim<T> to_prim(double q0, double q1, double q2, double q3, double q4,
                                           T gm1) {
  Prim<T> W;
  W.r = (T)q0;
  T inv = T(1) / W.r;
  W.u = (T)q1 * inv;
  W.v = (T)q2 * inv;
  W.w = (T)q3 * inv;
  W.p = gm1 * ((T)q4 - T(0.5) * W.r * (W.u * W.u + W.v * W.v + W.w * W.w));
  return W;
}

template <typename T>
__device__ __forceinline__ T limiter(T a, T b, T eps) {
  return (T(2) * a * b + eps) / (a * a + b * b + eps);
}

// Left and right states of one component at the face between cells c-1, c.
template <typename T>
__device__ __forceinline__ void muscl1(T wm2, T wm1, T w0, T wp1, T eps, T& wl, T& wr) {
  const T kap = T(1.0 / 3.0);
  T dm = wm1 - wm2;
  T dp = w0 - wm1;
  T s = limiter(dm, dp, eps);
  wl = wm1 + T(0.25) * s * ((T(1) - kap * s) * dm + (T(1) + kap * s) * dp);
  T dp2 = wp1 - w0;
  T s2 = limiter(dp, dp2, eps);
  wr = w0 - T(0.25) * s2 * ((T(1) - kap * s2) * dp2 + (T(1) + kap * s2) * dp);
}

template <typename T>
__device__ __forceinline__ void muscl(const Prim<T>& a, const Prim<T>& b, const Prim<T>& c,
                                      const Prim<T>& d, T eps, Prim<T>& L, Prim<T>& R) {
  muscl1(a.r, b.r, c.r, d.r, eps, L.r, R.r);
  muscl1(a.u, b.u, c.u, d.u, eps, L.u, R.u);
  muscl1(a.v, b.v, c.v, d.v, eps, L.v, R.v);
  muscl1(a.w, b.w, c.w, d.w, eps, L.w, R.w);
  muscl1(a.p, b.p, c.p, d.p, eps, L.p, R.p);
  // positivity fallback: first order on this face
  if (!(L.r > T(0)) || !(L.p > T(0)) || !(R.r > T(0)) || !(R.p > T(0))) {
    L = b;
    R = c;
  }
}

// Roe flux per unit area through a face with unit normal n (Roe 1981, Harten fix).
template <typename T>
__device__ __forceinline__ void roe(const Prim<T>& L, const Prim<T>& R, T nx, T ny, T nz,
                                    T gamma, T eps_h, T F[5]) {
  const T gm1 = gamma - T(1);
  const T gg = gamma / gm1;
  T Hl = gg * L.p / L.r + T(0.5) * (L.u * L.u + L.v * L.v + L.w * L.w);
  T Hr = gg * R.p / R.r + T(0.5) * (R.u * R.u + R.v * R.v + R.w * R.w);
  T r = sqrt(R.r / L.r);
  T rhat = r * L.r;
  T i1r = T(1) / (T(1) + r);
  T uh = (L.u + r * R.u) * i1r;
  T vh = (L.v + r * R.v) * i1r;
  T wh = (L.w + r * R.w) * i1r;
  T Hh = (Hl + r * Hr) * i1r;
  T q2 = uh * uh + vh * vh + wh * wh;
  T c2 = gm1 * (Hh - T(0.5) * q2);
  T ch = sqrt(c2);
  T Uh = uh * nx + vh * ny + wh * nz;
  T dr = R.r - L.r;
  T du = R.u - L.u, dv = R.v - L.v, dw = R.w - L.w;
  T dp = R.p - L.p;
  T dU = du * nx + dv * ny + dw * nz;
  T l1 = fabs(Uh - ch);
  T l2 = fabs(Uh);
  T l3 = fabs(Uh + ch);
  T delta = eps_h * (fabs(Uh) + ch);
  if (l1 < delta) l1 = (l1 * l1 + delta * delta) / (T(2) * delta);
  if (l3 < delta) l3 = (l3 * l3 + delta * delta) / (T(2) * delta);
  T i2c2 = T(1) / (T(2) * c2);
  T a1 = (dp - rhat * ch * dU) * i2c2;
  T a5 = (dp + rhat * ch * dU) * i2c2;
  T a2 = dr - dp / c2;
  T w1 = l1 * a1, w5 = l3 * a5, w2 = l2 * a2, ws = l2 * rhat;
  T D0 = w1 + w2 + w5;
  T D1 = w1 * (uh - ch * nx) + w2 * uh + ws * (du - dU * nx) + w5 * (uh + ch * nx);
  T D2 = w1 * (vh - ch * ny) + w2 * vh + ws * (dv - dU * ny) + w5 * (vh + ch * ny);
  T D3 = w1 * (wh - ch * nz) + w2 * wh + ws * (dw - dU * nz) + w5 * (wh + ch * nz);
  T D4 = w1 * (Hh - ch * Uh) + w2 * (T(0.5) * q2) + ws * (uh * du + vh * dv + wh * dw - Uh * dU) +
         w5 * (Hh + ch * Uh);
  T Ul = L.u * nx + L.v * ny + L.w * nz;
  T Ur = R.u * nx + R.v * ny + R.w * nz;
  T ml = L.r * Ul, mr = R.r * Ur;
  F[0] = T(0.5) * (ml + mr - D0);
  F[1] = T(0.5) * (ml * L.u + L.p * nx + mr * R.u + R.p * nx - D1);
  F[2] = T(0.5) * (ml * L.v + L.p * ny + mr * R.v + R.p * ny - D2);
  F[3] = T(0.5) * (ml * L.w + L.p * nz + mr * R.w + R.p * nz - D3);
  F[4] = T(0.5) * (ml * Hl + mr * Hr - D4);
}

template <typename T>
__device__ __forceinline__ T sutherland(T t, T mu_inf, T s_star) {
  return mu_inf * t * sqrt(t) * (T(1) + s_star) / (t + s_star);
}

// Viscous flux F_v . n per unit area through a face of unit normal n.
//  g[a][x]: gradient of phi_a (a = u, v, w, T) in direction x at the face;
//  uf: face velocity, tf: face temperature.
template <typename T>
__device__ __forceinline__ void viscous_n(const T g[4][3], const T uf[3], T tf, T nx, T ny, T nz,
                                          const Gas<T>& gas, T F[5]) {
  T mu = sutherland(tf, gas.mu_inf, gas.s_star);
  T kc = mu * gas.gamma / (gas.gm1 * gas.prandtl);
  T div = g[0][0] + g[1][1] + g[2][2];
  T lam = T(2.0 / 3.0) * div;
  T txx = mu * (g[0][0] + g[0][0] - lam);
  T tyy = mu * (g[1][1] + g[1][1] - lam);
  T tzz = mu * (g[2][2] + g[2][2] - lam);
  T txy = mu * (g[0][1] + g[1][0]);
  T txz = mu * (g[0][2] + g[2][0]);
  T tyz = mu * (g[1][2] + g[2][1]);
  F[0] = T(0);
  F[1] = txx * nx + txy * ny + txz * nz;
  F[2] = txy * nx + tyy * ny + tyz * nz;
  F[3] = txz * nx + tyz * ny + tzz * nz;
  F[4] = uf[0] * F[1] + uf[1] * F[2] + uf[2] * F[3] +
         kc * (g[3][0] * nx + g[3][1] * ny + g[3][2] * nz);
}

// Characteristic far-field boundary state (FP64): interior conserved state q,
// outward unit normal n; writes the boundary conserved state.
__device__ __forceinline__ void farfield_state(const double q[5], double nx, double ny, double nz,
                                               const StepParams& P, double out[5]) {
  const double g = P.gamma, gm1 = g - 1.0;
  double rho = q[0];
  double inv = 1.0 / rho;
  double u = q[1] * inv, v = q[2] * inv, w = q[3] * inv;
  double p = gm1 * (q[4] - 0.5 * rho * (u * u + v * v + w * w));
  double ci = sqrt(g * p / rho);
  double Ui = u * nx + v * ny + w * nz;
  double ux = P.uinf[0], uy = P.uinf[1], uz = P.uinf[2];
  double cinf = sqrt(g);
  double Uinf = ux * nx + uy * ny + uz * nz;
  double rb, pb, ub, vb, wb;
  if (Ui >= ci) {
    rb = rho; pb = p; ub = u; vb = v; wb = w;
  } else if (Ui <= -ci) {
    rb = 1.0; pb = 1.0; ub = ux; vb = uy; wb = uz;
  } else {
    double Rp = Ui + 2.0 * ci / gm1;
    double Rm = Uinf - 2.0 * cinf / gm1;
    double Ub = 0.5 * (Rp + Rm);
    double cb = 0.25 * gm1 * (Rp - Rm);
    double s, sx, sy, sz;
    if (Ub >= 0.0) {
      s = p / pow(rho, g); sx = u; sy = v; sz = w;
    } else {
      s = 1.0; sx = ux; sy = uy; sz = uz;
    }
    double Us = sx * nx + sy * ny + sz * nz;
    rb = pow(cb * cb / (g * s), 1.0 / gm1);
    pb = rb * cb * cb / g;
    ub = sx - Us * nx + Ub * nx;
    vb = sy - Us * ny + Ub * ny;
    wb = sz - Us * nz + Ub * nz;
  }
  out[0] = rb;
  out[1] = rb * ub;
  out[2] = rb * vb;
  out[3] = rb * wb;
  out[4] = pb / gm1 + 0.5 * rb * (ub * ub + vb * vb + wb * wb);
}

}  // namespace cfd
