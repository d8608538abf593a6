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

// FP64 reciprocal and square root of positive normal operands (densities,
// pressures, squared sound speeds, temperatures, volumes, face areas).
// 1 (default): the hardware estimates refined in FMA arithmetic, no
// special-case handling: reciprocal by two Newton-Raphson steps
// x' = x + x (1 - b x); square root by Goldschmidt's iteration from the
// reciprocal square root (g ~ sqrt(a), h ~ 1/(2 sqrt(a))) and two residual
// corrections g' = g + h (a - g^2) (Markstein, IBM J. Res. Dev. 34(1), 1990).
// Both stay within 1 ulp of the correctly rounded result and take about half
// the instructions of the IEEE sequences, which also scale denormal and
// infinite operands that never occur here.  Zero or negative operands give
// inf or NaN, which the non-finite counters report.  0: IEEE operations.
#ifndef CFD_FAST_F64
#define CFD_FAST_F64 1
#endif
#if CFD_FAST_F64
__device__ __forceinline__ double frcp(double b) {
  double x = __builtin_amdgcn_rcp(b);
  double e = __builtin_fma(-b, x, 1.0);
  x = __builtin_fma(x, e, x);
  e = __builtin_fma(-b, x, 1.0);
  return __builtin_fma(x, e, x);
}
__device__ __forceinline__ double fdiv(double a, double b) {
  const double x = frcp(b);
  const double q = a * x;
  return __builtin_fma(__builtin_fma(-b, q, a), x, q);
}
__device__ __forceinline__ double fsqrt(double a) {
  const double y = __builtin_amdgcn_rsq(a);
  double g = a * y, h = 0.5 * y;
  const double r = __builtin_fma(-g, h, 0.5);
  g = __builtin_fma(g, r, g);
  h = __builtin_fma(h, r, h);
  g = __builtin_fma(__builtin_fma(-g, g, a), h, g);
  return __builtin_fma(__builtin_fma(-g, g, a), h, g);
}
#else
__device__ __forceinline__ double frcp(double b) { return 1.0 / b; }
__device__ __forceinline__ double fdiv(double a, double b) { return a / b; }
__device__ __forceinline__ double fsqrt(double a) { return sqrt(a); }
#endif

// Reciprocal, quotient and square root in the flux precision: the FP64
// helpers above for double; the single-instruction hardware reciprocal and
// square root (1 ulp) for the FP32 flux variant, whose error budget is 1e-5.
__device__ __forceinline__ double rcp_t(double x) { return frcp(x); }
__device__ __forceinline__ float rcp_t(float x) { return __builtin_amdgcn_rcpf(x); }
__device__ __forceinline__ double div_t(double a, double b) { return fdiv(a, b); }
__device__ __forceinline__ float div_t(float a, float b) { return a * __builtin_amdgcn_rcpf(b); }
__device__ __forceinline__ double sqrt_t(double x) { return fsqrt(x); }
__device__ __forceinline__ float sqrt_t(float x) { return __builtin_amdgcn_sqrtf(x); }

template <typename T>
__device__ __forceinline__ Prim<T> to_prim(double q0, double q1, double q2, double q3, double q4,
                                           T gm1) {
  Prim<T> W;
  W.r = (T)q0;
  T inv = rcp_t(W.r);
  W.u = (T)q1 * inv;
  W.v = (T)q2 * inv;
  W.w = (T)q3 * inv;
  W.p = gm1 * ((T)q4 - T(0.5) * W.r * (W.u * W.u + W.v * W.v + W.w * W.w));
  return W;
}

// Reciprocals of n positive values.  FP64: one division and prefix products
// (Montgomery's batch inversion); denominators here lie in [eps, O(1e6)], so
// the products stay far inside the FP64 range.  FP32: hardware reciprocal.
template <int N>
__device__ __forceinline__ void batch_rcp(const double* den, double* inv) {
  double p[N];
  p[0] = den[0];
#pragma unroll
  for (int k = 1; k < N; ++k) p[k] = p[k - 1] * den[k];
  double r = frcp(p[N - 1]);
#pragma unroll
  for (int k = N - 1; k > 0; --k) {
    inv[k] = r * p[k - 1];
    r = r * den[k];
  }
  inv[0] = r;
}
template <int N>
__device__ __forceinline__ void batch_rcp(const float* den, float* inv) {
#pragma unroll
  for (int k = 0; k < N; ++k) inv[k] = __builtin_amdgcn_rcpf(den[k]);
}

// 1: Roe's flux divides through reciprocals (fewer FP64 divisions);
// 0: plain quotients.
#ifndef CFD_ROE_RCP
#define CFD_ROE_RCP 1
#endif

// How many limiter denominators share one reciprocal: 10 (one division per
// face), 5 (one per side) or 1 (a division each).
#ifndef CFD_LIMITER_BATCH
#define CFD_LIMITER_BATCH 5
#endif

template <typename T>
__device__ __forceinline__ void muscl(const Prim<T>& a, const Prim<T>& b, const Prim<T>& c,
                                      const Prim<T>& d, T eps, Prim<T>& L, Prim<T>& R) {
  const T A[5] = {a.r, a.u, a.v, a.w, a.p};
  const T Bv[5] = {b.r, b.u, b.v, b.w, b.p};
  const T Cv[5] = {c.r, c.u, c.v, c.w, c.p};
  const T D[5] = {d.r, d.u, d.v, d.w, d.p};
  T dm[5], dp[5], dp2[5], num[10], den[10], inv[10];
#pragma unroll
  for (int q = 0; q < 5; ++q) {
    dm[q] = Bv[q] - A[q];
    dp[q] = Cv[q] - Bv[q];
    dp2[q] = D[q] - Cv[q];
    num[q] = T(2) * dm[q] * dp[q] + eps;
    den[q] = dm[q] * dm[q] + dp[q] * dp[q] + eps;
    num[5 + q] = T(2) * dp[q] * dp2[q] + eps;
    den[5 + q] = dp[q] * dp[q] + dp2[q] * dp2[q] + eps;
  }
#if CFD_LIMITER_BATCH == 10
  batch_rcp<10>(den, inv);
#elif CFD_LIMITER_BATCH == 5
  batch_rcp<5>(den, inv);
  batch_rcp<5>(den + 5, inv + 5);
#else
#pragma unroll
  for (int k = 0; k < 10; ++k) inv[k] = rcp_t(den[k]);
#endif
  const T kap = T(1.0 / 3.0);
  T l[5], r[5];
#pragma unroll
  for (int q = 0; q < 5; ++q) {
    const T s = num[q] * inv[q];
    l[q] = Bv[q] + T(0.25) * s * ((T(1) - kap * s) * dm[q] + (T(1) + kap * s) * dp[q]);
    const T s2 = num[5 + q] * inv[5 + q];
    r[q] = Cv[q] - T(0.25) * s2 * ((T(1) - kap * s2) * dp2[q] + (T(1) + kap * s2) * dp[q]);
  }
  L.r = l[0]; L.u = l[1]; L.v = l[2]; L.w = l[3]; L.p = l[4];
  R.r = r[0]; R.u = r[1]; R.v = r[2]; R.w = r[3]; R.p = r[4];
  // positivity fallback: first order on this face
  if (!(L.r > T(0)) || !(L.p > T(0)) || !(R.r > T(0)) || !(R.p > T(0))) {
    L = b;
    R = c;
  }
}

// Roe flux per unit area through a face with unit normal n (Roe 1981, Harten fix).
template <typename T>
__device__ __forceinline__ void roe(const Prim<T>& L, const Prim<T>& R, T nx, T ny, T nz,
                                    const Gas<T>& gas, T F[5]) {
  const T gm1 = gas.gm1;
  const T gg = gas.gg;
  const T eps_h = gas.eps_h;
#if CFD_ROE_RCP
  const T iLr = rcp_t(L.r), iRr = rcp_t(R.r);
  T Hl = gg * L.p * iLr + T(0.5) * (L.u * L.u + L.v * L.v + L.w * L.w);
  T Hr = gg * R.p * iRr + T(0.5) * (R.u * R.u + R.v * R.v + R.w * R.w);
  T r = sqrt_t(R.r * iLr);
#else
  T Hl = div_t(gg * L.p, L.r) + T(0.5) * (L.u * L.u + L.v * L.v + L.w * L.w);
  T Hr = div_t(gg * R.p, R.r) + T(0.5) * (R.u * R.u + R.v * R.v + R.w * R.w);
  T r = sqrt_t(div_t(R.r, L.r));
#endif
  T rhat = r * L.r;
  T i1r = rcp_t(T(1) + r);
  T uh = (L.u + r * R.u) * i1r;
  T vh = (L.v + r * R.v) * i1r;
  T wh = (L.w + r * R.w) * i1r;
  T Hh = (Hl + r * Hr) * i1r;
  T q2 = uh * uh + vh * vh + wh * wh;
  T c2 = gm1 * (Hh - T(0.5) * q2);
  T ch = sqrt_t(c2);
  T Uh = uh * nx + vh * ny + wh * nz;
  T dr = R.r - L.r;
  T du = R.u - L.u, dv = R.v - L.v, dw = R.w - L.w;
  T dp = R.p - L.p;
  T dU = du * nx + dv * ny + dw * nz;
  T l1 = fabs(Uh - ch);
  T l2 = fabs(Uh);
  T l3 = fabs(Uh + ch);
  T delta = eps_h * (fabs(Uh) + ch);
#if CFD_ROE_RCP
  const T i2d = rcp_t(T(2) * delta);
  if (l1 < delta) l1 = (l1 * l1 + delta * delta) * i2d;
  if (l3 < delta) l3 = (l3 * l3 + delta * delta) * i2d;
#else
  if (l1 < delta) l1 = div_t(l1 * l1 + delta * delta, T(2) * delta);
  if (l3 < delta) l3 = div_t(l3 * l3 + delta * delta, T(2) * delta);
#endif
  T i2c2 = rcp_t(T(2) * c2);
  T a1 = (dp - rhat * ch * dU) * i2c2;
  T a5 = (dp + rhat * ch * dU) * i2c2;
  T a2 = dr - dp * (T(2) * i2c2);
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
  return div_t(mu_inf * t * sqrt_t(t) * (T(1) + s_star), t + s_star);
}

// Viscous flux F_v . n per unit area through a face of unit normal n.
//  g[a][x]: gradient of phi_a (a = u, v, w, T) in direction x at the face;
//  uf: face velocity, tf: face temperature.
template <typename T>
__device__ __forceinline__ void viscous_n(const T g[4][3], const T uf[3], T tf, T nx, T ny, T nz,
                                          const Gas<T>& gas, T F[5]) {
  T mu = sutherland(tf, gas.mu_inf, gas.s_star);
  T kc = mu * gas.kfac;   // k = mu gamma / ((gamma - 1) Pr)
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
                                               double g, const double uinf[3], double out[5]) {
  const double gm1 = g - 1.0;
  double rho = q[0];
  double inv = 1.0 / rho;
  double u = q[1] * inv, v = q[2] * inv, w = q[3] * inv;
  double p = gm1 * (q[4] - 0.5 * rho * (u * u + v * v + w * w));
  double ci = sqrt(g * p / rho);
  double Ui = u * nx + v * ny + w * nz;
  double ux = uinf[0], uy = uinf[1], uz = uinf[2];
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
