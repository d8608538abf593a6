// Device code shared by the stage kernels: one face-flux function fed by
// different gathers (straight from global memory, or from LDS planes), the
// cell update of Eqs. (4)-(6) and the norm partials.
//
// Both stage kernels call face_inviscid / face_viscous with bitwise identical
// inputs in the same order (the same
// primitives from the same Q, the same metric loads, the same averaging
// expressions), and the sources are built with -ffp-contract=on so the
// contraction of each expression is fixed by the source: every face flux is
// the same bits whichever kernel, tile shape or launch computed it.
#pragma once
#include <hip/hip_runtime.h>
#include "cfd_internal.hpp"
#include "physics.hpp"

namespace cfd {

template <typename T>
__device__ __forceinline__ Prim<T> ld_prim(const double* __restrict__ qb, int64_t o, int64_t sv, T gm1) {
  return to_prim<T>(qb[o], qb[o + sv], qb[o + 2 * sv], qb[o + 3 * sv], qb[o + 4 * sv], gm1);
}

__device__ __forceinline__ int64_t dstride(int d, int64_t sj, int64_t sk) {
  return d == 0 ? 1 : (d == 1 ? sj : sk);
}

// phi = (u, v, w, T) of a cell
template <typename T>
__device__ __forceinline__ void phi_of(const Prim<T>& W, T tc, T phi[4]) {
  phi[0] = W.u;
  phi[1] = W.v;
  phi[2] = W.w;
  phi[3] = tc;
}

template <typename T>
__device__ __forceinline__ T temp_of(const Prim<T>& W) {
  return div_t(W.p, W.r);
}

// transverse difference 1/4 (phi(L+e) + phi(R+e) - phi(L-e) - phi(R-e))
template <typename T>
__device__ __forceinline__ void tdiff(const T a[4], const T b[4], const T e[4], const T f[4], T out[4]) {
#pragma unroll
  for (int q = 0; q < 4; ++q) out[q] = T(0.25) * (a[q] + b[q] - e[q] - f[q]);
}

// Metric terms of the viscous face between cells cl (L) and c (R) in
// direction d: averaged transverse face vectors (ascending transverse order)
// and the auxiliary volume.  The grid is fixed, so these are evaluated once,
// when the blocks are created, into the viscous face metric arena; the stage
// kernels read them back with face_vmetrics (the same bits).
__device__ __forceinline__ void visc_metrics(const double* __restrict__ mb, int64_t sv, int64_t cl, int64_t c,
                                             int d, int64_t sj, int64_t sk, double St[2][3], double& vf) {
  int tt = 0;
#pragma unroll
  for (int t = 0; t < 3; ++t) {
    if (t == d) continue;
    const int64_t st = dstride(t, sj, sk);
#pragma unroll
    for (int x = 0; x < 3; ++x) {
      const int64_t mo = (int64_t)(3 * t + x) * sv;
      St[tt][x] = 0.25 * (mb[mo + cl] + mb[mo + cl + st] + mb[mo + c] + mb[mo + c + st]);
    }
    ++tt;
  }
  vf = 0.5 * (mb[9 * sv + cl] + mb[9 * sv + c]);
}

// Viscous metric terms of the lower d-face of cell c, from the arena vb.
__device__ __forceinline__ void face_vmetrics(const double* __restrict__ vb, int64_t sv, int64_t c, int d,
                                              double St[2][3], double& vf) {
#pragma unroll
  for (int u = 0; u < 2; ++u)
#pragma unroll
    for (int x = 0; x < 3; ++x) St[u][x] = vb[(int64_t)(7 * d + 3 * u + x) * sv + c];
  vf = vb[(int64_t)(7 * d + 6) * sv + c];
}

// Inviscid part of one face: MUSCL states from cells c-2, c-1 (L), c (R),
// c+1 along the face direction, then Roe's flux per unit area f through the
// face vector (sx, sy, sz).  Returns |S|; n receives the unit normal.
template <typename T>
__device__ __forceinline__ double face_inviscid(const Prim<T>& a, const Prim<T>& b, const Prim<T>& c,
                                                const Prim<T>& d, double sx, double sy, double sz,
                                                const Gas<T>& gas, T f[5], T n[3]) {
  Prim<T> L, R;
  muscl(a, b, c, d, gas.eps_lim, L, R);
  const double area = fsqrt(sx * sx + sy * sy + sz * sz);
  const double ia = frcp(area);
  n[0] = (T)(sx * ia);
  n[1] = (T)(sy * ia);
  n[2] = (T)(sz * ia);
  roe<T>(L, R, n[0], n[1], n[2], gas, f);
  return area;
}

// Viscous part: subtract F_v . n from f.  pl, pr: phi of L and R;
// dt1, dt2: transverse differences of phi (ascending transverse order);
// St, vf: averaged transverse face vectors and the auxiliary volume.
template <typename T>
__device__ __forceinline__ void face_viscous(const T pl[4], const T pr[4], double sx, double sy, double sz,
                                             const T n[3], const T dt1[4], const T dt2[4], const double St[2][3],
                                             double vf, const Gas<T>& gas, T f[5]) {
  const double iv = frcp(vf);
  const T sdx = (T)(sx * iv), sdy = (T)(sy * iv), sdz = (T)(sz * iv);
  const T s1x = (T)(St[0][0] * iv), s1y = (T)(St[0][1] * iv), s1z = (T)(St[0][2] * iv);
  const T s2x = (T)(St[1][0] * iv), s2y = (T)(St[1][1] * iv), s2z = (T)(St[1][2] * iv);
  T g[4][3];
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    const T dq = pr[q] - pl[q];
    g[q][0] = dq * sdx + dt1[q] * s1x + dt2[q] * s2x;
    g[q][1] = dq * sdy + dt1[q] * s1y + dt2[q] * s2y;
    g[q][2] = dq * sdz + dt1[q] * s1z + dt2[q] * s2z;
  }
  const T uf[3] = {T(0.5) * (pl[0] + pr[0]), T(0.5) * (pl[1] + pr[1]), T(0.5) * (pl[2] + pr[2])};
  const T tf = T(0.5) * (pl[3] + pr[3]);
  T fv[5];
  viscous_n<T>(g, uf, tf, n[0], n[1], n[2], gas, fv);
#pragma unroll
  for (int q = 0; q < 5; ++q) f[q] -= fv[q];
}

__device__ __forceinline__ void scale_flux_f64(const double f[5], double area, double F[5]) {
#pragma unroll
  for (int q = 0; q < 5; ++q) F[q] = f[q] * area;
}
__device__ __forceinline__ void scale_flux_f64(const float f[5], double area, double F[5]) {
#pragma unroll
  for (int q = 0; q < 5; ++q) F[q] = (double)f[q] * area;
}

// Face flux (F_inv - F_vis) . S on the lower d-face of cell c, every input
// read from global memory.
template <typename T, bool VISC>
__device__ __forceinline__ void face_flux_global(const double* __restrict__ qb, const double* __restrict__ mb,
                                                 const double* __restrict__ vb, const BlockDesc& B, int64_t c,
                                                 int d, const Gas<T>& gas, double F[5]) {
  const int64_t sd = dstride(d, B.sj, B.sk);
  const int64_t sv = B.sv;
  const double sx = mb[(3 * d) * sv + c], sy = mb[(3 * d + 1) * sv + c], sz = mb[(3 * d + 2) * sv + c];
  T f[5], n[3];
  T pl[4], pr[4];
  double area;
  {
    const Prim<T> wm2 = ld_prim<T>(qb, c - 2 * sd, sv, gas.gm1);
    const Prim<T> wm1 = ld_prim<T>(qb, c - sd, sv, gas.gm1);
    const Prim<T> w0 = ld_prim<T>(qb, c, sv, gas.gm1);
    const Prim<T> wp1 = ld_prim<T>(qb, c + sd, sv, gas.gm1);
    area = face_inviscid<T>(wm2, wm1, w0, wp1, sx, sy, sz, gas, f, n);
    if (VISC) {
      phi_of(wm1, temp_of(wm1), pl);
      phi_of(w0, temp_of(w0), pr);
    }
  }
  if (VISC) {
    const int64_t cl = c - sd;
    T dd[2][4];
    int tt = 0;
    for (int t = 0; t < 3; ++t) {
      if (t == d) continue;
      const int64_t st = dstride(t, B.sj, B.sk);
      T a[4], b[4], e[4], ff[4];
      Prim<T> W;
      W = ld_prim<T>(qb, cl + st, sv, gas.gm1);
      phi_of(W, temp_of(W), a);
      W = ld_prim<T>(qb, c + st, sv, gas.gm1);
      phi_of(W, temp_of(W), b);
      W = ld_prim<T>(qb, cl - st, sv, gas.gm1);
      phi_of(W, temp_of(W), e);
      W = ld_prim<T>(qb, c - st, sv, gas.gm1);
      phi_of(W, temp_of(W), ff);
      tdiff(a, b, e, ff, dd[tt]);
      ++tt;
    }
    double St[2][3], vf;
    face_vmetrics(vb, sv, c, d, St, vf);
    face_viscous<T>(pl, pr, sx, sy, sz, n, dd[0], dd[1], St, vf, gas, f);
  }
  scale_flux_f64(f, area, F);
}

__device__ __forceinline__ void init_partials(double acc[NPART]) {
#pragma unroll
  for (int q = 0; q < NPART; ++q) acc[q] = 0.0;
  acc[12] = __builtin_inf();
}

__device__ __forceinline__ bool finite(double x) { return !(isnan(x) || isinf(x)); }

// Admissible time step of one cell with conserved state q (FP64):
// dt_c = CFL V / (sum_d L_d + 4 sum_d Lv_d), S_d averaged over the cell's two
// d-faces (b[d]), L_d = |u . S_d| + c |S_d|,
// Lv_d = max(4/3, gamma/Pr)(mu/rho)|S_d|^2/V.
__device__ __forceinline__ double cell_dt_b(const double q[5], const double b[3][3], double vol,
                                            const StepParams& P) {
  const double gm1 = P.gamma - 1.0;
  const double r = q[0];
  const double inv = frcp(r);
  const double u = q[1] * inv, v = q[2] * inv, w = q[3] * inv;
  const double p = gm1 * (q[4] - 0.5 * r * (u * u + v * v + w * w));
  const double cs = fsqrt(P.gamma * p * inv);
  const double coefv = fmax(4.0 / 3.0, P.gamma / P.prandtl);
  double mu_r = 0.0;
  if (P.viscous) {
    const double t = p * inv;
    mu_r = P.mu_inf * t * fsqrt(t) * (1.0 + P.s_star) * frcp(t + P.s_star) * inv;
  }
  const double ivol = frcp(vol);
  double lam = 0.0, lamv = 0.0;
#pragma unroll
  for (int d = 0; d < 3; ++d) {
    const double bx = b[d][0], by = b[d][1], bz = b[d][2];
    const double m2 = bx * bx + by * by + bz * bz;
    lam += fabs(u * bx + v * by + w * bz) + cs * fsqrt(m2);
    if (P.viscous) lamv += coefv * mu_r * m2 * ivol;
  }
  return fdiv(P.cfl * vol, lam + 4.0 * lamv);
}

// The face-averaged area vectors of cell c: b[d] = (S_d(c) + S_d(c + e_d)) / 2.
__device__ __forceinline__ void dt_vectors(const double* __restrict__ mb, int64_t c, int64_t sv, int64_t sj,
                                           int64_t sk, double b[3][3]) {
#pragma unroll
  for (int d = 0; d < 3; ++d) {
    const int64_t sd = dstride(d, sj, sk);
#pragma unroll
    for (int x = 0; x < 3; ++x) b[d][x] = 0.5 * (mb[(3 * d + x) * sv + c] + mb[(3 * d + x) * sv + c + sd]);
  }
}

__device__ __forceinline__ double cell_dt(const double q[5], const double* __restrict__ mb, int64_t c,
                                          int64_t sv, int64_t sj, int64_t sk, const StepParams& P) {
  double b[3][3];
  dt_vectors(mb, c, sv, sj, sk, b);
  return cell_dt_b(q, b, mb[9 * sv + c], P);
}

// Inputs of one cell's update besides its flux differences.
struct CellIn {
  double qv[5], qn[5], dt, vol;
};

// Load them (qn only in mode 2, dt only in modes 1-2).  Every load of the
// update is issued before its first store: the output may alias the inputs
// as far as the compiler knows, so a load placed after a store would wait for
// that store (and, through the shared memory counter, for every store before
// it).  A kernel may load them early, before its face work, to hide latency.
template <int MODE>
__device__ __forceinline__ void load_cell(const StageArgs& A, const BlockDesc& B, int64_t c, CellIn& in) {
  in.vol = A.met[B.moff + 9 * B.sv + c];
  if (MODE == 0) return;
  in.dt = A.local_dt ? A.dt[B.soff + c] : A.dt[0];
  const double* qb = A.qs + B.qoff;
#pragma unroll
  for (int q = 0; q < 5; ++q) in.qv[q] = qb[q * B.sv + c];
  if (MODE >= 2) {
#pragma unroll
    for (int q = 0; q < 5; ++q) in.qn[q] = A.qn[B.qoff + q * B.sv + c];
  }
}

// R = ((Di + Dj) + Dk) / V, then write R (mode 0) or the stage update
// (modes 1-3; mode 1 also writes R for the norms if A.rout is set), less
// (A.fb dt) force when a multigrid level's forcing is given.  R is returned
// in Rc, the written state in Qo (modes 1-3).
template <int MODE>
__device__ __forceinline__ void update_cell(const StageArgs& A, const BlockDesc& B, int64_t c, const double Di[5],
                                            const double Dj[5], const double Dk[5], const CellIn& in,
                                            double Rc[5] = nullptr, double Qo[5] = nullptr,
                                            const double* force = nullptr) {
  double R[5];
  const double ivol = frcp(in.vol);
#pragma unroll
  for (int q = 0; q < 5; ++q) R[q] = ((Di[q] + Dj[q]) + Dk[q]) * ivol;
  if (MODE == 0) {
#pragma unroll
    for (int q = 0; q < 5; ++q) A.out[B.qoff + q * B.sv + c] = R[q];
  } else if (MODE == 1) {
#pragma unroll
    for (int q = 0; q < 5; ++q) {
      double o = in.qv[q] - in.dt * R[q];
      if (force) {
        const double h = A.fb * in.dt;
        o = o - h * force[B.qoff + q * B.sv + c];
      }
      A.out[B.qoff + q * B.sv + c] = o;
      if (A.rout) A.rout[B.qoff + q * B.sv + c] = R[q];
      if (Qo) Qo[q] = o;
    }
  } else {
#pragma unroll
    for (int q = 0; q < 5; ++q) {
      double o = A.a * in.qn[q] + A.b * (in.qv[q] - in.dt * R[q]);
      if (force) {
        const double h = A.fb * in.dt;
        o = o - h * force[B.qoff + q * B.sv + c];
      }
      A.out[B.qoff + q * B.sv + c] = o;
      if (Qo) Qo[q] = o;
    }
  }
  if (Rc) {
#pragma unroll
    for (int q = 0; q < 5; ++q) Rc[q] = R[q];
  }
}

template <int MODE>
__device__ __forceinline__ void finish_cell(const StageArgs& A, const BlockDesc& B, int64_t c, const double Di[5],
                                            const double Dj[5], const double Dk[5]) {
  CellIn in;
  load_cell<MODE>(A, B, c, in);
  update_cell<MODE>(A, B, c, Di, Dj, Dk, in, nullptr, nullptr, A.force);
}

// Fixed-order workgroup reduction of NPART partials; thread 0 writes the row.
// Slots: sums for [0,10) and 11, max for 10, min for 12.  red: LDS scratch of
// NPART x 16 doubles that no thread uses any more (the first barrier below
// orders the caller's last uses before it).
__device__ __forceinline__ void wg_reduce_partials(double acc[NPART], double* __restrict__ out_row,
                                                   double (*red)[16]) {
  const int lane = threadIdx.x & 63;
  const int wave = threadIdx.x >> 6;
  const int nwave = (blockDim.x + 63) >> 6;
  __syncthreads();
#pragma unroll
  for (int q = 0; q < NPART; ++q) {
    double v = acc[q];
    for (int off = 32; off > 0; off >>= 1) {
      const double o = __shfl_xor(v, off, 64);
      if (q == 10) v = fmax(v, o);
      else if (q == 12) v = fmin(v, o);
      else v = v + o;
    }
    if (lane == 0) red[q][wave] = v;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    for (int q = 0; q < NPART; ++q) {
      double v = red[q][0];
      for (int w = 1; w < nwave; ++w) {
        if (q == 10) v = fmax(v, red[q][w]);
        else if (q == 12) v = fmin(v, red[q][w]);
        else v = v + red[q][w];
      }
      out_row[q] = v;
    }
  }
  __syncthreads();
}
__device__ __forceinline__ void wg_reduce_partials(double acc[NPART], double* __restrict__ out_row) {
  __shared__ double red[NPART][16];
  wg_reduce_partials(acc, out_row, red);
}

}  // namespace cfd
