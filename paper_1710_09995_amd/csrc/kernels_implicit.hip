// Implicit step on the finite-volume residual: backward Euler
//   (V_c / dt_c + d(V R)_c / dQ) dQ = -V_c R_c
// with the first-order flux-split approximate Jacobian (frozen dissipation
// mu_f = lambda_f / 2 + lv_f per face) relaxed by point-Jacobi sweeps.  The
// paper's flowchart solves a sparse linear system per step (Section 2.3)
// without naming the method; this is the library's data-parallel reading (the
// same one as the WCNS-E-5 path's implicit step, on this residual).
//
// Work arrays (caller's workspace, each in the state arena's layout: per
// block 5 variables with the block's strides and offset):
//   R    the residual of Q^n (written by the stage kernel in mode 0);
//   dA   dQ iterate, dB the next iterate (ping-pong);
//   MU   variables 0-2: mu of the lower d-face of every cell position (index
//        0..n_d along d, so the last entry is the block's upper face), 3: the
//        diagonal D, 4: the per-cell time step.
// Every kernel walks the interior cells as the grid's 64-cell row chunks
// (chunks.hpp), one launch over all blocks, coalesced along i.
#include <hip/hip_runtime.h>
#include "cfd_internal.hpp"
#include "physics.hpp"
#include "stage_common.hpp"
#include "chunks.hpp"
#include "implicit.hpp"

namespace cfd {


// mu = lambda / 2 + lv on the face between cells a (below) and b (above) with
// area vector (sx, sy, sz): lambda of the mean primitive state of the two
// cells, lv the viscous radius with mean mu/rho and mean volume.
__device__ __forceinline__ double face_mu(const double qa[5], const double qb[5], double sx, double sy, double sz,
                                          double va, double vb, const ImplicitArgs& A) {
  const double gm1 = A.gamma - 1.0;
  const Prim<double> wa = to_prim<double>(qa[0], qa[1], qa[2], qa[3], qa[4], gm1);
  const Prim<double> wb = to_prim<double>(qb[0], qb[1], qb[2], qb[3], qb[4], gm1);
  const double rm = 0.5 * (wa.r + wb.r), um = 0.5 * (wa.u + wb.u), vm = 0.5 * (wa.v + wb.v),
               wm = 0.5 * (wa.w + wb.w), pm = 0.5 * (wa.p + wb.p);
  const double s2 = sx * sx + sy * sy + sz * sz;
  const double lam = fabs(um * sx + vm * sy + wm * sz) + fsqrt(A.gamma * pm * frcp(rm)) * fsqrt(s2);
  double mu = 0.5 * lam;
  if (A.viscous) {
    const double ta = wa.p * frcp(wa.r), tb = wb.p * frcp(wb.r);
    const double na = sutherland<double>(ta, A.mu_inf, A.s_star) * frcp(wa.r);
    const double nb = sutherland<double>(tb, A.mu_inf, A.s_star) * frcp(wb.r);
    mu += fmax(4.0 / 3.0, A.gamma / A.prandtl) * (0.5 * (na + nb)) * s2 * frcp(0.5 * (va + vb));
  }
  return mu;
}

// F(Q) . S of the inviscid flux of Eq. (1).
__device__ __forceinline__ void flux_dot(const double Q[5], double sx, double sy, double sz, double gm1, double F[5]) {
  const double ir = frcp(Q[0]);
  const double u = Q[1] * ir, v = Q[2] * ir, w = Q[3] * ir;
  const double p = gm1 * (Q[4] - 0.5 * Q[0] * (u * u + v * v + w * w));
  const double U = u * sx + v * sy + w * sz;
  F[0] = Q[0] * U;
  F[1] = Q[1] * U + p * sx;
  F[2] = Q[2] * U + p * sy;
  F[3] = Q[3] * U + p * sz;
  F[4] = (Q[4] + p) * U;
}

__device__ __forceinline__ void load5(const double* __restrict__ a, int64_t o, int64_t sv, double x[5]) {
#pragma unroll
  for (int v = 0; v < 5; ++v) x[v] = a[v * sv + o];
}

// mu of the three lower faces of every interior cell (and of the block's upper
// faces, by the last cell along each direction); the per-cell time step.
__global__ void __launch_bounds__(256) k_ifv_faces(ImplicitArgs A, const BlockDesc* __restrict__ blocks, int nblk,
                                                   int64_t nchunks, StepParams P) {
  const int lane = threadIdx.x & 63;
  int64_t r0, r1;
  wave_rows(nchunks, r0, r1);
  ChunkWalk W;
  if (r0 < r1) W.start(blocks, nblk, r0);
  for (int64_t u = r0; u < r1; ++u) {
    int i, j, k;
    if (!W.cell(u, lane, i, j, k)) continue;
    const BlockDesc& B = W.B;
    const int64_t c = (int64_t)(k + NG) * B.sk + (int64_t)(j + NG) * B.sj + (i + NG);
    const double* qb = A.q + B.qoff;
    const double* mb = A.met + B.moff;
    double* mub = A.mu + B.qoff;
    double qc[5];
    load5(qb, c, B.sv, qc);
    const double vc = mb[9 * B.sv + c];
    const int idx[3] = {i, j, k};
#pragma unroll
    for (int d = 0; d < 3; ++d) {
      const int64_t sd = d == 0 ? 1 : (d == 1 ? B.sj : B.sk);
      double qn[5];
      load5(qb, c - sd, B.sv, qn);
      mub[d * B.sv + c] = face_mu(qn, qc, mb[(3 * d) * B.sv + c], mb[(3 * d + 1) * B.sv + c],
                                  mb[(3 * d + 2) * B.sv + c], mb[9 * B.sv + c - sd], vc, A);
      if (idx[d] == B.n[d] - 1) {
        load5(qb, c + sd, B.sv, qn);
        const int64_t cu = c + sd;
        mub[d * B.sv + cu] = face_mu(qc, qn, mb[(3 * d) * B.sv + cu], mb[(3 * d + 1) * B.sv + cu],
                                     mb[(3 * d + 2) * B.sv + cu], vc, mb[9 * B.sv + cu], A);
      }
    }
    mub[4 * B.sv + c] = cell_dt(qc, mb, c, B.sv, B.sj, B.sk, P);
  }
}

// D = V/dt + the six faces' mu; first iterate dQ = -V R / D.
__global__ void __launch_bounds__(256) k_ifv_diag(ImplicitArgs A, const BlockDesc* __restrict__ blocks, int nblk,
                                                  int64_t nchunks) {
  const int lane = threadIdx.x & 63;
  int64_t r0, r1;
  wave_rows(nchunks, r0, r1);
  ChunkWalk W;
  if (r0 < r1) W.start(blocks, nblk, r0);
  for (int64_t u = r0; u < r1; ++u) {
    int i, j, k;
    if (!W.cell(u, lane, i, j, k)) continue;
    const BlockDesc& B = W.B;
    const int64_t c = (int64_t)(k + NG) * B.sk + (int64_t)(j + NG) * B.sj + (i + NG);
    const double* mb = A.met + B.moff;
    double* mub = A.mu + B.qoff;
    const double vc = mb[9 * B.sv + c];
    const double dtc = A.local ? mub[4 * B.sv + c] : A.dt[0];
    double D = vc / dtc;
#pragma unroll
    for (int d = 0; d < 3; ++d) {
      const int64_t sd = d == 0 ? 1 : (d == 1 ? B.sj : B.sk);
      D = D + mub[d * B.sv + c] + mub[d * B.sv + c + sd];
    }
    mub[3 * B.sv + c] = D;
    const double* rb = A.r + B.qoff;
    double* ob = A.dq_out + B.qoff;
#pragma unroll
    for (int v = 0; v < 5; ++v) ob[v * B.sv + c] = -vc * rb[v * B.sv + c] / D;
  }
}

// One point-Jacobi sweep: dQ_out = (-V R - O(dQ_in)) / D, where over each
// direction the upper face adds dF(c+e)/2 - mu dQ(c+e) and the lower face
// -dF(c-e)/2 - mu dQ(c-e), dF(m) = F(Q_m + dQ_m) . S - F(Q_m) . S.
__global__ void __launch_bounds__(256) k_ifv_sweep(ImplicitArgs A, const BlockDesc* __restrict__ blocks, int nblk,
                                                   int64_t nchunks) {
  const int lane = threadIdx.x & 63;
  const double gm1 = A.gamma - 1.0;
  int64_t r0, r1;
  wave_rows(nchunks, r0, r1);
  ChunkWalk W;
  if (r0 < r1) W.start(blocks, nblk, r0);
  for (int64_t u = r0; u < r1; ++u) {
    int i, j, k;
    if (!W.cell(u, lane, i, j, k)) continue;
    const BlockDesc& B = W.B;
    const int64_t c = (int64_t)(k + NG) * B.sk + (int64_t)(j + NG) * B.sj + (i + NG);
    const double* qb = A.q + B.qoff;
    const double* mb = A.met + B.moff;
    const double* mub = A.mu + B.qoff;
    const double* db = A.dq_in + B.qoff;
    double O[5] = {0.0, 0.0, 0.0, 0.0, 0.0};
#pragma unroll
    for (int d = 0; d < 3; ++d) {
      const int64_t sd = d == 0 ? 1 : (d == 1 ? B.sj : B.sk);
      double up[5], lo[5];
      {
        const int64_t m = c + sd;            // upper neighbour, through the cell's upper face
        double Qm[5], dQ[5], Qp[5], F0[5], F1[5];
        load5(qb, m, B.sv, Qm);
        load5(db, m, B.sv, dQ);
        const double sx = mb[(3 * d) * B.sv + m], sy = mb[(3 * d + 1) * B.sv + m], sz = mb[(3 * d + 2) * B.sv + m];
#pragma unroll
        for (int v = 0; v < 5; ++v) Qp[v] = Qm[v] + dQ[v];
        flux_dot(Qp, sx, sy, sz, gm1, F1);
        flux_dot(Qm, sx, sy, sz, gm1, F0);
        const double mu = mub[d * B.sv + m];
#pragma unroll
        for (int v = 0; v < 5; ++v) up[v] = 0.5 * (F1[v] - F0[v]) - mu * dQ[v];
      }
      {
        const int64_t m = c - sd;            // lower neighbour, through the cell's lower face
        double Qm[5], dQ[5], Qp[5], F0[5], F1[5];
        load5(qb, m, B.sv, Qm);
        load5(db, m, B.sv, dQ);
        const double sx = mb[(3 * d) * B.sv + c], sy = mb[(3 * d + 1) * B.sv + c], sz = mb[(3 * d + 2) * B.sv + c];
#pragma unroll
        for (int v = 0; v < 5; ++v) Qp[v] = Qm[v] + dQ[v];
        flux_dot(Qp, sx, sy, sz, gm1, F1);
        flux_dot(Qm, sx, sy, sz, gm1, F0);
        const double mu = mub[d * B.sv + c];
#pragma unroll
        for (int v = 0; v < 5; ++v) lo[v] = -0.5 * (F1[v] - F0[v]) - mu * dQ[v];
      }
#pragma unroll
      for (int v = 0; v < 5; ++v) O[v] = O[v] + (up[v] + lo[v]);
    }
    const double vc = mb[9 * B.sv + c];
    const double D = mub[3 * B.sv + c];
    const double* rb = A.r + B.qoff;
    double* ob = A.dq_out + B.qoff;
    double rhs[5];
#pragma unroll
    for (int v = 0; v < 5; ++v) rhs[v] = -vc * rb[v * B.sv + c];
#pragma unroll
    for (int v = 0; v < 5; ++v) ob[v * B.sv + c] = (rhs[v] - O[v]) / D;
  }
}

// Q += dQ on the interior cells.
__global__ void __launch_bounds__(256) k_ifv_apply(double* __restrict__ q, const double* __restrict__ dq,
                                                   const BlockDesc* __restrict__ blocks, int nblk, int64_t nchunks) {
  const int lane = threadIdx.x & 63;
  int64_t r0, r1;
  wave_rows(nchunks, r0, r1);
  ChunkWalk W;
  if (r0 < r1) W.start(blocks, nblk, r0);
  for (int64_t u = r0; u < r1; ++u) {
    int i, j, k;
    if (!W.cell(u, lane, i, j, k)) continue;
    const BlockDesc& B = W.B;
    const int64_t c = (int64_t)(k + NG) * B.sk + (int64_t)(j + NG) * B.sj + (i + NG);
    double x[5], y[5];
    load5(q + B.qoff, c, B.sv, x);
    load5(dq + B.qoff, c, B.sv, y);
#pragma unroll
    for (int v = 0; v < 5; ++v) q[B.qoff + v * B.sv + c] = x[v] + y[v];
  }
}

// ------------------------------------------------------------------ launchers

void launch_ifv_faces(const ImplicitArgs& A, const BlockDesc* blocks, int nblk, int64_t nchunks,
                      const StepParams& P, int nwg, hipStream_t s) {
  hipLaunchKernelGGL(k_ifv_faces, dim3(nwg), dim3(256), 0, s, A, blocks, nblk, nchunks, P);
}
void launch_ifv_diag(const ImplicitArgs& A, const BlockDesc* blocks, int nblk, int64_t nchunks, int nwg,
                     hipStream_t s) {
  hipLaunchKernelGGL(k_ifv_diag, dim3(nwg), dim3(256), 0, s, A, blocks, nblk, nchunks);
}
void launch_ifv_sweep(const ImplicitArgs& A, const BlockDesc* blocks, int nblk, int64_t nchunks, int nwg,
                      hipStream_t s) {
  hipLaunchKernelGGL(k_ifv_sweep, dim3(nwg), dim3(256), 0, s, A, blocks, nblk, nchunks);
}
void launch_ifv_apply(double* q, const double* dq, const BlockDesc* blocks, int nblk, int64_t nchunks, int nwg,
                      hipStream_t s) {
  hipLaunchKernelGGL(k_ifv_apply, dim3(nwg), dim3(256), 0, s, q, dq, blocks, nblk, nchunks);
}

}  // namespace cfd
