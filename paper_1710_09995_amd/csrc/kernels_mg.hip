// Multigrid (full approximation storage) kernels for steady marches: the
// forcing term of a coarse level's RK3 stages, the restriction of a level's
// state and forced residual to the next coarser level, the coarse forcing,
// and the injected coarse-grid correction.  A coarse cell (i, j, k) of block b
// is the union of the fine cells (2i + di, 2j + dj, 2k + dk) of the same block
// (the coarse grid keeps every second node).  All arrays are state arenas of
// their level (5 variables, ghost layers, the level's own strides); only
// interior cells are read or written.  The grids are cut into the 64-cell
// row chunks of their own level (chunks.hpp).
#include <hip/hip_runtime.h>

#include "cfd_internal.hpp"
#include "chunks.hpp"
#include "mg.hpp"

namespace cfd {

namespace {

__device__ __forceinline__ int64_t cell_index(const BlockDesc& B, int i, int j, int k) {
  return (int64_t)(k + NG) * B.sk + (int64_t)(j + NG) * B.sj + (i + NG);
}

// Q^(s) -= b dt F after a stage of Eqs. 4-6: with the stage's own update
// a Q^n + b (Q^(s-1) - dt R), this gives the stage of dQ/dt = -(R + F).
__global__ void __launch_bounds__(256) k_mg_force(double* __restrict__ q, const double* __restrict__ f,
                                                  const double* __restrict__ dt, int local, double b,
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
    const int64_t c = cell_index(B, i, j, k);
    const double h = b * (local ? dt[B.soff + c] : dt[0]);
    double x[5], y[5];
#pragma unroll
    for (int v = 0; v < 5; ++v) {
      x[v] = q[B.qoff + v * B.sv + c];
      y[v] = f[B.qoff + v * B.sv + c];
    }
#pragma unroll
    for (int v = 0; v < 5; ++v) q[B.qoff + v * B.sv + c] = x[v] - h * y[v];
  }
}

// Coarse state Q^0 = sum V Q / sum V over the 8 children (into qc and q0),
// and the restricted forced residual sum V (R + F) / V_c (into fc); the
// children in the order dk, dj, di (di fastest), each sum from the first
// child on.
__global__ void __launch_bounds__(256) k_mg_restrict(const double* __restrict__ qf, const double* __restrict__ metf,
                                                     const double* __restrict__ rf, const double* __restrict__ ff,
                                                     const BlockDesc* __restrict__ bf, double* __restrict__ qc,
                                                     double* __restrict__ q0, double* __restrict__ fc,
                                                     const double* __restrict__ metc,
                                                     const BlockDesc* __restrict__ bc, int nblk, int64_t nchunks) {
  const int lane = threadIdx.x & 63;
  int64_t r0, r1;
  wave_rows(nchunks, r0, r1);
  ChunkWalk W;
  if (r0 < r1) W.start(bc, nblk, r0);
  for (int64_t u = r0; u < r1; ++u) {
    int i, j, k;
    if (!W.cell(u, lane, i, j, k)) continue;
    const BlockDesc& C = W.B;
    const BlockDesc F = bf[W.b];
    double num[5], rs[5], den = 0.0;
    bool first = true;
#pragma unroll
    for (int dk = 0; dk < 2; ++dk)
#pragma unroll
      for (int dj = 0; dj < 2; ++dj)
#pragma unroll
        for (int di = 0; di < 2; ++di) {
          const int64_t c = cell_index(F, 2 * i + di, 2 * j + dj, 2 * k + dk);
          const double v = metf[F.moff + 9 * F.sv + c];
          double qv[5], rv[5];
#pragma unroll
          for (int x = 0; x < 5; ++x) {
            qv[x] = v * qf[F.qoff + x * F.sv + c];
            const double r = ff ? rf[F.qoff + x * F.sv + c] + ff[F.qoff + x * F.sv + c] : rf[F.qoff + x * F.sv + c];
            rv[x] = v * r;
          }
          if (first) {
#pragma unroll
            for (int x = 0; x < 5; ++x) {
              num[x] = qv[x];
              rs[x] = rv[x];
            }
            den = v;
            first = false;
          } else {
#pragma unroll
            for (int x = 0; x < 5; ++x) {
              num[x] += qv[x];
              rs[x] += rv[x];
            }
            den += v;
          }
        }
    const int64_t cc = cell_index(C, i, j, k);
    const double vc = metc[C.moff + 9 * C.sv + cc];
#pragma unroll
    for (int x = 0; x < 5; ++x) {
      const double s = num[x] / den;
      qc[C.qoff + x * C.sv + cc] = s;
      q0[C.qoff + x * C.sv + cc] = s;
      fc[C.qoff + x * C.sv + cc] = rs[x] / vc;
    }
  }
}

// F_c -= R_c(Q^0): the coarse forcing from the restricted forced residual.
__global__ void __launch_bounds__(256) k_mg_forcing(double* __restrict__ fc, const double* __restrict__ rc,
                                                    const BlockDesc* __restrict__ blocks, int nblk,
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
    const int64_t c = cell_index(B, i, j, k);
    double x[5], y[5];
#pragma unroll
    for (int v = 0; v < 5; ++v) {
      x[v] = fc[B.qoff + v * B.sv + c];
      y[v] = rc[B.qoff + v * B.sv + c];
    }
#pragma unroll
    for (int v = 0; v < 5; ++v) fc[B.qoff + v * B.sv + c] = x[v] - y[v];
  }
}

// Q_f += Q_c - Q^0_c of the parent cell (injection), over the fine grid.
__global__ void __launch_bounds__(256) k_mg_prolong(double* __restrict__ qf, const BlockDesc* __restrict__ bf,
                                                    const double* __restrict__ qc, const double* __restrict__ q0,
                                                    const BlockDesc* __restrict__ bc, int nblk, int64_t nchunks) {
  const int lane = threadIdx.x & 63;
  int64_t r0, r1;
  wave_rows(nchunks, r0, r1);
  ChunkWalk W;
  if (r0 < r1) W.start(bf, nblk, r0);
  for (int64_t u = r0; u < r1; ++u) {
    int i, j, k;
    if (!W.cell(u, lane, i, j, k)) continue;
    const BlockDesc& F = W.B;
    const BlockDesc C = bc[W.b];
    const int64_t c = cell_index(F, i, j, k);
    const int64_t p = cell_index(C, i >> 1, j >> 1, k >> 1);
    double x[5], a[5], z[5];
#pragma unroll
    for (int v = 0; v < 5; ++v) {
      x[v] = qf[F.qoff + v * F.sv + c];
      a[v] = qc[C.qoff + v * C.sv + p];
      z[v] = q0[C.qoff + v * C.sv + p];
    }
#pragma unroll
    for (int v = 0; v < 5; ++v) qf[F.qoff + v * F.sv + c] = x[v] + (a[v] - z[v]);
  }
}

}  // namespace

void launch_mg_force(double* q, const double* f, const double* dt, int local, double b, const BlockDesc* blocks,
                     int nblk, int64_t nchunks, int nwg, hipStream_t s) {
  hipLaunchKernelGGL(k_mg_force, dim3(nwg), dim3(256), 0, s, q, f, dt, local, b, blocks, nblk, nchunks);
}

void launch_mg_restrict(const double* qf, const double* metf, const double* rf, const double* ff,
                        const BlockDesc* bf, double* qc, double* q0, double* fc, const double* metc,
                        const BlockDesc* bc, int nblk, int64_t nchunks_c, int nwg, hipStream_t s) {
  hipLaunchKernelGGL(k_mg_restrict, dim3(nwg), dim3(256), 0, s, qf, metf, rf, ff, bf, qc, q0, fc, metc, bc, nblk,
                     nchunks_c);
}

void launch_mg_forcing(double* fc, const double* rc, const BlockDesc* bc, int nblk, int64_t nchunks_c, int nwg,
                       hipStream_t s) {
  hipLaunchKernelGGL(k_mg_forcing, dim3(nwg), dim3(256), 0, s, fc, rc, bc, nblk, nchunks_c);
}

void launch_mg_prolong(double* qf, const BlockDesc* bf, const double* qc, const double* q0, const BlockDesc* bc,
                       int nblk, int64_t nchunks_f, int nwg, hipStream_t s) {
  hipLaunchKernelGGL(k_mg_prolong, dim3(nwg), dim3(256), 0, s, qf, bf, qc, q0, bc, nblk, nchunks_f);
}

}  // namespace cfd
