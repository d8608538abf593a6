// Residual, time-stage update, time step and norm kernels.
//
// R_c = ((F_i+ - F_i-) + (F_j+ - F_j-) + (F_k+ - F_k-)) / V_c with
// F = (F_inv - F_vis) . S (Section 2.2, Eq. 3, dQ/dt = -R), and the stage
// update of Eqs. (4)-(6) with lambda = -dt:
//   stage 1: Q1   = Qn - dt R(Qn)
//   stage 2: Q2   = 3/4 Qn + 1/4 (Q1 - dt R(Q1))
//   stage 3: Qn+1 = 1/3 Qn + 2/3 (Q2 - dt R(Q2))
//
// All kernels run persistent over a tile work list that spans every block:
// workgroup w takes tiles w, w + G, w + 2G, ... (static round robin), so one
// launch covers all blocks of uneven sizes.  Reductions go wave64 butterfly
// -> LDS in fixed order -> one partial row per workgroup -> a single-workgroup
// finalize in fixed order, so results are bitwise reproducible.
//
// This file holds the simple per-cell kernel (every face read from global
// memory and computed by both of its cells); the tiled face-once kernel is in
// kernels_tiled.hip.
#include <hip/hip_runtime.h>
#include "cfd_internal.hpp"
#include "physics.hpp"
#include "stage_common.hpp"
#include "chunks.hpp"

namespace cfd {

// ------------------------------------------------- simple per-cell stage kernel
template <typename T, bool VISC, int MODE>
__global__ void __launch_bounds__(256) k_stage_simple(StageArgs A, const BlockDesc* __restrict__ blocks,
                                                      const TileDesc* __restrict__ tiles, Gas<T> gas) {
  const int tx = threadIdx.x & 63, ty = threadIdx.x >> 6;
  const int nty = blockDim.x >> 6;
  for (int tile = blockIdx.x; tile < A.ntiles; tile += gridDim.x) {
    const TileDesc td = tiles[tile];
    const BlockDesc B = blocks[td.blk];
    const int i = td.i0 + tx;
    const int kend = min(td.k0 + A.tile_k, B.n[2]);
    const double* qb = A.qs + B.qoff;
    const double* mb = A.met + B.moff;
    const double* vb = VISC ? A.vmet + B.voff : nullptr;
    for (int j = td.j0 + ty; j < min(td.j0 + A.tile_j, B.n[1]); j += nty) {
      if (i >= B.n[0]) break;
      for (int k = td.k0; k < kend; ++k) {
        const int64_t c = (int64_t)(k + NG) * B.sk + (int64_t)(j + NG) * B.sj + (i + NG);
        double Fl[5], Fu[5], D[3][5];
        for (int d = 0; d < 3; ++d) {
          face_flux_global<T, VISC>(qb, mb, vb, B, c, d, gas, Fl);
          face_flux_global<T, VISC>(qb, mb, vb, B, c + dstride(d, B.sj, B.sk), d, gas, Fu);
          for (int q = 0; q < 5; ++q) D[d][q] = Fu[q] - Fl[q];
        }
        finish_cell<MODE>(A, B, c, D[0], D[1], D[2]);
      }
    }
  }
}

// ------------------------------------------------------------- time step
// dt_c = CFL V / (sum_d L_d + 4 sum_d Lv_d) with S_d averaged over the cell's
// two d-faces; per-workgroup partials: minimum dt (slot 12), sum V Q
// (slots 5-9) and the count of non-finite Q values (slot 11); local steps
// stored.
__global__ void __launch_bounds__(256) k_dt(const double* __restrict__ q, const double* __restrict__ met,
                                            double* __restrict__ dtcell, double* __restrict__ partials,
                                            const BlockDesc* __restrict__ blocks, int nblk, int64_t nchunks,
                                            StepParams P) {
  double acc[NPART];
  init_partials(acc);
  const int lane = threadIdx.x & 63;
  int64_t r0, r1;
  wave_rows(nchunks, r0, r1);
  ChunkWalk W;
  if (r0 < r1) W.start(blocks, nblk, r0);
  for (int64_t u = r0; u < r1; ++u) {
    int i, j, k;
    if (!W.cell(u, lane, i, j, k)) continue;
    const BlockDesc& B = W.B;
    const double* qb = q + B.qoff;
    const double* mb = met + B.moff;
    const int64_t c = (int64_t)(k + NG) * B.sk + (int64_t)(j + NG) * B.sj + (i + NG);
    const double qc[5] = {qb[c], qb[B.sv + c], qb[2 * B.sv + c], qb[3 * B.sv + c], qb[4 * B.sv + c]};
    const double vol = mb[9 * B.sv + c];
    const double dtc = cell_dt(qc, mb, c, B.sv, B.sj, B.sk, P);
    if (P.local_dt) dtcell[B.soff + c] = dtc;
    acc[12] = fmin(acc[12], dtc);
#pragma unroll
    for (int v = 0; v < 5; ++v) {
      acc[5 + v] += vol * qc[v];
      if (!finite(qc[v])) acc[11] += 1.0;
    }
  }
  wg_reduce_partials(acc, partials + (int64_t)blockIdx.x * NPART);
}

// ------------------------------------------------------------- norms
// Partials of sum R^2 (slots 0-4), max |R_rho| (10) and the non-finite count
// (11) of r, and of sum V Q (5-9) and the non-finite count of q; either of q
// (then met too) and r may be null.  Same cut of the grid as k_dt, so its
// sum V Q rows are bitwise k_dt's.
__global__ void __launch_bounds__(256) k_norms(const double* __restrict__ q, const double* __restrict__ r,
                                               const double* __restrict__ met, double* __restrict__ partials,
                                               const BlockDesc* __restrict__ blocks, int nblk, int64_t nchunks) {
  double acc[NPART];
  init_partials(acc);
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
    if (q) {
      double qv[5];
#pragma unroll
      for (int v = 0; v < 5; ++v) qv[v] = q[B.qoff + v * B.sv + c];
      const double vol = met[B.moff + 9 * B.sv + c];
#pragma unroll
      for (int v = 0; v < 5; ++v) {
        acc[5 + v] += vol * qv[v];
        if (!finite(qv[v])) acc[11] += 1.0;
      }
    }
    if (r) {
      double rv[5];
#pragma unroll
      for (int v = 0; v < 5; ++v) rv[v] = r[B.qoff + v * B.sv + c];
#pragma unroll
      for (int v = 0; v < 5; ++v) {
        acc[v] += rv[v] * rv[v];
        if (!finite(rv[v])) acc[11] += 1.0;
      }
      acc[10] = fmax(acc[10], fabs(rv[0]));
    }
  }
  wg_reduce_partials(acc, partials + (int64_t)blockIdx.x * NPART);
}

// ------------------------------------------------------------- finalize
// One workgroup of 256 threads: thread t combines rows t, t+256, ... in
// order, then a fixed-shape tree.  mode 0: dt only (min of slot 12 -> dt);
// mode 1: history row [dt, L2 x5, sum VQ x5, max|R_rho|] and nonfinite count.
__global__ void __launch_bounds__(256) k_finalize(const double* __restrict__ partials, int nrows,
                                                  int mode, double inv_ncells, double* __restrict__ dt,
                                                  double* __restrict__ hist, double* __restrict__ nonfinite) {
  __shared__ double sh[NPART][256];
  const int t = threadIdx.x;
  double acc[NPART];
  init_partials(acc);
  for (int row = t; row < nrows; row += 256) {
    const double* p = partials + (int64_t)row * NPART;
    for (int q = 0; q < NPART; ++q) {
      if (q == 10) acc[q] = fmax(acc[q], p[q]);
      else if (q == 12) acc[q] = fmin(acc[q], p[q]);
      else acc[q] += p[q];
    }
  }
  for (int q = 0; q < NPART; ++q) sh[q][t] = acc[q];
  __syncthreads();
  for (int s = 128; s > 0; s >>= 1) {
    if (t < s) {
      for (int q = 0; q < NPART; ++q) {
        if (q == 10) sh[q][t] = fmax(sh[q][t], sh[q][t + s]);
        else if (q == 12) sh[q][t] = fmin(sh[q][t], sh[q][t + s]);
        else sh[q][t] = sh[q][t] + sh[q][t + s];
      }
    }
    __syncthreads();
  }
  if (t == 0) {
    if (mode == 0) {
      dt[0] = sh[12][0];
    } else {
      hist[0] = dt ? dt[0] : 0.0;
      for (int q = 0; q < 5; ++q) hist[1 + q] = sqrt(sh[q][0] * inv_ncells);
      for (int q = 0; q < 5; ++q) hist[6 + q] = sh[5 + q][0];
      hist[11] = sh[10][0];
      if (nonfinite) nonfinite[0] = sh[11][0];
    }
  }
}

// ---------------------------------------------------------------- launchers

template <typename T, bool VISC, int MODE>
static void launch_simple_t(const StageArgs& A, const BlockDesc* blocks, const TileDesc* tiles,
                            const Gas<T>& gas, int nwg, hipStream_t s) {
  hipLaunchKernelGGL((k_stage_simple<T, VISC, MODE>), dim3(nwg), dim3(256), 0, s, A, blocks, tiles,
                     gas);
}

void launch_stage_simple(const StageArgs& A, int mode, bool visc, bool fp32, const BlockDesc* blocks,
                         const TileDesc* tiles, const Gas<double>& g64, const Gas<float>& g32, int nwg,
                         hipStream_t s) {
#define CFD_DISPATCH(T, G, V)                                                    \
  if (mode == 0) launch_simple_t<T, V, 0>(A, blocks, tiles, G, nwg, s);          \
  else if (mode == 1) launch_simple_t<T, V, 1>(A, blocks, tiles, G, nwg, s);     \
  else launch_simple_t<T, V, 2>(A, blocks, tiles, G, nwg, s);
  if (fp32) {
    if (visc) { CFD_DISPATCH(float, g32, true) } else { CFD_DISPATCH(float, g32, false) }
  } else {
    if (visc) { CFD_DISPATCH(double, g64, true) } else { CFD_DISPATCH(double, g64, false) }
  }
#undef CFD_DISPATCH
}

void launch_dt(const double* q, const double* met, double* dtcell, double* partials, const BlockDesc* blocks,
               int nblk, int64_t nchunks, const StepParams& P, int nwg, hipStream_t s) {
  hipLaunchKernelGGL(k_dt, dim3(nwg), dim3(256), 0, s, q, met, dtcell, partials, blocks, nblk, nchunks, P);
}

void launch_norms(const double* q, const double* r, const double* met, double* partials, const BlockDesc* blocks,
                  int nblk, int64_t nchunks, int nwg, hipStream_t s) {
  hipLaunchKernelGGL(k_norms, dim3(nwg), dim3(256), 0, s, q, r, met, partials, blocks, nblk, nchunks);
}

void launch_finalize(const double* partials, int nrows, int mode, double inv_ncells, double* dt,
                     double* hist, double* nonfinite, hipStream_t s) {
  hipLaunchKernelGGL(k_finalize, dim3(1), dim3(256), 0, s, partials, nrows, mode, inv_ncells, dt, hist,
                     nonfinite);
}

}  // namespace cfd
