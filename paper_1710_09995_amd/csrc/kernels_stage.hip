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
#include <hip/hip_runtime.h>
#include "cfd_internal.hpp"
#include "physics.hpp"

namespace cfd {

// ------------------------------------------------------------------ helpers

template <typename T>
__device__ __forceinline__ Prim<T> ld_prim(const double* __restrict__ qb, int64_t o, int64_t sv,
                                           T gm1) {
  return to_prim<T>(qb[o], qb[o + sv], qb[o + 2 * sv], qb[o + 3 * sv], qb[o + 4 * sv], gm1);
}

template <typename T>
__device__ __forceinline__ void ld_phi(const double* __restrict__ qb, int64_t o, int64_t sv, T gm1,
                                       T phi[4]) {
  Prim<T> W = ld_prim<T>(qb, o, sv, gm1);
  phi[0] = W.u;
  phi[1] = W.v;
  phi[2] = W.w;
  phi[3] = W.p / W.r;
}

__device__ __forceinline__ int64_t dstride(int d, int64_t sj, int64_t sk) {
  return d == 0 ? 1 : (d == 1 ? sj : sk);
}

// (F_inv - F_vis) . S on the lower d-face of the cell at offset c (relative to
// the block's padded origin), read straight from global memory.
template <typename T, bool VISC>
__device__ __forceinline__ void face_flux_global(const double* __restrict__ qb,
                                                 const double* __restrict__ mb, const BlockDesc& B,
                                                 int64_t c, int d, const Gas<T>& gas,
                                                 double F[5]) {
  const int64_t sd = dstride(d, B.sj, B.sk);
  const int64_t sv = B.sv;
  Prim<T> wm2 = ld_prim<T>(qb, c - 2 * sd, sv, gas.gm1);
  Prim<T> wm1 = ld_prim<T>(qb, c - sd, sv, gas.gm1);
  Prim<T> w0 = ld_prim<T>(qb, c, sv, gas.gm1);
  Prim<T> wp1 = ld_prim<T>(qb, c + sd, sv, gas.gm1);
  Prim<T> L, R;
  muscl(wm2, wm1, w0, wp1, gas.eps_lim, L, R);
  const double sx = mb[(3 * d) * sv + c], sy = mb[(3 * d + 1) * sv + c], sz = mb[(3 * d + 2) * sv + c];
  const double area = sqrt(sx * sx + sy * sy + sz * sz);
  const double ia = 1.0 / area;
  const T nx = (T)(sx * ia), ny = (T)(sy * ia), nz = (T)(sz * ia);
  T f[5];
  roe<T>(L, R, nx, ny, nz, gas.gamma, gas.eps_h, f);
  if (VISC) {
    const int64_t cl = c - sd;
    T pl[4], pr[4];
    pl[0] = wm1.u; pl[1] = wm1.v; pl[2] = wm1.w; pl[3] = wm1.p / wm1.r;
    pr[0] = w0.u; pr[1] = w0.v; pr[2] = w0.w; pr[3] = w0.p / w0.r;
    T dd[2][4];
    double St[2][3];
    int tt = 0;
    for (int t = 0; t < 3; ++t) {
      if (t == d) continue;
      const int64_t st = dstride(t, B.sj, B.sk);
      T a[4], b[4], e[4], f4[4];
      ld_phi<T>(qb, cl + st, sv, gas.gm1, a);
      ld_phi<T>(qb, c + st, sv, gas.gm1, b);
      ld_phi<T>(qb, cl - st, sv, gas.gm1, e);
      ld_phi<T>(qb, c - st, sv, gas.gm1, f4);
      for (int q = 0; q < 4; ++q) dd[tt][q] = T(0.25) * (a[q] + b[q] - e[q] - f4[q]);
      for (int x = 0; x < 3; ++x) {
        const int64_t mo = (int64_t)(3 * t + x) * sv;
        St[tt][x] = 0.25 * (mb[mo + cl] + mb[mo + cl + st] + mb[mo + c] + mb[mo + c + st]);
      }
      ++tt;
    }
    const double vf = 0.5 * (mb[9 * sv + cl] + mb[9 * sv + c]);
    const double iv = 1.0 / vf;
    const T sdx = (T)(sx * iv), sdy = (T)(sy * iv), sdz = (T)(sz * iv);
    const T s1x = (T)(St[0][0] * iv), s1y = (T)(St[0][1] * iv), s1z = (T)(St[0][2] * iv);
    const T s2x = (T)(St[1][0] * iv), s2y = (T)(St[1][1] * iv), s2z = (T)(St[1][2] * iv);
    T g[4][3];
    for (int q = 0; q < 4; ++q) {
      const T dq = pr[q] - pl[q];
      g[q][0] = dq * sdx + dd[0][q] * s1x + dd[1][q] * s2x;
      g[q][1] = dq * sdy + dd[0][q] * s1y + dd[1][q] * s2y;
      g[q][2] = dq * sdz + dd[0][q] * s1z + dd[1][q] * s2z;
    }
    T uf[3] = {T(0.5) * (pl[0] + pr[0]), T(0.5) * (pl[1] + pr[1]), T(0.5) * (pl[2] + pr[2])};
    const T tf = T(0.5) * (pl[3] + pr[3]);
    T fv[5];
    viscous_n<T>(g, uf, tf, nx, ny, nz, gas, fv);
    for (int q = 0; q < 5; ++q) f[q] -= fv[q];
  }
  for (int q = 0; q < 5; ++q) F[q] = (double)f[q] * area;
}

// Fixed-order workgroup reduction of NPART partials; thread 0 writes the row.
// op: sums for [0,10), max for 10, sum for 11 (count), min for 12.
__device__ __forceinline__ void wg_reduce_partials(double acc[NPART], double* __restrict__ out_row) {
  __shared__ double red[NPART][16];
  const int lane = threadIdx.x & 63;
  const int wave = threadIdx.x >> 6;
  const int nwave = (blockDim.x + 63) >> 6;
#pragma unroll
  for (int q = 0; q < NPART; ++q) {
    double v = acc[q];
    for (int off = 32; off > 0; off >>= 1) {
      double o = __shfl_xor(v, off, 64);
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

__device__ __forceinline__ void init_partials(double acc[NPART]) {
#pragma unroll
  for (int q = 0; q < NPART; ++q) acc[q] = 0.0;
  acc[12] = __builtin_inf();
}

__device__ __forceinline__ bool finite(double x) { return !(isnan(x) || isinf(x)); }

// ------------------------------------------------- simple per-cell stage kernel
// MODE 0: write R; MODE 1: stage 1 (+ norm partials of R(Qn), V Qn);
// MODE 2: stages 2-3 with coefficients (a, b).
template <typename T, bool VISC, int MODE>
__global__ void __launch_bounds__(256) k_stage_simple(StageArgs A, const BlockDesc* __restrict__ blocks,
                                                      const TileDesc* __restrict__ tiles, Gas<T> gas) {
  double acc[NPART];
  init_partials(acc);
  const int tx = threadIdx.x & 63, ty = threadIdx.x >> 6;
  const int nty = blockDim.x >> 6;
  for (int tile = blockIdx.x; tile < A.ntiles; tile += gridDim.x) {
    const TileDesc td = tiles[tile];
    const BlockDesc B = blocks[td.blk];
    const int i = td.i0 + tx;
    const int kend = min(td.k0 + A.tile_k, B.n[2]);
    const double* qb = A.qs + B.qoff;
    const double* mb = A.met + B.moff;
    for (int j = td.j0 + ty; j < min(td.j0 + A.tile_j, B.n[1]); j += nty) {
      if (i >= B.n[0]) break;
      for (int k = td.k0; k < kend; ++k) {
        const int64_t c = (int64_t)(k + NG) * B.sk + (int64_t)(j + NG) * B.sj + (i + NG);
        double Fl[5], Fu[5], D[3][5];
        for (int d = 0; d < 3; ++d) {
          face_flux_global<T, VISC>(qb, mb, B, c, d, gas, Fl);
          face_flux_global<T, VISC>(qb, mb, B, c + dstride(d, B.sj, B.sk), d, gas, Fu);
          for (int q = 0; q < 5; ++q) D[d][q] = Fu[q] - Fl[q];
        }
        const double vol = mb[9 * B.sv + c];
        double R[5];
        for (int q = 0; q < 5; ++q) R[q] = ((D[0][q] + D[1][q]) + D[2][q]) / vol;
        if (MODE == 0) {
          for (int q = 0; q < 5; ++q) A.out[B.qoff + q * B.sv + c] = R[q];
          continue;
        }
        const double dt = A.local_dt ? A.dt[B.soff + c] : A.dt[0];
        if (MODE == 1) {
          for (int q = 0; q < 5; ++q) {
            const double qv = qb[q * B.sv + c];
            A.out[B.qoff + q * B.sv + c] = qv - dt * R[q];
            acc[q] += R[q] * R[q];
            acc[5 + q] += vol * qv;
            if (!finite(qv) || !finite(R[q])) acc[11] += 1.0;
          }
          acc[10] = fmax(acc[10], fabs(R[0]));
        } else {
          const double* qnb = A.qn + B.qoff;
          for (int q = 0; q < 5; ++q) {
            const double qv = qb[q * B.sv + c];
            A.out[B.qoff + q * B.sv + c] = A.a * qnb[q * B.sv + c] + A.b * (qv - dt * R[q]);
          }
        }
      }
    }
  }
  if (MODE == 1) wg_reduce_partials(acc, A.partials + (int64_t)blockIdx.x * NPART);
}

// ------------------------------------------------------------- time step
// dt_c = CFL V / (sum_d L_d + 4 sum_d Lv_d) with S_d averaged over the cell's
// two d-faces; per-workgroup minimum partial (slot 12); local steps stored.
__global__ void __launch_bounds__(256) k_dt(const double* __restrict__ q, const double* __restrict__ met,
                                            double* __restrict__ dtcell, double* __restrict__ partials,
                                            const BlockDesc* __restrict__ blocks,
                                            const TileDesc* __restrict__ tiles, int ntiles, int tile_j,
                                            int tile_k, StepParams P) {
  double acc[NPART];
  init_partials(acc);
  const int tx = threadIdx.x & 63, ty = threadIdx.x >> 6;
  const int nty = blockDim.x >> 6;
  const double gm1 = P.gamma - 1.0;
  const double coefv = fmax(4.0 / 3.0, P.gamma / P.prandtl);
  for (int tile = blockIdx.x; tile < ntiles; tile += gridDim.x) {
    const TileDesc td = tiles[tile];
    const BlockDesc B = blocks[td.blk];
    const int i = td.i0 + tx;
    if (i >= B.n[0]) continue;
    const double* qb = q + B.qoff;
    const double* mb = met + B.moff;
    for (int j = td.j0 + ty; j < min(td.j0 + tile_j, B.n[1]); j += nty) {
      for (int k = td.k0; k < min(td.k0 + tile_k, B.n[2]); ++k) {
        const int64_t c = (int64_t)(k + NG) * B.sk + (int64_t)(j + NG) * B.sj + (i + NG);
        const double r = qb[c];
        const double inv = 1.0 / r;
        const double u = qb[B.sv + c] * inv, v = qb[2 * B.sv + c] * inv, w = qb[3 * B.sv + c] * inv;
        const double p = gm1 * (qb[4 * B.sv + c] - 0.5 * r * (u * u + v * v + w * w));
        const double cs = sqrt(P.gamma * p / r);
        const double vol = mb[9 * B.sv + c];
        double lam = 0.0, lamv = 0.0;
        double mu_r = 0.0;
        if (P.viscous) {
          const double t = p / r;
          mu_r = P.mu_inf * t * sqrt(t) * (1.0 + P.s_star) / (t + P.s_star) / r;
        }
        for (int d = 0; d < 3; ++d) {
          const int64_t sd = dstride(d, B.sj, B.sk);
          const double bx = 0.5 * (mb[(3 * d) * B.sv + c] + mb[(3 * d) * B.sv + c + sd]);
          const double by = 0.5 * (mb[(3 * d + 1) * B.sv + c] + mb[(3 * d + 1) * B.sv + c + sd]);
          const double bz = 0.5 * (mb[(3 * d + 2) * B.sv + c] + mb[(3 * d + 2) * B.sv + c + sd]);
          const double mag = sqrt(bx * bx + by * by + bz * bz);
          lam += fabs(u * bx + v * by + w * bz) + cs * mag;
          if (P.viscous) lamv += coefv * mu_r * mag * mag / vol;
        }
        const double dtc = P.cfl * vol / (lam + 4.0 * lamv);
        if (P.local_dt) dtcell[B.soff + c] = dtc;
        acc[12] = fmin(acc[12], dtc);
      }
    }
  }
  wg_reduce_partials(acc, partials + (int64_t)blockIdx.x * NPART);
}

// ------------------------------------------------------------- norms only
__global__ void __launch_bounds__(256) k_norms(const double* __restrict__ q, const double* __restrict__ r,
                                               const double* __restrict__ met, double* __restrict__ partials,
                                               const BlockDesc* __restrict__ blocks,
                                               const TileDesc* __restrict__ tiles, int ntiles, int tile_j,
                                               int tile_k) {
  double acc[NPART];
  init_partials(acc);
  const int tx = threadIdx.x & 63, ty = threadIdx.x >> 6;
  const int nty = blockDim.x >> 6;
  for (int tile = blockIdx.x; tile < ntiles; tile += gridDim.x) {
    const TileDesc td = tiles[tile];
    const BlockDesc B = blocks[td.blk];
    const int i = td.i0 + tx;
    if (i >= B.n[0]) continue;
    for (int j = td.j0 + ty; j < min(td.j0 + tile_j, B.n[1]); j += nty) {
      for (int k = td.k0; k < min(td.k0 + tile_k, B.n[2]); ++k) {
        const int64_t c = (int64_t)(k + NG) * B.sk + (int64_t)(j + NG) * B.sj + (i + NG);
        const double vol = met[B.moff + 9 * B.sv + c];
        for (int v = 0; v < 5; ++v) {
          const double qv = q[B.qoff + v * B.sv + c];
          acc[5 + v] += vol * qv;
          if (!finite(qv)) acc[11] += 1.0;
          if (r) {
            const double rv = r[B.qoff + v * B.sv + c];
            acc[v] += rv * rv;
            if (!finite(rv)) acc[11] += 1.0;
            if (v == 0) acc[10] = fmax(acc[10], fabs(rv));
          }
        }
      }
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

void launch_dt(const double* q, const double* met, double* dtcell, double* partials,
               const BlockDesc* blocks, const TileDesc* tiles, int ntiles, int tile_j, int tile_k,
               const StepParams& P, int nwg, hipStream_t s) {
  hipLaunchKernelGGL(k_dt, dim3(nwg), dim3(256), 0, s, q, met, dtcell, partials, blocks, tiles, ntiles,
                     tile_j, tile_k, P);
}

void launch_norms(const double* q, const double* r, const double* met, double* partials,
                  const BlockDesc* blocks, const TileDesc* tiles, int ntiles, int tile_j, int tile_k,
                  int nwg, hipStream_t s) {
  hipLaunchKernelGGL(k_norms, dim3(nwg), dim3(256), 0, s, q, r, met, partials, blocks, tiles, ntiles,
                     tile_j, tile_k);
}

void launch_finalize(const double* partials, int nrows, int mode, double inv_ncells, double* dt,
                     double* hist, double* nonfinite, hipStream_t s) {
  hipLaunchKernelGGL(k_finalize, dim3(1), dim3(256), 0, s, partials, nrows, mode, inv_ncells, dt, hist,
                     nonfinite);
}

}  // namespace cfd
