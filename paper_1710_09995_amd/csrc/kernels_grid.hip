// Grid kernels: padded node copy, ghost nodes, metrics (face vectors and
// volumes), metric ghost copy across connections, and the per-stage ghost
// fill of the conserved state.
//
// Every kernel here is HBM-bound index work (copies and a few flops per
// element).  Patch kernels run one launch per sweep direction over all
// patches of all blocks: grid.y = patch, grid.x covers the patch's
// transverse points, each thread handles all g ghost layers of its point.
#include <hip/hip_runtime.h>
#include "cfd_internal.hpp"
#include "physics.hpp"
#include "stage_common.hpp"

namespace cfd {

__device__ __forceinline__ int64_t stride_of(int d, int64_t sj, int64_t sk) {
  return d == 0 ? 1 : (d == 1 ? sj : sk);
}

// Offset (relative to the padded origin) of logical index (a along d, p1
// along t1, p2 along t2) with t1 < t2 the transverse directions.
__device__ __forceinline__ int64_t pos3(int d, int a, int p1, int p2, int64_t sj, int64_t sk) {
  int i, j, k;
  if (d == 0) { i = a; j = p1; k = p2; }
  else if (d == 1) { j = a; i = p1; k = p2; }
  else { k = a; i = p1; j = p2; }
  return (int64_t)(k + NG) * sk + (int64_t)(j + NG) * sj + (i + NG);
}

__global__ void k_copy_nodes(const double* __restrict__ src, double* __restrict__ x, BlockDesc B) {
  const int ni = B.n[0], nj = B.n[1], nk = B.n[2];
  const int64_t total = (int64_t)3 * (nk + 1) * (nj + 1) * (ni + 1);
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < total;
       e += (int64_t)gridDim.x * blockDim.x) {
    int64_t r = e;
    int i = r % (ni + 1); r /= (ni + 1);
    int j = r % (nj + 1); r /= (nj + 1);
    int k = r % (nk + 1);
    int c = (int)(r / (nk + 1));
    x[B.xoff + c * B.xsv + (int64_t)(k + NG) * B.xsk + (int64_t)(j + NG) * B.xsj + (i + NG)] = src[e];
  }
}

// Ghost nodes of one sweep: connections copy the neighbour's node plus the
// shift; physical faces extrapolate linearly, x_{-m} = x_0 + m (x_0 - x_1).
__global__ void k_ghost_nodes(double* __restrict__ x, const BlockDesc* __restrict__ blocks,
                              const PatchDesc* __restrict__ patches) {
  const PatchDesc P = patches[blockIdx.y];
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= P.count) return;
  const int d = P.face >> 1, side = P.face & 1;
  const int t1 = d == 0 ? 1 : 0, t2 = d == 2 ? 1 : 2;
  const int w1 = P.hi[t1] - P.lo[t1];
  const int p1 = P.lo[t1] + t % w1, p2 = P.lo[t2] + t / w1;
  const BlockDesc B = blocks[P.blk];
  const int n = B.n[d];
  double* xb = x + B.xoff;
  if (P.kind == 0) {
    const BlockDesc N = blocks[P.nbr];
    const double* xn = x + N.xoff;
    const int nn = N.n[d];
    for (int m = 1; m <= NG; ++m) {
      const int gm = side == 0 ? -m : n + m;
      const int sm = side == 0 ? nn - m : m;
      const int64_t od = pos3(d, gm, p1, p2, B.xsj, B.xsk);
      const int64_t os = pos3(d, sm, p1 + P.noff[t1], p2 + P.noff[t2], N.xsj, N.xsk);
      for (int c = 0; c < 3; ++c) xb[c * B.xsv + od] = xn[c * N.xsv + os] + P.shift[c];
    }
  } else {
    const int a0 = side == 0 ? 0 : n, a1 = side == 0 ? 1 : n - 1;
    const int64_t o0 = pos3(d, a0, p1, p2, B.xsj, B.xsk);
    const int64_t o1 = pos3(d, a1, p1, p2, B.xsj, B.xsk);
    for (int m = 1; m <= NG; ++m) {
      const int gm = side == 0 ? -m : n + m;
      const int64_t od = pos3(d, gm, p1, p2, B.xsj, B.xsk);
      for (int c = 0; c < 3; ++c) {
        const double v0 = xb[c * B.xsv + o0], v1 = xb[c * B.xsv + o1];
        xb[c * B.xsv + od] = v0 + (double)m * (v0 - v1);
      }
    }
  }
}

struct V3 {
  double x, y, z;
};
__device__ __forceinline__ V3 sub(V3 a, V3 b) { return {a.x - b.x, a.y - b.y, a.z - b.z}; }
__device__ __forceinline__ V3 cross(V3 a, V3 b) {
  return {a.y * b.z - a.z * b.y, a.z * b.x - a.x * b.z, a.x * b.y - a.y * b.x};
}
__device__ __forceinline__ double dot(V3 a, V3 b) { return a.x * b.x + a.y * b.y + a.z * b.z; }

// Face vector of the d-face whose lowest node is at offset o (relative to a
// local origin x0): S = 1/2 (x[+t1+t2] - x[0]) x (x[+t2] - x[+t1]), with
// (t1, t2) cyclic after d.  Also returns the face's mean node position.
__device__ __forceinline__ void face_vec(const double* xb, const BlockDesc& B, int64_t o, int d,
                                         V3 x0, V3& S, V3& C) {
  const int c1 = (d + 1) % 3, c2 = (d + 2) % 3;
  const int64_t s1 = stride_of(c1, B.xsj, B.xsk), s2 = stride_of(c2, B.xsj, B.xsk);
  auto ld = [&](int64_t off) {
    V3 v = {xb[off], xb[B.xsv + off], xb[2 * B.xsv + off]};
    return sub(v, x0);
  };
  V3 p0 = ld(o), p1 = ld(o + s1), p2 = ld(o + s2), p12 = ld(o + s1 + s2);
  V3 a = sub(p12, p0), b = sub(p2, p1);
  V3 cr = cross(a, b);
  S = {0.5 * cr.x, 0.5 * cr.y, 0.5 * cr.z};
  C = {0.25 * (p0.x + p1.x + p2.x + p12.x), 0.25 * (p0.y + p1.y + p2.y + p12.y),
       0.25 * (p0.z + p1.z + p2.z + p12.z)};
}

// Metrics of every padded cell of one block: lower-face vectors S_i, S_j, S_k
// and the volume V = 1/3 sum_faces (face centre - x_c) . S_out, measured from
// the cell's lowest node x_c (the divergence theorem is origin-free; a local
// origin avoids cancellation on large coordinates).
__global__ void k_metrics(const double* __restrict__ x, double* __restrict__ met, BlockDesc B) {
  const int pi = B.n[0] + 2 * NG, pj = B.n[1] + 2 * NG, pk = B.n[2] + 2 * NG;
  const int64_t total = (int64_t)pi * pj * pk;
  const double* xb = x + B.xoff;
  double* mb = met + B.moff;
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < total;
       e += (int64_t)gridDim.x * blockDim.x) {
    const int ii = e % pi, jj = (e / pi) % pj, kk = (int)(e / ((int64_t)pi * pj));
    const int64_t o = (int64_t)kk * B.xsk + (int64_t)jj * B.xsj + ii;   // node at the cell's low corner
    const V3 x0 = {xb[o], xb[B.xsv + o], xb[2 * B.xsv + o]};
    const int64_t co = (int64_t)kk * B.sk + (int64_t)jj * B.sj + ii;
    double vol = 0.0;
    for (int d = 0; d < 3; ++d) {
      V3 Sl, Cl, Su, Cu;
      face_vec(xb, B, o, d, x0, Sl, Cl);
      face_vec(xb, B, o + stride_of(d, B.xsj, B.xsk), d, x0, Su, Cu);
      mb[(3 * d + 0) * B.sv + co] = Sl.x;
      mb[(3 * d + 1) * B.sv + co] = Sl.y;
      mb[(3 * d + 2) * B.sv + co] = Sl.z;
      vol += dot(Cu, Su) - dot(Cl, Sl);
    }
    mb[9 * B.sv + co] = vol / 3.0;
  }
}

// Metric ghost copy across connections (one sweep).  The seam face vector of
// the lower block becomes the upper block's own, so both see the same bits.
__global__ void k_metric_ghosts(double* __restrict__ met, const BlockDesc* __restrict__ blocks,
                                const PatchDesc* __restrict__ patches) {
  const PatchDesc P = patches[blockIdx.y];
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= P.count || P.kind != 0) return;
  const int d = P.face >> 1, side = P.face & 1;
  const int t1 = d == 0 ? 1 : 0, t2 = d == 2 ? 1 : 2;
  const int w1 = P.hi[t1] - P.lo[t1];
  const int p1 = P.lo[t1] + t % w1, p2 = P.lo[t2] + t / w1;
  const BlockDesc B = blocks[P.blk];
  const BlockDesc N = blocks[P.nbr];
  const int n = B.n[d], nn = N.n[d];
  for (int m = 1; m <= NG; ++m) {
    const int gm = side == 0 ? -m : n - 1 + m;
    const int sm = side == 0 ? nn - m : m - 1;
    const int64_t od = pos3(d, gm, p1, p2, B.sj, B.sk);
    const int64_t os = pos3(d, sm, p1 + P.noff[t1], p2 + P.noff[t2], N.sj, N.sk);
    for (int c = 0; c < NM; ++c) met[B.moff + c * B.sv + od] = met[N.moff + c * N.sv + os];
  }
}

// Ghost fill of the conserved state (one sweep, all patches of all blocks).
// One thread per transverse point, except on i-faces: there the NG ghost
// cells of a row are adjacent in memory while neighbouring points are a row
// apart, so a thread per (point, layer) puts a row's layers on adjacent lanes
// and halves the memory segments each access touches.
// With delta set, q is an update (the implicit step's dQ): connections copy it
// as they copy the state, and the ghost cells of physical patches get zero.
__global__ void k_ghost_q(double* __restrict__ q, const double* __restrict__ met,
                          const BlockDesc* __restrict__ blocks,
                          const PatchDesc* __restrict__ patches, StepParams SP, int delta) {
  const PatchDesc& P = patches[blockIdx.y];
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  const int d = P.face >> 1, side = P.face & 1;
  const int per = ghost_threads_per_point(P.kind, d);
  if (t >= P.count * per) return;
  const int pt = t / per;
  // transverse directions t1 < t2, selected without indexing (keeps P out of scratch)
  const int lo1 = d == 0 ? P.lo[1] : P.lo[0], hi1 = d == 0 ? P.hi[1] : P.hi[0];
  const int lo2 = d == 2 ? P.lo[1] : P.lo[2];
  const int w1 = hi1 - lo1;
  const int p1 = lo1 + pt % w1, p2 = lo2 + pt / w1;
  const BlockDesc& B = blocks[P.blk];
  const int n = d == 0 ? B.n[0] : (d == 1 ? B.n[1] : B.n[2]);
  double* qb = q + B.qoff;
  if (P.kind == 0) {
    const BlockDesc& N = blocks[P.nbr];
    const double* qn = q + N.qoff;
    const int nn = d == 0 ? N.n[0] : (d == 1 ? N.n[1] : N.n[2]);
    const int o1 = d == 0 ? P.noff[1] : P.noff[0], o2 = d == 2 ? P.noff[1] : P.noff[2];
    // Every load before the first store: source and destination share one
    // arena, so a load issued after a store would wait for it.
    if (per != 1) {     // this thread's layer only
      const int m = 1 + t % per;
      const int64_t od = pos3(d, side == 0 ? -m : n - 1 + m, p1, p2, B.sj, B.sk);
      const int64_t os = pos3(d, side == 0 ? nn - m : m - 1, p1 + o1, p2 + o2, N.sj, N.sk);
      double val[NV];
      for (int v = 0; v < NV; ++v) val[v] = qn[v * N.sv + os];
      for (int v = 0; v < NV; ++v) qb[v * B.sv + od] = val[v];
      return;
    }
    double val[NG][NV];
    int64_t od[NG];
    for (int m = 1; m <= NG; ++m) {
      const int gm = side == 0 ? -m : n - 1 + m;
      const int sm = side == 0 ? nn - m : m - 1;
      od[m - 1] = pos3(d, gm, p1, p2, B.sj, B.sk);
      const int64_t os = pos3(d, sm, p1 + o1, p2 + o2, N.sj, N.sk);
      for (int v = 0; v < NV; ++v) val[m - 1][v] = qn[v * N.sv + os];
    }
    for (int m = 0; m < NG; ++m)
      for (int v = 0; v < NV; ++v) qb[v * B.sv + od[m]] = val[m][v];
    return;
  }
  if (delta) {
    if (per != 1) {     // this thread's layer only
      const int m = 1 + t % per;
      const int64_t od = pos3(d, side == 0 ? -m : n - 1 + m, p1, p2, B.sj, B.sk);
      for (int v = 0; v < NV; ++v) qb[v * B.sv + od] = 0.0;
      return;
    }
    for (int m = 1; m <= NG; ++m) {
      const int64_t od = pos3(d, side == 0 ? -m : n - 1 + m, p1, p2, B.sj, B.sk);
      for (int v = 0; v < NV; ++v) qb[v * B.sv + od] = 0.0;
    }
    return;
  }
  // boundary face vector at this transverse position
  const int fa = side == 0 ? 0 : n;
  const int64_t of = pos3(d, fa, p1, p2, B.sj, B.sk);
  const double* mb = met + B.moff;
  const double sx = mb[(3 * d) * B.sv + of], sy = mb[(3 * d + 1) * B.sv + of],
               sz = mb[(3 * d + 2) * B.sv + of];
  const double nrm = sqrt(sx * sx + sy * sy + sz * sz);
  const double nx = sx / nrm, ny = sy / nrm, nz = sz / nrm;
  const int a0 = side == 0 ? 0 : n - 1;
  if (P.kind == CFD_BC_KIND_FARFIELD || P.kind == CFD_BC_KIND_EXTRAP) {
    const int64_t o0 = pos3(d, a0, p1, p2, B.sj, B.sk);
    double qi[5], qg[5];
    for (int v = 0; v < NV; ++v) qi[v] = qb[v * B.sv + o0];
    if (P.kind == CFD_BC_KIND_FARFIELD) {
      const double s = side == 0 ? -1.0 : 1.0;
      farfield_state(qi, s * nx, s * ny, s * nz, SP.gamma, P.uinf, qg);
    } else {
      for (int v = 0; v < NV; ++v) qg[v] = qi[v];
    }
    if (per != 1) {     // this thread's layer only
      const int m = 1 + t % per;
      const int64_t od = pos3(d, side == 0 ? -m : n - 1 + m, p1, p2, B.sj, B.sk);
      for (int v = 0; v < NV; ++v) qb[v * B.sv + od] = qg[v];
      return;
    }
    for (int m = 1; m <= NG; ++m) {
      const int gm = side == 0 ? -m : n - 1 + m;
      const int64_t od = pos3(d, gm, p1, p2, B.sj, B.sk);
      for (int v = 0; v < NV; ++v) qb[v * B.sv + od] = qg[v];
    }
    return;
  }
  // walls: ghost layer m mirrors interior cell m - 1
  auto wall = [&](const double w[NV], int64_t od) {
    const double mx = w[1], my = w[2], mz = w[3];
    double gx, gy, gz;
    if (P.kind == CFD_BC_KIND_SLIPWALL) {
      const double mn = mx * nx + my * ny + mz * nz;
      gx = mx - 2.0 * mn * nx;
      gy = my - 2.0 * mn * ny;
      gz = mz - 2.0 * mn * nz;
    } else {  // no-slip adiabatic
      gx = -mx;
      gy = -my;
      gz = -mz;
    }
    qb[od] = w[0];
    qb[B.sv + od] = gx;
    qb[2 * B.sv + od] = gy;
    qb[3 * B.sv + od] = gz;
    qb[4 * B.sv + od] = w[4];
  };
  if (per != 1) {       // this thread's layer only
    const int m = 1 + t % per;
    const int64_t oi = pos3(d, side == 0 ? m - 1 : n - m, p1, p2, B.sj, B.sk);
    double w[NV];
    for (int v = 0; v < NV; ++v) w[v] = qb[v * B.sv + oi];
    wall(w, pos3(d, side == 0 ? -m : n - 1 + m, p1, p2, B.sj, B.sk));
    return;
  }
  double wv[NG][NV];       // the mirrored interior cells, all loaded before any store
  for (int m = 1; m <= NG; ++m) {
    const int im = side == 0 ? m - 1 : n - m;
    const int64_t oi = pos3(d, im, p1, p2, B.sj, B.sk);
    for (int v = 0; v < NV; ++v) wv[m - 1][v] = qb[v * B.sv + oi];
  }
  for (int m = 1; m <= NG; ++m) wall(wv[m - 1], pos3(d, side == 0 ? -m : n - 1 + m, p1, p2, B.sj, B.sk));
}

// Viscous face metrics of one block: for every cell position (i, j, k) in
// [0, n]^3 and direction d, the terms of its lower d-face (see visc_metrics).
__global__ void k_visc_metrics(const double* __restrict__ met, double* __restrict__ vmet, BlockDesc B) {
  const int64_t wi = B.n[0] + 1, wj = B.n[1] + 1, total = wi * wj * (B.n[2] + 1);
  for (int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; t < total; t += (int64_t)gridDim.x * blockDim.x) {
    const int i = (int)(t % wi), j = (int)((t / wi) % wj), k = (int)(t / (wi * wj));
    const int64_t c = (int64_t)(k + NG) * B.sk + (int64_t)(j + NG) * B.sj + (i + NG);
    const double* mb = met + B.moff;
    double* vb = vmet + B.voff;
    for (int d = 0; d < 3; ++d) {
      double St[2][3], vf;
      visc_metrics(mb, B.sv, c - dstride(d, B.sj, B.sk), c, d, B.sj, B.sk, St, vf);
      for (int u = 0; u < 2; ++u)
        for (int x = 0; x < 3; ++x) vb[(int64_t)(7 * d + 3 * u + x) * B.sv + c] = St[u][x];
      vb[(int64_t)(7 * d + 6) * B.sv + c] = vf;
    }
  }
}

// ---------------------------------------------------------------- launchers

void launch_visc_metrics(const double* met, double* vmet, const BlockDesc& B, hipStream_t s) {
  const int64_t total = (int64_t)(B.n[0] + 1) * (B.n[1] + 1) * (B.n[2] + 1);
  int64_t nb = (total + 255) / 256;
  if (nb > 65535) nb = 65535;
  hipLaunchKernelGGL(k_visc_metrics, dim3((unsigned)nb), dim3(256), 0, s, met, vmet, B);
}

void launch_copy_nodes(const double* src, double* x, const BlockDesc& B, hipStream_t s) {
  const int64_t total = (int64_t)3 * (B.n[0] + 1) * (B.n[1] + 1) * (B.n[2] + 1);
  int64_t nb = (total + 255) / 256;
  if (nb > 65535) nb = 65535;
  hipLaunchKernelGGL(k_copy_nodes, dim3((unsigned)nb), dim3(256), 0, s, src, x, B);
}

void launch_ghost_nodes(double* x, const BlockDesc* blocks, const PatchDesc* patches, int npatch,
                        int maxcount, hipStream_t s) {
  if (npatch == 0) return;
  hipLaunchKernelGGL(k_ghost_nodes, dim3((maxcount + 127) / 128, npatch), dim3(128), 0, s, x,
                     blocks, patches);
}

void launch_metrics(const double* x, double* met, const BlockDesc& B, hipStream_t s) {
  const int64_t total = (int64_t)(B.n[0] + 2 * NG) * (B.n[1] + 2 * NG) * (B.n[2] + 2 * NG);
  int64_t nb = (total + 255) / 256;
  if (nb > 65535) nb = 65535;
  hipLaunchKernelGGL(k_metrics, dim3((unsigned)nb), dim3(256), 0, s, x, met, B);
}

void launch_metric_ghosts(double* met, const BlockDesc* blocks, const PatchDesc* patches,
                          int npatch, int maxcount, hipStream_t s) {
  if (npatch == 0) return;
  hipLaunchKernelGGL(k_metric_ghosts, dim3((maxcount + 127) / 128, npatch), dim3(128), 0, s, met,
                     blocks, patches);
}

void launch_ghost_q(double* q, const double* met, const BlockDesc* blocks,
                    const PatchDesc* patches, int npatch, int nthreads, const StepParams& SP,
                    hipStream_t s, int delta) {
  if (npatch == 0) return;
  hipLaunchKernelGGL(k_ghost_q, dim3((nthreads + 127) / 128, npatch), dim3(128), 0, s, q, met,
                     blocks, patches, SP, delta);
}

}  // namespace cfd
