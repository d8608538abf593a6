// Plane-ring face-once residual / stage kernel (64 x 8 or 64 x 4 tiles).
//
// Same tile decomposition and per-face arithmetic as the tiled kernel, with a
// different plane pipeline.  LDS holds a ring of three primitive planes
// W(k-1), W(k), W(k+1), each with a halo of 2 cells (rho, u, v, w, p [, T]).
// The viscous face gradients take phi = (u, v, w, T) of the neighbouring
// planes straight from the ring, so every plane is loaded and converted once
// and no separate phi planes are kept or copied.
//
// Per k-plane, two barriers:
//   A. faces of plane k (W(k-1..k+1) ready): the lower i-face and lower
//      j-face of every column, the tile-edge faces, the upper k-face (cells
//      k-1..k+1 from the ring, k+2 from a one-cell register queue);
//   B. after the barrier: the cell update of plane k (its inputs were loaded
//      before the faces) together with the fill of W(k+2) into the slot of
//      W(k-1) and the queue load of W(k+3), so their memory latencies overlap.
// Stage 1 accumulates the norm partials of R(Qn) in registers (this kernel
// has the register room) instead of writing R for a separate norms kernel
// (the totals sum V Qn come from a row-chunk kernel whose cut of the grid
// does not depend on the tiles), and stage 3 (mode 3) evaluates the CFL time
// step of the state it writes (the next step's), instead of a separate
// time-step kernel.
// The i-face fluxes are exchanged between neighbouring lanes of the wave
// (shuffle) instead of through LDS; only the tile's edge i-faces and the
// j-faces go through LDS.  Every face flux gets the same bits as in the
// other stage kernels (same primitives, same expressions).
#include <hip/hip_runtime.h>
#include "cfd_internal.hpp"
#include "physics.hpp"
#include "stage_common.hpp"

// Scheduling fence between face computations (register pressure), as in the
// tiled kernel.
#define CFD_FACE_FENCE_RING() __builtin_amdgcn_sched_barrier(0)

namespace cfd {

template <typename T, bool VISC, int TJ_>
struct RingLds {
  static constexpr int TJ = TJ_;
  static constexpr int WI = 68, WJ = TJ + 4;   // halo 2
  static constexpr int NW = VISC ? 6 : 5;
  static constexpr int PLANE = NW * WJ * WI;   // elements of one plane
  static constexpr int W_BYTES = (3 * PLANE * (int)sizeof(T) + 15) / 16 * 16;
  static constexpr int FJ = 5 * (TJ + 1) * 64;  // doubles: lower j-faces, TJ+1 rows
  static constexpr int FE = 5 * TJ;             // doubles: i-faces at i0+64
  static constexpr int TOTAL = W_BYTES + (FJ + FE) * 8;
  // stage 3 also keeps the area vectors of those faces for the time step
  static constexpr int SJ = 3 * (TJ + 1) * 64;  // doubles: S_j of the lower j-faces
  static constexpr int SE = 3 * TJ;             // doubles: S_i at i0+64
  static constexpr int TOTAL_DT = TOTAL + (SJ + SE) * 8;
};

// Minimum waves per SIMD asked of the register allocator: the FP32 Euler
// variants fit 128 VGPRs (4 waves per SIMD; LDS allows two 64x8 or three
// 64x4 workgroups per CU), the others take what they need.
template <typename T, bool VISC>
constexpr int ring_min_waves() {
  return (sizeof(T) == 4 && !VISC) ? 4 : 1;
}

template <typename T, bool VISC, int MODE, int TJ>
__global__ void __launch_bounds__(64 * TJ, (ring_min_waves<T, VISC>())) k_stage_ring(
    StageArgs A, const BlockDesc* __restrict__ blocks, const TileDesc* __restrict__ tiles, Gas<T> gas) {
  using LD = RingLds<T, VISC, TJ>;
  constexpr int NT = 64 * TJ;
  constexpr int WI = LD::WI, WJ = LD::WJ;
  __shared__ __attribute__((aligned(16))) char smem[MODE == 3 ? LD::TOTAL_DT : LD::TOTAL];
  T* sW = reinterpret_cast<T*>(smem);                                   // [3][NW][WJ][WI]
  double* sFj = reinterpret_cast<double*>(smem + LD::W_BYTES);          // [5][TJ+1][64]
  double* sFe = sFj + LD::FJ;                                           // [5][TJ]
  double* sSj = sFe + LD::FE;                                           // mode 3: [3][TJ+1][64]
  double* sSe = sSj + LD::SJ;                                           // mode 3: [3][TJ]

  auto W = [&](int slot, int v, int pj, int pi) -> T& { return sW[slot * LD::PLANE + (v * WJ + pj) * WI + pi]; };
  auto wprim = [&](int slot, int pj, int pi) {
    Prim<T> w;
    w.r = W(slot, 0, pj, pi);
    w.u = W(slot, 1, pj, pi);
    w.v = W(slot, 2, pj, pi);
    w.w = W(slot, 3, pj, pi);
    w.p = W(slot, 4, pj, pi);
    return w;
  };
  auto wphi = [&](int slot, int pj, int pi, T o[4]) {
    o[0] = W(slot, 1, pj, pi);
    o[1] = W(slot, 2, pj, pi);
    o[2] = W(slot, 3, pj, pi);
    o[3] = W(slot, VISC ? 5 : 4, pj, pi);
  };

  const int tid = threadIdx.x, tx = tid & 63, ty = tid >> 6;
  // partials: stage 1 (mode 1) sum R^2, max |R_rho|, non-finite count;
  // stage 3 (mode 3) minimum time step of the new state
  double acc[NPART];
  init_partials(acc);

  for (int tile = blockIdx.x; tile < A.ntiles; tile += gridDim.x) {
    const TileDesc td = tiles[tile];
    const BlockDesc B = blocks[td.blk];
    const int ni = B.n[0], nj = B.n[1], nk = B.n[2];
    const int i0 = td.i0, j0 = td.j0, k0 = td.k0;
    const int kend = min(k0 + A.tile_k, nk);
    const int i = i0 + tx, j = j0 + ty;
    const bool act = i < ni && j < nj;
    const bool fi_ok = i <= ni && j < nj;
    const bool fj_ok = j <= nj && i < ni;
    const bool has_xj = j0 + TJ <= nj && i0 + tx < ni;              // wave 0: j-faces of row j0+TJ
    const bool has_xi = tx < TJ && i0 + 64 <= ni && j0 + tx < nj;  // wave 1: i-faces at column i0+64
    const double* qb = A.qs + B.qoff;
    const double* mb = A.met + B.moff;
    const double* vb = VISC ? A.vmet + B.voff : nullptr;
    const int64_t sj = B.sj, sk = B.sk, sv = B.sv;
    auto off = [&](int ii, int jj, int kk) -> int64_t {
      return (int64_t)(kk + NG) * sk + (int64_t)(jj + NG) * sj + (ii + NG);
    };
    // W(kk) with halo 2 into ring slot `slot`; a fixed trip count, unrolled,
    // so that all of a thread's loads are in flight together
    auto fill = [&](int slot, int kk) {
      constexpr int NS = (WJ * WI + NT - 1) / NT;
#pragma unroll
      for (int it = 0; it < NS; ++it) {
        const int s = tid + it * NT;
        if (s >= WJ * WI) break;
        const int pj = s / WI, pi = s - (s / WI) * WI;
        const int gi = i0 - 2 + pi, gj = j0 - 2 + pj;
        Prim<T> w;
        w.r = T(1); w.u = T(0); w.v = T(0); w.w = T(0); w.p = T(1);
        if (gi <= ni + 1 && gj <= nj + 1) w = ld_prim<T>(qb, off(gi, gj, kk), sv, gas.gm1);
        W(slot, 0, pj, pi) = w.r;
        W(slot, 1, pj, pi) = w.u;
        W(slot, 2, pj, pi) = w.v;
        W(slot, 3, pj, pi) = w.w;
        W(slot, 4, pj, pi) = w.p;
        if (VISC) W(slot, 5, pj, pi) = temp_of(w);
      }
    };

    // lower k-face of the tile from global memory; queue cell W(k0+2)
    double Fklo[5] = {0, 0, 0, 0, 0};
    Prim<T> q3{};
    if (act) {
      const int64_t c0 = off(i, j, k0);
      face_flux_global<T, VISC>(qb, mb, vb, B, c0, 2, gas, Fklo);
      q3 = ld_prim<T>(qb, c0 + 2 * sk, sv, gas.gm1);
    }
    __syncthreads();   // the previous tile's LDS users are done
    int sm = 0, s0 = 1, sp = 2;   // ring slots of W(k-1), W(k), W(k+1)
    fill(sm, k0 - 1);
    fill(s0, k0);
    fill(sp, k0 + 1);
    __syncthreads();

    for (int k = k0; k < kend; ++k) {
      // inputs of this plane's cell update, loaded before the face work
      CellIn cin;
      if (act) load_cell<MODE>(A, B, off(i, j, k), cin);
      // ---- A. faces of plane k
      // lower i-face of cell (i0+ci, j0+rj): flux F, area vector S
      auto face_i = [&](int ci, int rj, double F[5], double S[3]) {
        const int pi = ci + 2, pj = rj + 2;
        const int64_t c = off(i0 + ci, j0 + rj, k);
        const double sx = mb[c], sy = mb[sv + c], sz = mb[2 * sv + c];
        S[0] = sx;
        S[1] = sy;
        S[2] = sz;
        T f[5], n[3];
        const double area = face_inviscid<T>(wprim(s0, pj, pi - 2), wprim(s0, pj, pi - 1), wprim(s0, pj, pi),
                                             wprim(s0, pj, pi + 1), sx, sy, sz, gas, f, n);
        if (VISC) {
          T pl[4], pr[4], d1[4], d2[4], a[4], b[4], e[4], g[4];
          wphi(s0, pj, pi - 1, pl);
          wphi(s0, pj, pi, pr);
          wphi(s0, pj + 1, pi - 1, a); wphi(s0, pj + 1, pi, b); wphi(s0, pj - 1, pi - 1, e); wphi(s0, pj - 1, pi, g);
          tdiff(a, b, e, g, d1);
          wphi(sp, pj, pi - 1, a); wphi(sp, pj, pi, b); wphi(sm, pj, pi - 1, e); wphi(sm, pj, pi, g);
          tdiff(a, b, e, g, d2);
          double St[2][3], vf;
          face_vmetrics(vb, sv, c, 0, St, vf);
          face_viscous<T>(pl, pr, sx, sy, sz, n, d1, d2, St, vf, gas, f);
        }
        scale_flux_f64(f, area, F);
      };
      auto face_j = [&](int ci, int rj) {   // lower j-face of cell (i0+ci, j0+rj) -> sFj
        const int pi = ci + 2, pj = rj + 2;
        const int64_t c = off(i0 + ci, j0 + rj, k);
        const double sx = mb[3 * sv + c], sy = mb[4 * sv + c], sz = mb[5 * sv + c];
        if (MODE == 3) {
          sSj[(0 * (TJ + 1) + rj) * 64 + ci] = sx;
          sSj[(1 * (TJ + 1) + rj) * 64 + ci] = sy;
          sSj[(2 * (TJ + 1) + rj) * 64 + ci] = sz;
        }
        T f[5], n[3];
        const double area = face_inviscid<T>(wprim(s0, pj - 2, pi), wprim(s0, pj - 1, pi), wprim(s0, pj, pi),
                                             wprim(s0, pj + 1, pi), sx, sy, sz, gas, f, n);
        if (VISC) {
          T pl[4], pr[4], d1[4], d2[4], a[4], b[4], e[4], g[4];
          wphi(s0, pj - 1, pi, pl);
          wphi(s0, pj, pi, pr);
          wphi(s0, pj - 1, pi + 1, a); wphi(s0, pj, pi + 1, b); wphi(s0, pj - 1, pi - 1, e); wphi(s0, pj, pi - 1, g);
          tdiff(a, b, e, g, d1);
          wphi(sp, pj - 1, pi, a); wphi(sp, pj, pi, b); wphi(sm, pj - 1, pi, e); wphi(sm, pj, pi, g);
          tdiff(a, b, e, g, d2);
          double St[2][3], vf;
          face_vmetrics(vb, sv, c, 1, St, vf);
          face_viscous<T>(pl, pr, sx, sy, sz, n, d1, d2, St, vf, gas, f);
        }
        double F[5];
        scale_flux_f64(f, area, F);
        for (int q = 0; q < 5; ++q) sFj[(q * (TJ + 1) + rj) * 64 + ci] = F[q];
      };
      double Fi[5] = {0, 0, 0, 0, 0};
      if (fi_ok) {
        double Si[3];
        face_i(tx, ty, Fi, Si);
      }
      CFD_FACE_FENCE_RING();
      if (fj_ok) face_j(tx, ty);
      CFD_FACE_FENCE_RING();
      if (ty == 0 && has_xj) face_j(tx, TJ);
      if (ty == 1 && has_xi) {
        double Fe[5], Se[3];
        face_i(64, tx, Fe, Se);
        for (int q = 0; q < 5; ++q) sFe[q * TJ + tx] = Fe[q];
        if (MODE == 3)
          for (int x = 0; x < 3; ++x) sSe[x * TJ + tx] = Se[x];
      }
      CFD_FACE_FENCE_RING();
      double Fku[5] = {0, 0, 0, 0, 0};
      if (act) {   // upper k-face between (i, j, k) and (i, j, k+1)
        const int pi = tx + 2, pj = ty + 2;
        const int64_t cu = off(i, j, k) + sk;
        const double sx = mb[6 * sv + cu], sy = mb[7 * sv + cu], sz = mb[8 * sv + cu];
        T f[5], n[3];
        const double area = face_inviscid<T>(wprim(sm, pj, pi), wprim(s0, pj, pi), wprim(sp, pj, pi), q3,
                                             sx, sy, sz, gas, f, n);
        if (VISC) {
          T pl[4], pr[4], d1[4], d2[4], a[4], b[4], e[4], g[4];
          wphi(s0, pj, pi, pl);
          wphi(sp, pj, pi, pr);
          wphi(s0, pj, pi + 1, a); wphi(sp, pj, pi + 1, b); wphi(s0, pj, pi - 1, e); wphi(sp, pj, pi - 1, g);
          tdiff(a, b, e, g, d1);
          wphi(s0, pj + 1, pi, a); wphi(sp, pj + 1, pi, b); wphi(s0, pj - 1, pi, e); wphi(sp, pj - 1, pi, g);
          tdiff(a, b, e, g, d2);
          double St[2][3], vf;
          face_vmetrics(vb, sv, cu, 2, St, vf);
          face_viscous<T>(pl, pr, sx, sy, sz, n, d1, d2, St, vf, gas, f);
        }
        scale_flux_f64(f, area, Fku);
      }
      // upper i-face flux of this cell = lower i-face flux of the next lane
      double Fiu[5];
      for (int q = 0; q < 5; ++q) Fiu[q] = __shfl_down(Fi[q], 1, 64);
      __syncthreads();   // j-face and edge fluxes stored; every read of W(k-1) done

      // ---- B. cell update of plane k; fill W(k+2) over W(k-1); queue W(k+3)
      const bool more = k + 1 < kend;
      Prim<T> q3n = q3;
      if (act && more) q3n = ld_prim<T>(qb, off(i, j, k) + 3 * sk, sv, gas.gm1);
      // mode 3: the cell's face-averaged area vectors b[d] = (S_d(c) + S_d(c + e_d)) / 2.
      // Upper faces from this plane's face work: S_i of the next lane
      // (shuffle; the tile-edge face from LDS for lane 63), S_j of the next
      // row (LDS), S_k from the k-face (registers).  The lower i- and k-faces
      // are loaded again (cheaper than keeping them live through the faces).
      double bdt[3][3];
      if (MODE == 3) {
        double Si[3] = {0, 0, 0}, Sk[3] = {0, 0, 0}, Sku[3] = {0, 0, 0};
        if (fi_ok) {
          const int64_t c = off(i, j, k);
          for (int x = 0; x < 3; ++x) Si[x] = mb[x * sv + c];
        }
        if (act) {
          const int64_t c = off(i, j, k);
          for (int x = 0; x < 3; ++x) Sk[x] = mb[(6 + x) * sv + c];
          for (int x = 0; x < 3; ++x) Sku[x] = mb[(6 + x) * sv + c + sk];
        }
        double Siu[3];
        for (int x = 0; x < 3; ++x) Siu[x] = __shfl_down(Si[x], 1, 64);
        if (act)
          for (int x = 0; x < 3; ++x) {
            const double su = tx == 63 ? sSe[x * TJ + ty] : Siu[x];
            bdt[0][x] = 0.5 * (Si[x] + su);
            bdt[1][x] = 0.5 * (sSj[(x * (TJ + 1) + ty) * 64 + tx] + sSj[(x * (TJ + 1) + ty + 1) * 64 + tx]);
            bdt[2][x] = 0.5 * (Sk[x] + Sku[x]);
          }
      }
      if (more) fill(sm, k + 2);
      if (act) {
        double Di[5], Dj[5], Dk[5];
        for (int q = 0; q < 5; ++q) {
          const double fu = tx == 63 ? sFe[q * TJ + ty] : Fiu[q];
          Di[q] = fu - Fi[q];
          Dj[q] = sFj[(q * (TJ + 1) + ty + 1) * 64 + tx] - sFj[(q * (TJ + 1) + ty) * 64 + tx];
          Dk[q] = Fku[q] - Fklo[q];
        }
        double Rc[5], Qo[5];
        update_cell<MODE>(A, B, off(i, j, k), Di, Dj, Dk, cin, Rc, Qo);
        if (MODE == 1) {
#pragma unroll
          for (int q = 0; q < 5; ++q) {
            acc[q] += Rc[q] * Rc[q];
            if (!finite(Rc[q])) acc[11] += 1.0;
            if (!finite(cin.qv[q])) acc[11] += 1.0;
          }
          acc[10] = fmax(acc[10], fabs(Rc[0]));
        }
        if (MODE == 3) {
          const double dtc = cell_dt_b(Qo, bdt, cin.vol, A.sp);
          if (A.sp.local_dt) A.dt_out[B.soff + off(i, j, k)] = dtc;
          acc[12] = fmin(acc[12], dtc);
        }
        for (int q = 0; q < 5; ++q) Fklo[q] = Fku[q];
      }
      q3 = q3n;
      const int t = sm;
      sm = s0;
      s0 = sp;
      sp = t;
      __syncthreads();   // W(k+2) filled; j-face and edge flux reads done
    }
  }
  // the j-face buffer is free once the tiles are done
  if (MODE == 1 || MODE == 3)
    wg_reduce_partials(acc, A.partials + (int64_t)blockIdx.x * NPART, reinterpret_cast<double(*)[16]>(sFj));
}

// ---------------------------------------------------------------- launchers

template <typename T, bool VISC, int MODE, int TJ>
static void launch_ring_t(const StageArgs& A, const BlockDesc* blocks, const TileDesc* tiles, const Gas<T>& gas,
                          int nwg, hipStream_t s) {
  hipLaunchKernelGGL((k_stage_ring<T, VISC, MODE, TJ>), dim3(nwg), dim3(64 * TJ), 0, s, A, blocks, tiles, gas);
}

template <typename T, bool VISC, int MODE, int TJ>
static int occ_ring_t() {
  int n = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, k_stage_ring<T, VISC, MODE, TJ>, 64 * TJ, 0) != hipSuccess)
    return 1;
  return n > 0 ? n : 1;
}

template <typename T, bool VISC, int TJ>
static void ring_mode(const StageArgs& A, int mode, const BlockDesc* blocks, const TileDesc* tiles,
                      const Gas<T>& gas, int nwg, hipStream_t s, int* occ) {
  if (occ) {
    *occ = mode == 0 ? occ_ring_t<T, VISC, 0, TJ>()
                     : (mode == 1 ? occ_ring_t<T, VISC, 1, TJ>()
                                  : (mode == 2 ? occ_ring_t<T, VISC, 2, TJ>() : occ_ring_t<T, VISC, 3, TJ>()));
    return;
  }
  if (mode == 0) launch_ring_t<T, VISC, 0, TJ>(A, blocks, tiles, gas, nwg, s);
  else if (mode == 1) launch_ring_t<T, VISC, 1, TJ>(A, blocks, tiles, gas, nwg, s);
  else if (mode == 2) launch_ring_t<T, VISC, 2, TJ>(A, blocks, tiles, gas, nwg, s);
  else launch_ring_t<T, VISC, 3, TJ>(A, blocks, tiles, gas, nwg, s);
}

template <typename T, bool VISC>
static bool ring_tj(const StageArgs& A, int mode, const BlockDesc* blocks, const TileDesc* tiles, const Gas<T>& gas,
                    int nwg, hipStream_t s, int* occ) {
  if (A.tile_j == 8) ring_mode<T, VISC, 8>(A, mode, blocks, tiles, gas, nwg, s, occ);
  else if (A.tile_j == 4) ring_mode<T, VISC, 4>(A, mode, blocks, tiles, gas, nwg, s, occ);
  else return false;
  return true;
}

// Launch (occ == nullptr) or query the resident workgroups per CU.  Takes
// A.tile_j = 4 or 8.
bool stage_ring(const StageArgs& A, int mode, bool visc, bool fp32, const BlockDesc* blocks, const TileDesc* tiles,
                const Gas<double>& g64, const Gas<float>& g32, int nwg, hipStream_t s, int* occ) {
  if (fp32) {
    return visc ? ring_tj<float, true>(A, mode, blocks, tiles, g32, nwg, s, occ)
                : ring_tj<float, false>(A, mode, blocks, tiles, g32, nwg, s, occ);
  }
  return visc ? ring_tj<double, true>(A, mode, blocks, tiles, g64, nwg, s, occ)
              : ring_tj<double, false>(A, mode, blocks, tiles, g64, nwg, s, occ);
}

}  // namespace cfd
