// Tiled face-once residual / stage kernel.
//
// A workgroup of 64 x TJ threads owns a tile of 64 (i) x TJ (j) cell columns
// and marches it through k.  Per k-plane:
//   1. the plane's primitives (rho, u, v, w, p [, T]) are built in LDS with a
//      halo of 2 cells (MUSCL stencil); for viscous flow the planes k-1 and
//      k+1 of phi = (u, v, w, T) are kept in LDS with a halo of 1;
//   2. each thread computes the lower i-face and lower j-face of its column
//      from LDS and the upper k-face from a register queue of its own column
//      (W at k-1 .. k+2); the faces on the tile's high i and j edges are
//      spread over the first waves; every face is computed once per tile and
//      its flux goes straight to an LDS exchange buffer;
//   3. every interior cell forms R = ((Di + Dj) + Dk) / V and its stage update.
// Metrics are read from global memory (cached; each is used by several faces);
// the viscous face terms come precomputed from the viscous face metric arena.
// The first k-face of a tile comes from the global-memory gather, which feeds
// face_inviscid / face_viscous the same bits in the same order, so results do
// not depend on the tile shape or on which kernel computed them.
#include <hip/hip_runtime.h>
#include "cfd_internal.hpp"
#include "physics.hpp"
#include "stage_common.hpp"

// Scheduling fence between face computations: keeps the compiler from
// hoisting one face's loads into another's live range (register pressure).
#ifndef CFD_SCHED_FENCE
#define CFD_SCHED_FENCE 1
#endif
#if CFD_SCHED_FENCE
#define CFD_FACE_FENCE() __builtin_amdgcn_sched_barrier(0)
#else
#define CFD_FACE_FENCE() ((void)0)
#endif
// Minimum waves per SIMD requested from the register allocator (0 = none).
#ifndef CFD_MIN_WAVES
#define CFD_MIN_WAVES 0
#endif
#if CFD_MIN_WAVES > 0
#define CFD_TILED_BOUNDS(n) __launch_bounds__(n, CFD_MIN_WAVES)
#else
#define CFD_TILED_BOUNDS(n) __launch_bounds__(n)
#endif

namespace cfd {

template <typename T, bool VISC, int TJ>
struct TiledLds {
  static constexpr int WI = 68, WJ = TJ + 4;   // primitive plane, halo 2
  static constexpr int PI = 66, PJ = TJ + 2;   // phi planes, halo 1
  static constexpr int NW = VISC ? 6 : 5;
  static constexpr int W_BYTES = (NW * WJ * WI * (int)sizeof(T) + 15) / 16 * 16;
  static constexpr int FI = 5 * TJ * 65;        // doubles: lower i-faces, 65 per row
  static constexpr int FJ = 5 * (TJ + 1) * 64;  // doubles: lower j-faces, TJ+1 rows
  static constexpr int F_BYTES = (FI + FJ) * 8;
  static constexpr int P_ELEMS = 4 * PJ * PI;
  static constexpr int P_BYTES = VISC ? 2 * P_ELEMS * (int)sizeof(T) : 0;
  static constexpr int TOTAL = F_BYTES + W_BYTES + P_BYTES;
};

template <typename T, bool VISC, int MODE, int TJ>
__global__ void CFD_TILED_BOUNDS(64 * TJ) k_stage_tiled(StageArgs A, const BlockDesc* __restrict__ blocks,
                                                        const TileDesc* __restrict__ tiles, Gas<T> gas) {
  using LD = TiledLds<T, VISC, TJ>;
  constexpr int NT = 64 * TJ;
  constexpr int WI = LD::WI, WJ = LD::WJ, PI = LD::PI, PJ = LD::PJ;
  __shared__ __attribute__((aligned(16))) char smem[LD::TOTAL];
  double* sFi = reinterpret_cast<double*>(smem);                 // [5][TJ][65]
  double* sFj = sFi + LD::FI;                                     // [5][TJ+1][64]
  T* sW = reinterpret_cast<T*>(smem + LD::F_BYTES);               // [NW][WJ][WI]
  T* sPm = reinterpret_cast<T*>(smem + LD::F_BYTES + LD::W_BYTES);   // phi(k-1) [4][PJ][PI]
  T* sPp = sPm + LD::P_ELEMS;                                     // phi(k+1)

  auto W = [&](int v, int pj, int pi) -> T& { return sW[(v * WJ + pj) * WI + pi]; };
  auto P = [&](T* buf, int v, int pj, int pi) -> T& { return buf[(v * PJ + pj) * PI + pi]; };
  auto wprim = [&](int pj, int pi) {
    Prim<T> w;
    w.r = W(0, pj, pi);
    w.u = W(1, pj, pi);
    w.v = W(2, pj, pi);
    w.w = W(3, pj, pi);
    w.p = W(4, pj, pi);
    return w;
  };
  auto wphi = [&](int pj, int pi, T o[4]) {
    o[0] = W(1, pj, pi);
    o[1] = W(2, pj, pi);
    o[2] = W(3, pj, pi);
    o[3] = W(VISC ? 5 : 4, pj, pi);
  };
  auto pphi = [&](T* buf, int pj, int pi, T o[4]) {
    o[0] = P(buf, 0, pj, pi);
    o[1] = P(buf, 1, pj, pi);
    o[2] = P(buf, 2, pj, pi);
    o[3] = P(buf, 3, pj, pi);
  };

  const int tid = threadIdx.x, tx = tid & 63, ty = tid >> 6;

  for (int tile = blockIdx.x; tile < A.ntiles; tile += gridDim.x) {
    const TileDesc td = tiles[tile];
    const BlockDesc B = blocks[td.blk];
    const int ni = B.n[0], nj = B.n[1], nk = B.n[2];
    const int i0 = td.i0, j0 = td.j0, k0 = td.k0;
    const int kend = min(k0 + A.tile_k, nk);
    const int i = i0 + tx, j = j0 + ty;
    const bool act = i < ni && j < nj;
    const bool fi_ok = i <= ni && j < nj;   // this thread's lower i-face is needed
    const bool fj_ok = j <= nj && i < ni;   // this thread's lower j-face is needed
    // faces on the tile's high edges: the j-faces of row j0+TJ (wave 0) and
    // the i-faces of column i0+64 (TJ lanes of wave 1)
    const bool has_xj = j0 + TJ <= nj && i0 + tx < ni;
    const bool has_xi = tx < TJ && i0 + 64 <= ni && j0 + tx < nj;
    const double* qb = A.qs + B.qoff;
    const double* mb = A.met + B.moff;
    const double* vb = VISC ? A.vmet + B.voff : nullptr;
    const int64_t sj = B.sj, sk = B.sk, sv = B.sv;
    auto off = [&](int ii, int jj, int kk) -> int64_t {
      return (int64_t)(kk + NG) * sk + (int64_t)(jj + NG) * sj + (ii + NG);
    };

    // own-column queue W(k-1), W(k), W(k+1), W(k+2) and the lower k-face
    Prim<T> q0{}, q1{}, q2{}, q3{};
    double Fklo[5] = {0, 0, 0, 0, 0};
    if (act) {
      const int64_t c0 = off(i, j, k0);
      face_flux_global<T, VISC>(qb, mb, vb, B, c0, 2, gas, Fklo);
      q0 = ld_prim<T>(qb, c0 - sk, sv, gas.gm1);
      q1 = ld_prim<T>(qb, c0, sv, gas.gm1);
      q2 = ld_prim<T>(qb, c0 + sk, sv, gas.gm1);
      q3 = ld_prim<T>(qb, c0 + 2 * sk, sv, gas.gm1);
    }
    auto fill_phi = [&](T* buf, int kk) {   // phi plane kk with halo 1
      for (int s = tid; s < PJ * PI; s += NT) {
        const int pj = s / PI, pi = s - (s / PI) * PI;
        const int gi = i0 - 1 + pi, gj = j0 - 1 + pj;
        T o[4] = {T(0), T(0), T(0), T(1)};
        if (gi <= ni + 1 && gj <= nj + 1) {
          const Prim<T> w = ld_prim<T>(qb, off(gi, gj, kk), sv, gas.gm1);
          phi_of(w, temp_of(w), o);
        }
        for (int v = 0; v < 4; ++v) P(buf, v, pj, pi) = o[v];
      }
    };
    __syncthreads();   // the previous tile's LDS users are done
    if (VISC) fill_phi(sPm, k0 - 1);

    for (int k = k0; k < kend; ++k) {
      // ---- 1. planes: W(k) with halo 2, phi(k+1) with halo 1
      for (int s = tid; s < WJ * WI; s += NT) {
        const int pj = s / WI, pi = s - (s / WI) * WI;
        const int gi = i0 - 2 + pi, gj = j0 - 2 + pj;
        Prim<T> w;
        w.r = T(1); w.u = T(0); w.v = T(0); w.w = T(0); w.p = T(1);
        if (gi <= ni + 1 && gj <= nj + 1) w = ld_prim<T>(qb, off(gi, gj, k), sv, gas.gm1);
        W(0, pj, pi) = w.r;
        W(1, pj, pi) = w.u;
        W(2, pj, pi) = w.v;
        W(3, pj, pi) = w.w;
        W(4, pj, pi) = w.p;
        if (VISC) W(5, pj, pi) = temp_of(w);
      }
      if (VISC) fill_phi(sPp, k + 1);
      __syncthreads();

      // ---- 2. faces, each flux stored to LDS as soon as it is known
      auto face_i = [&](int ci, int rj) {   // lower i-face of cell (i0+ci, j0+rj)
        const int pi = ci + 2, pj = rj + 2, qi = ci + 1, qj = rj + 1;
        const int64_t c = off(i0 + ci, j0 + rj, k);
        const double sx = mb[c], sy = mb[sv + c], sz = mb[2 * sv + c];
        T f[5], n[3];
        const double area = face_inviscid<T>(wprim(pj, pi - 2), wprim(pj, pi - 1), wprim(pj, pi),
                                             wprim(pj, pi + 1), sx, sy, sz, gas, f, n);
        if (VISC) {
          T pl[4], pr[4], d1[4], d2[4], a[4], b[4], e[4], g[4];
          wphi(pj, pi - 1, pl);
          wphi(pj, pi, pr);
          wphi(pj + 1, pi - 1, a); wphi(pj + 1, pi, b); wphi(pj - 1, pi - 1, e); wphi(pj - 1, pi, g);
          tdiff(a, b, e, g, d1);
          pphi(sPp, qj, qi - 1, a); pphi(sPp, qj, qi, b); pphi(sPm, qj, qi - 1, e); pphi(sPm, qj, qi, g);
          tdiff(a, b, e, g, d2);
          double St[2][3], vf;
          face_vmetrics(vb, sv, c, 0, St, vf);
          face_viscous<T>(pl, pr, sx, sy, sz, n, d1, d2, St, vf, gas, f);
        }
        double F[5];
        scale_flux_f64(f, area, F);
        for (int q = 0; q < 5; ++q) sFi[(q * TJ + rj) * 65 + ci] = F[q];
      };
      auto face_j = [&](int ci, int rj) {   // lower j-face of cell (i0+ci, j0+rj)
        const int pi = ci + 2, pj = rj + 2, qi = ci + 1, qj = rj + 1;
        const int64_t c = off(i0 + ci, j0 + rj, k);
        const double sx = mb[3 * sv + c], sy = mb[4 * sv + c], sz = mb[5 * sv + c];
        T f[5], n[3];
        const double area = face_inviscid<T>(wprim(pj - 2, pi), wprim(pj - 1, pi), wprim(pj, pi),
                                             wprim(pj + 1, pi), sx, sy, sz, gas, f, n);
        if (VISC) {
          T pl[4], pr[4], d1[4], d2[4], a[4], b[4], e[4], g[4];
          wphi(pj - 1, pi, pl);
          wphi(pj, pi, pr);
          wphi(pj - 1, pi + 1, a); wphi(pj, pi + 1, b); wphi(pj - 1, pi - 1, e); wphi(pj, pi - 1, g);
          tdiff(a, b, e, g, d1);
          pphi(sPp, qj - 1, qi, a); pphi(sPp, qj, qi, b); pphi(sPm, qj - 1, qi, e); pphi(sPm, qj, qi, g);
          tdiff(a, b, e, g, d2);
          double St[2][3], vf;
          face_vmetrics(vb, sv, c, 1, St, vf);
          face_viscous<T>(pl, pr, sx, sy, sz, n, d1, d2, St, vf, gas, f);
        }
        double F[5];
        scale_flux_f64(f, area, F);
        for (int q = 0; q < 5; ++q) sFj[(q * (TJ + 1) + rj) * 64 + ci] = F[q];
      };
      if (fi_ok) face_i(tx, ty);
      CFD_FACE_FENCE();
      if (fj_ok) face_j(tx, ty);
      CFD_FACE_FENCE();
      if (ty == 0 && has_xj) face_j(tx, TJ);
      if (ty == 1 && has_xi) face_i(64, tx);
      CFD_FACE_FENCE();
      double Fku[5] = {0, 0, 0, 0, 0};
      if (act) {   // upper k-face between (i, j, k) and (i, j, k+1)
        const int pi = tx + 2, pj = ty + 2, qi = tx + 1, qj = ty + 1;
        const int64_t cu = off(i, j, k) + sk;
        const double sx = mb[6 * sv + cu], sy = mb[7 * sv + cu], sz = mb[8 * sv + cu];
        T f[5], n[3];
        const double area = face_inviscid<T>(q0, q1, q2, q3, sx, sy, sz, gas, f, n);
        if (VISC) {
          T pl[4], pr[4], d1[4], d2[4], a[4], b[4], e[4], g[4];
          phi_of(q1, temp_of(q1), pl);
          phi_of(q2, temp_of(q2), pr);
          wphi(pj, pi + 1, a); pphi(sPp, qj, qi + 1, b); wphi(pj, pi - 1, e); pphi(sPp, qj, qi - 1, g);
          tdiff(a, b, e, g, d1);
          wphi(pj + 1, pi, a); pphi(sPp, qj + 1, qi, b); wphi(pj - 1, pi, e); pphi(sPp, qj - 1, qi, g);
          tdiff(a, b, e, g, d2);
          double St[2][3], vf;
          face_vmetrics(vb, sv, cu, 2, St, vf);
          face_viscous<T>(pl, pr, sx, sy, sz, n, d1, d2, St, vf, gas, f);
        }
        scale_flux_f64(f, area, Fku);
      }
      __syncthreads();   // fluxes stored; every read of sW / sPm / sPp for this plane done

      // ---- 3. keep phi(k) as the next plane's phi(k-1); finish the cells
      if (VISC) {
        for (int s = tid; s < PJ * PI; s += NT) {
          const int pj = s / PI, pi = s - (s / PI) * PI;
          T o[4];
          wphi(pj + 1, pi + 1, o);
          for (int v = 0; v < 4; ++v) P(sPm, v, pj, pi) = o[v];
        }
      }
      if (act) {
        double Di[5], Dj[5], Dk[5];
        for (int q = 0; q < 5; ++q) {
          Di[q] = sFi[(q * TJ + ty) * 65 + tx + 1] - sFi[(q * TJ + ty) * 65 + tx];
          Dj[q] = sFj[(q * (TJ + 1) + ty + 1) * 64 + tx] - sFj[(q * (TJ + 1) + ty) * 64 + tx];
          Dk[q] = Fku[q] - Fklo[q];
        }
        const int64_t c = off(i, j, k);
        q0 = q1;
        q1 = q2;
        q2 = q3;
        if (k + 1 < kend) q3 = ld_prim<T>(qb, c + 3 * sk, sv, gas.gm1);   // loads before the stores below
        finish_cell<MODE>(A, B, c, Di, Dj, Dk);
        for (int q = 0; q < 5; ++q) Fklo[q] = Fku[q];
      }
      __syncthreads();   // flux reads and the phi copy done before the next plane
    }
  }
}

// ---------------------------------------------------------------- launchers

template <typename T, bool VISC, int MODE, int TJ>
static void launch_t(const StageArgs& A, const BlockDesc* blocks, const TileDesc* tiles, const Gas<T>& gas,
                     int nwg, hipStream_t s) {
  hipLaunchKernelGGL((k_stage_tiled<T, VISC, MODE, TJ>), dim3(nwg), dim3(64 * TJ), 0, s, A, blocks, tiles, gas);
}

template <typename T, bool VISC, int MODE, int TJ>
static int occ_t() {
  int n = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, k_stage_tiled<T, VISC, MODE, TJ>, 64 * TJ, 0) != hipSuccess)
    return 1;
  return n > 0 ? n : 1;
}

template <typename T, bool VISC, int TJ>
static void dispatch_mode(const StageArgs& A, int mode, const BlockDesc* blocks, const TileDesc* tiles,
                          const Gas<T>& gas, int nwg, hipStream_t s, int* occ) {
  if (occ) {
    *occ = mode == 0 ? occ_t<T, VISC, 0, TJ>() : (mode == 1 ? occ_t<T, VISC, 1, TJ>() : occ_t<T, VISC, 2, TJ>());
    return;
  }
  if (mode == 0) launch_t<T, VISC, 0, TJ>(A, blocks, tiles, gas, nwg, s);
  else if (mode == 1) launch_t<T, VISC, 1, TJ>(A, blocks, tiles, gas, nwg, s);
  else launch_t<T, VISC, 2, TJ>(A, blocks, tiles, gas, nwg, s);
}

template <typename T, bool VISC>
static bool dispatch_tj(const StageArgs& A, int mode, int tj, const BlockDesc* blocks, const TileDesc* tiles,
                        const Gas<T>& gas, int nwg, hipStream_t s, int* occ) {
  switch (tj) {
    case 2: dispatch_mode<T, VISC, 2>(A, mode, blocks, tiles, gas, nwg, s, occ); return true;
    case 4: dispatch_mode<T, VISC, 4>(A, mode, blocks, tiles, gas, nwg, s, occ); return true;
    case 8: dispatch_mode<T, VISC, 8>(A, mode, blocks, tiles, gas, nwg, s, occ); return true;
  }
  return false;
}

// Launch (occ == nullptr) or query the resident workgroups per CU (occ != nullptr).
bool stage_tiled(const StageArgs& A, int mode, bool visc, bool fp32, const BlockDesc* blocks,
                 const TileDesc* tiles, const Gas<double>& g64, const Gas<float>& g32, int nwg,
                 hipStream_t s, int* occ) {
  if (fp32) {
    return visc ? dispatch_tj<float, true>(A, mode, A.tile_j, blocks, tiles, g32, nwg, s, occ)
                : dispatch_tj<float, false>(A, mode, A.tile_j, blocks, tiles, g32, nwg, s, occ);
  }
  return visc ? dispatch_tj<double, true>(A, mode, A.tile_j, blocks, tiles, g64, nwg, s, occ)
              : dispatch_tj<double, false>(A, mode, A.tile_j, blocks, tiles, g64, nwg, s, occ);
}

}  // namespace cfd
