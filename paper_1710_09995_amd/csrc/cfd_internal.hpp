// Internal device/host descriptors shared by the kernels and the host runtime.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace cfd {

constexpr int NG = 2;          // ghost layers
constexpr int NV = 5;          // conserved variables
constexpr int NM = 10;         // metric components: S_i(3), S_j(3), S_k(3), V
constexpr int NVM = 21;        // viscous face metrics: per direction d, on the lower d-face,
                               // the two averaged transverse face vectors (6) and the
                               // auxiliary-cell volume (1), at index 7 d + ...
constexpr int NHIST = 12;      // history row: dt, L2(R) x5, sum VQ x5, max|R_rho|
constexpr int NPART = 13;      // per-workgroup partials: sum R^2 x5, sum VQ x5, max|R_rho|, nonfinite, min dt

// physical boundary kinds (same values as cfd_bc_kind)
constexpr int CFD_BC_KIND_FARFIELD = 1;
constexpr int CFD_BC_KIND_SLIPWALL = 2;
constexpr int CFD_BC_KIND_NOSLIP = 3;
constexpr int CFD_BC_KIND_EXTRAP = 4;

// One block of the multi-block grid, as the kernels see it.
struct BlockDesc {
  int32_t n[3];        // interior cells ni, nj, nk
  int32_t pad0;
  int64_t qoff;        // state arena: element index of padded cell (-g,-g,-g), var 0
  int64_t moff;        // metrics arena offset (NM vars, same strides)
  int64_t soff;        // scalar arena offset (1 var, same strides)
  int64_t voff;        // viscous face metric arena offset (NVM vars, same strides)
  int64_t sv, sk, sj;  // element strides of var, k, j (i stride is 1)
  int64_t xoff;        // node scratch: element index of padded node (-g,-g,-g), coord 0
  int64_t xsv, xsk, xsj;
  int64_t coff;        // row chunks (runs of up to 64 cells along i) of the blocks before this one
};

// One patch of one sweep (connection or physical boundary), cells or nodes.
struct PatchDesc {
  int32_t blk, face, kind, nbr;   // kind 0 = connection, else cfd_bc_kind
  int32_t lo[3], hi[3];           // covered logical index range per direction (d entry unused)
  int32_t noff[3];                // neighbour index = own index + noff (transverse); unused for d
  int32_t count;                  // number of transverse points
  int32_t pad0;
  double shift[3];                // connections: added to neighbour node coordinates
  double uinf[3];                 // far field: freestream velocity of this patch
};

// Threads per transverse point of a state ghost sweep (k_ghost_q): one per
// ghost layer on i-faces, else one.
__host__ __device__ inline int ghost_threads_per_point(int /*kind*/, int d) { return d == 0 ? NG : 1; }

// One tile of the stage work list.
struct TileDesc {
  int32_t blk, i0, j0, k0;
};

// Flow constants in the precision of the flux evaluation.
template <typename T>
struct Gas {
  T gamma, gm1, prandtl, mu_inf, s_star, eps_h, eps_lim;
  T gg;     // gamma / (gamma - 1): enthalpy over p / rho
  T kfac;   // gamma / ((gamma - 1) Pr): conductivity over viscosity
  T uinf[3];
};

// Warm-start network geometry (padded parameter layout, training cache).
constexpr int MLP_KIN = 16;          // input features padded to one MFMA k-step
constexpr int MLP_NOUT = 16;         // outputs padded to one MFMA tile
constexpr int MLP_MAX_LAYERS = 9;
struct MlpDims {
  int d_in, d_hidden, n_hidden, d_out;
  int nlayer;                        // n_hidden + 1 weight matrices
  int K[MLP_MAX_LAYERS], N[MLP_MAX_LAYERS];
  int64_t woff[MLP_MAX_LAYERS];      // offset of W_l (elements)
  int64_t boff[MLP_MAX_LAYERS];      // offset of b_l
  int64_t hoff[MLP_MAX_LAYERS];      // cache: layer input h_l, per-point offset (floats)
  int64_t zoff[MLP_MAX_LAYERS];      // cache: pre-activation z_l, per-point offset
  int64_t nparam, cache_per_point;
};

// Interior cells of all blocks, numbered block by block (k, j, i; i fastest).
struct CellMap {
  const BlockDesc* blocks;
  const int64_t* cell_start;         // [nblk + 1] prefix sums of interior cell counts
  int nblk;
};

struct StepParams {
  double gamma, prandtl, mu_inf, s_star, cfl, eps_h, eps_lim;
  double uinf[3];
  int32_t viscous, flux_fp32, local_dt, pad0;
};

// Arguments of the residual / stage kernels.
// mode 0 writes R; mode 1 is stage 1: out = Qs - dt R(Qs), and either
// rout = R(Qs) (for the norms kernel) or, in the plane-ring kernel, the norm
// partials of R(Qs) per workgroup; mode 2 is stages 2-3:
// out = a Qn + b (Qs - dt R(Qs)); mode 3 (plane-ring kernel only) is stage 3
// plus the CFL time step of the new state (per-workgroup minimum into
// partials, per-cell steps into dt_out with local stepping).
struct StageArgs {
  const double* qs;   // stencil state Q^(s)
  const double* qn;   // Q^n (pointwise, mode 2)
  double* out;        // R (mode 0) or Q^(s+1)
  double* rout;       // R (mode 1, if not null), state-arena layout, interior cells only
  double* partials;   // [gridDim.x][NPART] partials (modes 1 and 3, plane-ring kernel)
  double* dt_out;     // per-cell steps of the new state (mode 3, local stepping)
  const double* met;
  const double* vmet; // viscous face metrics (viscous flow only)
  const double* dt;   // global dt (1 double) or per-cell scalar arena (local)
  double a, b;
  int32_t local_dt;
  int32_t ntiles;
  int32_t tile_j, tile_k;
  StepParams sp;      // flow and CFL parameters (mode 3)
  // A multigrid level's forcing, applied by the tiled and simple kernels in
  // modes 1-2 (null: none): out = out - (fb dt) F, rounded as the separate
  // forcing pass rounds it.
  const double* force;
  double fb;
};


}  // namespace cfd
