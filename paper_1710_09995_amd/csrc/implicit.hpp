// Arguments of the implicit-step kernels (kernels_implicit.hip), shared with
// the host runtime.
#pragma once
#include <stdint.h>
#include <hip/hip_runtime_api.h>

namespace cfd {

struct ImplicitArgs {
  const double* q;       // state arena (ghost cells filled)
  const double* met;     // metrics arena
  const double* r;       // R(Q^n), state layout
  double* mu;            // MU arena (state layout, 5 variables as above)
  const double* dq_in;   // current iterate (ghost cells filled)
  double* dq_out;        // next iterate
  const double* dt;      // global step (1 double) when !local
  int local;
  int viscous;
  double gamma, prandtl, mu_inf, s_star;
  double cfl;
};

struct BlockDesc;
struct StepParams;
void launch_ifv_faces(const ImplicitArgs& A, const BlockDesc* blocks, int nblk, int64_t nchunks,
                      const StepParams& P, int nwg, hipStream_t s);
void launch_ifv_diag(const ImplicitArgs& A, const BlockDesc* blocks, int nblk, int64_t nchunks, int nwg,
                     hipStream_t s);
void launch_ifv_sweep(const ImplicitArgs& A, const BlockDesc* blocks, int nblk, int64_t nchunks, int nwg,
                      hipStream_t s);
void launch_ifv_apply(double* q, const double* dq, const BlockDesc* blocks, int nblk, int64_t nchunks, int nwg,
                      hipStream_t s);

}  // namespace cfd
