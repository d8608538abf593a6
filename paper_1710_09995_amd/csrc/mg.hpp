// Launchers of the multigrid kernels (kernels_mg.hip).
#pragma once
#include <hip/hip_runtime.h>

#include "cfd_internal.hpp"

namespace cfd {

// q -= b dt F on the interior cells (dt: the per-cell step arena when local,
// else the one global step).
void launch_mg_force(double* q, const double* f, const double* dt, int local, double b, const BlockDesc* blocks,
                     int nblk, int64_t nchunks, int nwg, hipStream_t s);
// Coarse state and restricted forced residual from the fine level (ff may be
// null: no forcing on the fine level); the grid cuts the coarse chunks.
void launch_mg_restrict(const double* qf, const double* metf, const double* rf, const double* ff,
                        const BlockDesc* bf, double* qc, double* q0, double* fc, const double* metc,
                        const BlockDesc* bc, int nblk, int64_t nchunks_c, int nwg, hipStream_t s);
// fc -= rc on the coarse interior cells.
void launch_mg_forcing(double* fc, const double* rc, const BlockDesc* bc, int nblk, int64_t nchunks_c, int nwg,
                       hipStream_t s);
// qf += qc - q0 of each fine cell's parent; the grid cuts the fine chunks.
void launch_mg_prolong(double* qf, const BlockDesc* bf, const double* qc, const double* q0, const BlockDesc* bc,
                       int nblk, int64_t nchunks_f, int nwg, hipStream_t s);

}  // namespace cfd
