// Sixth-order staggered flux difference of Section 2.2, Eq. (2): the
// cell-centred derivative of a face-centred field along one index direction,
//   out_i = [75/64 (F_{i+1/2} - F_{i-1/2}) - 25/384 (F_{i+3/2} - F_{i-3/2})
//            + 3/640 (F_{i+5/2} - F_{i-5/2})] / h.
// One thread per (variable, cell); the six faces of a cell are adjacent along
// the direction, so neighbouring cells share them through L1/L2.  Each XCD
// (workgroup id mod 8, the grid being a multiple of 8) streams one contiguous
// eighth of the rows: the faces a stencil re-reads stay in that XCD's L2.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdint>
#include <string>

#include "../../include/cfd.h"
#include "host_services.hpp"

namespace cfd {

__device__ __forceinline__ int xcd_slot(int nb, int b) {   // XCD-contiguous order for grids that are multiples of 8
  return (nb & 7) == 0 ? (b & 7) * (nb >> 3) + (b >> 3) : b;
}

__device__ __forceinline__ double eq2(double c1, double c2, double c3, double f0, double f1, double f2, double f3,
                                      double f4, double f5) {
  return c1 * (f3 - f2) + c2 * (f4 - f1) + c3 * (f5 - f0);
}

// Along i: workgroup w takes a 256-cell segment of RI consecutive i-rows
// (row = (v, k, j)) and stages the rows' 261 faces each in LDS (coalesced,
// all rows' loads in flight before the one barrier); each lane then reads its
// six faces per row from LDS.
constexpr int RI = 4;
__global__ void __launch_bounds__(256) k_staggered_diff6_i(const double* __restrict__ f, double* __restrict__ out,
                                                           int ni, int nj, int nk, int nseg, int nrows, double c1,
                                                           double c2, double c3) {
  __shared__ double sf[RI][256 + 5];
  const int w = xcd_slot(gridDim.x, blockIdx.x);
  const int rg = w / nseg, seg = w - rg * nseg;
  const int i0 = seg * 256, t = (int)threadIdx.x;
  const int64_t ei = ni + 5;
#pragma unroll
  for (int q = 0; q < RI; ++q) {
    const int row = rg * RI + q;             // row = (v * nk + k) * nj + j
    const double* fr = f + (int64_t)row * ei;
    for (int s = t; s < 256 + 5; s += 256) sf[q][s] = row < nrows && i0 + s < ni + 5 ? fr[i0 + s] : 0.0;
  }
  __syncthreads();
  const int i = i0 + t;
  if (i >= ni) return;
#pragma unroll
  for (int q = 0; q < RI; ++q) {
    const int row = rg * RI + q;
    if (row < nrows)
      out[(int64_t)row * ni + i] =
          eq2(c1, c2, c3, sf[q][t], sf[q][t + 1], sf[q][t + 2], sf[q][t + 3], sf[q][t + 4], sf[q][t + 5]);
  }
}

// Along j or k: each lane marches CH cells of its i-column along the
// direction with a register window of CH + 5 faces (all loaded up front), so
// a face is loaded (CH + 5) / CH times instead of six.  Workgroup w takes a
// 256-cell i-segment of one chunk of one line (v, the other transverse index).
template <int CH>
__global__ void __launch_bounds__(256) k_staggered_diff6_march(const double* __restrict__ f, double* __restrict__ out,
                                                               int ni, int nj, int nk, int d, int nseg, int nchunk,
                                                               double c1, double c2, double c3) {
  const int w = xcd_slot(gridDim.x, blockIdx.x);
  const int seg = w % nseg;
  int r = w / nseg;
  const int chunk = r % nchunk;
  r /= nchunk;
  const int i = seg * 256 + (int)threadIdx.x;
  if (i >= ni) return;
  const int nd = d == 1 ? nj : nk;                 // cells along the direction
  const int no = d == 1 ? nk : nj;                 // the other transverse extent
  const int o = r % no, v = r / no;
  const int j = d == 1 ? 0 : o, k = d == 1 ? o : 0;
  const int64_t ej = nj + (d == 1 ? 5 : 0), ek = nk + (d == 2 ? 5 : 0);
  const int64_t sd = d == 1 ? ni : (int64_t)ni * ej;                 // face stride along d
  const int64_t so = d == 1 ? (int64_t)ni : (int64_t)nj * ni;          // cell stride along d in out
  const double* fp = f + (((int64_t)v * ek + k) * ej + j) * ni + i;    // face position 0 of this line
  double* op = out + (((int64_t)v * nk + k) * nj + j) * ni + i;        // cell 0 of this line
  const int c0 = chunk * CH;
  double win[CH + 5];
#pragma unroll
  for (int s = 0; s < CH + 5; ++s) win[s] = c0 + s < nd + 5 ? fp[(c0 + s) * sd] : 0.0;
#pragma unroll
  for (int s = 0; s < CH; ++s)
    if (c0 + s < nd)
      op[(c0 + s) * so] = eq2(c1, c2, c3, win[s], win[s + 1], win[s + 2], win[s + 3], win[s + 4], win[s + 5]);
}

}  // namespace cfd

extern "C" cfd_status cfd_staggered_diff6(const double* f_dev, double* out_dev, const int32_t n[3], int32_t d,
                                          int32_t nvar, double h, hipStream_t stream) {
  return cfd::host_guarded([&] {
    if (!f_dev || !out_dev || !n) cfd::host_fail(CFD_EINVAL, "NULL argument");
    if (d < 0 || d > 2) cfd::host_fail(CFD_EINVAL, "direction must be 0, 1 or 2");
    if (n[0] < 1 || n[1] < 1 || n[2] < 1) cfd::host_fail(CFD_EINVAL, "every extent must be >= 1");
    if (nvar < 1 || nvar > 64) cfd::host_fail(CFD_EINVAL, "nvar must be in [1, 64]");
    if (!(h > 0.0) || !std::isfinite(h)) cfd::host_fail(CFD_EINVAL, "h must be positive and finite");
    const int64_t cells = (int64_t)n[0] * n[1] * n[2];
    const int64_t total = cells * nvar;
    const int64_t faces = total + (int64_t)5 * nvar * (cells / n[d]);
    if (total > ((int64_t)1 << 40)) cfd::host_fail(CFD_EINVAL, "field too large");
    // the input and output ranges must not overlap
    const char *fa = reinterpret_cast<const char*>(f_dev), *fe = fa + faces * 8;
    const char *oa = reinterpret_cast<const char*>(out_dev), *oe = oa + total * 8;
    if (fa < oe && oa < fe) cfd::host_fail(CFD_EINVAL, "f and out overlap");
    const double c1 = 75.0 / (64.0 * h), c2 = -25.0 / (384.0 * h), c3 = 3.0 / (640.0 * h);
    const int64_t nseg = (n[0] + 255) / 256;
    if (d == 0) {
      const int64_t nrows = (int64_t)nvar * n[1] * n[2];
      const int64_t nwork = nseg * ((nrows + cfd::RI - 1) / cfd::RI);
      if (nwork > INT32_MAX || nrows > INT32_MAX) cfd::host_fail(CFD_EINVAL, "field too large");
      hipLaunchKernelGGL(cfd::k_staggered_diff6_i, dim3((unsigned)nwork), dim3(256), 0, stream, f_dev, out_dev, n[0],
                         n[1], n[2], (int)nseg, (int)nrows, c1, c2, c3);
    } else {
      constexpr int CH = 16;
      const int64_t nchunk = (n[d] + CH - 1) / CH;
      const int64_t nwork = nseg * nchunk * nvar * (d == 1 ? n[2] : n[1]);
      if (nwork > INT32_MAX) cfd::host_fail(CFD_EINVAL, "field too large");
      hipLaunchKernelGGL(cfd::k_staggered_diff6_march<CH>, dim3((unsigned)nwork), dim3(256), 0, stream, f_dev,
                         out_dev, n[0], n[1], n[2], d, (int)nseg, (int)nchunk, c1, c2, c3);
    }
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) cfd::host_fail(CFD_EHIP, std::string("kernel launch failed: ") + hipGetErrorString(e));
  });
}
