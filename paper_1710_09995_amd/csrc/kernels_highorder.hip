// High-order pieces of the paper's WCNS-E-5 scheme (Section 2.2), as operators
// on one block's fields along one index direction d:
//   - Eq. (2), the sixth-order staggered flux difference: the derivative at
//     the n cells from n + 5 face values,
//       out_i = [75/64 (F_{i+1/2} - F_{i-1/2}) - 25/384 (F_{i+3/2} - F_{i-3/2})
//                + 3/640 (F_{i+5/2} - F_{i-5/2})] / h;
//   - the fifth-order weighted cell-edge interpolation of WCNS-E-5: left and
//     right states at m faces from m + 5 cell values (the published
//     construction of the scheme; the paper names it without printing it).
// Both read a window of six consecutive entries along d per output entry p
// (entries p .. p + 5), so they share two kernel skeletons: along i a
// workgroup stages 4 rows of 261 entries in LDS (coalesced, all loads in
// flight before one barrier); along j and k each lane marches 16 outputs of
// its i-column with a register window of 21 entries.  Each input entry is thus
// loaded about once instead of six times.  With a grid that is a multiple of
// 8, each XCD (workgroup id mod 8) streams one contiguous eighth of the work.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdint>
#include <string>

#include "../../include/cfd.h"
#include "host_services.hpp"
#include "physics.hpp"

namespace cfd {

__device__ __forceinline__ int xcd_slot(int nb, int b) {
  return (nb & 7) == 0 ? (b & 7) * (nb >> 3) + (b >> 3) : b;
}

// Eq. (2): one output per window; ACC adds it to the output (sums over
// directions) instead of storing it.
template <bool ACC_>
struct Eq2OpT {
  static constexpr int NOUT = 1;
  static constexpr bool ACC = ACC_;
  double c1, c2, c3;
  __device__ __forceinline__ void operator()(const double* w, double* o) const {
    o[0] = c1 * (w[3] - w[2]) + c2 * (w[4] - w[1]) + c3 * (w[5] - w[0]);
  }
};

// WCNS-E-5 left state at the face between u0 and up1: three 3-cell Taylor
// candidates u0 + (h/2) g + (h^2/8) s, smoothness (h g)^2 + (h^2 s)^2, linear
// weights 1/16, 10/16, 5/16 made nonlinear by d_k / (eps + beta_k)^2.  Four
// refined hardware reciprocals (frcp, within 1 ulp) instead of six divisions.
__device__ __forceinline__ double wcns5_left(double um2, double um1, double u0, double up1, double up2, double eps) {
  const double g0 = (um2 - 4.0 * um1 + 3.0 * u0) / 2.0, g1 = (up1 - um1) / 2.0,
               g2 = (-3.0 * u0 + 4.0 * up1 - up2) / 2.0;
  const double s0 = um2 - 2.0 * um1 + u0, s1 = um1 - 2.0 * u0 + up1, s2 = u0 - 2.0 * up1 + up2;
  const double c0 = u0 + 0.5 * g0 + 0.125 * s0, c1 = u0 + 0.5 * g1 + 0.125 * s1, c2 = u0 + 0.5 * g2 + 0.125 * s2;
  const double b0 = eps + g0 * g0 + s0 * s0, b1 = eps + g1 * g1 + s1 * s1, b2 = eps + g2 * g2 + s2 * s2;
  const double a0 = (1.0 / 16.0) * frcp(b0 * b0), a1 = (10.0 / 16.0) * frcp(b1 * b1),
               a2 = (5.0 / 16.0) * frcp(b2 * b2);
  const double it = frcp(a0 + a1 + a2);
  return (a0 * it) * c0 + (a1 * it) * c1 + (a2 * it) * c2;
}

// The window of face p spans cells p .. p + 5; the face lies between the
// third and fourth.  Left state from cells p .. p + 4, right from p + 5 .. p + 1.
struct Wcns5Op {
  static constexpr int NOUT = 2;
  static constexpr bool ACC = false;
  double eps;
  __device__ __forceinline__ void operator()(const double* w, double* o) const {
    o[0] = wcns5_left(w[0], w[1], w[2], w[3], w[4], eps);
    o[1] = wcns5_left(w[5], w[4], w[3], w[2], w[1], eps);
  }
};

// Along i.  Output extents mi x mj x mk per variable (row = (v, k, j)); the
// input has mi + 5 entries along i.  Workgroup w takes a SEG-entry segment of
// RI consecutive rows; SEG = 264 lets one workgroup cover rows of up to 264
// outputs (256 cells plus the 5 extra faces of the edge interpolation),
// lanes 0..7 taking a second output.
constexpr int RI = 4;
constexpr int SEG = 264;
template <class Op>
__global__ void __launch_bounds__(256) k_window6_i(const double* __restrict__ in, double* __restrict__ out0,
                                                   double* __restrict__ out1, int mi, int nseg, int nrows, Op op) {
  __shared__ double sw[RI][SEG + 5];
  const int w = xcd_slot(gridDim.x, blockIdx.x);
  const int rg = w / nseg, seg = w - rg * nseg;
  const int i0 = seg * SEG, t = (int)threadIdx.x;
  const int64_t ei = mi + 5;
#pragma unroll
  for (int q = 0; q < RI; ++q) {
    const int row = rg * RI + q;
    const double* r = in + (int64_t)row * ei;
    for (int s = t; s < SEG + 5; s += 256) sw[q][s] = row < nrows && i0 + s < mi + 5 ? r[i0 + s] : 0.0;
  }
  __syncthreads();
  for (int tt = t; tt < SEG; tt += 256) {
    const int i = i0 + tt;
    if (i >= mi) break;
#pragma unroll
    for (int q = 0; q < RI; ++q) {
      const int row = rg * RI + q;
      if (row >= nrows) continue;
      double o[Op::NOUT];
      op(&sw[q][tt], o);
      const int64_t at = (int64_t)row * mi + i;
      if constexpr (Op::ACC) out0[at] += o[0]; else out0[at] = o[0];
      if constexpr (Op::NOUT > 1) out1[at] = o[Op::NOUT - 1];
    }
  }
}

// Along j (d = 1) or k (d = 2).  Output extents mi x mj x mk per variable; the
// input has 5 more entries along d.  Workgroup w takes a 256-entry i-segment
// of one chunk of CH outputs of one line (v, the other transverse index).
template <class Op, int CH>
__global__ void __launch_bounds__(256) k_window6_march(const double* __restrict__ in, double* __restrict__ out0,
                                                       double* __restrict__ out1, int mi, int mj, int mk, int d,
                                                       int nseg, int nchunk, Op op) {
  const int w = xcd_slot(gridDim.x, blockIdx.x);
  const int seg = w % nseg;
  int r = w / nseg;
  const int chunk = r % nchunk;
  r /= nchunk;
  const int i = seg * 256 + (int)threadIdx.x;
  if (i >= mi) return;
  const int md = d == 1 ? mj : mk;                  // outputs along the direction
  const int mo = d == 1 ? mk : mj;                  // the other transverse extent
  const int o2 = r % mo, v = r / mo;
  const int j = d == 1 ? 0 : o2, k = d == 1 ? o2 : 0;
  const int64_t ej = mj + (d == 1 ? 5 : 0), ek = mk + (d == 2 ? 5 : 0);
  const int64_t sin_ = d == 1 ? (int64_t)mi : (int64_t)mi * ej;       // input stride along d
  const int64_t sout = d == 1 ? (int64_t)mi : (int64_t)mi * mj;       // output stride along d
  const double* ip = in + (((int64_t)v * ek + k) * ej + j) * mi + i;  // input entry 0 of this line
  const int64_t ob = (((int64_t)v * mk + k) * mj + j) * mi + i;      // output entry 0 of this line
  const int c0 = chunk * CH;
  double win[CH + 5];
#pragma unroll
  for (int s = 0; s < CH + 5; ++s) win[s] = c0 + s < md + 5 ? ip[(c0 + s) * sin_] : 0.0;
#pragma unroll
  for (int s = 0; s < CH; ++s) {
    if (c0 + s >= md) break;
    double o[Op::NOUT];
    op(&win[s], o);
    const int64_t at = ob + (int64_t)(c0 + s) * sout;
    if constexpr (Op::ACC) out0[at] += o[0]; else out0[at] = o[0];
    if constexpr (Op::NOUT > 1) out1[at] = o[Op::NOUT - 1];
  }
}

// Launch an operator over output extents m (per variable) along direction d.
template <class Op>
void launch_window6(const double* in, double* out0, double* out1, const int64_t m[3], int d, int nvar, const Op& op,
                    hipStream_t stream) {
  if (d == 0) {
    const int64_t nseg = (m[0] + SEG - 1) / SEG;
    const int64_t nrows = (int64_t)nvar * m[1] * m[2];
    const int64_t nwork = nseg * ((nrows + RI - 1) / RI);
    if (nwork > INT32_MAX || nrows > INT32_MAX) host_fail(CFD_EINVAL, "field too large");
    hipLaunchKernelGGL(k_window6_i<Op>, dim3((unsigned)nwork), dim3(256), 0, stream, in, out0, out1, (int)m[0],
                       (int)nseg, (int)nrows, op);
  } else {
    const int64_t nseg = (m[0] + 255) / 256;
    constexpr int CH = 16;
    const int64_t nchunk = (m[d] + CH - 1) / CH;
    const int64_t nwork = nseg * nchunk * nvar * (d == 1 ? m[2] : m[1]);
    if (nwork > INT32_MAX) host_fail(CFD_EINVAL, "field too large");
    hipLaunchKernelGGL((k_window6_march<Op, CH>), dim3((unsigned)nwork), dim3(256), 0, stream, in, out0, out1,
                       (int)m[0], (int)m[1], (int)m[2], d, (int)nseg, (int)nchunk, op);
  }
  const hipError_t e = hipGetLastError();
  if (e != hipSuccess) host_fail(CFD_EHIP, std::string("kernel launch failed: ") + hipGetErrorString(e));
}

// Primitive variables of a periodic block, padded by five cells on each side
// along d: W[v][...p...] = prim(Q at cell (p - 5) mod n_d), p = 0 .. n_d + 9.
__global__ void __launch_bounds__(256) k_pad_prim_periodic(const double* __restrict__ q, double* __restrict__ w,
                                                           int ni, int nj, int nk, int d, double gm1) {
  const int64_t ei = ni + (d == 0 ? 10 : 0), ej = nj + (d == 1 ? 10 : 0), ek = nk + (d == 2 ? 10 : 0);
  const int64_t total = ei * ej * ek, cells = (int64_t)ni * nj * nk;
  for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < total; t += (int64_t)gridDim.x * blockDim.x) {
    int64_t a = t % ei, r = t / ei;
    int64_t b = r % ej, c = r / ej;
    if (d == 0) a = (a - 5 + 5 * (int64_t)ni) % ni;
    if (d == 1) b = (b - 5 + 5 * (int64_t)nj) % nj;
    if (d == 2) c = (c - 5 + 5 * (int64_t)nk) % nk;
    const int64_t src = (c * nj + b) * ni + a;
    const Prim<double> p = to_prim<double>(q[src], q[cells + src], q[2 * cells + src], q[3 * cells + src],
                                           q[4 * cells + src], gm1);
    w[t] = p.r;
    w[total + t] = p.u;
    w[2 * total + t] = p.v;
    w[3 * total + t] = p.w;
    w[4 * total + t] = p.p;
  }
}

// Roe's flux per unit area through faces of unit normal e_d, from the left
// and right primitive states (each [5][nf]).
__global__ void __launch_bounds__(256) k_roe_faces(const double* __restrict__ wl, const double* __restrict__ wr,
                                                   double* __restrict__ f, int64_t nf, int d, Gas<double> gas) {
  for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < nf; t += (int64_t)gridDim.x * blockDim.x) {
    const Prim<double> L{wl[t], wl[nf + t], wl[2 * nf + t], wl[3 * nf + t], wl[4 * nf + t]};
    const Prim<double> R{wr[t], wr[nf + t], wr[2 * nf + t], wr[3 * nf + t], wr[4 * nf + t]};
    double fl[5];
    roe<double>(L, R, d == 0 ? 1.0 : 0.0, d == 1 ? 1.0 : 0.0, d == 2 ? 1.0 : 0.0, gas, fl);
    for (int v = 0; v < 5; ++v) f[v * nf + t] = fl[v];
  }
}

int grid_for(int64_t n) { return (int)std::min<int64_t>((n + 255) / 256, 8192); }

// One Runge-Kutta stage of Eqs. (4)-(6) with lambda = -dt, in place:
// q <- a qn + b (q - dt r) (a = 0, b = 1: the first stage; then 3/4, 1/4 and
// 1/3, 2/3).  keep_qn also stores q into qn first (the step's start state).
__global__ void __launch_bounds__(256) k_rk3_stage(double* __restrict__ q, double* __restrict__ qn,
                                                   const double* __restrict__ r, int64_t n, double dt, double a,
                                                   double b, int keep_qn) {
  for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < n; t += (int64_t)gridDim.x * blockDim.x) {
    const double x = q[t], y = r[t];
    const double s = x - dt * y;
    if (keep_qn) {
      qn[t] = x;
      q[t] = s;
    } else {
      q[t] = a * qn[t] + b * s;
    }
  }
}

// Workspace of the periodic WCNS-E-5 residual (doubles): the padded primitives
// and the two face states and the face flux of the largest direction.
void wcns5_work(const int32_t n[3], int64_t& pmax, int64_t& fmax) {
  const int64_t cells = (int64_t)n[0] * n[1] * n[2];
  pmax = fmax = 0;
  for (int d = 0; d < 3; ++d) {
    pmax = std::max(pmax, 5 * (cells / n[d]) * (n[d] + 10));
    fmax = std::max(fmax, 5 * (cells / n[d]) * (n[d] + 5));
  }
}

// Shared argument checks: direction, extents, variables, and that the input
// range (in_elems doubles) and the output ranges (out_elems each) are disjoint.
void check_window6(const void* in, int64_t in_elems, const void* const* outs, int nout, int64_t out_elems,
                   const int32_t n[3], int32_t d, int32_t nvar) {
  if (!in) host_fail(CFD_EINVAL, "NULL argument");
  for (int q = 0; q < nout; ++q)
    if (!outs[q]) host_fail(CFD_EINVAL, "NULL argument");
  if (n[0] < 1 || n[1] < 1 || n[2] < 1) host_fail(CFD_EINVAL, "every extent must be >= 1");
  if (nvar < 1 || nvar > 64) host_fail(CFD_EINVAL, "nvar must be in [1, 64]");
  if (in_elems > ((int64_t)1 << 40)) host_fail(CFD_EINVAL, "field too large");
  auto overlap = [](const void* a, int64_t na, const void* b, int64_t nb) {
    const char *a0 = static_cast<const char*>(a), *b0 = static_cast<const char*>(b);
    return a0 < b0 + nb * 8 && b0 < a0 + na * 8;
  };
  for (int q = 0; q < nout; ++q) {
    if (overlap(in, in_elems, outs[q], out_elems)) host_fail(CFD_EINVAL, "input and output overlap");
    for (int r = q + 1; r < nout; ++r)
      if (overlap(outs[q], out_elems, outs[r], out_elems)) host_fail(CFD_EINVAL, "outputs overlap");
  }
}

// Entries of a field with extents m per variable and 5 more along d.
int64_t padded_elems(const int64_t m[3], int d, int nvar) {
  int64_t e[3] = {m[0], m[1], m[2]};
  e[d] += 5;
  return e[0] * e[1] * e[2] * nvar;
}

}  // namespace cfd

extern "C" cfd_status cfd_staggered_diff6(const double* f_dev, double* out_dev, const int32_t n[3], int32_t d,
                                          int32_t nvar, double h, hipStream_t stream) {
  return cfd::host_guarded([&] {
    if (!n) cfd::host_fail(CFD_EINVAL, "NULL argument");
    if (d < 0 || d > 2) cfd::host_fail(CFD_EINVAL, "direction must be 0, 1 or 2");
    if (!(h > 0.0) || !std::isfinite(h)) cfd::host_fail(CFD_EINVAL, "h must be positive and finite");
    const int64_t m[3] = {n[0], n[1], n[2]};          // the cells
    const void* outs[1] = {out_dev};
    cfd::check_window6(f_dev, cfd::padded_elems(m, d, nvar), outs, 1, m[0] * m[1] * m[2] * nvar, n, d, nvar);
    const cfd::Eq2OpT<false> op{75.0 / (64.0 * h), -25.0 / (384.0 * h), 3.0 / (640.0 * h)};
    cfd::launch_window6(f_dev, out_dev, nullptr, m, d, nvar, op, stream);
  });
}

extern "C" cfd_status cfd_wcns5_edges(const double* u_dev, double* left_dev, double* right_dev, const int32_t n[3],
                                      int32_t d, int32_t nvar, double eps, hipStream_t stream) {
  return cfd::host_guarded([&] {
    if (!n) cfd::host_fail(CFD_EINVAL, "NULL argument");
    if (d < 0 || d > 2) cfd::host_fail(CFD_EINVAL, "direction must be 0, 1 or 2");
    if (!(eps > 0.0) || !std::isfinite(eps)) cfd::host_fail(CFD_EINVAL, "eps must be positive and finite");
    int64_t m[3] = {n[0], n[1], n[2]};
    m[d] += 5;                                        // the faces i - 1/2, i = -2 .. n[d] + 2
    const void* outs[2] = {left_dev, right_dev};
    cfd::check_window6(u_dev, cfd::padded_elems(m, d, nvar), outs, 2, m[0] * m[1] * m[2] * nvar, n, d, nvar);
    cfd::launch_window6(u_dev, left_dev, right_dev, m, d, nvar, cfd::Wcns5Op{eps}, stream);
  });
}

extern "C" cfd_status cfd_wcns5_euler_work_bytes(const int32_t n[3], size_t* bytes) {
  return cfd::host_guarded([&] {
    if (!n || !bytes) cfd::host_fail(CFD_EINVAL, "NULL argument");
    if (n[0] < 1 || n[1] < 1 || n[2] < 1) cfd::host_fail(CFD_EINVAL, "every extent must be >= 1");
    int64_t pmax, fmax;
    cfd::wcns5_work(n, pmax, fmax);
    *bytes = (size_t)(8 * (pmax + 3 * fmax));
  });
}

extern "C" cfd_status cfd_wcns5_euler_residual_periodic(const double* q_dev, double* r_dev, void* work_dev,
                                                        size_t work_bytes, const int32_t n[3], const double h[3],
                                                        double gamma, double entropy_fix, double eps,
                                                        hipStream_t stream) {
  return cfd::host_guarded([&] {
    if (!q_dev || !r_dev || !work_dev || !n || !h) cfd::host_fail(CFD_EINVAL, "NULL argument");
    if (n[0] < 1 || n[1] < 1 || n[2] < 1) cfd::host_fail(CFD_EINVAL, "every extent must be >= 1");
    for (int d = 0; d < 3; ++d)
      if (!(h[d] > 0.0) || !std::isfinite(h[d])) cfd::host_fail(CFD_EINVAL, "spacings must be positive and finite");
    if (!(gamma > 1.0) || !std::isfinite(gamma)) cfd::host_fail(CFD_EINVAL, "gamma must exceed 1");
    if (!(entropy_fix >= 0.0) || !std::isfinite(entropy_fix)) cfd::host_fail(CFD_EINVAL, "bad entropy_fix");
    if (!(eps > 0.0) || !std::isfinite(eps)) cfd::host_fail(CFD_EINVAL, "eps must be positive and finite");
    int64_t pmax, fmax;
    cfd::wcns5_work(n, pmax, fmax);
    const size_t need = (size_t)(8 * (pmax + 3 * fmax));
    if (work_bytes < need) cfd::host_fail(CFD_ENOMEM, "workspace smaller than cfd_wcns5_euler_work_bytes()");
    const int64_t cells = (int64_t)n[0] * n[1] * n[2];
    auto apart = [](const void* a, int64_t na, const void* b, int64_t nb) {
      const char *a0 = static_cast<const char*>(a), *b0 = static_cast<const char*>(b);
      return a0 + na <= b0 || b0 + nb <= a0;
    };
    if (!apart(q_dev, 40 * cells, r_dev, 40 * cells) || !apart(q_dev, 40 * cells, work_dev, (int64_t)need) ||
        !apart(r_dev, 40 * cells, work_dev, (int64_t)need))
      cfd::host_fail(CFD_EINVAL, "q, r and the workspace must not overlap");
    double* W = static_cast<double*>(work_dev);
    double* WL = W + pmax;
    double* WR = WL + fmax;
    double* F = WR + fmax;
    cfd::Gas<double> gas{};
    gas.gamma = gamma;
    gas.gm1 = gamma - 1.0;
    gas.gg = gamma / (gamma - 1.0);
    gas.eps_h = entropy_fix;
    for (int d = 0; d < 3; ++d) {
      int64_t mp[3] = {n[0], n[1], n[2]}, mf[3] = {n[0], n[1], n[2]};
      mp[d] += 10;
      mf[d] += 5;
      const int64_t nf = mf[0] * mf[1] * mf[2];
      hipLaunchKernelGGL(cfd::k_pad_prim_periodic, dim3(cfd::grid_for(mp[0] * mp[1] * mp[2])), dim3(256), 0, stream,
                         q_dev, W, n[0], n[1], n[2], d, gamma - 1.0);
      cfd::launch_window6(W, WL, WR, mf, d, 5, cfd::Wcns5Op{eps}, stream);
      hipLaunchKernelGGL(cfd::k_roe_faces, dim3(cfd::grid_for(nf)), dim3(256), 0, stream, WL, WR, F, nf, d, gas);
      const int64_t m[3] = {n[0], n[1], n[2]};
      const double c1 = 75.0 / (64.0 * h[d]), c2 = -25.0 / (384.0 * h[d]), c3 = 3.0 / (640.0 * h[d]);
      if (d == 0)
        cfd::launch_window6(F, r_dev, nullptr, m, d, 5, cfd::Eq2OpT<false>{c1, c2, c3}, stream);
      else
        cfd::launch_window6(F, r_dev, nullptr, m, d, 5, cfd::Eq2OpT<true>{c1, c2, c3}, stream);
    }
  });
}

namespace {

size_t wcns5_residual_work(const int32_t n[3]) {
  int64_t pmax, fmax;
  cfd::wcns5_work(n, pmax, fmax);
  return (size_t)(8 * (pmax + 3 * fmax));
}

}  // namespace

extern "C" cfd_status cfd_wcns5_euler_step_work_bytes(const int32_t n[3], size_t* bytes) {
  return cfd::host_guarded([&] {
    if (!n || !bytes) cfd::host_fail(CFD_EINVAL, "NULL argument");
    if (n[0] < 1 || n[1] < 1 || n[2] < 1) cfd::host_fail(CFD_EINVAL, "every extent must be >= 1");
    *bytes = wcns5_residual_work(n) + (size_t)2 * 40 * ((size_t)n[0] * n[1] * n[2]);
  });
}

extern "C" cfd_status cfd_wcns5_euler_steps_periodic(double* q_dev, void* work_dev, size_t work_bytes,
                                                     const int32_t n[3], const double h[3], double gamma,
                                                     double entropy_fix, double eps, double dt, int32_t nsteps,
                                                     hipStream_t stream) {
  return cfd::host_guarded([&] {
    if (!q_dev || !work_dev || !n || !h) cfd::host_fail(CFD_EINVAL, "NULL argument");
    if (n[0] < 1 || n[1] < 1 || n[2] < 1) cfd::host_fail(CFD_EINVAL, "every extent must be >= 1");
    if (!(dt > 0.0) || !std::isfinite(dt)) cfd::host_fail(CFD_EINVAL, "dt must be positive and finite");
    if (nsteps < 0) cfd::host_fail(CFD_EINVAL, "nsteps must be >= 0");
    const int64_t cells = (int64_t)n[0] * n[1] * n[2];
    const size_t rw = wcns5_residual_work(n);
    if (work_bytes < rw + (size_t)2 * 40 * cells)
      cfd::host_fail(CFD_ENOMEM, "workspace smaller than cfd_wcns5_euler_step_work_bytes()");
    const char *qa = reinterpret_cast<const char*>(q_dev), *wa = static_cast<const char*>(work_dev);
    if (qa < wa + work_bytes && wa < qa + 40 * cells) cfd::host_fail(CFD_EINVAL, "q and the workspace overlap");
    double* qn = reinterpret_cast<double*>(static_cast<char*>(work_dev) + rw);
    double* r = qn + 5 * cells;
    const int64_t nv = 5 * cells;
    const int g = cfd::grid_for(nv);
    const double a[3] = {0.0, 0.75, 1.0 / 3.0}, b[3] = {1.0, 0.25, 2.0 / 3.0};
    for (int it = 0; it < nsteps; ++it)
      for (int st = 0; st < 3; ++st) {
        const cfd_status s = cfd_wcns5_euler_residual_periodic(q_dev, r, work_dev, rw, n, h, gamma, entropy_fix,
                                                               eps, stream);
        if (s != CFD_OK) cfd::host_fail(s, cfd_last_error(nullptr));
        hipLaunchKernelGGL(cfd::k_rk3_stage, dim3(g), dim3(256), 0, stream, q_dev, qn, r, nv, dt, a[st], b[st],
                           st == 0 ? 1 : 0);
      }
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) cfd::host_fail(CFD_EHIP, std::string("kernel launch failed: ") + hipGetErrorString(e));
  });
}

// ------------------------------------------- fourth-order central viscous terms
// The paper takes the viscous flux derivatives by fourth-order central
// differencing; on a uniform periodic grid the textbook forms, all exact for
// cubics: cell derivative (f_{i-2} - 8 f_{i-1} + 8 f_{i+1} - f_{i+2}) / 12h,
// face value (-f_{i-1} + 9 f_i + 9 f_{i+1} - f_{i+2}) / 16, face derivative
// (f_{i-1} - 27 f_i + 27 f_{i+1} - f_{i+2}) / 24h, and the flux difference
// (F_{i-3/2} - 27 F_{i-1/2} + 27 F_{i+1/2} - F_{i+3/2}) / 24h, a face array
// holding face i + 1/2 at index i.  Stress, Sutherland viscosity and
// conduction as in the finite-volume path.
namespace cfd {

struct Cells3 {
  int n[3];
  __device__ __forceinline__ int64_t at(int i, int j, int k) const {
    return ((int64_t)k * n[1] + j) * n[0] + i;
  }
  // index of the cell s steps from (i, j, k) along d, periodic
  __device__ __forceinline__ int64_t step(int i, int j, int k, int d, int s) const {
    int c[3] = {i, j, k};
    c[d] = ((c[d] + s) % n[d] + n[d]) % n[d];
    return at(c[0], c[1], c[2]);
  }
};

__global__ void __launch_bounds__(256) k_c4_phi(const double* __restrict__ q, double* __restrict__ phi, int64_t cells,
                                                double gm1) {
  for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < cells; t += (int64_t)gridDim.x * blockDim.x) {
    const Prim<double> p = to_prim<double>(q[t], q[cells + t], q[2 * cells + t], q[3 * cells + t], q[4 * cells + t],
                                           gm1);
    phi[t] = p.u;
    phi[cells + t] = p.v;
    phi[2 * cells + t] = p.w;
    phi[3 * cells + t] = p.p / p.r;
  }
}

// g[(a * 3 + t) * cells + c] = d phi_a / d x_t at cell c.
__global__ void __launch_bounds__(256) k_c4_grads(const double* __restrict__ phi, double* __restrict__ g, Cells3 C,
                                                  double ih0, double ih1, double ih2) {
  const int64_t cells = (int64_t)C.n[0] * C.n[1] * C.n[2];
  const double ih[3] = {ih0, ih1, ih2};
  for (int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; c < cells; c += (int64_t)gridDim.x * blockDim.x) {
    const int i = (int)(c % C.n[0]), j = (int)((c / C.n[0]) % C.n[1]), k = (int)(c / ((int64_t)C.n[0] * C.n[1]));
    for (int t = 0; t < 3; ++t) {
      const int64_t m2 = C.step(i, j, k, t, -2), m1 = C.step(i, j, k, t, -1), p1 = C.step(i, j, k, t, 1),
                    p2 = C.step(i, j, k, t, 2);
      for (int a = 0; a < 4; ++a) {
        const double* f = phi + a * cells;
        g[(a * 3 + t) * cells + c] = (f[m2] - 8.0 * f[m1] + 8.0 * f[p1] - f[p2]) * (ih[t] / 12.0);
      }
    }
  }
}

// Viscous flux (momentum x, y, z and energy) through face i + 1/2 along d,
// stored at the index of cell i.
__global__ void __launch_bounds__(256) k_c4_visc_faces(const double* __restrict__ phi, const double* __restrict__ g,
                                                       double* __restrict__ fv, Cells3 C, int d, double ihd,
                                                       Gas<double> gas) {
  const int64_t cells = (int64_t)C.n[0] * C.n[1] * C.n[2];
  for (int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; c < cells; c += (int64_t)gridDim.x * blockDim.x) {
    const int i = (int)(c % C.n[0]), j = (int)((c / C.n[0]) % C.n[1]), k = (int)(c / ((int64_t)C.n[0] * C.n[1]));
    const int64_t m1 = C.step(i, j, k, d, -1), p1 = C.step(i, j, k, d, 1), p2 = C.step(i, j, k, d, 2);
    double pf[4], grad[4][3];
    for (int a = 0; a < 4; ++a) {
      const double* f = phi + a * cells;
      pf[a] = (-f[m1] + 9.0 * f[c] + 9.0 * f[p1] - f[p2]) / 16.0;
      for (int t = 0; t < 3; ++t) {
        if (t == d) {
          grad[a][t] = (f[m1] - 27.0 * f[c] + 27.0 * f[p1] - f[p2]) * (ihd / 24.0);
        } else {
          const double* gt = g + (a * 3 + t) * cells;
          grad[a][t] = (-gt[m1] + 9.0 * gt[c] + 9.0 * gt[p1] - gt[p2]) / 16.0;
        }
      }
    }
    const double T = pf[3];
    const double mu = gas.mu_inf * T * sqrt(T) * (1.0 + gas.s_star) / (T + gas.s_star);
    const double kc = mu * gas.kfac;
    const double div = grad[0][0] + grad[1][1] + grad[2][2];
    double tau[3];
    for (int b = 0; b < 3; ++b) tau[b] = mu * (grad[d][b] + grad[b][d]);
    tau[d] = tau[d] - (2.0 / 3.0) * mu * div;
    fv[c] = tau[0];
    fv[cells + c] = tau[1];
    fv[2 * cells + c] = tau[2];
    fv[3 * cells + c] = pf[0] * tau[0] + pf[1] * tau[1] + pf[2] * tau[2] + kc * grad[3][d];
  }
}

// r[1 + v] -= (F_{i-3/2} - 27 F_{i-1/2} + 27 F_{i+1/2} - F_{i+3/2}) / 24h, v = 0..3.
__global__ void __launch_bounds__(256) k_c4_flux_sub(const double* __restrict__ fv, double* __restrict__ r, Cells3 C,
                                                     int d, double ihd) {
  const int64_t cells = (int64_t)C.n[0] * C.n[1] * C.n[2];
  for (int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; c < cells; c += (int64_t)gridDim.x * blockDim.x) {
    const int i = (int)(c % C.n[0]), j = (int)((c / C.n[0]) % C.n[1]), k = (int)(c / ((int64_t)C.n[0] * C.n[1]));
    const int64_t m2 = C.step(i, j, k, d, -2), m1 = C.step(i, j, k, d, -1), p1 = C.step(i, j, k, d, 1);
    for (int v = 0; v < 4; ++v) {
      const double* F = fv + v * cells;
      r[(1 + v) * cells + c] -= (F[m2] - 27.0 * F[m1] + 27.0 * F[c] - F[p1]) * (ihd / 24.0);
    }
  }
}

}  // namespace cfd

extern "C" cfd_status cfd_c4_viscous_work_bytes(const int32_t n[3], size_t* bytes) {
  return cfd::host_guarded([&] {
    if (!n || !bytes) cfd::host_fail(CFD_EINVAL, "NULL argument");
    if (n[0] < 1 || n[1] < 1 || n[2] < 1) cfd::host_fail(CFD_EINVAL, "every extent must be >= 1");
    *bytes = (size_t)8 * 20 * ((size_t)n[0] * n[1] * n[2]);      // phi (4), gradients (12), face flux (4)
  });
}

extern "C" cfd_status cfd_c4_viscous_add_periodic(const double* q_dev, double* r_dev, void* work_dev,
                                                  size_t work_bytes, const int32_t n[3], const double h[3],
                                                  double gamma, double prandtl, double mu_inf, double s_star,
                                                  hipStream_t stream) {
  return cfd::host_guarded([&] {
    if (!q_dev || !r_dev || !work_dev || !n || !h) cfd::host_fail(CFD_EINVAL, "NULL argument");
    if (n[0] < 1 || n[1] < 1 || n[2] < 1) cfd::host_fail(CFD_EINVAL, "every extent must be >= 1");
    for (int d = 0; d < 3; ++d)
      if (!(h[d] > 0.0) || !std::isfinite(h[d])) cfd::host_fail(CFD_EINVAL, "spacings must be positive and finite");
    if (!(gamma > 1.0) || !(prandtl > 0.0) || !(mu_inf >= 0.0) || !(s_star > 0.0) || !std::isfinite(mu_inf))
      cfd::host_fail(CFD_EINVAL, "bad gas parameters");
    const int64_t cells = (int64_t)n[0] * n[1] * n[2];
    const size_t need = (size_t)8 * 20 * cells;
    if (work_bytes < need) cfd::host_fail(CFD_ENOMEM, "workspace smaller than cfd_c4_viscous_work_bytes()");
    auto apart = [](const void* a, int64_t na, const void* b, int64_t nb) {
      const char *a0 = static_cast<const char*>(a), *b0 = static_cast<const char*>(b);
      return a0 + na <= b0 || b0 + nb <= a0;
    };
    if (!apart(q_dev, 40 * cells, r_dev, 40 * cells) || !apart(q_dev, 40 * cells, work_dev, (int64_t)need) ||
        !apart(r_dev, 40 * cells, work_dev, (int64_t)need))
      cfd::host_fail(CFD_EINVAL, "q, r and the workspace must not overlap");
    double* phi = static_cast<double*>(work_dev);
    double* g = phi + 4 * cells;
    double* fv = g + 12 * cells;
    cfd::Cells3 C{{n[0], n[1], n[2]}};
    cfd::Gas<double> gas{};
    gas.gamma = gamma;
    gas.gm1 = gamma - 1.0;
    gas.mu_inf = mu_inf;
    gas.s_star = s_star;
    gas.prandtl = prandtl;
    gas.kfac = gamma / ((gamma - 1.0) * prandtl);
    const int gr = cfd::grid_for(cells);
    hipLaunchKernelGGL(cfd::k_c4_phi, dim3(gr), dim3(256), 0, stream, q_dev, phi, cells, gamma - 1.0);
    hipLaunchKernelGGL(cfd::k_c4_grads, dim3(gr), dim3(256), 0, stream, phi, g, C, 1.0 / h[0], 1.0 / h[1], 1.0 / h[2]);
    for (int d = 0; d < 3; ++d) {
      hipLaunchKernelGGL(cfd::k_c4_visc_faces, dim3(gr), dim3(256), 0, stream, phi, g, fv, C, d, 1.0 / h[d], gas);
      hipLaunchKernelGGL(cfd::k_c4_flux_sub, dim3(gr), dim3(256), 0, stream, fv, r_dev, C, d, 1.0 / h[d]);
    }
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) cfd::host_fail(CFD_EHIP, std::string("kernel launch failed: ") + hipGetErrorString(e));
  });
}
