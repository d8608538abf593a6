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
// The residuals built from them run, on blocks large enough to fill the chip,
// as one pass per direction that keeps every intermediate on chip: an LDS row
// pass along i and register marches along j and k for the inviscid residual
// (primitives, edge states, Roe's flux, Eq. 2), the index derivatives of the
// viscous terms and their face fluxes with the staggered difference; smaller
// blocks take the padded-primitive, face and Eq. 2 passes, with the same bits.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdint>
#include <mutex>
#include <string>
#include <utility>
#include <vector>

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
  static constexpr bool DIV = false;
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
  static constexpr bool DIV = false;
  double eps;
  __device__ __forceinline__ void operator()(const double* w, double* o) const {
    o[0] = wcns5_left(w[0], w[1], w[2], w[3], w[4], eps);
    o[1] = wcns5_left(w[5], w[4], w[3], w[2], w[1], eps);
  }
};

// Eq. (2) added into the output, the sum then divided by J^{-1} of the cell:
// the last direction's pass of a curvilinear residual (along j or k only).
struct Eq2DivOp {
  static constexpr int NOUT = 1;
  static constexpr bool ACC = true;
  static constexpr bool DIV = true;
  double c1, c2, c3;
  const double* jinv;
  __device__ __forceinline__ void operator()(const double* w, double* o) const {
    o[0] = c1 * (w[3] - w[2]) + c2 * (w[4] - w[1]) + c3 * (w[5] - w[0]);
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
    if constexpr (Op::DIV) {
      out0[at] = (out0[at] + o[0]) / op.jinv[at - (int64_t)v * mi * mj * mk];
    } else if constexpr (Op::ACC) {
      out0[at] += o[0];
    } else {
      out0[at] = o[0];
    }
    if constexpr (Op::NOUT > 1) out1[at] = o[Op::NOUT - 1];
  }
}

// Launch an operator over output extents m (per variable) along direction d.
template <class Op>
void launch_window6(const double* in, double* out0, double* out1, const int64_t m[3], int d, int nvar, const Op& op,
                    hipStream_t stream) {
  if (Op::DIV && d == 0) host_fail(CFD_EINVAL, "the dividing Eq. 2 pass runs along j or k only");
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

int grid_for(int64_t n) { return (int)std::min<int64_t>((n + 255) / 256, 8192); }

// ------------------------------------------------------- curvilinear blocks
// Metrics of a periodic curvilinear block for the geometric conservation law
// the paper requires (Section 2.2).  Vertex v along a direction sits at index
// position v + 1/2, cells at integer positions.  D is Eq. (2) with h = 1 and
// I the sixth-order mid-point interpolation (150, -25, 3) / 256, both from six
// vertex positions to the centre position along one axis.  Face metrics in
// the symmetric conservative form
//   S_d = 1/2 [D_b (D_a X x I_a X) - D_a (D_b X x I_b X)], (a, b) = (d+1, d+2) mod 3,
// so that sum_d D_d S_d = 0 at every cell (D and I along different axes
// commute) and a uniform stream stays uniform; J^{-1} = det[X_xi X_eta X_zeta]
// at the cell, each column D along its axis of I along the other two.
constexpr double I1 = 150.0 / 256.0, I2 = -25.0 / 256.0, I3 = 3.0 / 256.0;
constexpr double E1 = 75.0 / 64.0, E2 = -25.0 / 384.0, E3 = 3.0 / 640.0;

struct PeriodicGrid {
  const double* xv;  // [3][nk][nj][ni]: vertex (i, j, k) is the upper corner of cell (i, j, k)
  int n[3];
  double P[3][3];    // P[d]: the displacement of the grid over one period along d
  // Coordinates of vertex (v0, v1, v2), any integers: the stored vertex of
  // the wrapped index plus the periods crossed.
  __device__ __forceinline__ void vertex(int v0, int v1, int v2, double X[3]) const {
    const int v[3] = {v0, v1, v2};
    int w[3];
    double q[3];
#pragma unroll
    for (int d = 0; d < 3; ++d) {
      const int qd = v[d] >= 0 ? v[d] / n[d] : -((-v[d] + n[d] - 1) / n[d]);
      w[d] = v[d] - qd * n[d];
      q[d] = (double)qd;
    }
    const int64_t cells = (int64_t)n[0] * n[1] * n[2];
    const int64_t idx = ((int64_t)w[2] * n[1] + w[1]) * n[0] + w[0];
#pragma unroll
    for (int c = 0; c < 3; ++c) X[c] = xv[c * cells + idx] + q[0] * P[0][c] + q[1] * P[1][c] + q[2] * P[2][c];
  }
};

// Coordinates from an explicit array of the vertices -3 .. n + 1 along each
// direction (a block of a larger grid: the caller supplies the vertices
// beyond its faces).  Every index the metric kernels ask for lies in that range.
struct ExtGrid {
  const double* xe;  // [3][nk + 5][nj + 5][ni + 5], vertex v at index v + 3
  int n[3];
  __device__ __forceinline__ void vertex(int v0, int v1, int v2, double X[3]) const {
    const int64_t e0 = n[0] + 5, e1 = n[1] + 5, ecells = e0 * e1 * (n[2] + 5);
    const int64_t idx = ((int64_t)(v2 + 3) * e1 + (v1 + 3)) * e0 + (v0 + 3);
#pragma unroll
    for (int c = 0; c < 3; ++c) X[c] = xe[c * ecells + idx];
  }
};

// D_a X x I_a X at position p (a centre along a, vertices along the others).
template <int A, class Grid>
__device__ __forceinline__ void metric_cross(const Grid& g, int p0, int p1, int p2, double out[3]) {
  double f[6][3];
#pragma unroll
  for (int m = 0; m < 6; ++m)
    g.vertex(p0 + (A == 0 ? m - 3 : 0), p1 + (A == 1 ? m - 3 : 0), p2 + (A == 2 ? m - 3 : 0), f[m]);
  double D[3], I[3];
#pragma unroll
  for (int c = 0; c < 3; ++c) {
    D[c] = E1 * (f[3][c] - f[2][c]) + E2 * (f[4][c] - f[1][c]) + E3 * (f[5][c] - f[0][c]);
    I[c] = I1 * (f[3][c] + f[2][c]) + I2 * (f[4][c] + f[1][c]) + I3 * (f[5][c] + f[0][c]);
  }
  out[0] = D[1] * I[2] - D[2] * I[1];
  out[1] = D[2] * I[0] - D[0] * I[2];
  out[2] = D[0] * I[1] - D[1] * I[0];
}

// S_d at the faces of direction d: s[(d * 3 + c) * cells + cell] holds
// component c of the face v + 1/2 with v the cell's index along d.
template <int DIR, class Grid>
__global__ void __launch_bounds__(256) k_metric_faces(Grid g, double* __restrict__ s) {
  constexpr int A = (DIR + 1) % 3, B = (DIR + 2) % 3;
  const int64_t cells = (int64_t)g.n[0] * g.n[1] * g.n[2];
  for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < cells; t += (int64_t)gridDim.x * blockDim.x) {
    const int p[3] = {(int)(t % g.n[0]), (int)((t / g.n[0]) % g.n[1]), (int)(t / ((int64_t)g.n[0] * g.n[1]))};
    const double wd[6] = {-E3, -E2, -E1, E1, E2, E3};
    double t1[3] = {0.0, 0.0, 0.0}, t2[3] = {0.0, 0.0, 0.0};
#pragma unroll 1
    for (int k = 0; k < 6; ++k) {                   // D_b of (D_a X x I_a X)
      double m[3];
      metric_cross<A, Grid>(g, p[0] + (B == 0 ? k - 3 : 0), p[1] + (B == 1 ? k - 3 : 0), p[2] + (B == 2 ? k - 3 : 0),
                            m);
      const double w = k == 0 ? wd[0] : k == 1 ? wd[1] : k == 2 ? wd[2] : k == 3 ? wd[3] : k == 4 ? wd[4] : wd[5];
#pragma unroll
      for (int c = 0; c < 3; ++c) t1[c] += w * m[c];
    }
#pragma unroll 1
    for (int k = 0; k < 6; ++k) {                   // D_a of (D_b X x I_b X)
      double m[3];
      metric_cross<B, Grid>(g, p[0] + (A == 0 ? k - 3 : 0), p[1] + (A == 1 ? k - 3 : 0), p[2] + (A == 2 ? k - 3 : 0),
                            m);
      const double w = k == 0 ? wd[0] : k == 1 ? wd[1] : k == 2 ? wd[2] : k == 3 ? wd[3] : k == 4 ? wd[4] : wd[5];
#pragma unroll
      for (int c = 0; c < 3; ++c) t2[c] += w * m[c];
    }
#pragma unroll
    for (int c = 0; c < 3; ++c) s[(DIR * 3 + c) * cells + t] = 0.5 * (t1[c] - t2[c]);
  }
}

// J^{-1} at the cells: one pass over the 6 x 6 x 6 vertices around the cell,
// column d weighted by D along d and I along the other two.
template <class Grid>
__global__ void __launch_bounds__(256) k_metric_jinv(Grid g, double* __restrict__ jinv) {
  const double wd[6] = {-E3, -E2, -E1, E1, E2, E3};
  const double wi[6] = {I3, I2, I1, I1, I2, I3};
  const int64_t cells = (int64_t)g.n[0] * g.n[1] * g.n[2];
  for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < cells; t += (int64_t)gridDim.x * blockDim.x) {
    const int i = (int)(t % g.n[0]), j = (int)((t / g.n[0]) % g.n[1]), k = (int)(t / ((int64_t)g.n[0] * g.n[1]));
    double col[3][3] = {{0, 0, 0}, {0, 0, 0}, {0, 0, 0}};
    for (int r2 = 0; r2 < 6; ++r2)
      for (int r1 = 0; r1 < 6; ++r1) {
#pragma unroll
        for (int r0 = 0; r0 < 6; ++r0) {
          double X[3];
          g.vertex(i - 3 + r0, j - 3 + r1, k - 3 + r2, X);
          const double w0 = wd[r0] * wi[r1] * wi[r2], w1 = wi[r0] * wd[r1] * wi[r2], w2 = wi[r0] * wi[r1] * wd[r2];
#pragma unroll
          for (int c = 0; c < 3; ++c) {
            col[0][c] += w0 * X[c];
            col[1][c] += w1 * X[c];
            col[2][c] += w2 * X[c];
          }
        }
      }
    const double cx = col[1][1] * col[2][2] - col[1][2] * col[2][1];
    const double cy = col[1][2] * col[2][0] - col[1][0] * col[2][2];
    const double cz = col[1][0] * col[2][1] - col[1][1] * col[2][0];
    jinv[t] = col[0][0] * cx + col[0][1] * cy + col[0][2] * cz;
  }
}


// Blocks joined face to face.  Index of cell (a, b, c) of a block whose
// extent along d is nd and whose other extents are the caller's.
__device__ __forceinline__ int64_t seam_index(int a, int b, int c, int d, int nd, int n0, int n1) {
  const int64_t e0 = d == 0 ? nd : n0, e1 = d == 1 ? nd : n1;
  return ((int64_t)c * e1 + b) * e0 + a;
}

// Face states and Roe's flux in one pass: thread per face p of the face grid
// (m_d = n_d + 5 along d) reads the six padded cells p .. p + 5 of the five
// primitives (extents m with m_d + 5 along d), forms the WCNS-E-5 left and
// right states (Wcns5Op's arithmetic) and Roe's flux (per unit area through
// e_d, or through the face's area vector): the face states never leave
// registers.  Without
// metrics (s == NULL) the face normal is e_d and the flux per unit area;
// else the area vector of face v = p - 3 comes from the block (0 <= v < n_d)
// or the neighbour below (v + nlo) or above (v - n_d), whose cells counts
// are slo/shi (a periodic block passes itself).
__global__ void __launch_bounds__(256) k_wcns5_roe_faces(const double* __restrict__ w, double* __restrict__ f,
                                                         int m0, int m1, int m2, int d, double eps,
                                                         const double* __restrict__ s,
                                                         const double* __restrict__ slo,
                                                         const double* __restrict__ shi, int n0, int n1, int n2,
                                                         int nlo, int nhi, Gas<double> gas) {
  const int64_t nf = (int64_t)m0 * m1 * m2;
  const int64_t p0 = m0 + (d == 0 ? 5 : 0), p1 = m1 + (d == 1 ? 5 : 0);
  const int64_t np = p0 * p1 * (m2 + (d == 2 ? 5 : 0));
  const int64_t step = d == 0 ? 1 : (d == 1 ? p0 : p0 * p1);
  const int nd = d == 0 ? n0 : (d == 1 ? n1 : n2);
  for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < nf; t += (int64_t)gridDim.x * blockDim.x) {
    int a = (int)(t % m0), b = (int)((t / m0) % m1), c = (int)(t / ((int64_t)m0 * m1));
    const int64_t base = ((int64_t)c * p1 + b) * p0 + a;   // padded cell p of the window (index p along d)
    double L[5], R[5];
#pragma unroll
    for (int v = 0; v < 5; ++v) {
      const double* wv = w + v * np + base;
      const double u0 = wv[0], u1 = wv[step], u2 = wv[2 * step], u3 = wv[3 * step], u4 = wv[4 * step],
                   u5 = wv[5 * step];
      L[v] = wcns5_left(u0, u1, u2, u3, u4, eps);
      R[v] = wcns5_left(u5, u4, u3, u2, u1, eps);
    }
    const Prim<double> PL{L[0], L[1], L[2], L[3], L[4]};
    const Prim<double> PR{R[0], R[1], R[2], R[3], R[4]};
    double fl[5];
    if (!s) {
      roe<double>(PL, PR, d == 0 ? 1.0 : 0.0, d == 1 ? 1.0 : 0.0, d == 2 ? 1.0 : 0.0, gas, fl);
      for (int q = 0; q < 5; ++q) f[q * nf + t] = fl[q];
    } else {
      // v in [-3, n_d + 1]; a modulo (not one wrap) keeps a periodic block
      // thinner than three cells, which passes itself, inside its faces
      int v = (d == 0 ? a : (d == 1 ? b : c)) - 3;
      const double* src = s;
      int sd = nd;
      if (v < 0) {
        src = slo;
        sd = nlo;
        v = ((v % nlo) + nlo) % nlo;
      } else if (v >= nd) {
        src = shi;
        sd = nhi;
        v = (v - nd) % nhi;
      }
      if (d == 0) a = v;
      if (d == 1) b = v;
      if (d == 2) c = v;
      const int64_t scells = (int64_t)(d == 0 ? sd : n0) * (d == 1 ? sd : n1) * (d == 2 ? sd : n2);
      const int64_t ci = seam_index(a, b, c, d, sd, n0, n1);
      const double* sdv = src + 3 * d * scells;
      const double sx = sdv[ci], sy = sdv[scells + ci], sz = sdv[2 * scells + ci];
      const double area = fsqrt(sx * sx + sy * sy + sz * sz);
      const double ia = frcp(area);
      roe<double>(PL, PR, sx * ia, sy * ia, sz * ia, gas, fl);
      for (int q = 0; q < 5; ++q) f[q * nf + t] = fl[q] * area;
    }
  }
}

template <class Grid>
void launch_metrics(const Grid& g, double* s_dev, double* jinv_dev, int64_t cells, hipStream_t stream) {
  const dim3 grid(grid_for(cells));
  hipLaunchKernelGGL((k_metric_faces<0, Grid>), grid, dim3(256), 0, stream, g, s_dev);
  hipLaunchKernelGGL((k_metric_faces<1, Grid>), grid, dim3(256), 0, stream, g, s_dev);
  hipLaunchKernelGGL((k_metric_faces<2, Grid>), grid, dim3(256), 0, stream, g, s_dev);
  hipLaunchKernelGGL(k_metric_jinv<Grid>, grid, dim3(256), 0, stream, g, jinv_dev);
}


// Primitives padded by five cells on each side along d, those beyond the
// block taken from the neighbours across its two d-faces (qlo: its last five
// cells along d, qhi: its first five).
__global__ void __launch_bounds__(256) k_pad_prim_blocks(const double* __restrict__ q, const double* __restrict__ qlo,
                                                         const double* __restrict__ qhi, double* __restrict__ w,
                                                         int n0, int n1, int n2, int d, int nlo, int nhi,
                                                         double gm1) {
  const int nd = d == 0 ? n0 : (d == 1 ? n1 : n2);
  const int64_t e0 = n0 + (d == 0 ? 10 : 0), e1 = n1 + (d == 1 ? 10 : 0), e2 = n2 + (d == 2 ? 10 : 0);
  const int64_t total = e0 * e1 * e2;
  for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < total; t += (int64_t)gridDim.x * blockDim.x) {
    int a = (int)(t % e0), b = (int)((t / e0) % e1), c = (int)(t / (e0 * e1));
    int x = (d == 0 ? a : (d == 1 ? b : c)) - 5;
    const double* src = q;
    int sd = nd;
    if (x < 0) {
      src = qlo;
      sd = nlo;
      x += nlo;
    } else if (x >= nd) {
      src = qhi;
      sd = nhi;
      x -= nd;
    }
    if (d == 0) a = x;
    if (d == 1) b = x;
    if (d == 2) c = x;
    const int64_t scells = (int64_t)(d == 0 ? sd : n0) * (d == 1 ? sd : n1) * (d == 2 ? sd : n2);
    const int64_t i = seam_index(a, b, c, d, sd, n0, n1);
    const Prim<double> p = to_prim<double>(src[i], src[scells + i], src[2 * scells + i], src[3 * scells + i],
                                           src[4 * scells + i], gm1);
    w[t] = p.r;
    w[total + t] = p.u;
    w[2 * total + t] = p.v;
    w[3 * total + t] = p.w;
    w[4 * total + t] = p.p;
  }
}

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

// Workspace of the WCNS-E-5 residual (doubles): the padded primitives and the
// face flux of the largest direction.
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
    *bytes = (size_t)(8 * (pmax + fmax));
  });
}

namespace cfd {

bool apart(const void* a, int64_t na, const void* b, int64_t nb) {
  const char *a0 = static_cast<const char*>(a), *b0 = static_cast<const char*>(b);
  return a0 + na <= b0 || b0 + nb <= a0;
}

// Interior cells of block b of a dims table (3 entries per block).
int64_t block_cells(const int32_t* dims, int b) {
  return (int64_t)dims[3 * b] * dims[3 * b + 1] * dims[3 * b + 2];
}

// One argument buffer of a multi-block call: `bytes` bytes at p, written by
// the call or only read.
struct ArgSpan {
  uintptr_t p;
  int64_t bytes;
  bool written;
};
ArgSpan span(const void* p, int64_t bytes, bool written) {
  return ArgSpan{reinterpret_cast<uintptr_t>(p), bytes, written};
}

// Fails with msg when a written buffer overlaps any other one (read-only
// buffers may share memory).  In the order of start addresses a buffer
// overlaps an earlier one exactly when it starts below the largest end among
// them, so one pass after the sort checks all pairs: O(n log n) however many
// blocks a call names.
void check_spans(std::vector<ArgSpan>& v, const char* msg) {
  std::sort(v.begin(), v.end(), [](const ArgSpan& a, const ArgSpan& b) { return a.p < b.p; });
  uintptr_t end_any = 0, end_written = 0;
  for (const ArgSpan& a : v) {
    if (a.bytes <= 0) continue;
    if (a.p < end_written || (a.written && a.p < end_any)) host_fail(CFD_EINVAL, msg);
    const uintptr_t e = a.p + (uintptr_t)a.bytes;
    end_any = std::max(end_any, e);
    if (a.written) end_written = std::max(end_written, e);
  }
}

// A family of fields along direction d around a block: field f of the block
// at own[f * cown + cell], of the neighbours below and above at lo / hi
// (their extents along d nlo / nhi; the other extents are the block's).  A
// periodic block is its own neighbour.
struct Line {
  const double* own;
  const double* lo;
  const double* hi;
  int64_t cown, clo, chi;  // field strides: the cells of each block
  int nlo, nhi;            // the neighbours' extents along d
};

// Field f at the cell s steps along d from (i, j, k) of a block of extents n
// (|s| <= 2; a neighbour is at least five cells deep).
__device__ __forceinline__ double line_at(const Line& L, int f, int i, int j, int k, int s, int d, const int n[3]) {
  int c[3] = {i, j, k};
  int x = c[d] + s;
  const double* base = L.own;
  int64_t cells = L.cown;
  int nd = n[d];
  if (x < 0) {
    base = L.lo;
    cells = L.clo;
    x += L.nlo;
    nd = L.nlo;
  } else if (x >= n[d]) {
    base = L.hi;
    cells = L.chi;
    x -= n[d];
    nd = L.nhi;
  }
  c[d] = x;
  const int64_t e0 = d == 0 ? nd : n[0], e1 = d == 1 ? nd : n[1];
  return base[f * cells + ((int64_t)c[2] * e1 + c[1]) * e0 + c[0]];
}

struct Dims3 {
  int n[3];
};

// A neighbour resolved once: field f of the cell s steps along d is at
// base[f * cells + idx], whichever block holds it.
struct LineRef {
  const double* base;
  int64_t cells, idx;
  __device__ __forceinline__ double operator[](int f) const { return base[f * cells + idx]; }
};

__device__ __forceinline__ LineRef line_ref(const Line& L, int i, int j, int k, int s, int d, const int n[3]) {
  int c[3] = {i, j, k};
  int x = c[d] + s;
  LineRef r{L.own, L.cown, 0};
  int nd = n[d];
  if (x < 0) {
    r.base = L.lo;
    r.cells = L.clo;
    x += L.nlo;
    nd = L.nlo;
  } else if (x >= n[d]) {
    r.base = L.hi;
    r.cells = L.chi;
    x -= n[d];
    nd = L.nhi;
  }
  c[d] = x;
  const int64_t e0 = d == 0 ? nd : n[0], e1 = d == 1 ? nd : n[1];
  r.idx = ((int64_t)c[2] * e1 + c[1]) * e0 + c[0];
  return r;
}

// The cell s steps away along d (x = the coordinate along d, possibly outside
// the block): with a neighbour at least five cells deep one step across the
// seam; a block that is its own neighbour and thinner than the stencil wraps
// as often as needed (the periodic single block).
__device__ __forceinline__ LineRef wrap_ref(const Line& L, const int c0[3], int x, int d, const int n[3]) {
  int c[3] = {c0[0], c0[1], c0[2]};
  LineRef r{L.own, L.cown, 0};
  int nd = n[d];
  if (x < 0) {
    r.base = L.lo;
    r.cells = L.clo;
    nd = L.nlo;
    x += nd;
    if (x < 0) x = (x % nd + nd) % nd;
  } else if (x >= nd) {
    r.base = L.hi;
    r.cells = L.chi;
    x -= nd;
    nd = L.nhi;
    if (x >= nd) x %= nd;
  }
  c[d] = x;
  const int64_t e0 = d == 0 ? nd : n[0], e1 = d == 1 ? nd : n[1];
  r.idx = ((int64_t)c[2] * e1 + c[1]) * e0 + c[0];
  return r;
}

// The inviscid residual along d = 1 or 2 in one pass (Eq. 2 of the WCNS-E-5
// face fluxes): each thread marches a line of cells along d (lanes along i,
// coalesced rows) over a chunk of cells, converting each cell's state to
// primitives once, keeping the six cells around the current face and the last
// six face fluxes in registers, so neither the padded primitives nor the face
// fluxes go through memory.  Face v (between cells v and v + 1) takes its left
// state from cells v - 2 .. v + 2 and its right state from v + 3 .. v - 1
// (k_wcns5_roe_faces' arithmetic); cell x takes Eq. 2 of faces x - 3 .. x + 2.
// Q: the state arrays (5 fields) along d; S: the face metrics along d (own ==
// NULL: per unit area through e_d).  MODE 1: r += Eq. 2; MODE 2: r = (r +
// Eq. 2) / J^{-1} (the last direction of a curvilinear residual).
template <int D, int MODE>
__global__ void __launch_bounds__(256) k_wcns5_euler_march(Line Q, Line S, double* __restrict__ r,
                                                           const double* __restrict__ jinv, Dims3 Dm, int chunk,
                                                           double eps, double c1, double c2, double c3,
                                                           Gas<double> gas) {
  constexpr int O = D == 1 ? 2 : 1;
  const int* n = Dm.n;
  const int nD = n[D], nO = n[O], n0 = n[0];
  const int nch = (nD + chunk - 1) / chunk;
  const int64_t cells = (int64_t)n0 * n[1] * n[2];
  const int64_t total = (int64_t)n0 * nO * nch;
  for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < total; t += (int64_t)gridDim.x * blockDim.x) {
    int c0[3];
    c0[0] = (int)(t % n0);
    const int64_t rest = t / n0;
    c0[O] = (int)(rest % nO);
    c0[D] = 0;
    const int x0 = (int)(rest / nO) * chunk, x1 = min(x0 + chunk, nD);
    double W[6][5], F[6][5];
    auto load = [&](int x, double* w) {
      const LineRef q = wrap_ref(Q, c0, x, D, n);
      const Prim<double> p = to_prim<double>(q[0], q[1], q[2], q[3], q[4], gas.gm1);
      w[0] = p.r;
      w[1] = p.u;
      w[2] = p.v;
      w[3] = p.w;
      w[4] = p.p;
    };
#pragma unroll
    for (int k = 1; k < 6; ++k) load(x0 - 6 + k, W[k]);
    for (int v = x0 - 3; v <= x1 + 1; ++v) {
#pragma unroll
      for (int k = 0; k < 5; ++k)
#pragma unroll
        for (int q = 0; q < 5; ++q) {
          W[k][q] = W[k + 1][q];
          F[k][q] = F[k + 1][q];
        }
      load(v + 3, W[5]);
      double L[5], R[5];
#pragma unroll
      for (int q = 0; q < 5; ++q) {
        L[q] = wcns5_left(W[0][q], W[1][q], W[2][q], W[3][q], W[4][q], eps);
        R[q] = wcns5_left(W[5][q], W[4][q], W[3][q], W[2][q], W[1][q], eps);
      }
      const Prim<double> PL{L[0], L[1], L[2], L[3], L[4]};
      const Prim<double> PR{R[0], R[1], R[2], R[3], R[4]};
      double fl[5];
      if (!S.own) {
        roe<double>(PL, PR, D == 0 ? 1.0 : 0.0, D == 1 ? 1.0 : 0.0, D == 2 ? 1.0 : 0.0, gas, fl);
#pragma unroll
        for (int q = 0; q < 5; ++q) F[5][q] = fl[q];
      } else {
        const LineRef sr = wrap_ref(S, c0, v, D, n);
        const double sx = sr[3 * D], sy = sr[3 * D + 1], sz = sr[3 * D + 2];
        const double area = fsqrt(sx * sx + sy * sy + sz * sz);
        const double ia = frcp(area);
        roe<double>(PL, PR, sx * ia, sy * ia, sz * ia, gas, fl);
#pragma unroll
        for (int q = 0; q < 5; ++q) F[5][q] = fl[q] * area;
      }
      if (v >= x0 + 2) {   // cell v - 2: faces v - 5 .. v
        int p[3] = {c0[0], c0[1], c0[2]};
        p[D] = v - 2;
        const int64_t c = ((int64_t)p[2] * n[1] + p[1]) * n0 + p[0];
#pragma unroll
        for (int q = 0; q < 5; ++q) {
          const double o = c1 * (F[3][q] - F[2][q]) + c2 * (F[4][q] - F[1][q]) + c3 * (F[5][q] - F[0][q]);
          double* at = r + q * cells + c;
          if constexpr (MODE == 2) *at = (*at + o) / jinv[c];
          else *at += o;
        }
      }
    }
  }
}

// The inviscid marches take chunks of 32 cells: each chunk computes five
// extra faces (and converts ten extra cells), an overhead that shorter chunks
// make larger than the passes they replace.  A block whose lines give fewer
// than 64 k such chunks (too few workgroups to fill the chip) keeps the
// padded-primitive, face and Eq. 2 passes instead (measured: 128 x 64 x 64
// blocks ran 1.4 % slower per step with 8-cell chunks).
constexpr int EULER_CHUNK = 32;
bool euler_march_ok(const int n[3], int d) {
  return (int64_t)n[0] * n[d == 1 ? 2 : 1] * ((n[d] + EULER_CHUNK - 1) / EULER_CHUNK) >= (int64_t)1 << 16;
}

// One direction d (1 or 2) of the inviscid residual of a block added into r;
// div: the sum then divided by J^{-1} (curvilinear, last direction).
void euler_march_launch(const Line& Q, const Line& S, double* r, const double* jinv, const int n[3], int d, bool div,
                        double eps, double c1, double c2, double c3, const Gas<double>& gas, hipStream_t stream) {
  const Dims3 D{{n[0], n[1], n[2]}};
  const int ch = EULER_CHUNK;
  const int64_t th = (int64_t)n[0] * n[d == 1 ? 2 : 1] * ((n[d] + ch - 1) / ch);
  const dim3 g(grid_for(th)), b(256);
  if (d == 1 && !div) hipLaunchKernelGGL((k_wcns5_euler_march<1, 1>), g, b, 0, stream, Q, S, r, jinv, D, ch, eps, c1, c2, c3, gas);
  else if (d == 1) hipLaunchKernelGGL((k_wcns5_euler_march<1, 2>), g, b, 0, stream, Q, S, r, jinv, D, ch, eps, c1, c2, c3, gas);
  else if (!div) hipLaunchKernelGGL((k_wcns5_euler_march<2, 1>), g, b, 0, stream, Q, S, r, jinv, D, ch, eps, c1, c2, c3, gas);
  else hipLaunchKernelGGL((k_wcns5_euler_march<2, 2>), g, b, 0, stream, Q, S, r, jinv, D, ch, eps, c1, c2, c3, gas);
}

// The inviscid residual along i in one pass: each wave takes a segment of 59
// cells of a row, converts the 69 cells around it to primitives into LDS
// (coalesced along i), computes the segment's 64 face fluxes, one per lane,
// into LDS, then stores Eq. 2 of each cell into R (the first direction).  The
// arithmetic is that of k_pad_prim_*, k_wcns5_roe_faces and the Eq. 2 pass.
constexpr int EROW_SEG = 59, EROW_CELLS = EROW_SEG + 10, EROW_FACES = EROW_SEG + 5;

__global__ void __launch_bounds__(256) k_wcns5_euler_rows(Line Q, Line S, double* __restrict__ r, Dims3 Dm,
                                                          double eps, double c1, double c2, double c3,
                                                          Gas<double> gas) {
  __shared__ double sp[4][5][EROW_CELLS + 3];
  __shared__ double sf[4][5][EROW_FACES];
  const int* n = Dm.n;
  const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int nseg = (n[0] + EROW_SEG - 1) / EROW_SEG;
  const int64_t cells = (int64_t)n[0] * n[1] * n[2];
  const int64_t items = (int64_t)n[1] * n[2] * nseg;
  for (int64_t base = (int64_t)blockIdx.x * 4; base < items; base += (int64_t)gridDim.x * 4) {
    const int64_t it = base + w;
    const bool act = it < items;
    int c0[3] = {0, 0, 0}, x0 = 0, x1 = 0;
    if (act) {
      const int64_t row = it / nseg;
      x0 = (int)(it % nseg) * EROW_SEG;
      x1 = min(x0 + EROW_SEG, n[0]);
      c0[1] = (int)(row % n[1]);
      c0[2] = (int)(row / n[1]);
      for (int e = lane; e < EROW_CELLS; e += 64) {
        const int x = x0 - 5 + e;
        if (x <= x1 + 4) {
          const LineRef q = wrap_ref(Q, c0, x, 0, n);
          const Prim<double> p = to_prim<double>(q[0], q[1], q[2], q[3], q[4], gas.gm1);
          sp[w][0][e] = p.r;
          sp[w][1][e] = p.u;
          sp[w][2][e] = p.v;
          sp[w][3][e] = p.w;
          sp[w][4][e] = p.p;
        }
      }
    }
    __syncthreads();
    if (act) {
      const int v = x0 - 3 + lane;   // face between cells v and v + 1: cells v - 2 .. v + 3 at lane .. lane + 5
      if (v <= x1 + 1) {
        double L[5], R[5];
#pragma unroll
        for (int q = 0; q < 5; ++q) {
          const double* u = &sp[w][q][lane];
          L[q] = wcns5_left(u[0], u[1], u[2], u[3], u[4], eps);
          R[q] = wcns5_left(u[5], u[4], u[3], u[2], u[1], eps);
        }
        const Prim<double> PL{L[0], L[1], L[2], L[3], L[4]};
        const Prim<double> PR{R[0], R[1], R[2], R[3], R[4]};
        double fl[5];
        if (!S.own) {
          roe<double>(PL, PR, 1.0, 0.0, 0.0, gas, fl);
#pragma unroll
          for (int q = 0; q < 5; ++q) sf[w][q][lane] = fl[q];
        } else {
          const LineRef sr = wrap_ref(S, c0, v, 0, n);
          const double sx = sr[0], sy = sr[1], sz = sr[2];
          const double area = fsqrt(sx * sx + sy * sy + sz * sz);
          const double ia = frcp(area);
          roe<double>(PL, PR, sx * ia, sy * ia, sz * ia, gas, fl);
#pragma unroll
          for (int q = 0; q < 5; ++q) sf[w][q][lane] = fl[q] * area;
        }
      }
    }
    __syncthreads();
    if (act && lane < EROW_SEG) {
      const int x = x0 + lane;   // faces x - 3 .. x + 2 at lane .. lane + 5
      if (x < x1) {
        const int64_t c = ((int64_t)c0[2] * n[1] + c0[1]) * n[0] + x;
#pragma unroll
        for (int q = 0; q < 5; ++q) {
          const double* F = &sf[w][q][lane];
          r[q * cells + c] = c1 * (F[3] - F[2]) + c2 * (F[4] - F[1]) + c3 * (F[5] - F[0]);
        }
      }
    }
    __syncthreads();
  }
}

// Rows of n cells leave idle lanes in the last segment's faces; the row pass
// is used where its face slots stay within 1.25 times the n + 5 faces needed
// (256- and 512-cell rows: 1.23, 1.11; 128 cells: 1.44).
bool euler_rows_ok(int n0) {
  const int64_t nseg = (n0 + EROW_SEG - 1) / EROW_SEG;
  return nseg * 64 * 4 <= (int64_t)(n0 + 5) * 5;
}

void euler_rows_launch(const Line& Q, const Line& S, double* r, const int n[3], double eps, double c1, double c2,
                       double c3, const Gas<double>& gas, hipStream_t stream) {
  const Dims3 D{{n[0], n[1], n[2]}};
  const int64_t items = (int64_t)n[1] * n[2] * ((n[0] + EROW_SEG - 1) / EROW_SEG);
  const int grid = (int)std::min<int64_t>((items + 3) / 4, 1 << 16);
  hipLaunchKernelGGL(k_wcns5_euler_rows, dim3(grid), dim3(256), 0, stream, Q, S, r, D, eps, c1, c2, c3, gas);
}

// The periodic WCNS-E-5 residual along the three directions.  Cartesian when
// s is NULL (face normals e_d, Eq. (2) with the spacings h); else curvilinear:
// Roe's flux through the face area vectors s, Eq. (2) in index units and a
// final division by jinv.  Arguments checked by the callers.
void wcns5_residual_core(const double* q_dev, const double* s_dev, const double* jinv_dev, double* r_dev,
                         void* work_dev, size_t work_bytes, const int32_t n[3], const double* h, double gamma,
                         double entropy_fix, double eps, hipStream_t stream) {
  if (!(gamma > 1.0) || !std::isfinite(gamma)) host_fail(CFD_EINVAL, "gamma must exceed 1");
  if (!(entropy_fix >= 0.0) || !std::isfinite(entropy_fix)) host_fail(CFD_EINVAL, "bad entropy_fix");
  if (!(eps > 0.0) || !std::isfinite(eps)) host_fail(CFD_EINVAL, "eps must be positive and finite");
  int64_t pmax, fmax;
  wcns5_work(n, pmax, fmax);
  const size_t need = (size_t)(8 * (pmax + fmax));
  if (work_bytes < need) host_fail(CFD_ENOMEM, "workspace smaller than cfd_wcns5_euler_work_bytes()");
  const int64_t cells = (int64_t)n[0] * n[1] * n[2];
  if (!apart(q_dev, 40 * cells, r_dev, 40 * cells) || !apart(q_dev, 40 * cells, work_dev, (int64_t)need) ||
      !apart(r_dev, 40 * cells, work_dev, (int64_t)need))
    host_fail(CFD_EINVAL, "q, r and the workspace must not overlap");
  if (s_dev && (!apart(r_dev, 40 * cells, s_dev, 72 * cells) || !apart(r_dev, 40 * cells, jinv_dev, 8 * cells) ||
                !apart(work_dev, (int64_t)need, s_dev, 72 * cells) ||
                !apart(work_dev, (int64_t)need, jinv_dev, 8 * cells)))
    host_fail(CFD_EINVAL, "r and the workspace must not overlap the metrics");
  double* W = static_cast<double*>(work_dev);
  double* F = W + pmax;
  Gas<double> gas{};
  gas.gamma = gamma;
  gas.gm1 = gamma - 1.0;
  gas.gg = gamma / (gamma - 1.0);
  gas.eps_h = entropy_fix;
  for (int d = 0; d < 3; ++d) {
    const double hd = s_dev ? 1.0 : h[d];
    const double c1 = 75.0 / (64.0 * hd), c2 = -25.0 / (384.0 * hd), c3 = 3.0 / (640.0 * hd);
    if (d == 0 && euler_rows_ok(n[0])) {   // i: one row pass
      const Line Q{q_dev, q_dev, q_dev, cells, cells, cells, n[0], n[0]};
      const Line S{s_dev, s_dev, s_dev, cells, cells, cells, n[0], n[0]};
      euler_rows_launch(Q, S, r_dev, n, eps, c1, c2, c3, gas, stream);
      continue;
    }
    if (d > 0 && euler_march_ok(n, d)) {   // j and k: one marching pass (the last one divides the sum by J^{-1})
      const Line Q{q_dev, q_dev, q_dev, cells, cells, cells, n[d], n[d]};
      const Line S{s_dev, s_dev, s_dev, cells, cells, cells, n[d], n[d]};
      euler_march_launch(Q, S, r_dev, jinv_dev, n, d, d == 2 && s_dev, eps, c1, c2, c3, gas, stream);
      continue;
    }
    int64_t mp[3] = {n[0], n[1], n[2]}, mf[3] = {n[0], n[1], n[2]};
    mp[d] += 10;
    mf[d] += 5;
    const int64_t nf = mf[0] * mf[1] * mf[2];
    hipLaunchKernelGGL(k_pad_prim_periodic, dim3(grid_for(mp[0] * mp[1] * mp[2])), dim3(256), 0, stream, q_dev, W,
                       n[0], n[1], n[2], d, gamma - 1.0);
    hipLaunchKernelGGL(k_wcns5_roe_faces, dim3(grid_for(nf)), dim3(256), 0, stream, W, F, (int)mf[0], (int)mf[1],
                       (int)mf[2], d, eps, s_dev, s_dev, s_dev, n[0], n[1], n[2], n[d], n[d], gas);
    const int64_t m[3] = {n[0], n[1], n[2]};
    if (d == 0)
      launch_window6(F, r_dev, nullptr, m, d, 5, Eq2OpT<false>{c1, c2, c3}, stream);
    else if (d == 2 && s_dev)       // the last pass also divides the sum by J^{-1}
      launch_window6(F, r_dev, nullptr, m, d, 5, Eq2DivOp{c1, c2, c3, jinv_dev}, stream);
    else
      launch_window6(F, r_dev, nullptr, m, d, 5, Eq2OpT<true>{c1, c2, c3}, stream);
  }
  const hipError_t e = hipGetLastError();
  if (e != hipSuccess) host_fail(CFD_EHIP, std::string("kernel launch failed: ") + hipGetErrorString(e));
}

}  // namespace cfd

extern "C" cfd_status cfd_wcns5_euler_residual_periodic(const double* q_dev, double* r_dev, void* work_dev,
                                                        size_t work_bytes, const int32_t n[3], const double h[3],
                                                        double gamma, double entropy_fix, double eps,
                                                        hipStream_t stream) {
  return cfd::host_guarded([&] {
    if (!q_dev || !r_dev || !work_dev || !n || !h) cfd::host_fail(CFD_EINVAL, "NULL argument");
    if (n[0] < 1 || n[1] < 1 || n[2] < 1) cfd::host_fail(CFD_EINVAL, "every extent must be >= 1");
    for (int d = 0; d < 3; ++d)
      if (!(h[d] > 0.0) || !std::isfinite(h[d])) cfd::host_fail(CFD_EINVAL, "spacings must be positive and finite");
    cfd::wcns5_residual_core(q_dev, nullptr, nullptr, r_dev, work_dev, work_bytes, n, h, gamma, entropy_fix, eps,
                             stream);
  });
}

// Scratch of cfd_wcns5_euler_residual_periodic_noalloc: every device the
// library runs on holds its own copy from module load to process end.  In host
// code the name is only a handle; the device address comes from
// hipGetSymbolAddress, once per device, and only that address reaches kernels.
static __device__ __align__(256) double scratch[CFD_WCNS5_NOALLOC_MAX_BYTES / sizeof(double)];

namespace {

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_addr[kMaxDevices] = {};

// The device address of `scratch` on the current device, which must be the
// stream's device; looked up on the first call on each device.
void* scratch_address(hipStream_t stream) {
  int dev = -1;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) cfd::host_fail(CFD_EHIP, std::string("hipGetDevice: ") + hipGetErrorString(e));
  if (dev < 0 || dev >= kMaxDevices) cfd::host_fail(CFD_EUNSUPPORTED, "device ordinal beyond the scratch table");
  hipDevice_t sdev = -1;
  e = hipStreamGetDevice(stream, &sdev);
  if (e != hipSuccess) cfd::host_fail(CFD_EHIP, std::string("hipStreamGetDevice: ") + hipGetErrorString(e));
  if (sdev != dev) cfd::host_fail(CFD_EINVAL, "the stream is not on the current device");
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_addr[dev]) {
    void* p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p)
      cfd::host_fail(CFD_EHIP, std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e));
    g_scratch_addr[dev] = p;
  }
  return g_scratch_addr[dev];
}

}  // namespace

extern "C" cfd_status cfd_wcns5_euler_residual_periodic_noalloc(const double* q_dev, double* r_dev,
                                                                const int32_t n[3], const double h[3], double gamma,
                                                                double entropy_fix, double eps, hipStream_t stream) {
  return cfd::host_guarded([&] {
    if (!q_dev || !r_dev || !n || !h) cfd::host_fail(CFD_EINVAL, "NULL argument");
    if (n[0] < 1 || n[1] < 1 || n[2] < 1) cfd::host_fail(CFD_EINVAL, "every extent must be >= 1");
    for (int d = 0; d < 3; ++d)
      if (!(h[d] > 0.0) || !std::isfinite(h[d])) cfd::host_fail(CFD_EINVAL, "spacings must be positive and finite");
    // at least 80 bytes per cell (padded primitives and face flux): reject
    // huge extents before the exact count, whose products could overflow
    double need = 80.0 * (double)n[0] * (double)n[1] * (double)n[2];
    if (need <= (double)CFD_WCNS5_NOALLOC_MAX_BYTES) {
      int64_t pmax, fmax;
      cfd::wcns5_work(n, pmax, fmax);
      need = 8.0 * ((double)pmax + (double)fmax);
    }
    if (need > (double)CFD_WCNS5_NOALLOC_MAX_BYTES)
      cfd::host_fail(CFD_ENOMEM, "block needs " + std::to_string((long long)need) +
                                     " bytes of scratch, more than CFD_WCNS5_NOALLOC_MAX_BYTES = " +
                                     std::to_string((long long)CFD_WCNS5_NOALLOC_MAX_BYTES));
    void* work = scratch_address(stream);
    cfd::wcns5_residual_core(q_dev, nullptr, nullptr, r_dev, work, CFD_WCNS5_NOALLOC_MAX_BYTES, n, h, gamma,
                             entropy_fix, eps, stream);
  });
}

extern "C" cfd_status cfd_wcns5_metrics_periodic(const double* xv_dev, const double period[9], const int32_t n[3],
                                                 double* s_dev, double* jinv_dev, hipStream_t stream) {
  return cfd::host_guarded([&] {
    if (!xv_dev || !period || !n || !s_dev || !jinv_dev) cfd::host_fail(CFD_EINVAL, "NULL argument");
    if (n[0] < 1 || n[1] < 1 || n[2] < 1) cfd::host_fail(CFD_EINVAL, "every extent must be >= 1");
    for (int t = 0; t < 9; ++t)
      if (!std::isfinite(period[t])) cfd::host_fail(CFD_EINVAL, "periods must be finite");
    const int64_t cells = (int64_t)n[0] * n[1] * n[2];
    if (cells > ((int64_t)1 << 34)) cfd::host_fail(CFD_EINVAL, "block too large");
    if (!cfd::apart(xv_dev, 24 * cells, s_dev, 72 * cells) || !cfd::apart(xv_dev, 24 * cells, jinv_dev, 8 * cells) ||
        !cfd::apart(s_dev, 72 * cells, jinv_dev, 8 * cells))
      cfd::host_fail(CFD_EINVAL, "vertices, metrics and jinv must not overlap");
    cfd::PeriodicGrid g{};
    g.xv = xv_dev;
    for (int d = 0; d < 3; ++d) {
      g.n[d] = n[d];
      for (int c = 0; c < 3; ++c) g.P[d][c] = period[3 * d + c];
    }
    const dim3 grid(cfd::grid_for(cells));
    cfd::launch_metrics(g, s_dev, jinv_dev, cells, stream);
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) cfd::host_fail(CFD_EHIP, std::string("kernel launch failed: ") + hipGetErrorString(e));
  });
}

extern "C" cfd_status cfd_wcns5_euler_residual_curv_periodic(const double* q_dev, const double* s_dev,
                                                             const double* jinv_dev, double* r_dev, void* work_dev,
                                                             size_t work_bytes, const int32_t n[3], double gamma,
                                                             double entropy_fix, double eps, hipStream_t stream) {
  return cfd::host_guarded([&] {
    if (!q_dev || !s_dev || !jinv_dev || !r_dev || !work_dev || !n) cfd::host_fail(CFD_EINVAL, "NULL argument");
    if (n[0] < 1 || n[1] < 1 || n[2] < 1) cfd::host_fail(CFD_EINVAL, "every extent must be >= 1");
    cfd::wcns5_residual_core(q_dev, s_dev, jinv_dev, r_dev, work_dev, work_bytes, n, nullptr, gamma, entropy_fix, eps,
                             stream);
  });
}

namespace {

size_t wcns5_residual_work(const int32_t n[3]) {
  int64_t pmax, fmax;
  cfd::wcns5_work(n, pmax, fmax);
  return (size_t)(8 * (pmax + fmax));
}

}  // namespace

extern "C" cfd_status cfd_wcns5_euler_step_work_bytes(const int32_t n[3], size_t* bytes) {
  return cfd::host_guarded([&] {
    if (!n || !bytes) cfd::host_fail(CFD_EINVAL, "NULL argument");
    if (n[0] < 1 || n[1] < 1 || n[2] < 1) cfd::host_fail(CFD_EINVAL, "every extent must be >= 1");
    *bytes = wcns5_residual_work(n) + (size_t)2 * 40 * ((size_t)n[0] * n[1] * n[2]);
  });
}

namespace cfd {

// nsteps RK3 steps in place on q with the residual core (Cartesian when s is
// NULL).  The workspace: the residual's, then the step's start state and R.
Gas<double> viscous_gas(double gamma, double prandtl, double mu_inf, double s_star);
// Viscous scratch of a periodic block: phi (4) and index gradients (12) per
// cell, shared with the residual's scratch; the face metrics (21 per cell)
// are computed once per call and kept apart from it.
constexpr int VW_FIELDS = 16, FM_FIELDS = 21;
void c4_face_metrics_curv(const double* s_dev, const double* jinv_dev, double* sc_tmp, double* fm, const int32_t n[3],
                          hipStream_t stream);
// The RK3 stage a Q^n + b (Q^(s-1) - dt R) of Eqs. 4-6 for a pass that
// applies it (keep: the first stage, which saves Q^n).
struct RkArgs {
  double* q;
  double* qn;
  double dt, a, b;
  int keep;
};
// Whether a block's last viscous pass applies the RK3 stage itself: only where
// its k march runs whole 32-cell chunks (on 128 x 64 x 64 blocks, with 8-cell
// chunks, the fused update measured 3 % slower per step than a separate pass).
int visc_chunk(const int n[3], int d);
inline bool rk_fused(const int n[3]) { return visc_chunk(n, 2) >= 32; }
void c4_viscous_curv_core(const double* q_dev, const double* s_dev, const double* jinv_dev, double* r_dev,
                          double* work, const double* fm, const int32_t n[3], const Gas<double>& gas,
                          hipStream_t stream, const RkArgs* rk = nullptr);
// Bytes of a periodic block's residual-or-viscous scratch followed by its
// face metrics (the metrics start at visc_fm_offset).
size_t visc_fm_offset(size_t rw0, int64_t cells) { return std::max(rw0, (size_t)8 * VW_FIELDS * cells); }
size_t visc_region(size_t rw0, int64_t cells) { return visc_fm_offset(rw0, cells) + (size_t)8 * FM_FIELDS * cells; }

// With visc (curvilinear blocks only) each stage adds the fourth-order
// viscous terms to the residual; their scratch shares the residual's, which
// is free again once R is formed.
void wcns5_steps_core(double* q_dev, const double* s_dev, const double* jinv_dev, void* work_dev, size_t work_bytes,
                      const int32_t n[3], const double* h, double gamma, double entropy_fix, double eps, double dt,
                      int32_t nsteps, hipStream_t stream, const Gas<double>* visc = nullptr) {
  if (n[0] < 1 || n[1] < 1 || n[2] < 1) host_fail(CFD_EINVAL, "every extent must be >= 1");
  if (!(dt > 0.0) || !std::isfinite(dt)) host_fail(CFD_EINVAL, "dt must be positive and finite");
  if (nsteps < 0) host_fail(CFD_EINVAL, "nsteps must be >= 0");
  const int64_t cells = (int64_t)n[0] * n[1] * n[2];
  const size_t rw0 = wcns5_residual_work(n);
  const size_t rw = visc ? visc_region(rw0, cells) : rw0;
  if (work_bytes < rw + (size_t)2 * 40 * cells)
    host_fail(CFD_ENOMEM, visc ? "workspace smaller than cfd_wcns5_ns_step_work_bytes()"
                               : "workspace smaller than cfd_wcns5_euler_step_work_bytes()");
  if (!apart(q_dev, 40 * cells, work_dev, (int64_t)work_bytes)) host_fail(CFD_EINVAL, "q and the workspace overlap");
  if (s_dev && (!apart(q_dev, 40 * cells, s_dev, 72 * cells) || !apart(q_dev, 40 * cells, jinv_dev, 8 * cells)))
    host_fail(CFD_EINVAL, "q must not overlap the metrics");
  double* qn = reinterpret_cast<double*>(static_cast<char*>(work_dev) + rw);
  double* r = qn + 5 * cells;
  const int64_t nv = 5 * cells;
  const int g = grid_for(nv);
  const double a[3] = {0.0, 0.75, 1.0 / 3.0}, b[3] = {1.0, 0.25, 2.0 / 3.0};
  double* fm = visc ? reinterpret_cast<double*>(static_cast<char*>(work_dev) + visc_fm_offset(rw0, cells)) : nullptr;
  if (visc && nsteps > 0) c4_face_metrics_curv(s_dev, jinv_dev, static_cast<double*>(work_dev), fm, n, stream);
  for (int it = 0; it < nsteps; ++it)
    for (int st = 0; st < 3; ++st) {
      wcns5_residual_core(q_dev, s_dev, jinv_dev, r, work_dev, rw0, n, h, gamma, entropy_fix, eps, stream);
      if (visc && rk_fused(n)) {   // the last viscous pass applies the stage
        const RkArgs K{q_dev, qn, dt, a[st], b[st], st == 0 ? 1 : 0};
        c4_viscous_curv_core(q_dev, s_dev, jinv_dev, r, static_cast<double*>(work_dev), fm, n, *visc, stream, &K);
      } else {
        if (visc) c4_viscous_curv_core(q_dev, s_dev, jinv_dev, r, static_cast<double*>(work_dev), fm, n, *visc, stream);
        hipLaunchKernelGGL(k_rk3_stage, dim3(g), dim3(256), 0, stream, q_dev, qn, r, nv, dt, a[st], b[st],
                           st == 0 ? 1 : 0);
      }
    }
  const hipError_t e = hipGetLastError();
  if (e != hipSuccess) host_fail(CFD_EHIP, std::string("kernel launch failed: ") + hipGetErrorString(e));
}

}  // namespace cfd

extern "C" cfd_status cfd_wcns5_euler_steps_periodic(double* q_dev, void* work_dev, size_t work_bytes,
                                                     const int32_t n[3], const double h[3], double gamma,
                                                     double entropy_fix, double eps, double dt, int32_t nsteps,
                                                     hipStream_t stream) {
  return cfd::host_guarded([&] {
    if (!q_dev || !work_dev || !n || !h) cfd::host_fail(CFD_EINVAL, "NULL argument");
    if (n[0] < 1 || n[1] < 1 || n[2] < 1) cfd::host_fail(CFD_EINVAL, "every extent must be >= 1");
    for (int d = 0; d < 3; ++d)
      if (!(h[d] > 0.0) || !std::isfinite(h[d])) cfd::host_fail(CFD_EINVAL, "spacings must be positive and finite");
    cfd::wcns5_steps_core(q_dev, nullptr, nullptr, work_dev, work_bytes, n, h, gamma, entropy_fix, eps, dt, nsteps,
                          stream);
  });
}

extern "C" cfd_status cfd_wcns5_euler_steps_curv_periodic(double* q_dev, const double* s_dev, const double* jinv_dev,
                                                          void* work_dev, size_t work_bytes, const int32_t n[3],
                                                          double gamma, double entropy_fix, double eps, double dt,
                                                          int32_t nsteps, hipStream_t stream) {
  return cfd::host_guarded([&] {
    if (!q_dev || !s_dev || !jinv_dev || !work_dev || !n) cfd::host_fail(CFD_EINVAL, "NULL argument");
    cfd::wcns5_steps_core(q_dev, s_dev, jinv_dev, work_dev, work_bytes, n, nullptr, gamma, entropy_fix, eps, dt,
                          nsteps, stream);
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

// r[1 + v] -= (F_{i-3/2} - 27 F_{i-1/2} + 27 F_{i+1/2} - F_{i+3/2}) / 24h, v = 0..3;
// with jinv (curvilinear blocks, h = 1) the difference is divided by J^{-1}.
__global__ void __launch_bounds__(256) k_c4_flux_sub(const double* __restrict__ fv, double* __restrict__ r, Cells3 C,
                                                     int d, double ihd, const double* __restrict__ jinv) {
  const int64_t cells = (int64_t)C.n[0] * C.n[1] * C.n[2];
  for (int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; c < cells; c += (int64_t)gridDim.x * blockDim.x) {
    const int i = (int)(c % C.n[0]), j = (int)((c / C.n[0]) % C.n[1]), k = (int)(c / ((int64_t)C.n[0] * C.n[1]));
    const int64_t m2 = C.step(i, j, k, d, -2), m1 = C.step(i, j, k, d, -1), p1 = C.step(i, j, k, d, 1);
    for (int v = 0; v < 4; ++v) {
      const double* F = fv + v * cells;
      const double dF = (F[m2] - 27.0 * F[m1] + 27.0 * F[c] - F[p1]) * (ihd / 24.0);
      r[(1 + v) * cells + c] -= jinv ? dF / jinv[c] : dF;
    }
  }
}

// Curvilinear blocks: the metrics at the cells, each S_t interpolated from its
// faces along t: sc[(t * 3 + x) * cells + c] (faces i + 1/2 at index i).
__global__ void __launch_bounds__(256) k_c4_cell_metrics(const double* __restrict__ s, double* __restrict__ sc,
                                                         Cells3 C) {
  const int64_t cells = (int64_t)C.n[0] * C.n[1] * C.n[2];
  for (int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; c < cells; c += (int64_t)gridDim.x * blockDim.x) {
    const int i = (int)(c % C.n[0]), j = (int)((c / C.n[0]) % C.n[1]), k = (int)(c / ((int64_t)C.n[0] * C.n[1]));
    for (int t = 0; t < 3; ++t) {
      const int64_t m2 = C.step(i, j, k, t, -2), m1 = C.step(i, j, k, t, -1), p1 = C.step(i, j, k, t, 1);
      for (int x = 0; x < 3; ++x) {
        const double* f = s + (t * 3 + x) * cells;
        sc[(t * 3 + x) * cells + c] = (-f[m2] + 9.0 * f[m1] + 9.0 * f[c] - f[p1]) / 16.0;
      }
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
      hipLaunchKernelGGL(cfd::k_c4_flux_sub, dim3(gr), dim3(256), 0, stream, fv, r_dev, C, d, 1.0 / h[d],
                         static_cast<const double*>(nullptr));
    }
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) cfd::host_fail(CFD_EHIP, std::string("kernel launch failed: ") + hipGetErrorString(e));
  });
}

namespace cfd {

Gas<double> viscous_gas(double gamma, double prandtl, double mu_inf, double s_star) {
  Gas<double> gas{};
  gas.gamma = gamma;
  gas.gm1 = gamma - 1.0;
  gas.mu_inf = mu_inf;
  gas.s_star = s_star;
  gas.prandtl = prandtl;
  gas.kfac = gamma / ((gamma - 1.0) * prandtl);
  return gas;
}

}  // namespace cfd

extern "C" cfd_status cfd_c4_viscous_curv_work_bytes(const int32_t n[3], size_t* bytes) {
  return cfd::host_guarded([&] {
    if (!n || !bytes) cfd::host_fail(CFD_EINVAL, "NULL argument");
    if (n[0] < 1 || n[1] < 1 || n[2] < 1) cfd::host_fail(CFD_EINVAL, "every extent must be >= 1");
    *bytes = (size_t)8 * (cfd::VW_FIELDS + cfd::FM_FIELDS) * ((size_t)n[0] * n[1] * n[2]);  // phi, gradients, face metrics
  });
}

extern "C" cfd_status cfd_c4_viscous_add_curv_periodic(const double* q_dev, const double* s_dev,
                                                       const double* jinv_dev, double* r_dev, void* work_dev,
                                                       size_t work_bytes, const int32_t n[3], double gamma,
                                                       double prandtl, double mu_inf, double s_star,
                                                       hipStream_t stream) {
  return cfd::host_guarded([&] {
    if (!q_dev || !s_dev || !jinv_dev || !r_dev || !work_dev || !n) cfd::host_fail(CFD_EINVAL, "NULL argument");
    if (n[0] < 1 || n[1] < 1 || n[2] < 1) cfd::host_fail(CFD_EINVAL, "every extent must be >= 1");
    if (!(gamma > 1.0) || !(prandtl > 0.0) || !(mu_inf >= 0.0) || !(s_star > 0.0) || !std::isfinite(mu_inf))
      cfd::host_fail(CFD_EINVAL, "bad gas parameters");
    const int64_t cells = (int64_t)n[0] * n[1] * n[2];
    const size_t need = (size_t)8 * (cfd::VW_FIELDS + cfd::FM_FIELDS) * cells;
    if (work_bytes < need) cfd::host_fail(CFD_ENOMEM, "workspace smaller than cfd_c4_viscous_curv_work_bytes()");
    const void* ins[3] = {q_dev, s_dev, jinv_dev};
    const int64_t in_bytes[3] = {40 * cells, 72 * cells, 8 * cells};
    for (int t = 0; t < 3; ++t)
      if (!cfd::apart(ins[t], in_bytes[t], r_dev, 40 * cells) || !cfd::apart(ins[t], in_bytes[t], work_dev, (int64_t)need))
        cfd::host_fail(CFD_EINVAL, "r and the workspace must not overlap q, the metrics or each other");
    if (!cfd::apart(r_dev, 40 * cells, work_dev, (int64_t)need))
      cfd::host_fail(CFD_EINVAL, "r and the workspace must not overlap q, the metrics or each other");
    double* w = static_cast<double*>(work_dev);
    double* fm = w + cfd::VW_FIELDS * cells;
    cfd::c4_face_metrics_curv(s_dev, jinv_dev, w, fm, n, stream);
    cfd::c4_viscous_curv_core(q_dev, s_dev, jinv_dev, r_dev, w, fm, n, cfd::viscous_gas(gamma, prandtl, mu_inf, s_star),
                              stream);
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) cfd::host_fail(CFD_EHIP, std::string("kernel launch failed: ") + hipGetErrorString(e));
  });
}

// ------------------------------------------------------------ time step
// The paper leaves the step size open; the finite-volume path's reading on
// these blocks: dt_c = CFL J^{-1} / (sum_d L_d + 4 sum_d Lv_d) with
// L_d = |u . Sb_d| + c |Sb_d|, Lv_d = max(4/3, gamma/Pr)(mu/rho)|Sb_d|^2/J^{-1}
// (viscous flow only), Sb_d the mean of the cell's two d-face area vectors;
// the step is the least dt_c.  Each workgroup reduces its cells in LDS and
// takes one atomic minimum on the bits of the result (ordered like the
// values for positive doubles, so the outcome does not depend on the order).
namespace cfd {

__global__ void k_dt_init(unsigned long long* out) {
  if (threadIdx.x == 0 && blockIdx.x == 0) *out = 0x7FF0000000000000ull;   // +inf
}

__global__ void __launch_bounds__(256) k_cfl_dt_curv(const double* __restrict__ q, const double* __restrict__ s,
                                                     const double* __restrict__ jinv, Cells3 C, Gas<double> gas,
                                                     double cfl, int viscous, unsigned long long* out) {
  __shared__ double red[256];
  const int64_t cells = (int64_t)C.n[0] * C.n[1] * C.n[2];
  const double coef = fmax(4.0 / 3.0, gas.gamma / gas.prandtl);
  double best = __longlong_as_double(0x7FF0000000000000ll);
  for (int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; c < cells; c += (int64_t)gridDim.x * blockDim.x) {
    const int i = (int)(c % C.n[0]), j = (int)((c / C.n[0]) % C.n[1]), k = (int)(c / ((int64_t)C.n[0] * C.n[1]));
    const Prim<double> p = to_prim<double>(q[c], q[cells + c], q[2 * cells + c], q[3 * cells + c], q[4 * cells + c],
                                           gas.gm1);
    const double a = sqrt(gas.gamma * p.p / p.r);
    const double V = jinv[c];
    double mu = 0.0;
    if (viscous) {
      const double T = p.p / p.r;
      mu = gas.mu_inf * T * sqrt(T) * (1.0 + gas.s_star) / (T + gas.s_star);
    }
    double lam = 0.0, lamv = 0.0;
    for (int d = 0; d < 3; ++d) {
      const int64_t lo = C.step(i, j, k, d, -1);
      const double* sd = s + 3 * d * cells;
      const double bx = 0.5 * (sd[lo] + sd[c]), by = 0.5 * (sd[cells + lo] + sd[cells + c]),
                   bz = 0.5 * (sd[2 * cells + lo] + sd[2 * cells + c]);
      const double mag = sqrt(bx * bx + by * by + bz * bz);
      lam = lam + (fabs(p.u * bx + p.v * by + p.w * bz) + a * mag);
      if (viscous) lamv = lamv + coef * (mu / p.r) * mag * mag / V;
    }
    double dt = cfl * V / (lam + 4.0 * lamv);
    if (!(dt > 0.0)) dt = 0.0;                  // a non-physical cell or J^{-1} <= 0 gives a step of 0
    best = fmin(best, dt);
  }
  red[threadIdx.x] = best;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) red[threadIdx.x] = fmin(red[threadIdx.x], red[threadIdx.x + w]);
    __syncthreads();
  }
  if (threadIdx.x == 0) atomicMin(out, (unsigned long long)__double_as_longlong(red[0]));
}

}  // namespace cfd

extern "C" cfd_status cfd_wcns5_time_step_curv_periodic(const double* q_dev, const double* s_dev,
                                                        const double* jinv_dev, const int32_t n[3], double gamma,
                                                        double cfl, int32_t viscous, double prandtl, double mu_inf,
                                                        double s_star, double* dt_dev, hipStream_t stream) {
  return cfd::host_guarded([&] {
    if (!q_dev || !s_dev || !jinv_dev || !n || !dt_dev) cfd::host_fail(CFD_EINVAL, "NULL argument");
    if (n[0] < 1 || n[1] < 1 || n[2] < 1) cfd::host_fail(CFD_EINVAL, "every extent must be >= 1");
    if (!(gamma > 1.0) || !std::isfinite(gamma)) cfd::host_fail(CFD_EINVAL, "gamma must exceed 1");
    if (!(cfl > 0.0) || !std::isfinite(cfl)) cfd::host_fail(CFD_EINVAL, "cfl must be positive and finite");
    if (viscous && (!(prandtl > 0.0) || !(mu_inf >= 0.0) || !(s_star > 0.0) || !std::isfinite(mu_inf)))
      cfd::host_fail(CFD_EINVAL, "bad gas parameters");
    const int64_t cells = (int64_t)n[0] * n[1] * n[2];
    if (!cfd::apart(dt_dev, 8, q_dev, 40 * cells) || !cfd::apart(dt_dev, 8, s_dev, 72 * cells) ||
        !cfd::apart(dt_dev, 8, jinv_dev, 8 * cells))
      cfd::host_fail(CFD_EINVAL, "dt must not overlap the inputs");
    if ((reinterpret_cast<uintptr_t>(dt_dev) & 7) != 0) cfd::host_fail(CFD_EINVAL, "dt must be 8-byte aligned");
    cfd::Cells3 C{{n[0], n[1], n[2]}};
    cfd::Gas<double> gas{};
    gas.gamma = gamma;
    gas.gm1 = gamma - 1.0;
    gas.mu_inf = mu_inf;
    gas.s_star = s_star;
    gas.prandtl = viscous ? prandtl : 1.0;
    auto* out = reinterpret_cast<unsigned long long*>(dt_dev);
    hipLaunchKernelGGL(cfd::k_dt_init, dim3(1), dim3(64), 0, stream, out);
    hipLaunchKernelGGL(cfd::k_cfl_dt_curv, dim3(cfd::grid_for(cells)), dim3(256), 0, stream, q_dev, s_dev, jinv_dev, C,
                       gas, cfl, viscous ? 1 : 0, out);
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) cfd::host_fail(CFD_EHIP, std::string("kernel launch failed: ") + hipGetErrorString(e));
  });
}

// ------------------------------------------------------------ block seams
extern "C" cfd_status cfd_wcns5_metrics_ext(const double* xe_dev, const int32_t n[3], double* s_dev, double* jinv_dev,
                                            hipStream_t stream) {
  return cfd::host_guarded([&] {
    if (!xe_dev || !n || !s_dev || !jinv_dev) cfd::host_fail(CFD_EINVAL, "NULL argument");
    if (n[0] < 1 || n[1] < 1 || n[2] < 1) cfd::host_fail(CFD_EINVAL, "every extent must be >= 1");
    const int64_t cells = (int64_t)n[0] * n[1] * n[2];
    if (cells > ((int64_t)1 << 34)) cfd::host_fail(CFD_EINVAL, "block too large");
    const int64_t ecells = (int64_t)(n[0] + 5) * (n[1] + 5) * (n[2] + 5);
    if (!cfd::apart(xe_dev, 24 * ecells, s_dev, 72 * cells) || !cfd::apart(xe_dev, 24 * ecells, jinv_dev, 8 * cells) ||
        !cfd::apart(s_dev, 72 * cells, jinv_dev, 8 * cells))
      cfd::host_fail(CFD_EINVAL, "vertices, metrics and jinv must not overlap");
    cfd::ExtGrid g{xe_dev, {n[0], n[1], n[2]}};
    cfd::launch_metrics(g, s_dev, jinv_dev, cells, stream);
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) cfd::host_fail(CFD_EHIP, std::string("kernel launch failed: ") + hipGetErrorString(e));
  });
}

namespace {

// Checks the face-to-face table: every neighbour in range, the link returned
// by the neighbour's opposite face, the same transverse extents, at least
// five cells across the seam.  Returns the largest residual workspace.
size_t check_seams(int32_t nblk, const int32_t* dims, const int32_t* nbr) {
  if (nblk < 1 || nblk > 65536) cfd::host_fail(CFD_EINVAL, "nblk must be in [1, 65536]");
  if (!dims || !nbr) cfd::host_fail(CFD_EINVAL, "NULL argument");
  size_t most = 0;
  for (int b = 0; b < nblk; ++b) {
    const int32_t* n = dims + 3 * b;
    if (n[0] < 1 || n[1] < 1 || n[2] < 1) cfd::host_fail(CFD_EINVAL, "every extent must be >= 1");
    if ((int64_t)n[0] * n[1] * n[2] > ((int64_t)1 << 34)) cfd::host_fail(CFD_EINVAL, "block too large");
  }
  for (int b = 0; b < nblk; ++b) {
    const int32_t* n = dims + 3 * b;
    for (int f = 0; f < 6; ++f) {
      const int d = f / 2, c = nbr[6 * b + f];
      if (c < 0 || c >= nblk) cfd::host_fail(CFD_EINVAL, "neighbour index out of range");
      if (nbr[6 * c + (f ^ 1)] != b) cfd::host_fail(CFD_EINVAL, "neighbour links must be mutual (face f <-> f^1)");
      for (int t = 0; t < 3; ++t)
        if (t != d && dims[3 * c + t] != n[t]) cfd::host_fail(CFD_EINVAL, "joined faces must have the same extents");
      if (dims[3 * c + d] < 5) cfd::host_fail(CFD_EINVAL, "a neighbour must be at least 5 cells across the seam");
    }
    int64_t pmax, fmax;
    cfd::wcns5_work(n, pmax, fmax);
    most = std::max(most, (size_t)(8 * (pmax + fmax)));
  }
  return most;
}

}  // namespace

namespace cfd {

// The residual of blocks joined face to face (arguments checked by the caller).
void wcns5_blocks_residual_launch(int32_t nblk, const int32_t* dims, const int32_t* nbr, const double* const* q_dev,
                                  const double* const* s_dev, const double* const* jinv_dev, double* const* r_dev,
                                  void* work_dev, double gamma, double entropy_fix, double eps, hipStream_t stream,
                                  const char* skip = nullptr) {
  Gas<double> gas{};
  gas.gamma = gamma;
  gas.gm1 = gamma - 1.0;
  gas.gg = gamma / (gamma - 1.0);
  gas.eps_h = entropy_fix;
  for (int b = 0; b < nblk; ++b) {
    if (skip && skip[b]) continue;   // a block whose residual nobody reads (a refilled ghost block)
    const int32_t* n = dims + 3 * b;
    int64_t pmax, fmax;
    wcns5_work(n, pmax, fmax);
    double* W = static_cast<double*>(work_dev);
    double* F = W + pmax;
    for (int d = 0; d < 3; ++d) {
      const int lo = nbr[6 * b + 2 * d], hi = nbr[6 * b + 2 * d + 1];
      const int nlo = dims[3 * lo + d], nhi = dims[3 * hi + d];
      if (d == 0 && euler_rows_ok(n[0])) {   // i: one row pass across the seams
        const Line Q{q_dev[b], q_dev[lo], q_dev[hi], block_cells(dims, b), block_cells(dims, lo),
                     block_cells(dims, hi), nlo, nhi};
        const Line S{s_dev[b], s_dev[lo], s_dev[hi], block_cells(dims, b), block_cells(dims, lo),
                     block_cells(dims, hi), nlo, nhi};
        euler_rows_launch(Q, S, r_dev[b], n, eps, 75.0 / 64.0, -25.0 / 384.0, 3.0 / 640.0, gas, stream);
        continue;
      }
      if (d > 0 && euler_march_ok(n, d)) {   // j and k: one marching pass across the seams (the last divides by J^{-1})
        const Line Q{q_dev[b], q_dev[lo], q_dev[hi], block_cells(dims, b), block_cells(dims, lo),
                     block_cells(dims, hi), nlo, nhi};
        const Line S{s_dev[b], s_dev[lo], s_dev[hi], block_cells(dims, b), block_cells(dims, lo),
                     block_cells(dims, hi), nlo, nhi};
        euler_march_launch(Q, S, r_dev[b], jinv_dev[b], n, d, d == 2, eps, 75.0 / 64.0, -25.0 / 384.0,
                           3.0 / 640.0, gas, stream);
        continue;
      }
      int64_t mp[3] = {n[0], n[1], n[2]}, mf[3] = {n[0], n[1], n[2]};
      mp[d] += 10;
      mf[d] += 5;
      const int64_t nf = mf[0] * mf[1] * mf[2];
      hipLaunchKernelGGL(k_pad_prim_blocks, dim3(grid_for(mp[0] * mp[1] * mp[2])), dim3(256), 0, stream,
                         q_dev[b], q_dev[lo], q_dev[hi], W, n[0], n[1], n[2], d, nlo, nhi, gamma - 1.0);
      hipLaunchKernelGGL(k_wcns5_roe_faces, dim3(grid_for(nf)), dim3(256), 0, stream, W, F, (int)mf[0],
                         (int)mf[1], (int)mf[2], d, eps, s_dev[b], s_dev[lo], s_dev[hi], n[0], n[1], n[2], nlo, nhi,
                         gas);
      const int64_t m[3] = {n[0], n[1], n[2]};
      const double c1 = 75.0 / 64.0, c2 = -25.0 / 384.0, c3 = 3.0 / 640.0;
      if (d == 0)
        launch_window6(F, r_dev[b], nullptr, m, d, 5, Eq2OpT<false>{c1, c2, c3}, stream);
      else if (d == 2)            // the last pass also divides the sum by J^{-1}
        launch_window6(F, r_dev[b], nullptr, m, d, 5, Eq2DivOp{c1, c2, c3, jinv_dev[b]}, stream);
      else
        launch_window6(F, r_dev[b], nullptr, m, d, 5, Eq2OpT<true>{c1, c2, c3}, stream);
    }
  }
}

}  // namespace cfd

extern "C" cfd_status cfd_wcns5_euler_blocks_work_bytes(int32_t nblk, const int32_t* dims, const int32_t* nbr,
                                                        size_t* bytes) {
  return cfd::host_guarded([&] {
    if (!bytes) cfd::host_fail(CFD_EINVAL, "NULL argument");
    *bytes = check_seams(nblk, dims, nbr);
  });
}

extern "C" cfd_status cfd_wcns5_euler_residual_blocks(int32_t nblk, const int32_t* dims, const int32_t* nbr,
                                                      const double* const* q_dev, const double* const* s_dev,
                                                      const double* const* jinv_dev, double* const* r_dev,
                                                      void* work_dev, size_t work_bytes, double gamma,
                                                      double entropy_fix, double eps, hipStream_t stream) {
  return cfd::host_guarded([&] {
    const size_t need = check_seams(nblk, dims, nbr);
    if (!q_dev || !s_dev || !jinv_dev || !r_dev || !work_dev) cfd::host_fail(CFD_EINVAL, "NULL argument");
    if (!(gamma > 1.0) || !std::isfinite(gamma)) cfd::host_fail(CFD_EINVAL, "gamma must exceed 1");
    if (!(entropy_fix >= 0.0) || !std::isfinite(entropy_fix)) cfd::host_fail(CFD_EINVAL, "bad entropy_fix");
    if (!(eps > 0.0) || !std::isfinite(eps)) cfd::host_fail(CFD_EINVAL, "eps must be positive and finite");
    if (work_bytes < need) cfd::host_fail(CFD_ENOMEM, "workspace smaller than cfd_wcns5_euler_blocks_work_bytes()");
    std::vector<cfd::ArgSpan> spans{cfd::span(work_dev, (int64_t)need, true)};
    for (int b = 0; b < nblk; ++b) {
      if (!q_dev[b] || !s_dev[b] || !jinv_dev[b] || !r_dev[b]) cfd::host_fail(CFD_EINVAL, "NULL block pointer");
      const int64_t cb = cfd::block_cells(dims, b);
      spans.insert(spans.end(), {cfd::span(q_dev[b], 40 * cb, false), cfd::span(s_dev[b], 72 * cb, false),
                                 cfd::span(jinv_dev[b], 8 * cb, false), cfd::span(r_dev[b], 40 * cb, true)});
    }
    cfd::check_spans(spans, "a residual or the workspace overlaps an input, another residual or the workspace");
    cfd::wcns5_blocks_residual_launch(nblk, dims, nbr, q_dev, s_dev, jinv_dev, r_dev, work_dev, gamma, entropy_fix, eps,
                                      stream);
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) cfd::host_fail(CFD_EHIP, std::string("kernel launch failed: ") + hipGetErrorString(e));
  });
}

// ------------------------------------------- viscous terms across block seams
// The curvilinear viscous kernels above with every four-point stencil along
// d reading across the block's two d-faces: a Line names a family of fields
// (field f of a block at f * cells + cell) in the block and in its two
// neighbours along d.  The arithmetic is that of the periodic kernels.
namespace cfd {

// u, v, w, T of a block's cells (phi, 4 fields) and their index derivatives
// along i (g[(a * 3 + 0) * cells + c]) in one pass: each wave takes 60 cells
// of a row, converts the 64 cells around them (the neighbours' across the
// i-faces included) in registers, keeps those in LDS for the derivatives, and
// writes phi of its own 60 cells.
constexpr int PGI_SEG = 60;

__global__ void __launch_bounds__(256) k_c4_phi_grads_i(Line Q, double* __restrict__ phi, double* __restrict__ g,
                                                        Dims3 Dm, double gm1) {
  __shared__ double sp[4][4][64];
  const int* n = Dm.n;
  const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int nseg = (n[0] + PGI_SEG - 1) / PGI_SEG;
  const int64_t cells = (int64_t)n[0] * n[1] * n[2];
  const int64_t items = (int64_t)n[1] * n[2] * nseg;
  for (int64_t base = (int64_t)blockIdx.x * 4; base < items; base += (int64_t)gridDim.x * 4) {
    const int64_t it = base + w;
    const bool act = it < items;
    int c0[3] = {0, 0, 0}, x0 = 0, x1 = 0;
    int64_t rb = 0;
    if (act) {
      const int64_t row = it / nseg;
      x0 = (int)(it % nseg) * PGI_SEG;
      x1 = min(x0 + PGI_SEG, n[0]);
      c0[1] = (int)(row % n[1]);
      c0[2] = (int)(row / n[1]);
      rb = ((int64_t)c0[2] * n[1] + c0[1]) * n[0];
      const int x = x0 - 2 + lane;   // cells x0 - 2 .. x0 + 61 at lanes 0 .. 63
      if (x <= x1 + 1) {
        const LineRef q = wrap_ref(Q, c0, x, 0, n);
        const Prim<double> p = to_prim<double>(q[0], q[1], q[2], q[3], q[4], gm1);
        const double f[4] = {p.u, p.v, p.w, p.p / p.r};
#pragma unroll
        for (int a = 0; a < 4; ++a) sp[w][a][lane] = f[a];
        if (x >= x0 && x < x1)
#pragma unroll
          for (int a = 0; a < 4; ++a) phi[a * cells + rb + x] = f[a];
      }
    }
    __syncthreads();
    if (act && lane < PGI_SEG) {
      const int x = x0 + lane;   // cells x - 2 .. x + 2 at lanes lane .. lane + 4
      if (x < x1) {
#pragma unroll
        for (int a = 0; a < 4; ++a) {
          const double m2 = sp[w][a][lane], m1 = sp[w][a][lane + 1], p1 = sp[w][a][lane + 3],
                       p2 = sp[w][a][lane + 4];
          g[(a * 3) * cells + rb + x] = (m2 - 8.0 * m1 + 8.0 * p1 - p2) * (1.0 / 12.0);
        }
      }
    }
    __syncthreads();
  }
}

// The same along j or k: each lane marches a line of cells (lanes along i,
// coalesced rows) over a chunk, keeping five cells of u, v, w, T in registers,
// so every cell is read once per chunk instead of four times from other rows
// or planes.
template <int D>
__global__ void __launch_bounds__(256) k_c4_grads_march(Line phi, double* __restrict__ g, Dims3 Dm, int chunk) {
  constexpr int O = D == 1 ? 2 : 1;
  const int* n = Dm.n;
  const int nD = n[D], nO = n[O], n0 = n[0];
  const int nch = (nD + chunk - 1) / chunk;
  const int64_t cells = (int64_t)n0 * n[1] * n[2];
  const int64_t total = (int64_t)n0 * nO * nch;
  for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < total; t += (int64_t)gridDim.x * blockDim.x) {
    int c0[3];
    c0[0] = (int)(t % n0);
    const int64_t rest = t / n0;
    c0[O] = (int)(rest % nO);
    c0[D] = 0;
    const int x0 = (int)(rest / nO) * chunk, x1 = min(x0 + chunk, nD);
    double w[5][4];
    auto load = [&](int x, double* v) {
      const LineRef r = wrap_ref(phi, c0, x, D, n);
#pragma unroll
      for (int a = 0; a < 4; ++a) v[a] = r[a];
    };
#pragma unroll
    for (int k = 1; k < 5; ++k) load(x0 - 3 + k, w[k]);
    for (int x = x0; x < x1; ++x) {
#pragma unroll
      for (int k = 0; k < 4; ++k)
#pragma unroll
        for (int a = 0; a < 4; ++a) w[k][a] = w[k + 1][a];
      load(x + 2, w[4]);
      int p[3] = {c0[0], c0[1], c0[2]};
      p[D] = x;
      const int64_t c = ((int64_t)p[2] * n[1] + p[1]) * n0 + p[0];
#pragma unroll
      for (int a = 0; a < 4; ++a) {
        const double m2 = w[0][a], m1 = w[1][a], p1 = w[3][a], p2 = w[4][a];
        g[(a * 3 + D) * cells + c] = (m2 - 8.0 * m1 + 8.0 * p1 - p2) * (1.0 / 12.0);
      }
    }
  }
}

// Chunk of the gradient marches: 32 cells, halved (down to 8) while the grid
// gives fewer than 128 k threads.
int grads_chunk(const int n[3], int d) {
  const int o = d == 1 ? 2 : 1;
  int chunk = 32;
  while (chunk > 8 && (int64_t)n[0] * n[o] * ((n[d] + chunk - 1) / chunk) < (int64_t)1 << 17) chunk /= 2;
  return chunk;
}

// phi and its index derivatives along i of a block (Qi: its state line along
// i), into phi (4 fields) and g (12 fields).
void phi_grads_i_launch(const Line& Qi, double* phi, double* g, const int n[3], double gm1, hipStream_t stream) {
  const Dims3 D{{n[0], n[1], n[2]}};
  const int64_t items = (int64_t)n[1] * n[2] * ((n[0] + PGI_SEG - 1) / PGI_SEG);
  const int grid = (int)std::min<int64_t>((items + 3) / 4, 1 << 16);
  hipLaunchKernelGGL(k_c4_phi_grads_i, dim3(grid), dim3(256), 0, stream, Qi, phi, g, D, gm1);
}

// The index derivatives along j and k of a block's u, v, w, T (lines P[d]
// over its phi fields and the neighbours', which must all be written) into g.
void grads_jk_launch(const Line* P, double* g, const int n[3], hipStream_t stream) {
  const Dims3 D{{n[0], n[1], n[2]}};
  const int c1 = grads_chunk(n, 1), c2 = grads_chunk(n, 2);
  const int64_t t1 = (int64_t)n[0] * n[2] * ((n[1] + c1 - 1) / c1), t2 = (int64_t)n[0] * n[1] * ((n[2] + c2 - 1) / c2);
  hipLaunchKernelGGL(k_c4_grads_march<1>, dim3(grid_for(t1)), dim3(256), 0, stream, P[1], g, D, c1);
  hipLaunchKernelGGL(k_c4_grads_march<2>, dim3(grid_for(t2)), dim3(256), 0, stream, P[2], g, D, c2);
}

// sc[(t * 3 + x) * cells + c]: S_t at the cells from its faces along t.
__global__ void __launch_bounds__(256) k_c4_cell_metrics_line(Line S, double* __restrict__ sc, Dims3 D, int t) {
  const int64_t cells = (int64_t)D.n[0] * D.n[1] * D.n[2];
  for (int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; c < cells; c += (int64_t)gridDim.x * blockDim.x) {
    const int i = (int)(c % D.n[0]), j = (int)((c / D.n[0]) % D.n[1]), k = (int)(c / ((int64_t)D.n[0] * D.n[1]));
    const LineRef rm2 = line_ref(S, i, j, k, -2, t, D.n), rm1 = line_ref(S, i, j, k, -1, t, D.n),
                  r0 = line_ref(S, i, j, k, 0, t, D.n), rp1 = line_ref(S, i, j, k, 1, t, D.n);
    for (int x = 0; x < 3; ++x) {
      const int f = t * 3 + x;
      sc[f * cells + c] = (-rm2[f] + 9.0 * rm1[f] + 9.0 * r0[f] - rp1[f]) / 16.0;
    }
  }
}

// Fields of a block's viscous workspace: phi 0..3 and the index gradients
// g 4..15 (g[a * 3 + t]: phi_a along t); the face metrics, 21 per cell, sit in
// an array of their own (fm[(d * 7 + m) * cells + c] at the d-face above cell
// c: m = 0..5 the cell metrics S_t, t != d in increasing t, interpolated to
// the face; m = 6 the inverse of J^{-1} interpolated likewise).
constexpr int VW_PHI = 0, VW_G = 4;

// Face metrics along d from the cell metrics sc (9 fields, S_t[x] at t * 3 + x)
// and J^{-1}, four-point face values across the seams.
__global__ void __launch_bounds__(256) k_c4_face_metrics(Line SC, Line J, double* __restrict__ fm, Dims3 D, int d) {
  const int64_t cells = (int64_t)D.n[0] * D.n[1] * D.n[2];
  for (int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; c < cells; c += (int64_t)gridDim.x * blockDim.x) {
    const int p[3] = {(int)(c % D.n[0]), (int)((c / D.n[0]) % D.n[1]), (int)(c / ((int64_t)D.n[0] * D.n[1]))};
    const LineRef a = wrap_ref(SC, p, p[d] - 1, d, D.n), b = wrap_ref(SC, p, p[d], d, D.n),
                  e = wrap_ref(SC, p, p[d] + 1, d, D.n), f = wrap_ref(SC, p, p[d] + 2, d, D.n);
    int m = 0;
    for (int t = 0; t < 3; ++t) {
      if (t == d) continue;
      for (int x = 0; x < 3; ++x) {
        const int v = t * 3 + x;
        fm[(d * 7 + m++) * cells + c] = (-a[v] + 9.0 * b[v] + 9.0 * e[v] - f[v]) / 16.0;
      }
    }
    const LineRef ja = wrap_ref(J, p, p[d] - 1, d, D.n), jb = wrap_ref(J, p, p[d], d, D.n),
                  je = wrap_ref(J, p, p[d] + 1, d, D.n), jf = wrap_ref(J, p, p[d] + 2, d, D.n);
    fm[(d * 7 + 6) * cells + c] = 1.0 / ((-ja[0] + 9.0 * jb[0] + 9.0 * je[0] - jf[0]) / 16.0);
  }
}

// A cell's inputs of the d-face fluxes: phi (4) and the index derivatives of
// phi across d (8: a * 2 + u, u-th direction other than d).
template <int D>
__device__ __forceinline__ void load_visc_cell(const Line& PG, const int c0[3], int x, const int n[3], double w[12]) {
  const LineRef r = wrap_ref(PG, c0, x, D, n);
#pragma unroll
  for (int a = 0; a < 4; ++a) w[a] = r[VW_PHI + a];
#pragma unroll
  for (int a = 0; a < 4; ++a) {
    int u = 0;
#pragma unroll
    for (int t = 0; t < 3; ++t)
      if (t != D) w[4 + a * 2 + u++] = r[VW_G + a * 3 + t];
  }
}

// Viscous flux (momentum x, y, z and energy) through the d-face between the
// second and third of four consecutive cells A, B, C, E along d: face values of
// u, v, w, T and of their index derivatives across d, the compact derivative
// along d, the physical gradient by the chain rule J sum_t S_t d/dxi_t, the
// stress and heat flux contracted with the face's area vector sd; m: the
// face's metrics (six S_t, t != d, then J).
template <int D>
__device__ __forceinline__ void visc_face_flux(const double A[12], const double B[12], const double C[12],
                                               const double E[12], const double m[7], const double sd[3],
                                               const Gas<double>& gas, double out[4]) {
  auto fval = [](double a, double b, double c, double e) { return (-a + 9.0 * b + 9.0 * c - e) / 16.0; };
  double Sf[3][3];
  {
    int k = 0;
#pragma unroll
    for (int t = 0; t < 3; ++t)
#pragma unroll
      for (int x = 0; x < 3; ++x) Sf[t][x] = t == D ? sd[x] : m[k++];
  }
  const double Jf = m[6];
  double pf[4], grad[4][3];
#pragma unroll
  for (int a = 0; a < 4; ++a) {
    pf[a] = fval(A[a], B[a], C[a], E[a]);
    double dxi[3];
    int u = 0;
#pragma unroll
    for (int t = 0; t < 3; ++t) {
      if (t == D) {
        dxi[t] = (A[a] - 27.0 * B[a] + 27.0 * C[a] - E[a]) * (1.0 / 24.0);
      } else {
        const int f = 4 + a * 2 + u++;
        dxi[t] = fval(A[f], B[f], C[f], E[f]);
      }
    }
#pragma unroll
    for (int x = 0; x < 3; ++x) grad[a][x] = Jf * (Sf[0][x] * dxi[0] + Sf[1][x] * dxi[1] + Sf[2][x] * dxi[2]);
  }
  const double T = pf[3];
  const double mu = gas.mu_inf * T * sqrt(T) * (1.0 + gas.s_star) / (T + gas.s_star);
  const double kc = mu * gas.kfac;
  const double div = grad[0][0] + grad[1][1] + grad[2][2];
  double tau[3][3];
#pragma unroll
  for (int x = 0; x < 3; ++x)
#pragma unroll
    for (int y = 0; y < 3; ++y) tau[x][y] = mu * (grad[x][y] + grad[y][x]);
#pragma unroll
  for (int x = 0; x < 3; ++x) tau[x][x] = tau[x][x] - (2.0 / 3.0) * mu * div;
  double e[3];
#pragma unroll
  for (int x = 0; x < 3; ++x) e[x] = pf[0] * tau[x][0] + pf[1] * tau[x][1] + pf[2] * tau[x][2] + kc * grad[3][x];
#pragma unroll
  for (int q = 0; q < 3; ++q) out[q] = sd[0] * tau[0][q] + sd[1] * tau[1][q] + sd[2] * tau[2][q];
  out[3] = sd[0] * e[0] + sd[1] * e[1] + sd[2] * e[2];
}

template <int D>
__device__ __forceinline__ void visc_face_at(const Line& FM, const Line& S, const int c0[3], int f, const int n[3],
                                             const double* A, const double* B, const double* C, const double* E,
                                             const Gas<double>& gas, double out[4]) {
  const LineRef mr = wrap_ref(FM, c0, f, D, n), sr = wrap_ref(S, c0, f, D, n);
  double m[7], sd[3];
#pragma unroll
  for (int k = 0; k < 7; ++k) m[k] = mr[D * 7 + k];
#pragma unroll
  for (int x = 0; x < 3; ++x) sd[x] = sr[D * 3 + x];
  visc_face_flux<D>(A, B, C, E, m, sd, gas, out);
}

// r[1 + v] -= (F_{c-3/2} - 27 F_{c-1/2} + 27 F_{c+1/2} - F_{c+3/2}) / 24 / J^{-1}.
__device__ __forceinline__ void visc_flux_sub(double* __restrict__ r, const double* __restrict__ jinv, int64_t cells,
                                              int64_t c, const double* Fm2, const double* Fm1, const double* F0,
                                              const double* Fp1) {
  const double ji = jinv[c];
#pragma unroll
  for (int v = 0; v < 4; ++v) {
    const double dF = (Fm2[v] - 27.0 * Fm1[v] + 27.0 * F0[v] - Fp1[v]) * (1.0 / 24.0);
    r[(1 + v) * cells + c] -= dF / ji;
  }
}

// The RK3 stage of Eqs. 4-6 applied by the last viscous pass of a step's
// stage, cell by cell, once its residual is complete (nothing reads the
// state after that pass; RkArgs: Q^(s) = a Q^n + b (Q^(s-1) - dt R), Q^n
// kept from Q by the first stage).  The residual itself is not stored.

__device__ __forceinline__ void visc_flux_sub_rk(const double* __restrict__ r, const double* __restrict__ jinv,
                                                 int64_t cells, int64_t c, const double* Fm2, const double* Fm1,
                                                 const double* F0, const double* Fp1, const RkArgs& K) {
  const double ji = jinv[c];
  double R[5];
  R[0] = r[c];
#pragma unroll
  for (int v = 0; v < 4; ++v) {
    const double dF = (Fm2[v] - 27.0 * Fm1[v] + 27.0 * F0[v] - Fp1[v]) * (1.0 / 24.0);
    R[1 + v] = r[(1 + v) * cells + c] - dF / ji;
  }
#pragma unroll
  for (int v = 0; v < 5; ++v) {
    const int64_t t = v * cells + c;
    const double x = K.q[t], y = R[v];
    const double s = x - K.dt * y;
    if (K.keep) {
      K.qn[t] = x;
      K.q[t] = s;
    } else {
      K.q[t] = K.a * K.qn[t] + K.b * s;
    }
  }
}

// The viscous terms along d = 1 or 2 added into r: each thread marches one
// line of cells along d (lanes along i, so every load is a coalesced row)
// over a chunk of `chunk` cells, keeping the four cells around the current
// face and the last four face fluxes in registers: each cell's inputs are
// loaded once per chunk instead of once per face stencil, and the face
// fluxes never leave the chip.
template <int D, bool RK>
__global__ void __launch_bounds__(256) k_c4_visc_march(Line PG, Line FM, Line S, double* __restrict__ r,
                                                       const double* __restrict__ jinv, Dims3 Dm, int chunk,
                                                       Gas<double> gas, RkArgs K) {
  constexpr int O = D == 1 ? 2 : 1;
  const int* n = Dm.n;
  const int nD = n[D], nO = n[O], n0 = n[0];
  const int nch = (nD + chunk - 1) / chunk;
  const int64_t cells = (int64_t)n0 * n[1] * n[2];
  const int64_t total = (int64_t)n0 * nO * nch;
  for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < total; t += (int64_t)gridDim.x * blockDim.x) {
    int c0[3];
    c0[0] = (int)(t % n0);
    const int64_t rest = t / n0;
    c0[O] = (int)(rest % nO);
    c0[D] = 0;
    const int x0 = (int)(rest / nO) * chunk, x1 = min(x0 + chunk, nD);
    auto cell_index = [&](int x) {
      int p[3] = {c0[0], c0[1], c0[2]};
      p[D] = x;
      return ((int64_t)p[2] * n[1] + p[1]) * n0 + p[0];
    };
    double W0[12], W1[12], W2[12], W3[12];
    double F0[4], F1[4], F2[4], F3[4];
    load_visc_cell<D>(PG, c0, x0 - 3, n, W0);
    load_visc_cell<D>(PG, c0, x0 - 2, n, W1);
    load_visc_cell<D>(PG, c0, x0 - 1, n, W2);
    // face g (between cells g and g + 1) needs cells g - 1 .. g + 2; cell
    // g - 1 is finished with face g.  Window and face slots rotate by one per
    // face: four faces per trip, each with its own register names.
#define CFD_VSTEP(U, A, B, C, E, FN, FA, FB, FC)                                    \
  {                                                                               \
    const int g = f + U;                                                          \
    if (g <= x1) {                                                                \
      load_visc_cell<D>(PG, c0, g + 2, n, E);                                     \
      visc_face_at<D>(FM, S, c0, g, n, A, B, C, E, gas, FN);                      \
      if (g > x0) {                                                               \
        if constexpr (RK) visc_flux_sub_rk(r, jinv, cells, cell_index(g - 1), FA, FB, FC, FN, K); \
        else visc_flux_sub(r, jinv, cells, cell_index(g - 1), FA, FB, FC, FN);   \
      }                                                                           \
    }                                                                             \
  }
    for (int f = x0 - 2; f <= x1; f += 4) {
      CFD_VSTEP(0, W0, W1, W2, W3, F0, F1, F2, F3)
      CFD_VSTEP(1, W1, W2, W3, W0, F1, F2, F3, F0)
      CFD_VSTEP(2, W2, W3, W0, W1, F2, F3, F0, F1)
      CFD_VSTEP(3, W3, W0, W1, W2, F3, F0, F1, F2)
    }
#undef CFD_VSTEP
  }
}

// The viscous terms along i added into r: each wave takes 64 cells of one
// row, stages the inputs of the 70 cells around them in LDS (coalesced along
// i), computes the 67 face fluxes they need into LDS, then the differences.
constexpr int VROW_CELLS = 70, VROW_FACES = 67;

__global__ void __launch_bounds__(256) k_c4_visc_rows(Line PG, Line FM, Line S, double* __restrict__ r,
                                                      const double* __restrict__ jinv, Dims3 Dm, Gas<double> gas) {
  __shared__ double sw[4][12][VROW_CELLS + 2];
  __shared__ double sf[4][4][VROW_FACES + 1];
  const int* n = Dm.n;
  const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int nseg = (n[0] + 63) / 64;
  const int64_t cells = (int64_t)n[0] * n[1] * n[2];
  const int64_t items = (int64_t)n[1] * n[2] * nseg;
  for (int64_t base = (int64_t)blockIdx.x * 4; base < items; base += (int64_t)gridDim.x * 4) {
    const int64_t it = base + w;
    const bool act = it < items;
    int c0[3] = {0, 0, 0}, x0 = 0, x1 = 0;
    if (act) {
      const int64_t row = it / nseg;
      x0 = (int)(it % nseg) * 64;
      x1 = min(x0 + 64, n[0]);
      c0[1] = (int)(row % n[1]);
      c0[2] = (int)(row / n[1]);
      for (int e = lane; e < VROW_CELLS; e += 64) {
        const int x = x0 - 3 + e;
        if (x <= x1 + 2) {
          double v[12];
          load_visc_cell<0>(PG, c0, x, n, v);
#pragma unroll
          for (int f = 0; f < 12; ++f) sw[w][f][e] = v[f];
        }
      }
    }
    __syncthreads();
    if (act) {
      for (int e = lane; e < VROW_FACES; e += 64) {
        const int g = x0 - 2 + e;
        if (g <= x1) {
          double A[12], B[12], C[12], E[12], out[4];
#pragma unroll
          for (int f = 0; f < 12; ++f) {
            A[f] = sw[w][f][e];
            B[f] = sw[w][f][e + 1];
            C[f] = sw[w][f][e + 2];
            E[f] = sw[w][f][e + 3];
          }
          visc_face_at<0>(FM, S, c0, g, n, A, B, C, E, gas, out);
#pragma unroll
          for (int v = 0; v < 4; ++v) sf[w][v][e] = out[v];
        }
      }
    }
    __syncthreads();
    if (act) {
      const int x = x0 + lane;
      if (x < x1) {
        double Fm2[4], Fm1[4], F0[4], Fp1[4];
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          Fm2[v] = sf[w][v][lane];
          Fm1[v] = sf[w][v][lane + 1];
          F0[v] = sf[w][v][lane + 2];
          Fp1[v] = sf[w][v][lane + 3];
        }
        visc_flux_sub(r, jinv, cells, ((int64_t)c0[2] * n[1] + c0[1]) * n[0] + x, Fm2, Fm1, F0, Fp1);
      }
    }
    __syncthreads();
  }
}

// Chunk of the march kernels: 32 cells, halved (down to 8) while the grid
// gives fewer than 128 k threads.
int visc_chunk(const int n[3], int d) {
  const int o = d == 1 ? 2 : 1;
  int chunk = 32;
  while (chunk > 8 && (int64_t)n[0] * n[o] * ((n[d] + chunk - 1) / chunk) < (int64_t)1 << 17) chunk /= 2;
  return chunk;
}

// The fused viscous passes of one block (lines built by the caller): i rows,
// then the j and k marches, each subtracting its differences from r; with
// rk (not NULL) the k march applies the RK3 stage to the block's state
// instead of storing the finished residual.
void visc_fused_launch(const Line* PG, const Line* FM, const Line* S, double* r, const double* jinv, const int n[3],
                       const Gas<double>& gas, hipStream_t stream, const RkArgs* rk = nullptr) {
  const Dims3 D{{n[0], n[1], n[2]}};
  const int64_t rows = (int64_t)n[1] * n[2] * ((n[0] + 63) / 64);
  const int grows = (int)std::min<int64_t>((rows + 3) / 4, 1 << 16);
  hipLaunchKernelGGL(k_c4_visc_rows, dim3(grows), dim3(256), 0, stream, PG[0], FM[0], S[0], r, jinv, D, gas);
  const int c1 = visc_chunk(n, 1), c2 = visc_chunk(n, 2);
  const int64_t t1 = (int64_t)n[0] * n[2] * ((n[1] + c1 - 1) / c1), t2 = (int64_t)n[0] * n[1] * ((n[2] + c2 - 1) / c2);
  const RkArgs none{};
  hipLaunchKernelGGL((k_c4_visc_march<1, false>), dim3(grid_for(t1)), dim3(256), 0, stream, PG[1], FM[1], S[1], r, jinv,
                     D, c1, gas, none);
  if (rk)
    hipLaunchKernelGGL((k_c4_visc_march<2, true>), dim3(grid_for(t2)), dim3(256), 0, stream, PG[2], FM[2], S[2], r,
                       jinv, D, c2, gas, *rk);
  else
    hipLaunchKernelGGL((k_c4_visc_march<2, false>), dim3(grid_for(t2)), dim3(256), 0, stream, PG[2], FM[2], S[2], r,
                       jinv, D, c2, gas, none);
}

// A periodic block's lines: every neighbour the block itself.
Line self_line(const double* base, int64_t cells, int nd) { return Line{base, base, base, cells, cells, cells, nd, nd}; }

void c4_face_metrics_curv(const double* s_dev, const double* jinv_dev, double* sc_tmp, double* fm, const int32_t n[3],
                          hipStream_t stream) {
  const int64_t cells = (int64_t)n[0] * n[1] * n[2];
  const Cells3 C{{n[0], n[1], n[2]}};
  const Dims3 D{{n[0], n[1], n[2]}};
  const int gr = grid_for(cells);
  hipLaunchKernelGGL(k_c4_cell_metrics, dim3(gr), dim3(256), 0, stream, s_dev, sc_tmp, C);
  for (int d = 0; d < 3; ++d)
    hipLaunchKernelGGL(k_c4_face_metrics, dim3(gr), dim3(256), 0, stream, self_line(sc_tmp, cells, n[d]),
                       self_line(jinv_dev, cells, n[d]), fm, D, d);
}

// The curvilinear viscous terms of a periodic block added into r (work: phi
// and gradients, 16 doubles per cell; fm: its face metrics).
void c4_viscous_curv_core(const double* q_dev, const double* s_dev, const double* jinv_dev, double* r_dev,
                          double* work, const double* fm, const int32_t n[3], const Gas<double>& gas,
                          hipStream_t stream, const RkArgs* rk) {
  const int64_t cells = (int64_t)n[0] * n[1] * n[2];
  double* phi = work;
  double* g = phi + 4 * cells;
  Line PG[3], FM[3], S[3];
  for (int d = 0; d < 3; ++d) {
    PG[d] = self_line(work, cells, n[d]);
    FM[d] = self_line(fm, cells, n[d]);
    S[d] = self_line(s_dev, cells, n[d]);
  }
  phi_grads_i_launch(self_line(q_dev, cells, n[0]), phi, g, n, gas.gm1, stream);
  grads_jk_launch(PG, g, n, stream);
  visc_fused_launch(PG, FM, S, r_dev, jinv_dev, n, gas, stream, rk);
}

}  // namespace cfd

namespace {

using cfd::block_cells;

}  // namespace

namespace cfd {

// Per-block offsets (in doubles) of `per` fields per cell.
std::vector<int64_t> field_offsets(int32_t nblk, const int32_t* dims, int per) {
  std::vector<int64_t> off(nblk + 1, 0);
  for (int b = 0; b < nblk; ++b) off[b + 1] = off[b] + per * block_cells(dims, b);
  return off;
}

// The line along d around block b over per-block arrays.
Line block_line(int b, int d, const int32_t* dims, const int32_t* nbr, const double* const* bases) {
  const int lo = nbr[6 * b + 2 * d], hi = nbr[6 * b + 2 * d + 1];
  return Line{bases[b], bases[lo], bases[hi], block_cells(dims, b), block_cells(dims, lo), block_cells(dims, hi),
              dims[3 * lo + d], dims[3 * hi + d]};
}

// Face metrics of blocks joined face to face into FM (21 doubles per cell of
// every block), once per grid; W (16 doubles per cell of every block) holds
// the cell metrics meanwhile.
void c4_face_metrics_blocks(int32_t nblk, const int32_t* dims, const int32_t* nbr, const double* const* s_dev,
                            const double* const* jinv_dev, double* W, double* FM, hipStream_t stream) {
  const std::vector<int64_t> off = field_offsets(nblk, dims, VW_FIELDS), offm = field_offsets(nblk, dims, FM_FIELDS);
  std::vector<const double*> sc(nblk);
  for (int b = 0; b < nblk; ++b) sc[b] = W + off[b];
  for (int b = 0; b < nblk; ++b) {
    const int64_t cb = block_cells(dims, b);
    const Dims3 D{{dims[3 * b], dims[3 * b + 1], dims[3 * b + 2]}};
    for (int t = 0; t < 3; ++t)
      hipLaunchKernelGGL(k_c4_cell_metrics_line, dim3(grid_for(cb)), dim3(256), 0, stream,
                         block_line(b, t, dims, nbr, s_dev), W + off[b], D, t);
  }
  for (int b = 0; b < nblk; ++b) {
    const int64_t cb = block_cells(dims, b);
    const Dims3 D{{dims[3 * b], dims[3 * b + 1], dims[3 * b + 2]}};
    for (int d = 0; d < 3; ++d)
      hipLaunchKernelGGL(k_c4_face_metrics, dim3(grid_for(cb)), dim3(256), 0, stream,
                         block_line(b, d, dims, nbr, sc.data()), block_line(b, d, dims, nbr, jinv_dev), FM + offm[b],
                         D, d);
  }
}

// The viscous terms of blocks joined face to face added into r (arguments
// checked by the caller; W: 16 doubles per cell of every block; FM: their
// face metrics from c4_face_metrics_blocks).
void c4_viscous_blocks_launch(int32_t nblk, const int32_t* dims, const int32_t* nbr, const double* const* q_dev,
                              const double* const* s_dev, const double* const* jinv_dev, double* const* r_dev,
                              double* W, const double* FM, const Gas<double>& gas, hipStream_t stream,
                              const char* skip = nullptr, const RkArgs* rk = nullptr) {
  const std::vector<int64_t> off = field_offsets(nblk, dims, VW_FIELDS), offm = field_offsets(nblk, dims, FM_FIELDS);
  std::vector<const double*> wb(nblk), fb(nblk);
  for (int b = 0; b < nblk; ++b) {
    wb[b] = W + off[b];
    fb[b] = FM + offm[b];
  }
  for (int b = 0; b < nblk; ++b) {
    const int64_t cb = block_cells(dims, b);
    phi_grads_i_launch(block_line(b, 0, dims, nbr, q_dev), W + off[b], W + off[b] + VW_G * cb, dims + 3 * b, gas.gm1,
                       stream);
  }
  for (int b = 0; b < nblk; ++b) {
    const int64_t cb = block_cells(dims, b);
    const Line P[3] = {block_line(b, 0, dims, nbr, wb.data()), block_line(b, 1, dims, nbr, wb.data()),
                       block_line(b, 2, dims, nbr, wb.data())};
    grads_jk_launch(P, W + off[b] + VW_G * cb, dims + 3 * b, stream);
  }
  for (int b = 0; b < nblk; ++b) {
    if (skip && skip[b]) continue;   // its u, v, w, T and gradients still serve the neighbours' stencils
    Line PG[3], FL[3], S[3];
    for (int d = 0; d < 3; ++d) {
      PG[d] = block_line(b, d, dims, nbr, wb.data());
      FL[d] = block_line(b, d, dims, nbr, fb.data());
      S[d] = block_line(b, d, dims, nbr, s_dev);
    }
    visc_fused_launch(PG, FL, S, r_dev[b], jinv_dev[b], dims + 3 * b, gas, stream, rk && rk[b].q ? rk + b : nullptr);
  }
}

}  // namespace cfd

extern "C" cfd_status cfd_c4_viscous_blocks_work_bytes(int32_t nblk, const int32_t* dims, const int32_t* nbr,
                                                       size_t* bytes) {
  return cfd::host_guarded([&] {
    if (!bytes) cfd::host_fail(CFD_EINVAL, "NULL argument");
    check_seams(nblk, dims, nbr);
    size_t total = 0;
    for (int b = 0; b < nblk; ++b) total += (size_t)8 * (cfd::VW_FIELDS + cfd::FM_FIELDS) * block_cells(dims, b);
    *bytes = total;
  });
}

extern "C" cfd_status cfd_c4_viscous_add_blocks(int32_t nblk, const int32_t* dims, const int32_t* nbr,
                                                const double* const* q_dev, const double* const* s_dev,
                                                const double* const* jinv_dev, double* const* r_dev, void* work_dev,
                                                size_t work_bytes, double gamma, double prandtl, double mu_inf,
                                                double s_star, hipStream_t stream) {
  return cfd::host_guarded([&] {
    check_seams(nblk, dims, nbr);
    if (!q_dev || !s_dev || !jinv_dev || !r_dev || !work_dev) cfd::host_fail(CFD_EINVAL, "NULL argument");
    if (!(gamma > 1.0) || !(prandtl > 0.0) || !(mu_inf >= 0.0) || !(s_star > 0.0) || !std::isfinite(mu_inf))
      cfd::host_fail(CFD_EINVAL, "bad gas parameters");
    const std::vector<int64_t> off = cfd::field_offsets(nblk, dims, cfd::VW_FIELDS + cfd::FM_FIELDS);
    const size_t need = (size_t)8 * off[nblk];
    if (work_bytes < need) cfd::host_fail(CFD_ENOMEM, "workspace smaller than cfd_c4_viscous_blocks_work_bytes()");
    std::vector<cfd::ArgSpan> spans{cfd::span(work_dev, (int64_t)need, true)};
    for (int b = 0; b < nblk; ++b) {
      if (!q_dev[b] || !s_dev[b] || !jinv_dev[b] || !r_dev[b]) cfd::host_fail(CFD_EINVAL, "NULL block pointer");
      const int64_t cb = cfd::block_cells(dims, b);
      spans.insert(spans.end(), {cfd::span(q_dev[b], 40 * cb, false), cfd::span(s_dev[b], 72 * cb, false),
                                 cfd::span(jinv_dev[b], 8 * cb, false), cfd::span(r_dev[b], 40 * cb, true)});
    }
    cfd::check_spans(spans, "a residual or the workspace overlaps an input, another residual or the workspace");
    double* W = static_cast<double*>(work_dev);
    double* FM = W + cfd::field_offsets(nblk, dims, cfd::VW_FIELDS)[nblk];
    cfd::c4_face_metrics_blocks(nblk, dims, nbr, s_dev, jinv_dev, W, FM, stream);
    cfd::c4_viscous_blocks_launch(nblk, dims, nbr, q_dev, s_dev, jinv_dev, r_dev, W, FM,
                                  cfd::viscous_gas(gamma, prandtl, mu_inf, s_star), stream);
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) cfd::host_fail(CFD_EHIP, std::string("kernel launch failed: ") + hipGetErrorString(e));
  });
}

// ------------------------------------------------ Navier-Stokes RK3 steps
extern "C" cfd_status cfd_wcns5_ns_step_work_bytes(const int32_t n[3], size_t* bytes) {
  return cfd::host_guarded([&] {
    if (!n || !bytes) cfd::host_fail(CFD_EINVAL, "NULL argument");
    if (n[0] < 1 || n[1] < 1 || n[2] < 1) cfd::host_fail(CFD_EINVAL, "every extent must be >= 1");
    const int64_t cells = (int64_t)n[0] * n[1] * n[2];
    *bytes = cfd::visc_region(wcns5_residual_work(n), cells) + (size_t)2 * 40 * cells;
  });
}

extern "C" cfd_status cfd_wcns5_ns_steps_curv_periodic(double* q_dev, const double* s_dev, const double* jinv_dev,
                                                       void* work_dev, size_t work_bytes, const int32_t n[3],
                                                       double gamma, double entropy_fix, double eps, double prandtl,
                                                       double mu_inf, double s_star, double dt, int32_t nsteps,
                                                       hipStream_t stream) {
  return cfd::host_guarded([&] {
    if (!q_dev || !s_dev || !jinv_dev || !work_dev || !n) cfd::host_fail(CFD_EINVAL, "NULL argument");
    if (!(gamma > 1.0) || !(prandtl > 0.0) || !(mu_inf >= 0.0) || !(s_star > 0.0) || !std::isfinite(mu_inf))
      cfd::host_fail(CFD_EINVAL, "bad gas parameters");
    const cfd::Gas<double> gas = cfd::viscous_gas(gamma, prandtl, mu_inf, s_star);
    cfd::wcns5_steps_core(q_dev, s_dev, jinv_dev, work_dev, work_bytes, n, nullptr, gamma, entropy_fix, eps, dt, nsteps,
                          stream, &gas);
  });
}

// ------------------------------------------------------------ implicit step
// Backward Euler (I/dt + dR/dQ) dQ = -R on a periodic curvilinear block with
// the flux-split approximate Jacobian A+- = (A +- lambda I)/2 at every face
// (lambda = |u . S| + c |S| of the mean primitive state of the face's two
// cells) relaxed by point-Jacobi sweeps: the paper's flowchart solves a sparse
// linear system per step without naming the method; this one is data parallel.
//   D_i = 1/dt + J_i sum_d (lambda_{i+1/2} + lambda_{i-1/2}) / 2
//   dQ_i <- (-R_i - J_i sum_d [(dF_{i+1} - lambda_{i+1/2} dQ_{i+1})
//                              - (dF_{i-1} + lambda_{i-1/2} dQ_{i-1})] / 2) / D_i
// with dF_m = F(Q_m + dQ_m) . S - F(Q_m) . S through the face between.
namespace cfd {

__device__ __forceinline__ void euler_flux_dot(double q0, double q1, double q2, double q3, double q4, double sx,
                                               double sy, double sz, double gm1, double F[5]) {
  const Prim<double> w = to_prim<double>(q0, q1, q2, q3, q4, gm1);
  const double U = w.u * sx + w.v * sy + w.w * sz;
  F[0] = q0 * U;
  F[1] = q1 * U + w.p * sx;
  F[2] = q2 * U + w.p * sy;
  F[3] = q3 * U + w.p * sz;
  F[4] = (q4 + w.p) * U;
}

// lam[d * cells + c]: the spectral radius at face c + 1/2 along d.
__global__ void __launch_bounds__(256) k_impl_lambda(const double* __restrict__ q, const double* __restrict__ s,
                                                     const double* __restrict__ jinv, double* __restrict__ lam,
                                                     double* __restrict__ lamv, Cells3 C, double gamma,
                                                     Gas<double> visc, int viscous) {
  const int64_t cells = (int64_t)C.n[0] * C.n[1] * C.n[2];
  const double gm1 = gamma - 1.0;
  for (int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; c < cells; c += (int64_t)gridDim.x * blockDim.x) {
    const int i = (int)(c % C.n[0]), j = (int)((c / C.n[0]) % C.n[1]), k = (int)(c / ((int64_t)C.n[0] * C.n[1]));
    const Prim<double> a = to_prim<double>(q[c], q[cells + c], q[2 * cells + c], q[3 * cells + c], q[4 * cells + c],
                                           gm1);
    for (int d = 0; d < 3; ++d) {
      const int64_t p = C.step(i, j, k, d, 1);
      const Prim<double> b = to_prim<double>(q[p], q[cells + p], q[2 * cells + p], q[3 * cells + p],
                                             q[4 * cells + p], gm1);
      const double r = 0.5 * (a.r + b.r), u = 0.5 * (a.u + b.u), v = 0.5 * (a.v + b.v), w = 0.5 * (a.w + b.w),
                   pr = 0.5 * (a.p + b.p);
      const double* sd = s + 3 * d * cells;
      const double sx = sd[c], sy = sd[cells + c], sz = sd[2 * cells + c];
      lam[d * cells + c] = fabs(u * sx + v * sy + w * sz) + sqrt(gamma * pr / r) * sqrt(sx * sx + sy * sy + sz * sz);
      if (viscous) {
        const double Ta = a.p / a.r, Tb = b.p / b.r;
        const double na = visc.mu_inf * Ta * sqrt(Ta) * (1.0 + visc.s_star) / (Ta + visc.s_star) / a.r;
        const double nb = visc.mu_inf * Tb * sqrt(Tb) * (1.0 + visc.s_star) / (Tb + visc.s_star) / b.r;
        const double num = 0.5 * (na + nb), jm = 0.5 * (jinv[c] + jinv[p]);
        lamv[d * cells + c] = fmax(4.0 / 3.0, gamma / visc.prandtl) * num * (sx * sx + sy * sy + sz * sz) / jm;
      }
    }
  }
}

// The diagonal D and the first iterate dQ = -R / D.
__global__ void __launch_bounds__(256) k_impl_diag(const double* __restrict__ r, const double* __restrict__ lam,
                                                   const double* __restrict__ lamv, const double* __restrict__ jinv,
                                                   double* __restrict__ diag, double* __restrict__ dq, Cells3 C,
                                                   double dt, int viscous) {
  const int64_t cells = (int64_t)C.n[0] * C.n[1] * C.n[2];
  for (int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; c < cells; c += (int64_t)gridDim.x * blockDim.x) {
    const int i = (int)(c % C.n[0]), j = (int)((c / C.n[0]) % C.n[1]), k = (int)(c / ((int64_t)C.n[0] * C.n[1]));
    double sum = 0.0;
    for (int d = 0; d < 3; ++d) {
      const int64_t m = C.step(i, j, k, d, -1);
      const double t = 0.5 * (lam[d * cells + c] + lam[d * cells + m]);
      sum = sum + (viscous ? t + (lamv[d * cells + c] + lamv[d * cells + m]) : t);
    }
    const double D = 1.0 / dt + (1.0 / jinv[c]) * sum;
    diag[c] = D;
    for (int v = 0; v < 5; ++v) dq[v * cells + c] = -r[v * cells + c] / D;
  }
}

// One Jacobi sweep: dq_in -> dq_out.
__global__ void __launch_bounds__(256) k_impl_sweep(const double* __restrict__ q, const double* __restrict__ r,
                                                    const double* __restrict__ s, const double* __restrict__ lam,
                                                    const double* __restrict__ lamv, const double* __restrict__ jinv,
                                                    const double* __restrict__ diag, const double* __restrict__ dq_in,
                                                    double* __restrict__ dq_out, Cells3 C, double gm1, int viscous) {
  const int64_t cells = (int64_t)C.n[0] * C.n[1] * C.n[2];
  for (int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; c < cells; c += (int64_t)gridDim.x * blockDim.x) {
    const int i = (int)(c % C.n[0]), j = (int)((c / C.n[0]) % C.n[1]), k = (int)(c / ((int64_t)C.n[0] * C.n[1]));
    double O[5] = {0.0, 0.0, 0.0, 0.0, 0.0};
    for (int d = 0; d < 3; ++d) {
      const int64_t p = C.step(i, j, k, d, 1), m = C.step(i, j, k, d, -1);
      const double* sd = s + 3 * d * cells;
      const double lp = lam[d * cells + c], lm = lam[d * cells + m];
      double Fa[5], Fb[5], dFp[5], dFm[5];
      {
        const double sx = sd[c], sy = sd[cells + c], sz = sd[2 * cells + c];
        euler_flux_dot(q[p] + dq_in[p], q[cells + p] + dq_in[cells + p], q[2 * cells + p] + dq_in[2 * cells + p],
                       q[3 * cells + p] + dq_in[3 * cells + p], q[4 * cells + p] + dq_in[4 * cells + p], sx, sy, sz,
                       gm1, Fa);
        euler_flux_dot(q[p], q[cells + p], q[2 * cells + p], q[3 * cells + p], q[4 * cells + p], sx, sy, sz, gm1, Fb);
        for (int v = 0; v < 5; ++v) dFp[v] = Fa[v] - Fb[v];
      }
      {
        const double sx = sd[m], sy = sd[cells + m], sz = sd[2 * cells + m];
        euler_flux_dot(q[m] + dq_in[m], q[cells + m] + dq_in[cells + m], q[2 * cells + m] + dq_in[2 * cells + m],
                       q[3 * cells + m] + dq_in[3 * cells + m], q[4 * cells + m] + dq_in[4 * cells + m], sx, sy, sz,
                       gm1, Fa);
        euler_flux_dot(q[m], q[cells + m], q[2 * cells + m], q[3 * cells + m], q[4 * cells + m], sx, sy, sz, gm1, Fb);
        for (int v = 0; v < 5; ++v) dFm[v] = Fa[v] - Fb[v];
      }
      const double vp = viscous ? lamv[d * cells + c] : 0.0, vm = viscous ? lamv[d * cells + m] : 0.0;
      for (int v = 0; v < 5; ++v) {
        O[v] = O[v] + 0.5 * ((dFp[v] - lp * dq_in[v * cells + p]) - (dFm[v] + lm * dq_in[v * cells + m]));
        if (viscous) O[v] = O[v] - (vp * dq_in[v * cells + p] + vm * dq_in[v * cells + m]);
      }
    }
    const double J = 1.0 / jinv[c], D = diag[c];
    for (int v = 0; v < 5; ++v) dq_out[v * cells + c] = (-r[v * cells + c] - J * O[v]) / D;
  }
}

__global__ void __launch_bounds__(256) k_impl_apply(double* __restrict__ q, const double* __restrict__ dq, int64_t n) {
  for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < n; t += (int64_t)gridDim.x * blockDim.x)
    q[t] = q[t] + dq[t];
}

}  // namespace cfd

extern "C" cfd_status cfd_wcns5_implicit_step_work_bytes(const int32_t n[3], size_t* bytes) {
  return cfd::host_guarded([&] {
    if (!n || !bytes) cfd::host_fail(CFD_EINVAL, "NULL argument");
    if (n[0] < 1 || n[1] < 1 || n[2] < 1) cfd::host_fail(CFD_EINVAL, "every extent must be >= 1");
    const int64_t cells = (int64_t)n[0] * n[1] * n[2];
    // scratch of the residual or the viscous terms, the viscous face metrics, then R, two dQ, lambda (3),
    // viscous lambda (3), D
    *bytes = cfd::visc_region(wcns5_residual_work(n), cells) + (size_t)8 * 22 * cells;
  });
}

extern "C" cfd_status cfd_wcns5_implicit_steps_curv_periodic(double* q_dev, const double* s_dev,
                                                             const double* jinv_dev, void* work_dev,
                                                             size_t work_bytes, const int32_t n[3], double gamma,
                                                             double entropy_fix, double eps, int32_t viscous,
                                                             double prandtl, double mu_inf, double s_star, double dt,
                                                             int32_t nsteps, int32_t sweeps, hipStream_t stream) {
  return cfd::host_guarded([&] {
    if (!q_dev || !s_dev || !jinv_dev || !work_dev || !n) cfd::host_fail(CFD_EINVAL, "NULL argument");
    if (n[0] < 1 || n[1] < 1 || n[2] < 1) cfd::host_fail(CFD_EINVAL, "every extent must be >= 1");
    if (!(dt > 0.0) || !std::isfinite(dt)) cfd::host_fail(CFD_EINVAL, "dt must be positive and finite");
    if (nsteps < 0 || sweeps < 0 || sweeps > 1000) cfd::host_fail(CFD_EINVAL, "nsteps >= 0, sweeps in [0, 1000]");
    if (!(gamma > 1.0) || !std::isfinite(gamma)) cfd::host_fail(CFD_EINVAL, "gamma must exceed 1");
    if (viscous && (!(prandtl > 0.0) || !(mu_inf >= 0.0) || !(s_star > 0.0) || !std::isfinite(mu_inf)))
      cfd::host_fail(CFD_EINVAL, "bad gas parameters");
    const int64_t cells = (int64_t)n[0] * n[1] * n[2];
    const size_t rw0 = wcns5_residual_work(n);
    const size_t rw = cfd::visc_region(rw0, cells);
    const size_t need = rw + (size_t)8 * 22 * cells;
    if (work_bytes < need) cfd::host_fail(CFD_ENOMEM, "workspace smaller than cfd_wcns5_implicit_step_work_bytes()");
    if (!cfd::apart(q_dev, 40 * cells, work_dev, (int64_t)work_bytes) ||
        !cfd::apart(q_dev, 40 * cells, s_dev, 72 * cells) || !cfd::apart(q_dev, 40 * cells, jinv_dev, 8 * cells))
      cfd::host_fail(CFD_EINVAL, "q must not overlap the workspace or the metrics");
    if (!cfd::apart(work_dev, (int64_t)work_bytes, s_dev, 72 * cells) ||
        !cfd::apart(work_dev, (int64_t)work_bytes, jinv_dev, 8 * cells))
      cfd::host_fail(CFD_EINVAL, "the workspace must not overlap the metrics");
    double* R = reinterpret_cast<double*>(static_cast<char*>(work_dev) + rw);
    double* dqa = R + 5 * cells;
    double* dqb = dqa + 5 * cells;
    double* lam = dqb + 5 * cells;
    double* lamv = lam + 3 * cells;
    double* diag = lamv + 3 * cells;
    const cfd::Gas<double> vgas = cfd::viscous_gas(gamma, viscous ? prandtl : 1.0, mu_inf, s_star);
    const cfd::Cells3 C{{n[0], n[1], n[2]}};
    const int gr = cfd::grid_for(cells);
    double* fm = reinterpret_cast<double*>(static_cast<char*>(work_dev) + cfd::visc_fm_offset(rw0, cells));
    if (viscous && nsteps > 0)
      cfd::c4_face_metrics_curv(s_dev, jinv_dev, static_cast<double*>(work_dev), fm, n, stream);
    for (int it = 0; it < nsteps; ++it) {
      cfd::wcns5_residual_core(q_dev, s_dev, jinv_dev, R, work_dev, rw0, n, nullptr, gamma, entropy_fix, eps, stream);
      if (viscous)
        cfd::c4_viscous_curv_core(q_dev, s_dev, jinv_dev, R, static_cast<double*>(work_dev), fm, n, vgas, stream);
      hipLaunchKernelGGL(cfd::k_impl_lambda, dim3(gr), dim3(256), 0, stream, q_dev, s_dev, jinv_dev, lam, lamv, C,
                         gamma, vgas, viscous ? 1 : 0);
      hipLaunchKernelGGL(cfd::k_impl_diag, dim3(gr), dim3(256), 0, stream, R, lam, lamv, jinv_dev, diag, dqa, C, dt,
                         viscous ? 1 : 0);
      double *cur = dqa, *nxt = dqb;
      for (int k = 0; k < sweeps; ++k) {
        hipLaunchKernelGGL(cfd::k_impl_sweep, dim3(gr), dim3(256), 0, stream, q_dev, R, s_dev, lam, lamv, jinv_dev,
                           diag, cur, nxt, C, gamma - 1.0, viscous ? 1 : 0);
        std::swap(cur, nxt);
      }
      hipLaunchKernelGGL(cfd::k_impl_apply, dim3(cfd::grid_for(5 * cells)), dim3(256), 0, stream, q_dev, cur,
                         5 * cells);
    }
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) cfd::host_fail(CFD_EHIP, std::string("kernel launch failed: ") + hipGetErrorString(e));
  });
}

// ------------------------------------------- implicit steps on joined blocks
// The implicit kernels above with every neighbour read through the tables of
// blocks joined face to face (Line): a sweep reads only the previous iterate,
// so the iteration, and its bits, do not depend on how the domain is cut.
namespace cfd {

struct Lines3 {
  Line l[3];
};

__global__ void __launch_bounds__(256) k_impl_lambda_line(const double* __restrict__ q, Lines3 Q,
                                                          const double* __restrict__ s,
                                                          const double* __restrict__ jinv, Lines3 JL,
                                                          double* __restrict__ lam, double* __restrict__ lamv,
                                                          Dims3 D, double gamma, Gas<double> visc, int viscous) {
  const int64_t cells = (int64_t)D.n[0] * D.n[1] * D.n[2];
  const double gm1 = gamma - 1.0;
  for (int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; c < cells; c += (int64_t)gridDim.x * blockDim.x) {
    const int i = (int)(c % D.n[0]), j = (int)((c / D.n[0]) % D.n[1]), k = (int)(c / ((int64_t)D.n[0] * D.n[1]));
    const Prim<double> a = to_prim<double>(q[c], q[cells + c], q[2 * cells + c], q[3 * cells + c], q[4 * cells + c],
                                           gm1);
    for (int d = 0; d < 3; ++d) {
      const Line& L = Q.l[d];
      const Prim<double> b = to_prim<double>(line_at(L, 0, i, j, k, 1, d, D.n), line_at(L, 1, i, j, k, 1, d, D.n),
                                             line_at(L, 2, i, j, k, 1, d, D.n), line_at(L, 3, i, j, k, 1, d, D.n),
                                             line_at(L, 4, i, j, k, 1, d, D.n), gm1);
      const double r = 0.5 * (a.r + b.r), u = 0.5 * (a.u + b.u), v = 0.5 * (a.v + b.v), w = 0.5 * (a.w + b.w),
                   pr = 0.5 * (a.p + b.p);
      const double* sd = s + 3 * d * cells;
      const double sx = sd[c], sy = sd[cells + c], sz = sd[2 * cells + c];
      lam[d * cells + c] = fabs(u * sx + v * sy + w * sz) + sqrt(gamma * pr / r) * sqrt(sx * sx + sy * sy + sz * sz);
      if (viscous) {
        const double Ta = a.p / a.r, Tb = b.p / b.r;
        const double na = visc.mu_inf * Ta * sqrt(Ta) * (1.0 + visc.s_star) / (Ta + visc.s_star) / a.r;
        const double nb = visc.mu_inf * Tb * sqrt(Tb) * (1.0 + visc.s_star) / (Tb + visc.s_star) / b.r;
        const double num = 0.5 * (na + nb), jm = 0.5 * (jinv[c] + line_at(JL.l[d], 0, i, j, k, 1, d, D.n));
        lamv[d * cells + c] = fmax(4.0 / 3.0, gamma / visc.prandtl) * num * (sx * sx + sy * sy + sz * sz) / jm;
      }
    }
  }
}

__global__ void __launch_bounds__(256) k_impl_diag_line(const double* __restrict__ r, const double* __restrict__ lam,
                                                        Lines3 L, const double* __restrict__ lamv, Lines3 LV,
                                                        const double* __restrict__ jinv, double* __restrict__ diag,
                                                        double* __restrict__ dq, Dims3 D, double dt, int viscous) {
  const int64_t cells = (int64_t)D.n[0] * D.n[1] * D.n[2];
  for (int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; c < cells; c += (int64_t)gridDim.x * blockDim.x) {
    const int i = (int)(c % D.n[0]), j = (int)((c / D.n[0]) % D.n[1]), k = (int)(c / ((int64_t)D.n[0] * D.n[1]));
    double sum = 0.0;
    for (int d = 0; d < 3; ++d) {
      const double t = 0.5 * (lam[d * cells + c] + line_at(L.l[d], d, i, j, k, -1, d, D.n));
      sum = sum + (viscous ? t + (lamv[d * cells + c] + line_at(LV.l[d], d, i, j, k, -1, d, D.n)) : t);
    }
    const double Dg = 1.0 / dt + (1.0 / jinv[c]) * sum;
    diag[c] = Dg;
    for (int v = 0; v < 5; ++v) dq[v * cells + c] = -r[v * cells + c] / Dg;
  }
}

__global__ void __launch_bounds__(256) k_impl_sweep_line(Lines3 Q, Lines3 DQ, Lines3 S, Lines3 L, Lines3 LV,
                                                         int viscous, const double* __restrict__ r,
                                                         const double* __restrict__ s, const double* __restrict__ lam,
                                                         const double* __restrict__ lamv,
                                                         const double* __restrict__ jinv,
                                                         const double* __restrict__ diag, double* __restrict__ dq_out,
                                                         Dims3 D, double gm1) {
  const int64_t cells = (int64_t)D.n[0] * D.n[1] * D.n[2];
  for (int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; c < cells; c += (int64_t)gridDim.x * blockDim.x) {
    const int i = (int)(c % D.n[0]), j = (int)((c / D.n[0]) % D.n[1]), k = (int)(c / ((int64_t)D.n[0] * D.n[1]));
    double O[5] = {0.0, 0.0, 0.0, 0.0, 0.0};
    for (int d = 0; d < 3; ++d) {
      double qp[5], dqp[5], qm[5], dqm[5];
      for (int v = 0; v < 5; ++v) {
        qp[v] = line_at(Q.l[d], v, i, j, k, 1, d, D.n);
        dqp[v] = line_at(DQ.l[d], v, i, j, k, 1, d, D.n);
        qm[v] = line_at(Q.l[d], v, i, j, k, -1, d, D.n);
        dqm[v] = line_at(DQ.l[d], v, i, j, k, -1, d, D.n);
      }
      const double* sd = s + 3 * d * cells;
      const double lp = lam[d * cells + c], lm = line_at(L.l[d], d, i, j, k, -1, d, D.n);
      double Fa[5], Fb[5], dFp[5], dFm[5];
      {
        const double sx = sd[c], sy = sd[cells + c], sz = sd[2 * cells + c];
        euler_flux_dot(qp[0] + dqp[0], qp[1] + dqp[1], qp[2] + dqp[2], qp[3] + dqp[3], qp[4] + dqp[4], sx, sy, sz,
                       gm1, Fa);
        euler_flux_dot(qp[0], qp[1], qp[2], qp[3], qp[4], sx, sy, sz, gm1, Fb);
        for (int v = 0; v < 5; ++v) dFp[v] = Fa[v] - Fb[v];
      }
      {
        const double sx = line_at(S.l[d], 3 * d, i, j, k, -1, d, D.n),
                     sy = line_at(S.l[d], 3 * d + 1, i, j, k, -1, d, D.n),
                     sz = line_at(S.l[d], 3 * d + 2, i, j, k, -1, d, D.n);
        euler_flux_dot(qm[0] + dqm[0], qm[1] + dqm[1], qm[2] + dqm[2], qm[3] + dqm[3], qm[4] + dqm[4], sx, sy, sz,
                       gm1, Fa);
        euler_flux_dot(qm[0], qm[1], qm[2], qm[3], qm[4], sx, sy, sz, gm1, Fb);
        for (int v = 0; v < 5; ++v) dFm[v] = Fa[v] - Fb[v];
      }
      const double vp = viscous ? lamv[d * cells + c] : 0.0,
                   vm = viscous ? line_at(LV.l[d], d, i, j, k, -1, d, D.n) : 0.0;
      for (int v = 0; v < 5; ++v) {
        O[v] = O[v] + 0.5 * ((dFp[v] - lp * dqp[v]) - (dFm[v] + lm * dqm[v]));
        if (viscous) O[v] = O[v] - (vp * dqp[v] + vm * dqm[v]);
      }
    }
    const double J = 1.0 / jinv[c], Dg = diag[c];
    for (int v = 0; v < 5; ++v) dq_out[v * cells + c] = (-r[v * cells + c] - J * O[v]) / Dg;
  }
}

}  // namespace cfd

extern "C" cfd_status cfd_wcns5_implicit_blocks_work_bytes(int32_t nblk, const int32_t* dims, const int32_t* nbr,
                                                           size_t* bytes) {
  return cfd::host_guarded([&] {
    if (!bytes) cfd::host_fail(CFD_EINVAL, "NULL argument");
    const size_t rscratch = check_seams(nblk, dims, nbr);
    size_t vscratch = 0, fmb = 0, rest = 0;
    for (int b = 0; b < nblk; ++b) {
      vscratch += (size_t)8 * cfd::VW_FIELDS * block_cells(dims, b);   // the viscous terms' scratch
      fmb += (size_t)8 * cfd::FM_FIELDS * block_cells(dims, b);        // their face metrics
      rest += (size_t)8 * 22 * block_cells(dims, b);                   // R, two dQ, radii (3 + 3), D
    }
    *bytes = std::max(rscratch, vscratch) + fmb + rest;
  });
}

extern "C" cfd_status cfd_wcns5_implicit_steps_blocks(int32_t nblk, const int32_t* dims, const int32_t* nbr,
                                                      double* const* q_dev, const double* const* s_dev,
                                                      const double* const* jinv_dev, void* work_dev,
                                                      size_t work_bytes, double gamma, double entropy_fix, double eps,
                                                      int32_t viscous, double prandtl, double mu_inf, double s_star,
                                                      double dt, int32_t nsteps, int32_t sweeps, hipStream_t stream) {
  return cfd::host_guarded([&] {
    const size_t rscratch = check_seams(nblk, dims, nbr);
    if (viscous && (!(prandtl > 0.0) || !(mu_inf >= 0.0) || !(s_star > 0.0) || !std::isfinite(mu_inf)))
      cfd::host_fail(CFD_EINVAL, "bad gas parameters");
    size_t vscratch = 0, fmb = 0;
    for (int b = 0; b < nblk; ++b) {
      vscratch += (size_t)8 * cfd::VW_FIELDS * block_cells(dims, b);
      fmb += (size_t)8 * cfd::FM_FIELDS * block_cells(dims, b);
    }
    const size_t shared = std::max(rscratch, vscratch);
    const size_t scratch = shared + fmb;
    if (!q_dev || !s_dev || !jinv_dev || !work_dev) cfd::host_fail(CFD_EINVAL, "NULL argument");
    if (!(gamma > 1.0) || !std::isfinite(gamma)) cfd::host_fail(CFD_EINVAL, "gamma must exceed 1");
    if (!(entropy_fix >= 0.0) || !std::isfinite(entropy_fix)) cfd::host_fail(CFD_EINVAL, "bad entropy_fix");
    if (!(eps > 0.0) || !std::isfinite(eps)) cfd::host_fail(CFD_EINVAL, "eps must be positive and finite");
    if (!(dt > 0.0) || !std::isfinite(dt)) cfd::host_fail(CFD_EINVAL, "dt must be positive and finite");
    if (nsteps < 0 || sweeps < 0 || sweeps > 1000) cfd::host_fail(CFD_EINVAL, "nsteps >= 0, sweeps in [0, 1000]");
    std::vector<int64_t> off(nblk + 1, 0);
    for (int b = 0; b < nblk; ++b) off[b + 1] = off[b] + 22 * block_cells(dims, b);
    const size_t need = scratch + (size_t)8 * off[nblk];
    if (work_bytes < need) cfd::host_fail(CFD_ENOMEM, "workspace smaller than cfd_wcns5_implicit_blocks_work_bytes()");
    std::vector<cfd::ArgSpan> spans{cfd::span(work_dev, (int64_t)need, true)};
    for (int b = 0; b < nblk; ++b) {
      if (!q_dev[b] || !s_dev[b] || !jinv_dev[b]) cfd::host_fail(CFD_EINVAL, "NULL block pointer");
      const int64_t cb = cfd::block_cells(dims, b);
      spans.insert(spans.end(), {cfd::span(q_dev[b], 40 * cb, true), cfd::span(s_dev[b], 72 * cb, false),
                                 cfd::span(jinv_dev[b], 8 * cb, false)});
    }
    cfd::check_spans(spans, "a state or the workspace overlaps the metrics, another state or the workspace");
    double* base = reinterpret_cast<double*>(static_cast<char*>(work_dev) + scratch);
    std::vector<double*> R(nblk), dqa(nblk), dqb(nblk), lam(nblk), lamv(nblk), diag(nblk);
    for (int b = 0; b < nblk; ++b) {
      const int64_t cb = block_cells(dims, b);
      R[b] = base + off[b];
      dqa[b] = R[b] + 5 * cb;
      dqb[b] = dqa[b] + 5 * cb;
      lam[b] = dqb[b] + 5 * cb;
      lamv[b] = lam[b] + 3 * cb;
      diag[b] = lamv[b] + 3 * cb;
    }
    const cfd::Gas<double> vgas = cfd::viscous_gas(gamma, viscous ? prandtl : 1.0, mu_inf, s_star);
    auto lines = [&](int b, const std::vector<const double*>& arr) {
      cfd::Lines3 L{};
      for (int d = 0; d < 3; ++d) {
        const int lo = nbr[6 * b + 2 * d], hi = nbr[6 * b + 2 * d + 1];
        L.l[d] = cfd::Line{arr[b], arr[lo], arr[hi], block_cells(dims, b), block_cells(dims, lo), block_cells(dims, hi),
                           dims[3 * lo + d], dims[3 * hi + d]};
      }
      return L;
    };
    std::vector<const double*> qv(q_dev, q_dev + nblk), sv(s_dev, s_dev + nblk), jv(jinv_dev, jinv_dev + nblk),
        lamc(lam.begin(), lam.end()), lamvc(lamv.begin(), lamv.end());
    std::vector<double*> rv(R.begin(), R.end());
    double* FM = reinterpret_cast<double*>(static_cast<char*>(work_dev) + shared);
    if (viscous && nsteps > 0)
      cfd::c4_face_metrics_blocks(nblk, dims, nbr, s_dev, jinv_dev, static_cast<double*>(work_dev), FM, stream);
    for (int it = 0; it < nsteps; ++it) {
      cfd::wcns5_blocks_residual_launch(nblk, dims, nbr, q_dev, s_dev, jinv_dev, rv.data(), work_dev, gamma,
                                        entropy_fix, eps, stream);
      if (viscous)
        cfd::c4_viscous_blocks_launch(nblk, dims, nbr, q_dev, s_dev, jinv_dev, rv.data(),
                                      static_cast<double*>(work_dev), FM, vgas, stream);
      for (int b = 0; b < nblk; ++b) {
        const int64_t cb = block_cells(dims, b);
        const cfd::Dims3 D{{dims[3 * b], dims[3 * b + 1], dims[3 * b + 2]}};
        hipLaunchKernelGGL(cfd::k_impl_lambda_line, dim3(cfd::grid_for(cb)), dim3(256), 0, stream, q_dev[b],
                           lines(b, qv), s_dev[b], jinv_dev[b], lines(b, jv), lam[b], lamv[b], D, gamma, vgas,
                           viscous ? 1 : 0);
      }
      for (int b = 0; b < nblk; ++b) {
        const int64_t cb = block_cells(dims, b);
        const cfd::Dims3 D{{dims[3 * b], dims[3 * b + 1], dims[3 * b + 2]}};
        hipLaunchKernelGGL(cfd::k_impl_diag_line, dim3(cfd::grid_for(cb)), dim3(256), 0, stream, R[b], lam[b],
                           lines(b, lamc), lamv[b], lines(b, lamvc), jinv_dev[b], diag[b], dqa[b], D, dt,
                           viscous ? 1 : 0);
      }
      std::vector<double*> cur = dqa, nxt = dqb;
      for (int k = 0; k < sweeps; ++k) {
        std::vector<const double*> curv(cur.begin(), cur.end());
        for (int b = 0; b < nblk; ++b) {
          const int64_t cb = block_cells(dims, b);
          const cfd::Dims3 D{{dims[3 * b], dims[3 * b + 1], dims[3 * b + 2]}};
          hipLaunchKernelGGL(cfd::k_impl_sweep_line, dim3(cfd::grid_for(cb)), dim3(256), 0, stream, lines(b, qv),
                             lines(b, curv), lines(b, sv), lines(b, lamc), lines(b, lamvc), viscous ? 1 : 0, R[b],
                             s_dev[b], lam[b], lamv[b], jinv_dev[b], diag[b], nxt[b], D, gamma - 1.0);
        }
        std::swap(cur, nxt);
      }
      for (int b = 0; b < nblk; ++b) {
        const int64_t cb = block_cells(dims, b);
        hipLaunchKernelGGL(cfd::k_impl_apply, dim3(cfd::grid_for(5 * cb)), dim3(256), 0, stream, q_dev[b], cur[b],
                           5 * cb);
      }
    }
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) cfd::host_fail(CFD_EHIP, std::string("kernel launch failed: ") + hipGetErrorString(e));
  });
}

// ------------------------------------- Navier-Stokes RK3 steps on joined blocks
extern "C" cfd_status cfd_wcns5_ns_blocks_work_bytes(int32_t nblk, const int32_t* dims, const int32_t* nbr,
                                                     size_t* bytes) {
  return cfd::host_guarded([&] {
    if (!bytes) cfd::host_fail(CFD_EINVAL, "NULL argument");
    const size_t rscratch = check_seams(nblk, dims, nbr);
    size_t vscratch = 0, states = 0;
    for (int b = 0; b < nblk; ++b) {
      vscratch += (size_t)8 * cfd::VW_FIELDS * block_cells(dims, b);
      states += (size_t)8 * (10 + cfd::FM_FIELDS) * block_cells(dims, b);   // Q^n, R, viscous face metrics
    }
    *bytes = std::max(rscratch, vscratch) + states;
  });
}

namespace cfd {

// ------------------------------------------------ closures at physical faces
// Walls and the far field of the WCNS-E-5 scheme as ghost blocks: five-cell
// blocks joined to an owner across the two faces of one bounded direction
// (whose transverse directions are periodic), with metrics from the owner's
// vertex lines extended by linear extrapolation and states refilled from the
// owner before every residual (mirrored for walls, the characteristic state
// for the far field).  The owner's residual is then the joined-block residual.

constexpr int WCNS_GHOST = 5;

struct Period9 {
  double p[9];   // displacement over one period along direction d: p[3 d + component]
};

// Vertices of a block extended for its metrics and its ghost blocks'
// (cfd_wcns5_extend_vertices_mask): along a periodic direction vertex v of
// the output is vertex v mod n plus floor(v / n) periods; along a bounded one
// plane pl = -XL .. n + XL, copied for 0 <= pl <= n, else continued linearly
// from the two planes at that end.  With two bounded directions the first
// (lower) is continued first and the second from those values, so a corner
// vertex continues the continued planes.
__global__ void __launch_bounds__(256) k_extend_vertices(const double* __restrict__ xv, int ni, int nj, int nk,
                                                         int mask, Period9 P, double* __restrict__ xe, int ei,
                                                         int ej, int ek) {
  const int n[3] = {ni, nj, nk};
  const int s[3] = {ni + ((mask >> 0) & 1), nj + ((mask >> 1) & 1), nk + ((mask >> 2) & 1)};
  const int64_t scells = (int64_t)s[0] * s[1] * s[2];
  const int64_t total = (int64_t)ei * ej * ek;
  int bd[2] = {-1, -1}, nb = 0;
  for (int d = 0; d < 3; ++d)
    if ((mask >> d) & 1) bd[nb++] = d;
  for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < total; t += (int64_t)gridDim.x * blockDim.x) {
    const int e[3] = {(int)(t % ei), (int)((t / ei) % ej), (int)(t / ((int64_t)ei * ej))};
    int src[3], q[3] = {0, 0, 0}, a[3] = {0, 0, 0}, b[3] = {0, 0, 0}, m[3] = {0, 0, 0};
    for (int d = 0; d < 3; ++d) {
      if ((mask >> d) & 1) {
        const int pl = e[d] - CFD_WCNS5_XLAYERS;
        if (pl < 0) {
          a[d] = 0, b[d] = 1, m[d] = -pl;
        } else if (pl > n[d]) {
          a[d] = n[d], b[d] = n[d] - 1, m[d] = pl - n[d];
        } else {
          a[d] = pl, b[d] = pl, m[d] = 0;
        }
        src[d] = 0;
      } else {
        const int v = e[d] - 3;
        const int w = ((v % n[d]) + n[d]) % n[d];
        src[d] = w;
        q[d] = (v - w) / n[d];
      }
    }
    for (int c = 0; c < 3; ++c) {
      // the wrapped vertex at the bounded-direction indices idx, plus its periods
      auto at = [&](const int idx[3]) {
        double x = xv[c * scells + ((int64_t)idx[2] * s[1] + idx[1]) * s[0] + idx[0]];
        for (int d = 0; d < 3; ++d)
          if (!((mask >> d) & 1)) x = x + (double)q[d] * P.p[3 * d + c];
        return x;
      };
      // continued along the first bounded direction (if any) at second-direction plane p2
      auto first = [&](int p2) {
        int i0[3] = {src[0], src[1], src[2]}, i1[3] = {src[0], src[1], src[2]};
        if (nb > 0) {
          i0[bd[0]] = a[bd[0]];
          i1[bd[0]] = b[bd[0]];
        }
        if (nb > 1) i0[bd[1]] = i1[bd[1]] = p2;
        const double x0 = at(i0);
        if (nb == 0 || m[bd[0]] == 0) return x0;
        const double x1 = at(i1);
        return x0 + (double)m[bd[0]] * (x0 - x1);
      };
      double x;
      if (nb < 2) {
        x = first(0);
      } else {
        const double y0 = first(a[bd[1]]);
        if (m[bd[1]] == 0) {
          x = y0;
        } else {
          const double y1 = first(b[bd[1]]);
          x = y0 + (double)m[bd[1]] * (y0 - y1);
        }
      }
      xe[c * total + t] = x;
    }
  }
}

// Ghost-block states (cfd_wcns5_fill_ghost_blocks): one thread per side,
// layer m = 1 .. 5 and transverse point.
__global__ void __launch_bounds__(256) k_fill_ghost_blocks(const double* __restrict__ q, double* __restrict__ qlo,
                                                           double* __restrict__ qhi, const double* __restrict__ slo,
                                                           const double* __restrict__ sown, int ni, int nj, int nk,
                                                           int d, int kind_lo, int kind_hi, double gamma, double ux,
                                                           double uy, double uz) {
  const int n[3] = {ni, nj, nk};
  const int t1 = (d + 1) % 3, t2 = (d + 2) % 3;
  const int64_t npt = (int64_t)n[t1] * n[t2];
  const int64_t total = 2 * WCNS_GHOST * npt;
  int gd[3] = {ni, nj, nk};
  gd[d] = WCNS_GHOST;
  const int64_t ocells = (int64_t)ni * nj * nk, gcells = (int64_t)gd[0] * gd[1] * gd[2];
  const double uinf[3] = {ux, uy, uz};
  for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < total; t += (int64_t)gridDim.x * blockDim.x) {
    const int64_t pt = t % npt;
    const int m = 1 + (int)((t / npt) % WCNS_GHOST);
    const int side = (int)(t / (npt * WCNS_GHOST));
    int c[3];
    c[t1] = (int)(pt % n[t1]);
    c[t2] = (int)(pt / n[t1]);
    auto own_at = [&](int along) {
      int x[3] = {c[0], c[1], c[2]};
      x[d] = along;
      return ((int64_t)x[2] * nj + x[1]) * ni + x[0];
    };
    auto ghost_at = [&](int along) {
      int x[3] = {c[0], c[1], c[2]};
      x[d] = along;
      return ((int64_t)x[2] * gd[1] + x[1]) * gd[0] + x[0];
    };
    // unit normal (+d) of the boundary face: the low ghost block's last face,
    // or the owner's last face
    const double* sb = side == 0 ? slo : sown;
    const int64_t fb = side == 0 ? ghost_at(WCNS_GHOST - 1) : own_at(n[d] - 1);
    const int64_t fc = side == 0 ? gcells : ocells;
    const double sx = sb[(3 * d) * fc + fb], sy = sb[(3 * d + 1) * fc + fb], sz = sb[(3 * d + 2) * fc + fb];
    const double nrm = sqrt(sx * sx + sy * sy + sz * sz);
    const double nx = sx / nrm, ny = sy / nrm, nz = sz / nrm;
    const int kind = side == 0 ? kind_lo : kind_hi;
    double qi[5], qg[5];
    if (kind == CFD_BC_FARFIELD) {
      const int64_t o0 = own_at(side == 0 ? 0 : n[d] - 1);
      for (int v = 0; v < 5; ++v) qi[v] = q[v * ocells + o0];
      const double sg = side == 0 ? -1.0 : 1.0;
      farfield_state(qi, sg * nx, sg * ny, sg * nz, gamma, uinf, qg);
    } else {
      const int64_t om = own_at(side == 0 ? m - 1 : n[d] - m);
      for (int v = 0; v < 5; ++v) qi[v] = q[v * ocells + om];
      qg[0] = qi[0];
      qg[4] = qi[4];
      if (kind == CFD_BC_SLIPWALL) {
        const double mn = qi[1] * nx + qi[2] * ny + qi[3] * nz;
        qg[1] = qi[1] - 2.0 * mn * nx;
        qg[2] = qi[2] - 2.0 * mn * ny;
        qg[3] = qi[3] - 2.0 * mn * nz;
      } else {
        qg[1] = -qi[1];
        qg[2] = -qi[2];
        qg[3] = -qi[3];
      }
    }
    double* qd = side == 0 ? qlo : qhi;
    const int64_t og = ghost_at(side == 0 ? WCNS_GHOST - m : m - 1);
    for (int v = 0; v < 5; ++v) qd[v * gcells + og] = qg[v];
  }
}

void fill_ghost_blocks_launch(const double* q, double* qlo, double* qhi, const double* slo, const double* sown,
                              const int32_t n[3], int d, const int32_t kind[2], double gamma, const double uinf[3],
                              hipStream_t stream) {
  const int64_t total = 2 * WCNS_GHOST * (int64_t)n[(d + 1) % 3] * n[(d + 2) % 3];
  hipLaunchKernelGGL(k_fill_ghost_blocks, dim3(grid_for(total)), dim3(256), 0, stream, q, qlo, qhi, slo, sown, n[0],
                     n[1], n[2], d, kind[0], kind[1], gamma, uinf[0], uinf[1], uinf[2]);
}

}  // namespace cfd

namespace {

// Checks a closure against the joined-block table: indices in range and
// distinct, the ghost blocks five cells across the bounded direction with the
// owner's transverse extents and joined to the owner's two faces, the kinds
// known, the far-field velocity finite.
void check_closure(int32_t nblk, const int32_t* dims, const int32_t* nbr, const cfd_wcns5_closure& c) {
  const int d = c.bounded;
  if (d < 0 || d > 2) cfd::host_fail(CFD_EINVAL, "closure: bounded must be 0, 1 or 2");
  const int32_t b[3] = {c.owner, c.ghost_lo, c.ghost_hi};
  for (int x = 0; x < 3; ++x)
    if (b[x] < 0 || b[x] >= nblk) cfd::host_fail(CFD_EINVAL, "closure: block index out of range");
  if (b[0] == b[1] || b[0] == b[2] || b[1] == b[2]) cfd::host_fail(CFD_EINVAL, "closure: blocks must be distinct");
  for (int x = 1; x < 3; ++x)
    for (int t = 0; t < 3; ++t) {
      const int want = t == d ? cfd::WCNS_GHOST : dims[3 * c.owner + t];
      if (dims[3 * b[x] + t] != want)
        cfd::host_fail(CFD_EINVAL, "closure: a ghost block must be 5 cells across the bounded direction, with the "
                                   "owner's transverse extents");
    }
  if (nbr[6 * c.owner + 2 * d] != c.ghost_lo || nbr[6 * c.owner + 2 * d + 1] != c.ghost_hi)
    cfd::host_fail(CFD_EINVAL, "closure: the ghost blocks must be joined to the owner's two bounded faces");
  for (int x = 0; x < 2; ++x)
    if (c.kind[x] != CFD_BC_FARFIELD && c.kind[x] != CFD_BC_SLIPWALL && c.kind[x] != CFD_BC_NOSLIP_ADIABATIC)
      cfd::host_fail(CFD_EINVAL, "closure: kind must be CFD_BC_FARFIELD, CFD_BC_SLIPWALL or CFD_BC_NOSLIP_ADIABATIC");
  for (int x = 0; x < 3; ++x)
    if (!std::isfinite(c.uinf[x])) cfd::host_fail(CFD_EINVAL, "closure: far-field velocity must be finite");
}

// RK3 steps on joined blocks (cfd_wcns5_ns_steps_blocks), with the ghost
// blocks of the nclosures closures refilled before every stage and the
// viscous terms only when `viscous`.
cfd_status ns_steps_blocks_impl(int32_t nblk, const int32_t* dims, const int32_t* nbr, double* const* q_dev,
                                const double* const* s_dev, const double* const* jinv_dev,
                                const cfd_wcns5_closure* closures, int32_t nclosures, bool viscous, void* work_dev,
                                size_t work_bytes,
                                double gamma, double entropy_fix, double eps, double prandtl, double mu_inf,
                                double s_star, double dt, int32_t nsteps, hipStream_t stream) {
  return cfd::host_guarded([&] {
    const size_t rscratch = check_seams(nblk, dims, nbr);
    if (!q_dev || !s_dev || !jinv_dev || !work_dev) cfd::host_fail(CFD_EINVAL, "NULL argument");
    if (!(gamma > 1.0) || !std::isfinite(gamma)) cfd::host_fail(CFD_EINVAL, "gamma must exceed 1");
    if (!(entropy_fix >= 0.0) || !std::isfinite(entropy_fix)) cfd::host_fail(CFD_EINVAL, "bad entropy_fix");
    if (!(eps > 0.0) || !std::isfinite(eps)) cfd::host_fail(CFD_EINVAL, "eps must be positive and finite");
    if (!(prandtl > 0.0) || !(mu_inf >= 0.0) || !(s_star > 0.0) || !std::isfinite(mu_inf))
      cfd::host_fail(CFD_EINVAL, "bad gas parameters");
    if (!(dt > 0.0) || !std::isfinite(dt)) cfd::host_fail(CFD_EINVAL, "dt must be positive and finite");
    if (nsteps < 0) cfd::host_fail(CFD_EINVAL, "nsteps must be >= 0");
    if (nclosures < 0 || (nclosures > 0 && !closures)) cfd::host_fail(CFD_EINVAL, "bad closure list");
    // ghost blocks: refilled from their owners before every stage, so their
    // own residual and update are never read (their states after a call are
    // scratch) and are skipped
    std::vector<char> ghost(nblk, 0);
    if (nclosures > 0) {
      // a block is the ghost block of at most one closure; an owner may be the
      // ghost block of an earlier closure (corner blocks filled from a face's
      // ghost block), never of a later one (it would be read before written)
      std::vector<char> owner(nblk, 0);
      for (int c = 0; c < nclosures; ++c) {
        const cfd_wcns5_closure& cl = closures[c];
        check_closure(nblk, dims, nbr, cl);
        owner[cl.owner] = 1;
        for (int32_t b : {cl.ghost_lo, cl.ghost_hi}) {
          if (ghost[b]) cfd::host_fail(CFD_EINVAL, "closure: a block is the ghost block of two closures");
          if (owner[b]) cfd::host_fail(CFD_EINVAL, "closure: a ghost block is the owner of an earlier closure");
          ghost[b] = 1;
        }
      }
    }
    std::vector<int64_t> off(nblk + 1, 0);
    size_t vscratch = 0;
    for (int b = 0; b < nblk; ++b) {
      off[b + 1] = off[b] + 10 * block_cells(dims, b);
      vscratch += (size_t)8 * cfd::VW_FIELDS * block_cells(dims, b);
    }
    const size_t scratch = std::max(rscratch, vscratch);
    const size_t need = scratch + (size_t)8 * off[nblk] + (size_t)8 * cfd::FM_FIELDS * (off[nblk] / 10);
    if (work_bytes < need) cfd::host_fail(CFD_ENOMEM, "workspace smaller than cfd_wcns5_ns_blocks_work_bytes()");
    std::vector<cfd::ArgSpan> spans{cfd::span(work_dev, (int64_t)need, true)};
    for (int b = 0; b < nblk; ++b) {
      if (!q_dev[b] || !s_dev[b] || !jinv_dev[b]) cfd::host_fail(CFD_EINVAL, "NULL block pointer");
      const int64_t cb = cfd::block_cells(dims, b);
      spans.insert(spans.end(), {cfd::span(q_dev[b], 40 * cb, true), cfd::span(s_dev[b], 72 * cb, false),
                                 cfd::span(jinv_dev[b], 8 * cb, false)});
    }
    cfd::check_spans(spans, "a state or the workspace overlaps the metrics, another state or the workspace");
    double* base = reinterpret_cast<double*>(static_cast<char*>(work_dev) + scratch);
    std::vector<double*> qn(nblk), R(nblk);
    for (int b = 0; b < nblk; ++b) {
      qn[b] = base + off[b];
      R[b] = qn[b] + 5 * block_cells(dims, b);
    }
    const cfd::Gas<double> vgas = cfd::viscous_gas(gamma, prandtl, mu_inf, s_star);
    const double a[3] = {0.0, 0.75, 1.0 / 3.0}, bb[3] = {1.0, 0.25, 2.0 / 3.0};
    double* FM = base + off[nblk];      // the viscous face metrics, once per call
    if (viscous && nsteps > 0)
      cfd::c4_face_metrics_blocks(nblk, dims, nbr, s_dev, jinv_dev, static_cast<double*>(work_dev), FM, stream);
    for (int it = 0; it < nsteps; ++it)
      for (int st = 0; st < 3; ++st) {
        for (int c = 0; c < nclosures; ++c) {
          const cfd_wcns5_closure& cl = closures[c];
          cfd::fill_ghost_blocks_launch(q_dev[cl.owner], q_dev[cl.ghost_lo], q_dev[cl.ghost_hi], s_dev[cl.ghost_lo],
                                        s_dev[cl.owner], dims + 3 * cl.owner, cl.bounded, cl.kind, gamma, cl.uinf,
                                        stream);
        }
        cfd::wcns5_blocks_residual_launch(nblk, dims, nbr, q_dev, s_dev, jinv_dev, R.data(), work_dev, gamma,
                                          entropy_fix, eps, stream, ghost.data());
        // the last viscous pass of a large block applies the stage (K[b].q set)
        std::vector<cfd::RkArgs> K(nblk);
        for (int b = 0; b < nblk; ++b)
          if (viscous && cfd::rk_fused(dims + 3 * b))
            K[b] = cfd::RkArgs{q_dev[b], qn[b], dt, a[st], bb[st], st == 0 ? 1 : 0};
        if (viscous)
          cfd::c4_viscous_blocks_launch(nblk, dims, nbr, q_dev, s_dev, jinv_dev, R.data(),
                                        static_cast<double*>(work_dev), FM, vgas, stream, ghost.data(), K.data());
        for (int b = 0; b < nblk; ++b) {
          if (ghost[b] || K[b].q) continue;
          const int64_t nv = 5 * block_cells(dims, b);
          hipLaunchKernelGGL(cfd::k_rk3_stage, dim3(cfd::grid_for(nv)), dim3(256), 0, stream, q_dev[b], qn[b], R[b],
                             nv, dt, a[st], bb[st], st == 0 ? 1 : 0);
        }
      }
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) cfd::host_fail(CFD_EHIP, std::string("kernel launch failed: ") + hipGetErrorString(e));
  });
}

}  // namespace

extern "C" cfd_status cfd_wcns5_ns_steps_blocks(int32_t nblk, const int32_t* dims, const int32_t* nbr,
                                                double* const* q_dev, const double* const* s_dev,
                                                const double* const* jinv_dev, void* work_dev, size_t work_bytes,
                                                double gamma, double entropy_fix, double eps, double prandtl,
                                                double mu_inf, double s_star, double dt, int32_t nsteps,
                                                hipStream_t stream) {
  return ns_steps_blocks_impl(nblk, dims, nbr, q_dev, s_dev, jinv_dev, nullptr, 0, true, work_dev, work_bytes, gamma,
                              entropy_fix, eps, prandtl, mu_inf, s_star, dt, nsteps, stream);
}

extern "C" cfd_status cfd_wcns5_steps_blocks_closed(int32_t nblk, const int32_t* dims, const int32_t* nbr,
                                                    double* const* q_dev, const double* const* s_dev,
                                                    const double* const* jinv_dev,
                                                    const cfd_wcns5_closure* closures, int32_t nclosures,
                                                    int32_t viscous, void* work_dev, size_t work_bytes, double gamma,
                                                    double entropy_fix, double eps, double prandtl, double mu_inf,
                                                    double s_star, double dt, int32_t nsteps, hipStream_t stream) {
  if (!closures || nclosures < 1)
    return cfd::host_guarded([] { cfd::host_fail(CFD_EINVAL, "at least one closure is needed"); });
  return ns_steps_blocks_impl(nblk, dims, nbr, q_dev, s_dev, jinv_dev, closures, nclosures, viscous != 0, work_dev,
                              work_bytes, gamma, entropy_fix, eps, prandtl, mu_inf, s_star, dt, nsteps, stream);
}

extern "C" cfd_status cfd_wcns5_extend_vertices_mask(const double* xv_dev, const int32_t n[3], int32_t bounded_mask,
                                                     const double period[9], double* xe_dev, hipStream_t stream) {
  return cfd::host_guarded([&] {
    if (!xv_dev || !n || !period || !xe_dev) cfd::host_fail(CFD_EINVAL, "NULL argument");
    if (bounded_mask < 0 || bounded_mask > 7 || bounded_mask == 7)
      cfd::host_fail(CFD_EINVAL, "bounded_mask must name at most two directions");
    if (n[0] < 1 || n[1] < 1 || n[2] < 1) cfd::host_fail(CFD_EINVAL, "every extent must be >= 1");
    for (int x = 0; x < 9; ++x)
      if (!std::isfinite(period[x])) cfd::host_fail(CFD_EINVAL, "period must be finite");
    int64_t e[3], sv = 1, ev = 1;
    for (int d = 0; d < 3; ++d) {
      const bool b = (bounded_mask >> d) & 1;
      e[d] = b ? n[d] + 1 + 2 * CFD_WCNS5_XLAYERS : n[d] + 5;
      sv *= n[d] + (b ? 1 : 0);
      ev *= e[d];
    }
    if (ev > ((int64_t)1 << 34)) cfd::host_fail(CFD_EINVAL, "block too large");
    if (!cfd::apart(xv_dev, 24 * sv, xe_dev, 24 * ev)) cfd::host_fail(CFD_EINVAL, "input and output overlap");
    cfd::Period9 P;
    for (int x = 0; x < 9; ++x) P.p[x] = period[x];
    hipLaunchKernelGGL(cfd::k_extend_vertices, dim3(cfd::grid_for(ev)), dim3(256), 0, stream, xv_dev, n[0], n[1], n[2],
                       (int)bounded_mask, P, xe_dev, (int)e[0], (int)e[1], (int)e[2]);
    const hipError_t err = hipGetLastError();
    if (err != hipSuccess) cfd::host_fail(CFD_EHIP, std::string("kernel launch failed: ") + hipGetErrorString(err));
  });
}

extern "C" cfd_status cfd_wcns5_extend_vertices(const double* xv_dev, const int32_t n[3], int32_t bounded,
                                                const double period[9], double* xe_dev, hipStream_t stream) {
  if (bounded < -1 || bounded > 2)
    return cfd::host_guarded([] { cfd::host_fail(CFD_EINVAL, "bounded must be -1, 0, 1 or 2"); });
  return cfd_wcns5_extend_vertices_mask(xv_dev, n, bounded < 0 ? 0 : 1 << bounded, period, xe_dev, stream);
}

extern "C" cfd_status cfd_wcns5_fill_ghost_blocks(const double* q_dev, double* q_lo_dev, double* q_hi_dev,
                                                  const double* s_dev, const double* s_lo_dev, const int32_t n[3],
                                                  int32_t bounded, const int32_t kind[2], double gamma,
                                                  const double uinf[3], hipStream_t stream) {
  return cfd::host_guarded([&] {
    if (!q_dev || !q_lo_dev || !q_hi_dev || !s_dev || !s_lo_dev || !n || !kind || !uinf)
      cfd::host_fail(CFD_EINVAL, "NULL argument");
    if (bounded < 0 || bounded > 2) cfd::host_fail(CFD_EINVAL, "bounded must be 0, 1 or 2");
    if (n[0] < 1 || n[1] < 1 || n[2] < 1) cfd::host_fail(CFD_EINVAL, "every extent must be >= 1");
    if (!(gamma > 1.0) || !std::isfinite(gamma)) cfd::host_fail(CFD_EINVAL, "gamma must exceed 1");
    for (int x = 0; x < 2; ++x)
      if (kind[x] != CFD_BC_FARFIELD && kind[x] != CFD_BC_SLIPWALL && kind[x] != CFD_BC_NOSLIP_ADIABATIC)
        cfd::host_fail(CFD_EINVAL, "kind must be CFD_BC_FARFIELD, CFD_BC_SLIPWALL or CFD_BC_NOSLIP_ADIABATIC");
    for (int x = 0; x < 3; ++x)
      if (!std::isfinite(uinf[x])) cfd::host_fail(CFD_EINVAL, "uinf must be finite");
    const int64_t oc = (int64_t)n[0] * n[1] * n[2];
    if (oc > ((int64_t)1 << 34)) cfd::host_fail(CFD_EINVAL, "block too large");
    const int64_t gc = oc / n[bounded] * cfd::WCNS_GHOST;
    std::vector<cfd::ArgSpan> spans{cfd::span(q_dev, 40 * oc, false), cfd::span(s_dev, 72 * oc, false),
                                    cfd::span(s_lo_dev, 72 * gc, false), cfd::span(q_lo_dev, 40 * gc, true),
                                    cfd::span(q_hi_dev, 40 * gc, true)};
    cfd::check_spans(spans, "a ghost state overlaps the owner's state, a metric array or the other ghost state");
    cfd::fill_ghost_blocks_launch(q_dev, q_lo_dev, q_hi_dev, s_lo_dev, s_dev, n, bounded, kind, gamma, uinf, stream);
    const hipError_t err = hipGetLastError();
    if (err != hipSuccess) cfd::host_fail(CFD_EHIP, std::string("kernel launch failed: ") + hipGetErrorString(err));
  });
}
