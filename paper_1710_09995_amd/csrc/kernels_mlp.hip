// Learned warm start: a small MLP (features -> SiLU hidden layers -> linear
// output) evaluated with BF16 MFMA (FP32 accumulate), trained with FP32
// backward kernels and Adam, plus the conversions between the solver's
// state arena and the network's features / targets / outputs.
//
// Parameter layout (padded, shared by the BF16 copy, the FP32 master copy,
// Adam moments and gradients): for layer l = 0 .. n_hidden, W_l as [N_l][K_l]
// (output-major) followed by b_l [N_l], with K_0 = 16 (inputs zero-padded),
// K_l = N_l = d_hidden for hidden-to-hidden layers and N_out = 16 (outputs
// zero-padded).  Padded weights start at zero and receive zero gradients, so
// they stay zero.
#include <hip/hip_runtime.h>
#include <stdint.h>
#include "cfd_internal.hpp"

namespace cfd {

typedef short short4_t __attribute__((ext_vector_type(4)));
typedef float float4_t __attribute__((ext_vector_type(4)));

__device__ __forceinline__ uint16_t f2bf(float f) {   // round to nearest even
  uint32_t u = __float_as_uint(f);
  u += 0x7FFFu + ((u >> 16) & 1u);
  return (uint16_t)(u >> 16);
}
__device__ __forceinline__ float bf2f(uint16_t h) { return __uint_as_float(((uint32_t)h) << 16); }
__device__ __forceinline__ float silu_f(float z) { return z / (1.0f + __expf(-z)); }
__device__ __forceinline__ float silu_grad_f(float z) {
  const float s = 1.0f / (1.0f + __expf(-z));
  return s * (1.0f + z * (1.0f - s));
}

// ------------------------------------------------------------------ forward
// One wave evaluates 16 points; a workgroup holds 4 waves.  Activations of
// the 16 points live in LDS as BF16 [16][128] (ping-pong per wave).  Each
// 16x16 output tile accumulates K/16 MFMA steps:
//   A (16 points x 16 k):  lane l holds rows l%16, k = 4 (l/16) .. +3
//   B (16 k x 16 outputs): lane l holds column l%16, k = 4 (l/16) .. +3
//   D (16 points x 16 outputs): lane l holds rows 4 (l/16) .. +3, column l%16
constexpr int MLP_WAVES = 4;
constexpr int MLP_ACT_W = 128;   // d_hidden for the LDS activation tiles

__global__ void __launch_bounds__(64 * MLP_WAVES) k_mlp_forward(MlpDims D, const uint16_t* __restrict__ P,
                                                                 const float* __restrict__ x,
                                                                 const int32_t* __restrict__ idx, int64_t n,
                                                                 float* __restrict__ y, float* __restrict__ cache) {
  __shared__ __attribute__((aligned(16))) uint16_t act[MLP_WAVES][2][16][MLP_ACT_W];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int64_t p0 = ((int64_t)blockIdx.x * MLP_WAVES + wave) * 16;
  if (p0 >= n) return;   // whole wave inactive (no block-level sync below)
  const int r16 = lane & 15, kq = (lane >> 4) * 4;
  // input layer activations (zero padded to K_0 = 16)
  for (int e = lane; e < 16 * MLP_KIN; e += 64) {
    const int pr = e / MLP_KIN, k = e % MLP_KIN;
    const int64_t p = p0 + pr;
    float v = 0.f;
    if (p < n && k < D.d_in) {
      const int64_t src = idx ? (int64_t)idx[p] : p;
      v = x[src * D.d_in + k];
    }
    const uint16_t hb = f2bf(v);
    act[wave][0][pr][k] = hb;
    if (cache && p < n) cache[p * D.cache_per_point + D.hoff[0] + k] = bf2f(hb);
  }
  __builtin_amdgcn_wave_barrier();
  int cur = 0;
  for (int l = 0; l < D.nlayer; ++l) {
    const int K = D.K[l], N = D.N[l];
    const bool last = l == D.nlayer - 1;
    const uint16_t* W = P + D.woff[l];
    const uint16_t* B = P + D.boff[l];
    for (int nt = 0; nt < N / 16; ++nt) {
      float4_t acc = {0.f, 0.f, 0.f, 0.f};
      const int col = nt * 16 + r16;
      for (int ks = 0; ks < K / 16; ++ks) {
        const int k0 = ks * 16 + kq;
        short4_t a, b;
        const uint16_t* ap = &act[wave][cur][r16][k0];
        const uint16_t* bp = W + (int64_t)col * K + k0;
        a[0] = (short)ap[0]; a[1] = (short)ap[1]; a[2] = (short)ap[2]; a[3] = (short)ap[3];
        b[0] = (short)bp[0]; b[1] = (short)bp[1]; b[2] = (short)bp[2]; b[3] = (short)bp[3];
        acc = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a, b, acc, 0, 0, 0);
      }
      const float bias = bf2f(B[col]);
      for (int r = 0; r < 4; ++r) {
        const int row = kq + r;
        const int64_t p = p0 + row;
        const float z = acc[r] + bias;
        if (last) {
          if (p < n && col < D.d_out) y[p * D.d_out + col] = z;
          if (cache && p < n) cache[p * D.cache_per_point + D.zoff[l] + col] = z;
        } else {
          const uint16_t hb = f2bf(silu_f(z));
          act[wave][cur ^ 1][row][col] = hb;
          if (cache && p < n) {
            cache[p * D.cache_per_point + D.zoff[l] + col] = z;
            cache[p * D.cache_per_point + D.hoff[l + 1] + col] = bf2f(hb);
          }
        }
      }
    }
    __builtin_amdgcn_wave_barrier();
    cur ^= 1;
  }
}

// ------------------------------------------------------------------ loss
// dy = 2 (y - t) / (n d_out) on the d_out outputs; per-workgroup loss
// partials (fixed-order tree) for a deterministic mean squared error.
__global__ void __launch_bounds__(256) k_mlp_mse(const float* __restrict__ y, const float* __restrict__ t,
                                                 const int32_t* __restrict__ idx, int64_t n, int d_out,
                                                 float* __restrict__ dy, double* __restrict__ partials) {
  __shared__ double red[256];
  double acc = 0.0;
  const int64_t total = n * d_out;
  const float scale = 2.0f / (float)total;
  for (int64_t e = blockIdx.x * 256 + threadIdx.x; e < total; e += (int64_t)gridDim.x * 256) {
    const int64_t p = e / d_out;
    const int o = (int)(e - p * d_out);
    const int64_t src = idx ? (int64_t)idx[p] : p;
    const float d = y[e] - t[src * d_out + o];
    dy[e] = scale * d;
    acc += (double)d * (double)d;
  }
  red[threadIdx.x] = acc;
  __syncthreads();
  for (int s = 128; s > 0; s >>= 1) {
    if (threadIdx.x < s) red[threadIdx.x] += red[threadIdx.x + s];
    __syncthreads();
  }
  if (threadIdx.x == 0) partials[blockIdx.x] = red[0];
}

__global__ void k_mlp_mse_final(const double* __restrict__ partials, int nrows, int64_t count,
                                double* __restrict__ loss) {
  if (threadIdx.x == 0 && blockIdx.x == 0) {
    double s = 0.0;
    for (int r = 0; r < nrows; ++r) s += partials[r];
    loss[0] = s / (double)count;
  }
}

// ------------------------------------------------------------------ backward
// dZ of the output layer: the loss gradient, zero padded to N_out.
__global__ void k_mlp_dz_out(const float* __restrict__ dy, int64_t n, int d_out, int N, float* __restrict__ dz) {
  const int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (e >= n * N) return;
  const int64_t p = e / N;
  const int o = (int)(e - p * N);
  dz[e] = o < d_out ? dy[p * d_out + o] : 0.f;
}

// dZ_l = dA_l * silu'(z_l) for a hidden layer.
__global__ void k_mlp_dz_hidden(const float* __restrict__ da, const float* __restrict__ cache, int64_t cpp,
                                int64_t zoff, int64_t n, int N, float* __restrict__ dz) {
  const int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (e >= n * N) return;
  const int64_t p = e / N;
  const int c = (int)(e - p * N);
  dz[e] = da[e] * silu_grad_f(cache[p * cpp + zoff + c]);
}

// Partial weight/bias gradients over point chunk ch: grid (N*K+N threads, chunks).
__global__ void k_mlp_dw_partial(const float* __restrict__ dz, const float* __restrict__ cache, int64_t cpp,
                                 int64_t hoff, int64_t n, int N, int K, int64_t chunk,
                                 float* __restrict__ part) {
  const int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  const int64_t nw = (int64_t)N * K + N;
  if (e >= nw) return;
  const int64_t pa = blockIdx.y * chunk, pb = min(n, pa + chunk);
  float s = 0.f;
  if (e < (int64_t)N * K) {
    const int o = (int)(e / K), k = (int)(e - (int64_t)o * K);
    for (int64_t p = pa; p < pb; ++p) s += dz[p * N + o] * cache[p * cpp + hoff + k];
  } else {
    const int o = (int)(e - (int64_t)N * K);
    for (int64_t p = pa; p < pb; ++p) s += dz[p * N + o];
  }
  part[blockIdx.y * nw + e] = s;
}

// Sum the chunk partials in order into the gradient slots of layer l.
__global__ void k_mlp_dw_reduce(const float* __restrict__ part, int nchunk, int N, int K, int64_t woff,
                                int64_t boff, float* __restrict__ grad) {
  const int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  const int64_t nw = (int64_t)N * K + N;
  if (e >= nw) return;
  float s = 0.f;
  for (int c = 0; c < nchunk; ++c) s += part[c * nw + e];
  if (e < (int64_t)N * K) grad[woff + e] = s;
  else grad[boff + (e - (int64_t)N * K)] = s;
}

// dA_{l} (gradient w.r.t. layer l's input) = dZ_l W_l (weights from the BF16 copy).
__global__ void k_mlp_da(const float* __restrict__ dz, const uint16_t* __restrict__ P, int64_t woff, int64_t n,
                         int N, int K, float* __restrict__ da) {
  const int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (e >= n * K) return;
  const int64_t p = e / K;
  const int k = (int)(e - p * K);
  float s = 0.f;
  for (int o = 0; o < N; ++o) s += dz[p * N + o] * bf2f(P[woff + (int64_t)o * K + k]);
  da[e] = s;
}

// ------------------------------------------------------------------ Adam
__global__ void k_mlp_adam(int64_t np, float* __restrict__ master, float* __restrict__ m, float* __restrict__ v,
                           const float* __restrict__ g, uint16_t* __restrict__ pbf, float lr, float b1, float b2,
                           float eps, float c1, float c2) {
  const int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (e >= np) return;
  const float ge = g[e];
  const float me = b1 * m[e] + (1.f - b1) * ge;
  const float ve = b2 * v[e] + (1.f - b2) * ge * ge;
  m[e] = me;
  v[e] = ve;
  const float th = master[e] - lr * (me / c1) / (sqrtf(ve / c2) + eps);
  master[e] = th;
  pbf[e] = f2bf(th);
}

__global__ void k_mlp_to_bf16(int64_t np, const float* __restrict__ master, uint16_t* __restrict__ pbf) {
  const int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (e < np) pbf[e] = f2bf(master[e]);
}

// ------------------------------------------------------------ state <-> features
// Interior cells of all blocks in order (block, k, j, i); thread per cell.
// Features: [(M - 0.675)/0.175, (h - 0.06)/0.04, 2 xi - 1, 2 eta - 1, 2 zeta - 1].
__device__ __forceinline__ int find_block(const CellMap& M, int64_t e) {
  int lo = 0, hi = M.nblk - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (M.cell_start[mid] <= e) lo = mid;
    else hi = mid - 1;
  }
  return lo;
}

__global__ void k_mlp_features(CellMap M, int64_t ncells, const double* __restrict__ cond, float* __restrict__ x) {
  const int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (e >= ncells) return;
  const int b = find_block(M, e);
  const BlockDesc B = M.blocks[b];
  const int64_t r = e - M.cell_start[b];
  const int ni = B.n[0], nj = B.n[1], nk = B.n[2];
  const int i = (int)(r % ni), j = (int)((r / ni) % nj), k = (int)(r / ((int64_t)ni * nj));
  float* o = x + e * 5;
  o[0] = (float)((cond[2 * b] - 0.675) / 0.175);
  o[1] = (float)((cond[2 * b + 1] - 0.06) / 0.04);
  o[2] = (float)(2.0 * (i + 0.5) / ni - 1.0);
  o[3] = (float)(2.0 * (j + 0.5) / nj - 1.0);
  o[4] = (float)(2.0 * (k + 0.5) / nk - 1.0);
}

// Targets: primitive deviations from each block's inflow stream.
__global__ void k_mlp_targets(CellMap M, int64_t ncells, const double* __restrict__ q,
                              const double* __restrict__ cond, double gamma, float* __restrict__ t) {
  const int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (e >= ncells) return;
  const int b = find_block(M, e);
  const BlockDesc B = M.blocks[b];
  const int64_t r = e - M.cell_start[b];
  const int ni = B.n[0], nj = B.n[1];
  const int i = (int)(r % ni), j = (int)((r / ni) % nj), k = (int)(r / ((int64_t)ni * nj));
  const int64_t c = B.qoff + (int64_t)(k + NG) * B.sk + (int64_t)(j + NG) * B.sj + (i + NG);
  const double rho = q[c], inv = 1.0 / rho;
  const double u = q[B.sv + c] * inv, v = q[2 * B.sv + c] * inv, w = q[3 * B.sv + c] * inv;
  const double p = (gamma - 1.0) * (q[4 * B.sv + c] - 0.5 * rho * (u * u + v * v + w * w));
  float* o = t + e * 5;
  o[0] = (float)(rho - 1.0);
  o[1] = (float)(u - cond[2 * b] * sqrt(gamma));
  o[2] = (float)v;
  o[3] = (float)w;
  o[4] = (float)(p - 1.0);
}

// Network outputs -> conserved state of the interior cells (FP64).
__global__ void k_mlp_to_state(CellMap M, int64_t ncells, const float* __restrict__ yv,
                               const double* __restrict__ cond, double gamma, double* __restrict__ q) {
  const int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (e >= ncells) return;
  const int b = find_block(M, e);
  const BlockDesc B = M.blocks[b];
  const int64_t r = e - M.cell_start[b];
  const int ni = B.n[0], nj = B.n[1];
  const int i = (int)(r % ni), j = (int)((r / ni) % nj), k = (int)(r / ((int64_t)ni * nj));
  const int64_t c = B.qoff + (int64_t)(k + NG) * B.sk + (int64_t)(j + NG) * B.sj + (i + NG);
  const float* o = yv + e * 5;
  const double rho = 1.0 + (double)o[0];
  const double u = cond[2 * b] * sqrt(gamma) + (double)o[1];
  const double v = (double)o[2], w = (double)o[3];
  const double p = 1.0 + (double)o[4];
  q[c] = rho;
  q[B.sv + c] = rho * u;
  q[2 * B.sv + c] = rho * v;
  q[3 * B.sv + c] = rho * w;
  q[4 * B.sv + c] = p / (gamma - 1.0) + 0.5 * rho * (u * u + v * v + w * w);
}

// ------------------------------------------------------------------ launchers

static unsigned blocks_for(int64_t n, int t) { return (unsigned)((n + t - 1) / t); }

void mlp_forward(const MlpDims& D, const uint16_t* P, const float* x, const int32_t* idx, int64_t n, float* y,
                 float* cache, hipStream_t s) {
  const int64_t waves = (n + 15) / 16;
  hipLaunchKernelGGL(k_mlp_forward, dim3(blocks_for(waves, MLP_WAVES)), dim3(64 * MLP_WAVES), 0, s, D, P, x, idx,
                     n, y, cache);
}

int mlp_mse(const float* y, const float* t, const int32_t* idx, int64_t n, int d_out, float* dy, double* partials,
            int max_rows, double* loss, hipStream_t s) {
  int nb = (int)std::min<int64_t>(max_rows, std::max<int64_t>(1, (n * d_out + 255) / 256));
  hipLaunchKernelGGL(k_mlp_mse, dim3(nb), dim3(256), 0, s, y, t, idx, n, d_out, dy, partials);
  hipLaunchKernelGGL(k_mlp_mse_final, dim3(1), dim3(64), 0, s, partials, nb, n * d_out, loss);
  return nb;
}

void mlp_backward(const MlpDims& D, const uint16_t* P, const float* cache, const float* dy, int64_t n, float* grad,
                  float* dz, float* da, float* part, int nchunk, hipStream_t s) {
  const int64_t chunk = (n + nchunk - 1) / nchunk;
  for (int l = D.nlayer - 1; l >= 0; --l) {
    const int N = D.N[l], K = D.K[l];
    if (l == D.nlayer - 1)
      hipLaunchKernelGGL(k_mlp_dz_out, dim3(blocks_for(n * N, 256)), dim3(256), 0, s, dy, n, D.d_out, N, dz);
    else
      hipLaunchKernelGGL(k_mlp_dz_hidden, dim3(blocks_for(n * N, 256)), dim3(256), 0, s, da, cache,
                         D.cache_per_point, D.zoff[l], n, N, dz);
    const int64_t nw = (int64_t)N * K + N;
    hipLaunchKernelGGL(k_mlp_dw_partial, dim3(blocks_for(nw, 256), nchunk), dim3(256), 0, s, dz, cache,
                       D.cache_per_point, D.hoff[l], n, N, K, chunk, part);
    hipLaunchKernelGGL(k_mlp_dw_reduce, dim3(blocks_for(nw, 256)), dim3(256), 0, s, part, nchunk, N, K, D.woff[l],
                       D.boff[l], grad);
    if (l > 0)
      hipLaunchKernelGGL(k_mlp_da, dim3(blocks_for(n * K, 256)), dim3(256), 0, s, dz, P, D.woff[l], n, N, K, da);
  }
}

void mlp_adam(int64_t np, float* master, float* m, float* v, const float* g, uint16_t* pbf, float lr, float b1,
              float b2, float eps, int t, hipStream_t s) {
  const float c1 = 1.f - powf(b1, (float)t), c2 = 1.f - powf(b2, (float)t);
  hipLaunchKernelGGL(k_mlp_adam, dim3(blocks_for(np, 256)), dim3(256), 0, s, np, master, m, v, g, pbf, lr, b1, b2,
                     eps, c1, c2);
}

void mlp_to_bf16(int64_t np, const float* master, uint16_t* pbf, hipStream_t s) {
  hipLaunchKernelGGL(k_mlp_to_bf16, dim3(blocks_for(np, 256)), dim3(256), 0, s, np, master, pbf);
}

void mlp_features(const CellMap& M, int64_t ncells, const double* cond, float* x, hipStream_t s) {
  hipLaunchKernelGGL(k_mlp_features, dim3(blocks_for(ncells, 256)), dim3(256), 0, s, M, ncells, cond, x);
}

void mlp_targets(const CellMap& M, int64_t ncells, const double* q, const double* cond, double gamma, float* t,
                 hipStream_t s) {
  hipLaunchKernelGGL(k_mlp_targets, dim3(blocks_for(ncells, 256)), dim3(256), 0, s, M, ncells, q, cond, gamma, t);
}

void mlp_to_state(const CellMap& M, int64_t ncells, const float* y, const double* cond, double gamma, double* q,
                  hipStream_t s) {
  hipLaunchKernelGGL(k_mlp_to_state, dim3(blocks_for(ncells, 256)), dim3(256), 0, s, M, ncells, y, cond, gamma, q);
}

}  // namespace cfd
