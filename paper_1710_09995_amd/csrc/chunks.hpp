// Row chunks of the grid and their cut into contiguous runs per wave (the
// time-step, norms and implicit kernels).
#pragma once
#include <hip/hip_runtime.h>
#include "cfd_internal.hpp"

namespace cfd {

// ------------------------------------------------- row-per-wave reductions
// The time-step and norms kernels give every wave a contiguous run of the
// grid's 64-cell row chunks (below).  With a grid that is a multiple of 8,
// workgroup b runs on XCD b % 8 and the runs of one XCD's workgroups are
// adjacent, so a row's j+1 and k+1 neighbours are mostly read through the
// same L2.
__device__ __forceinline__ void wave_rows(int64_t nrows, int64_t& r0, int64_t& r1) {
  const int wpb = blockDim.x >> 6;
  const int nb = gridDim.x, b = blockIdx.x;
  const int slot = (nb & 7) == 0 ? (b & 7) * (nb >> 3) + (b >> 3) : b;
  const int64_t w = __builtin_amdgcn_readfirstlane((int)slot * wpb + (int)(threadIdx.x >> 6));
  const int64_t nw = (int64_t)nb * wpb;
  r0 = nrows * w / nw;
  r1 = nrows * (w + 1) / nw;
}

// The grid's row chunks, numbered block by block and, within a block, i
// chunk fastest, then j, then k: chunk u of block b (coff[b] <= u < coff[b+1])
// covers cells i = 64 ic .. 64 ic + 63 of row (j, k).  The time-step and norms
// kernels cut this numbering alone into contiguous runs per wave, with a grid
// that depends on the chunk count only, so their per-workgroup partials (and
// the fixed-order sums of them) do not depend on the stage kernels' tiles.
__device__ __forceinline__ int block_of_chunk(const BlockDesc* __restrict__ blocks, int nblk, int64_t u) {
  int lo = 0, hi = nblk - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (blocks[mid].coff <= u) lo = mid;
    else hi = mid - 1;
  }
  return lo;
}

struct ChunkWalk {
  const BlockDesc* blocks;
  int nblk, b;
  BlockDesc B;
  __device__ void start(const BlockDesc* bl, int nb, int64_t u) {
    blocks = bl;
    nblk = nb;
    b = block_of_chunk(bl, nb, u);
    B = bl[b];
  }
  // cell (i, j, k) of this lane in chunk u (u ascending over calls); false past the row's end
  __device__ bool cell(int64_t u, int lane, int& i, int& j, int& k) {
    while (b + 1 < nblk && u >= blocks[b + 1].coff) B = blocks[++b];
    const int nci = (B.n[0] + 63) >> 6;
    const int64_t v = u - B.coff;
    const int64_t row = v / nci;
    i = (int)(v - row * nci) * 64 + lane;
    j = (int)(row % B.n[1]);
    k = (int)(row / B.n[1]);
    return i < B.n[0];
  }
};

}  // namespace cfd
