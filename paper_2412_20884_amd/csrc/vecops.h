// Column-blocked streaming helpers shared by the iterative solvers (multi-shift CG, PCG):
// an n x r row-major block is swept with thread t on column t % r, rows t / r + k * rps
// (rps = 256 / r rows per sweep), a workgroup covering `rows_per_block` consecutive rows; per
// column sums go through fixed-order workgroup records, so every reduction is deterministic.
#pragma once

#include "common.h"

namespace gpk {

constexpr int kVecBlocksMax = 2048;

// Row tiling of the streaming kernels: thread t handles column t % r of rows t / r, t / r + rps,
// ... with rps = 256 / r rows per sweep; a block covers `rows_per_block` consecutive rows.
struct VecGrid {
  int rps;
  int64_t rows_per_block;
  int64_t blocks;
};

inline VecGrid vec_grid(int64_t n, int r) {
  VecGrid g;
  g.rps = kThreads / r;
  int64_t blocks = (n + g.rps - 1) / g.rps;
  if (blocks > kVecBlocksMax) blocks = kVecBlocksMax;
  int64_t rpb = (n + blocks - 1) / blocks;
  rpb = ((rpb + g.rps - 1) / g.rps) * g.rps;
  g.rows_per_block = rpb;
  g.blocks = (n + rpb - 1) / rpb;
  return g;
}

// Fixed-order per-column sum of the block's thread partials into part[blockIdx.x * r + c].
__device__ inline void block_column_sum(double v, double *sh, int r, int rps, double *part) {
  const int t = threadIdx.x;
  sh[t] = v;
  __syncthreads();
  if (t < r) {
    double s = 0.0;
    for (int l = 0; l < rps; ++l) s += sh[l * r + t];
    part[(int64_t)blockIdx.x * r + t] = s;
  }
}

// Fixed-order sum of part[b * r + c] over the blocks, by all threads of the (single) block.
// Totals of every column c < r (r <= blockDim.x) of part[blocks][r] into tot[c] (LDS): G groups
// of r threads each sum every G-th block, then a pairwise tree over the groups; the order
// depends on blocks and r only.  red: blockDim.x doubles of LDS.
__device__ inline void column_totals(const double *part, int64_t blocks, int r, double *red,
                                     double *tot) {
  const int t = threadIdx.x;
  int G = 1;
  while (2 * G * r <= (int)blockDim.x) G *= 2;
  const int g = t / r, c = t - g * r;
  double s = 0.0;
  if (g < G)
    for (int64_t b = g; b < blocks; b += G) s += part[b * r + c];
  red[t] = s;
  __syncthreads();
  for (int h = G / 2; h > 0; h /= 2) {
    if (g < h) red[t] += red[t + h * r];
    __syncthreads();
  }
  if (t < r) tot[t] = red[t];
  __syncthreads();
}

__device__ inline double column_total(const double *part, int64_t blocks, int r, int c, double *red) {
  const int t = threadIdx.x;
  double s = 0.0;
  for (int64_t b = t; b < blocks; b += blockDim.x) s += part[b * r + c];
  red[t] = s;
  __syncthreads();
  for (int w = blockDim.x / 2; w >= 1; w >>= 1) {
    if (t < w) red[t] += red[t + w];
    __syncthreads();
  }
  const double tot = red[0];
  __syncthreads();
  return tot;
}

}  // namespace gpk
