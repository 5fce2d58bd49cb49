// Shared device/host definitions of libgpk.
//
// Coordinate pre-scaling (stage step of every product): with s_k = sqrt(log2(e)/2) / l_k and
// x~_ik = (x_ik - c_k) s_k for any fixed centre c,
//     K_ij = alpha exp(-1/2 sum_k (x_ik - x_jk)^2 / l_k^2) = exp2(log2(alpha) - rho_ij),
//     rho_ij = sum_k (x~_ik - x~_jk)^2,
// and the length-scale derivative factor (x_ik - x_jk)^2 / l_k^2 equals 2 ln(2) (x~_ik - x~_jk)^2.
// The centre (the coordinate mean) only reduces the magnitude of the rounded coordinates.
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

namespace gpk {

constexpr double kLog2e = 1.4426950408889634074;
constexpr double kLn2 = 0.69314718055994530942;
constexpr double kScale = 0.84932180028801904272;  // sqrt(log2(e) / 2)

constexpr int kThreads = 256;     // threads per block of the VALU kernels
constexpr int kMaxD = 64;         // largest supported spatial dimension
constexpr int kMaxRPass = 32;     // right-hand sides handled in one pass
constexpr int kCentreBlocks = 64; // blocks of the coordinate-mean reduction

// Padded coordinate width used by the kernels: d is zero-padded to one of these.
inline int padded_dim(int d) {
  if (d <= 4) return 4;
  if (d <= 8) return 8;
  if (d <= 16) return 16;
  if (d <= 32) return 32;
  return 64;
}

inline int pow2_at_least(int r) {
  int p = 1;
  while (p < r) p <<= 1;
  return p;
}

template <typename T>
__device__ __forceinline__ T gexp2(T t);
template <>
__device__ __forceinline__ float gexp2<float>(float t) {
  return __builtin_amdgcn_exp2f(t);
}
template <>
__device__ __forceinline__ double gexp2<double>(double t) {
  return exp2(t);
}

// Sum over the 64 lanes of a wavefront (fixed butterfly order, deterministic).
__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}

// Layout of one product call's workspace: all offsets are 256-byte aligned.
struct WsLayout {
  size_t centre_part;  // double [kCentreBlocks][kMaxD]
  size_t centre;       // double [kMaxD]
  size_t xs;           // T [n][dp] scaled, centred coordinates
  size_t outp;         // double [splits][n][rpass] split partial sums
  size_t rec_pair;     // double [pair blocks][nrec]
  size_t rec_fin;      // double [finalise blocks][nrec]
  size_t scratch;      // matrix-core pass scratch
  size_t total;
};

inline size_t align256(size_t x) { return (x + 255) & ~size_t(255); }

// Smallest column chunk of a split: below some 32k points the row blocks alone cannot fill
// 256 CUs, and 256 columns per block still amortise its row-side setup.
constexpr int64_t kMinSplitCols = 256;

// Column splits of the pair grid: enough blocks to fill 256 CUs several times over, with at
// least kMinSplitCols columns per split.
inline int choose_splits(int64_t n, int rows_per_block) {
  int64_t rb = (n + rows_per_block - 1) / rows_per_block;
  int64_t s = (4096 + rb - 1) / rb;
  int64_t max_s = n / kMinSplitCols;
  if (s > max_s) s = max_s;
  if (s > 64) s = 64;
  if (s < 1) s = 1;
  return (int)s;
}

inline WsLayout ws_layout(int64_t n, int dp, size_t tsize, int rpass, int splits,
                          int64_t pair_blocks, int64_t fin_blocks, int nrec,
                          size_t scratch_bytes) {
  WsLayout L;
  size_t o = 0;
  L.centre_part = o;
  o = align256(o + sizeof(double) * kCentreBlocks * kMaxD);
  L.centre = o;
  o = align256(o + sizeof(double) * kMaxD);
  L.xs = o;
  o = align256(o + tsize * (size_t)n * dp);
  L.outp = o;
  o = align256(o + (splits > 1 ? sizeof(double) * (size_t)splits * n * rpass : 0));
  L.rec_pair = o;
  o = align256(o + sizeof(double) * (size_t)pair_blocks * nrec);
  L.rec_fin = o;
  o = align256(o + sizeof(double) * (size_t)fin_blocks * nrec);
  L.scratch = o;
  o = align256(o + scratch_bytes);
  L.total = o;
  return L;
}

}  // namespace gpk
