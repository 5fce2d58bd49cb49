// Host-side description of one pair pass and the launchers of the product kernels.
#pragma once

#include "common.h"

namespace gpk {

enum Prec { kF64 = 0, kF32 = 1, kBF16X = 2 };

// One pass over all pairs (i, j) of a point set.  For every row i it forms
//   (A Y)_ic = sum_j K_ij Y_jc + (sigma^2 [unless no_noise] + shift_c) Y_ic
// and, when P is set, the gradient sums of sum_c w_c P_c^T A Q_c; when D is set, the
// per-column sums q_c = sum_i D_ic (A Y)_ic and, with P set, sigma^2 sum_c w_c P_c . Q_c.
// Per-block records (nrec = n_theta + R doubles) are written for the final reduction:
//   [0] sum K S, [1..L] sum K S rho_k (scaled), [L+1] sigma^2 term, [n_theta + c] q_c.
struct PassDesc {
  int prec;
  int kind;  // 0 iso, 1 ard
  int d, dp;
  int64_t n;
  int R;
  const void *xs;
  const double *theta;
  const void *Y;
  int64_t ldy;
  const void *P;
  int64_t ldp;
  const void *Q;
  int64_t ldq;
  const double *w;
  const void *D;
  int64_t ldd;
  const double *col_shift;
  int no_noise;
  void *out;
  int64_t ldo;
  int splits;
  double *outp;
  double *rec_pair;
  double *rec_fin;
  int nth;
  int nrec;
  int use_mfma;  // 1: matrix-core pair kernel (float, 8 <= R <= 32, d <= 16); 2: cross-term
                 //    kernel (GP_BF16X, d <= 64)
  void *mfma_scratch;  // scale exponents and partial maxima of the matrix-core pass
  int ib;              // matrix-core kernel: 16-row blocks per wave requested (1 or 2)
};

// Rows per block of the pair kernels (VALU and MFMA variants).  The matrix-core kernel uses
// 256 rows, or 128 for the per-coordinate gradient at d >= 8; workspaces are sized for the
// smaller block.
constexpr int kRowsValu = kThreads;
constexpr int kRowsMfma = 256;
constexpr int kRowsMfmaMin = 128;
int mfma_rows_per_block(int kind, int d, int has_grad, int ib_request);
int mfma_ib(int kind, int d, int has_grad, int ib_request);

int64_t pair_blocks(const PassDesc &p);
int64_t fin_blocks(const PassDesc &p);

hipError_t launch_stage(int prec, const void *X, int64_t n, int d, int dp, int kind,
                        const double *theta, char *ws, const WsLayout &L, hipStream_t s);
hipError_t launch_pass(const PassDesc &p, hipStream_t s);
// quad receives the first nq column sums (nq < 0: all of them).
hipError_t launch_reduce(const PassDesc &p, double *grad, double *quad, hipStream_t s, int nq = -1);

bool mfma_supported(int prec, int kind, int d, int R);
size_t mfma_scratch_bytes(int64_t n, int dp);

// typed entry points, defined per precision
hipError_t launch_pass_f32(const PassDesc &p, hipStream_t s);
hipError_t launch_pass_f64(const PassDesc &p, hipStream_t s);
hipError_t launch_pass_mfma(const PassDesc &p, hipStream_t s);
hipError_t launch_pass_xm(const PassDesc &p, hipStream_t s);
int xm_rows_per_block(int has_grad_ard);
size_t xm_scratch_bytes(int64_t n, int d);
hipError_t launch_stage_f32(const void *X, int64_t n, int d, int dp, int kind,
                            const double *theta, char *ws, const WsLayout &L, hipStream_t s);
hipError_t launch_stage_f64(const void *X, int64_t n, int d, int dp, int kind,
                            const double *theta, char *ws, const WsLayout &L, hipStream_t s);

}  // namespace gpk
