// Randomized Nystrom preconditioner (Section 3.1 after eq. pex; Section 3.2.3; rank 5 in
// Section 4.1, rank 500 in Section 4.3) and batched preconditioned conjugate gradients.
//
// Nystrom factor, in the order of the randomized construction the paper uses (Frangella, Tropp
// and Udell), for an n x l Gaussian test matrix Omega supplied by the caller:
//     Q = orth(Omega)            Cholesky-QR applied twice (Gram on the device, l x l Cholesky on
//                                the host in double)
//     Y = K Q                    gp_kmatvec with GP_NO_NOISE, l right-hand sides
//     nu = sqrt(n) eps |Y|_F     Y_nu = Y + nu Q
//     C^T C = Q^T Y_nu,  B = Y_nu C^{-1}
//     B = U S V^T                from the l x l eigendecomposition of B^T B (Householder + QL on the
//                                host): U = B V S^{-1}
//     lam = max(0, S^2 - nu),    K ~ U diag(lam) U^T.
// Preconditioner for A + lambda I = K + mu I (mu = sigma^2 + lambda, so one factor serves every
// shift through the Woodbury identity):
//     P^{-1} r = r + U ((lam_l + mu) / (lam + mu) - 1) U^T r.
// The tall-skinny products (Gram matrices A^T B and right multiplications A M) run in the
// kernels below with double accumulation and fixed-order chunk sums.
#include <math.h>

#include <algorithm>
#include <cmath>
#include <vector>

#include "common.h"
#include "gpk.h"
#include "nystrom.h"
#include "vecops.h"

namespace gpk {

gp_status fail(gp_status st, const char *fmt, ...);
void clear_error();
gp_status hip_fail(hipError_t e, const char *where);

namespace {

constexpr int kRankMax = 512;
constexpr int kPcgMaxR = 32;
constexpr int kCheckEvery = 4;
constexpr int kGT = 32;          // Gram output tile
constexpr int kMR = 64, kMC = 32, kMK = 32;  // right-multiplication tiles

// ---- tall-skinny kernels --------------------------------------------------------------------

// part[chunk][i][j] = sum over the chunk's rows of A[row][i] B[row][j]; i < l1, j < l2.
template <typename T>
__global__ __launch_bounds__(256) void gram_partial(int64_t n, int l1, const T *A, int64_t lda,
                                                    int l2, const T *B, int64_t ldb,
                                                    int64_t rows_per_chunk, double *part) {
  __shared__ double sa[kGT][kGT + 1], sb[kGT][kGT + 1];
  const int t = threadIdx.x;
  const int tiles_j = (l2 + kGT - 1) / kGT;
  const int i0 = (blockIdx.y / tiles_j) * kGT, j0 = (blockIdx.y % tiles_j) * kGT;
  const int ii = t / 8, jj = (t % 8) * 4;
  const int64_t r0 = (int64_t)blockIdx.x * rows_per_chunk;
  const int64_t r1 = min(n, r0 + rows_per_chunk);
  double acc[4] = {0.0, 0.0, 0.0, 0.0};
  for (int64_t rb = r0; rb < r1; rb += kGT) {
    for (int e = t; e < kGT * kGT; e += 256) {
      const int rr = e / kGT, cc = e % kGT;
      const int64_t row = rb + rr;
      sa[rr][cc] = (row < r1 && i0 + cc < l1) ? (double)A[row * lda + i0 + cc] : 0.0;
      sb[rr][cc] = (row < r1 && j0 + cc < l2) ? (double)B[row * ldb + j0 + cc] : 0.0;
    }
    __syncthreads();
    for (int rr = 0; rr < kGT; ++rr) {
      const double a = sa[rr][ii];
#pragma unroll
      for (int q = 0; q < 4; ++q) acc[q] += a * sb[rr][jj + q];
    }
    __syncthreads();
  }
  double *out = part + (int64_t)blockIdx.x * l1 * l2;
  if (i0 + ii < l1)
    for (int q = 0; q < 4; ++q)
      if (j0 + jj + q < l2) out[(int64_t)(i0 + ii) * l2 + j0 + jj + q] = acc[q];
}

// The same partials for l2 <= L2P <= 32 columns of B (the preconditioner's U^T v): one thread per
// row i of A^T streams its column of A (coalesced across threads), the chunk's rows of B are
// staged in LDS 64 at a time; many small chunks keep the grid wide at any n.
template <typename T, int L2P>
__global__ __launch_bounds__(256) void gram_skinny(int64_t n, int l1, const T *A, int64_t lda,
                                                   int l2, const T *B, int64_t ldb,
                                                   int64_t rows_per_chunk, double *part) {
  __shared__ double sb[64][L2P];
  const int i = blockIdx.y * 256 + threadIdx.x;
  const int64_t r0 = (int64_t)blockIdx.x * rows_per_chunk;
  const int64_t r1 = min(n, r0 + rows_per_chunk);
  double acc[L2P];
#pragma unroll
  for (int j = 0; j < L2P; ++j) acc[j] = 0.0;
  for (int64_t rb = r0; rb < r1; rb += 64) {
    const int nr = (int)min((int64_t)64, r1 - rb);
    __syncthreads();
    for (int e = threadIdx.x; e < 64 * L2P; e += 256) {
      const int rr = e / L2P, c = e % L2P;
      sb[rr][c] = (rr < nr && c < l2) ? (double)B[(rb + rr) * ldb + c] : 0.0;
    }
    __syncthreads();
    if (i < l1) {
      const T *a = A + rb * lda + i;
      for (int rr = 0; rr < nr; ++rr) {
        const double av = (double)a[rr * lda];
#pragma unroll
        for (int j = 0; j < L2P; ++j) acc[j] += av * sb[rr][j];
      }
    }
  }
  if (i < l1) {
    double *out = part + ((int64_t)blockIdx.x * l1 + i) * l2;
#pragma unroll
    for (int j = 0; j < L2P; ++j)
      if (j < l2) out[j] = acc[j];
  }
}

// G[e] = sum over chunks of part[chunk][e], one wave per output (lanes over chunks, fixed order).
__global__ __launch_bounds__(256) void gram_final_wave(int nchunk, int64_t m, const double *part,
                                                       double *G) {
  const int64_t e = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
  const int lane = threadIdx.x & 63;
  double v = 0.0;
  if (e < m)
    for (int c = lane; c < nchunk; c += 64) v += part[(int64_t)c * m + e];
  v = wave_sum(v);
  if (e < m && lane == 0) G[e] = v;
}

__global__ void gram_final(int nchunk, int64_t m, const double *part, double *G) {
  const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (e >= m) return;
  double s = 0.0;
  for (int c = 0; c < nchunk; ++c) s += part[(int64_t)c * m + e];
  G[e] = s;
}

// out[row][c] = Cin[row][c] (if given) + sum_k A[row][k] M[k][c]; M is l x m, row-major, double.
template <typename T>
__global__ __launch_bounds__(256) void right_mul(int64_t n, int l, const T *A, int64_t lda,
                                                 const double *M, int m, const T *Cin,
                                                 int64_t ldc, T *out, int64_t ldo, int kper,
                                                 double *part) {
  __shared__ double sa[kMR][kMK + 1], sm[kMK][kMC + 1];
  const int t = threadIdx.x;
  const int64_t row0 = (int64_t)blockIdx.x * kMR;
  const int c0 = blockIdx.y * kMC;
  const int rr = t / 4, cc = (t % 4) * 8;
  // split over the inner dimension (gridDim.z > 1): this block's kper of the l terms, its
  // partial sums to part[z][n][m] for right_mul_sum
  const int kb = blockIdx.z * kper, ke = min(l, kb + kper);
  double acc[8] = {0, 0, 0, 0, 0, 0, 0, 0};
  for (int k0 = kb; k0 < ke; k0 += kMK) {
    for (int e = t; e < kMR * kMK; e += 256) {
      const int a = e / kMK, b = e % kMK;
      const int64_t row = row0 + a;
      sa[a][b] = (row < n && k0 + b < ke) ? (double)A[row * lda + k0 + b] : 0.0;
    }
    for (int e = t; e < kMK * kMC; e += 256) {
      const int a = e / kMC, b = e % kMC;
      sm[a][b] = (k0 + a < ke && c0 + b < m) ? M[(int64_t)(k0 + a) * m + c0 + b] : 0.0;
    }
    __syncthreads();
    for (int k = 0; k < kMK; ++k) {
      const double a = sa[rr][k];
#pragma unroll
      for (int q = 0; q < 8; ++q) acc[q] += a * sm[k][cc + q];
    }
    __syncthreads();
  }
  const int64_t row = row0 + rr;
  if (row < n)
    for (int q = 0; q < 8; ++q) {
      const int c = c0 + cc + q;
      if (c < m) {
        if (part) {
          part[((int64_t)blockIdx.z * n + row) * m + c] = acc[q];
        } else {
          const double base = Cin ? (double)Cin[row * ldc + c] : 0.0;
          out[row * ldo + c] = (T)(base + acc[q]);
        }
      }
    }
}

// out = Cin + the nz partial products of a split right_mul, summed in split order.
template <typename T>
__global__ void right_mul_sum(int64_t n, int m, int nz, const double *part, const T *Cin,
                              int64_t ldc, T *out, int64_t ldo) {
  const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (e >= n * m) return;
  const int64_t row = e / m;
  const int c = (int)(e - row * m);
  double s = 0.0;
  for (int z = 0; z < nz; ++z) s += part[(int64_t)z * n * m + e];
  const double base = Cin ? (double)Cin[row * ldc + c] : 0.0;
  out[row * ldo + c] = (T)(base + s);
}

template <typename T>
__global__ __launch_bounds__(256) void sumsq_partial(int64_t m, const T *a, double *part) {
  __shared__ double sh[4];
  double s = 0.0;
  for (int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x; e < m; e += (int64_t)gridDim.x * 256) {
    const double v = (double)a[e];
    s += v * v;
  }
  s = wave_sum(s);
  if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = s;
  __syncthreads();
  if (threadIdx.x == 0) part[blockIdx.x] = (sh[0] + sh[1]) + (sh[2] + sh[3]);
}

template <typename T>
__global__ __launch_bounds__(256) void axpy_inplace(int64_t m, double a, const T *x, T *y) {
  const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (e < m) y[e] = (T)((double)y[e] + a * (double)x[e]);
}

// ---- host dense linear algebra (l x l, double, row-major) ----------------------------------

// G = C^T C with C upper triangular; false if G is not numerically positive definite.
bool chol_upper(const std::vector<double> &G, int l, std::vector<double> &C) {
  C.assign((size_t)l * l, 0.0);
  for (int j = 0; j < l; ++j) {
    double s = G[(size_t)j * l + j];
    for (int k = 0; k < j; ++k) s -= C[(size_t)k * l + j] * C[(size_t)k * l + j];
    if (!(s > 0.0)) return false;
    const double d = sqrt(s);
    C[(size_t)j * l + j] = d;
    for (int i = j + 1; i < l; ++i) {
      double t = G[(size_t)j * l + i];
      for (int k = 0; k < j; ++k) t -= C[(size_t)k * l + j] * C[(size_t)k * l + i];
      C[(size_t)j * l + i] = t / d;
    }
  }
  return true;
}

// Inverse of an upper-triangular matrix (upper triangular).
void inv_upper(const std::vector<double> &C, int l, std::vector<double> &Ci) {
  Ci.assign((size_t)l * l, 0.0);
  for (int j = 0; j < l; ++j) {
    Ci[(size_t)j * l + j] = 1.0 / C[(size_t)j * l + j];
    for (int i = j - 1; i >= 0; --i) {
      double s = 0.0;
      for (int k = i + 1; k <= j; ++k) s += C[(size_t)i * l + k] * Ci[(size_t)k * l + j];
      Ci[(size_t)i * l + j] = -s / C[(size_t)i * l + i];
    }
  }
}

// Eigenvalues (descending) and orthonormal eigenvectors (columns of V, row-major l x l) of a
// symmetric matrix: Householder reduction to tridiagonal form T = Q^T S Q, then the implicit
// shifted QL iteration on T (Wilkinson-type shift from the leading 2 x 2 block of the active
// part), each plane rotation applied to the accumulated Q.
void sym_eig(std::vector<double> S, int l, std::vector<double> &ev, std::vector<double> &V) {
  const int n = l;
  std::vector<double> Q((size_t)n * n, 0.0), d(n), e(n, 0.0), v(n), p(n), w(n);
  for (int i = 0; i < n; ++i) Q[(size_t)i * n + i] = 1.0;
  auto A = [&](int i, int j) -> double & { return S[(size_t)i * n + j]; };
  // Householder: for column k, reflect rows k+1..n-1 so that A(k+2.., k) = 0
  for (int k = 0; k + 2 < n; ++k) {
    double sig = 0.0;
    for (int i = k + 1; i < n; ++i) sig += A(i, k) * A(i, k);
    const double xn = std::sqrt(sig);
    if (xn == 0.0) continue;
    const double x0 = A(k + 1, k);
    const double alpha = x0 > 0.0 ? -xn : xn;
    // v = x - alpha e1, unit length
    double vn2 = 0.0;
    for (int i = k + 1; i < n; ++i) {
      v[i] = A(i, k) - (i == k + 1 ? alpha : 0.0);
      vn2 += v[i] * v[i];
    }
    if (vn2 == 0.0) continue;
    const double inv = 1.0 / std::sqrt(vn2);
    for (int i = k + 1; i < n; ++i) v[i] *= inv;
    // H A H on rows/columns k.. with H = I - 2 v v^T (v zero above k+1): p = A v over the
    // trailing block (and row k), K = v^T p, w = p - K v, A -= 2 (v w^T + w v^T)
    for (int i = k; i < n; ++i) {
      double t = 0.0;
      for (int j = k + 1; j < n; ++j) t += A(i, j) * v[j];
      p[i] = t;
    }
    double K = 0.0;
    for (int i = k + 1; i < n; ++i) K += v[i] * p[i];
    for (int i = k; i < n; ++i) w[i] = p[i] - (i > k ? K * v[i] : 0.0);
    for (int i = k; i < n; ++i) {
      const double vi = i > k ? v[i] : 0.0;
      for (int j = k; j < n; ++j) {
        const double vj = j > k ? v[j] : 0.0;
        A(i, j) -= 2.0 * (vi * w[j] + w[i] * vj);
      }
    }
    // Q <- Q H
    for (int r = 0; r < n; ++r) {
      double t = 0.0;
      for (int j = k + 1; j < n; ++j) t += Q[(size_t)r * n + j] * v[j];
      t *= 2.0;
      for (int j = k + 1; j < n; ++j) Q[(size_t)r * n + j] -= t * v[j];
    }
  }
  for (int i = 0; i < n; ++i) d[i] = A(i, i);
  for (int i = 0; i + 1 < n; ++i) e[i] = A(i + 1, i);  // e[i] couples i and i + 1
  // implicit QL: deflate from the top; the active block is lo..m with e[m] negligible
  for (int lo = 0; lo < n; ++lo) {
    for (int iter = 0; iter < 60; ++iter) {
      int m = lo;
      for (; m + 1 < n; ++m) {
        const double dd = std::fabs(d[m]) + std::fabs(d[m + 1]);
        if (std::fabs(e[m]) <= 1e-16 * dd) break;
      }
      if (m == lo) break;
      // shift: the eigenvalue of the leading 2 x 2 block [d_lo e_lo; e_lo d_lo+1] nearer d_lo
      double g = (d[lo + 1] - d[lo]) / (2.0 * e[lo]);
      double r = std::hypot(g, 1.0);
      g = d[m] - d[lo] + e[lo] / (g + (g >= 0.0 ? r : -r));
      double s = 1.0, c = 1.0, pp = 0.0;
      int i = m - 1;
      bool early = false;
      for (; i >= lo; --i) {
        const double f = s * e[i], b = c * e[i];
        r = std::hypot(f, g);
        e[i + 1] = r;
        if (r == 0.0) {  // underflow: the block splits here
          d[i + 1] -= pp;
          e[m] = 0.0;
          early = true;
          break;
        }
        s = f / r;
        c = g / r;
        g = d[i + 1] - pp;
        r = (d[i] - g) * s + 2.0 * c * b;
        pp = s * r;
        d[i + 1] = g + pp;
        g = c * r - b;
        for (int k = 0; k < n; ++k) {  // rotate columns i, i + 1 of Q
          const double qa = Q[(size_t)k * n + i], qb = Q[(size_t)k * n + i + 1];
          Q[(size_t)k * n + i + 1] = s * qa + c * qb;
          Q[(size_t)k * n + i] = c * qa - s * qb;
        }
      }
      if (early) continue;
      d[lo] -= pp;
      e[lo] = g;
      e[m] = 0.0;
    }
  }
  // descending order
  std::vector<int> idx(n);
  for (int i = 0; i < n; ++i) idx[i] = i;
  std::sort(idx.begin(), idx.end(), [&](int a, int b) { return d[a] > d[b]; });
  ev.resize(n);
  V.assign((size_t)n * n, 0.0);
  for (int j = 0; j < n; ++j) {
    ev[j] = d[idx[j]];
    for (int k = 0; k < n; ++k) V[(size_t)k * n + j] = Q[(size_t)k * n + idx[j]];
  }
}

// ---- workspace helpers ------------------------------------------------------------------------

int gram_chunks(int64_t n) {
  int64_t c = (n + 4095) / 4096;
  return (int)std::max<int64_t>(1, std::min<int64_t>(64, c));
}

struct Gram {
  int nchunk;
  int64_t rows_per_chunk;
};

Gram gram_plan(int64_t n) {
  Gram g;
  g.nchunk = gram_chunks(n);
  g.rows_per_chunk = (n + g.nchunk - 1) / g.nchunk;
  g.nchunk = (int)((n + g.rows_per_chunk - 1) / g.rows_per_chunk);
  return g;
}

// Chunks of the skinny Gram (l2 <= 32): about 512 rows each, or for small n as many chunks of at
// least 64 rows as make about 512 workgroups (a 3000 x 500 by 15 Gram in 6 chunks, 12
// workgroups, took 214 us); at most ~2^20 partial doubles.
Gram skinny_plan(int64_t n, int l1, int l2) {
  Gram g;
  const int64_t cap = std::max<int64_t>(1, ((int64_t)1 << 20) / ((int64_t)l1 * l2));
  const int64_t ytiles = (l1 + 255) / 256;
  const int64_t want = std::min<int64_t>((n + 63) / 64, (512 + ytiles - 1) / ytiles);
  g.nchunk = (int)std::max<int64_t>(1, std::min<int64_t>(cap, std::max<int64_t>((n + 511) / 512, want)));
  g.rows_per_chunk = (n + g.nchunk - 1) / g.nchunk;
  g.nchunk = (int)((n + g.rows_per_chunk - 1) / g.rows_per_chunk);
  return g;
}

template <typename T, int L2P>
void launch_skinny(const Gram &g, int64_t n, int l1, const T *A, int64_t lda, int l2, const T *B,
                   int64_t ldb, double *part, hipStream_t s) {
  gram_skinny<T, L2P><<<dim3((unsigned)g.nchunk, (unsigned)((l1 + 255) / 256)), 256, 0, s>>>(
      n, l1, A, lda, l2, B, ldb, g.rows_per_chunk, part);
}

// Partial doubles gram() writes for an l1 x l2 product over n rows (sizes its part buffer).
int64_t gram_part_doubles(int64_t n, int l1, int l2) {
  const int nchunk = l2 <= 32 ? skinny_plan(n, l1, l2).nchunk : gram_plan(n).nchunk;
  return (int64_t)nchunk * l1 * l2;
}

template <typename T>
hipError_t gram(int64_t n, int l1, const T *A, int64_t lda, int l2, const T *B, int64_t ldb,
                double *part, double *G, hipStream_t s) {
  if (l2 <= 32) {
    const Gram g = skinny_plan(n, l1, l2);
    if (l2 == 1) launch_skinny<T, 1>(g, n, l1, A, lda, l2, B, ldb, part, s);
    else if (l2 <= 2) launch_skinny<T, 2>(g, n, l1, A, lda, l2, B, ldb, part, s);
    else if (l2 <= 4) launch_skinny<T, 4>(g, n, l1, A, lda, l2, B, ldb, part, s);
    else if (l2 <= 8) launch_skinny<T, 8>(g, n, l1, A, lda, l2, B, ldb, part, s);
    else if (l2 <= 16) launch_skinny<T, 16>(g, n, l1, A, lda, l2, B, ldb, part, s);
    else launch_skinny<T, 32>(g, n, l1, A, lda, l2, B, ldb, part, s);
    const int64_t m = (int64_t)l1 * l2;
    gram_final_wave<<<(unsigned)((m + 3) / 4), 256, 0, s>>>(g.nchunk, m, part, G);
    return hipGetLastError();
  }
  const Gram g = gram_plan(n);
  const int tiles = ((l1 + kGT - 1) / kGT) * ((l2 + kGT - 1) / kGT);
  gram_partial<T><<<dim3((unsigned)g.nchunk, (unsigned)tiles), 256, 0, s>>>(n, l1, A, lda, l2, B, ldb,
                                                                           g.rows_per_chunk, part);
  const int64_t m = (int64_t)l1 * l2;
  gram_final<<<(unsigned)((m + 255) / 256), 256, 0, s>>>(g.nchunk, m, part, G);
  return hipGetLastError();
}

// Splits of the inner dimension for a small right multiplication (about 512 blocks in all, at
// least 64 terms each, at most kMulSplitMax; a 3000 x 500 by 15 product ran 47 blocks, 94 us),
// and the partial-product doubles they need.
constexpr int kMulSplitMax = 8;
constexpr int64_t kMulSplitRows = 8192;  // larger n: enough blocks without a split
int mul_splits(int64_t n, int l, int m) {
  const int64_t blocks = ((n + kMR - 1) / kMR) * ((m + kMC - 1) / kMC);
  if (n > kMulSplitRows || blocks >= 256) return 1;
  int64_t z = std::min<int64_t>(kMulSplitMax, (512 + blocks - 1) / blocks);
  z = std::min<int64_t>(z, std::max<int64_t>(1, l / 64));
  return (int)std::max<int64_t>(1, z);
}
size_t mul_split_doubles(int64_t n, int l, int m) {
  const int z = mul_splits(n, l, m);
  return z > 1 ? (size_t)z * n * m : 0;
}

// out = Cin + A M (A n x l, M l x m); split over l into `split` (mul_split_doubles scratch) when
// that is given and the product is small.
template <typename T>
hipError_t rmul(int64_t n, int l, const T *A, int64_t lda, const double *M, int m, const T *Cin,
                int64_t ldc, T *out, int64_t ldo, hipStream_t s, double *split = nullptr) {
  const int z = split ? mul_splits(n, l, m) : 1;
  const int kper = z > 1 ? (((l + z - 1) / z + kMK - 1) / kMK) * kMK : l;
  const int nz = (l + kper - 1) / kper;
  right_mul<T><<<dim3((unsigned)((n + kMR - 1) / kMR), (unsigned)((m + kMC - 1) / kMC), (unsigned)nz),
                 256, 0, s>>>(n, l, A, lda, M, m, Cin, ldc, out, ldo, kper, nz > 1 ? split : nullptr);
  if (nz > 1)
    right_mul_sum<T><<<(unsigned)((n * m + 255) / 256), 256, 0, s>>>(n, m, nz, split, Cin, ldc, out,
                                                                    ldo);
  return hipGetLastError();
}

gp_status to_host(std::vector<double> &h, const double *d, size_t m, hipStream_t s) {
  h.resize(m);
  hipError_t e = hipMemcpyAsync(h.data(), d, sizeof(double) * m, hipMemcpyDeviceToHost, s);
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  return e == hipSuccess ? GP_OK : hip_fail(e, "device -> host");
}

gp_status to_dev(double *d, const std::vector<double> &h, hipStream_t s) {
  hipError_t e = hipMemcpyAsync(d, h.data(), sizeof(double) * h.size(), hipMemcpyHostToDevice, s);
  if (e == hipSuccess) e = hipStreamSynchronize(s);  // h is a local of the caller
  return e == hipSuccess ? GP_OK : hip_fail(e, "host -> device");
}

struct NysLayout {
  size_t prod, prod_bytes, q, y, w, part, G, M, ss, total;
};

gp_kernel no_noise_of(const gp_kernel *k) {
  gp_kernel kk = *k;
  kk.flags |= GP_NO_NOISE;
  return kk;
}

NysLayout nys_layout(const gp_kernel *k, int64_t n, int l) {
  NysLayout L;
  const size_t es = k->prec == GP_F64 ? 8 : 4;
  const gp_kernel kk = no_noise_of(k);
  size_t o = 0;
  L.prod = o;
  L.prod_bytes = gp_workspace_size(&kk, n, l);
  o += align256(L.prod_bytes);
  L.q = o;
  o += align256(es * n * l);
  L.y = o;
  o += align256(es * n * l);
  L.w = o;
  o += align256(es * n * l);
  L.part = o;
  o += align256(sizeof(double) * (size_t)gram_part_doubles(n, l, l));
  L.G = o;
  o += align256(sizeof(double) * l * l);
  L.M = o;
  o += align256(sizeof(double) * l * l);
  L.ss = o;
  o += align256(sizeof(double) * 1024);
  L.total = o;
  return L;
}

// Q = W R^{-1}, R from the Cholesky factor of W^T W (one Cholesky-QR step).
template <typename T>
gp_status cholqr_step(int64_t n, int l, const T *W, T *Q, const NysLayout &L, char *w,
                      hipStream_t s) {
  double *part = (double *)(w + L.part), *G = (double *)(w + L.G), *M = (double *)(w + L.M);
  hipError_t e = gram<T>(n, l, W, l, l, W, l, part, G, s);
  if (e != hipSuccess) return hip_fail(e, "Gram");
  std::vector<double> hG, C, Ci;
  gp_status st = to_host(hG, G, (size_t)l * l, s);
  if (st) return st;
  if (!chol_upper(hG, l, C)) return fail(GP_ERR_ARG, "the test matrix is rank deficient");
  inv_upper(C, l, Ci);
  st = to_dev(M, Ci, s);
  if (st) return st;
  e = rmul<T>(n, l, W, l, M, l, nullptr, 0, Q, l, s);
  return e == hipSuccess ? GP_OK : hip_fail(e, "right multiplication");
}

template <typename T>
gp_status run_nystrom(const gp_kernel *k, int64_t n, const void *X, const double *theta, int l,
                      const T *omega, T *U, double *lam, char *w, const NysLayout &L,
                      hipStream_t s) {
  T *Q = (T *)(w + L.q), *Y = (T *)(w + L.y), *W = (T *)(w + L.w);
  double *part = (double *)(w + L.part), *G = (double *)(w + L.G), *M = (double *)(w + L.M);
  // Q = orth(Omega): Cholesky-QR twice
  gp_status st = cholqr_step<T>(n, l, omega, W, L, w, s);
  if (st) return st;
  st = cholqr_step<T>(n, l, W, Q, L, w, s);
  if (st) return st;
  // Y = K Q
  const gp_kernel kk = no_noise_of(k);
  st = gp_kmatvec(&kk, n, X, theta, l, Q, l, nullptr, Y, l, w + L.prod, L.prod_bytes, s);
  if (st) return st;
  // nu = sqrt(n) eps |Y|_F, Y += nu Q
  const int64_t m = n * l;
  const int sb = (int)std::min<int64_t>(1024, (m + 255) / 256);
  sumsq_partial<T><<<sb, 256, 0, s>>>(m, Y, (double *)(w + L.ss));
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return hip_fail(e, "norm");
  std::vector<double> hs;
  st = to_host(hs, (const double *)(w + L.ss), sb, s);
  if (st) return st;
  double ss = 0.0;
  for (int b = 0; b < sb; ++b) ss += hs[b];
  const double eps = k->prec == GP_F64 ? 2.220446049250313e-16 : 1.1920928955078125e-07;
  const double nu = sqrt((double)n) * eps * sqrt(ss);
  axpy_inplace<T><<<(unsigned)((m + 255) / 256), 256, 0, s>>>(m, nu, Q, Y);
  // C^T C = Q^T Y_nu (symmetrised), B = Y_nu C^{-1} into W
  e = gram<T>(n, l, Q, l, l, Y, l, part, G, s);
  if (e != hipSuccess) return hip_fail(e, "Gram");
  std::vector<double> hG, C, Ci;
  st = to_host(hG, G, (size_t)l * l, s);
  if (st) return st;
  for (int i = 0; i < l; ++i)
    for (int j = 0; j < i; ++j) {
      const double a = 0.5 * (hG[(size_t)i * l + j] + hG[(size_t)j * l + i]);
      hG[(size_t)i * l + j] = a;
      hG[(size_t)j * l + i] = a;
    }
  if (!chol_upper(hG, l, C)) return fail(GP_ERR_ARG, "Q^T (K + nu I) Q is not positive definite");
  inv_upper(C, l, Ci);
  st = to_dev(M, Ci, s);
  if (st) return st;
  e = rmul<T>(n, l, Y, l, M, l, nullptr, 0, W, l, s);
  if (e != hipSuccess) return hip_fail(e, "right multiplication");
  // B^T B = V S^2 V^T, U = B V S^{-1}, lam = max(0, S^2 - nu)
  e = gram<T>(n, l, W, l, l, W, l, part, G, s);
  if (e != hipSuccess) return hip_fail(e, "Gram");
  st = to_host(hG, G, (size_t)l * l, s);
  if (st) return st;
  std::vector<double> ev, V;
  sym_eig(hG, l, ev, V);
  std::vector<double> hM((size_t)l * l), hl(l);
  for (int j = 0; j < l; ++j) {
    const double s2 = ev[j] > 0.0 ? ev[j] : 0.0;
    const double inv = s2 > 0.0 ? 1.0 / sqrt(s2) : 0.0;
    for (int i = 0; i < l; ++i) hM[(size_t)i * l + j] = V[(size_t)i * l + j] * inv;
    hl[j] = std::max(0.0, s2 - nu);
  }
  st = to_dev(M, hM, s);
  if (st) return st;
  e = rmul<T>(n, l, W, l, M, l, nullptr, 0, U, l, s);
  if (e != hipSuccess) return hip_fail(e, "right multiplication");
  return to_dev(lam, hl, s);
}

// ---- preconditioned CG ------------------------------------------------------------------------

struct PcgCol {
  double rz, bb, a, beta;
  int32_t done, iters, status, pad;
};

template <typename T>
__global__ __launch_bounds__(256) void pcg_residual(int64_t n, int r, VecGrid g, const T *B,
                                                    int64_t ldb, const T *q, T *rv, double *part) {
  __shared__ double sh[kThreads];
  const int t = threadIdx.x, c = t % r, l = t / r;
  double acc = 0.0;
  if (l < g.rps) {
    const int64_t i1 = min(n, (int64_t)(blockIdx.x + 1) * g.rows_per_block);
    for (int64_t i = (int64_t)blockIdx.x * g.rows_per_block + l; i < i1; i += g.rps) {
      const double b = (double)B[i * ldb + c];
      rv[i * r + c] = (T)(b - (double)q[i * r + c]);
      acc += b * b;
    }
  }
  block_column_sum(acc, sh, r, g.rps, part);
}

// part = per-column partial sums of a . b
template <typename T>
__global__ __launch_bounds__(256) void pcg_dot(int64_t n, int r, VecGrid g, const T *a, const T *b,
                                               double *part) {
  __shared__ double sh[kThreads];
  const int t = threadIdx.x, c = t % r, l = t / r;
  double acc = 0.0;
  if (l < g.rps) {
    const int64_t i1 = min(n, (int64_t)(blockIdx.x + 1) * g.rows_per_block);
    for (int64_t i = (int64_t)blockIdx.x * g.rows_per_block + l; i < i1; i += g.rps)
      acc += (double)a[i * r + c] * (double)b[i * r + c];
  }
  block_column_sum(acc, sh, r, g.rps, part);
}

// x += a p, r -= a q for live columns; partial sums of the new r . r
template <typename T>
__global__ __launch_bounds__(256) void pcg_update(int64_t n, int r, VecGrid g, const PcgCol *col,
                                                  const T *p, const T *q, T *x, int64_t ldx, T *rv,
                                                  double *part) {
  __shared__ double sh[kThreads];
  const int t = threadIdx.x, c = t % r, l = t / r;
  double acc = 0.0;
  if (l < g.rps && !col[c].done) {
    const double a = col[c].a;
    const int64_t i1 = min(n, (int64_t)(blockIdx.x + 1) * g.rows_per_block);
    for (int64_t i = (int64_t)blockIdx.x * g.rows_per_block + l; i < i1; i += g.rps) {
      x[i * ldx + c] = (T)((double)x[i * ldx + c] + a * (double)p[i * r + c]);
      const T rn = (T)((double)rv[i * r + c] - a * (double)q[i * r + c]);
      rv[i * r + c] = rn;
      acc += (double)rn * (double)rn;
    }
  }
  block_column_sum(acc, sh, r, g.rps, part);
}

template <typename T>
__global__ __launch_bounds__(256) void pcg_direction(int64_t n, int r, VecGrid g, const PcgCol *col,
                                                     const T *z, T *p, int first) {
  const int t = threadIdx.x, c = t % r, l = t / r;
  if (l >= g.rps || col[c].done) return;
  const double beta = first ? 0.0 : col[c].beta;
  const int64_t i1 = min(n, (int64_t)(blockIdx.x + 1) * g.rows_per_block);
  for (int64_t i = (int64_t)blockIdx.x * g.rows_per_block + l; i < i1; i += g.rps)
    p[i * r + c] = (T)((double)z[i * r + c] + (first ? 0.0 : beta * (double)p[i * r + c]));
}

// M[k][c] = ((lam_l + mu_c) / (lam_k + mu_c) - 1) t[k][c], mu_c = sigma^2 + shift_c
__global__ void pcg_prec_scale(int l, int r, const double *lam, const double *theta, int nth,
                               const double *shift, const double *tkc, double *M) {
  const int e = blockIdx.x * 256 + threadIdx.x;
  if (e >= l * r) return;
  const int kk = e / r, c = e % r;
  const double mu = exp(theta[nth - 1]) + (shift ? shift[c] : 0.0);
  M[e] = ((lam[l - 1] + mu) / (lam[kk] + mu) - 1.0) * tkc[e];
}

// Column scalars.  stage 0: bb, rr from part0 / part1 (set-up); stage 1: a = rz / (p.q);
// stage 2: convergence on r.r; stage 3: beta from the new r.z.
__global__ void pcg_scalars(int stage, int r, int64_t blocks, const double *part, double tol,
                            int it, PcgCol *col, int32_t *remaining) {
  __shared__ double red[kThreads];
  __shared__ double tot[kThreads];
  __shared__ int32_t left;
  if (threadIdx.x == 0) left = 0;
  column_totals(part, blocks, r, red, tot);
  for (int c = 0; c < r; ++c) {
    const double v = tot[c];
    if (threadIdx.x == 0) {
      PcgCol s = col[c];
      if (stage == 0) {
        s.bb = v;
        s.done = 0;
        s.iters = 0;
        s.status = isfinite(v) ? 0 : GP_CG_NONFINITE;
        s.rz = 0.0;
        s.a = 0.0;
        s.beta = 0.0;
        s.pad = 0;
      } else if (!s.done) {
        if (stage == 1) {
          s.a = s.rz / v;
          if (!(isfinite(s.a) && v > 0.0)) {
            s.status |= GP_CG_NONFINITE;
            s.done = 1;
          }
        } else if (stage == 2) {
          // iterations taken: `it` is 1 inside an iteration, 0 for the set-up's test (the
          // launches carry no iteration index, so a captured group of them can be replayed)
          s.iters += it;
          if (!isfinite(v)) {
            s.status |= GP_CG_NONFINITE;
            s.done = 1;
          } else if (v <= tol * tol * s.bb) {
            s.done = 1;
          }
        } else if (stage == 3) {
          s.beta = v / s.rz;
          s.rz = v;
          if (!isfinite(s.beta)) {
            s.status |= GP_CG_NONFINITE;
            s.done = 1;
          }
        } else if (stage == 4) {  // initial r . z
          s.rz = v;
        }
      }
      left += 1 - s.done;
      col[c] = s;
    }
  }
  __syncthreads();
  if (threadIdx.x == 0 && remaining) *remaining = left;
}

__global__ void pcg_finish(int r, int maxit, const PcgCol *col, int32_t *status, int32_t *iters) {
  const int c = threadIdx.x;
  if (c >= r) return;
  const PcgCol s = col[c];
  if (status) status[c] = s.status | (s.done ? 0 : GP_CG_MAXIT);
  if (iters) iters[c] = s.done ? s.iters : maxit;
}

template <typename T>
__global__ void copy_block(int64_t n, int r, const T *a, T *b) {
  const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (e < n * r) b[e] = a[e];
}

struct PcgLayout {
  size_t prod, prod_bytes, rv, zv, pv, qv, part, scr, col, remaining, total;
};

PcgLayout pcg_layout(const gp_kernel *k, int64_t n, int r, int rank) {
  PcgLayout L;
  const size_t es = k->prec == GP_F64 ? 8 : 4;
  size_t o = 0;
  L.prod = o;
  L.prod_bytes = gp_workspace_size(k, n, r);
  o += align256(L.prod_bytes);
  L.rv = o;
  o += align256(es * n * r);
  L.zv = o;
  o += align256(es * n * r);
  L.pv = o;
  o += align256(es * n * r);
  L.qv = o;
  o += align256(es * n * r);
  L.part = o;
  o += align256(sizeof(double) * kVecBlocksMax * r);
  L.scr = o;
  o += align256(nystrom_apply_scratch(n, std::max(rank, 1), r));
  L.col = o;
  o += align256(sizeof(PcgCol) * r);
  L.remaining = o;
  o += 256;
  L.total = o;
  return L;
}

template <typename T>
gp_status run_pcg(const gp_kernel *k, int64_t n, const void *X, const double *theta, int r,
                  const T *B, int64_t ldb, T *x, int64_t ldx, const double *shift, int rank,
                  const T *U, const double *lam, double tol, int maxit, int32_t *status,
                  int32_t *iters, char *w, const PcgLayout &L, hipStream_t s) {
  T *rv = (T *)(w + L.rv), *zv = (T *)(w + L.zv), *pv = (T *)(w + L.pv), *qv = (T *)(w + L.qv);
  double *part = (double *)(w + L.part);
  PcgCol *col = (PcgCol *)(w + L.col);
  int32_t *remaining = (int32_t *)(w + L.remaining);
  const int nth = gp_n_theta(k);
  const VecGrid g = vec_grid(n, r);
  const unsigned vb = (unsigned)g.blocks;
  const unsigned eb = (unsigned)((n * r + 255) / 256);
  auto precond = [&](hipStream_t q) -> gp_status {  // z = P^{-1} r
    hipError_t e;
    if (rank == 0) {
      copy_block<T><<<eb, 256, 0, q>>>(n, r, rv, zv);
      e = hipGetLastError();
    } else {
      e = nystrom_apply<T>(n, rank, U, lam, theta, nth, shift, r, rv, zv, w + L.scr, q);
    }
    return e == hipSuccess ? GP_OK : hip_fail(e, "preconditioner");
  };
  // r = b - (A + shift) x, |b|^2
  gp_status st = gp_kmatvec(k, n, X, theta, r, x, ldx, shift, qv, r, w + L.prod, L.prod_bytes, s);
  if (st) return st;
  pcg_residual<T><<<vb, 256, 0, s>>>(n, r, g, B, ldb, qv, rv, part);
  pcg_scalars<<<1, 256, 0, s>>>(0, r, g.blocks, part, tol, 0, col, nullptr);
  pcg_dot<T><<<vb, 256, 0, s>>>(n, r, g, rv, rv, part);
  pcg_scalars<<<1, 256, 0, s>>>(2, r, g.blocks, part, tol, 0, col, remaining);
  st = precond(s);
  if (st) return st;
  pcg_dot<T><<<vb, 256, 0, s>>>(n, r, g, rv, zv, part);
  pcg_scalars<<<1, 256, 0, s>>>(4, r, g.blocks, part, tol, 0, col, nullptr);
  pcg_direction<T><<<vb, 256, 0, s>>>(n, r, g, col, zv, pv, 1);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return hip_fail(e, "PCG set-up");
  // one iteration: the same launches every time (finished columns skip their updates), so
  // kCheckEvery of them are captured once as a graph and replayed between convergence checks;
  // the iterations past the last whole group run eagerly, so no more than maxit are taken
  auto iteration = [&](hipStream_t q) -> gp_status {
    gp_status r2 = gp_kmatvec(k, n, X, theta, r, pv, r, shift, qv, r, w + L.prod, L.prod_bytes, q);
    if (r2 == GP_OK) {
      pcg_dot<T><<<vb, 256, 0, q>>>(n, r, g, pv, qv, part);
      pcg_scalars<<<1, 256, 0, q>>>(1, r, g.blocks, part, tol, 0, col, nullptr);
      pcg_update<T><<<vb, 256, 0, q>>>(n, r, g, col, pv, qv, x, ldx, rv, part);
      pcg_scalars<<<1, 256, 0, q>>>(2, r, g.blocks, part, tol, 1, col, remaining);
      r2 = precond(q);
    }
    if (r2 == GP_OK) {
      pcg_dot<T><<<vb, 256, 0, q>>>(n, r, g, rv, zv, part);
      pcg_scalars<<<1, 256, 0, q>>>(3, r, g.blocks, part, tol, 0, col, nullptr);
      pcg_direction<T><<<vb, 256, 0, q>>>(n, r, g, col, zv, pv, 0);
      const hipError_t he = hipGetLastError();
      if (he != hipSuccess) r2 = hip_fail(he, "PCG iteration");
    }
    return r2;
  };
  hipGraphExec_t exec = nullptr;
  if (maxit >= kCheckEvery) {
    hipStream_t cap;
    e = hipStreamCreateWithFlags(&cap, hipStreamNonBlocking);
    if (e != hipSuccess) return hip_fail(e, "capture stream");
    hipGraph_t graph = nullptr;
    gp_status sc = GP_OK;
    e = hipStreamBeginCapture(cap, hipStreamCaptureModeThreadLocal);
    if (e == hipSuccess) {
      for (int i = 0; i < kCheckEvery && sc == GP_OK; ++i) sc = iteration(cap);
      const hipError_t ee = hipStreamEndCapture(cap, &graph);
      if (e == hipSuccess) e = ee;
    }
    if (e == hipSuccess && sc == GP_OK) e = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
    if (graph) (void)hipGraphDestroy(graph);
    (void)hipStreamDestroy(cap);
    if (sc != GP_OK) return sc;
    if (e != hipSuccess) return hip_fail(e, "PCG graph");
  }
  for (int it = 0; it < maxit;) {
    int32_t left = 0;
    e = hipMemcpyAsync(&left, remaining, sizeof(int32_t), hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess || left == 0) break;
    if (exec && maxit - it >= kCheckEvery) {
      e = hipGraphLaunch(exec, s);
      if (e != hipSuccess) break;
      it += kCheckEvery;
    } else {
      st = iteration(s);
      if (st) break;
      ++it;
    }
  }
  if (exec) (void)hipGraphExecDestroy(exec);
  if (st) return st;
  if (e != hipSuccess) return hip_fail(e, "PCG iterations");
  pcg_finish<<<1, 64, 0, s>>>(r, maxit, col, status, iters);
  e = hipGetLastError();
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  return e == hipSuccess ? GP_OK : hip_fail(e, "PCG finish");
}

bool ranges_overlap(const void *a, int64_t rows, int64_t lda, int cols, const void *b, int64_t ldb,
                    int bcols, size_t es) {
  const char *a0 = (const char *)a, *b0 = (const char *)b;
  const char *a1 = a0 + ((rows - 1) * lda + cols) * (int64_t)es;
  const char *b1 = b0 + ((rows - 1) * ldb + bcols) * (int64_t)es;
  return a0 < b1 && b0 < a1;
}

}  // namespace

size_t nystrom_apply_scratch(int64_t n, int rank, int r) {
  return align256(sizeof(double) * (size_t)gram_part_doubles(n, rank, r)) +
         2 * align256(sizeof(double) * (size_t)rank * r) +
         align256(sizeof(double) * mul_split_doubles(n, rank, r));
}

template <typename T>
hipError_t nystrom_apply(int64_t n, int rank, const T *U, const double *lam, const double *theta,
                         int nth, const double *shift, int r, const T *v, T *z, char *scratch,
                         hipStream_t s) {
  double *gpart = (double *)scratch;
  double *tkc = (double *)(scratch + align256(sizeof(double) * (size_t)gram_part_doubles(n, rank, r)));
  double *M = tkc + align256(sizeof(double) * (size_t)rank * r) / sizeof(double);
  double *split = M + align256(sizeof(double) * (size_t)rank * r) / sizeof(double);
  hipError_t e = gram<T>(n, rank, U, rank, r, v, r, gpart, tkc, s);
  if (e != hipSuccess) return e;
  pcg_prec_scale<<<(unsigned)((rank * r + 255) / 256), 256, 0, s>>>(rank, r, lam, theta, nth, shift,
                                                                    tkc, M);
  return rmul<T>(n, rank, U, rank, M, r, v, r, z, r, s, split);
}

template hipError_t nystrom_apply<float>(int64_t, int, const float *, const double *,
                                         const double *, int, const double *, int, const float *,
                                         float *, char *, hipStream_t);
template hipError_t nystrom_apply<double>(int64_t, int, const double *, const double *,
                                          const double *, int, const double *, int, const double *,
                                          double *, char *, hipStream_t);

}  // namespace gpk

using namespace gpk;

extern "C" {

size_t gp_nystrom_workspace_size(const gp_kernel *k, int64_t n, int32_t rank) {
  if (gp_n_theta(k) < 0 || n < 1 || rank < 1 || rank > kRankMax || rank > n) return 0;
  return nys_layout(k, n, rank).total;
}

gp_status gp_nystrom(const gp_kernel *k, int64_t n, const void *X, const double *theta,
                     int32_t rank, const void *omega, void *U, double *lam, void *ws,
                     size_t ws_bytes, hipStream_t stream) {
  clear_error();
  if (gp_n_theta(k) < 0) return fail(GP_ERR_ARG, "invalid kernel description");
  if (n < 1) return fail(GP_ERR_SHAPE, "n = %lld < 1", (long long)n);
  if (rank < 1 || rank > kRankMax || rank > n)
    return fail(GP_ERR_SHAPE, "rank = %d outside 1..min(n, %d)", rank, kRankMax);
  if (!X || !theta || !omega || !U || !lam)
    return fail(GP_ERR_ARG, "X, theta, omega, U and lam must be non-NULL");
  const size_t es = k->prec == GP_F64 ? 8 : 4;
  if (ranges_overlap(omega, n, rank, rank, U, rank, rank, es)) return fail(GP_ERR_ARG, "U overlaps omega");
  const NysLayout L = nys_layout(k, n, rank);
  if (!ws || ws_bytes < L.total)
    return fail(GP_ERR_WORKSPACE, "workspace of %zu bytes needed, %zu given", L.total,
                ws ? ws_bytes : (size_t)0);
  if (k->prec == GP_F64)
    return run_nystrom<double>(k, n, X, theta, rank, (const double *)omega, (double *)U, lam,
                               (char *)ws, L, stream);
  return run_nystrom<float>(k, n, X, theta, rank, (const float *)omega, (float *)U, lam, (char *)ws,
                            L, stream);
}

size_t gp_pcg_workspace_size(const gp_kernel *k, int64_t n, int32_t r, int32_t rank) {
  if (gp_n_theta(k) < 0 || (k->flags & GP_NO_NOISE) || n < 1 || r < 1 || r > kPcgMaxR || rank < 0 ||
      rank > kRankMax)
    return 0;
  return pcg_layout(k, n, r, rank).total;
}

gp_status gp_pcg_solve(const gp_kernel *k, int64_t n, const void *X, const double *theta,
                       int32_t r, const void *B, int64_t ldb, void *x, int64_t ldx,
                       const double *col_shift, int32_t rank, const void *U, const double *lam,
                       double tol, int32_t maxit, int32_t *status, int32_t *iters, void *ws,
                       size_t ws_bytes, hipStream_t stream) {
  clear_error();
  if (gp_n_theta(k) < 0) return fail(GP_ERR_ARG, "invalid kernel description");
  if (k->flags & GP_NO_NOISE) return fail(GP_ERR_ARG, "GP_NO_NOISE: K alone need not be invertible");
  if (n < 1) return fail(GP_ERR_SHAPE, "n = %lld < 1", (long long)n);
  if (r < 1 || r > kPcgMaxR) return fail(GP_ERR_SHAPE, "r = %d outside 1..%d", r, kPcgMaxR);
  if (rank < 0 || rank > kRankMax) return fail(GP_ERR_SHAPE, "rank = %d outside 0..%d", rank, kRankMax);
  if (!X || !theta || !B || !x) return fail(GP_ERR_ARG, "X, theta, B and x must be non-NULL");
  if (rank > 0 && (!U || !lam)) return fail(GP_ERR_ARG, "rank > 0 needs U and lam");
  if (ldb < r || ldx < r) return fail(GP_ERR_SHAPE, "leading dimensions must be >= r = %d", r);
  if (!(tol > 0.0)) return fail(GP_ERR_ARG, "tol must be > 0");
  if (maxit < 0) return fail(GP_ERR_ARG, "maxit must be >= 0");
  const size_t es = k->prec == GP_F64 ? 8 : 4;
  if (ranges_overlap(B, n, ldb, r, x, ldx, r, es)) return fail(GP_ERR_ARG, "x overlaps B");
  const PcgLayout L = pcg_layout(k, n, r, rank);
  if (!ws || ws_bytes < L.total)
    return fail(GP_ERR_WORKSPACE, "workspace of %zu bytes needed, %zu given", L.total,
                ws ? ws_bytes : (size_t)0);
  if (k->prec == GP_F64)
    return run_pcg<double>(k, n, X, theta, r, (const double *)B, ldb, (double *)x, ldx, col_shift,
                           rank, (const double *)U, lam, tol, maxit, status, iters, (char *)ws, L,
                           stream);
  return run_pcg<float>(k, n, X, theta, r, (const float *)B, ldb, (float *)x, ldx, col_shift, rank,
                        (const float *)U, lam, tol, maxit, status, iters, (char *)ws, L, stream);
}

}  // extern "C"
