// Gibbs refresh of phi: phi = A^{-1/2} xi (Section 3.1) through the pole expansion
//     A^{-1/2} ~ sum_p w_p (A + lambda_p I)^{-1}                       (eq. pex)
// with the weights and shifts of Appendix A (eq. msqdisc).
//
// Weights and shifts (host, double): elliptic.h, with the lower bound m = sigma^2 (every
// eigenvalue of A = sigma^2 I + K is at least the noise variance).
//
// Shifted solves.  All N_p systems (A + lambda_p I) x_p = xi share one Krylov space, so one
// conjugate-gradient iteration on A drives all of them (multi-shift CG): the shifted residuals
// stay collinear with the unshifted one, r_p = zeta_p r, and zeta_p, the shifted step lengths and
// directions follow from the unshifted CG scalars by a three-term recurrence.  Each iteration
// costs ONE product A p (for every right-hand side at once) plus streaming updates of the N_p
// shifted directions; phi = sum_p w_p x_p is accumulated directly, so the x_p are never stored.
// A shifted system is frozen once its residual |zeta_p| |r| falls below tol |xi|; the smallest
// shift is positive, so every shifted system converges no later than the unshifted one.
//
// The host replays a captured graph of a few iterations and checks for convergence after each
// replay (the call synchronises its stream).  Scalars are kept in double on the device; vectors are in the
// precision of the products (float for GP_F32 and GP_BF16X, double for GP_F64).
#include <math.h>
#include <string.h>

#include <vector>

#include "common.h"
#include "elliptic.h"
#include "gpk.h"
#include "vecops.h"

namespace gpk {

gp_status fail(gp_status st, const char *fmt, ...);
void clear_error();
gp_status hip_fail(hipError_t e, const char *where);

namespace {

constexpr int kPoleMax = 64;     // most poles per call
constexpr int kPhiMaxR = 32;     // most right-hand sides per call
constexpr int kCheckEvery = 4;   // host convergence check period, iterations
constexpr int kPcgBatch = 32;    // pole columns per preconditioned batch (gp_pcg_solve's limit)

// ---- device kernels ---------------------------------------------------------------------------

struct PoleCol {      // one right-hand side
  double rr;          // r . r of the unshifted residual
  double rr0;         // xi . xi
  double a;           // step length of the current iteration (0 once finished)
  double a_prev;      // step length of the previous iteration (1 before the first)
  double b_prev;      // direction coefficient of the previous iteration (0 before the first)
  double beta;        // direction coefficient of the current iteration
  int32_t done;
  int32_t iters;
  int32_t status;
  int32_t pad;
};

struct PoleShift {    // one (right-hand side, pole) pair
  double z_prev, z;   // zeta of the previous and current iteration
  double z_next;      // zeta of the next iteration, set by the step scalars
  double coefx;       // w_p * shifted step length: phi += coefx * p_p
  double zp, bp;      // this iteration's shifted direction is zp * r + bp * (previous one)
  int32_t act;
  int32_t pad;
};

// r = p = xi, phi = 0, partial sums of xi . xi.
template <typename T>
__global__ void __launch_bounds__(kThreads) phi_init(int64_t n, int r, VecGrid g, const T *xi,
                                                     int64_t ldxi, T *rv, T *pv, T *phi,
                                                     int64_t ldphi, double *part) {
  __shared__ double sh[kThreads];
  const int t = threadIdx.x;
  const int c = t % r, l = t / r;
  double acc = 0.0;
  if (l < g.rps) {
    const int64_t i1 = min(n, (int64_t)(blockIdx.x + 1) * g.rows_per_block);
    for (int64_t i = (int64_t)blockIdx.x * g.rows_per_block + l; i < i1; i += g.rps) {
      const T v = xi[i * ldxi + c];
      rv[i * r + c] = v;
      pv[i * r + c] = v;
      phi[i * ldphi + c] = (T)0;
      acc += (double)v * (double)v;
    }
  }
  block_column_sum(acc, sh, r, g.rps, part);
}

// Partial sums of p . q per column.
template <typename T>
__global__ void __launch_bounds__(kThreads) phi_dot(int64_t n, int r, VecGrid g, const T *pv,
                                                    const T *qv, double *part) {
  __shared__ double sh[kThreads];
  const int t = threadIdx.x;
  const int c = t % r, l = t / r;
  double acc = 0.0;
  if (l < g.rps) {
    const int64_t i1 = min(n, (int64_t)(blockIdx.x + 1) * g.rows_per_block);
    for (int64_t i = (int64_t)blockIdx.x * g.rows_per_block + l; i < i1; i += g.rps)
      acc += (double)pv[i * r + c] * (double)qv[i * r + c];
  }
  block_column_sum(acc, sh, r, g.rps, part);
}

// Column and shift states before the first iteration.
__global__ void phi_setup(int r, int np, int64_t blocks, const double *part, PoleCol *col,
                          PoleShift *sh, int32_t *remaining) {
  __shared__ double red[kThreads];
  __shared__ double tot[kPhiMaxR];
  __shared__ int32_t left;
  if (threadIdx.x == 0) left = 0;
  column_totals(part, blocks, r, red, tot);
  for (int c = 0; c < r; ++c) {
    const double rr0 = tot[c];
    if (threadIdx.x == 0) {
      PoleCol s;
      s.rr = rr0;
      s.rr0 = rr0;
      s.a = 0.0;
      s.a_prev = 1.0;
      s.b_prev = 0.0;
      s.beta = 0.0;
      s.iters = 0;
      s.pad = 0;
      s.status = isfinite(rr0) ? 0 : GP_PHI_NONFINITE;
      s.done = (rr0 == 0.0 || !isfinite(rr0)) ? 1 : 0;  // xi = 0: phi = 0
      left += 1 - s.done;
      col[c] = s;
    }
  }
  __syncthreads();
  for (int e = threadIdx.x; e < r * np; e += blockDim.x) {
    PoleShift s;
    s.z_prev = 1.0;
    s.z = 1.0;
    s.z_next = 1.0;
    s.coefx = 0.0;
    s.zp = 1.0;
    s.bp = 0.0;
    s.act = 1;
    s.pad = 0;
    sh[e] = s;
  }
  if (threadIdx.x == 0) *remaining = left;
}

// Step scalars: a = rr / (p . q), next zeta and shifted step lengths of every active pole.
__global__ void phi_scalars_a(int r, int np, int64_t blocks, const double *part,
                              const double *w, const double *lam, PoleCol *col, PoleShift *sh) {
  __shared__ double red[kThreads];
  __shared__ double a_sh[kPhiMaxR];
  __shared__ double tot[kPhiMaxR];
  column_totals(part, blocks, r, red, tot);
  for (int c = 0; c < r; ++c) {
    const double pq = tot[c];
    if (threadIdx.x == 0) {
      PoleCol s = col[c];
      double a = 0.0;
      if (!s.done) {
        a = s.rr / pq;
        if (!(isfinite(a) && a > 0.0)) {  // breakdown: A p . p not positive, or overflow
          s.status |= GP_PHI_NONFINITE;
          s.done = 1;
          a = 0.0;
        }
      }
      s.a = a;
      col[c] = s;
      a_sh[c] = a;
    }
  }
  __syncthreads();
  for (int e = threadIdx.x; e < r * np; e += blockDim.x) {
    const int c = e / np, p = e % np;
    PoleShift s = sh[e];
    const double a = a_sh[c];
    if (a == 0.0 || !s.act) {
      s.coefx = 0.0;
      s.act = a == 0.0 ? 0 : s.act;
    } else {
      const PoleCol cs = col[c];
      const double den = a * cs.b_prev * (s.z_prev - s.z) + s.z_prev * cs.a_prev * (1.0 + lam[p] * a);
      const double zn = s.z * s.z_prev * cs.a_prev / den;
      s.z_next = zn;
      s.coefx = w[p] * a * zn / s.z;
      if (!isfinite(s.coefx)) {  // zeta underflow: the shifted residual is far below any tol
        s.coefx = 0.0;
        s.act = 0;
      }
    }
    sh[e] = s;
  }
}

// One streaming pass: form this iteration's shifted directions, accumulate phi, update r, and
// the partial sums of the new r . r.
template <typename T>
__global__ void __launch_bounds__(kThreads) phi_update(int64_t n, int r, int np, VecGrid g,
                                                       const PoleCol *col, const PoleShift *shs,
                                                       T *ps, T *rv, const T *qv, T *phi,
                                                       int64_t ldphi, double *part) {
  __shared__ double sh[kThreads];
  extern __shared__ double coef[];  // [3][r * np] + [r]
  double *cz = coef, *cb = coef + r * np, *cx = coef + 2 * r * np, *ca = coef + 3 * r * np;
  for (int e = threadIdx.x; e < r * np; e += blockDim.x) {
    const PoleShift s = shs[e];
    // an inactive pole keeps its direction (zp = 0, bp = 1) and adds nothing
    cz[e] = s.act ? s.zp : 0.0;
    cb[e] = s.act ? s.bp : 1.0;
    cx[e] = s.act ? s.coefx : 0.0;
  }
  for (int c = threadIdx.x; c < r; c += blockDim.x) ca[c] = col[c].done ? 0.0 : col[c].a;
  __syncthreads();
  const int t = threadIdx.x;
  const int c = t % r, l = t / r;
  double acc = 0.0;
  if (l < g.rps && ca[c] != 0.0) {
    const double a = ca[c];
    const int64_t nr = n * r;
    const int64_t i1 = min(n, (int64_t)(blockIdx.x + 1) * g.rows_per_block);
    for (int64_t i = (int64_t)blockIdx.x * g.rows_per_block + l; i < i1; i += g.rps) {
      const int64_t e = i * r + c;
      const double ri = (double)rv[e];
      double ph = 0.0;
      for (int p = 0; p < np; ++p) {
        const double x = cx[c * np + p], zp = cz[c * np + p], bp = cb[c * np + p];
        if (zp == 0.0 && x == 0.0) continue;  // frozen pole: direction unchanged
        const double old = bp != 0.0 ? (double)ps[p * nr + e] : 0.0;
        const double dir = zp * ri + bp * old;
        const T dt = (T)dir;
        ps[p * nr + e] = dt;
        ph += x * (double)dt;
      }
      phi[i * ldphi + c] = (T)((double)phi[i * ldphi + c] + ph);
      const double rn = ri - a * (double)qv[e];
      const T rt = (T)rn;
      rv[e] = rt;
      acc += (double)rt * (double)rt;
    }
  }
  block_column_sum(acc, sh, r, g.rps, part);
}

// Direction scalars: beta = rr_new / rr, shifted direction coefficients, convergence of every
// pole and column.
__global__ void phi_scalars_b(int r, int np, int64_t blocks, const double *part, double tol,
                              PoleCol *col, PoleShift *sh, int32_t *remaining) {
  __shared__ double red[kThreads];
  __shared__ double rn_sh[kPhiMaxR];
  __shared__ int32_t alive[kPhiMaxR];
  __shared__ double tot[kPhiMaxR];
  column_totals(part, blocks, r, red, tot);
  for (int c = 0; c < r; ++c) {
    const double rn = tot[c];
    if (threadIdx.x == 0) {
      rn_sh[c] = rn;
      alive[c] = 0;
    }
  }
  __syncthreads();
  for (int e = threadIdx.x; e < r * np; e += blockDim.x) {
    const int c = e / np;
    const PoleCol cs = col[c];
    PoleShift s = sh[e];
    if (!cs.done && s.act) {
      const double rn = rn_sh[c];
      const double beta = rn / cs.rr;
      const double q = s.z_next / s.z;
      s.zp = s.z_next;
      s.bp = beta * q * q;
      s.z_prev = s.z;
      s.z = s.z_next;
      s.act = (fabs(s.z) * sqrt(rn) > tol * sqrt(cs.rr0)) ? 1 : 0;
      if (!isfinite(s.bp) || !isfinite(s.z)) s.act = 0;
      if (s.act) atomicOr(&alive[c], 1);
    }
    sh[e] = s;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    int32_t left = 0;
    for (int c = 0; c < r; ++c) {
      PoleCol s = col[c];
      if (!s.done) {
        const double rn = rn_sh[c];
        s.iters += 1;
        if (!isfinite(rn)) {
          s.status |= GP_PHI_NONFINITE;
          s.done = 1;
        } else {
          s.beta = rn / s.rr;
          s.a_prev = s.a;
          s.b_prev = s.beta;
          s.rr = rn;
          if (!alive[c]) s.done = 1;
        }
        col[c] = s;
      }
      left += 1 - s.done;
    }
    *remaining = left;
  }
}

// p = r + beta p for the columns still iterating.
template <typename T>
__global__ void __launch_bounds__(kThreads) phi_direction(int64_t n, int r, VecGrid g,
                                                          const PoleCol *col, const T *rv, T *pv) {
  const int t = threadIdx.x;
  const int c = t % r, l = t / r;
  if (l >= g.rps || col[c].done) return;
  const double beta = col[c].beta;
  const int64_t i1 = min(n, (int64_t)(blockIdx.x + 1) * g.rows_per_block);
  for (int64_t i = (int64_t)blockIdx.x * g.rows_per_block + l; i < i1; i += g.rps)
    pv[i * r + c] = (T)((double)rv[i * r + c] + beta * (double)pv[i * r + c]);
}

__global__ void phi_finish(int r, const PoleCol *col, int32_t *status, int32_t *iters) {
  const int c = threadIdx.x;
  if (c >= r) return;
  const PoleCol s = col[c];
  if (status) status[c] = s.status | (s.done ? 0 : GP_PHI_CG_MAXIT);
  if (iters) iters[c] = s.iters;
}

__global__ void phi_empty(int r, int32_t *status, int32_t *iters) {
  const int c = threadIdx.x;
  if (c >= r) return;
  if (status) status[c] = 0;
  if (iters) iters[c] = 0;
}

// Largest entry of a vector (the Gershgorin bound: A has positive entries, so its largest
// absolute row sum is max_i (A 1)_i).  part[b] per block, then one block.
template <typename T>
__global__ void __launch_bounds__(kThreads) row_max(int64_t n, const T *v, double *part) {
  __shared__ double red[kThreads];
  double m = -INFINITY;
  for (int64_t i = (int64_t)blockIdx.x * kThreads + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * kThreads) {
    const double x = (double)v[i];
    m = (x > m || x != x) ? x : m;  // a NaN propagates
  }
  red[threadIdx.x] = m;
  __syncthreads();
  for (int w = kThreads / 2; w >= 1; w >>= 1) {
    if (threadIdx.x < w) {
      const double o = red[threadIdx.x + w];
      if (o > red[threadIdx.x] || o != o) red[threadIdx.x] = o;
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) part[blockIdx.x] = red[0];
}

template <typename T>
__global__ void fill_value(T *a, int64_t m, T v) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e < m) a[e] = v;
}

// Preconditioned path: column c of xi replicated into the npc pole columns of b (n x npc).
template <typename T>
__global__ void phi_replicate(int64_t n, int npc, const T *xi, int64_t ldxi, int c, T *b) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e < n * npc) b[e] = xi[(e / npc) * ldxi + c];
}

// phi_ic (+)= sum_p w_p x_ip over one batch of pole columns (fixed order in p), in double.
template <typename T>
__global__ void phi_combine(int64_t n, int npc, const T *x, const double *w, T *phi, int64_t ldphi,
                            int c, int first) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  double s = first ? 0.0 : (double)phi[i * ldphi + c];
  for (int p = 0; p < npc; ++p) s += w[p] * (double)x[i * npc + p];
  phi[i * ldphi + c] = (T)s;
}

// Column status: the OR of the poles' bits (GP_CG_* and GP_PHI_* share their values), iterations
// the largest pole's.
__global__ void phi_pole_status(int npc, const int32_t *pst, const int32_t *pit, int32_t *status,
                                int32_t *iters, int c, int first) {
  if (threadIdx.x != 0) return;
  int32_t s = 0, it = 0;
  for (int p = 0; p < npc; ++p) {
    s |= pst[p];
    it = pit[p] > it ? pit[p] : it;
  }
  if (status) status[c] = first ? s : (status[c] | s);
  if (iters) iters[c] = first ? it : (iters[c] > it ? iters[c] : it);
}

// ---- workspace --------------------------------------------------------------------------------

struct PhiLayout {
  size_t prod;      // product workspace
  size_t prod_bytes;
  size_t ps;        // T [np][n][r] shifted directions
  size_t rv, pv, qv;  // T [n][r]
  size_t part;      // double [kVecBlocksMax][r]
  size_t col;       // PoleCol [r]
  size_t shift;     // PoleShift [r][np]
  size_t wl;        // double [2][np] weights, shifts
  size_t remaining; // int32
  // preconditioned path: PCG workspace, replicated right-hand side and solutions (T [n][npc]),
  // per-pole status and iterations
  size_t pcg = 0, pcg_bytes = 0, pb = 0, px = 0, pst = 0;
  size_t total;
};

PhiLayout phi_layout(const gp_kernel *k, int64_t n, int r, int np, int rank) {
  PhiLayout L;
  const size_t es = k->prec == GP_F64 ? 8 : 4;
  const size_t p1 = gp_workspace_size(k, n, 1), pr = gp_workspace_size(k, n, r);
  L.prod_bytes = p1 > pr ? p1 : pr;
  size_t o = 0;
  L.prod = o;
  o += align256(L.prod_bytes);
  if (rank > 0) {
    // preconditioned: one batch of pole columns at a time (no shifted directions kept)
    const int npc = np < kPcgBatch ? np : kPcgBatch;
    L.pcg_bytes = gp_pcg_workspace_size(k, n, npc, rank);
    L.pcg = o;
    o += align256(L.pcg_bytes);
    L.pb = o;
    o += align256(es * (size_t)n * npc);
    L.px = o;
    o += align256(es * (size_t)n * npc);
    L.pst = o;
    o += align256(2 * sizeof(int32_t) * kPcgBatch);
  }
  L.ps = o;
  o += rank > 0 ? 0 : align256(es * (size_t)np * n * r);
  L.rv = o;
  o += align256(es * (size_t)n * r);
  L.pv = o;
  o += align256(es * (size_t)n * r);
  L.qv = o;
  o += align256(es * (size_t)n * r);
  L.part = o;
  o += align256(sizeof(double) * kVecBlocksMax * (r > 1 ? r : 1));
  L.col = o;
  o += align256(sizeof(PoleCol) * r);
  L.shift = o;
  o += align256(sizeof(PoleShift) * r * np);
  L.wl = o;
  o += align256(sizeof(double) * 2 * np);
  L.remaining = o;
  o += 256;
  L.total = o;
  return L;
}

bool ranges_overlap(const void *a, int64_t rows, int64_t lda, int cols, const void *b,
                    int64_t ldb, size_t es) {
  const char *a0 = (const char *)a, *b0 = (const char *)b;
  const char *a1 = a0 + ((rows - 1) * lda + cols) * (int64_t)es;
  const char *b1 = b0 + ((rows - 1) * ldb + cols) * (int64_t)es;
  return a0 < b1 && b0 < a1;
}

template <typename T>
gp_status run_phi(const gp_kernel *k, const gp_phi_params *pp, int64_t n, const void *X,
                  const double *theta, int32_t r, const T *xi, int64_t ldxi, T *phi,
                  int64_t ldphi, int32_t *status, int32_t *iters, double *bounds, char *ws,
                  const PhiLayout &L, hipStream_t stream) {
  const int np = pp->n_poles;
  const int nth = gp_n_theta(k);
  // m = sigma^2 from theta
  double th[kMaxD + 2];
  hipError_t e = hipMemcpyAsync(th, theta, sizeof(double) * nth, hipMemcpyDeviceToHost, stream);
  if (e == hipSuccess) e = hipStreamSynchronize(stream);
  if (e != hipSuccess) return hip_fail(e, "reading theta");
  const double m = exp(th[nth - 1]);
  if (!(m > 0.0) || !isfinite(m)) return fail(GP_ERR_ARG, "sigma^2 = %g is not a positive number", m);

  char *prod = ws + L.prod;
  T *ps = (T *)(ws + L.ps);
  T *rv = (T *)(ws + L.rv);
  T *pv = (T *)(ws + L.pv);
  T *qv = (T *)(ws + L.qv);
  double *part = (double *)(ws + L.part);
  PoleCol *col = (PoleCol *)(ws + L.col);
  PoleShift *shf = (PoleShift *)(ws + L.shift);
  double *wl = (double *)(ws + L.wl);
  int32_t *remaining = (int32_t *)(ws + L.remaining);

  // M: given, or the Gershgorin bound max_i (A 1)_i, widened by a few rounding units of the
  // product so that it stays an upper bound
  double M = pp->lambda_max;
  if (!(M > 0.0)) {
    fill_value<T><<<(unsigned)((n + 255) / 256), 256, 0, stream>>>(pv, n, (T)1);
    e = hipGetLastError();
    if (e != hipSuccess) return hip_fail(e, "Gershgorin ones");
    gp_status st = gp_kmatvec(k, n, X, theta, 1, pv, 1, nullptr, qv, 1, prod, L.prod_bytes, stream);
    if (st) return st;
    const int mb = (int)((n + kThreads - 1) / kThreads < 1024 ? (n + kThreads - 1) / kThreads : 1024);
    row_max<T><<<mb, kThreads, 0, stream>>>(n, qv, part);
    row_max<double><<<1, kThreads, 0, stream>>>(mb, part, part + kVecBlocksMax - 1);
    e = hipGetLastError();
    if (e == hipSuccess)
      e = hipMemcpyAsync(&M, part + kVecBlocksMax - 1, sizeof(double), hipMemcpyDeviceToHost, stream);
    if (e == hipSuccess) e = hipStreamSynchronize(stream);
    if (e != hipSuccess) return hip_fail(e, "Gershgorin bound");
    const double widen = k->prec == GP_F64 ? 1e-12 : (k->prec == GP_F32 ? 1e-5 : 1e-3);
    M *= 1.0 + widen;
    if (!isfinite(M)) return fail(GP_ERR_ARG, "the Gershgorin bound is not finite");
  }
  if (M < m) M = m;  // A = sigma^2 I (no kernel mass): a single-point spectrum
  std::vector<double> hw(2 * np);
  gp_status st = gp_pole_weights(m, M, np, hw.data(), hw.data() + np);
  if (st) return st;
  if (bounds) {
    bounds[0] = m;
    bounds[1] = M;
  }
  e = hipMemcpyAsync(wl, hw.data(), sizeof(double) * 2 * np, hipMemcpyHostToDevice, stream);
  if (e != hipSuccess) return hip_fail(e, "uploading the pole weights");

  if (pp->precond_rank > 0) {
    // Nystrom-preconditioned CG for the shifted systems of each column, then phi = sum_p w_p x_p
    const int rank = pp->precond_rank;
    T *pb = (T *)(ws + L.pb), *px = (T *)(ws + L.px);
    int32_t *pst = (int32_t *)(ws + L.pst), *pit = pst + kPcgBatch;
    const double *w_dev = wl, *shift_dev = wl + np;
    const int nb = np < kPcgBatch ? np : kPcgBatch;  // width of the replicated right-hand side
    for (int c = 0; c < r; ++c) {
      // xi's column is read once, before any batch writes phi (which may be xi itself)
      phi_replicate<T><<<(unsigned)((n * nb + 255) / 256), 256, 0, stream>>>(n, nb, xi, ldxi, c, pb);
      for (int p0 = 0; p0 < np; p0 += kPcgBatch) {
        const int npc = np - p0 < kPcgBatch ? np - p0 : kPcgBatch;
        const unsigned eb = (unsigned)((n * npc + 255) / 256);
        fill_value<T><<<eb, 256, 0, stream>>>(px, n * npc, (T)0);
        e = hipGetLastError();
        if (e != hipSuccess) return hip_fail(e, "preconditioned phi set-up");
        st = gp_pcg_solve(k, n, X, theta, npc, pb, nb, px, npc, shift_dev + p0, rank,
                          pp->precond_U, pp->precond_lam, pp->tol, pp->maxit, pst, pit,
                          ws + L.pcg, L.pcg_bytes, stream);
        if (st) return st;
        phi_combine<T><<<(unsigned)((n + 255) / 256), 256, 0, stream>>>(n, npc, px, w_dev + p0, phi,
                                                                       ldphi, c, p0 == 0);
        phi_pole_status<<<1, 64, 0, stream>>>(npc, pst, pit, status, iters, c, p0 == 0);
        e = hipGetLastError();
        if (e != hipSuccess) return hip_fail(e, "preconditioned phi combine");
      }
    }
    e = hipStreamSynchronize(stream);
    return e == hipSuccess ? GP_OK : hip_fail(e, "phi finish");
  }

  const VecGrid g = vec_grid(n, r);
  const unsigned vb = (unsigned)g.blocks;
  phi_init<T><<<vb, kThreads, 0, stream>>>(n, r, g, xi, ldxi, rv, pv, phi, ldphi, part);
  phi_setup<<<1, kThreads, 0, stream>>>(r, np, g.blocks, part, col, shf, remaining);
  e = hipGetLastError();
  if (e != hipSuccess) return hip_fail(e, "phi set-up");
  // one iteration: the same launches every time (finished columns skip their updates), so
  // kCheckEvery of them are captured once as a graph and replayed between convergence checks;
  // the iterations past the last whole group run eagerly, so no more than maxit are taken
  auto iteration = [&](hipStream_t q) -> gp_status {
    gp_status r2 = gp_kmatvec(k, n, X, theta, r, pv, r, nullptr, qv, r, prod, L.prod_bytes, q);
    if (r2) return r2;
    phi_dot<T><<<vb, kThreads, 0, q>>>(n, r, g, pv, qv, part);
    phi_scalars_a<<<1, kThreads, 0, q>>>(r, np, g.blocks, part, wl, wl + np, col, shf);
    phi_update<T><<<vb, kThreads, sizeof(double) * (3 * r * np + r), q>>>(n, r, np, g, col, shf, ps, rv, qv, phi, ldphi, part);
    phi_scalars_b<<<1, kThreads, 0, q>>>(r, np, g.blocks, part, pp->tol, col, shf, remaining);
    phi_direction<T><<<vb, kThreads, 0, q>>>(n, r, g, col, rv, pv);
    const hipError_t he = hipGetLastError();
    return he == hipSuccess ? GP_OK : hip_fail(he, "multi-shift CG iteration");
  };
  hipGraphExec_t exec = nullptr;
  if (pp->maxit >= kCheckEvery) {
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
    if (e != hipSuccess) return hip_fail(e, "multi-shift CG graph");
  }
  for (int it = 0; it < pp->maxit;) {
    int32_t left = 0;
    e = hipMemcpyAsync(&left, remaining, sizeof(int32_t), hipMemcpyDeviceToHost, stream);
    if (e == hipSuccess) e = hipStreamSynchronize(stream);
    if (e != hipSuccess) break;
    if (left == 0) break;
    if (exec && pp->maxit - it >= kCheckEvery) {
      e = hipGraphLaunch(exec, stream);
      if (e != hipSuccess) break;
      it += kCheckEvery;
    } else {
      st = iteration(stream);
      if (st) break;
      ++it;
    }
  }
  if (exec) (void)hipGraphExecDestroy(exec);
  if (st) return st;
  if (e != hipSuccess) return hip_fail(e, "multi-shift CG");
  phi_finish<<<1, 64, 0, stream>>>(r, col, status, iters);
  e = hipGetLastError();
  if (e == hipSuccess) e = hipStreamSynchronize(stream);
  if (e != hipSuccess) return hip_fail(e, "phi finish");
  return GP_OK;
}

gp_status check_phi(const gp_kernel *k, const gp_phi_params *p, int64_t n, int32_t r) {
  if (!k || !p) return fail(GP_ERR_ARG, "kernel description or parameters are NULL");
  if (gp_n_theta(k) < 0) return fail(GP_ERR_ARG, "invalid kernel description");
  if (k->flags & GP_NO_NOISE) return fail(GP_ERR_ARG, "GP_NO_NOISE: A has no positive lower bound");
  if (n < 0) return fail(GP_ERR_SHAPE, "n = %lld < 0", (long long)n);
  if (r < 1 || r > kPhiMaxR) return fail(GP_ERR_SHAPE, "r = %d outside 1..%d", r, kPhiMaxR);
  if (p->n_poles < 1 || p->n_poles > kPoleMax)
    return fail(GP_ERR_ARG, "n_poles = %d outside 1..%d", p->n_poles, kPoleMax);
  if (!(p->tol > 0.0)) return fail(GP_ERR_ARG, "tol must be > 0");
  if (p->maxit < 1) return fail(GP_ERR_ARG, "maxit must be >= 1");
  if (!(p->lambda_max <= 0.0 || isfinite(p->lambda_max)))
    return fail(GP_ERR_ARG, "lambda_max must be finite");
  if (p->precond_rank < 0 || p->precond_rank > 512 || (n > 0 && p->precond_rank > n))
    return fail(GP_ERR_SHAPE, "precond_rank = %d outside 0..min(n, 512)", p->precond_rank);
  if (p->precond_rank > 0 && (!p->precond_U || !p->precond_lam))
    return fail(GP_ERR_ARG, "precond_rank > 0 needs precond_U and precond_lam");
  return GP_OK;
}

}  // namespace
}  // namespace gpk

using namespace gpk;

extern "C" {

gp_status gp_pole_weights(double m, double M, int32_t n_poles, double *w, double *shift) {
  clear_error();
  if (!w || !shift) return fail(GP_ERR_ARG, "w and shift must be non-NULL");
  if (n_poles < 1) return fail(GP_ERR_ARG, "n_poles = %d < 1", n_poles);
  if (!(m > 0.0) || !(M >= m) || !isfinite(M))
    return fail(GP_ERR_ARG, "need 0 < m <= M < inf (m = %g, M = %g)", m, M);
  const double k = sqrt(m / M);
  const double kp = ellk_complement(k);
  double sa[kAgmMax], sc[kAgmMax];
  const int ns = agm_scale(k, sa, sc);
  for (int j = 0; j < n_poles; ++j) pole_node(m, M, n_poles, j, k, kp, sa, sc, ns, w + j, shift + j);
  return GP_OK;
}

size_t gp_phi_workspace_size(const gp_kernel *k, const gp_phi_params *p, int64_t n, int32_t r) {
  if (check_phi(k, p, n, r) != GP_OK || n == 0) return 0;  // n = 0 needs no workspace
  return phi_layout(k, n, r, p->n_poles, p->precond_rank).total;
}

gp_status gp_phi_refresh(const gp_kernel *k, const gp_phi_params *p, int64_t n, const void *X,
                         const double *theta, int32_t r, const void *xi, int64_t ldxi, void *phi,
                         int64_t ldphi, int32_t *status, int32_t *iters, double *bounds, void *ws,
                         size_t ws_bytes, hipStream_t stream) {
  clear_error();
  gp_status st = check_phi(k, p, n, r);
  if (st) return st;
  if (n > 0 && (!X || !theta || !xi || !phi)) return fail(GP_ERR_ARG, "X, theta, xi and phi must be non-NULL");
  if (n > 0 && (ldxi < r || ldphi < r))
    return fail(GP_ERR_SHAPE, "leading dimensions ldxi=%lld ldphi=%lld must be >= r=%d",
                (long long)ldxi, (long long)ldphi, r);
  const size_t es = k->prec == GP_F64 ? 8 : 4;
  if (n > 0 && !(xi == phi && ldxi == ldphi) && ranges_overlap(xi, n, ldxi, r, phi, ldphi, es))
    return fail(GP_ERR_ARG, "phi overlaps xi (only phi == xi with equal leading dimensions is allowed)");
  if (n > 0 && ranges_overlap(X, n, k->d, k->d, phi, ldphi, es)) return fail(GP_ERR_ARG, "phi overlaps X");
  const PhiLayout L = phi_layout(k, n, r, p->n_poles, p->precond_rank);
  if (n == 0) {  // nothing to solve: every column converged in 0 iterations
    phi_empty<<<1, 64, 0, stream>>>(r, status, iters);
    hipError_t e = hipGetLastError();
    if (e == hipSuccess) e = hipStreamSynchronize(stream);
    return e == hipSuccess ? GP_OK : hip_fail(e, "phi (n = 0)");
  }
  if (!ws || ws_bytes < L.total)
    return fail(GP_ERR_WORKSPACE, "workspace of %zu bytes needed, %zu given", L.total,
                ws ? ws_bytes : (size_t)0);
  if (k->prec == GP_F64)
    return run_phi<double>(k, p, n, X, theta, r, (const double *)xi, ldxi, (double *)phi, ldphi,
                           status, iters, bounds, (char *)ws, L, stream);
  return run_phi<float>(k, p, n, X, theta, r, (const float *)xi, ldxi, (float *)phi, ldphi, status,
                        iters, bounds, (char *)ws, L, stream);
}

}  // extern "C"
