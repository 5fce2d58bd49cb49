// HMC trajectory with the implicit midpoint integrator (Section 3.2.3) solved by Anderson-
// accelerated fixed-point iteration (Appendix B).
//
// One step solves eq. (implicitsystem) for (theta_1, pi_1, x) as the fixed point of eq. (Phi):
//     Phi(theta, pi, x) = ( theta_0 + dt (pi_0 + pi) / 2,
//                           pi_0 - dt F(m, x),                 m = (theta_0 + theta) / 2
//                           x + R (y - A(m) x) ),               R = I / c,  c ~ rho(A(theta_0))
// where F(m, x) is the frozen-x force of Section 3.2.1.  F(m, x) and A(m) x come from ONE fused
// quadratic-form pass over [x | phi] at m (gp_quadform_grad, w = (-1/2, +1/2)).  The unknowns are
// stacked into one vector v = (theta, pi, x); Anderson acceleration with history k keeps the
// last k pairs (f_i = Phi(v_i) - v_i, g_i = Phi(v_i)) and sets v = sum_i alpha_i g_i with
// alpha minimising |sum_i alpha_i f_i| subject to sum_i alpha_i = 1 (k = 0: plain Picard
// iteration).  Everything of an iteration runs on the device: the (theta, pi) parts and the
// history's Gram matrix in double in a small state block, the convergence test, the
// least-squares weights and the combination in one single-workgroup kernel (imp_update), the x
// parts in the streaming kernels below.  Every iteration enqueues the same launches, so kCheck
// of them are captured once per trajectory as a graph, which the host replays, reading the
// state's convergence flag after each replay (iterations after convergence change nothing).  c comes from power iterations
// on A(theta_0) (ten in the paper); with a Nystrom factor R = P^{-1} / c, P the preconditioner of
// A(theta_0) and c ~ rho(P^{-1} A(theta_0)).  The trajectory ends with a solve at theta_1 for the energy,
// as for the leapfrog integrator, and the Metropolis decision of Algorithm 1.
#include <math.h>

#include <algorithm>
#include <vector>

#include "common.h"
#include "gpk.h"
#include "nystrom.h"

namespace gpk {

gp_status fail(gp_status st, const char *fmt, ...);
void clear_error();
gp_status hip_fail(hipError_t e, const char *where);

namespace {

constexpr int kHistMax = 20;
constexpr int kCheck = 4;          // fixed-point iterations between host convergence checks
constexpr int kTh = kMaxD + 4;     // stride of the theta / pi parts of the device state
constexpr size_t kImpDoubles = 4 * kTh + 2 * (size_t)kHistMax * 2 * kTh + (size_t)kHistMax * kHistMax;
constexpr int kDotBlocks = 512;
// Transfer block of a fixed-point iteration: the force pass's gradient, the block partials of
// |y - A(m) x|^2 and those of the new Gram row, fetched to the host together.
constexpr int kXfGrad = 0;
constexpr int kXfRes = kMaxD + 4;
constexpr int kXfRow = kXfRes + kDotBlocks;
constexpr int kXfDoubles = kXfRow + kDotBlocks * kHistMax;

// out[b][j] = partial sums over this block's rows of a[i] * H[j][i] for j < m (H rows of length n)
template <typename T>
__device__ void multi_dot_body(int64_t n, int m, const T *a, const T *H, int64_t ldh, double *out);

template <typename T>
__global__ __launch_bounds__(256) void multi_dot(int64_t n, int m, const T *a, const T *H,
                                                 int64_t ldh, double *out) {
  multi_dot_body<T>(n, m, a, H, ldh, out);
}

// The Gram row of the fixed-point iteration: m = min(it + 1, kh) rows, it = flags[4] the
// iteration's index within its step.
template <typename T>
__global__ __launch_bounds__(256) void multi_dot_hist(int64_t n, const int32_t *flags, int kh,
                                                      const T *a, const T *H, int64_t ldh,
                                                      double *out) {
  multi_dot_body<T>(n, min(flags[4] + 1, kh), a, H, ldh, out);
}

template <typename T>
__device__ void multi_dot_body(int64_t n, int m, const T *a, const T *H, int64_t ldh, double *out) {
  __shared__ double sh[4][kHistMax + 1];
  double acc[kHistMax + 1];
  for (int j = 0; j < m; ++j) acc[j] = 0.0;
  for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (int64_t)gridDim.x * 256) {
    const double ai = (double)a[i];
    for (int j = 0; j < m; ++j) acc[j] += ai * (double)H[(int64_t)j * ldh + i];
  }
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  for (int j = 0; j < m; ++j) {
    const double v = wave_sum(acc[j]);
    if (lane == 0) sh[wave][j] = v;
  }
  __syncthreads();
  for (int j = threadIdx.x; j < m; j += 256)
    out[(int64_t)blockIdx.x * m + j] = (sh[0][j] + sh[1][j]) + (sh[2][j] + sh[3][j]);
}

// Z = [x | phi] (n x 2)
template <typename T>
__global__ void pack_z(int64_t n, const T *x, const T *phi, T *Z) {
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (i >= n) return;
  Z[2 * i] = x[i];
  Z[2 * i + 1] = phi[i];
}

// res = y - A x with A x = AZ[:, 0]
template <typename T>
__global__ void linear_residual(int64_t n, const T *y, const T *AZ, T *res) {
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (i < n) res[i] = (T)((double)y[i] - (double)AZ[2 * i]);
}

// fx = src / c (src = the residual, preconditioned or not), gx = x + fx
template <typename T>
__global__ void fixed_point_x(int64_t n, const T *src, const T *x, double inv_c, T *fx, T *gx) {
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (i >= n) return;
  const double f = (double)src[i] * inv_c;
  fx[i] = (T)f;
  gx[i] = (T)((double)x[i] + f);
}

template <typename T>
__global__ void scale_copy(int64_t n, const T *a, double s, T *b) {
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (i < n) b[i] = (T)((double)a[i] * s);
}

struct ImpLayout {
  size_t qf, qf_bytes, pcg, pcg_bytes, Z, AZ, x, v, rb, fx, gx, Fh, Gh, part, alpha, grad, th0,
      xf, wts, nys, ist, iflags, total;
};

ImpLayout imp_layout(const gp_kernel *k, int64_t n, int hist, int rank) {
  ImpLayout L;
  const size_t es = k->prec == GP_F64 ? 8 : 4;
  const int hs = hist > 0 ? hist : 1;
  size_t o = 0;
  L.qf = o;
  L.qf_bytes = std::max(gp_workspace_size(k, n, 2), gp_workspace_size(k, n, 1));
  o += align256(L.qf_bytes);
  L.pcg = o;
  L.pcg_bytes = gp_pcg_workspace_size(k, n, 1, rank);
  o += align256(L.pcg_bytes);
  L.Z = o;
  o += align256(es * 2 * n);
  L.AZ = o;
  o += align256(es * 2 * n);
  L.x = o;
  o += align256(es * n);
  L.v = o;
  o += align256(es * n);
  L.rb = o;
  o += align256(es * n);
  L.fx = o;
  o += align256(es * n);
  L.gx = o;
  o += align256(es * n);
  L.Fh = o;
  o += align256(es * n * hs);
  L.Gh = o;
  o += align256(es * n * hs);
  L.part = o;
  o += align256(sizeof(double) * kDotBlocks * (kHistMax + 1));
  L.alpha = o;
  o += align256(sizeof(double) * (kHistMax + 1));
  L.grad = o;
  o += align256(sizeof(double) * (kMaxD + 4 + 2 + 8));
  L.th0 = o;
  o += align256(sizeof(double) * (kMaxD + 4));
  L.xf = o;  // a fixed-point iteration's force, residual and Gram-row partials (kXf* offsets)
  o += align256(sizeof(double) * kXfDoubles);
  L.wts = o;
  o += align256(sizeof(double) * 2);
  L.nys = o;
  o += align256(rank > 0 ? nystrom_apply_scratch(n, rank, 1) : 0);
  L.ist = o;
  o += align256(sizeof(double) * kImpDoubles);
  L.iflags = o;
  o += align256(sizeof(int32_t) * 8);
  L.total = o;
  return L;
}

// Device state of the fixed-point iteration (double): the step's start (ths, pis), the current
// iterate (th, pi), the parameter parts of the history's f and g ([kHistMax][2 kTh]) and its
// Gram matrix ([kHistMax][kHistMax]); flags: [0] converged, [1] status bits, [2] iterations
// taken, [3] the x update of the iteration (0 none, 1 Anderson combination, 2 x = g), [4] the
// iteration's index within its step (the history holds min(it + 1, k) pairs, the newest in slot
// it mod k), so that every iteration enqueues the same launches.
struct ImpDev {
  double *ths, *pis, *th, *pi, *hf, *hg, *G;
  int32_t *flags;
};

// Minimise |sum alpha_i f_i|^2 subject to sum alpha_i = 1 from the Gram matrix a (LDS, m x m,
// row stride kHistMax, overwritten): alpha = G^{-1} 1 / (1^T G^{-1} 1), with a small ridge for a
// near-singular history; Gaussian elimination with partial pivoting (the pivot search and the
// back substitution by lane 0, the row updates one row per lane).  A degenerate history gives
// the plain fixed-point step (alpha = e_m).  One wave; b, z and alpha in LDS (kHistMax each).
__device__ void anderson_weights(double *a, int m, double *b, double *z, double *alpha) {
  const int t = threadIdx.x;
  __shared__ int s_piv;
  __shared__ double s_tr;
  if (t == 0) {
    double tr = 0.0;
    for (int i = 0; i < m; ++i) tr += a[i * kHistMax + i];
    s_tr = tr;
  }
  __syncthreads();
  if (t < m) {
    a[t * kHistMax + t] += 1e-12 * s_tr / m;
    b[t] = 1.0;
  }
  __syncthreads();
  for (int c = 0; c < m; ++c) {
    if (t == 0) {
      int p = c;
      for (int r = c + 1; r < m; ++r)
        if (fabs(a[r * kHistMax + c]) > fabs(a[p * kHistMax + c])) p = r;
      s_piv = p;
    }
    __syncthreads();
    const int p = s_piv;
    if (p != c) {
      if (t < m) {
        const double u = a[c * kHistMax + t];
        a[c * kHistMax + t] = a[p * kHistMax + t];
        a[p * kHistMax + t] = u;
      }
      if (t == 0) {
        const double u = b[c];
        b[c] = b[p];
        b[p] = u;
      }
    }
    __syncthreads();
    const double d = a[c * kHistMax + c];
    if (fabs(d) >= 1e-300 && t > c && t < m) {
      const double f = a[t * kHistMax + c] / d;
      for (int j = c; j < m; ++j) a[t * kHistMax + j] -= f * a[c * kHistMax + j];
      b[t] -= f * b[c];
    }
    __syncthreads();
  }
  if (t == 0) {
    for (int r = m - 1; r >= 0; --r) {
      double u = b[r];
      for (int j = r + 1; j < m; ++j) u -= a[r * kHistMax + j] * z[j];
      const double d = a[r * kHistMax + r];
      z[r] = fabs(d) < 1e-300 ? 0.0 : u / d;
    }
    double sum = 0.0;
    for (int i = 0; i < m; ++i) sum += z[i];
    const bool degenerate = !(fabs(sum) > 0.0) || !isfinite(sum);
    for (int i = 0; i < m; ++i) alpha[i] = degenerate ? (i == m - 1 ? 1.0 : 0.0) : z[i] / sum;
  }
  __syncthreads();
}

// Start of a step: (ths, pis) = (th, pi), nothing converged yet.
__global__ void imp_begin_step(ImpDev s, int nth) {
  if (threadIdx.x != 0) return;
  for (int k = 0; k < nth; ++k) {
    s.ths[k] = s.th[k];
    s.pis[k] = s.pi[k];
  }
  s.flags[0] = 0;
  s.flags[3] = 0;
  s.flags[4] = 0;
}

// (f, g) of x into the history slot of this iteration.
template <typename T>
__global__ void hist_store(int64_t n, const int32_t *flags, int kh, const T *fx, const T *gx, T *Fh,
                           T *Gh) {
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (i >= n) return;
  const int64_t o = (int64_t)(flags[4] % kh) * n + i;
  Fh[o] = fx[i];
  Gh[o] = gx[i];
}

// The midpoint (theta_0 + theta) / 2 at which the iteration's force pass runs.
__global__ void imp_midpoint(ImpDev s, int nth, double *mid) {
  const int k = threadIdx.x;
  if (s.flags[0] || s.flags[1] || k >= nth) return;
  mid[k] = 0.5 * (s.ths[k] + s.th[k]);
}

__device__ __forceinline__ double wave_max(double v) {
  for (int o = 32; o >= 1; o >>= 1) v = fmax(v, __shfl_xor(v, o, 64));
  return v;
}

// One fixed-point iteration's bookkeeping, one wave of 64 lanes working in LDS: g = Phi(v) and
// f = g - v for the parameter parts from the force F (one component per lane), the convergence
// test on f and on |y - A(m) x| (the block partials of its square), then the next iterate: g
// (Picard, or the converged iteration's map value) or the Anderson combination over the last
// m_new pairs (slot `head` just written; the x parts' Gram row arrives as block partials).
__global__ __launch_bounds__(64) void imp_update(ImpDev s, int nth, double dt, double tol,
                                                 double ynorm, int kh, int maxit, int nb,
                                                 const double *F, const double *res_part,
                                                 const double *row_part, double *alpha_d) {
  __shared__ double gtp[2 * kTh], ftp[2 * kTh];
  __shared__ double a[kHistMax * kHistMax], b[kHistMax], z[kHistMax], alpha[kHistMax];
  const int t = threadIdx.x;
  const int it = s.flags[4];
  __syncthreads();  // every lane has read the index before lane 0 advances it
  if (t == 0) s.flags[4] = it + 1;
  // converged, failed or past the iteration limit: iterations after it change nothing
  if (s.flags[0] || s.flags[1] || it >= maxit) {
    if (t == 0) s.flags[3] = 0;
    return;
  }
  const int m_new = kh > 0 ? min(it + 1, kh) : 0, head = kh > 0 ? it % kh : 0;
  double fm = 0.0, vm = 0.0;
  for (int k = t; k < nth; k += 64) {
    const double th = s.th[k], pi = s.pi[k], ths = s.ths[k], pis = s.pis[k];
    const double g0 = ths + dt * 0.5 * (pis + pi), g1 = pis - dt * F[k];
    gtp[k] = g0;
    gtp[nth + k] = g1;
    ftp[k] = g0 - th;
    ftp[nth + k] = g1 - pi;
    const double af = fmax(fabs(g0 - th), fabs(g1 - pi)), av = fmax(fabs(th), fabs(pi));
    fm = (af > fm || af != af) ? af : fm;  // a NaN propagates
    vm = fmax(vm, av);
  }
  fm = wave_max(fm);
  vm = wave_max(vm);
  double rr2 = 0.0;
  for (int q = t; q < nb; q += 64) rr2 += res_part[q];
  rr2 = wave_sum(rr2);
  __syncthreads();
  if (!isfinite(fm)) {
    if (t == 0) {
      s.flags[1] |= GP_CHAIN_NONFINITE_THETA;
      s.flags[3] = 0;
      s.flags[2] += 1;
    }
    return;
  }
  const bool conv = fm <= tol * (1.0 + vm) && sqrt(rr2) <= tol * ynorm;
  if (conv || kh == 0) {
    for (int k = t; k < nth; k += 64) {
      s.th[k] = gtp[k];
      s.pi[k] = gtp[nth + k];
    }
    if (t == 0) {
      s.flags[0] = conv ? 1 : 0;
      s.flags[3] = conv ? 0 : 2;
      s.flags[2] += 1;
    }
    return;
  }
  const int w = 2 * kTh;
  double *hfh = s.hf + head * w;
  for (int k = t; k < 2 * nth; k += 64) {
    hfh[k] = ftp[k];
    s.hg[head * w + k] = gtp[k];
  }
  // the new Gram row, entry j < m_new: the row blocks' x-part partials plus the parameter
  // parts' product, spread over the lanes (every lane's loads in flight together), each entry
  // then summed by the butterfly (fixed order)
  double u[kHistMax];
#pragma unroll
  for (int j = 0; j < kHistMax; ++j) u[j] = 0.0;
  for (int q = t; q < nb; q += 64) {
#pragma unroll
    for (int j = 0; j < kHistMax; ++j)
      if (j < m_new) u[j] += row_part[q * m_new + j];
  }
  for (int k = t; k < 2 * nth; k += 64) {
    const double fk = ftp[k];
#pragma unroll
    for (int j = 0; j < kHistMax; ++j)
      if (j < m_new) u[j] += fk * (j == head ? fk : s.hf[j * w + k]);
  }
#pragma unroll
  for (int j = 0; j < kHistMax; ++j) {
    if (j < m_new) {
      const double v = wave_sum(u[j]);
      if (t == 0) {
        s.G[head * kHistMax + j] = v;
        s.G[j * kHistMax + head] = v;
      }
    }
  }
  __threadfence_block();
  __syncthreads();
  for (int e = t; e < m_new * m_new; e += 64) {
    const int i = e / m_new, j = e % m_new;
    a[i * kHistMax + j] = s.G[i * kHistMax + j];
  }
  __syncthreads();
  anderson_weights(a, m_new, b, z, alpha);
  for (int k = t; k < nth; k += 64) {
    double u = 0.0, v = 0.0;
    for (int j = 0; j < m_new; ++j) {
      u += alpha[j] * s.hg[j * w + k];
      v += alpha[j] * s.hg[j * w + nth + k];
    }
    s.th[k] = u;
    s.pi[k] = v;
  }
  if (t < m_new) alpha_d[t] = alpha[t];
  if (t == 0) {
    s.flags[3] = 1;
    s.flags[2] += 1;
  }
}

// x = sum_j alpha_j G[j] (Anderson, over the min(it + 1, kh) pairs of the iteration just
// taken), x = g (Picard), or unchanged, as imp_update decided.
template <typename T>
__global__ void imp_x_update(int64_t n, int kh, const int32_t *flags, const double *alpha,
                             const T *G, int64_t ldg, const T *gx, T *x) {
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  const int mode = flags[3];
  const int m = min(flags[4], kh);  // imp_update has advanced the index past this iteration
  if (i >= n || mode == 0) return;
  if (mode == 2) {
    x[i] = gx[i];
    return;
  }
  double t = 0.0;
  for (int j = 0; j < m; ++j) t += alpha[j] * (double)G[(int64_t)j * ldg + i];
  x[i] = (T)t;
}

template <typename T>
struct Ctx {
  const gp_kernel *k;
  const gp_implicit_params *p;
  int64_t n;
  int nth;
  const void *X;
  const T *y, *phi;
  int rank;
  const void *U;
  const double *lam;
  char *w;
  ImpLayout L;
  hipStream_t s;
  double *thd;  // device theta used for the passes (the caller's theta array)
};

template <typename T>
gp_status h2d(double *d, const double *h, int m, hipStream_t s) {
  hipError_t e = hipMemcpyAsync(d, h, sizeof(double) * m, hipMemcpyHostToDevice, s);
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  return e == hipSuccess ? GP_OK : hip_fail(e, "host -> device");
}

gp_status d2h(double *h, const double *d, int m, hipStream_t s) {
  hipError_t e = hipMemcpyAsync(h, d, sizeof(double) * m, hipMemcpyDeviceToHost, s);
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  return e == hipSuccess ? GP_OK : hip_fail(e, "device -> host");
}

// sum_i a_i H[j][i] for j < m, on the host in double (fixed order over blocks)
template <typename T>
gp_status dots(const Ctx<T> &c, const T *a, const T *H, int64_t ldh, int m, double *out) {
  const int nb = (int)std::min<int64_t>(kDotBlocks, (c.n + 255) / 256);
  double *part = (double *)(c.w + c.L.part);
  multi_dot<T><<<nb, 256, 0, c.s>>>(c.n, m, a, H, ldh, part);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return hip_fail(e, "dots");
  std::vector<double> h((size_t)nb * m);
  gp_status st = d2h(h.data(), part, nb * m, c.s);
  if (st) return st;
  for (int j = 0; j < m; ++j) {
    double t = 0.0;
    for (int b = 0; b < nb; ++b) t += h[(size_t)b * m + j];
    out[j] = t;
  }
  return GP_OK;
}

// Energy H = 1/2 (2 y.x - x^T A x) + 1/2 phi^T A phi + 1/2 pi.pi at theta (on the device array
// c.thd), with x solved there by (preconditioned) CG from the warm start x.
template <typename T>
gp_status energy(const Ctx<T> &c, const std::vector<double> &theta, const std::vector<double> &pi,
                 T *x, double *H, int32_t *cg_status, int32_t *cg_iters) {
  gp_status st = h2d<T>(c.thd, theta.data(), c.nth, c.s);
  if (st) return st;
  int32_t *sd = (int32_t *)(c.w + c.L.grad + sizeof(double) * (kMaxD + 4 + 2));
  st = gp_pcg_solve(c.k, c.n, c.X, c.thd, 1, c.y, 1, x, 1, nullptr, c.rank, c.U, c.lam, c.p->cg_tol,
                    c.p->cg_maxit, sd, sd + 1, c.w + c.L.pcg, c.L.pcg_bytes, c.s);
  if (st) return st;
  int32_t hs[2];
  hipError_t e = hipMemcpyAsync(hs, sd, sizeof(hs), hipMemcpyDeviceToHost, c.s);
  if (e == hipSuccess) e = hipStreamSynchronize(c.s);
  if (e != hipSuccess) return hip_fail(e, "solve status");
  *cg_status = hs[0];
  *cg_iters = hs[1];
  T *Z = (T *)(c.w + c.L.Z);
  pack_z<T><<<(unsigned)((c.n + 255) / 256), 256, 0, c.s>>>(c.n, x, c.phi, Z);
  double *q = (double *)(c.w + c.L.grad);
  st = gp_quadform_grad(c.k, c.n, c.X, c.thd, 2, Z, 2, Z, 2, nullptr, nullptr, q, nullptr, 0,
                        nullptr, 0, c.w + c.L.qf, c.L.qf_bytes, c.s);
  if (st) return st;
  double hq[2], yx;
  st = d2h(hq, q, 2, c.s);
  if (st) return st;
  st = dots<T>(c, c.y, x, c.n, 1, &yx);
  if (st) return st;
  double pp = 0.0;
  for (double v : pi) pp += v * v;
  *H = 0.5 * (2.0 * yx - hq[0]) + 0.5 * hq[1] + 0.5 * pp;
  return GP_OK;
}

template <typename T>
gp_status run_implicit(Ctx<T> &c, double *theta_d, double *pi_d, T *x_warm, const double *u_d,
                       double *H0_d, double *H1_d, int32_t *acc_d, int32_t *status_d,
                       int32_t *iters_d) {
  const gp_implicit_params &p = *c.p;
  const int nth = c.nth;
  const int64_t n = c.n;
  const int kh = p.history;
  const unsigned gb = (unsigned)((n + 255) / 256);
  std::vector<double> th0(nth), pi0(nth);
  gp_status st = d2h(th0.data(), theta_d, nth, c.s);
  if (st) return st;
  st = d2h(pi0.data(), pi_d, nth, c.s);
  if (st) return st;
  double u = -1.0;
  if (u_d) {
    st = d2h(&u, u_d, 1, c.s);
    if (st) return st;
  }
  c.thd = theta_d;
  T *x = (T *)(c.w + c.L.x);
  T *v = (T *)(c.w + c.L.v);
  T *Z = (T *)(c.w + c.L.Z), *AZ = (T *)(c.w + c.L.AZ);
  T *fx = (T *)(c.w + c.L.fx), *gx = (T *)(c.w + c.L.gx);
  T *Fh = (T *)(c.w + c.L.Fh), *Gh = (T *)(c.w + c.L.Gh);
  double *alpha_d = (double *)(c.w + c.L.alpha);
  int32_t status = 0, total_it = 0, cs = 0, ci = 0;

  // start: solve at theta_0 (warm), H_0
  hipError_t e = hipMemcpyAsync(x, x_warm, sizeof(T) * n, hipMemcpyDeviceToDevice, c.s);
  if (e != hipSuccess) return hip_fail(e, "copy");
  double H0 = 0.0;
  st = energy<T>(c, th0, pi0, x, &H0, &cs, &ci);
  if (st) return st;
  if (cs) status |= GP_CHAIN_CG_MAXIT;

  // R = I / c with c ~ rho(A(theta_0)), or with a Nystrom factor R = P^{-1} / c, c ~ rho(P^{-1} A)
  // (P built at theta_0), c by power iterations from y / |y|
  double *th0_d = (double *)(c.w + c.L.th0);
  st = h2d<T>(th0_d, th0.data(), nth, c.s);
  if (st) return st;
  T *rb = (T *)(c.w + c.L.rb);
  double yy;
  st = dots<T>(c, c.y, c.y, n, 1, &yy);
  if (st) return st;
  scale_copy<T><<<gb, 256, 0, c.s>>>(n, c.y, 1.0 / sqrt(yy > 0 ? yy : 1.0), v);
  double rho = 1.0;
  for (int it = 0; it < p.power_its; ++it) {
    st = gp_kmatvec(c.k, n, c.X, th0_d, 1, v, 1, nullptr, gx, 1, c.w + c.L.qf, c.L.qf_bytes, c.s);
    if (st) return st;
    if (c.rank > 0) {
      e = nystrom_apply<T>(n, c.rank, (const T *)c.U, c.lam, th0_d, nth, nullptr, 1, gx, rb,
                           c.w + c.L.nys, c.s);
      if (e != hipSuccess) return hip_fail(e, "Nystrom apply");
      e = hipMemcpyAsync(gx, rb, sizeof(T) * n, hipMemcpyDeviceToDevice, c.s);
      if (e != hipSuccess) return hip_fail(e, "copy");
    }
    double nn;
    st = dots<T>(c, gx, gx, n, 1, &nn);
    if (st) return st;
    rho = sqrt(nn);
    scale_copy<T><<<gb, 256, 0, c.s>>>(n, gx, 1.0 / rho, v);
  }
  const double inv_c = 1.0 / rho;
  const double ynorm = sqrt(yy);

  std::vector<double> th = th0, pi = pi0;
  const int nb = (int)std::min<int64_t>(kDotBlocks, (n + 255) / 256);
  double *xf = (double *)(c.w + c.L.xf);
  double *wts_d = (double *)(c.w + c.L.wts);
  const double wts[2] = {-0.5, 0.5};
  st = h2d<T>(wts_d, wts, 2, c.s);
  if (st) return st;
  // the device state: (th, pi) = (theta_0, pi_0), nothing taken yet
  double *ist = (double *)(c.w + c.L.ist);
  ImpDev ds;
  ds.ths = ist;
  ds.pis = ist + kTh;
  ds.th = ist + 2 * kTh;
  ds.pi = ist + 3 * kTh;
  ds.hf = ist + 4 * kTh;
  ds.hg = ds.hf + (size_t)kHistMax * 2 * kTh;
  ds.G = ds.hg + (size_t)kHistMax * 2 * kTh;
  ds.flags = (int32_t *)(c.w + c.L.iflags);
  {
    std::vector<double> v0(2 * kTh, 0.0);
    std::copy(th0.begin(), th0.end(), v0.begin());
    std::copy(pi0.begin(), pi0.end(), v0.begin() + kTh);
    e = hipMemcpyAsync(ds.th, v0.data(), sizeof(double) * 2 * kTh, hipMemcpyHostToDevice, c.s);
    const int32_t f0[8] = {0, 0, 0, 0, 0, 0, 0, 0};
    if (e == hipSuccess) e = hipMemcpyAsync(ds.flags, f0, sizeof(f0), hipMemcpyHostToDevice, c.s);
    if (e == hipSuccess) e = hipStreamSynchronize(c.s);
    if (e != hipSuccess) return hip_fail(e, "fixed-point state");
  }
  // kCheck iterations, each the same launches (the history's size and slot and the iteration
  // limit are read on the device), captured once as a graph and replayed between host checks
  auto enqueue_iteration = [&](hipStream_t q) -> gp_status {
    imp_midpoint<<<1, kTh, 0, q>>>(ds, nth, c.thd);
    pack_z<T><<<gb, 256, 0, q>>>(n, x, c.phi, Z);
    gp_status r = gp_quadform_grad(c.k, n, c.X, c.thd, 2, Z, 2, Z, 2, wts_d, xf + kXfGrad, nullptr,
                                   AZ, 2, nullptr, 0, c.w + c.L.qf, c.L.qf_bytes, q);
    if (r) return r;
    linear_residual<T><<<gb, 256, 0, q>>>(n, c.y, AZ, rb);
    multi_dot<T><<<nb, 256, 0, q>>>(n, 1, rb, rb, n, xf + kXfRes);
    hipError_t he = hipSuccess;
    if (c.rank > 0) {
      he = nystrom_apply<T>(n, c.rank, (const T *)c.U, c.lam, th0_d, nth, nullptr, 1, rb, fx,
                            c.w + c.L.nys, q);
      if (he != hipSuccess) return hip_fail(he, "Nystrom apply");
      fixed_point_x<T><<<gb, 256, 0, q>>>(n, fx, x, inv_c, fx, gx);
    } else {
      fixed_point_x<T><<<gb, 256, 0, q>>>(n, rb, x, inv_c, fx, gx);
    }
    if (kh > 0) {  // (f, g) of x into the iteration's slot, the x parts of the new Gram row
      hist_store<T><<<gb, 256, 0, q>>>(n, ds.flags, kh, fx, gx, Fh, Gh);
      multi_dot_hist<T><<<nb, 256, 0, q>>>(n, ds.flags, kh, fx, Fh, n, xf + kXfRow);
    }
    imp_update<<<1, 64, 0, q>>>(ds, nth, p.dt, p.tol, ynorm, kh, p.maxit, nb, xf + kXfGrad,
                                xf + kXfRes, xf + kXfRow, alpha_d);
    imp_x_update<T><<<gb, 256, 0, q>>>(n, kh, ds.flags, alpha_d, Gh, n, gx, x);
    he = hipGetLastError();
    return he == hipSuccess ? GP_OK : hip_fail(he, "fixed-point kernels");
  };
  hipGraphExec_t exec = nullptr;
  {
    hipStream_t cap;
    e = hipStreamCreateWithFlags(&cap, hipStreamNonBlocking);
    if (e != hipSuccess) return hip_fail(e, "capture stream");
    hipGraph_t graph = nullptr;
    gp_status sc = GP_OK;
    e = hipStreamBeginCapture(cap, hipStreamCaptureModeThreadLocal);
    if (e == hipSuccess) {
      for (int i = 0; i < kCheck && sc == GP_OK; ++i) sc = enqueue_iteration(cap);
      const hipError_t ee = hipStreamEndCapture(cap, &graph);
      if (e == hipSuccess) e = ee;
    }
    if (e == hipSuccess && sc == GP_OK) e = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
    if (graph) (void)hipGraphDestroy(graph);
    (void)hipStreamDestroy(cap);
    if (sc != GP_OK) return sc;
    if (e != hipSuccess) return hip_fail(e, "fixed-point graph");
  }
  int32_t fl[5] = {0, 0, 0, 0, 0};
  for (int step = 0; step < p.n_steps && status == 0 && st == GP_OK; ++step) {
    imp_begin_step<<<1, 64, 0, c.s>>>(ds, nth);
    e = hipGetLastError();
    for (int it = 0; it < p.maxit && e == hipSuccess; it += kCheck) {
      e = hipGraphLaunch(exec, c.s);
      if (e == hipSuccess) e = hipMemcpyAsync(fl, ds.flags, sizeof(fl), hipMemcpyDeviceToHost, c.s);
      if (e == hipSuccess) e = hipStreamSynchronize(c.s);
      if (e == hipSuccess && (fl[0] || fl[1])) break;
    }
    if (e != hipSuccess) break;
    status |= fl[1];
    if (!fl[0] && status == 0) status |= GP_CHAIN_FP_MAXIT;
  }
  (void)hipGraphExecDestroy(exec);
  if (e != hipSuccess) return hip_fail(e, "fixed-point iterations");
  total_it = fl[2];
  {
    std::vector<double> v1(2 * kTh);
    st = d2h(v1.data(), ds.th, 2 * kTh, c.s);
    if (st) return st;
    std::copy(v1.begin(), v1.begin() + nth, th.begin());
    std::copy(v1.begin() + kTh, v1.begin() + kTh + nth, pi.begin());
  }

  // end: solve at theta_1, H_1, Metropolis decision
  double H1 = NAN;
  if (status == 0) {
    st = energy<T>(c, th, pi, x, &H1, &cs, &ci);
    if (st) return st;
    if (cs) status |= GP_CHAIN_CG_MAXIT;
    if (!isfinite(H1)) status |= GP_CHAIN_NONFINITE_H;
  }
  bool acc = status == 0;
  if (acc && u_d) acc = (u <= 0.0) || (log(u) <= H0 - H1);
  const std::vector<double> &tho = acc ? th : th0;
  const std::vector<double> &pio = acc ? pi : pi0;
  st = h2d<T>(theta_d, tho.data(), nth, c.s);
  if (st) return st;
  st = h2d<T>(pi_d, pio.data(), nth, c.s);
  if (st) return st;
  if (acc) {
    e = hipMemcpyAsync(x_warm, x, sizeof(T) * n, hipMemcpyDeviceToDevice, c.s);
    if (e != hipSuccess) return hip_fail(e, "copy");
  }
  st = h2d<T>(H0_d, &H0, 1, c.s);
  if (!st) st = h2d<T>(H1_d, &H1, 1, c.s);
  if (st) return st;
  const int32_t outs[3] = {acc ? 1 : 0, status, total_it};
  e = hipMemcpyAsync(acc_d, &outs[0], sizeof(int32_t), hipMemcpyHostToDevice, c.s);
  if (e == hipSuccess) e = hipMemcpyAsync(status_d, &outs[1], sizeof(int32_t), hipMemcpyHostToDevice, c.s);
  if (e == hipSuccess && iters_d)
    e = hipMemcpyAsync(iters_d, &outs[2], sizeof(int32_t), hipMemcpyHostToDevice, c.s);
  if (e == hipSuccess) e = hipStreamSynchronize(c.s);
  return e == hipSuccess ? GP_OK : hip_fail(e, "outputs");
}

gp_status check_imp(const gp_kernel *k, const gp_implicit_params *p, int64_t n, int32_t rank) {
  if (gp_n_theta(k) < 0) return fail(GP_ERR_ARG, "invalid kernel description");
  if (k->flags & GP_NO_NOISE) return fail(GP_ERR_ARG, "GP_NO_NOISE is not accepted");
  if (!p) return fail(GP_ERR_ARG, "params are NULL");
  if (p->n_steps < 0) return fail(GP_ERR_ARG, "n_steps < 0");
  if (p->history < 0 || p->history > kHistMax)
    return fail(GP_ERR_ARG, "history = %d outside 0..%d", p->history, kHistMax);
  if (!(p->tol > 0.0) || !(p->cg_tol > 0.0)) return fail(GP_ERR_ARG, "tolerances must be > 0");
  if (p->maxit < 1 || p->cg_maxit < 1) return fail(GP_ERR_ARG, "iteration limits must be >= 1");
  if (p->power_its < 1) return fail(GP_ERR_ARG, "power_its must be >= 1");
  if (n < 1) return fail(GP_ERR_SHAPE, "n = %lld < 1", (long long)n);
  if (rank < 0 || rank > 512) return fail(GP_ERR_SHAPE, "rank = %d outside 0..512", rank);
  return GP_OK;
}

}  // namespace
}  // namespace gpk

using namespace gpk;

extern "C" {

size_t gp_implicit_workspace_size(const gp_kernel *k, const gp_implicit_params *p, int64_t n,
                                  int32_t rank) {
  if (check_imp(k, p, n, rank) != GP_OK) return 0;
  return imp_layout(k, n, p->history, rank).total;
}

gp_status gp_hmc_implicit(const gp_kernel *k, const gp_implicit_params *p, int64_t n,
                          const void *X, const void *y, const void *phi, double *theta, double *pi,
                          void *x_warm, const double *u_accept, int32_t rank, const void *U,
                          const double *lam, double *H0, double *H1, int32_t *accepted,
                          int32_t *status, int32_t *iters, void *ws, size_t ws_bytes,
                          hipStream_t stream) {
  clear_error();
  gp_status st = check_imp(k, p, n, rank);
  if (st) return st;
  if (!X || !y || !phi || !theta || !pi || !x_warm || !H0 || !H1 || !accepted || !status)
    return fail(GP_ERR_ARG, "X, y, phi, theta, pi, x_warm, H0, H1, accepted and status must be non-NULL");
  if (rank > 0 && (!U || !lam)) return fail(GP_ERR_ARG, "rank > 0 needs U and lam");
  const ImpLayout L = imp_layout(k, n, p->history, rank);
  if (!ws || ws_bytes < L.total)
    return fail(GP_ERR_WORKSPACE, "workspace of %zu bytes needed, %zu given", L.total,
                ws ? ws_bytes : (size_t)0);
  if (k->prec == GP_F64) {
    Ctx<double> c{k, p, n, gp_n_theta(k), X, (const double *)y, (const double *)phi, rank, U, lam,
                  (char *)ws, L, stream, nullptr};
    return run_implicit<double>(c, theta, pi, (double *)x_warm, u_accept, H0, H1, accepted, status,
                                iters);
  }
  Ctx<float> c{k, p, n, gp_n_theta(k), X, (const float *)y, (const float *)phi, rank, U, lam,
               (char *)ws, L, stream, nullptr};
  return run_implicit<float>(c, theta, pi, (float *)x_warm, u_accept, H0, H1, accepted, status,
                             iters);
}

}  // extern "C"
