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
// iteration).  The (theta, pi) parts live on the host in double, the x parts on the device; the
// inner products and the combination run in the kernels below.  c comes from power iterations
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
constexpr int kDotBlocks = 512;
// Transfer block of a fixed-point iteration: the force pass's gradient, the block partials of
// |y - A(m) x|^2 and those of the new Gram row, fetched to the host together.
constexpr int kXfGrad = 0;
constexpr int kXfRes = kMaxD + 4;
constexpr int kXfRow = kXfRes + kDotBlocks;
constexpr int kXfDoubles = kXfRow + kDotBlocks * kHistMax;

// out[b][j] = partial sums over this block's rows of a[i] * H[j][i] for j < m (H rows of length n)
template <typename T>
__global__ __launch_bounds__(256) void multi_dot(int64_t n, int m, const T *a, const T *H,
                                                 int64_t ldh, double *out) {
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

// x = sum_j alpha_j G[j]
template <typename T>
__global__ void combine(int64_t n, int m, const double *alpha, const T *G, int64_t ldg, T *x) {
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (i >= n) return;
  double s = 0.0;
  for (int j = 0; j < m; ++j) s += alpha[j] * (double)G[(int64_t)j * ldg + i];
  x[i] = (T)s;
}

template <typename T>
__global__ void scale_copy(int64_t n, const T *a, double s, T *b) {
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (i < n) b[i] = (T)((double)a[i] * s);
}

struct ImpLayout {
  size_t qf, qf_bytes, pcg, pcg_bytes, Z, AZ, x, v, rb, fx, gx, Fh, Gh, part, alpha, grad, th0,
      xf, wts, nys, total;
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
  L.xf = o;  // one device -> host transfer per fixed-point iteration (kXf* offsets)
  o += align256(sizeof(double) * kXfDoubles);
  L.wts = o;
  o += align256(sizeof(double) * 2);
  L.nys = o;
  o += align256(rank > 0 ? nystrom_apply_scratch(n, rank, 1) : 0);
  L.total = o;
  return L;
}

// Minimise |sum alpha_i f_i|^2 subject to sum alpha_i = 1 from the Gram matrix G (m x m):
// alpha = G^{-1} 1 / (1^T G^{-1} 1), with a small ridge for a near-singular history.
std::vector<double> anderson_weights(const std::vector<double> &G, int m) {
  double tr = 0.0;
  for (int i = 0; i < m; ++i) tr += G[(size_t)i * m + i];
  std::vector<double> a((size_t)m * m), b(m, 1.0);
  for (int i = 0; i < m; ++i)
    for (int j = 0; j < m; ++j) a[(size_t)i * m + j] = G[(size_t)i * m + j] + (i == j ? 1e-12 * tr / m : 0.0);
  // Gaussian elimination with partial pivoting
  for (int c = 0; c < m; ++c) {
    int p = c;
    for (int r = c + 1; r < m; ++r)
      if (fabs(a[(size_t)r * m + c]) > fabs(a[(size_t)p * m + c])) p = r;
    if (p != c) {
      for (int j = 0; j < m; ++j) std::swap(a[(size_t)c * m + j], a[(size_t)p * m + j]);
      std::swap(b[c], b[p]);
    }
    const double d = a[(size_t)c * m + c];
    if (fabs(d) < 1e-300) continue;
    for (int r = c + 1; r < m; ++r) {
      const double f = a[(size_t)r * m + c] / d;
      for (int j = c; j < m; ++j) a[(size_t)r * m + j] -= f * a[(size_t)c * m + j];
      b[r] -= f * b[c];
    }
  }
  std::vector<double> z(m, 0.0);
  for (int r = m - 1; r >= 0; --r) {
    double s = b[r];
    for (int j = r + 1; j < m; ++j) s -= a[(size_t)r * m + j] * z[j];
    const double d = a[(size_t)r * m + r];
    z[r] = fabs(d) < 1e-300 ? 0.0 : s / d;
  }
  double sum = 0.0;
  for (int i = 0; i < m; ++i) sum += z[i];
  std::vector<double> alpha(m, 0.0);
  if (!(fabs(sum) > 0.0) || !isfinite(sum)) {
    alpha[m - 1] = 1.0;  // degenerate history: plain fixed-point step
    return alpha;
  }
  for (int i = 0; i < m; ++i) alpha[i] = z[i] / sum;
  return alpha;
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
  std::vector<double> hf((size_t)kHistMax * 2 * nth), hg((size_t)kHistMax * 2 * nth);  // host parts
  std::vector<double> G((size_t)kHistMax * kHistMax);
  // One host round trip per fixed-point iteration: the midpoint theta and the Anderson weights
  // go up without a wait (the host buffers are not touched again before the next transfer
  // down, which follows them on the stream), and the device work of the iteration is enqueued
  // whole before its one transfer down.
  const int nb = (int)std::min<int64_t>(kDotBlocks, (n + 255) / 256);
  double *xf = (double *)(c.w + c.L.xf);
  double *wts_d = (double *)(c.w + c.L.wts);
  const double wts[2] = {-0.5, 0.5};
  st = h2d<T>(wts_d, wts, 2, c.s);
  if (st) return st;
  std::vector<double> hx(kXfDoubles), mid(nth), alpha_h(kHistMax);
  for (int step = 0; step < p.n_steps && status == 0; ++step) {
    const std::vector<double> ths = th, pis = pi;
    int m = 0, head = 0;  // history size, next slot
    bool conv = false;
    // the current iterate v = (th, pi, x)
    for (int it = 0; it < p.maxit; ++it) {
      ++total_it;
      for (int kx = 0; kx < nth; ++kx) mid[kx] = 0.5 * (ths[kx] + th[kx]);
      e = hipMemcpyAsync(c.thd, mid.data(), sizeof(double) * nth, hipMemcpyHostToDevice, c.s);
      if (e != hipSuccess) return hip_fail(e, "host -> device");
      pack_z<T><<<gb, 256, 0, c.s>>>(n, x, c.phi, Z);
      st = gp_quadform_grad(c.k, n, c.X, c.thd, 2, Z, 2, Z, 2, wts_d, xf + kXfGrad, nullptr, AZ, 2,
                            nullptr, 0, c.w + c.L.qf, c.L.qf_bytes, c.s);
      if (st) return st;
      linear_residual<T><<<gb, 256, 0, c.s>>>(n, c.y, AZ, rb);
      multi_dot<T><<<nb, 256, 0, c.s>>>(n, 1, rb, rb, n, xf + kXfRes);
      if (c.rank > 0) {
        e = nystrom_apply<T>(n, c.rank, (const T *)c.U, c.lam, th0_d, nth, nullptr, 1, rb, fx,
                             c.w + c.L.nys, c.s);
        if (e != hipSuccess) return hip_fail(e, "Nystrom apply");
        fixed_point_x<T><<<gb, 256, 0, c.s>>>(n, fx, x, inv_c, fx, gx);
      } else {
        fixed_point_x<T><<<gb, 256, 0, c.s>>>(n, rb, x, inv_c, fx, gx);
      }
      // Anderson history: (f, g) into slot `head` and the new Gram row, ahead of the host's
      // convergence test (a converged iteration leaves them unused)
      const int m_new = kh > 0 ? std::min(m + 1, kh) : 0;
      if (kh > 0) {
        e = hipMemcpyAsync(Fh + (size_t)head * n, fx, sizeof(T) * n, hipMemcpyDeviceToDevice, c.s);
        if (e == hipSuccess)
          e = hipMemcpyAsync(Gh + (size_t)head * n, gx, sizeof(T) * n, hipMemcpyDeviceToDevice, c.s);
        if (e != hipSuccess) return hip_fail(e, "history");
        multi_dot<T><<<nb, 256, 0, c.s>>>(n, m_new, fx, Fh, n, xf + kXfRow);
      }
      e = hipGetLastError();
      if (e != hipSuccess) return hip_fail(e, "fixed-point kernels");
      st = d2h(hx.data(), xf, kXfRow + nb * m_new, c.s);
      if (st) return st;
      // g = Phi(v), f = g - v
      const double *F = hx.data() + kXfGrad;
      std::vector<double> g_tp(2 * nth), f_tp(2 * nth);
      double fmax = 0.0, vmax = 0.0;
      for (int kx = 0; kx < nth; ++kx) {
        g_tp[kx] = ths[kx] + p.dt * 0.5 * (pis[kx] + pi[kx]);
        g_tp[nth + kx] = pis[kx] - p.dt * F[kx];
        f_tp[kx] = g_tp[kx] - th[kx];
        f_tp[nth + kx] = g_tp[nth + kx] - pi[kx];
        fmax = std::max(fmax, std::max(fabs(f_tp[kx]), fabs(f_tp[nth + kx])));
        vmax = std::max(vmax, std::max(fabs(th[kx]), fabs(pi[kx])));
      }
      if (!isfinite(fmax)) {
        status |= GP_CHAIN_NONFINITE_THETA;
        break;
      }
      double rr2 = 0.0;
      for (int b = 0; b < nb; ++b) rr2 += hx[(size_t)kXfRes + b];
      const double res = sqrt(rr2);  // |y - A(m) x|
      if (fmax <= p.tol * (1.0 + vmax) && res <= p.tol * ynorm) {
        conv = true;
        // take the last map value: theta_1, pi_1 from g
        for (int kx = 0; kx < nth; ++kx) {
          th[kx] = g_tp[kx];
          pi[kx] = g_tp[nth + kx];
        }
        break;
      }
      if (kh == 0) {  // Picard
        for (int kx = 0; kx < nth; ++kx) {
          th[kx] = g_tp[kx];
          pi[kx] = g_tp[nth + kx];
        }
        e = hipMemcpyAsync(x, gx, sizeof(T) * n, hipMemcpyDeviceToDevice, c.s);
        if (e != hipSuccess) return hip_fail(e, "copy");
        continue;
      }
      // Anderson: the parameter parts of (f, g) in slot `head`, the Gram row, the combination
      for (int kx = 0; kx < 2 * nth; ++kx) {
        hf[(size_t)head * 2 * nth + kx] = f_tp[kx];
        hg[(size_t)head * 2 * nth + kx] = g_tp[kx];
      }
      m = m_new;
      for (int j = 0; j < m; ++j) {
        double t = 0.0;
        for (int b = 0; b < nb; ++b) t += hx[(size_t)kXfRow + (size_t)b * m + j];
        for (int kx = 0; kx < 2 * nth; ++kx) t += hf[(size_t)head * 2 * nth + kx] * hf[(size_t)j * 2 * nth + kx];
        G[(size_t)head * kHistMax + j] = t;
        G[(size_t)j * kHistMax + head] = t;
      }
      std::vector<double> Gm((size_t)m * m);
      for (int i = 0; i < m; ++i)
        for (int j = 0; j < m; ++j) Gm[(size_t)i * m + j] = G[(size_t)i * kHistMax + j];
      const std::vector<double> alpha = anderson_weights(Gm, m);
      for (int kx = 0; kx < nth; ++kx) {
        double a = 0.0, b = 0.0;
        for (int j = 0; j < m; ++j) {
          a += alpha[j] * hg[(size_t)j * 2 * nth + kx];
          b += alpha[j] * hg[(size_t)j * 2 * nth + nth + kx];
        }
        th[kx] = a;
        pi[kx] = b;
      }
      std::copy(alpha.begin(), alpha.end(), alpha_h.begin());
      e = hipMemcpyAsync(alpha_d, alpha_h.data(), sizeof(double) * m, hipMemcpyHostToDevice, c.s);
      if (e != hipSuccess) return hip_fail(e, "host -> device");
      combine<T><<<gb, 256, 0, c.s>>>(n, m, alpha_d, Gh, n, x);
      e = hipGetLastError();
      if (e != hipSuccess) return hip_fail(e, "Anderson combination");
      head = (head + 1) % kh;
    }
    if (!conv && status == 0) status |= GP_CHAIN_FP_MAXIT;
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
