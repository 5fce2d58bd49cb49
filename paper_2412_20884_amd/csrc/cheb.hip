// Products and quadratic-form gradients of the Chebyshev-amplitude kernel of Section 4:
//     K_ij = e^{C(x_i)} e^{C(x_j)} K~_ij,   K~_ij = exp(-|x_i - x_j|^2 / (2 l^2)),
//     C(x) = sum_m Theta_m phi_m(x),        phi_m(x) = prod_k T_{m_k}(x^k),
// i.e. K = D K~ D with D = diag(e^{C(x_i)}).  Every pairwise sum runs in the isotropic SE pair
// kernels (unit amplitude, no noise) on amplitude-scaled operands; the amplitudes, the
// scalings and the Theta-gradient run in the kernels of this file:
//     A V = sigma^2 V + D (K~ (D V))
//     dQ/dTheta_m = sum_i phi_m(x_i) s_i,  s_i = e^{C(x_i)} sum_c w_c [u_ic (K~ D v_c)_i + v_ic (K~ D u_c)_i]
//     dQ/dlog l   = the SE length-scale gradient of sum_c w_c (D u_c)^T K~ (D v_c)
//     q_c = (D u_c)^T K~ (D v_c) + sigma^2 u_c . v_c,   dQ/dlog sigma^2 = sigma^2 sum_c w_c u_c . v_c
// The Chebyshev polynomials are evaluated by their three-term recurrence.
#include "cheb.h"

namespace gpk {

gp_status fail(gp_status st, const char *fmt, ...);
gp_status hip_fail(hipError_t e, const char *where);

namespace {

constexpr int kChebMaxTerms = 64;   // N_cheb^d
constexpr int kRowsBlk = 256;

// T_m(x^k) for m < nc, k < d, into tt[k * nc + m]; d * nc <= 64 whenever nc^d <= 64.
template <typename T>
__device__ void cheb_table(const T *x, int d, int nc, double *tt) {
  for (int k = 0; k < d; ++k) {
    const double xv = (double)x[k];
    double tm1 = 1.0, t = xv;
    tt[k * nc] = 1.0;
    if (nc > 1) tt[k * nc + 1] = xv;
    for (int m = 2; m < nc; ++m) {
      const double tn = 2.0 * xv * t - tm1;
      tm1 = t;
      t = tn;
      tt[k * nc + m] = tn;
    }
  }
}

// phi_t(x) for the multi-index of term t (m_1 slowest).
__device__ __forceinline__ double cheb_term(const double *tt, int d, int nc, int t) {
  double p = 1.0;
  for (int k = d - 1; k >= 0; --k) {
    const int m = t % nc;
    t /= nc;
    p *= tt[k * nc + m];
  }
  return p;
}

template <typename T>
__global__ __launch_bounds__(kRowsBlk) void cheb_amp(const T *X, int64_t n, int d, int nc, int nt,
                                                    const double *theta, double *amp) {
  const int64_t i = (int64_t)blockIdx.x * kRowsBlk + threadIdx.x;
  if (i >= n) return;
  double tt[kChebMaxTerms];
  cheb_table(X + i * d, d, nc, tt);
  double c = 0.0;
  for (int t = 0; t < nt; ++t) c += theta[t] * cheb_term(tt, d, nc, t);
  amp[i] = exp(c);
}

// The SE parameters (log alpha = 0, log l, log sigma^2) from the Chebyshev theta.
__global__ void cheb_theta_se(const double *theta, int nth, double *th_se) {
  if (threadIdx.x == 0) {
    th_se[0] = 0.0;
    th_se[1] = theta[nth - 2];
    th_se[2] = theta[nth - 1];
  }
}

template <typename T>
__global__ __launch_bounds__(kRowsBlk) void cheb_scale(int64_t n, int r, const double *amp,
                                                      const T *V, int64_t ldv, T *out) {
  const int64_t e = (int64_t)blockIdx.x * kRowsBlk + threadIdx.x;
  if (e >= n * r) return;
  const int64_t i = e / r;
  const int c = (int)(e - i * r);
  out[e] = (T)(amp[i] * (double)V[i * ldv + c]);
}

// out = (sigma^2 + shift_c) V + D (K~ D V)
template <typename T>
__global__ __launch_bounds__(kRowsBlk) void cheb_mv_finish(int64_t n, int r, const double *amp,
                                                          const T *V, int64_t ldv, const T *kv,
                                                          const double *theta, int nth,
                                                          int no_noise, const double *shift,
                                                          T *out, int64_t ldo) {
  const int64_t e = (int64_t)blockIdx.x * kRowsBlk + threadIdx.x;
  if (e >= n * r) return;
  const int64_t i = e / r;
  const int c = (int)(e - i * r);
  const double diag = (no_noise ? 0.0 : exp(theta[nth - 1])) + (shift ? shift[c] : 0.0);
  out[i * ldo + c] = (T)(diag * (double)V[i * ldv + c] + amp[i] * (double)kv[e]);
}

// Per block of rows: sum_i phi_t(x_i) s_i for every term t, and u_c . v_c per column; the
// products A U, A V on request.  part[block][nt + r].
template <typename T>
__global__ __launch_bounds__(kRowsBlk) void cheb_grad_rows(
    int64_t n, int r, const T *X, int d, int nc, int nt, const double *theta, int nth,
    int no_noise, const double *amp, const T *U, int64_t ldu, const T *V, int64_t ldv,
    const double *w, const T *ku, const T *kv, T *AU, int64_t ldau, T *AV, int64_t ldav,
    double *part) {
  __shared__ double red[kRowsBlk / 64][kChebMaxTerms + 32];
  const int64_t i = (int64_t)blockIdx.x * kRowsBlk + threadIdx.x;
  const bool live = i < n;
  const double sigma2 = no_noise ? 0.0 : exp(theta[nth - 1]);
  double s = 0.0;
  double uv[32];
  for (int c = 0; c < r; ++c) uv[c] = 0.0;
  double tt[kChebMaxTerms];
  if (live) {
    const double a = amp[i];
    for (int c = 0; c < r; ++c) {
      const double u = (double)U[i * ldu + c], v = (double)V[i * ldv + c];
      const double kuv = (double)ku[i * r + c], kvv = (double)kv[i * r + c];
      const double wc = w ? w[c] : 1.0;
      s += wc * (u * kvv + v * kuv);
      uv[c] = u * v;
      if (AU) AU[i * ldau + c] = (T)(sigma2 * u + a * kuv);
      if (AV) AV[i * ldav + c] = (T)(sigma2 * v + a * kvv);
    }
    s *= a;
    cheb_table(X + i * d, d, nc, tt);
  }
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  for (int t = 0; t < nt + r; ++t) {
    double v = 0.0;
    if (live) v = t < nt ? cheb_term(tt, d, nc, t) * s : uv[t - nt];
    v = wave_sum(v);
    if (lane == 0) red[wave][t] = v;
  }
  __syncthreads();
  for (int t = threadIdx.x; t < nt + r; t += kRowsBlk) {
    double tot = 0.0;
    for (int wv = 0; wv < kRowsBlk / 64; ++wv) tot += red[wv][t];
    part[(int64_t)blockIdx.x * (nt + r) + t] = tot;
  }
}

// Fixed-order sums of the block records, then the gradient and the forms.
__global__ void cheb_grad_final(int64_t blocks, int nt, int r, const double *part,
                                const double *gse, const double *qse, const double *w,
                                const double *theta, int nth, int no_noise, double *grad,
                                double *quad) {
  __shared__ double tot[kChebMaxTerms + 32];
  const int e = threadIdx.x;
  if (e < nt + r) {
    double s = 0.0;
    for (int64_t b = 0; b < blocks; ++b) s += part[b * (nt + r) + e];
    tot[e] = s;
  }
  __syncthreads();
  if (e == 0) {
    const double sigma2 = no_noise ? 0.0 : exp(theta[nth - 1]);
    if (grad) {
      for (int t = 0; t < nt; ++t) grad[t] = tot[t];
      grad[nt] = gse[1];
      double g = 0.0;
      for (int c = 0; c < r; ++c) g += (w ? w[c] : 1.0) * tot[nt + c];
      grad[nt + 1] = sigma2 * g;
    }
    if (quad)
      for (int c = 0; c < r; ++c) quad[c] = qse[c] + sigma2 * tot[nt + c];
  }
}

struct ChebLayout {
  size_t se, se_bytes, th_se, amp, up, vp, ku, kv, gq, part, total;
  int64_t blocks;
};

gp_kernel se_of(const gp_kernel *k) {
  gp_kernel s = *k;
  s.kind = GP_SE_ISO;
  s.flags = GP_NO_NOISE;
  s.n_cheb = 0;
  return s;
}

ChebLayout cheb_layout(const gp_kernel *k, int64_t n, int r) {
  ChebLayout L;
  const gp_kernel se = se_of(k);
  const size_t es = k->prec == GP_F64 ? 8 : 4;
  const int nt = cheb_terms(k);
  L.blocks = (n + kRowsBlk - 1) / kRowsBlk;
  size_t o = 0;
  L.se = o;
  L.se_bytes = gp_workspace_size(&se, n, r);
  o += align256(L.se_bytes);
  L.th_se = o;
  o += 256;
  L.amp = o;
  o += align256(sizeof(double) * n);
  L.up = o;
  o += align256(es * n * r);
  L.vp = o;
  o += align256(es * n * r);
  L.ku = o;
  o += align256(es * n * r);
  L.kv = o;
  o += align256(es * n * r);
  L.gq = o;
  o += align256(sizeof(double) * (3 + kMaxRPass));
  L.part = o;
  o += align256(sizeof(double) * L.blocks * (nt + r));
  L.total = o;
  return L;
}

template <typename T>
gp_status run_prep(const gp_kernel *k, int64_t n, const void *X, const double *theta,
                   const ChebLayout &L, char *w, hipStream_t s) {
  const int nt = cheb_terms(k), nth = nt + 2;
  const unsigned gb = (unsigned)((n + kRowsBlk - 1) / kRowsBlk);
  cheb_theta_se<<<1, 64, 0, s>>>(theta, nth, (double *)(w + L.th_se));
  cheb_amp<T><<<gb, kRowsBlk, 0, s>>>((const T *)X, n, k->d, k->n_cheb, nt, theta,
                                      (double *)(w + L.amp));
  hipError_t e = hipGetLastError();
  return e == hipSuccess ? GP_OK : hip_fail(e, "Chebyshev amplitudes");
}

template <typename T>
gp_status run_kmatvec(const gp_kernel *k, int64_t n, const void *X, const double *theta, int r,
                      const void *V, int64_t ldv, const double *shift, void *out, int64_t ldo,
                      char *w, const ChebLayout &L, hipStream_t s) {
  gp_status st = run_prep<T>(k, n, X, theta, L, w, s);
  if (st) return st;
  const gp_kernel se = se_of(k);
  const double *amp = (const double *)(w + L.amp);
  const unsigned eb = (unsigned)((n * r + kRowsBlk - 1) / kRowsBlk);
  cheb_scale<T><<<eb, kRowsBlk, 0, s>>>(n, r, amp, (const T *)V, ldv, (T *)(w + L.up));
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return hip_fail(e, "Chebyshev scaling");
  st = gp_kmatvec(&se, n, X, (const double *)(w + L.th_se), r, w + L.up, r, nullptr, w + L.ku, r,
                  w + L.se, L.se_bytes, s);
  if (st) return st;
  cheb_mv_finish<T><<<eb, kRowsBlk, 0, s>>>(n, r, amp, (const T *)V, ldv, (const T *)(w + L.ku),
                                            theta, cheb_terms(k) + 2,
                                            (k->flags & GP_NO_NOISE) ? 1 : 0, shift, (T *)out, ldo);
  e = hipGetLastError();
  return e == hipSuccess ? GP_OK : hip_fail(e, "Chebyshev product");
}

template <typename T>
gp_status run_quadform(const gp_kernel *k, int64_t n, const void *X, const double *theta, int r,
                       const void *U, int64_t ldu, const void *V, int64_t ldv, const double *wgt,
                       double *grad, double *quad, void *AU, int64_t ldau, void *AV, int64_t ldav,
                       char *w, const ChebLayout &L, hipStream_t s) {
  gp_status st = run_prep<T>(k, n, X, theta, L, w, s);
  if (st) return st;
  const gp_kernel se = se_of(k);
  const int nt = cheb_terms(k);
  const double *amp = (const double *)(w + L.amp);
  const bool sym = U == V && ldu == ldv;
  const unsigned eb = (unsigned)((n * r + kRowsBlk - 1) / kRowsBlk);
  T *up = (T *)(w + L.up);
  T *vp = sym ? up : (T *)(w + L.vp);
  T *ku = (T *)(w + L.ku);
  T *kv = sym ? ku : (T *)(w + L.kv);
  cheb_scale<T><<<eb, kRowsBlk, 0, s>>>(n, r, amp, (const T *)U, ldu, up);
  if (!sym) cheb_scale<T><<<eb, kRowsBlk, 0, s>>>(n, r, amp, (const T *)V, ldv, vp);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return hip_fail(e, "Chebyshev scaling");
  double *gse = (double *)(w + L.gq);
  double *qse = gse + 3;
  // the SE pass: length-scale gradient, (D u_c)^T K~ (D v_c), K~ D U and K~ D V
  st = gp_quadform_grad(&se, n, X, (const double *)(w + L.th_se), r, up, r, vp, r, wgt, gse, qse,
                        ku, r, sym ? nullptr : kv, r, w + L.se, L.se_bytes, s);
  if (st) return st;
  const int no_noise = (k->flags & GP_NO_NOISE) ? 1 : 0;
  cheb_grad_rows<T><<<(unsigned)L.blocks, kRowsBlk, 0, s>>>(
      n, r, (const T *)X, k->d, k->n_cheb, nt, theta, nt + 2, no_noise, amp, (const T *)U, ldu,
      (const T *)V, ldv, wgt, ku, kv, (T *)AU, ldau, (T *)AV, ldav, (double *)(w + L.part));
  cheb_grad_final<<<1, 128, 0, s>>>(L.blocks, nt, r, (const double *)(w + L.part), gse, qse, wgt,
                                    theta, nt + 2, no_noise, grad, quad);
  e = hipGetLastError();
  return e == hipSuccess ? GP_OK : hip_fail(e, "Chebyshev gradient");
}

}  // namespace

int cheb_terms(const gp_kernel *k) {
  if (!k || k->n_cheb < 1 || k->d < 1) return -1;
  int64_t t = 1;
  for (int i = 0; i < k->d; ++i) {
    t *= k->n_cheb;
    if (t > kChebMaxTerms) return -1;
  }
  return (int)t;
}

size_t cheb_workspace_size(const gp_kernel *k, int64_t n, int r) {
  if (cheb_terms(k) < 0 || n < 1 || r < 1) return 0;
  return cheb_layout(k, n, r).total;
}

gp_status cheb_kmatvec(const gp_kernel *k, int64_t n, const void *X, const double *theta, int r,
                       const void *V, int64_t ldv, const double *col_shift, void *out,
                       int64_t ldo, void *ws, size_t ws_bytes, hipStream_t s) {
  const ChebLayout L = cheb_layout(k, n, r);
  if (!ws || ws_bytes < L.total)
    return fail(GP_ERR_WORKSPACE, "workspace of %zu bytes needed, %zu given", L.total,
                ws ? ws_bytes : (size_t)0);
  if (k->prec == GP_F64)
    return run_kmatvec<double>(k, n, X, theta, r, V, ldv, col_shift, out, ldo, (char *)ws, L, s);
  return run_kmatvec<float>(k, n, X, theta, r, V, ldv, col_shift, out, ldo, (char *)ws, L, s);
}

gp_status cheb_quadform_grad(const gp_kernel *k, int64_t n, const void *X, const double *theta,
                             int r, const void *U, int64_t ldu, const void *V, int64_t ldv,
                             const double *w, double *grad, double *quad, void *AU, int64_t ldau,
                             void *AV, int64_t ldav, void *ws, size_t ws_bytes, hipStream_t s) {
  const ChebLayout L = cheb_layout(k, n, r);
  if (!ws || ws_bytes < L.total)
    return fail(GP_ERR_WORKSPACE, "workspace of %zu bytes needed, %zu given", L.total,
                ws ? ws_bytes : (size_t)0);
  if (k->prec == GP_F64)
    return run_quadform<double>(k, n, X, theta, r, U, ldu, V, ldv, w, grad, quad, AU, ldau, AV,
                                ldav, (char *)ws, L, s);
  return run_quadform<float>(k, n, X, theta, r, U, ldu, V, ldv, w, grad, quad, AU, ldau, AV, ldav,
                             (char *)ws, L, s);
}

}  // namespace gpk
