// C ABI of libgpk: argument validation, workspace sizing and dispatch of the product kernels.
// Every argument check happens before the first HIP call of an entry point.
#include <stdarg.h>
#include <stdio.h>
#include <string.h>

#include "cheb.h"
#include "gpk.h"
#include "pass.h"
#include "tune.h"

namespace gpk {

static thread_local char g_err[512];

gp_status fail(gp_status st, const char *fmt, ...) {
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(g_err, sizeof(g_err), fmt, ap);
  va_end(ap);
  return st;
}

void clear_error() { g_err[0] = 0; }

gp_status hip_fail(hipError_t e, const char *where) {
  return fail(GP_ERR_HIP, "%s: %s", where, hipGetErrorString(e));
}

// Final fixed-order sum of the per-block records; grad receives the theta entries, quad the
// first nq column sums.
__global__ __launch_bounds__(256) void reduce_records(const double *rp, int64_t np,
                                                      const double *rf, int64_t nf, int nrec,
                                                      int nth, int L, double *grad, double *quad,
                                                      int nq) {
  // G (a power of two) groups of nrec threads: group g sums the records g, g + G, ... of the
  // pair blocks, then of the final blocks, with 8 loads in flight; then a pairwise tree over
  // the groups.  The order depends on nrec and the record counts only: deterministic.
  __shared__ double part[256];
  int G = 1;
  while (2 * G * nrec <= 256) G *= 2;
  const int t = threadIdx.x, g = t / nrec, e = t - g * nrec;
  double s = 0.0;
  if (g < G) {
    for (int pass = 0; pass < 2; ++pass) {
      const double *r = pass ? rf : rp;
      const int64_t m = pass ? nf : np;
      for (int64_t b0 = g; b0 < m; b0 += 8 * (int64_t)G) {
        double v[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) {
          const int64_t b = b0 + (int64_t)u * G;
          v[u] = b < m ? r[b * nrec + e] : 0.0;
        }
#pragma unroll
        for (int u = 0; u < 8; ++u) s += v[u];
      }
    }
  }
  part[t] = s;
  __syncthreads();
  for (int h = G / 2; h > 0; h /= 2) {
    if (g < h) part[t] += part[t + h * nrec];
    __syncthreads();
  }
  if (t >= nrec) return;
  s = part[t];
  if (t < nth) {
    const double f = (t >= 1 && t <= L) ? 2.0 * kLn2 : 1.0;
    if (grad) grad[t] = s * f;
  } else if (quad && t - nth < nq) {
    quad[t - nth] = s;
  }
}

// Operands of the one-pass form of sum_c w_c u_c^T A v_c with both A U and A V (U != V):
// Y = [U | V] and D = [V | U] (n x 2r), and the weights [w | 0].
template <typename T>
__global__ void pack_pair(int64_t n, int r, const T *U, int64_t ldu, const T *V, int64_t ldv,
                          T *Y, T *D) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= n * r) return;
  const int64_t i = e / r;
  const int c = (int)(e - i * r);
  const T u = U[i * ldu + c], v = V[i * ldv + c];
  Y[i * 2 * r + c] = u;
  Y[i * 2 * r + r + c] = v;
  D[i * 2 * r + c] = v;
  D[i * 2 * r + r + c] = u;
}

__global__ void pack_weights(int r, const double *w, double *w2) {
  const int c = threadIdx.x;
  if (c < r) {
    w2[c] = w ? w[c] : 1.0;
    w2[r + c] = 0.0;
  }
}

__global__ void fill_zero(double *a, int64_t m) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e < m) a[e] = 0.0;
}

hipError_t zero_doubles(double *a, int64_t m, hipStream_t s) {
  if (!a || m <= 0) return hipSuccess;
  fill_zero<<<(unsigned)((m + 255) / 256), 256, 0, s>>>(a, m);
  return hipGetLastError();
}

int64_t pair_blocks(const PassDesc &p) {
  const int rows = p.use_mfma == 2   ? xm_rows_per_block(p.P && p.kind != 0)
                   : p.use_mfma == 1 ? mfma_rows_per_block(p.kind, p.d, p.P ? 1 : 0, p.ib)
                                     : kRowsValu;
  return ((p.n + rows - 1) / rows) * p.splits;
}

int64_t fin_blocks(const PassDesc &p) {
  return p.splits > 1 ? (p.n + kThreads - 1) / kThreads : 0;
}

hipError_t launch_stage(int prec, const void *X, int64_t n, int d, int dp, int kind,
                        const double *theta, char *ws, const WsLayout &L, hipStream_t s) {
  if (prec == kF64) return launch_stage_f64(X, n, d, dp, kind, theta, ws, L, s);
  return launch_stage_f32(X, n, d, dp, kind, theta, ws, L, s);
}

hipError_t launch_pass(const PassDesc &p, hipStream_t s) {
  if (p.use_mfma == 2) return launch_pass_xm(p, s);
  if (p.use_mfma) return launch_pass_mfma(p, s);
  if (p.prec == kF64) return launch_pass_f64(p, s);
  return launch_pass_f32(p, s);
}

hipError_t launch_reduce(const PassDesc &p, double *grad, double *quad, hipStream_t s, int nq) {
  if (!grad && !quad) return hipSuccess;
  reduce_records<<<1, 256, 0, s>>>(p.rec_pair, pair_blocks(p), p.rec_fin, fin_blocks(p),
                                   p.nrec, p.nth, p.kind == 0 ? 1 : p.d, grad, quad,
                                   nq < 0 ? p.nrec - p.nth : nq);
  return hipGetLastError();
}

// ---- shared validation ------------------------------------------------------------------

static gp_status check_kernel(const gp_kernel *k, bool allow_no_noise) {
  if (!k) return fail(GP_ERR_ARG, "kernel description is NULL");
  if (k->kind != GP_SE_ISO && k->kind != GP_SE_ARD && k->kind != GP_SE_CHEB)
    return fail(GP_ERR_ARG, "kernel kind %d is not GP_SE_ISO, GP_SE_ARD or GP_SE_CHEB", k->kind);
  if (k->prec != GP_F64 && k->prec != GP_F32 && k->prec != GP_BF16X)
    return fail(GP_ERR_ARG, "precision %d is not GP_F64, GP_F32 or GP_BF16X", k->prec);
  if (k->d < 1 || k->d > kMaxD) return fail(GP_ERR_SHAPE, "d = %d outside 1..%d", k->d, kMaxD);
  if (k->flags & ~GP_NO_NOISE) return fail(GP_ERR_ARG, "unknown flag bits 0x%x", k->flags);
  if (!allow_no_noise && (k->flags & GP_NO_NOISE))
    return fail(GP_ERR_ARG, "GP_NO_NOISE is not accepted by this entry point");
  if (k->kind == GP_SE_CHEB && cheb_terms(k) < 0)
    return fail(GP_ERR_ARG, "GP_SE_CHEB needs n_cheb >= 1 with n_cheb^d <= 64 (n_cheb = %d, d = %d)",
                k->n_cheb, k->d);
  return GP_OK;
}

static int nth_of(const gp_kernel *k) {
  if (k->kind == GP_SE_CHEB) return cheb_terms(k) + 2;
  return k->kind == GP_SE_ISO ? 3 : k->d + 2;
}

static size_t elem_size(int prec) { return prec == GP_F64 ? sizeof(double) : sizeof(float); }

static bool overlap(const void *a, int64_t rows_a, int64_t ld_a, int cols_a, const void *b,
                    int64_t rows_b, int64_t ld_b, int cols_b, size_t es) {
  if (!a || !b) return false;
  const char *a0 = (const char *)a, *b0 = (const char *)b;
  const char *a1 = a0 + ((rows_a - 1) * ld_a + cols_a) * (int64_t)es;
  const char *b1 = b0 + ((rows_b - 1) * ld_b + cols_b) * (int64_t)es;
  return a0 < b1 && b0 < a1;
}

struct Plan {
  int dp;
  int rpass;
  int splits;
  int max_splits;
  int ib;
  int use_mfma;
  int nrec;
  WsLayout L;
};

// Largest column-split count a workspace is sized for: at most 64, at least kMinSplitCols
// columns per split, and at most 1 GiB of split partials.
static int max_splits_for(int64_t n, int rpass) {
  int64_t m = 64;
  if (n / kMinSplitCols < m) m = n / kMinSplitCols;
  const int64_t cap = ((int64_t)1 << 30) / (8 * n * (int64_t)rpass);
  if (cap < m) m = cap;
  return m < 1 ? 1 : (int)m;
}

static thread_local bool t_forced = false;
static thread_local TuneCfg t_force_cfg;

static WsLayout plan_layout(const gp_kernel *k, const Plan &pl, int64_t n) {
  const int rows_min = pl.use_mfma ? kRowsMfmaMin : kRowsValu;
  const int64_t pb = ((n + rows_min - 1) / rows_min) * pl.max_splits;
  const int64_t fb = pl.max_splits > 1 ? (n + kThreads - 1) / kThreads : 0;
  const size_t scr = pl.use_mfma == 2 ? xm_scratch_bytes(n, k->d)
                     : pl.use_mfma    ? mfma_scratch_bytes(n, pl.dp)
                                      : 0;
  return ws_layout(n, pl.dp, elem_size(k->prec), pl.rpass, pl.max_splits, pb, fb, pl.nrec, scr);
}

// Plan of a product pass.  With cap > 0 the workspace must fit in cap bytes: the column-split
// count (the only size that is a choice) is halved until it does; if one split does not fit,
// pl.L.total is left above cap.
static Plan make_plan(const gp_kernel *k, int64_t n, int r, int op, size_t cap = 0) {
  Plan pl;
  pl.dp = padded_dim(k->d);
  pl.rpass = r < kMaxRPass ? r : kMaxRPass;
  if (pl.rpass < 1) pl.rpass = 1;
  pl.use_mfma = k->prec == GP_BF16X ? 2 : (mfma_supported(k->prec, k->kind, k->d, pl.rpass) ? 1 : 0);
  const int rows = pl.use_mfma ? kRowsMfma : kRowsValu;
  pl.max_splits = max_splits_for(n, pl.rpass);
  pl.nrec = nth_of(k) + pl.rpass;
  if (cap > 0) {
    while (pl.max_splits > 1 && plan_layout(k, pl, n).total > cap) pl.max_splits /= 2;
  }
  pl.splits = choose_splits(n, rows);
  if (pl.splits > pl.max_splits) pl.splits = pl.max_splits;
  pl.ib = 2;
  TuneCfg c;
  bool have = false;
  if (t_forced) {
    c = t_force_cfg;
    have = true;
  } else if (op >= 0) {
    have = tune_lookup(tune_key(op, k->prec, k->kind, k->d, pl.rpass, n), &c);
  }
  if (have) {
    pl.splits = c.splits < 1 ? 1 : (c.splits > pl.max_splits ? pl.max_splits : c.splits);
    pl.ib = c.ib == 1 ? 1 : 2;
  }
  pl.L = plan_layout(k, pl, n);
  return pl;
}

static PassDesc base_desc(const gp_kernel *k, const Plan &pl, int64_t n, const double *theta,
                          char *ws) {
  PassDesc p;
  memset(&p, 0, sizeof(p));
  p.prec = k->prec == GP_F64 ? kF64 : kF32;
  p.kind = k->kind;
  p.d = k->d;
  p.dp = pl.dp;
  p.n = n;
  p.xs = ws + pl.L.xs;
  p.theta = theta;
  p.splits = pl.splits;
  p.outp = (double *)(ws + pl.L.outp);
  p.rec_pair = (double *)(ws + pl.L.rec_pair);
  p.rec_fin = (double *)(ws + pl.L.rec_fin);
  p.nth = nth_of(k);
  p.use_mfma = pl.use_mfma;
  p.mfma_scratch = ws + pl.L.scratch;
  p.ib = pl.ib;
  p.no_noise = (k->flags & GP_NO_NOISE) ? 1 : 0;
  return p;
}

// gp_quadform_grad with U != V and both A U and A V for 2r <= kMaxRPass runs one pass of 2r
// columns: its plan's workspace, then Y = [U | V], D = [V | U], the output [A U | A V] (n x 2r
// each) and the weights [w | 0].
static bool pair_pass(const gp_kernel *k, int r) { return k->kind != GP_SE_CHEB && 2 * r <= kMaxRPass; }

static size_t pair_pack_offset(const gp_kernel *k, int64_t n, int r) {
  return align256(make_plan(k, n, 2 * r, 1).L.total);
}

static size_t pair_pass_bytes(const gp_kernel *k, int64_t n, int r) {
  if (!pair_pass(k, r)) return 0;
  const size_t blk = align256(elem_size(k->prec) * (size_t)n * 2 * r);
  return pair_pack_offset(k, n, r) + 3 * blk + align256(sizeof(double) * 2 * r);
}

void tune_force(const TuneCfg *c) {
  t_forced = c != nullptr;
  if (c) t_force_cfg = *c;
}

std::vector<TuneCfg> tune_candidates(const gp_kernel *k, int64_t n, int r, int with_grad) {
  const Plan pl = make_plan(k, n, r, -1);
  std::vector<TuneCfg> out;
  const bool two = pl.use_mfma == 1 && mfma_ib(k->kind, k->d, with_grad, 2) == 2;
  for (int s = 1; s <= pl.max_splits; s *= 2) {
    for (int ib = two ? 1 : 2; ib <= 2; ++ib) {
      TuneCfg c;
      c.splits = s;
      c.ib = ib;
      c.ms = 0.f;
      out.push_back(c);
    }
  }
  return out;
}

}  // namespace gpk

using namespace gpk;

extern "C" {

const char *gp_last_error(void) { return g_err; }

const char *gp_status_string(gp_status s) {
  switch (s) {
    case GP_OK: return "GP_OK";
    case GP_ERR_ARG: return "GP_ERR_ARG";
    case GP_ERR_SHAPE: return "GP_ERR_SHAPE";
    case GP_ERR_UNSUPPORTED: return "GP_ERR_UNSUPPORTED";
    case GP_ERR_WORKSPACE: return "GP_ERR_WORKSPACE";
    case GP_ERR_HIP: return "GP_ERR_HIP";
    default: return "GP_UNKNOWN_STATUS";
  }
}

int32_t gp_n_theta(const gp_kernel *k) {
  if (check_kernel(k, true) != GP_OK) return -1;
  return nth_of(k);
}

size_t gp_workspace_size(const gp_kernel *k, int64_t n, int32_t r) {
  if (check_kernel(k, true) != GP_OK || n < 0 || r < 0) return 0;
  if (n == 0 || r == 0) return 0;
  if (k->kind == GP_SE_CHEB) return cheb_workspace_size(k, n, r);
  const size_t one = make_plan(k, n, r, -1).L.total;
  const size_t pair = pair_pass_bytes(k, n, r);
  return one > pair ? one : pair;
}

}  // extern "C"

namespace gpk {

// gp_kmatvec with the workspace planned to fit cap bytes (cap = 0: the full plan).  dry: every
// check (the workspace fit included, the workspace pointer excluded) and no HIP call.
gp_status kmatvec_run(const gp_kernel *k, int64_t n, const void *X, const double *theta,
                      int32_t r, const void *V, int64_t ldv, const double *col_shift, void *out,
                      int64_t ldo, void *ws, size_t ws_bytes, hipStream_t stream, size_t cap,
                      bool dry) {
  gp_status st = check_kernel(k, true);
  if (st) return st;
  if (n < 0) return fail(GP_ERR_SHAPE, "n = %lld < 0", (long long)n);
  if (r < 0) return fail(GP_ERR_SHAPE, "r = %d < 0", r);
  if (n == 0 || r == 0) return GP_OK;
  if (!X || !theta || !V || !out) return fail(GP_ERR_ARG, "X, theta, V and out must be non-NULL");
  if (ldv < r || ldo < r)
    return fail(GP_ERR_SHAPE, "leading dimensions ldv=%lld ldo=%lld must be >= r=%d",
                (long long)ldv, (long long)ldo, r);
  const size_t es = elem_size(k->prec);
  if (overlap(V, n, ldv, r, out, n, ldo, r, es)) return fail(GP_ERR_ARG, "out overlaps V");
  if (k->kind == GP_SE_CHEB) {
    if (cap > 0 && cheb_workspace_size(k, n, r) > cap)
      return fail(GP_ERR_WORKSPACE, "the product needs %zu bytes of workspace, the limit is %zu",
                  cheb_workspace_size(k, n, r), cap);
    if (dry) return GP_OK;
    return cheb_kmatvec(k, n, X, theta, r, V, ldv, col_shift, out, ldo, ws, ws_bytes, stream);
  }
  const Plan pl = make_plan(k, n, r, 0, cap);
  if (cap > 0 && pl.L.total > cap)
    return fail(GP_ERR_WORKSPACE, "the product needs %zu bytes of workspace, the limit is %zu",
                pl.L.total, cap);
  if (dry) return GP_OK;
  if (!ws || ws_bytes < pl.L.total)
    return fail(GP_ERR_WORKSPACE, "workspace of %zu bytes needed, %zu given", pl.L.total,
                ws ? ws_bytes : (size_t)0);
  char *w = (char *)ws;
  hipError_t e = launch_stage(k->prec == GP_F64 ? kF64 : kF32, X, n, k->d, pl.dp, k->kind, theta,
                              w, pl.L, stream);
  if (e != hipSuccess) return hip_fail(e, "stage");
  for (int c0 = 0; c0 < r; c0 += pl.rpass) {
    const int rc = r - c0 < pl.rpass ? r - c0 : pl.rpass;
    PassDesc p = base_desc(k, pl, n, theta, w);
    p.R = rc;
    p.nrec = nth_of(k) + rc;
    // GP_BF16X runs every chunk on its cross-term kernel; for the fp16-split kernel a narrow
    // trailing chunk runs on the VALU kernel (same rows per block and split count)
    p.use_mfma = pl.use_mfma == 2 ? 2 : (mfma_supported(k->prec, k->kind, k->d, rc) ? pl.use_mfma : 0);
    p.Y = (const char *)V + c0 * es;
    p.ldy = ldv;
    p.col_shift = col_shift ? col_shift + c0 : nullptr;
    p.no_noise = (k->flags & GP_NO_NOISE) ? 1 : 0;
    p.out = (char *)out + c0 * es;
    p.ldo = ldo;
    e = launch_pass(p, stream);
    if (e != hipSuccess) return hip_fail(e, "kmatvec pass");
  }
  return GP_OK;
}

}  // namespace gpk

extern "C" {

gp_status gp_kmatvec(const gp_kernel *k, int64_t n, const void *X, const double *theta,
                     int32_t r, const void *V, int64_t ldv, const double *col_shift, void *out,
                     int64_t ldo, void *ws, size_t ws_bytes, hipStream_t stream) {
  clear_error();
  return kmatvec_run(k, n, X, theta, r, V, ldv, col_shift, out, ldo, ws, ws_bytes, stream, 0,
                     false);
}

gp_status gp_quadform_grad(const gp_kernel *k, int64_t n, const void *X, const double *theta,
                           int32_t r, const void *U, int64_t ldu, const void *V, int64_t ldv,
                           const double *w, double *grad_theta, double *quad, void *AU,
                           int64_t ldau, void *AV, int64_t ldav, void *ws, size_t ws_bytes,
                           hipStream_t stream) {
  clear_error();
  gp_status st = check_kernel(k, true);
  if (st) return st;
  if (n < 0) return fail(GP_ERR_SHAPE, "n = %lld < 0", (long long)n);
  if (r < 1 || r > kMaxRPass) return fail(GP_ERR_SHAPE, "r = %d outside 1..%d", r, kMaxRPass);
  if (!grad_theta && !quad && !AU && !AV)
    return fail(GP_ERR_ARG, "at least one of grad_theta, quad, AU, AV must be non-NULL");
  if (n == 0) {
    // empty point set: Q = 0 and its gradient is 0
    hipError_t e = zero_doubles(grad_theta, nth_of(k), stream);
    if (e == hipSuccess) e = zero_doubles(quad, r, stream);
    if (e != hipSuccess) return hip_fail(e, "zero fill");
    return GP_OK;
  }
  if (!X || !theta || !U || !V) return fail(GP_ERR_ARG, "X, theta, U and V must be non-NULL");
  if (ldu < r || ldv < r || (AU && ldau < r) || (AV && ldav < r))
    return fail(GP_ERR_SHAPE, "a leading dimension is smaller than r=%d", r);
  const size_t es = elem_size(k->prec);
  const bool sym = (U == V && ldu == ldv);
  if (overlap(AU, n, ldau, r, U, n, ldu, r, es) || overlap(AU, n, ldau, r, V, n, ldv, r, es) ||
      overlap(AV, n, ldav, r, U, n, ldu, r, es) || overlap(AV, n, ldav, r, V, n, ldv, r, es) ||
      overlap(AU, n, ldau, r, AV, n, ldav, r, es))
    return fail(GP_ERR_ARG, "an output overlaps an input or the other output");
  if (k->kind == GP_SE_CHEB)
    return cheb_quadform_grad(k, n, X, theta, r, U, ldu, V, ldv, w, grad_theta, quad, AU, ldau,
                              AV, ldav, ws, ws_bytes, stream);
  const bool both = !sym && AU && AV && pair_pass(k, r);
  const Plan pl = make_plan(k, n, both ? 2 * r : r, 1);
  const size_t need = both ? pair_pass_bytes(k, n, r) : pl.L.total;
  if (!ws || ws_bytes < need)
    return fail(GP_ERR_WORKSPACE, "workspace of %zu bytes needed, %zu given", need,
                ws ? ws_bytes : (size_t)0);
  char *wsp = (char *)ws;
  hipError_t e = launch_stage(k->prec == GP_F64 ? kF64 : kF32, X, n, k->d, pl.dp, k->kind,
                              theta, wsp, pl.L, stream);
  if (e != hipSuccess) return hip_fail(e, "stage");

  if (both) {
    // one pass of 2r columns: Y = P = [U | V], D = Q = [V | U], weights [w | 0]; then
    // S_ij = sum_c w_c u_ic v_jc, q_c = v_c^T (A u_c) for c < r, the sigma^2 term
    // sigma^2 sum_c w_c u_c . v_c, and the product [A U | A V]
    const size_t blk = align256(es * (size_t)n * 2 * r);
    char *Y2 = wsp + pair_pack_offset(k, n, r);
    char *D2 = Y2 + blk, *O2 = D2 + blk;
    double *w2 = (double *)(O2 + blk);
    const unsigned eb = (unsigned)((n * r + 255) / 256);
    if (k->prec == GP_F64)
      pack_pair<double><<<eb, 256, 0, stream>>>(n, r, (const double *)U, ldu, (const double *)V,
                                                ldv, (double *)Y2, (double *)D2);
    else
      pack_pair<float><<<eb, 256, 0, stream>>>(n, r, (const float *)U, ldu, (const float *)V, ldv,
                                               (float *)Y2, (float *)D2);
    pack_weights<<<1, 64, 0, stream>>>(r, w, w2);
    e = hipGetLastError();
    if (e != hipSuccess) return hip_fail(e, "pack");
    PassDesc p = base_desc(k, pl, n, theta, wsp);
    p.R = 2 * r;
    p.nrec = nth_of(k) + 2 * r;
    p.P = p.Y = Y2;
    p.Q = p.D = D2;
    p.ldp = p.ldq = p.ldy = p.ldd = 2 * r;
    p.w = w2;
    p.out = O2;
    p.ldo = 2 * r;
    e = launch_pass(p, stream);
    if (e != hipSuccess) return hip_fail(e, "quadform pass");
    e = launch_reduce(p, grad_theta, quad, stream, r);
    if (e != hipSuccess) return hip_fail(e, "reduce");
    e = hipMemcpy2DAsync(AU, ldau * es, O2, 2 * r * es, r * es, n, hipMemcpyDeviceToDevice, stream);
    if (e == hipSuccess)
      e = hipMemcpy2DAsync(AV, ldav * es, O2 + r * es, 2 * r * es, r * es, n,
                           hipMemcpyDeviceToDevice, stream);
    return e == hipSuccess ? GP_OK : hip_fail(e, "copy A U, A V");
  }

  // Pass 1: gradient, q_c and one of the products.  Y is the operand whose product is wanted;
  // D is the other operand, so q_c = sum_i D_ic (A Y)_ic = u_c^T A v_c either way.
  PassDesc p = base_desc(k, pl, n, theta, wsp);
  p.R = r;
  p.nrec = nth_of(k) + r;
  p.P = U;
  p.ldp = ldu;
  p.Q = V;
  p.ldq = ldv;
  p.w = w;
  if (sym) {
    p.Y = U;
    p.ldy = ldu;
    p.D = U;
    p.ldd = ldu;
    p.out = AU ? AU : AV;
    p.ldo = AU ? ldau : ldav;
  } else if (AV && !AU) {
    p.Y = V;
    p.ldy = ldv;
    p.D = U;
    p.ldd = ldu;
    p.out = AV;
    p.ldo = ldav;
  } else {
    p.Y = U;
    p.ldy = ldu;
    p.D = V;
    p.ldd = ldv;
    p.out = AU;
    p.ldo = ldau;
  }
  e = launch_pass(p, stream);
  if (e != hipSuccess) return hip_fail(e, "quadform pass");
  e = launch_reduce(p, grad_theta, quad, stream);
  if (e != hipSuccess) return hip_fail(e, "reduce");
  if (sym && AU && AV) {
    e = hipMemcpy2DAsync(AV, ldav * es, AU, ldau * es, r * es, n, hipMemcpyDeviceToDevice,
                         stream);
    if (e != hipSuccess) return hip_fail(e, "copy AU -> AV");
  } else if (!sym && AU && AV) {
    // r > kMaxRPass / 2: pass 2, the second product without gradient sums.
    PassDesc q = base_desc(k, pl, n, theta, wsp);
    q.R = r;
    q.nrec = nth_of(k) + r;
    q.Y = V;
    q.ldy = ldv;
    q.out = AV;
    q.ldo = ldav;
    e = launch_pass(q, stream);
    if (e != hipSuccess) return hip_fail(e, "quadform second product");
  }
  return GP_OK;
}

}  // extern "C"
