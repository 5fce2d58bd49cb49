// Autotuner of the product kernels: for a problem class (operation, precision, kernel kind,
// padded d, padded R, log2 N) it times every candidate configuration (column splits x rows per
// wave of the matrix-core kernel) on synthetic inputs placed in the caller's workspace and
// keeps the fastest in a process-wide table, which gp_kmatvec / gp_quadform_grad consult.
// The table can be saved to and loaded from a small JSON file (one entry per line).
#include <stdio.h>
#include <string.h>

#include <map>
#include <mutex>
#include <tuple>
#include <vector>

#include "gpk.h"
#include "tune.h"

namespace gpk {

gp_status fail(gp_status st, const char *fmt, ...);
void clear_error();
gp_status hip_fail(hipError_t e, const char *where);

namespace {

std::mutex g_tmu;
std::map<std::tuple<int, int, int, int, int, int>, TuneCfg> g_table;
bool g_env_loaded = false;

std::tuple<int, int, int, int, int, int> as_tuple(const TuneKey &k) {
  return std::make_tuple(k.op, k.prec, k.kind, k.dp, k.rb, k.nb);
}

// Deterministic synthetic inputs: X uniform in [0,1)^d, V uniform in [-1,1).
__device__ __forceinline__ float hash01(uint64_t i) {
  uint64_t z = i * 0x9E3779B97F4A7C15ull + 0x632BE59BD9B4E019ull;
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  z ^= z >> 31;
  return (float)((z >> 40) * (1.0 / 16777216.0));
}

template <typename T>
__global__ void synth(T *a, int64_t m, float lo, float hi, uint64_t salt) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e < m) a[e] = (T)(lo + (hi - lo) * hash01((uint64_t)e + salt));
}

__global__ void synth_theta(double *th, int nth, double log_ell) {
  const int k = threadIdx.x;
  if (k < nth) th[k] = (k == 0) ? 0.0 : (k == nth - 1 ? -4.605170185988091 : log_ell);
}

// One table line (the format gp_tune_save writes); trajectory entries carry three more fields.
bool parse_entry(const char *line, TuneKey *k, TuneCfg *c) {
  int n = sscanf(line, " {\"op\": %d, \"prec\": %d, \"kind\": %d, \"dp\": %d, \"rb\": %d, "
                       "\"nb\": %d, \"splits\": %d, \"ib\": %d, \"ms\": %f, \"waves\": %d, "
                       "\"cpt_lo\": %d, \"cpt_hi\": %d}",
                 &k->op, &k->prec, &k->kind, &k->dp, &k->rb, &k->nb, &c->splits, &c->ib, &c->ms,
                 &c->waves, &c->cpt_lo, &c->cpt_hi);
  if (n < 9) return false;
  if (n < 12) c->waves = c->cpt_lo = c->cpt_hi = 0;
  if (k->op == 2) return c->waves >= 1 && c->waves <= 4;
  return c->splits >= 1 && (c->ib == 1 || c->ib == 2);
}

void load_env_once() {
  if (g_env_loaded) return;
  g_env_loaded = true;
  const char *p = getenv("GPK_TUNE_CACHE");
  if (!p || !*p) return;
  FILE *f = fopen(p, "r");
  if (!f) return;
  char line[512];
  while (fgets(line, sizeof(line), f)) {
    TuneKey k;
    TuneCfg c;
    if (parse_entry(line, &k, &c)) g_table[as_tuple(k)] = c;
  }
  fclose(f);
}

}  // namespace

TuneKey tune_key(int op, int prec, int kind, int d, int rpass, int64_t n) {
  TuneKey k;
  k.op = op;
  k.prec = prec;
  k.kind = kind;
  k.dp = padded_dim(d);
  k.rb = pow2_at_least(rpass < 1 ? 1 : rpass);
  int nb = 0;
  while (((int64_t)1 << (nb + 1)) <= n) ++nb;
  k.nb = nb;
  return k;
}

bool tune_lookup(const TuneKey &k, TuneCfg *out) {
  std::lock_guard<std::mutex> lock(g_tmu);
  load_env_once();
  auto it = g_table.find(as_tuple(k));
  if (it == g_table.end()) return false;
  *out = it->second;
  return true;
}

void tune_store(const TuneKey &k, const TuneCfg &c) {
  std::lock_guard<std::mutex> lock(g_tmu);
  load_env_once();
  g_table[as_tuple(k)] = c;
}

}  // namespace gpk

using namespace gpk;

extern "C" {

size_t gp_tune_workspace_size(const gp_kernel *k, int64_t n, int32_t r) {
  if (!k || n < 1 || r < 1 || k->kind == GP_SE_CHEB) return 0;
  const size_t es = k->prec == GP_F64 ? 8 : 4;
  const size_t prod = gp_workspace_size(k, n, r);
  if (prod == 0) return 0;
  size_t o = align256(prod);
  o += align256(es * (size_t)n * k->d);      // X
  o += 2 * align256(es * (size_t)n * r);     // V, out
  o += align256(sizeof(double) * (2 * (kMaxD + 2) + kMaxRPass));  // theta, grad, quad
  return o;
}

gp_status gp_tune_products(const gp_kernel *k, int64_t n, int32_t r, int32_t with_grad,
                           void *ws, size_t ws_bytes, hipStream_t stream) {
  clear_error();
  if (!k) return fail(GP_ERR_ARG, "kernel description is NULL");
  if (k->kind == GP_SE_CHEB)
    return fail(GP_ERR_UNSUPPORTED, "GP_SE_CHEB runs on the GP_SE_ISO kernels: tune those");
  if (n < 1 || r < 1) return fail(GP_ERR_SHAPE, "n and r must be >= 1");
  if (with_grad && r > kMaxRPass) return fail(GP_ERR_SHAPE, "r = %d > %d with gradient", r, kMaxRPass);
  const int32_t nth = gp_n_theta(k);
  if (nth < 0) return fail(GP_ERR_ARG, "invalid kernel description");
  if (with_grad && (k->flags & GP_NO_NOISE)) return fail(GP_ERR_ARG, "GP_NO_NOISE with gradient");
  const size_t need = gp_tune_workspace_size(k, n, r);
  if (need == 0) return fail(GP_ERR_UNSUPPORTED, "no product kernels for this description");
  if (!ws || ws_bytes < need)
    return fail(GP_ERR_WORKSPACE, "workspace of %zu bytes needed, %zu given", need,
                ws ? ws_bytes : (size_t)0);
  const size_t es = k->prec == GP_F64 ? 8 : 4;
  const size_t prod = gp_workspace_size(k, n, r);
  char *w = (char *)ws;
  char *X = w + align256(prod);
  char *V = X + align256(es * (size_t)n * k->d);
  char *O = V + align256(es * (size_t)n * r);
  double *th = (double *)(O + align256(es * (size_t)n * r));
  double *gq = th + kMaxD + 2;
  const int64_t mx = n * k->d, mv = n * r;
  const double log_ell = log(0.5 * pow((double)n, -1.0 / k->d) * 8.0);
  if (k->prec == GP_F64) {
    synth<double><<<(unsigned)((mx + 255) / 256), 256, 0, stream>>>((double *)X, mx, 0.f, 1.f, 1);
    synth<double><<<(unsigned)((mv + 255) / 256), 256, 0, stream>>>((double *)V, mv, -1.f, 1.f, 7);
  } else {
    synth<float><<<(unsigned)((mx + 255) / 256), 256, 0, stream>>>((float *)X, mx, 0.f, 1.f, 1);
    synth<float><<<(unsigned)((mv + 255) / 256), 256, 0, stream>>>((float *)V, mv, -1.f, 1.f, 7);
  }
  synth_theta<<<1, 128, 0, stream>>>(th, nth, log_ell);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return hip_fail(e, "tuner inputs");

  const int rpass = r < kMaxRPass ? r : kMaxRPass;
  const TuneKey key = tune_key(with_grad ? 1 : 0, k->prec, k->kind, k->d, rpass, n);
  const std::vector<TuneCfg> cands = tune_candidates(k, n, r, with_grad);
  hipEvent_t e0 = nullptr, e1 = nullptr;
  e = hipEventCreate(&e0);
  if (e == hipSuccess) e = hipEventCreate(&e1);
  if (e != hipSuccess) {
    if (e0) (void)hipEventDestroy(e0);
    return hip_fail(e, "tuner events");
  }
  auto cleanup = [&] {
    tune_force(nullptr);
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
  };
  TuneCfg best;
  best.ms = 1e30f;
  best.splits = 1;
  best.ib = 2;
  for (const TuneCfg &c : cands) {
    tune_force(&c);
    float ms_min = 1e30f;
    for (int rep = 0; rep < 2; ++rep) {
      e = hipEventRecord(e0, stream);
      gp_status st = GP_OK;
      if (e == hipSuccess) {
        if (with_grad)
          st = gp_quadform_grad(k, n, X, th, r, V, r, V, r, nullptr, gq, gq + nth, O, r, nullptr, 0,
                                ws, prod, stream);
        else
          st = gp_kmatvec(k, n, X, th, r, V, r, nullptr, O, r, ws, prod, stream);
      }
      if (st != GP_OK) {
        cleanup();
        return st;
      }
      if (e == hipSuccess) e = hipEventRecord(e1, stream);
      if (e == hipSuccess) e = hipEventSynchronize(e1);
      float ms = 0.f;
      if (e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
      if (e != hipSuccess) {
        cleanup();
        return hip_fail(e, "tuner timing");
      }
      if (rep > 0 && ms < ms_min) ms_min = ms;
    }
    if (ms_min < best.ms) {
      best = c;
      best.ms = ms_min;
    }
  }
  cleanup();
  tune_store(key, best);
  return GP_OK;
}

gp_status gp_tune_save(const char *path) {
  clear_error();
  if (!path) return fail(GP_ERR_ARG, "path is NULL");
  std::lock_guard<std::mutex> lock(g_tmu);
  FILE *f = fopen(path, "w");
  if (!f) return fail(GP_ERR_ARG, "cannot open %s for writing", path);
  fprintf(f, "{\"version\": 1, \"entries\": [\n");
  size_t i = 0;
  for (const auto &kv : g_table) {
    const auto &t = kv.first;
    const TuneCfg &c = kv.second;
    fprintf(f, " {\"op\": %d, \"prec\": %d, \"kind\": %d, \"dp\": %d, \"rb\": %d, \"nb\": %d, "
               "\"splits\": %d, \"ib\": %d, \"ms\": %.6f, \"waves\": %d, \"cpt_lo\": %d, "
               "\"cpt_hi\": %d}%s\n",
            std::get<0>(t), std::get<1>(t), std::get<2>(t), std::get<3>(t), std::get<4>(t),
            std::get<5>(t), c.splits, c.ib, c.ms, c.waves, c.cpt_lo, c.cpt_hi,
            ++i < g_table.size() ? "," : "");
  }
  fprintf(f, "]}\n");
  fclose(f);
  return GP_OK;
}

gp_status gp_tune_load(const char *path) {
  clear_error();
  if (!path) return fail(GP_ERR_ARG, "path is NULL");
  FILE *f = fopen(path, "r");
  if (!f) return fail(GP_ERR_ARG, "cannot open %s", path);
  std::lock_guard<std::mutex> lock(g_tmu);
  g_env_loaded = true;
  char line[512];
  int got = 0;
  while (fgets(line, sizeof(line), f)) {
    TuneKey k;
    TuneCfg c;
    if (parse_entry(line, &k, &c)) {
      g_table[as_tuple(k)] = c;
      ++got;
    }
  }
  fclose(f);
  (void)got;
  return GP_OK;
}

int32_t gp_tune_entries(void) {
  std::lock_guard<std::mutex> lock(g_tmu);
  return (int32_t)g_table.size();
}

void gp_tune_clear(void) {
  std::lock_guard<std::mutex> lock(g_tmu);
  g_table.clear();
  g_env_loaded = true;
}

}  // extern "C"
