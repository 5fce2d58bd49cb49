// gp_hmc_leapfrog host side: validation, workspace layout, per-chain descriptors and the three
// schedulers (plain per-op launches, one persistent launch, a captured graph of it).
#include <string.h>

#include <algorithm>
#include <cmath>
#include <map>
#include <mutex>
#include <numeric>
#include <vector>

#include "gpk.h"
#include "hmc.h"
#include "tune.h"

namespace gpk {

gp_status fail(gp_status st, const char *fmt, ...);
void clear_error();
gp_status hip_fail(hipError_t e, const char *where);

hipError_t hmc_kickoff_f32(void *, int, const HmcRunParams &, const HmcQueue &, int, hipStream_t);
hipError_t hmc_kickoff_f64(void *, int, const HmcRunParams &, const HmcQueue &, int, hipStream_t);
hipError_t hmc_tiles_f32(void *, int, int, int, int, int, hipStream_t);
hipError_t hmc_tiles_f64(void *, int, int, int, int, int, hipStream_t);
hipError_t hmc_epilogue_f32(void *, const HmcRunParams &, int, hipStream_t);
hipError_t hmc_epilogue_f64(void *, const HmcRunParams &, int, hipStream_t);
hipError_t hmc_gather_f32(void *, int, int, hipStream_t);
hipError_t hmc_gather_f64(void *, int, int, hipStream_t);
hipError_t hmc_persistent_f32(void *, int, const HmcRunParams &, const HmcQueue &, int, long long,
                              int, int, int, int, int, hipStream_t);
hipError_t hmc_persistent_f64(void *, int, const HmcRunParams &, const HmcQueue &, int, long long,
                              int, int, int, int, int, hipStream_t);
hipError_t hmc_reset_f32(const HmcQueue &, hipStream_t);
hipError_t hmc_reset_f64(const HmcQueue &, hipStream_t);
hipError_t hmc_check_f32(void *, int, hipStream_t);
hipError_t hmc_check_f64(void *, int, hipStream_t);
hipError_t hmc_phi_poles_f32(void *, int, const HmcRunParams &, hipStream_t);
hipError_t hmc_phi_poles_f64(void *, int, const HmcRunParams &, hipStream_t);

namespace {

// Launch configuration of the batched and graph modes: waves per SIMD of the persistent kernel
// (0: hmc_waves_default) and the product jobs' columns per trip for chains with padded d <= 8
// and above (0: the default of the tile).  The autotuner forces one on its own thread while it
// times the candidates; otherwise the tuning table's entry for the batch's class, if any.
struct LaunchCfg {
  int waves = 0, cpt_lo = 0, cpt_hi = 0;
};
thread_local const LaunchCfg *tl_force = nullptr;

struct InstInfo {
  int64_t n, off, xoff;
  int d, dp, nth;
  int64_t tofs;  // sum of n_theta over the instances before this one
};

constexpr int kMaxPrecondRank = kHmcMaxRank;

struct ChainLayout {
  size_t hdr_word, hdr_fin, hdr_cnt, hdr_order, chains;
  std::vector<size_t> per_chain;  // offset of each chain's region
  std::vector<int> n_rb, n_cs;
  size_t total;
};

size_t chain_bytes(int prec) { return prec == GP_F64 ? sizeof(HmcChain<double>) : sizeof(HmcChain<float>); }

// Padded cross-term width of a GP_BF16X chain (its jobs run on the matrix-core tiles), else 0.
int xm_width(int prec, int d) { return prec == GP_BF16X ? xmt::dpx_of(d) : 0; }

// Row blocks of a chain's jobs: 256-row tiles, or the 64-row stage / force-pass blocks of a
// GP_BF16X chain (its 128-row product jobs use the first half of the ids).
int64_t row_blocks(int64_t n, int xm) {
  const int64_t rows = xm ? xmt::kRowsStage : kHmcTile;
  return (n + rows - 1) / rows;
}

template <int DPX>
size_t xm_bytes(int64_t n_rb, int ard) {
  using G = xmt::Geo<DPX>;
  const int64_t nrow = n_rb * xmt::kRowsStage;
  size_t o = 2 * align256(2 * (size_t)nrow * G::XSTR);            // xh, xl
  o += align256(4 * (size_t)nrow);                               // nrm
  if (ard) o += align256((size_t)(nrow / xmt::TJ) * G::kBB);  // bimg
  return o;
}

constexpr int kPlainCheck = 4;  // plain mode: jobs between host checks of a tile chain

int plain_splits(int64_t n) {
  const int64_t rb = (n + kHmcTile - 1) / kHmcTile;
  int64_t s = (1024 + rb - 1) / rb;
  const int64_t smax = std::max<int64_t>(1, n / 512);
  s = std::min<int64_t>(std::min<int64_t>(s, smax), 64);
  return (int)std::max<int64_t>(1, s);
}

// Persistent launches: a batch with fewer row-block jobs than kSplitTarget splits every product
// and force-pass job's columns (at most kMaxSplits ways, at least kMinSplitCols columns each)
// until it has about that many, so a few chains still fill the GPU (one FP64 row-block job of a
// 3000-point chain is ~150 us of one workgroup).  Not for GP_BF16X chains (their jobs take no
// splits).  The split partials are summed in the chain's epilogue, or for preconditioned chains
// (whose row-block partials of U^T w need the complete q) by a gather job over the row blocks,
// which costs a scheduling round per CG iteration and so is used only from kMinPcSplits splits
// on (with 2 splits the 32-chain float batch ran 170 -> 137 chain-steps/s).  The epilogue's
// latency grows with the split count: on 10 FP64 chains of 3000 points a multi-shift iteration took 429 / 263 / 204 /
// 287 / 333 / 370 us with at most 1 / 2 / 4 / 6 / 8 / 16 splits, a CG iteration 379 / 209 / 224 /
// 230 / 259 / 312 us.  The target: 32 float chains of 6k-19k points (about 1,500 row blocks) ran
// 20-step trajectories at 107.7 / 137.6 / 130.7 / 126.1 chain-steps/s with 1 / 2 / 3 / 4 splits
// (the splits shorten the end of the launch, when only the largest chains still have jobs).
constexpr int64_t kSplitTarget = 4096;
constexpr int kMaxSplits = 4;
constexpr int64_t kMinSplitCols = 256;
constexpr int kMinPcSplits = 4;

int persistent_splits(const std::vector<InstInfo> &inst, int chains, int prec, int prank) {
  int64_t jobs = 0;
  for (const InstInfo &in : inst) {
    if (xm_width(prec, in.d)) return 1;
    jobs += row_blocks(in.n, 0) * chains;
  }
  const int s = (int)std::max<int64_t>(1, std::min<int64_t>(kMaxSplits, kSplitTarget / std::max<int64_t>(1, jobs)));
  return prank > 0 && s < kMinPcSplits ? 1 : s;
}

// Per-chain workspace; np > 0: a refresh of phi with np poles (shifted directions and pole state).
size_t region_bytes(const InstInfo &in, int prec, int kind, int n_cs, int prank, int np) {
  const size_t es = prec == GP_F64 ? 8 : 4;
  const int64_t n = in.n;
  const int xm = xm_width(prec, in.d);
  const int n_rb = (int)row_blocks(n, xm);
  size_t o = 0;
  if (xm) o += xm == 64 ? xm_bytes<64>(n_rb, kind == GP_SE_ARD) : xm_bytes<32>(n_rb, kind == GP_SE_ARD);
  o += align256(es * n * in.dp);     // xs
  o += 4 * align256(es * n);         // r, p, q, x0
  o += align256(es * 2 * n);         // Z
  o += align256(es * n);             // lc (Chebyshev-amplitude log2 amplitudes)
  if (n_cs > 1) o += align256(sizeof(double) * n_cs * n);
  o += align256(sizeof(double) * (size_t)n_rb * n_cs * kHmcRec);
  if (prank > 0) o += align256(sizeof(double) * (size_t)(2 * n_rb + 2) * prank);  // pgp, pg, ph
  if (np > 0) o += align256(es * (size_t)np * n) + align256(sizeof(double) * kPst * np);  // ps, pst
  return o;
}

ChainLayout make_layout(const std::vector<InstInfo> &inst, int chains, int prec, int mode,
                        int kind, int n_cheb, int prank, int np = 0) {
  ChainLayout L;
  const int nc = (int)inst.size() * chains;
  size_t o = 0;
  L.hdr_word = o;
  o = align256(o + 8 * (size_t)nc);
  L.hdr_fin = o;
  o = align256(o + 4 * (size_t)nc);
  L.hdr_cnt = o;
  o = align256(o + 16);
  L.hdr_order = o;
  o = align256(o + 4 * (size_t)nc);
  L.chains = o;
  o = align256(o + chain_bytes(prec) * (size_t)nc);
  const int ps = persistent_splits(inst, chains, prec, prank);
  for (const InstInfo &in : inst) {
    const int xm = xm_width(prec, in.d);
    int n_cs = 1;
    if (!xm) n_cs = mode == GP_HMC_PLAIN ? plain_splits(in.n) : std::min<int64_t>(ps, std::max<int64_t>(1, in.n / kMinSplitCols));
    const int n_rb = (int)row_blocks(in.n, xm);
    for (int h = 0; h < chains; ++h) {
      L.per_chain.push_back(o);
      L.n_rb.push_back(n_rb);
      L.n_cs.push_back(n_cs);
      o += region_bytes(in, prec, kind, n_cs, prank, np);
    }
  }
  (void)n_cheb;
  L.total = o;
  return L;
}

gp_status collect(const gp_kernel *k, const gp_hmc_params *p, const gp_batch *b,
                  std::vector<InstInfo> &inst) {
  if (!k) return fail(GP_ERR_ARG, "kernel description is NULL");
  if (k->kind != GP_SE_ISO && k->kind != GP_SE_ARD && k->kind != GP_SE_CHEB)
    return fail(GP_ERR_ARG, "bad kernel kind");
  if (k->prec != GP_F64 && k->prec != GP_F32 && k->prec != GP_BF16X)
    return fail(GP_ERR_ARG, "precision %d is not GP_F64, GP_F32 or GP_BF16X", k->prec);
  if (k->flags != 0) return fail(GP_ERR_ARG, "kernel flags must be 0 for gp_hmc_leapfrog");
  if (!p) return fail(GP_ERR_ARG, "params are NULL");
  if (p->n_steps < 0) return fail(GP_ERR_ARG, "n_steps < 0");
  if (!(p->cg_tol > 0.0)) return fail(GP_ERR_ARG, "cg_tol must be > 0");
  if (p->cg_maxit < 1) return fail(GP_ERR_ARG, "cg_maxit must be >= 1");
  if (p->mode != GP_HMC_PLAIN && p->mode != GP_HMC_BATCHED && p->mode != GP_HMC_GRAPH)
    return fail(GP_ERR_ARG, "unknown mode %d", p->mode);
  if (k->prec == GP_BF16X && k->kind == GP_SE_CHEB)
    return fail(GP_ERR_UNSUPPORTED,
                "GP_BF16X trajectories take GP_SE_ISO or GP_SE_ARD (the Chebyshev-amplitude kernel "
                "has d <= 6, where the cross term gains nothing)");
  if (k->prec == GP_BF16X && p->precond_rank > 0)
    return fail(GP_ERR_UNSUPPORTED, "GP_BF16X trajectories take no preconditioner");
  if (!b) return fail(GP_ERR_ARG, "batch is NULL");
  if (b->n_inst < 1 || b->chains_per_inst < 1)
    return fail(GP_ERR_SHAPE, "n_inst and chains_per_inst must be >= 1");
  if (!b->n_points || !b->offsets) return fail(GP_ERR_ARG, "n_points and offsets are required");
  if (p->precond_rank < 0 || p->precond_rank > kMaxPrecondRank)
    return fail(GP_ERR_ARG, "precond_rank = %d outside 0..%d", p->precond_rank, kMaxPrecondRank);
  if (p->precond_rank > 0 && (!p->precond_U || !p->precond_lam))
    return fail(GP_ERR_ARG, "precond_U and precond_lam are required when precond_rank > 0");
  inst.clear();
  int64_t xo = 0, tofs = 0;
  for (int i = 0; i < b->n_inst; ++i) {
    InstInfo in;
    in.n = b->n_points[i];
    in.off = b->offsets[i];
    in.d = b->d ? b->d[i] : k->d;
    if (in.n < 1) return fail(GP_ERR_SHAPE, "instance %d has n = %lld", i, (long long)in.n);
    if (in.off < 0) return fail(GP_ERR_SHAPE, "instance %d has a negative offset", i);
    if (in.d < 1 || in.d > kMaxD) return fail(GP_ERR_SHAPE, "instance %d has d = %d", i, in.d);
    in.dp = padded_dim(in.d);
    if (k->kind == GP_SE_CHEB) {
      gp_kernel kk = *k;
      kk.d = in.d;
      const int32_t nt = gp_n_theta(&kk);
      if (nt < 0)
        return fail(GP_ERR_ARG, "instance %d: n_cheb = %d with d = %d gives more than 64 terms", i,
                    k->n_cheb, in.d);
      in.nth = nt;
    } else {
      in.nth = k->kind == GP_SE_ISO ? 3 : in.d + 2;
    }
    in.xoff = b->x_offsets ? b->x_offsets[i] : in.off * in.d;
    if (in.xoff < 0) return fail(GP_ERR_SHAPE, "instance %d has a negative x offset", i);
    if (p->precond_rank > in.n)
      return fail(GP_ERR_SHAPE, "precond_rank %d exceeds instance %d's %lld points",
                  p->precond_rank, i, (long long)in.n);
    in.tofs = tofs;
    if (p->inv_mass) {
      for (int t = 0; t < in.nth; ++t) {
        const double m = p->inv_mass[tofs + t];
        if (!(m >= 0.0) || !std::isfinite(m))
          return fail(GP_ERR_ARG, "inv_mass[%lld] = %g is not finite and >= 0",
                      (long long)(tofs + t), m);
      }
    }
    tofs += in.nth;
    (void)xo;
    inst.push_back(in);
  }
  // row ranges must not overlap
  std::vector<int> idx(inst.size());
  std::iota(idx.begin(), idx.end(), 0);
  std::sort(idx.begin(), idx.end(), [&](int a, int c) { return inst[a].off < inst[c].off; });
  for (size_t t = 1; t < idx.size(); ++t)
    if (inst[idx[t - 1]].off + inst[idx[t - 1]].n > inst[idx[t]].off)
      return fail(GP_ERR_ARG, "row ranges of instances %d and %d overlap", idx[t - 1], idx[t]);
  return GP_OK;
}

// Arguments of the refresh of phi (chain program kProgPhi); null for trajectories.
struct PhiArgs {
  const gp_phi_params *pp;
  const void *xi;
  void *phi;
  double *bounds;
};

template <class P>
P *at(P *base, int64_t off) {
  return base ? base + off : nullptr;
}

template <typename T>
void fill_chains(const std::vector<InstInfo> &inst, int kind, int n_cheb, int chains,
                 const ChainLayout &L,
                 char *ws, const gp_hmc_params *p,
                 const void *X, const void *y, const void *phi, double *theta, double *pi,
                 void *x_warm, const double *u, double *H0, double *H1, int32_t *acc,
                 int32_t *status, int32_t *iters, int prec, const LaunchCfg &cfg,
                 const PhiArgs *pa, std::vector<HmcChain<T>> &out) {
  out.assign(inst.size() * chains, HmcChain<T>());
  int64_t tofs = 0;
  int c = 0;
  for (size_t b = 0; b < inst.size(); ++b) {
    const InstInfo &in = inst[b];
    for (int h = 0; h < chains; ++h, ++c) {
      HmcChain<T> &ch = out[c];
      memset(&ch, 0, sizeof(ch));
      ch.X = (const T *)X + in.xoff;
      ch.y = at((const T *)y, in.off);
      const int64_t vo = (int64_t)chains * in.off + (int64_t)h * in.n;
      ch.phi = at((const T *)phi, vo);
      ch.x = at((T *)x_warm, vo);
      const int64_t to = (int64_t)chains * tofs + (int64_t)h * in.nth;
      ch.theta = theta + to;
      ch.pi = at(pi, to);
      ch.u = at(u, c);
      ch.H0out = at(H0, c);
      ch.H1out = at(H1, c);
      ch.acc_out = at(acc, c);
      ch.status_out = status + c;
      ch.iters_out = at(iters, c);
      if (pa) {
        ch.prog = kProgPhi;
        ch.xi = (const T *)pa->xi + vo;
        ch.phio = (T *)pa->phi + vo;
        ch.bounds_out = at(pa->bounds, 2 * (int64_t)c);
      }
      for (int t = 0; t < in.nth; ++t) ch.minv[t] = p->inv_mass ? p->inv_mass[in.tofs + t] : 1.0;
      ch.prank = p->precond_rank;
      if (ch.prank > 0) {
        ch.pU = (const T *)p->precond_U + in.off * (int64_t)ch.prank;
        ch.plam = p->precond_lam + (int64_t)b * ch.prank;
      }
      ch.n = in.n;
      ch.d = in.d;
      ch.dp = in.dp;
      ch.kind = kind;
      ch.nth = in.nth;
      char *r = ws + L.per_chain[c];
      const size_t es = sizeof(T);
      const int64_t n = in.n;
      ch.xm = xm_width(prec, in.d);
      if (ch.xm) {
        const int64_t nrow = (int64_t)L.n_rb[c] * xmt::kRowsStage;
        const int xstr = ch.xm + 8;
        const int kbb = ch.xm == 64 ? xmt::Geo<64>::kBB : xmt::Geo<32>::kBB;
        ch.xh = (uint16_t *)r;
        r += align256(2 * (size_t)nrow * xstr);
        ch.xl = (uint16_t *)r;
        r += align256(2 * (size_t)nrow * xstr);
        ch.nrm = (float *)r;
        r += align256(4 * (size_t)nrow);
        if (kind == GP_SE_ARD) {
          ch.bimg = (uint16_t *)r;
          r += align256((size_t)(nrow / xmt::TJ) * kbb);
        }
      }
      ch.xs = (T *)r;
      r += align256(es * n * in.dp);
      const size_t vb = align256(es * n);
      ch.r = (T *)r;
      ch.p = (T *)(r + vb);
      ch.q = (T *)(r + 2 * vb);
      ch.x0 = (T *)(r + 3 * vb);
      r += 4 * vb;
      ch.Z = (T *)r;
      r += align256(es * 2 * n);
      ch.lc = (T *)r;
      r += align256(es * n);
      ch.ncheb = kind == GP_SE_CHEB ? n_cheb : 0;
      ch.n_rb = L.n_rb[c];
      ch.n_cs = L.n_cs[c];
      ch.cpt = in.dp <= 8 ? cfg.cpt_lo : cfg.cpt_hi;
      ch.n_jobs = ch.n_rb * ch.n_cs;
      ch.col_chunk = (n + ch.n_cs - 1) / ch.n_cs;
      if (ch.n_cs > 1) {
        ch.qpart = (double *)r;
        r += align256(sizeof(double) * ch.n_cs * n);
      }
      ch.rec = (double *)r;
      r += align256(sizeof(double) * (size_t)ch.n_jobs * kHmcRec);
      if (ch.prank > 0) {
        ch.pgp = (double *)r;
        ch.pg = ch.pgp + (size_t)2 * ch.n_rb * ch.prank;
        ch.ph = ch.pg + ch.prank;
        r += align256(sizeof(double) * (size_t)(2 * ch.n_rb + 2) * ch.prank);
      }
      if (pa) {
        const int np = pa->pp->n_poles;
        ch.ps = (T *)r;
        r += align256(es * (size_t)np * n);
        ch.pst = (double *)r;
        r += align256(sizeof(double) * kPst * np);
      }
    }
    tofs += in.nth;
  }
}

struct GraphEntry {
  std::vector<char> key;
  hipGraphExec_t exec = nullptr;
};

std::mutex g_mu;
std::map<void *, std::vector<char>> g_uploaded;  // ws -> descriptor bytes last uploaded
std::map<void *, GraphEntry> g_graphs;           // ws -> captured trajectory

// Class of a batch in the tuning table: precision, kind, largest padded d, kernel variant and
// floor(log2) of the number of chains (in rb, above the variant bits), floor(log2) of the
// largest instance.
TuneKey traj_key(const gp_kernel *k, const std::vector<InstInfo> &inst, int chains, int pc) {
  TuneKey key;
  key.op = 2;
  key.prec = k->prec;
  key.kind = k->kind;
  int dpmax = 4;
  int64_t nmax = 1;
  for (const InstInfo &in : inst) {
    dpmax = std::max(dpmax, in.dp);
    nmax = std::max(nmax, in.n);
  }
  key.dp = dpmax;
  int cb = 0;
  while (((int64_t)1 << (cb + 1)) <= (int64_t)inst.size() * chains) ++cb;
  key.rb = (pc ? 1 : 0) | (k->kind == GP_SE_CHEB ? 2 : 0) | (k->prec == GP_BF16X ? 4 : 0) | (cb << 3);
  int nb = 0;
  while (((int64_t)1 << (nb + 1)) <= nmax) ++nb;
  key.nb = nb;
  return key;
}

}  // namespace
}  // namespace gpk

using namespace gpk;

extern "C" {

size_t gp_hmc_workspace_size(const gp_kernel *k, const gp_hmc_params *p, const gp_batch *b) {
  std::vector<InstInfo> inst;
  if (collect(k, p, b, inst) != GP_OK) return 0;
  return make_layout(inst, b->chains_per_inst, k->prec, p->mode, k->kind, k->n_cheb,
                     p->precond_rank).total;
}

// One trajectory (rwm = 0) or one random-walk Metropolis update (rwm = 1) of every chain.
static gp_status run_chains(const gp_kernel *k, const gp_hmc_params *p, const gp_batch *b,
                            const void *X, const void *y, const void *phi, double *theta,
                            double *pi, void *x_warm, const double *u_accept, double *H0,
                            double *H1, int32_t *accepted, int32_t *status, int32_t *cg_iters,
                            void *ws, size_t ws_bytes, hipStream_t stream, int rwm,
                            const PhiArgs *pa = nullptr) {
  std::vector<InstInfo> inst;
  gp_status st = collect(k, p, b, inst);
  if (st) return st;
  if (pa) {
    if (!X || !theta || !pa->xi || !pa->phi || !status)
      return fail(GP_ERR_ARG, "X, theta, xi, phi and status must be non-NULL");
  } else if (!X || !y || !phi || !theta || !pi || !x_warm || !H0 || !H1 || !accepted || !status) {
    return fail(GP_ERR_ARG, "X, y, phi, theta, pi, x_warm, H0, H1, accepted and status must be non-NULL");
  }
  const int chains = b->chains_per_inst;
  const ChainLayout L = make_layout(inst, chains, k->prec, p->mode, k->kind, k->n_cheb,
                                    p->precond_rank, pa ? pa->pp->n_poles : 0);
  if (!ws || ws_bytes < L.total)
    return fail(GP_ERR_WORKSPACE, "workspace of %zu bytes needed, %zu given", L.total,
                ws ? ws_bytes : (size_t)0);
  const int nc = (int)inst.size() * chains;
  char *w = (char *)ws;
  const int pc = p->precond_rank > 0 ? 1 : 0;

  LaunchCfg cfg;
  if (tl_force) {
    cfg = *tl_force;
  } else {
    TuneCfg tc;
    if (tune_lookup(traj_key(k, inst, chains, pc), &tc)) {
      cfg.waves = tc.waves;
      cfg.cpt_lo = tc.cpt_lo;
      cfg.cpt_hi = tc.cpt_hi;
    }
  }

  std::vector<char> desc;
  if (k->prec == GP_F64) {
    std::vector<HmcChain<double>> v;
    fill_chains<double>(inst, k->kind, k->n_cheb, chains, L, w, p, X, y, phi, theta, pi, x_warm, u_accept, H0, H1,
                        accepted, status, cg_iters, k->prec, cfg, pa, v);
    desc.assign((const char *)v.data(), (const char *)(v.data() + v.size()));
  } else {
    std::vector<HmcChain<float>> v;
    fill_chains<float>(inst, k->kind, k->n_cheb, chains, L, w, p, X, y, phi, theta, pi, x_warm, u_accept, H0, H1,
                       accepted, status, cg_iters, k->prec, cfg, pa, v);
    desc.assign((const char *)v.data(), (const char *)(v.data() + v.size()));
  }
  // chain order for the batched scheduler: largest problems first
  std::vector<unsigned> order(nc);
  std::iota(order.begin(), order.end(), 0u);
  std::stable_sort(order.begin(), order.end(), [&](unsigned a, unsigned c) {
    return inst[a / chains].n * inst[a / chains].n * inst[a / chains].dp >
           inst[c / chains].n * inst[c / chains].n * inst[c / chains].dp;
  });
  std::vector<char> upload = desc;
  upload.insert(upload.end(), (const char *)order.data(), (const char *)(order.data() + nc));

  std::lock_guard<std::mutex> lock(g_mu);
  hipError_t e;
  auto itu = g_uploaded.find(ws);
  const bool changed = itu == g_uploaded.end() || itu->second != upload;
  if (changed) {
    // the workspace may still be in use by earlier work on the stream
    e = hipStreamSynchronize(stream);
    if (e != hipSuccess) return hip_fail(e, "stream sync");
    e = hipMemcpy(w + L.chains, desc.data(), desc.size(), hipMemcpyHostToDevice);
    if (e != hipSuccess) return hip_fail(e, "descriptor upload");
    e = hipMemcpy(w + L.hdr_order, order.data(), sizeof(unsigned) * nc, hipMemcpyHostToDevice);
    if (e != hipSuccess) return hip_fail(e, "order upload");
    g_uploaded[ws] = upload;
    auto itg = g_graphs.find(ws);
    if (itg != g_graphs.end()) {
      (void)hipGraphExecDestroy(itg->second.exec);  // a stale graph: nothing to do on failure
      g_graphs.erase(itg);
    }
  }

  HmcRunParams prm;
  memset(&prm, 0, sizeof(prm));  // the bytes key the graph cache
  prm.n_steps = rwm ? 0 : p->n_steps;
  prm.dt = p->dt;
  prm.tol2 = p->cg_tol * p->cg_tol;
  prm.cg_maxit = p->cg_maxit;
  // a preconditioned CG iteration is two or three jobs (the product, with split columns in a
  // persistent launch the gather job, and the z job); a solve adds its first product and gather,
  // the force pass and (GP_BF16X) the stage job
  const int64_t per_it = p->precond_rank > 0 ? 3 : 1;
  prm.max_jobs = (int)std::min<int64_t>((int64_t)(prm.n_steps + 2) * (per_it * p->cg_maxit + 4) + 4,
                                        (int64_t)1 << 30);
  prm.rwm = rwm;
  prm.epi_gather = p->mode != GP_HMC_PLAIN;
  // the refresh of phi: without the caller's bound, a launch for the Gershgorin bound first
  // (prm_b: the stage job and one product); then the poles; then the iteration (prm: the stage
  // job and maxit products)
  HmcRunParams prm_b;
  const bool bound_launch = pa && !(pa->pp->lambda_max > 0.0);
  if (pa) {
    prm.prog = kProgPhi;
    prm.n_poles = pa->pp->n_poles;
    prm.phi_tol = pa->pp->tol;
    prm.phi_lmax = pa->pp->lambda_max > 0.0 ? pa->pp->lambda_max : 0.0;
    prm.phi_widen = k->prec == GP_F64 ? 1e-12 : (k->prec == GP_F32 ? 1e-5 : 1e-3);
    prm.max_jobs = pa->pp->maxit + 4;
    prm_b = prm;
    prm_b.prog = kProgPhiBound;
    prm_b.max_jobs = 4;
  }
  HmcQueue qu;
  qu.word = (unsigned long long *)(w + L.hdr_word);
  qu.finished = (unsigned *)(w + L.hdr_fin);
  qu.chains_done = (unsigned *)(w + L.hdr_cnt);
  qu.abort = (unsigned *)(w + L.hdr_cnt + 4);
  qu.order = (unsigned *)(w + L.hdr_order);
  qu.progress = p->progress;
  void *chains_dev = w + L.chains;
  const bool f64 = k->prec == GP_F64;
  const int ch = k->kind == GP_SE_CHEB ? 1 : 0;
  const size_t cb = chain_bytes(k->prec);

  constexpr int kJobToDone = 6;
  static_assert(offsetof(HmcChain<double>, done) - offsetof(HmcChain<double>, job) == kJobToDone * sizeof(int) &&
                    offsetof(HmcChain<float>, done) - offsetof(HmcChain<float>, job) == kJobToDone * sizeof(int),
                "the plain-mode state read assumes job .. done are adjacent ints");
  // Plain mode: chain c's kickoff, then its jobs one launch at a time until it is done.
  auto plain_chain = [&](void *cp, int c, const HmcRunParams &pr) -> gp_status {
    hipError_t e = f64 ? hmc_kickoff_f64(cp, 1, pr, qu, 0, stream) : hmc_kickoff_f32(cp, 1, pr, qu, 0, stream);
    if (e != hipSuccess) return hip_fail(e, "kickoff");
    const size_t off_job = f64 ? offsetof(HmcChain<double>, job) : offsetof(HmcChain<float>, job);
    const int n_jobs = L.n_rb[c] * L.n_cs[c];
    const int xm = xm_width(k->prec, inst[c / chains].d);
    // chains are checked every kPlainCheck jobs: on a finished chain the tiles and the epilogue
    // do nothing, so a few surplus launches are harmless
    for (int64_t guard = 0;; ++guard) {
      if (guard > (int64_t)pr.max_jobs + 2 + kPlainCheck)
        return fail(GP_ERR_HIP, "plain-mode chain %d did not finish", c);
      // job .. done are adjacent ints of the chain state: one read brings both
      int state[kJobToDone + 1] = {};
      if (guard % kPlainCheck == 0) {
        e = hipMemcpyAsync(state, (char *)cp + off_job, sizeof(state), hipMemcpyDeviceToHost, stream);
        if (e == hipSuccess) e = hipStreamSynchronize(stream);
        if (e != hipSuccess) return hip_fail(e, "plain-mode state read");
        if (state[kJobToDone]) break;
      }
      const int dpc = inst[c / chains].dp;
      e = f64 ? hmc_tiles_f64(cp, n_jobs, dpc, ch, pc, 0, stream)
              : hmc_tiles_f32(cp, n_jobs, dpc, ch, pc, xm, stream);
      // with column splits the product is gathered by a multi-workgroup pass before the
      // (single-workgroup) epilogue
      if (e == hipSuccess && L.n_cs[c] > 1)
        e = f64 ? hmc_gather_f64(cp, L.n_rb[c], pc, stream)
                : hmc_gather_f32(cp, L.n_rb[c], pc, stream);
      if (e == hipSuccess)
        e = f64 ? hmc_epilogue_f64(cp, pr, pc, stream) : hmc_epilogue_f32(cp, pr, pc, stream);
      if (e != hipSuccess) return hip_fail(e, "plain-mode step");
    }
    return GP_OK;
  };

  if (p->mode == GP_HMC_PLAIN) {
    for (int c = 0; c < nc; ++c) {
      void *cp = (char *)chains_dev + cb * c;
      if (pa) {
        if (bound_launch) {
          st = plain_chain(cp, c, prm_b);
          if (st) return st;
        }
        e = f64 ? hmc_phi_poles_f64(cp, 1, prm, stream) : hmc_phi_poles_f32(cp, 1, prm, stream);
        if (e != hipSuccess) return hip_fail(e, "pole weights");
      }
      st = plain_chain(cp, c, prm);
      if (st) return st;
    }
    return GP_OK;
  }
  // the defaults stand if a query fails
  int dev = 0, cus = 256, clk_khz = 100000;
  (void)hipGetDevice(&dev);
  (void)hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
  (void)hipDeviceGetAttribute(&clk_khz, hipDeviceAttributeWallClockRate, dev);
  int dpmax = 4, xmax = 0;
  for (const InstInfo &in : inst) {
    dpmax = std::max(dpmax, in.dp);
    xmax = std::max(xmax, xm_width(k->prec, in.d));
  }
  int64_t total_jobs = 0;
  for (int c = 0; c < nc; ++c) total_jobs += (int64_t)L.n_rb[c] * L.n_cs[c];
  // the register allocation of the launch (waves per SIMD) and as many workgroups as can be
  // resident with it: one wave per SIMD each, so `waves` workgroups per CU
  const int w_def = hmc_waves_default(!f64, dpmax, xmax);
  const int waves = cfg.waves == hmc_waves_alt(!f64, dpmax, xmax) ? cfg.waves : w_def;
  const int grid = (int)std::max<int64_t>(1, std::min<int64_t>((int64_t)cus * waves, total_jobs));
  // an idle workgroup gives up after 20 s without claimable work
  const long long idle_limit = (long long)clk_khz * 1000LL * 20LL;

  // one persistent launch of program pr: queue reset, every chain's kickoff, the scheduler, and
  // the report of chains it did not finish
  auto launch = [&](const HmcRunParams &pr, hipStream_t s) -> hipError_t {
    hipError_t r = f64 ? hmc_reset_f64(qu, s) : hmc_reset_f32(qu, s);
    if (r != hipSuccess) return r;
    r = f64 ? hmc_kickoff_f64(chains_dev, nc, pr, qu, 1, s)
            : hmc_kickoff_f32(chains_dev, nc, pr, qu, 1, s);
    if (r != hipSuccess) return r;
    r = f64 ? hmc_persistent_f64(chains_dev, nc, pr, qu, grid, idle_limit, dpmax, pc, ch, 0, waves, s)
            : hmc_persistent_f32(chains_dev, nc, pr, qu, grid, idle_limit, dpmax, pc, ch, xmax,
                                 waves, s);
    if (r != hipSuccess) return r;
    return f64 ? hmc_check_f64(chains_dev, nc, s) : hmc_check_f32(chains_dev, nc, s);
  };
  auto enqueue = [&](hipStream_t s) -> hipError_t {
    if (pa) {
      if (bound_launch) {
        hipError_t r = launch(prm_b, s);
        if (r != hipSuccess) return r;
      }
      hipError_t r = f64 ? hmc_phi_poles_f64(chains_dev, nc, prm, s)
                         : hmc_phi_poles_f32(chains_dev, nc, prm, s);
      if (r != hipSuccess) return r;
    }
    return launch(prm, s);
  };

  if (p->mode == GP_HMC_BATCHED) {
    e = enqueue(stream);
    if (e != hipSuccess) return hip_fail(e, "batched launch");
    return GP_OK;
  }

  // GP_HMC_GRAPH: capture once per (workspace, descriptors, parameters), then replay.
  std::vector<char> key((const char *)&prm, (const char *)(&prm + 1));
  key.insert(key.end(), (const char *)&grid, (const char *)(&grid + 1));
  key.insert(key.end(), (const char *)&dpmax, (const char *)(&dpmax + 1));
  key.insert(key.end(), (const char *)&pc, (const char *)(&pc + 1));
  key.insert(key.end(), (const char *)&ch, (const char *)(&ch + 1));
  key.insert(key.end(), (const char *)&xmax, (const char *)(&xmax + 1));
  key.insert(key.end(), (const char *)&waves, (const char *)(&waves + 1));
  key.insert(key.end(), (const char *)&qu.progress, (const char *)(&qu.progress + 1));
  GraphEntry &ge = g_graphs[ws];
  if (!ge.exec || ge.key != key) {
    if (ge.exec) {
      (void)hipGraphExecDestroy(ge.exec);
      ge.exec = nullptr;
    }
    hipStream_t cap;
    e = hipStreamCreateWithFlags(&cap, hipStreamNonBlocking);
    if (e != hipSuccess) return hip_fail(e, "capture stream");
    hipGraph_t graph;
    e = hipStreamBeginCapture(cap, hipStreamCaptureModeThreadLocal);
    if (e == hipSuccess) {
      hipError_t el = enqueue(cap);
      e = hipStreamEndCapture(cap, &graph);
      if (el != hipSuccess) e = el;
    }
    if (e == hipSuccess) {
      e = hipGraphInstantiate(&ge.exec, graph, nullptr, nullptr, 0);
      (void)hipGraphDestroy(graph);
    }
    (void)hipStreamDestroy(cap);
    if (e != hipSuccess) {
      ge.exec = nullptr;
      return hip_fail(e, "graph capture");
    }
    ge.key = key;
  }
  e = hipGraphLaunch(ge.exec, stream);
  if (e != hipSuccess) return hip_fail(e, "graph launch");
  return GP_OK;
}


gp_status gp_hmc_leapfrog(const gp_kernel *k, const gp_hmc_params *p, const gp_batch *b,
                          const void *X, const void *y, const void *phi, double *theta,
                          double *pi, void *x_warm, const double *u_accept, double *H0,
                          double *H1, int32_t *accepted, int32_t *status, int32_t *cg_iters,
                          void *ws, size_t ws_bytes, hipStream_t stream) {
  clear_error();
  return run_chains(k, p, b, X, y, phi, theta, pi, x_warm, u_accept, H0, H1, accepted, status,
                    cg_iters, ws, ws_bytes, stream, 0);
}

gp_status gp_rwm(const gp_kernel *k, const gp_hmc_params *p, const gp_batch *b, const void *X,
                 const void *y, const void *phi, double *theta, double *xi, void *x_warm,
                 const double *u_accept, double *U0, double *U1, int32_t *accepted,
                 int32_t *status, int32_t *cg_iters, void *ws, size_t ws_bytes,
                 hipStream_t stream) {
  clear_error();
  return run_chains(k, p, b, X, y, phi, theta, xi, x_warm, u_accept, U0, U1, accepted, status,
                    cg_iters, ws, ws_bytes, stream, 1);
}
}  // extern "C"

namespace gpk {
namespace {

// The refresh's own parameters, and the trajectory parameters that carry them through the
// batch validation and the schedulers.
gp_status phi_chain_params(const gp_kernel *k, const gp_phi_params *pp, int32_t mode,
                           gp_hmc_params *hp) {
  if (!k) return fail(GP_ERR_ARG, "kernel description is NULL");
  if (!pp) return fail(GP_ERR_ARG, "phi parameters are NULL");
  if (k->flags & GP_NO_NOISE) return fail(GP_ERR_ARG, "GP_NO_NOISE: A has no positive lower bound");
  if (pp->n_poles < 1 || pp->n_poles > kPhiPoleMax)
    return fail(GP_ERR_ARG, "n_poles = %d outside 1..%d", pp->n_poles, kPhiPoleMax);
  if (!(pp->tol > 0.0)) return fail(GP_ERR_ARG, "tol must be > 0");
  if (pp->maxit < 1) return fail(GP_ERR_ARG, "maxit must be >= 1");
  if (!(pp->lambda_max <= 0.0 || std::isfinite(pp->lambda_max)))
    return fail(GP_ERR_ARG, "lambda_max must be finite");
  if (pp->precond_rank != 0)
    return fail(GP_ERR_UNSUPPORTED,
                "gp_phi_refresh_chains solves by multi-shift CG without a preconditioner "
                "(precond_rank must be 0; gp_phi_refresh takes a Nystrom factor)");
  memset(hp, 0, sizeof(*hp));
  hp->cg_tol = pp->tol;
  hp->cg_maxit = pp->maxit;
  hp->mode = mode;
  return GP_OK;
}

}  // namespace
}  // namespace gpk

extern "C" {

size_t gp_phi_chains_workspace_size(const gp_kernel *k, const gp_phi_params *p, int32_t mode,
                                    const gp_batch *b) {
  gp_hmc_params hp;
  std::vector<InstInfo> inst;
  if (phi_chain_params(k, p, mode, &hp) != GP_OK || collect(k, &hp, b, inst) != GP_OK) return 0;
  return make_layout(inst, b->chains_per_inst, k->prec, mode, k->kind, k->n_cheb, 0, p->n_poles)
      .total;
}

gp_status gp_phi_refresh_chains(const gp_kernel *k, const gp_phi_params *p, int32_t mode,
                                const gp_batch *b, const void *X, const double *theta,
                                const void *xi, void *phi, int32_t *status, int32_t *iters,
                                double *bounds, void *ws, size_t ws_bytes, hipStream_t stream) {
  clear_error();
  gp_hmc_params hp;
  gp_status st = phi_chain_params(k, p, mode, &hp);
  if (st) return st;
  std::vector<InstInfo> inst;
  st = collect(k, &hp, b, inst);
  if (st) return st;
  if (xi && phi && xi != phi) {
    // xi and phi are packed alike: either the same array or disjoint
    int64_t rows = 0;
    for (const InstInfo &in : inst) rows = std::max(rows, in.off + in.n);
    const size_t bytes = (size_t)rows * b->chains_per_inst * (k->prec == GP_F64 ? 8 : 4);
    const char *a0 = (const char *)xi, *b0 = (const char *)phi;
    if (a0 < b0 + bytes && b0 < a0 + bytes)
      return fail(GP_ERR_ARG, "phi overlaps xi (only phi == xi is allowed)");
  }
  PhiArgs pa{p, xi, phi, bounds};
  // the refresh reads theta and writes none of the trajectory outputs
  return run_chains(k, &hp, b, X, nullptr, nullptr, const_cast<double *>(theta), nullptr, nullptr,
                    nullptr, nullptr, nullptr, nullptr, status, iters, ws, ws_bytes, stream, 0, &pa);
}
}  // extern "C"

// ---- autotuning of the trajectory launch ---------------------------------------------------

namespace gpk {
namespace {

constexpr float kTuneMargin = 0.04f;  // relative gain a trajectory candidate needs to be chosen

// Tuning workspace: the trajectory workspace of the tuning run, then its synthetic inputs.
struct TuneLayout {
  size_t hmc, X, y, phi, xw, th, pi, H, ints, U, lam, total;
  int64_t nrows, nx, nth;
};

gp_hmc_params tune_params(const gp_hmc_params *p) {
  gp_hmc_params q;
  memset(&q, 0, sizeof(q));
  q.n_steps = 1;
  q.dt = 0.0;          // theta stays put: every candidate runs the same jobs
  q.cg_tol = 1e-300;   // every solve runs cg_maxit iterations
  q.cg_maxit = 8;
  q.mode = GP_HMC_BATCHED;
  q.precond_rank = p->precond_rank;
  return q;
}

TuneLayout tune_layout(const gp_kernel *k, const gp_hmc_params *q, const gp_batch *b,
                       const std::vector<InstInfo> &inst) {
  TuneLayout t;
  const size_t es = k->prec == GP_F64 ? 8 : 4;
  const int chains = b->chains_per_inst;
  t.nrows = t.nx = t.nth = 0;
  for (const InstInfo &in : inst) {
    t.nrows += in.n;
    t.nx += in.n * in.d;
    t.nth += in.nth;
  }
  const int64_t nc = (int64_t)inst.size() * chains;
  size_t o = 0;
  t.hmc = o;
  o += align256(make_layout(inst, chains, k->prec, q->mode, k->kind, k->n_cheb, q->precond_rank).total);
  t.X = o;
  o += align256(es * t.nx);
  t.y = o;
  o += align256(es * t.nrows);
  t.phi = o;
  o += align256(es * t.nrows * chains);
  t.xw = o;
  o += align256(es * t.nrows * chains);
  t.th = o;
  o += align256(8 * t.nth * chains);
  t.pi = o;
  o += align256(8 * t.nth * chains);
  t.H = o;
  o += align256(8 * 2 * nc);
  t.ints = o;
  o += align256(4 * 3 * nc);
  t.U = o;
  o += align256(es * t.nrows * q->precond_rank);
  t.lam = o;
  o += align256(8 * inst.size() * q->precond_rank);
  t.total = o;
  return t;
}

template <typename T>
__global__ void tune_fill(T *a, int64_t m, float lo, float hi, uint64_t salt) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= m) return;
  uint64_t z = ((uint64_t)e + salt) * 0x9E3779B97F4A7C15ull + 0x632BE59BD9B4E019ull;
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  z ^= z >> 31;
  a[e] = (T)(lo + (hi - lo) * (float)((z >> 40) * (1.0 / 16777216.0)));
}

template <typename T>
hipError_t tune_fill_launch(void *a, int64_t m, float lo, float hi, uint64_t salt, hipStream_t s) {
  if (m < 1) return hipSuccess;
  tune_fill<T><<<(unsigned)((m + 255) / 256), 256, 0, s>>>((T *)a, m, lo, hi, salt);
  return hipGetLastError();
}

}  // namespace
}  // namespace gpk

extern "C" {

size_t gp_tune_hmc_workspace_size(const gp_kernel *k, const gp_hmc_params *p, const gp_batch *b) {
  std::vector<InstInfo> inst;
  if (!p || collect(k, p, b, inst) != GP_OK) return 0;
  const gp_hmc_params q = tune_params(p);
  return tune_layout(k, &q, b, inst).total;
}

gp_status gp_tune_hmc(const gp_kernel *k, const gp_hmc_params *p, const gp_batch *b, void *ws,
                      size_t ws_bytes, hipStream_t stream) {
  clear_error();
  std::vector<InstInfo> inst;
  gp_status st = collect(k, p, b, inst);
  if (st) return st;
  const gp_hmc_params q = tune_params(p);
  const TuneLayout t = tune_layout(k, &q, b, inst);
  if (!ws || ws_bytes < t.total)
    return fail(GP_ERR_WORKSPACE, "workspace of %zu bytes needed, %zu given", t.total,
                ws ? ws_bytes : (size_t)0);
  const bool f64 = k->prec == GP_F64;
  const int chains = b->chains_per_inst;
  const int n_inst = (int)inst.size();
  const int nc = n_inst * chains;
  char *w = (char *)ws;
  // synthetic inputs packed instance after instance
  std::vector<int64_t> npts(n_inst), offs(n_inst), xoffs(n_inst);
  std::vector<int32_t> dims(n_inst);
  std::vector<double> th0;
  int64_t ro = 0, xo = 0;
  int dpmax = 4, xmax = 0, any_lo = 0, any_hi = 0;
  for (int i = 0; i < n_inst; ++i) {
    npts[i] = inst[i].n;
    offs[i] = ro;
    xoffs[i] = xo;
    dims[i] = inst[i].d;
    ro += inst[i].n;
    xo += inst[i].n * inst[i].d;
    dpmax = std::max(dpmax, inst[i].dp);
    xmax = std::max(xmax, xm_width(k->prec, inst[i].d));
    (inst[i].dp <= 8 ? any_lo : any_hi) = 1;
    for (int h = 0; h < chains; ++h)
      for (int j = 0; j < inst[i].nth; ++j)
        th0.push_back(j == inst[i].nth - 1 ? std::log(0.1) : (j == 0 ? 0.0 : std::log(0.5)));
  }
  if (k->kind == GP_SE_CHEB)  // Theta = 0 (unit amplitude), log l = log 0.5
    for (size_t j = 0, c = 0; c < (size_t)nc; ++c) {
      const int nth = inst[c / chains].nth;
      for (int q2 = 0; q2 < nth - 2; ++q2) th0[j + q2] = 0.0;
      j += nth;
    }
  gp_batch sb = *b;
  sb.n_points = npts.data();
  sb.offsets = offs.data();
  sb.x_offsets = xoffs.data();
  sb.d = dims.data();
  gp_hmc_params qq = q;
  if (q.precond_rank > 0) {
    qq.precond_U = w + t.U;
    qq.precond_lam = (const double *)(w + t.lam);
  }
  hipError_t e = hipSuccess;
  const int64_t rows = t.nrows;
  auto fill = [&](size_t off, int64_t m, float lo, float hi, uint64_t salt) {
    if (e != hipSuccess) return;
    e = f64 ? tune_fill_launch<double>(w + off, m, lo, hi, salt, stream)
            : tune_fill_launch<float>(w + off, m, lo, hi, salt, stream);
  };
  fill(t.X, t.nx, 0.f, 1.f, 11);
  fill(t.y, rows, -1.f, 1.f, 12);
  fill(t.phi, rows * chains, -1.f, 1.f, 13);
  if (e == hipSuccess) e = hipMemsetAsync(w + t.U, 0, (f64 ? 8 : 4) * rows * q.precond_rank, stream);
  if (e != hipSuccess) return hip_fail(e, "tuner inputs");
  std::vector<double> lam((size_t)n_inst * q.precond_rank, 1.0);
  if (!lam.empty()) {
    e = hipMemcpyAsync(w + t.lam, lam.data(), 8 * lam.size(), hipMemcpyHostToDevice, stream);
    if (e == hipSuccess) e = hipStreamSynchronize(stream);
    if (e != hipSuccess) return hip_fail(e, "tuner inputs");
  }
  // candidates, one knob at a time from the defaults: the alternative register allocation, then
  // the other columns per trip for the chains with padded d <= 8, then for those above
  const int wopt[2] = {hmc_waves_default(!f64, dpmax, xmax), hmc_waves_alt(!f64, dpmax, xmax)};
  const int lo_opt[2] = {4, 2}, hi_opt[2] = {2, 1};
  const int n_knobs = xmax ? 1 : 3;
  hipEvent_t e0 = nullptr, e1 = nullptr;
  e = hipEventCreate(&e0);
  if (e == hipSuccess) e = hipEventCreate(&e1);
  if (e != hipSuccess) {
    if (e0) (void)hipEventDestroy(e0);
    return hip_fail(e, "tuner events");
  }
  const size_t es = f64 ? 8 : 4;
  char *X = w + t.X, *y = w + t.y, *phi = w + t.phi, *xw = w + t.xw;
  double *th = (double *)(w + t.th), *pi = (double *)(w + t.pi), *H = (double *)(w + t.H);
  int32_t *ints = (int32_t *)(w + t.ints);
  const size_t hmc_bytes = t.X - t.hmc;
  // one timed run of configuration c (after a run that uploads its descriptors)
  auto time_cfg = [&](const LaunchCfg &c) -> float {
    tl_force = &c;
    float ms_min = 1e30f;
    for (int rep = 0; rep < 2 && st == GP_OK && e == hipSuccess; ++rep) {
      // the same start for every run: theta, pi = 0 and x = 0
      e = hipMemcpyAsync(th, th0.data(), 8 * th0.size(), hipMemcpyHostToDevice, stream);
      if (e == hipSuccess) e = hipMemsetAsync(pi, 0, 8 * th0.size(), stream);
      if (e == hipSuccess) e = hipMemsetAsync(xw, 0, es * rows * chains, stream);
      if (e == hipSuccess) e = hipStreamSynchronize(stream);
      if (e == hipSuccess) e = hipEventRecord(e0, stream);
      if (e != hipSuccess) break;
      st = run_chains(k, &qq, &sb, X, y, phi, th, pi, xw, nullptr, H, H + nc, ints, ints + nc,
                      ints + 2 * nc, w + t.hmc, hmc_bytes, stream, 0);
      if (st != GP_OK) break;
      e = hipEventRecord(e1, stream);
      if (e == hipSuccess) e = hipEventSynchronize(e1);
      float ms = 0.f;
      if (e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
      if (rep > 0 && ms < ms_min) ms_min = ms;
    }
    tl_force = nullptr;
    return ms_min;
  };
  LaunchCfg cur;
  cur.waves = wopt[0];
  cur.cpt_lo = any_lo && !xmax ? lo_opt[0] : 0;
  cur.cpt_hi = any_hi && !xmax ? hi_opt[0] : 0;
  float cur_ms = time_cfg(cur);
  for (int knob = 0; knob < n_knobs && st == GP_OK && e == hipSuccess; ++knob) {
    if ((knob == 1 && !any_lo) || (knob == 2 && !any_hi)) continue;
    LaunchCfg c = cur;
    if (knob == 0) c.waves = wopt[1];
    if (knob == 1) c.cpt_lo = lo_opt[1];
    if (knob == 2) c.cpt_hi = hi_opt[1];
    // a candidate must win clearly: the proxy runs every chain in lock-step for a few
    // iterations, so small differences do not carry over to trajectories whose chains finish
    // at different times (on the batched leapfrog workload a 2% proxy gain was an 8% loss)
    const float ms = time_cfg(c);
    if (ms < (1.0f - kTuneMargin) * cur_ms) {
      cur = c;
      cur_ms = ms;
    }
  }
  TuneCfg best;
  best.splits = 1;
  best.ib = 1;
  best.ms = cur_ms;
  best.waves = cur.waves;
  best.cpt_lo = cur.cpt_lo;
  best.cpt_hi = cur.cpt_hi;
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  {
    // the tuning workspace belongs to the caller again: forget its descriptors and graph
    std::lock_guard<std::mutex> lock(g_mu);
    g_uploaded.erase(w + t.hmc);
    auto itg = g_graphs.find(w + t.hmc);
    if (itg != g_graphs.end()) {
      if (itg->second.exec) (void)hipGraphExecDestroy(itg->second.exec);
      g_graphs.erase(itg);
    }
  }
  if (st != GP_OK) return st;
  if (e != hipSuccess) return hip_fail(e, "tuner timing");
  tune_store(traj_key(k, inst, chains, q.precond_rank > 0 ? 1 : 0), best);
  return GP_OK;
}
}  // extern "C"
