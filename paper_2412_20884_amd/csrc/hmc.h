// Device-resident chain state of the HMC trajectories and the job/phase encoding shared by the
// plain (host-scheduled) and batched (persistent work-queue) schedulers.
#pragma once

#include "common.h"
#include "gpk.h"

namespace gpk {

// Jobs a chain can publish; every job is split into n_rb row blocks x n_cs column splits.
// kJobGather: preconditioned chains with column splits in a persistent launch, after a product
// job (gsrc = kJobMvX or kJobMvP): q from the split partials, v . q and the preconditioner's
// partials, one row block per job id.
enum HmcJob { kJobNone = 0, kJobMvX = 1, kJobMvP = 2, kJobQf = 3, kJobZ = 4, kJobStage = 5,
              kJobGather = 6 };
// Why the current solve + quadratic-form pass is being done.
enum HmcCtxKind { kCtxEnergy0 = 0, kCtxForce = 1, kCtxEnergy1 = 2 };

// doubles per tile record: [0..7] scalars, [8 + k] length-scale gradient; the Chebyshev-amplitude
// kernel adds its N_cheb^d <= 64 coefficient sums at [9 + m]
constexpr int kHmcRec = 80;
constexpr int kHmcTile = 256;      // rows per tile (one per thread)
constexpr int kHmcMaxTheta = kMaxD + 2;
constexpr int kHmcMaxRank = 512;   // largest Nystrom rank of the preconditioned solves

// Geometry of the GP_BF16X trajectory jobs: 32-column tiles whose LDS image is the bfloat16 hi
// and lo coordinate rows (padded to XSTR halves against bank conflicts), the 32 norms, the column
// operand (up to 2 floats per column) and, for the force pass of ARD chains, the image of
// [X~ | 1]^T: KB2 blocks of 16 rows of kStr halves (slot-ordered columns) of hi parts, then the
// KB2 - 1 blocks of lo parts of X~ (the ones row needs none).
namespace xmt {
constexpr int TJ = 32;           // columns per tile
constexpr int kStr = 40;         // halves per row of the transposed column image
constexpr int kRowsStage = 64;   // rows per stage job (one job id)
constexpr int kRowsJob = 128;    // rows per product or force-pass job
template <int DPX>
struct Geo {
  static constexpr int XSTR = DPX + 8;
  static constexpr int KB2 = DPX / 16 + 1;
  static constexpr int kXB = TJ * XSTR * 2;
  static constexpr int kNB = TJ * 4;
  static constexpr int kVB = TJ * 2 * 4;
  static constexpr int kBBH = KB2 * 16 * kStr * 2;
  static constexpr int kBBL = (KB2 - 1) * 16 * kStr * 2;
  static constexpr int kBB = kBBH + kBBL;  // bytes of one tile's [X~ | 1]^T image
  static constexpr int oXL = kXB, oN = 2 * kXB, oV = oN + kNB, oBH = oV + kVB, oBL = oBH + kBBH;
  static constexpr int kBytes = oBH + kBB;
};
inline int dpx_of(int d) { return d <= 32 ? 32 : 64; }
}  // namespace xmt

template <typename T>
struct HmcChain {
  // problem (caller memory)
  const T *X;
  const T *y;
  const T *phi;
  double *theta;
  double *pi;
  T *x;
  const double *u;  // uniform for the accept test, or null
  double *H0out, *H1out;
  int32_t *acc_out, *status_out, *iters_out;
  int64_t n;
  int d, dp, kind, nth;
  // workspace
  T *xs;       // n x dp scaled coordinates
  T *r, *p, *q, *x0;
  T *Z;        // n x 2: [x | phi]
  T *lc;       // GP_SE_CHEB: log2 of the amplitude e^{C(x_i)} at the current theta (n)
  int ncheb;   // GP_SE_CHEB: N_cheb
  double *qpart;  // n_cs x n partial products (n_cs > 1 only)
  double *rec;    // n_jobs x kHmcRec
  double theta0[kHmcMaxTheta], pi0[kHmcMaxTheta], F[kHmcMaxTheta];
  double minv[kHmcMaxTheta];  // diagonal of the inverse mass matrix
  // Nystrom preconditioner of the solves (prank = 0: plain CG): U n x prank, lam prank; in the
  // workspace the row blocks' partial sums of U^T w1, U^T w2 [n_rb][2][prank], g = U^T r and
  // h = c o g [prank]
  const T *pU;
  const double *plam;
  int prank;
  int zfirst;     // the pending z job starts a solve (p = z) rather than continuing it
  int gsrc;       // the product job a pending gather job completes (kJobMvX or kJobMvP)
  double *pgp, *pg, *ph;
  double centre[kMaxD];
  // schedule
  int n_rb, n_cs, n_jobs;
  int cpt;  // columns per trip of the product jobs (0: the default for the chain's d)
  int64_t col_chunk;
  // state
  int job;       // job being run by the tiles
  int ctx;       // HmcCtxKind
  int step;      // leapfrog step index
  int it;        // CG iterations in the current solve
  int cg_total;  // CG iterations over the trajectory
  int status;
  int done;
  int jobs_run;  // jobs completed in this trajectory (bounded, see HmcRunParams::max_jobs)
  double rr, yy, H0, H1;
  double rz;  // r^T z of the preconditioned CG (z = P^{-1} r)
  // GP_BF16X chains (xm = padded cross-term width 32 or 64, else 0): the squared distances come
  // from the norm expansion with the cross term on the matrix cores.  A stage job (64 rows per
  // job) writes, for every theta, the bfloat16 hi / lo coordinates xh, xl ([n_rb * 64][xm + 8],
  // rows past n zero), the compensated norms nrm (rows past n: 1e30, so their kernel values
  // vanish) and, for ARD chains, bimg: the column-side image of [X~ | 1]^T per 32-column tile
  // (Geo::kBB bytes a tile, bfloat16 in slot order).
  int xm;
  uint16_t *xh, *xl, *bimg;
  float *nrm;
  double cscale[kMaxD];  // per-dimension coordinate scale of the theta being solved at
  // Gibbs refresh of phi (prog != kProgTrajectory): right-hand side xi and output phi (per chain,
  // caller memory), bounds out [m, M] or null; in the workspace the shifted directions ps
  // [np][n] and the per-pole state pst [np][kPst]; the unshifted CG scalars.
  int prog;
  const T *xi;
  T *phio;
  double *bounds_out;
  T *ps;
  double *pst;
  double rr0, a_prev, b_prev, lmin, lmax;
};

// Chain programs: one trajectory (or random-walk update) of theta, or the Gibbs refresh of phi
// (its Gershgorin bound, then its multi-shift iteration).
enum HmcProg { kProgTrajectory = 0, kProgPhi = 1, kProgPhiBound = 2 };
// Doubles of per-pole state of the refresh: weight, shift, zeta of the previous, current and next
// iteration, the shifted step coefficient w_p alpha_p, the direction coefficients zp and bp, and
// the active flag.
namespace phs {
enum { kW = 0, kLam, kZprev, kZ, kZnext, kCx, kZp, kBp, kAct };
}
constexpr int kPst = 9;
constexpr int kPhiPoleMax = 64;  // most poles of the batched refresh

// Waves per SIMD the persistent trajectory kernel is compiled for.  The default: in float the
// tile variants up to d = 8 fit 128 VGPRs (4 waves) and those up to d = 16 fit 168 with a few
// spills (3 waves), which the batched leapfrog measures faster than 2 waves without spills; the
// GP_BF16X jobs (xm != 0) run at 3 waves (their spills sit outside the pair loops: 1.01 s
// against 1.14 s at 2 waves for a 2-step d = 64 trajectory).  Each launch also has the
// alternative instantiation, which the trajectory autotuner can choose.
constexpr int hmc_waves_default(bool f32, int dpmax, int xm) {
  return xm ? 3 : (!f32 ? 1 : (dpmax <= 8 ? 4 : (dpmax <= 16 ? 3 : 1)));
}
constexpr int hmc_waves_alt(bool f32, int dpmax, int xm) {
  return xm ? 2 : (!f32 ? 2 : (dpmax <= 8 ? 3 : (dpmax <= 16 ? 2 : 2)));
}

struct HmcRunParams {
  int n_steps;
  double dt;
  double tol2;  // cg_tol^2
  int cg_maxit;
  int max_jobs;  // (n_steps + 2) * (cg_maxit + 2) + 4: no trajectory can need more jobs
  int rwm;       // 1: random-walk Metropolis update theta' = theta + dt * pi, no kinetic energy
  // Gibbs refresh (prog != kProgTrajectory): poles, per-pole tolerance, the caller's upper bound
  // (<= 0: Gershgorin) and the relative widening of the Gershgorin bound for the product's rounding
  int prog;
  int n_poles;
  double phi_tol;
  double phi_lmax;
  double phi_widen;
  // 1: the chain's epilogue forms q from the column-split partials (persistent launches); 0: the
  // plain mode's gather kernel has formed it
  int epi_gather;
};

// Scheduling words of the batched launch, one per chain: (generation << 32) | claimed tiles.
struct HmcQueue {
  unsigned long long *word;
  unsigned int *finished;    // per chain: tiles finished in the current generation
  unsigned int *chains_done;
  unsigned int *abort;
  unsigned int *order;       // chain indices, largest problems first
  int *progress;             // caller's progress word (finished chains), or null
};

}  // namespace gpk
