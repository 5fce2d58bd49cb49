/*
 * gpk.h -- C ABI of libgpk: matrix-free kernel-matrix products, quadratic-form gradients and
 * HMC leapfrog trajectories for determinant-free fully Bayesian Gaussian process regression,
 * on hand-written gfx950 (MI355X) kernels.
 *
 * Notation (Kielstra & Lindsey, "A gradient-based and determinant-free framework for fully
 * Bayesian Gaussian process regression"):
 *   A(theta) = sigma^2 I + K(theta)          Section 2, eq. (kerdef); K is eq. (kernmat)
 *   K_ij = alpha exp(-1/2 sum_k (x_ik - x_jk)^2 / l_k^2)
 *                                            squared-exponential kernel of Section 1; one
 *                                            length-scale (GP_SE_ISO) or one per coordinate
 *                                            (GP_SE_ARD)
 *   theta = (log alpha, log l_1 .. log l_L, log sigma^2), natural logs, L = 1 (ISO) or d (ARD),
 *   n_theta = L + 2.  In this library "K_theta" always means the full A(theta) unless
 *   GP_NO_NOISE is set.
 *   GP_SE_CHEB, the non-stationary amplitude kernel of Section 4:
 *     K_ij = exp(C(x_i)) exp(C(x_j)) exp(-|x_i - x_j|^2 / (2 l^2)),
 *     C(x) = sum_{m_1..m_d < N_cheb} Theta_{m_1..m_d} T_{m_1}(x^1) ... T_{m_d}(x^d),
 *   T_m the Chebyshev polynomials of the first kind (points are meant to lie in [-1, 1]^d);
 *   theta = (Theta flattened with m_1 slowest, log l, log sigma^2), n_theta = N_cheb^d + 2.
 *
 * Conventions common to every entry point
 *   - Ownership: every array argument is caller-owned memory; the library never allocates,
 *     frees or retains caller memory.  Arrays marked "device" must be device memory of the
 *     current HIP device; arrays marked "host" are read during the call only.
 *   - Asynchrony: work is enqueued on `stream` (0 = the null stream); results are valid once
 *     the stream has been synchronised.  The call returns after enqueueing.
 *   - Validation: every argument error is detected on the host before anything is enqueued;
 *     the call then returns a nonzero status with no side effect and gp_last_error() describes
 *     it.  GP_ERR_HIP reports a failed HIP launch or runtime call.
 *   - Layout: matrices are row-major with a leading dimension (elements between consecutive
 *     rows); point sets X are N x d row-major with leading dimension d.
 *   - Precision (gp_kernel.prec): GP_F64 -> all real arrays are double; GP_F32 -> X, V, U, out
 *     are float (parameters, weights, gradients, quadratic forms and energies stay double);
 *     GP_BF16X -> as GP_F32 in memory, but the coordinate cross term is formed from bfloat16
 *     hi/lo splits on the matrix cores with float accumulation.
 *   - Determinism: no floating-point atomics; for a fixed (n, r, d, precision) the summation
 *     order is fixed, so repeated calls give bitwise-identical results.
 *   - Thread safety: calls on distinct streams with distinct workspaces may run concurrently.
 *   - Workspace: `ws` is device scratch of at least the size the matching *_workspace_size
 *     function returns (0 bytes allowed when that size is 0); its contents on entry are
 *     irrelevant.
 */
#ifndef GPK_H
#define GPK_H

#include <stddef.h>
#include <stdint.h>

#include <hip/hip_runtime_api.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int32_t gp_status;
enum {
  GP_OK = 0,
  GP_ERR_ARG = 1,         /* null pointer, bad enum, aliasing, bad parameter value */
  GP_ERR_SHAPE = 2,       /* n, r, d or a leading dimension out of range */
  GP_ERR_UNSUPPORTED = 3, /* valid but not implemented combination */
  GP_ERR_WORKSPACE = 4,   /* ws missing or smaller than the required size */
  GP_ERR_HIP = 5          /* a HIP launch or runtime call failed */
};

enum { GP_SE_ISO = 0, GP_SE_ARD = 1, GP_SE_CHEB = 2 };
enum { GP_F64 = 0, GP_F32 = 1, GP_BF16X = 2 };
enum { GP_NO_NOISE = 1 /* apply K(theta) (eq. kernmat) instead of A(theta) */ };

/* Kernel description.  d: 1..64 coordinates. */
typedef struct {
  int32_t kind;   /* GP_SE_ISO, GP_SE_ARD or GP_SE_CHEB */
  int32_t prec;   /* GP_F64, GP_F32 or GP_BF16X */
  int32_t d;      /* spatial dimension */
  int32_t flags;  /* 0 or GP_NO_NOISE */
  int32_t n_cheb; /* GP_SE_CHEB: Chebyshev order N_cheb >= 1 with N_cheb^d <= 64; else ignored */
} gp_kernel;

/* Per-chain status bits written by gp_hmc_leapfrog; any set bit forces a reject. */
enum {
  GP_CHAIN_CG_MAXIT = 1,        /* a linear solve hit cg_maxit before reaching cg_tol */
  GP_CHAIN_NONFINITE_H = 2,     /* an energy was NaN or infinite */
  GP_CHAIN_NONFINITE_THETA = 4, /* theta or pi became NaN or infinite */
  GP_CHAIN_ABORTED = 8,         /* the batched scheduler stopped before the chain finished */
  GP_CHAIN_FP_MAXIT = 16        /* an implicit step's fixed point was not reached in maxit */
};

/* Message of the last failed call on the calling thread ("" if none).  Valid until the next
 * gp_* call on the same thread. */
const char *gp_last_error(void);
/* Static name of a status code. */
const char *gp_status_string(gp_status s);
/* n_theta for a kernel description, or -1 if it is invalid. */
int32_t gp_n_theta(const gp_kernel *k);

/* Bytes of workspace that gp_kmatvec and gp_quadform_grad need for n points and r columns.
 * Returns 0 for an invalid description. */
size_t gp_workspace_size(const gp_kernel *k, int64_t n, int32_t r);

/*
 * gp_kmatvec -- out = (A(theta) + diag(col_shift)) V, column by column, matrix-free.
 *
 * The matrix-free product with A(theta) of eq. (kerdef) (or K of eq. (kernmat) with
 * GP_NO_NOISE): entries are recomputed on the fly, memory stays O(N (d + r)).  Section 2 and the
 * discussion of matrix-free primitives in Section 1; each conjugate-gradient iteration of the
 * solves in Section 3.2.1 (eq. xtheta) and of the shifted solves of the pole expansion
 * (Section 3.1, eq. pex) is one such product.
 *
 *   X        device, n x d, leading dimension d
 *   theta    device double[n_theta]; read on the device, so a captured graph sees updates
 *   r        number of right-hand sides, r >= 0 (r = 0 or n = 0: nothing is done)
 *   V        device, n x r, leading dimension ldv >= r
 *   col_shift device double[r]: lambda_c added to the diagonal for column c, or NULL (= 0)
 *   out      device, n x r, leading dimension ldo >= r; must not overlap V
 */
gp_status gp_kmatvec(const gp_kernel *k, int64_t n, const void *X, const double *theta,
                     int32_t r, const void *V, int64_t ldv, const double *col_shift,
                     void *out, int64_t ldo, void *ws, size_t ws_bytes, hipStream_t stream);

/*
 * gp_kmatvec_noalloc -- gp_kmatvec for callers that cannot allocate device memory (code under
 * HIP graph capture, serving loops that must not call hipMalloc, harnesses that forbid it).
 *
 * Same product, arguments and validation as gp_kmatvec, without a workspace argument: the
 * workspace is a 64 MiB array in device memory that the library holds on every device it runs
 * on until the process ends; it makes no allocation of its own.  The column-split count of the
 * pass is reduced until the workspace fits, so results equal gp_kmatvec's up to the order of
 * floating-point sums.  A product whose workspace cannot fit in 64 MiB returns GP_ERR_WORKSPACE
 * before anything is enqueued; the limit is set by the staged column tiles of the matrix-core
 * passes: about 170,000 points for GP_F32 with 8 <= r <= 32 and d <= 16, about 37,000 for
 * GP_BF16X at d = 64, and 2 to 4 million for the VALU passes (GP_F64, or r < 8).  The first call on a device looks up the array's device address
 * (a HIP runtime query, no allocation).
 * Calls on one device share the array: two calls whose work overlaps on the device (different
 * streams, or host threads without ordering) race on it and give undefined results.  Calls
 * ordered on one stream are safe; no state carries over from one call to the next.
 */
gp_status gp_kmatvec_noalloc(const gp_kernel *k, int64_t n, const void *X, const double *theta,
                             int32_t r, const void *V, int64_t ldv, const double *col_shift,
                             void *out, int64_t ldo, hipStream_t stream);

/*
 * gp_quadform_grad -- Q = sum_c w_c u_c^T A(theta) v_c, its theta-gradient and A U, A V in one
 * pass over the pairs.
 *
 * The force of Section 3.2.1 needs only solves and the theta-gradient of quadratic forms in
 * A(theta) (capacity (3)); with U = V = [x | phi] and w = (-1/2, +1/2) the gradient is the force
 * of eq. (u) at x frozen.  The derivatives are
 *   dQ/dlog alpha   = sum_ij K_ij S_ij,        S_ij = sum_c w_c u_ic v_jc
 *   dQ/dlog l_k     = sum_ij K_ij (x_ik - x_jk)^2 / l_k^2 S_ij   (ISO: r_ij^2 / l^2)
 *   dQ/dlog sigma^2 = sigma^2 sum_c w_c u_c . v_c
 * and for GP_SE_CHEB (Section 4), with phi_m(x) = prod_k T_{m_k}(x^k),
 *   dQ/dTheta_m     = sum_ij K_ij (phi_m(x_i) + phi_m(x_j)) S_ij
 *                   = sum_i phi_m(x_i) e^{C(x_i)} sum_c w_c [u_ic (K~ D v_c)_i + v_ic (K~ D u_c)_i]
 * (K~ the unit-amplitude SE kernel, D = diag(e^{C(x_i)})), computed from the products of the
 * same pass.  Kernel entries are recomputed, never stored.  With GP_NO_NOISE the form is in
 * K(theta) (eq. kernmat) and the sigma^2 component of the gradient is 0.
 *
 *   U, V       device, n x r (r in 1..32), leading dimensions ldu, ldv >= r; U may equal V
 *   w          device double[r] weights, or NULL (all 1)
 *   grad_theta device double[n_theta] (dQ/dtheta), or NULL
 *   quad       device double[r], q_c = u_c^T A v_c (unweighted), or NULL
 *   AU, AV     device, n x r, leading dimensions ldau, ldav >= r, or NULL; A U is dQ/dv per
 *              column up to w_c, A V is dQ/du.  They must not overlap U or V or each other.
 *              With U != V and both requested, r <= 16 runs as one pass of 2r columns
 *              ([U | V] against [V | U], weights [w | 0]); larger r takes a second pass for A V.
 * At least one output must be non-NULL.
 */
gp_status gp_quadform_grad(const gp_kernel *k, int64_t n, const void *X, const double *theta,
                           int32_t r, const void *U, int64_t ldu, const void *V, int64_t ldv,
                           const double *w, double *grad_theta, double *quad, void *AU,
                           int64_t ldau, void *AV, int64_t ldav, void *ws, size_t ws_bytes,
                           hipStream_t stream);

/*
 * Autotuning of the product kernels.  For the problem class of (k, n, r) -- operation
 * (with_grad: gp_quadform_grad, else gp_kmatvec), precision, kernel kind, padded d, padded r and
 * floor(log2 n) -- gp_tune_products times every candidate configuration (column splits of the
 * pair grid; rows per wavefront of the matrix-core kernel) on synthetic inputs it generates in
 * `ws` (at least gp_tune_workspace_size bytes) and records the fastest in a process-wide table
 * that later calls of that class use.  The call synchronises `stream`.  Results of a product do
 * not depend on the configuration beyond the order of its floating-point sums.
 * gp_tune_save / gp_tune_load write / read the table as JSON; if the environment variable
 * GPK_TUNE_CACHE names a file, it is loaded on first use.
 */
size_t gp_tune_workspace_size(const gp_kernel *k, int64_t n, int32_t r);
gp_status gp_tune_products(const gp_kernel *k, int64_t n, int32_t r, int32_t with_grad,
                           void *ws, size_t ws_bytes, hipStream_t stream);
gp_status gp_tune_save(const char *path);
gp_status gp_tune_load(const char *path);
int32_t gp_tune_entries(void);
void gp_tune_clear(void);

/* Trajectory parameters.
 *
 * inv_mass: the diagonal of M^{-1} in H = U_phi + 1/2 pi^T M^{-1} pi (Section 3.2; the paper's
 * runs use M = I).  Host array packed per instance like one chain's theta (instance b's n_theta_b
 * entries at the sum of n_theta over the instances before it), shared by the instance's chains;
 * entries finite and >= 0.  A zero entry is the limit of an infinite mass: that component of theta
 * stays fixed and its momentum adds no kinetic energy (a hyperparameter held at its value).
 * NULL: M = I.
 *
 * precond_rank, precond_U, precond_lam: an optional randomized Nystrom factor K ~ U diag(lam) U^T
 * per instance (gp_nystrom's output; Section 3.1 after eq. pex, rank 5 in Section 4.1 and 500 in
 * Section 4.3) with which every conjugate-gradient solve of the trajectory is preconditioned by
 * P^{-1} = U diag((lam_rank + mu) / (lam + mu)) U^T + (I - U U^T), mu = sigma^2 at the theta of
 * the solve (the Woodbury form of gp_pcg_solve).  precond_U: device, kernel precision, instance
 * b's n_b x rank block (row-major, orthonormal columns) at element offset offsets[b] * rank;
 * precond_lam: device double, instance b's rank values (descending, >= 0) at b * rank.  The factor
 * may come from any theta (for example the chains' current one): the solves converge to the same
 * tolerance with any factor, only the iteration count depends on it.  precond_rank = 0: plain CG.
 */
typedef struct {
  int32_t n_steps;  /* leapfrog steps per trajectory, N_int >= 0 */
  double dt;        /* step size */
  double cg_tol;    /* relative residual |y - A x|_2 / |y|_2 at which CG stops, > 0 */
  int32_t cg_maxit; /* CG iteration limit per solve, >= 1 */
  int32_t mode;     /* GP_HMC_PLAIN, GP_HMC_BATCHED or GP_HMC_GRAPH */
  const double *inv_mass;    /* host, packed per instance, or NULL (M = I) */
  int32_t precond_rank;      /* 0..512; rank <= n_b for every instance */
  const void *precond_U;     /* device, packed per instance, or NULL when precond_rank = 0 */
  const double *precond_lam; /* device, packed per instance, or NULL when precond_rank = 0 */
  int32_t *progress;  /* host-pinned (hipHostMalloc) or device int32, or NULL: in the batched and
                         graph modes, the number of chains finished so far, stored as chains finish
                         (a long launch can be watched from the host) */
} gp_hmc_params;

enum {
  GP_HMC_PLAIN = 0,   /* one chain at a time, one kernel per operation, host-checked CG */
  GP_HMC_BATCHED = 1, /* every chain of every instance in one persistent launch */
  GP_HMC_GRAPH = 2    /* as GP_HMC_BATCHED, launched by replaying a captured hipGraph */
};

/* A batch of independent GPR instances, each with `chains_per_inst` chains.  Instance b has
 * n_points[b] points of dimension d[b] (or k->d if d is NULL).  Packing (all host arrays):
 *   X      element offset x_offsets[b] (or offsets[b] * d_b if x_offsets is NULL), n_b x d_b
 *   y      row offset offsets[b]
 *   phi, x_warm  chain h of instance b at  chains_per_inst * offsets[b] + h * n_b
 *   theta, pi    chain h of instance b at  chains_per_inst * tofs_b + h * n_theta_b, where
 *                tofs_b = sum of n_theta over instances before b
 *   per-chain scalars  index b * chains_per_inst + h
 * The row ranges [offsets[b], offsets[b] + n_b) must not overlap. */
typedef struct {
  int32_t n_inst;
  int32_t chains_per_inst;
  const int64_t *n_points;  /* host [n_inst], each >= 1 */
  const int64_t *offsets;   /* host [n_inst] */
  const int32_t *d;         /* host [n_inst] or NULL */
  const int64_t *x_offsets; /* host [n_inst] or NULL */
} gp_batch;

/* Bytes of workspace gp_hmc_leapfrog needs; 0 for an invalid description. */
size_t gp_hmc_workspace_size(const gp_kernel *k, const gp_hmc_params *p, const gp_batch *b);

/*
 * gp_hmc_leapfrog -- one HMC trajectory of theta given phi for every chain: the Hamiltonian
 * H = U_phi(theta) + 1/2 pi^T M^{-1} pi (Section 3.2, eq. U; M^{-1} = diag(p->inv_mass), or I),
 * n_steps drift-kick-drift
 * Stormer-Verlet steps (Section 3.2.2) with the force of Section 3.2.1 (solve A x = y by
 * conjugate gradients warm-started from x_warm, then the frozen-x gradient of eq. (u) as one
 * quadratic-form pass), and the Metropolis decision of Algorithm 1 (steps 6-10).
 *
 * The energy uses the variational form y^T A^{-1} y ~ 2 y^T x - x^T A x of the solved x.
 * Randomness is supplied by the caller: pi already drawn, u_accept uniform on [0, 1).
 *
 *   X, y        device, packed per gp_batch; X in the kernel precision, y likewise
 *   phi         device, per chain, kernel precision
 *   theta, pi   device double, in/out: on return theta is the accepted state (the start state
 *               if rejected) and pi the proposal's end momentum (start momentum if rejected)
 *   x_warm      device, in/out, kernel precision: CG start at theta on entry; on return the
 *               solve at the returned theta
 *   u_accept    device double per chain, or NULL: no decision, every proposal is kept
 *   H0, H1      device double per chain: energies at the start and at the proposal
 *   accepted    device int32 per chain (1 accepted, 0 rejected)
 *   status      device int32 per chain, GP_CHAIN_* bits
 *   cg_iters    device int32 per chain: CG iterations used over the trajectory, or NULL
 */
gp_status gp_hmc_leapfrog(const gp_kernel *k, const gp_hmc_params *p, const gp_batch *b,
                          const void *X, const void *y, const void *phi, double *theta,
                          double *pi, void *x_warm, const double *u_accept, double *H0,
                          double *H1, int32_t *accepted, int32_t *status, int32_t *cg_iters,
                          void *ws, size_t ws_bytes, hipStream_t stream);

/*
 * gp_rwm -- one random-walk Metropolis update of theta given phi for every chain (the update of
 * theta in Section 3 may be RWM or HMC; the proposal and acceptance rule are those given at the
 * start of Section 4): the proposal
 * theta' = theta + dt * xi, with xi ~ N(0, I) drawn by the caller, is accepted when
 * log u <= U_phi(theta) - U_phi(theta').  Both energies U_phi (eq. U, without a kinetic term) come
 * from one conjugate-gradient solve warm-started from x_warm and one quadratic-form pass each,
 * exactly as the end-point energies of gp_hmc_leapfrog.  With p->inv_mass the step is
 * dt * sqrt(inv_mass) * xi (proposal covariance dt^2 M^{-1}; a zero entry holds that component).  Parameters, batch packing, workspace
 * (gp_hmc_workspace_size) and modes are those of gp_hmc_leapfrog; p->n_steps is ignored and
 * p->dt is the proposal scale.
 *
 *   xi          device double per chain (packed as theta), in: the proposal direction; unchanged
 *               on return
 *   theta       device double, in/out: the accepted proposal, or the start state if rejected
 *   x_warm      device, in/out: CG start at theta on entry; on return the solve at the returned
 *               theta
 *   u_accept    device double per chain, or NULL: no decision, every proposal is kept
 *   U0, U1      device double per chain: U_phi at theta and at the proposal
 *   accepted, status, cg_iters   as for gp_hmc_leapfrog
 */
gp_status gp_rwm(const gp_kernel *k, const gp_hmc_params *p, const gp_batch *b, const void *X,
                 const void *y, const void *phi, double *theta, double *xi, void *x_warm,
                 const double *u_accept, double *U0, double *U1, int32_t *accepted,
                 int32_t *status, int32_t *cg_iters, void *ws, size_t ws_bytes,
                 hipStream_t stream);

/*
 * Autotuning of the trajectory launch (batched and graph modes).  For the class of a batch --
 * precision, kernel kind, largest padded d, kernel variant (preconditioned, Chebyshev-amplitude,
 * GP_BF16X), floor(log2) of its number of chains and of its largest N -- gp_tune_hmc times launch
 * configurations on synthetic inputs of the batch's geometry (the instances' N and d and the
 * chains per instance of `b`; a 1-step trajectory with 8 CG iterations per solve, so every
 * configuration runs the same jobs), one knob at a time from the defaults (a candidate must be
 * more than 4% faster to replace the current choice), and records the winner in the tuning
 * table of gp_tune_products, which later gp_hmc_leapfrog / gp_rwm calls of
 * that class use.  Knobs: the persistent kernel compiled for its default or its alternative
 * number of waves per SIMD, and the product jobs' columns per trip (4 or 2 for padded d <= 8,
 * 2 or 1 above).  No configuration changes any result: the sums run in the same order.  `p` supplies the preconditioner rank
 * (its factor is not read); its other fields are ignored.  `ws`: at least
 * gp_tune_hmc_workspace_size bytes of device memory; the call synchronises `stream`.
 */
size_t gp_tune_hmc_workspace_size(const gp_kernel *k, const gp_hmc_params *p, const gp_batch *b);
gp_status gp_tune_hmc(const gp_kernel *k, const gp_hmc_params *p, const gp_batch *b, void *ws,
                      size_t ws_bytes, hipStream_t stream);

/*
 * Gibbs refresh of phi (Section 3.1): given theta, phi | theta ~ N(0, A^{-1}) is drawn as
 * phi = A^{-1/2} xi with xi ~ N(0, I) supplied by the caller, through the pole expansion
 * A^{-1/2} ~ sum_p w_p (A + lambda_p I)^{-1} (eq. pex) with the weights and shifts of
 * Appendix A (eq. msqdisc) on the spectral interval [m, M].
 *
 * gp_pole_weights -- host only (no GPU use): the n_poles weights w[j] and shifts shift[j] >= 0 for
 * 0 < m <= M.  K(1 - k^2), k^2 = m / M, and the Jacobi functions at the imaginary nodes come from
 * the arithmetic-geometric mean; Jacobi's imaginary transformation makes every node real.
 * The approximation error of the expansion on [m, M] decays like exp(-2 pi K(k^2) N_p / K(1-k^2)).
 */
gp_status gp_pole_weights(double m, double M, int32_t n_poles, double *w, double *shift);

enum {
  GP_PHI_CG_MAXIT = 1,  /* some shifted system had not reached tol after maxit iterations */
  GP_PHI_NONFINITE = 2, /* a NaN or infinity appeared (or A p . p <= 0): phi is not usable */
  GP_PHI_ABORTED = 4    /* gp_phi_refresh_chains: the scheduler stopped before the chain finished */
};

typedef struct {
  int32_t n_poles;    /* N_p, 1..64 (15 gives ~1e-11 relative accuracy at condition 1e4) */
  double tol;         /* relative residual |xi - (A + lambda_p I) x_p| / |xi| of every pole, > 0 */
  int32_t maxit;      /* iteration limit, >= 1 */
  double lambda_max;  /* M >= lambda_max(A); <= 0: the Gershgorin bound max_i (A 1)_i is used */
  int32_t precond_rank;      /* 0: multi-shift CG; 1..512: Nystrom-preconditioned CG per pole */
  const void *precond_U;     /* device n x rank (gp_nystrom's U), kernel precision, or NULL */
  const double *precond_lam; /* device rank values (gp_nystrom's lam), or NULL */
} gp_phi_params;

/* Bytes of workspace gp_phi_refresh needs; 0 for an invalid description or n = 0. */
size_t gp_phi_workspace_size(const gp_kernel *k, const gp_phi_params *p, int64_t n, int32_t r);

/*
 * gp_phi_refresh -- phi = A(theta)^{-1/2} xi for r right-hand sides at once.
 *
 * The lower spectral bound is m = sigma^2 (read from theta).  Without a preconditioner all N_p
 * shifted systems are solved together by multi-shift conjugate gradients on A: one product with A
 * per iteration for every right-hand side, the shifted iterates following from the unshifted CG
 * scalars; phi accumulates sum_p w_p x_p directly.  With a Nystrom factor (precond_rank > 0; the
 * factor of K at any theta, reused across the shifts as Section 3.1 describes) the shifted systems
 * of each column are solved as one batch of preconditioned CG columns by gp_pcg_solve (the
 * preconditioner of A + lambda_p I uses mu = sigma^2 + lambda_p), then combined; iters reports the
 * largest pole's count.  Iteration stops per column once every pole's residual is below tol.
 * The host checks convergence every few iterations; the call synchronises `stream`.
 *
 *   X         device, n x d, kernel precision (GP_NO_NOISE is rejected: no lower bound m)
 *   theta     device double[n_theta]
 *   xi        device, n x r (r in 1..32), leading dimension ldxi >= r, kernel precision
 *   phi       device out, n x r, leading dimension ldphi >= r; may be xi itself (same ld),
 *             must not overlap it otherwise
 *   status    device int32[r] or NULL: GP_PHI_* bits per column (0 = converged)
 *   iters     device int32[r] or NULL: iterations used per column
 *   bounds    host double[2] or NULL: the m and M used
 * Vectors are kept in the kernel precision (float for GP_F32 / GP_BF16X); scalars in double.
 */
gp_status gp_phi_refresh(const gp_kernel *k, const gp_phi_params *p, int64_t n, const void *X,
                         const double *theta, int32_t r, const void *xi, int64_t ldxi, void *phi,
                         int64_t ldphi, int32_t *status, int32_t *iters, double *bounds, void *ws,
                         size_t ws_bytes, hipStream_t stream);

/* Bytes of workspace gp_phi_refresh_chains needs; 0 for an invalid description. */
size_t gp_phi_chains_workspace_size(const gp_kernel *k, const gp_phi_params *p, int32_t mode,
                                    const gp_batch *b);

/*
 * gp_phi_refresh_chains -- the Gibbs step phi | theta of Algorithm 1 for every chain of a batch,
 * each at its own theta: phi_c = A(theta_c)^{-1/2} xi_c by the pole expansion of Section 3.1
 * (eq. pex) with the weights and shifts of Appendix A (eq. msqdisc), all shifted systems of a
 * chain solved by multi-shift CG on A(theta_c).  The chains run as the trajectory chains of
 * gp_hmc_leapfrog do (same batch packing and modes: GP_HMC_PLAIN, GP_HMC_BATCHED, or
 * GP_HMC_GRAPH, one persistent launch in which every chain's products share the GPU); each
 * chain's weights and shifts are computed on the device for m = sigma^2_c and M = p->lambda_max
 * or, when that is <= 0, the chain's Gershgorin bound max_i (A 1)_i (one extra product).
 * p->precond_rank must be 0 (GP_ERR_UNSUPPORTED otherwise; gp_phi_refresh takes a Nystrom
 * factor for one theta).  A pole is frozen once its residual is below p->tol |xi_c|; a chain
 * ends when all of its poles are frozen, or after p->maxit iterations.  In the batched and graph
 * modes nothing is synchronised; the plain mode reads each chain's state every few jobs.
 *
 *   X        device, packed per gp_batch, kernel precision (GP_NO_NOISE is rejected)
 *   theta    device double, packed per chain as for gp_hmc_leapfrog; read only
 *   xi       device, per chain as phi in gp_hmc_leapfrog, kernel precision
 *   phi      device out, packed as xi; may be xi itself, must not overlap it otherwise
 *   status   device int32 per chain: GP_PHI_* bits (0 = converged)
 *   iters    device int32 per chain or NULL: multi-shift iterations used
 *   bounds   device double[2] per chain or NULL: the m and M used
 *   ws       gp_phi_chains_workspace_size bytes; the graph mode keys its captured launch by ws,
 *            so a workspace shared with gp_hmc_leapfrog calls is recaptured at every switch
 * Vectors are kept in the kernel precision (float for GP_F32 / GP_BF16X); scalars in double.
 */
gp_status gp_phi_refresh_chains(const gp_kernel *k, const gp_phi_params *p, int32_t mode,
                                const gp_batch *b, const void *X, const double *theta,
                                const void *xi, void *phi, int32_t *status, int32_t *iters,
                                double *bounds, void *ws, size_t ws_bytes, hipStream_t stream);

/*
 * Randomized Nystrom preconditioner (Section 3.1 after eq. pex, Section 3.2.3; rank 5 in
 * Section 4.1 and 500 in Section 4.3): a low-rank factor K ~ U diag(lam) U^T of the kernel
 * matrix, which through the Woodbury identity gives an approximate inverse of A + lambda I =
 * K + (sigma^2 + lambda) I for every shift lambda from the same factor.
 *
 * gp_nystrom -- U and lam for the Gaussian test matrix omega supplied by the caller:
 * Q = orth(omega) (Cholesky-QR, twice), Y = K Q, nu = sqrt(n) eps |Y|_F, C^T C = Q^T (Y + nu Q),
 * B = (Y + nu Q) C^{-1} = U S V^T, lam = max(0, S^2 - nu) (descending).  The l x l Cholesky
 * factorisations and the eigendecomposition of B^T B run on the host in double; the call
 * synchronises `stream`.
 *   omega   device, n x rank, contiguous (leading dimension rank), kernel precision
 *   U       device out, n x rank, contiguous, kernel precision (orthonormal columns)
 *   lam     device out, double[rank]
 *   rank    1..min(n, 512)
 */
size_t gp_nystrom_workspace_size(const gp_kernel *k, int64_t n, int32_t rank);
gp_status gp_nystrom(const gp_kernel *k, int64_t n, const void *X, const double *theta,
                     int32_t rank, const void *omega, void *U, double *lam, void *ws,
                     size_t ws_bytes, hipStream_t stream);

enum {
  GP_CG_MAXIT = 1,     /* the column had not reached tol after maxit iterations */
  GP_CG_NONFINITE = 2  /* a NaN or infinity appeared (or p^T A p <= 0) */
};

/*
 * gp_pcg_solve -- (A(theta) + lambda_c I) x_c = b_c for r columns at once by conjugate
 * gradients, preconditioned with P^{-1} = U diag((lam_rank + mu_c) / (lam + mu_c)) U^T +
 * (I - U U^T), mu_c = sigma^2 + lambda_c, when rank > 0 (plain CG when rank = 0).  These are
 * the solves of eq. (xtheta) (lambda = 0) and of the pole expansion eq. (pex) (lambda = the
 * shifts).  Each column stops at |b_c - (A + lambda_c) x_c| <= tol |b_c| (recurrence residual).
 * The host checks convergence every few iterations; the call synchronises `stream`.
 *   B        device, n x r (r in 1..32), leading dimension ldb >= r
 *   x        device, n x r, leading dimension ldx >= r: start on entry, solution on return
 *   col_shift device double[r] or NULL (all 0)
 *   U, lam   the gp_nystrom factor (U n x rank contiguous), or NULL with rank = 0
 *   status   device int32[r] or NULL: GP_CG_* bits per column (0 = converged)
 *   iters    device int32[r] or NULL: iterations used per column
 * GP_NO_NOISE is rejected.
 */
size_t gp_pcg_workspace_size(const gp_kernel *k, int64_t n, int32_t r, int32_t rank);
gp_status gp_pcg_solve(const gp_kernel *k, int64_t n, const void *X, const double *theta,
                       int32_t r, const void *B, int64_t ldb, void *x, int64_t ldx,
                       const double *col_shift, int32_t rank, const void *U, const double *lam,
                       double tol, int32_t maxit, int32_t *status, int32_t *iters, void *ws,
                       size_t ws_bytes, hipStream_t stream);

/*
 * Implicit midpoint HMC (Section 3.2.3, eq. implicitsystem) solved by Anderson-accelerated
 * fixed-point iteration of eq. (Phi) (Appendix B), for one chain.
 *
 * Each step seeks (theta_1, pi_1, x) with theta_1 = theta_0 + dt (pi_0 + pi_1)/2,
 * pi_1 = pi_0 - dt F(m, x) and A(m) x = y at m = (theta_0 + theta_1)/2, as the fixed point of
 * Phi(theta, pi, x) = (theta_0 + dt (pi_0 + pi)/2, pi_0 - dt F(m, x), x + (y - A(m) x)/c), where
 * F is the frozen-x force of Section 3.2.1 and c ~ rho(A(theta_0)) from power iterations (the
 * rescaling preconditioner R = I/c); with a Nystrom factor (rank > 0) R = P^{-1}/c instead, P
 * the Nystrom preconditioner of A(theta_0) and c ~ rho(P^{-1} A(theta_0)) (the Nystrom-based R of
 * Section 3.2.3).  Every evaluation of Phi is one fused quadratic-form pass
 * over [x | phi].  The unknowns are stacked into one vector and accelerated with Anderson
 * mixing of depth `history` (0: plain fixed-point iteration).  A step has converged when the
 * (theta, pi) update is below tol (max norm, relative to 1 + |(theta, pi)|) and
 * |y - A(m) x| <= tol |y|.  The energies use solves at theta_0 and theta_1 by gp_pcg_solve
 * (Nystrom-preconditioned when rank > 0) and the variational form of y^T A^{-1} y; the
 * Metropolis decision is that of Algorithm 1.  The fixed-point iteration runs on the device
 * (the Anderson least-squares problem included) as a captured graph of four iterations, which
 * the host replays and checks for convergence after each replay; the call synchronises
 * `stream`.
 *   X, y, phi     device, n x d / n / n, kernel precision
 *   theta, pi     device double[n_theta], in/out (accepted state or the start state); theta is
 *                 also used as scratch during the call
 *   x_warm        device, n: start of the first solve; on acceptance the solve at theta_1
 *   u_accept      device double or NULL (no decision: the proposal is kept)
 *   U, lam, rank  optional Nystrom factor (at theta_0) for R and the endpoint solves (rank 0: none)
 *   H0, H1        device double; accepted, status (GP_CHAIN_* bits), iters (Anderson
 *                 iterations over the trajectory) device int32
 */
typedef struct {
  int32_t n_steps;   /* implicit steps per trajectory, N_int >= 0 */
  double dt;         /* step size */
  int32_t history;   /* Anderson depth k, 0..20 (10 in the paper) */
  double tol;        /* fixed-point tolerance on (theta, pi) and on the linear part, > 0 */
  int32_t maxit;     /* fixed-point iterations per step, >= 1 */
  double cg_tol;     /* relative residual of the endpoint solves (energies at theta_0, theta_1) */
  int32_t cg_maxit;  /* iteration limit of the endpoint solves */
  int32_t power_its; /* power iterations for c (10 in the paper), >= 1 */
} gp_implicit_params;

size_t gp_implicit_workspace_size(const gp_kernel *k, const gp_implicit_params *p, int64_t n,
                                  int32_t rank);
gp_status gp_hmc_implicit(const gp_kernel *k, const gp_implicit_params *p, int64_t n,
                          const void *X, const void *y, const void *phi, double *theta, double *pi,
                          void *x_warm, const double *u_accept, int32_t rank, const void *U,
                          const double *lam, double *H0, double *H1, int32_t *accepted,
                          int32_t *status, int32_t *iters, void *ws, size_t ws_bytes,
                          hipStream_t stream);

#ifdef __cplusplus
}
#endif

#endif /* GPK_H */
