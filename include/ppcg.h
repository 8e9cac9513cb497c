/*
 * ppcg.h -- C ABI of the prior-preconditioned conjugate-gradient sampler.
 *
 * Nishimura & Suchard, "Prior-preconditioned conjugate gradient method for
 * accelerated Gibbs sampling in 'large n & large p' Bayesian sparse
 * regression".  The library draws
 *
 *     beta ~ N(Phi^-1 X^T Omega z, Phi^-1),  Phi = X^T Omega X + tau^-2 Lambda^-2
 *
 * (Section 1, eq. beta_conditional) by Prop 2.1: it forms the random vector
 *
 *     b = X^T Omega z + X^T Omega^1/2 eta + tau^-1 Lambda^-1 delta
 *
 * (eq. cg_sampler_target_vector) and solves Phi beta = b (eq.
 * linear_system_for_cg_sampler) by conjugate gradient (Supplement S2)
 * preconditioned with the prior precision M = tau^-2 Lambda^-2 (Section 2.4),
 * touching X only through the products v -> X v and w -> X^T w.
 *
 * Conventions shared by every entry point
 * ----------------------------------------
 * - X is binary (every stored entry equals one) and is given once as CSR
 *   index arrays; the handle owns device copies of the CSR and CSC index
 *   arrays and of its workspace.
 * - Vector arguments are DEVICE pointers owned by the caller, contiguous, with
 *   element type given by `dtype` (PPCG_F64: double, PPCG_F32: float).  The
 *   library keeps no pointer to them after the call returns.
 * - Work is enqueued on `stream` (a hipStream_t; NULL is the null stream).
 *   Entry points that take a `ppcg_info*` block the host until the result is
 *   written (the solver checks convergence from the host between batches of
 *   iterations); the others are asynchronous on `stream`.
 * - tau > 0, omega_i > 0 and lambda_j > 0 are the caller's responsibility for
 *   device vectors (they are not read back); violations give non-finite
 *   results or PPCG_EBREAKDOWN, not memory faults.
 * - Return values report synchronous problems (PPCG_EINVAL, PPCG_ENOMEM,
 *   PPCG_EHIP).  Convergence problems (PPCG_ENOTCONV, PPCG_EBREAKDOWN) are
 *   reported in ppcg_info.status and are also returned.
 * - No C++ exception crosses this interface.  A handle must not be used by
 *   two calls at the same time (it holds the solver's workspace).
 * - Results are bitwise reproducible: every reduction is summed in a fixed
 *   order (per-block partials, no floating-point atomics), so the same call
 *   on the same inputs and handle gives the same bits, and a batched chain
 *   on its own design gives the bits of the same chain drawn alone (chains
 *   that share one design run the K-wide passes, summed in another order).
 *   There is no non-deterministic mode, hence no option to select one.
 */
#ifndef PPCG_H
#define PPCG_H

#include <stdint.h>
#include <hip/hip_runtime_api.h>

#ifdef __cplusplus
extern "C" {
#endif

/* Status codes. */
#define PPCG_OK 0
#define PPCG_EINVAL 1     /* bad argument (size, pointer, index out of range, unsorted) */
#define PPCG_ENOMEM 2     /* device or host allocation failed                         */
#define PPCG_EHIP 3       /* a HIP runtime call or kernel launch failed               */
#define PPCG_ENOTCONV 4   /* max_iter reached; the last iterate is returned           */
#define PPCG_EBREAKDOWN 5 /* <s, Phi s> <= 0 or non-finite (Phi not positive definite) */
#define PPCG_ENODEV 6     /* no HIP device                                            */
#define PPCG_ETOOBIG 7    /* needs more scratch than an entry point that allocates nothing has */

/* Element type of vector arguments (and of the CG iteration's matvecs). */
#define PPCG_F64 0 /* FP64 vectors and matvecs throughout                               */
#define PPCG_F32 1 /* FP32 matvec vectors; FP64 state, inner products, scalars, RHS,
                      true residual; optional FP64-residual refinement restart       */

/* Stopping rules, all on the prior-preconditioned residual r~ = tau lambda (b - Phi beta)
 * of Supplement S4.2 (|| r~ ||^2 = <r, M^-1 r>) unless noted. */
#define PPCG_REL_PRECOND 0     /* ||r~_k|| <= tol * ||tau lambda b||                        */
#define PPCG_RMS_PRECOND_ABS 1 /* p^-1/2 ||r~_k|| <= tol  (eq. mean_sq_resid_for_cg_termination) */
#define PPCG_REL_PLAIN 2       /* ||r_k|| <= tol * ||b||  (the usual l2 rule, for comparison) */

/* Where ppcg_matrix_create reads its index arrays from. */
#define PPCG_MEM_HOST 0
#define PPCG_MEM_DEVICE 1

/* Random streams of the counter-based generator (ppcg_normals). */
#define PPCG_STREAM_ETA 0
#define PPCG_STREAM_DELTA 1

typedef struct ppcg_matrix ppcg_matrix;
typedef struct ppcg_batch ppcg_batch;

typedef struct ppcg_options {
  int32_t dtype;      /* PPCG_F64 or PPCG_F32                                        */
  int32_t criterion;  /* PPCG_REL_PRECOND (default), PPCG_RMS_PRECOND_ABS, PPCG_REL_PLAIN */
  int32_t max_iter;   /* cap on CG iterations per phase; <= 0 means p (CG is exact
                         in p steps in exact arithmetic, Section 2.2)             */
  int32_t refine;     /* 1: after convergence, if the FP64 true residual misses the
                         rule, restart once from it; -1: default (1 for F32, 0 for F64) */
  double tol;         /* tolerance of the stopping rule (default 1e-6)           */
  int32_t true_resid; /* 1 (default): recompute b - Phi beta in FP64 at the end     */
  int32_t check_every;/* host convergence check period in iterations (0: default 16);
                         a batch queued when the decay of the rule measure
                         predicts the end within one period is shortened to
                         the predicted remainder plus one iteration.  The
                         first batch of a solve phase (first solve from
                         zero, first solve from a given beta0, refinement
                         restart) runs to 2 iterations short of the same
                         handle's previous phase of that kind and
                         precision, with 3 more queued behind it, when that
                         phase converged; results do not depend on batching */
  double loop_factor; /* the recursion runs to loop_factor * tol before the FP64
                         check (0: default, 0.5 for F32 and 1 for F64)         */
  int32_t no_graph;   /* batched loops: 0 (default) replays each check batch as a
                         captured HIP graph; 1 launches its kernels directly   */
  int32_t reserved[3];
} ppcg_options;

typedef struct ppcg_info {
  int32_t status;       /* PPCG_OK, PPCG_ENOTCONV or PPCG_EBREAKDOWN               */
  int32_t iters;        /* CG iterations of the first phase                        */
  int32_t refine_iters; /* CG iterations of the refinement restart (0 if none)     */
  int32_t refined;      /* 1 if the refinement restart ran                          */
  double resid_rec;     /* rule value of the recursive residual at exit, divided by
                           tol (<= 1 means the rule holds)                          */
  double resid_true;    /* the same for the FP64 true residual b - Phi beta (-1 when
                           not computed)                                            */
  double rms_precond;   /* p^-1/2 ||tau lambda (b - Phi beta)|| (the paper's measure) */
  double bnorm_precond; /* ||tau lambda b||                                         */
  double resid_true_first; /* resid_true after the first phase, before any
                              refinement (-1 when not computed)                   */
} ppcg_info;

/* Fills `opt` with the defaults listed above for the given dtype. */
void ppcg_options_default(ppcg_options* opt, int32_t dtype);

/* Static string for a status code. */
const char* ppcg_status_string(int status);

/* Library version string. */
const char* ppcg_version(void);

/*
 * Creates a handle for the n x p binary design X (Section 1; the application's
 * X is sparse and binary, Section 4).  `row_ptr` (int64, n+1 entries, row_ptr[0]
 * = 0, non-decreasing, row_ptr[n] = nnz) and `col_idx` (int32, nnz entries,
 * strictly increasing within each row, in [0, p)) are host or device pointers
 * as `mem` says; they are copied.  `values` must be NULL (binary X).  Validates
 * the arrays (PPCG_EINVAL on any violation) and builds the CSC twin and the
 * chunk tables of the matvec kernels.  n, p >= 1; nnz >= 0.
 */
int ppcg_matrix_create(ppcg_matrix** out, int64_t n, int64_t p, int64_t nnz,
                       const int64_t* row_ptr, const int32_t* col_idx,
                       const void* values, int32_t mem, hipStream_t stream);

/* Releases the handle and its device memory (NULL is allowed). */
int ppcg_matrix_destroy(ppcg_matrix* X);

/* Sizes of a handle (any output pointer may be NULL). */
/*
 * The same handle from the column-major (CSC) index arrays of X: col_ptr
 * (p + 1, int64) and row_idx (nnz, int32, strictly increasing within each
 * column), on the host or the device as `mem` says.  Validation and
 * errors as ppcg_matrix_create; the row orientation is built from them.
 * For designs generated or stored column by column.
 */
int ppcg_matrix_create_csc(ppcg_matrix** out, int64_t n, int64_t p, int64_t nnz,
                           const int64_t* col_ptr, const int32_t* row_idx, const void* values,
                           int32_t mem, hipStream_t stream);

int ppcg_matrix_shape(const ppcg_matrix* X, int64_t* n, int64_t* p, int64_t* nnz);

/*
 * out = Phi v = X^T (omega .* (X v)) + tau^-2 lambda^-2 .* v  (the product CG
 * needs, Section 2.2; Phi from eq. beta_conditional).  omega: n, lambda, v,
 * out: p, all `dtype`.  Asynchronous on `stream`.
 */
int ppcg_phi_matvec(const ppcg_matrix* X, const void* omega, const void* lambda,
                    double tau, const void* v, void* out, int32_t dtype,
                    hipStream_t stream);

/*
 * ppcg_phi_matvec for callers that cannot allocate device memory (code under
 * HIP graph capture, tight serving loops, harnesses that forbid
 * hipMalloc): the same result from the same kernels (bitwise equal), with
 * every intermediate (d = tau^-2 lambda^-2, both passes' per-panel partial
 * sums and piece sums, the combined X^T u) in a fixed device array of
 * PPCG_NOALLOC_SCRATCH_BYTES per device that the library holds from its
 * first use on that device until the process ends, instead of the handle's
 * workspace (which it does not touch).  The call allocates nothing and
 * calls no allocating routine; it zero-fills what must start at zero with
 * kernels (no memset nodes), so it may be captured into a graph.  Scratch
 * needed, in bytes, each term rounded up to 256: 2 x 8p + sv (P_r n + N_r +
 * P_c p + N_c + p) with sv = 8 (PPCG_F64) or 4 (PPCG_F32), P_r, P_c the
 * panels and N_r, N_c (at least 1) the pieces of the row and column tables
 * of that precision; PPCG_ETOOBIG (nothing enqueued) when that exceeds
 * PPCG_NOALLOC_SCRATCH_BYTES (e.g. n = 5e5, p = 5e4 needs about 23 MB in
 * FP64).  Every call on a device shares that device's array: calls that
 * overlap on one device (two streams, or two threads) race and must be
 * ordered by the caller.  The handle's device must be the current device
 * (PPCG_EINVAL otherwise).  Arguments and errors otherwise as
 * ppcg_phi_matvec; asynchronous on `stream`.
 */
#define PPCG_NOALLOC_SCRATCH_BYTES (32u * 1024u * 1024u)
int ppcg_phi_matvec_noalloc(const ppcg_matrix* X, const void* omega, const void* lambda,
                            double tau, const void* v, void* out, int32_t dtype,
                            hipStream_t stream);

/*
 * Writes `count` standard normals of one stream of the counter-based generator
 * (FP64, device pointer `out`): Philox4x64-10 with key (seed, 0) and counter
 * (i, stream_id, chain, draw_index); block i gives elements 4i..4i+3 by the
 * Box-Muller transform.  These are the eta (stream 0) and delta (stream 1) of
 * Prop 2.1 for draw (seed, chain, draw_index).  Asynchronous.
 */
int ppcg_normals(uint64_t seed, uint64_t stream_id, uint64_t chain,
                 uint64_t draw_index, int64_t count, double* out,
                 hipStream_t stream);

/*
 * b = X^T Omega z + X^T Omega^1/2 eta + tau^-1 Lambda^-1 delta (Prop 2.1,
 * eq. cg_sampler_target_vector) with eta, delta from the generator above.
 * omega, z: n; lambda: p, all `dtype`; b_out: p doubles (always FP64).
 * Asynchronous.
 */
int ppcg_rhs(const ppcg_matrix* X, const void* omega, const void* z,
             const void* lambda, double tau, uint64_t seed, uint64_t chain,
             uint64_t draw_index, int32_t dtype, double* b_out,
             hipStream_t stream);

/*
 * Solves Phi beta = b (eq. linear_system_for_cg_sampler) by CG preconditioned
 * with M = tau^-2 Lambda^-2 (Section 2.4), starting from beta0 (NULL: zero,
 * Section 2.7).  omega: n; lambda, b, beta0, beta_out: p; all opt->dtype.
 * `opt` NULL means defaults for PPCG_F64.  `info` (host pointer, may be NULL)
 * receives iteration counts and residuals.  Blocks until beta_out is written.
 */
int ppcg_solve(const ppcg_matrix* X, const void* omega, const void* lambda,
               double tau, const void* b, const void* beta0,
               const ppcg_options* opt, void* beta_out, ppcg_info* info,
               hipStream_t stream);

/*
 * One draw of beta ~ N(Phi^-1 X^T Omega z, Phi^-1) by Prop 2.1: eta, delta from
 * (seed, chain, draw_index), b as in ppcg_rhs, then ppcg_solve from zero.  The
 * draw is a pure function of its arguments.  omega, z: n; lambda, beta_out: p;
 * all opt->dtype.  Blocks until beta_out is written.
 */
int ppcg_draw(const ppcg_matrix* X, const void* omega, const void* z,
              const void* lambda, double tau, uint64_t seed, uint64_t chain,
              uint64_t draw_index, const ppcg_options* opt, void* beta_out,
              ppcg_info* info, hipStream_t stream);

/*
 * General diagonal prior and preconditioner (Supplement S4.3): coefficients
 * estimated without shrinkage (an intercept, effects of interest) take
 * independent N(0, sigma_j^2) priors, flat when sigma_j is infinite, so
 *   Phi = X^T Omega X + diag(prior_prec),   M^-1 = diag(precond_inv),
 * with prior_prec_j = sigma_j^-2 (0 for a flat prior) for those and
 * tau^-2 lambda_j^-2 for shrunk ones, and precond_inv_j = gamma_j^2 for
 * unshrunk ones (the supplement takes gamma_j = c times an estimate of
 * beta_j's posterior scale, c >= 1) and (tau lambda_j)^2 for shrunk ones.
 * prior_prec (>= 0) and precond_inv (> 0, or NULL for 1 / prior_prec, which
 * needs every prior_prec_j > 0) are FP64 device arrays of p owned by the
 * caller; the other arguments are as in ppcg_solve.  The stopping rules
 * measure the residual in the norm of this M.  A flat prior needs a proper
 * likelihood (X^T Omega X positive on those coordinates) for Phi to be
 * positive definite; otherwise CG reports PPCG_EBREAKDOWN.
 */
int ppcg_solve_general(const ppcg_matrix* X, const void* omega, const double* prior_prec,
                       const double* precond_inv, const void* b, const void* beta0,
                       const ppcg_options* opt, void* beta_out, ppcg_info* info,
                       hipStream_t stream);

/*
 * One draw under the general prior: Prop 2.1 with the prior precision
 * diag(prior_prec), b = X^T Omega z + X^T Omega^1/2 eta +
 * diag(prior_prec)^1/2 delta (eta, delta from (seed, chain, draw_index) as in
 * ppcg_draw), then ppcg_solve_general from beta0 (NULL: zero; a warm start
 * such as the running mean of earlier draws, Section 2.7, saves iterations
 * without changing the law of the draw).
 */
int ppcg_draw_general(const ppcg_matrix* X, const void* omega, const void* z,
                      const double* prior_prec, const double* precond_inv, const void* beta0,
                      uint64_t seed, uint64_t chain, uint64_t draw_index,
                      const ppcg_options* opt, void* beta_out, ppcg_info* info,
                      hipStream_t stream);

/*
 * diag(Phi)_j = sum over the non-zeros of column j of omega_i, plus
 * prior_prec_j: one column pass.  Its reciprocal is the Jacobi
 * preconditioner's M^-1, the alternative the paper compares with (Section
 * 2.4) — pass it as precond_inv.  omega: n of `dtype`; prior_prec, diag_out:
 * FP64 device arrays of p.  Blocks until diag_out is written.
 */
int ppcg_phi_diag(const ppcg_matrix* X, const void* omega, int32_t dtype,
                  const double* prior_prec, double* diag_out, hipStream_t stream);

/*
 * Initial vector of the CG sampler (Supplement S4.1, choice of initial vector:
 * the rescaled running mean).  After draw i, acc += beta^(i) / (tau_prev
 * lambda_prev), with the scales that draw was conditioned on; before the next
 * draw, beta0 = tau lambda * (acc / count) with its scales, passed as beta0 of
 * ppcg_draw_general.  acc: FP64 device array of p owned by the caller (zero
 * it first); beta, lambda, beta0: p of `dtype`; count, tau > 0.  Asynchronous
 * on `stream`; PPCG_EINVAL for bad arguments.
 */
int ppcg_warm_start_accumulate(double* acc, const void* beta, const void* lambda_prev,
                               double tau_prev, int32_t dtype, int64_t p, hipStream_t stream);
int ppcg_warm_start_vector(void* beta0, const double* acc, double count, const void* lambda,
                           double tau, int32_t dtype, int64_t p, hipStream_t stream);

/*
 * Scales of unshrunk coefficients (Supplement S4.3).  The leading q1
 * coefficients (an intercept, effects of interest) get N(0, sigma_j^2)
 * priors (sigma_j^-2 = 0: flat) and preconditioner scales gamma_j =
 * c eta_hat_j, eta_hat_j^2 the variance of beta_j over earlier draws.
 *
 * ppcg_moments_update: Welford's update of the running mean and sum of
 * squared deviations of beta[0:q1) with the count-th draw (count = 1 for the
 * first; zero both arrays before it).  mean, m2: FP64 device arrays of q1;
 * beta: p (only q1 read) of `dtype`.
 *
 * ppcg_unshrunk_setup: writes prior_prec (d) and, if not NULL, precond_inv
 * (m = M^-1) for ppcg_draw_general: d_j = sigma_inv2[j], m_j = c^2 m2[j] /
 * (count - 1) for j < q1 (NaN where that variance is not positive, so a solve
 * with it reports PPCG_EBREAKDOWN); d_j = (tau lambda_j)^-2, m_j = (tau
 * lambda_j)^2 beyond.  q1 = 0 gives the shrinkage prior and preconditioner
 * (sigma_inv2, m2 unused).  lambda: p of `dtype` (entries below q1 unused);
 * sigma_inv2, m2: FP64 device arrays of q1; count >= 2 and c > 0 (the paper
 * takes c >= 1) when precond_inv is wanted and q1 > 0.
 *
 * Both are asynchronous on `stream`; PPCG_EINVAL for bad arguments.
 */
int ppcg_moments_update(double* mean, double* m2, const void* beta, int32_t dtype, int64_t q1,
                        int64_t count, hipStream_t stream);
int ppcg_unshrunk_setup(double* prior_prec, double* precond_inv, const double* sigma_inv2,
                        const double* m2, int64_t count, double c, const void* lambda, double tau,
                        int32_t dtype, int64_t q1, int64_t p, hipStream_t stream);

/*
 * Jacobi preconditioner (the alternative of Sections 2.4 and 3.3): writes
 * precond_inv = 1 / diag(Phi) = 1 / (X^T omega + prior_prec), one column
 * pass over omega.  Arguments as ppcg_phi_diag; precond_inv: FP64 device
 * array of p.  Asynchronous on `stream`.
 */
int ppcg_jacobi_precond(const ppcg_matrix* X, const void* omega, int32_t dtype,
                        const double* prior_prec, double* precond_inv, hipStream_t stream);

/*
 * Polya-Gamma omega update of the Gibbs cycle (Supplement S1, step 3, and
 * eq. pg_augmented_likelihood).
 *
 * ppcg_pg_update: psi = X beta (one FP64 row pass), omega_i ~ PG(1, psi_i)
 * and z_i = (y_i - 1/2) / omega_i, ready for ppcg_draw / ppcg_draw_general.
 * beta: p of `dtype`; y: n device bytes, 0 or 1; omega_out, z_out: n of
 * `dtype`.  Uses the handle's n-sized workspace, so it is ordered with the
 * handle's other calls on `stream`.  Asynchronous.
 *
 * ppcg_pg_sample: omega_i ~ PG(1, c_i) for given FP64 tilts c (device, n),
 * FP64 output.  Asynchronous.
 *
 * Draws are exact (Devroye's alternating-series sampler, as in Polson, Scott
 * & Windle 2013): PG(1, c) = J*(1, |c|/2) / 4.  Element i uses its own
 * Philox4x64-10 stream: uniform k is word k % 4 of the block with counter
 * (i, 2 | (k / 4) << 8, chain, draw_index) and key (seed, 0), mapped to
 * ((w >> 11) + 1/2) 2^-53; stream word 2 sits beside eta (0) and delta (1).
 * PPCG_EINVAL for bad arguments.
 */
int ppcg_pg_update(const ppcg_matrix* X, const void* beta, const uint8_t* y, uint64_t seed,
                   uint64_t chain, uint64_t draw_index, int32_t dtype, void* omega_out,
                   void* z_out, hipStream_t stream);
int ppcg_pg_sample(const double* c, int64_t n, uint64_t seed, uint64_t chain,
                   uint64_t draw_index, double* omega_out, hipStream_t stream);

/*
 * Adaptive choice between the prior and the Jacobi preconditioner
 * (Supplement S5.3: compare the two every so many Gibbs iterations and keep
 * the better).  A switch serves one chain of dimension p on one stream at a
 * time and owns p-sized device workspace (the Jacobi M^-1 and a second
 * draw).
 *
 * ppcg_draw_switch draws as ppcg_draw_general with the caller's prior
 * preconditioner `precond_inv` (NULL: 1 / prior_prec) or with the Jacobi
 * one, whichever the switch holds.  Its first draw and every period-th
 * after it is a trial: the same draw (same b, same beta0) is solved under
 * both, the one that met the stopping rule in fewer CG iterations (first
 * phase plus refinement) is kept and its result returned; a tie, or a Jacobi
 * solve that did not converge, keeps the prior preconditioner (the paper's
 * first choice).  The Jacobi solve runs first and the prior one is stopped
 * at its count (it can win only within it), so a trial costs at most about
 * twice the cheaper solve; the prior count reported is then at most the
 * Jacobi count plus one phase's refinement.  The Jacobi M^-1 is recomputed
 * each draw it is used
 * (omega changes between Gibbs steps).  Returns and blocks as
 * ppcg_draw_general.
 *
 * ppcg_switch_state: the current choice (PPCG_PRECOND_*), the draws made
 * and the two iteration counts of the last trial (-1 before the first);
 * NULL outputs are skipped.
 */
#define PPCG_PRECOND_PRIOR 0
#define PPCG_PRECOND_JACOBI 1
typedef struct ppcg_switch ppcg_switch;
int ppcg_switch_create(ppcg_switch** out, int64_t p, int32_t period);
int ppcg_switch_destroy(ppcg_switch* S);
int ppcg_switch_state(const ppcg_switch* S, int32_t* choice, int64_t* draws,
                      int32_t* iters_prior, int32_t* iters_jacobi);
int ppcg_draw_switch(ppcg_switch* S, const ppcg_matrix* X, const void* omega, const void* z,
                     const double* prior_prec, const double* precond_inv, const void* beta0,
                     uint64_t seed, uint64_t chain, uint64_t draw_index, const ppcg_options* opt,
                     void* beta_out, ppcg_info* info, hipStream_t stream);

/*
 * Adjoint of beta = Phi(lambda, tau)^-1 b for a loss L with g = dL/dbeta:
 * solves Phi a = g with the same preconditioned CG, then
 *   grad_b = a,  grad_loglambda_j = 2 d_j a_j beta_j,  grad_logtau = sum_j of those,
 * d_j = tau^-2 lambda_j^-2 (differentiating eq. beta_conditional: only the
 * prior term of Phi depends on lambda and tau).  b is an independent input.
 * beta, grad_beta, grad_b, grad_loglambda: p, opt->dtype; grad_logtau: one
 * double in device memory.  Blocks until the outputs are written.
 */
int ppcg_solve_backward(const ppcg_matrix* X, const void* omega,
                        const void* lambda, double tau, const void* beta,
                        const void* grad_beta, const ppcg_options* opt,
                        void* grad_b, void* grad_loglambda,
                        double* grad_logtau, ppcg_info* info,
                        hipStream_t stream);

/*
 * Kernel timing of the two X passes of the CG iteration (v -> omega .* X v
 * and w -> X^T w, the products Section 2.2 says dominate each iteration's
 * cost).  With `enable` != 0 the handle has the dispatch of both passes of one
 * iteration in every fourth convergence-check batch of a solve phase,
 * starting with its first (iteration check_every / 2 of the batch, when the
 * batch is longer than that and the iteration runs)
 * stamp HIP events on the caller's stream and accumulates their elapsed
 * times: a sample of the loop's launches, since event-stamped dispatches
 * leave the device idle for microseconds each.  Enabling resets the totals.  Host-only bookkeeping; PPCG_EINVAL
 * for a NULL handle.
 */
int ppcg_matrix_profile(ppcg_matrix* X, int32_t enable);

/*
 * Totals since the last ppcg_matrix_profile(X, 1): milliseconds and launch
 * counts of the row pass (CSR, v -> omega .* X v) and of the column pass (CSC,
 * w -> X^T w).  Any output pointer may be NULL.
 */
int ppcg_matrix_stats(const ppcg_matrix* X, double* csr_ms, int64_t* csr_launches,
                      double* csc_ms, int64_t* csc_launches);

/*
 * Algorithmic bytes of one launch of each X pass in the handle's format for
 * vectors of `dtype`: the index stream (16-byte groups) with its padding, the
 * per-chunk tables, segment boundaries and output slots, the gathered
 * vector read once, and the per-panel partial outputs.  Host-only.
 */
int ppcg_matrix_pass_bytes(const ppcg_matrix* X, int32_t dtype, int64_t* row_pass_bytes,
                           int64_t* col_pass_bytes);

/*
 * Many chains at once (independent Gibbs chains, each drawing as Prop 2.1
 * by the prior-preconditioned CG of Section 2.4 and Supplement S2; the
 * paper runs one).  A batch binds C chains, chain c to the design X[c]
 * (the same handle may serve several chains; sizes may differ between
 * chains).  Each call runs every chain's CG with the per-iteration phases of
 * all chains issued as one launch each (X passes, inner products, updates):
 * a chain that has converged drops out of the launches at once, and the
 * host waits until every chain has.  The result of each chain is the one
 * ppcg_draw / ppcg_solve gives for it (bitwise: the same kernels, blocks and
 * summation order).  `dtype` (PPCG_F64 or PPCG_F32) is fixed per batch; the
 * options passed to the calls must have the same dtype.  The batch owns its
 * workspace (one copy per chain) and keeps pointers to the X handles, which
 * must outlive it.  PPCG_EINVAL for nchains < 1, a NULL handle or bad dtype.
 */
int ppcg_batch_create(ppcg_batch** out, int32_t nchains, const ppcg_matrix* const* X,
                      int32_t dtype, hipStream_t stream);

/*
 * A batch of nchains (1..8) chains on ONE design X (given as for
 * ppcg_matrix_create; copied), each drawing as Prop 2.1 with its own omega,
 * lambda and tau.  Each X pass reads X's indices once for a
 * group of K chains: the group's vectors are interleaved and a panel of the
 * gathered vectors holds K values per entry.  K is 2 for up to two chains,
 * else 4: five to eight chains run as two groups, one pass of each per CG
 * step, the chains dealt to the groups by falling iteration count of the
 * previous call (a group whose chains have all stopped skips its passes).
 * Each chain's omega, z, lambda, tau, b and random stream are its
 * own (ppcg_chain), so the chains' Phi differ and their CG runs are
 * independent (a chain that has converged keeps its result while the
 * others iterate).  Results agree with the single-chain calls to the solver
 * tolerance, not bitwise (the panels are narrower, so sums group
 * differently).  Used with ppcg_draw_batched / ppcg_solve_batched and
 * released by ppcg_batch_destroy.
 */
int ppcg_batch_create_shared(ppcg_batch** out, int32_t nchains, int64_t n, int64_t p,
                             int64_t nnz, const int64_t* row_ptr, const int32_t* col_idx,
                             int32_t mem, int32_t dtype, hipStream_t stream);

/* Releases a batch (not its X handles; NULL is allowed). */
int ppcg_batch_destroy(ppcg_batch* B);

/*
 * One chain's arguments of a batched call (host array of C entries; the
 * vectors are device pointers of the batch's dtype, lengths those of the
 * chain's X: omega, z: n_c; lambda, b, beta_out: p_c).  Draws read z, seed,
 * chain and draw_index (the draw is ppcg_draw's for these); solves read b.
 */
typedef struct ppcg_chain {
  const void* omega;
  const void* z;
  const void* b;
  const void* lambda;
  void* beta_out;
  double tau;
  uint64_t seed;
  uint64_t chain;
  uint64_t draw_index;
} ppcg_chain;

/*
 * One draw for every chain of the batch (Prop 2.1 per chain, as ppcg_draw).
 * `infos` (host array of C entries, may be NULL) receives each chain's
 * result.  Returns PPCG_OK when every chain converged, else the first
 * chain's non-OK status; blocks until every beta_out is written.
 */
int ppcg_draw_batched(ppcg_batch* B, const ppcg_chain* chains, const ppcg_options* opt,
                      ppcg_info* infos, hipStream_t stream);

/* Phi_c beta_c = b_c for every chain (as ppcg_solve from zero). */
int ppcg_solve_batched(ppcg_batch* B, const ppcg_chain* chains, const ppcg_options* opt,
                       ppcg_info* infos, hipStream_t stream);

#ifdef __cplusplus
}
#endif

#endif /* PPCG_H */
