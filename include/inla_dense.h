/*
 * inla_dense.h - C-ABI of the MI355X (gfx950) dense-INLA Laplace-evaluation library.
 *
 * The library evaluates, for a batch of hyperparameter points theta, the per-theta
 * hot path of dense INLA (arXiv 2311.08050, "INLA+"): it assembles the dense
 * posterior precision Q*(theta) = Q_prior(theta) + A^T W(x) A, factors it with a
 * blocked Cholesky, takes log-determinants, runs the Newton iteration for the mode
 * of a non-Gaussian likelihood, corrects every iterate onto the linear constraints
 * C x = e by kriging, and forms the Laplace approximation of log pi(theta | y) and
 * the marginal variances diag(Q*^{-1}) (constraint-corrected).
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 *  - Latent Gaussian model of the paper's Introduction:
 *        y_i | x, theta ~ f(eta_i, theta),  eta = offset + A x,  x | theta ~ N(0, Q_prior^{-1}),
 *    with A = I (m = n observations, one per latent element).
 *  - Matrices are column-major; a symmetric matrix is read from its lower triangle
 *    only.  Constraint matrices C are k x n row-major.
 *  - "device" pointers are HIP device memory owned by the caller; "host" pointers
 *    are ordinary host memory owned by the caller.  The library never frees or
 *    retains caller memory after a call returns.  The handle owns its own
 *    workspace (grown on demand, released by inla_destroy).
 *  - Work is enqueued on the handle's stream.  inla_logdet, inla_constrained_mode,
 *    inla_laplace_eval and inla_marginal_var return only after their results are
 *    complete (the Newton iteration makes host decisions on device flags), so host
 *    outputs are valid on return and device outputs are valid for any later work
 *    on the handle's stream.
 *  - Return value: INLA_OK (0), -i when the i-th argument (1-based) is invalid,
 *    INLA_ERR_HIP on a HIP runtime failure, INLA_ERR_NOMEM when the workspace
 *    cannot be allocated.  Numerical outcomes are reported per theta in `info`
 *    (see INLA_INFO_*); the library never aborts the process.
 *
 * Hyperparameter layout (row b of `theta`, stride `ldtheta` doubles): prior
 * parameters first, then the likelihood parameter.
 *    INLA_PRIOR_EXPCOV          (log tau, log rho, lik)
 *    INLA_PRIOR_KRON_RW1_EXPCOV (log tau, log rho, log delta, lik)
 *    INLA_PRIOR_DENSE           (lik)
 *    lik = log sigma^2 for INLA_LIK_GAUSSIAN (eta = x),
 *          beta0       for INLA_LIK_POISSON  (eta = beta0 + x).
 */
#ifndef INLA_DENSE_H
#define INLA_DENSE_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ------------------------------------------------------------ return codes */
#define INLA_OK 0
#define INLA_ERR_HIP (-1000)
#define INLA_ERR_NOMEM (-1001)
#define INLA_ERR_UNSUPPORTED (-1002)
#define INLA_ERR_TOO_LARGE (-1003)   /* inla_logdet_noalloc: the batch needs more than its fixed scratch */

/* ----------------------------------------------------- per-theta info codes */
/* info == j > 0: the leading minor of order j of the matrix being factored is
 * not positive definite (LAPACK convention). */
#define INLA_INFO_OK 0
#define INLA_INFO_NEWTON_MAXIT (-1)     /* no convergence within max_iter; last iterate returned */
#define INLA_INFO_CONSTRAINT_RANK (-2)  /* C Q^{-1} C^T not positive definite: C lacks full row rank */
#define INLA_INFO_NONFINITE (-3)        /* NaN/Inf in theta, a start vector or an iterate */
#define INLA_INFO_EIG_MAXIT (-4)        /* inla_pinv: Jacobi sweeps did not converge; result from the
                                           last sweep */

/* ----------------------------------------------------------------- enums */
enum { INLA_LIK_GAUSSIAN = 0, INLA_LIK_POISSON = 1 };
enum {
  INLA_PRIOR_DENSE = 0,           /* Q_prior supplied by the caller (model.Qprior)       */
  INLA_PRIOR_EXPCOV = 1,          /* Q_prior = tau Sigma(rho)^{-1}, Sigma_ij = exp(-d_ij/rho) */
  INLA_PRIOR_KRON_RW1_EXPCOV = 2, /* Q_prior = tau (R_t kron Sigma_s(rho)^{-1} + delta I),
                                     R_t the unscaled first-order random walk on n_t
                                     steps, latent index t*n_s + s */
  INLA_PRIOR_PINV = 3             /* inla_woodbury_eval only: model.Qprior holds the
                                     Moore-Penrose inverse Q_prior^+ (full symmetric
                                     storage, model.ldq) of an intrinsic prior */
};
/* Precision of the Newton and final-pass factorisations (extension to the
 * paper's FP64 method).
 *  FP64: everything in FP64.
 *  FP32: FP32 storage and FP32 MFMA (FP32 accumulate) for the blocked Cholesky
 *        of Q*.  The prior pass, the log-det sums, the k x k kriging system and
 *        the residuals stay FP64.  Newton is run inexactly while far from the
 *        mode; once the previous step is below 1e-3 of the iterate's scale (and
 *        always for a Gaussian likelihood) the constrained (KKT) solve is refined
 *        with FP64 residuals until the correction is below 1e-13 relative, and
 *        only a refined step can end the iteration.  The last Newton factor
 *        gives log|Q*|.  A theta whose refinement does not converge within its
 *        budget, whose FP32 (or BF16-operand) factorisation of Q* meets a
 *        non-positive pivot, or whose kriging system built from that factor is
 *        numerically singular, is re-evaluated in FP64 and flagged in
 *        inla_result.fallback (bit 0); its info then comes from the FP64
 *        evaluation.
 *  BF16: as FP32, but the factorisations of the unrefined Newton steps round
 *        the panel operands of the trailing update of Q* to BF16 (FP32 storage,
 *        FP32 accumulation; the border rows keep FP32 operands), and each such
 *        step takes one refinement step with its own factor; refined steps, and
 *        so the factor giving log|Q*|, use FP32.  inla_logdet with BF16 uses
 *        BF16 trailing updates throughout. */
enum { INLA_PREC_FP64 = 0, INLA_PREC_FP32 = 1, INLA_PREC_BF16 = 2, INLA_PREC_COUNT = 3 };

typedef struct inla_handle inla_handle;

/* One latent Gaussian model.  The struct itself is host memory; the arrays it
 * points to are device memory. */
typedef struct inla_model {
  int32_t n;      /* latent size = number of observations (A = I); n >= 1          */
  int32_t k;      /* number of constraint rows (0: unconstrained); k < n            */
  int32_t lik;    /* INLA_LIK_*                                                     */
  int32_t prior;  /* INLA_PRIOR_*                                                   */
  int32_t n_s;    /* EXPCOV: must equal n; KRON: number of regions                  */
  int32_t n_t;    /* EXPCOV: 1; KRON: number of time points, n = n_s * n_t          */
  int32_t ldq;    /* DENSE: leading dimension of Qprior (>= n); otherwise ignored    */
  int32_t reserved;
  const double *y;      /* device [n] observations                                  */
  const double *E;      /* device [n] Poisson exposure phi, or NULL for all ones    */
  const double *C;      /* device [k*n] constraint rows, row-major; NULL iff k == 0 */
  const double *e;      /* device [k] constraint right-hand side, or NULL for zeros */
  const double *coords; /* device [n_s*2] points (x, y) row-major (EXPCOV, KRON)    */
  const double *Qprior; /* device, DENSE only: column-major n x n, lower triangle   */
  /* Design matrix A (eta = offset + A x, the LGM of the Introduction).  m = 0:
   * A = I and y, E have n entries.  m >= 1: A is m x n in CSR form (device
   * arrays A_rowptr [m + 1], A_col [nnz], A_val [nnz], column indices in
   * [0, n), A_rowptr[0] = 0, A_rowptr[m] = nnz) and y, E have m entries.
   * Then Q* = Q_prior + A^T W A, whose pattern the library derives on the host
   * once per call; such models are evaluated in FP64 (INLA_PREC_FP64 only)
   * and the variational-Bayes correction is not available for them. */
  int32_t m;
  int32_t nnz;
  const int32_t *A_rowptr;
  const int32_t *A_col;
  const double *A_val;
} inla_model;

/* Newton options (appendix "Gaussian approximation strategy", algorithm
 * "Gaussian Approximation"; the paper leaves norm and tolerance open, here
 * ||x_new - x||_inf <= tol * max(1, ||x_new||_inf)). */
typedef struct inla_opts {
  int32_t prec;      /* INLA_PREC_FP64, INLA_PREC_FP32 or INLA_PREC_BF16             */
  int32_t max_iter;  /* <= 0: 50                                                     */
  double tol;        /* <= 0: 1e-11                                                  */
  int32_t start;     /* 0: start from x = 0; 1: start from the vectors in x (a warm
                        start, e.g. inla_mlp_predict_modes or a previous mode).  A warm
                        start that fails or exceeds max_iter is retried from x = 0
                        with the default budget (result.fallback bit 1).          */
  int32_t reserved;
} inla_opts;

/* Per-theta results of inla_laplace_eval / inla_constrained_mode (host). */
typedef struct inla_result {
  double objective;     /* log pi~(y | theta) with pi(theta) excluded, Eq. (41)      */
  double logdet_qprior; /* log|Q_prior|                                              */
  double logdet_sprior; /* log|C Q_prior^{-1} C^T| (0 if k = 0)                      */
  double ese;           /* e^T (C Q_prior^{-1} C^T)^{-1} e (0 if k = 0)               */
  double xqx;           /* x*^T Q_prior x*                                           */
  double loglik;        /* sum_i log pi(y_i | eta*_i), normalising constants included */
  double logdet_qstar;  /* log|Q*| at the mode                                       */
  double logdet_s;      /* log|C Q*^{-1} C^T| at the mode (0 if k = 0)               */
  double step;          /* last Newton step ||x_new - x||_inf                        */
  int32_t iters;        /* Newton iterations taken                                   */
  int32_t info;         /* INLA_INFO_* or leading-minor index                        */
  int32_t ir_steps;     /* mixed precision: refinement steps summed over iterations  */
  int32_t fallback;     /* bit 0: re-evaluated in FP64 (refinement did not converge);
                           bit 1: warm start failed, re-evaluated from x = 0          */
} inla_result;

/* ------------------------------------------------------------ lifecycle */
/* Create a handle bound to `stream` (a hipStream_t; NULL = the null stream) on
 * the current HIP device.  *h receives the handle.  Returns INLA_OK or an error. */
int inla_create(inla_handle **h, void *stream);
/* Release the handle and its workspace.  NULL is accepted. */
int inla_destroy(inla_handle *h);
/* Rebind the handle to another stream of the same device. */
int inla_set_stream(inla_handle *h, void *stream);

/* ------------------------------------------------------------ hot path */

/* log-determinants of B symmetric positive-definite matrices (the Gaussian
 * normalisers of Eq. (41)): Q_b = L_b L_b^T by blocked Cholesky, log|Q_b| =
 * 2 sum_i log (L_b)_ii.
 *   B        number of matrices (>= 0)
 *   n        host [B] orders (>= 0; 0 gives log-det 0)
 *   Q        host [B] of device pointers, column-major, lower triangle read; on
 *            return the lower triangle holds L_b (strict upper triangle untouched)
 *   ldq      host [B] leading dimensions (>= max(1, n_b))
 *   prec     INLA_PREC_FP64, or INLA_PREC_FP32 / INLA_PREC_BF16 for a factor
 *            stored in FP32 (trailing updates with FP32 or BF16 operands, FP32
 *            accumulation; the log-sum of the diagonal in FP64).  The returned
 *            L is the factor converted to FP64.
 *   logdet   host [B] output
 *   info     host [B] output: 0, or j > 0 if the leading minor j is not positive
 *            definite (then logdet is NaN and Q_b holds a partial factor).
 * Returns INLA_ERR_UNSUPPORTED for an unknown precision. */
int inla_logdet(inla_handle *h, int32_t B, const int32_t *n, double *const *Q, const int32_t *ldq, int32_t prec,
                double *logdet, int32_t *info);

/* inla_logdet for callers that cannot allocate device memory: code under HIP
 * graph capture, tight serving loops, harnesses that forbid hipMalloc.  Same
 * arguments, results and status codes as inla_logdet (the same kernels), but
 * the call allocates nothing: every scratch buffer of the factorisation
 * (padded working matrices, diagonal-block inverses, result slots and status
 * words, BF16 panel copies) lives in one fixed device array of
 * INLA_NOALLOC_SCRATCH_BYTES per GPU, reserved when the library is loaded and
 * held until the process ends; descriptors go through the handle's upload
 * ring (allocated by inla_create); launch chains run without graphs (a new
 * graph would allocate), without lookahead and without profiling events.
 * Needed scratch per matrix of order n (np = n rounded up to 128, e = 8 bytes
 * for FP64, 4 for FP32 and BF16): e np^2 + 64 e np + 8 (4 np + 80) bytes, each
 * term rounded up to 256, plus 28 bytes per matrix of status words and
 * results, plus for BF16 2048 np bytes (512-wide panels); e.g. one FP64 matrix
 * up to n = 2816, or seven of n = 1024.  A larger batch returns
 * INLA_ERR_TOO_LARGE before any work is enqueued.  Every call on a GPU
 * shares that GPU's array, which keeps the last call's contents (the status
 * words are cleared by the call itself): calls that overlap on one GPU, from
 * two handles or two host threads, race and must be serialised by the caller. */
#define INLA_NOALLOC_SCRATCH_BYTES (64 << 20)
int inla_logdet_noalloc(inla_handle *h, int32_t B, const int32_t *n, double *const *Q, const int32_t *ldq,
                        int32_t prec, double *logdet, int32_t *info);

/* Constrained Newton mode of the Gaussian approximation for B theta points
 * (algorithm "Gaussian Approximation": Q* = Q_prior + Q_l(x), b = grad + Q_l x,
 * solve Q* x = b; each iterate conditioned on C x = e by kriging, section
 * "Identifiability constraints" and the appendix on an IGMRF under linear
 * constraints).
 *   models   host [B] model descriptions (may repeat; n may differ across b)
 *   theta    host [B * ldtheta] hyperparameters (layout above)
 *   x        host [B] of device pointers to [n_b] doubles: start vector when
 *            opts->start == 1, the mode on return
 *   opts     host options, NULL for defaults
 *   res      host [B] results: iters, step and info are set (other fields 0). */
int inla_constrained_mode(inla_handle *h, int32_t B, const inla_model *models, const double *theta,
                          int32_t ldtheta, double *const *x, const inla_opts *opts, inla_result *res);

/* Laplace approximation of log pi(theta | y) at B theta points (Eq. (41),
 * mode-approx), with the constraint terms of conditioning on C x = e:
 *   objective = 1/2 log|Q_p| + 1/2 log|S_p| + 1/2 e^T S_p^{-1} e - 1/2 x*^T Q_p x*
 *               + sum_i log pi(y_i | eta*_i) - 1/2 log|Q*| - 1/2 log|S|,
 *   S_p = C Q_p^{-1} C^T, S = C Q*^{-1} C^T, Q* refactored at the mode x*.
 * Arguments as inla_constrained_mode; every field of res[b] is set. */
int inla_laplace_eval(inla_handle *h, int32_t B, const inla_model *models, const double *theta,
                      int32_t ldtheta, double *const *x, const inla_opts *opts, inla_result *res);

/* Marginal variances at a given mode (Eq. (VBA): x | theta ~ N(x*, Q*^{-1}),
 * with the kriging correction of the appendix on an IGMRF under constraints):
 *   var_i = (Q*^{-1})_ii - (V S^{-1} V^T)_ii,  V = Q*^{-1} C^T,  S = C V.
 *   x_mode   host [B] of device pointers to [n_b] modes (read)
 *   var      host [B] of device pointers to [n_b] outputs
 *   info     host [B] outputs (0, leading-minor index, or INLA_INFO_CONSTRAINT_RANK) */
int inla_marginal_var(inla_handle *h, int32_t B, const inla_model *models, const double *theta,
                      int32_t ldtheta, const double *const *x_mode, double *const *var, int32_t *info);

/* ------------------------------------------------------------ learned warm start */
/* A multilayer perceptron u -> x0 that predicts the Newton mode from the
 * normalised hyperparameters u = (theta - centre) / scale, trained on modes the
 * method itself produced.  It only supplies a start vector: the Newton iteration
 * of inla_laplace_eval (opts.start = 1) still decides the result, and a failed
 * warm start falls back to x = 0.
 *   h1 = GELU(W1 u + b1), h2 = GELU(W2 h1 + b2), x0 = W3 h2 + b3,
 *   GELU(z) = z (1 + erf(z / sqrt 2)) / 2, FP32.
 * Parameters are one flat FP32 device array: W1 (H x I, row-major), b1 (H),
 * W2 (H x H), b2 (H), W3 (O x H), b3 (O).  All array arguments are device
 * memory unless marked host; calls complete before returning. */
typedef struct inla_mlp inla_mlp;
/* Create an I -> H -> H -> O network on the handle's device and stream; weights
 * uniform(+-sqrt(6/fan_in)) (last layer +-sqrt(3/H)) from a counter-based
 * generator seeded by `seed`, zero biases, zero Adam moments. */
int inla_mlp_create(inla_handle *h, int32_t n_in, int32_t n_hidden, int32_t n_out, uint64_t seed, inla_mlp **m);
int inla_mlp_destroy(inla_mlp *m);
/* Number of FP32 parameters (host output). */
int inla_mlp_num_params(const inla_mlp *m, int64_t *count);
/* Copy the flat parameter array out / in (set also clears the Adam state). */
int inla_mlp_get_params(inla_mlp *m, float *dst);
int inla_mlp_set_params(inla_mlp *m, const float *src);
/* y (B x O, row-major) = network(x (B x I, row-major)). */
int inla_mlp_forward(inla_mlp *m, int32_t B, const float *x, float *y);
/* Mean-squared-error loss over all B x O outputs against target (B x O, FP64,
 * e.g. modes written by inla_constrained_mode into rows of one array) and its
 * gradient with respect to every parameter (flat layout, written to grad if not
 * NULL); *loss (host) receives the loss if loss is not NULL. */
int inla_mlp_grad(inla_mlp *m, int32_t B, const float *x, const double *target, float *grad, double *loss);
/* One Adam step (beta1 0.9, beta2 0.999, eps 1e-8, learning rate lr) on the
 * mean-squared-error loss of a batch; *loss (host) receives the loss before the
 * step.  With loss NULL the call only enqueues the step on the handle's stream
 * and returns without waiting for the device. */
int inla_mlp_train_step(inla_mlp *m, int32_t B, const float *x, const double *target, float lr, double *loss);
/* Warm starts for inla_laplace_eval: theta (host, B x ldtheta, ldtheta <= 8)
 * normalised with centre[I], scale[I] (host), predicted modes written as FP64
 * into x[b] (host array of B device pointers to O doubles). */
int inla_mlp_predict_modes(inla_mlp *m, int32_t B, const double *theta, int32_t ldtheta, const double *centre,
                           const double *scale, double *const *x);

/* ------------------------------------------- variational-Bayes mean correction */
/* Correction of the posterior mean by variational Bayes (appendix "Variational
 * Bayes approximation strategy", algorithm "Correction of Posterior Mean using
 * Variational Bayes"): x | y, theta ~ N(mu + lambda, Q*^{-1}) with Q* and the
 * marginal variances s_i^2 of the Laplace approximation fixed; each iteration
 * solves (Q_prior + diag I'') lambda = -(I' + Q_prior mu) (the minimiser of the
 * second-order expansion of E[-log pi(y | eta)] + KLD, with the paper's sign of
 * c taken so that lambda minimises), kriged so that C mu stays e, and sets
 * mu <- mu + lambda, until ||lambda||_inf <= tol max(1, ||mu||_inf).  I' and I''
 * are the expectations of -d log pi / d eta and -d^2 log pi / d eta^2 over
 * eta_i ~ N(eta_i(mu), s_i^2) by n_gh-point Gauss-Hermite quadrature (<= 0: 20,
 * at most 64; rule by Golub-Welsch on the host).  A Gaussian likelihood's
 * correction is zero.  var[b]: device [n] marginal variances at the Laplace
 * mode (e.g. from inla_marginal_var); x[b]: device [n], the Laplace mode on
 * input, the corrected mean on output (left unchanged where info != 0).  opts:
 * max_iter (<= 0: 50) and tol (<= 0: 1e-11) are used; prec must be FP64.
 * iters, info: host [B] (INLA_INFO_* codes).  Returns -i for an invalid i-th
 * argument, INLA_ERR_UNSUPPORTED for another precision. */
int inla_vb_mean(inla_handle *h, int32_t B, const inla_model *models, const double *theta, int32_t ldtheta,
                 const double *const *var, double *const *x, int32_t n_gh, const inla_opts *opts, int32_t *iters,
                 int32_t *info);

/* --------------------------------------------- hyperparameter mode and CCD */
/* Stage 1 of the method (section "Stage 1", appendix "Marginal posteriors of the
 * hyperparameters"): theta* = argmin -log pi~(theta | y) with
 * log pi~(theta | y) = log pi~(y | theta) (inla_laplace_eval's objective, Eq. (41))
 * + log pi(theta), by BFGS (Nocedal and Wright's inverse-Hessian update, scaled
 * by s^T y / y^T y at the first update, steepest descent restart on a
 * non-descent direction), with central-difference gradients.  Every gradient
 * (2t points) and every round of the backtracking line search (Armijo,
 * c1 = 1e-4, step lengths 1, 1/2, ..., 1/2^11 in rounds of four) is one batched
 * inla_laplace_eval call, warm-started from the mode at the current point.  The
 * step is first scaled so that its largest component is at most max_step. */
typedef double (*inla_log_prior_fn)(const double *theta, int32_t t, void *user);  /* log pi(theta), host */
typedef struct inla_theta_opts {
  int32_t max_iter;   /* BFGS iterations, <= 0: 100                                        */
  int32_t reserved;
  double h;           /* central-difference step in theta, <= 0: 1e-3                      */
  double gtol;        /* stop when ||gradient||_inf <= gtol, <= 0: 1e-3                    */
  double ftol;        /* stop when the decrease of -log pi~ <= ftol max(1, |value|), <= 0: 1e-12 */
  double max_step;    /* largest component of a step before the line search, <= 0: 1      */
  inla_opts eval;     /* options of every Laplace evaluation (start is managed here)       */
} inla_theta_opts;
#define INLA_THETA_OK 0            /* converged (gradient or decrease test)                  */
#define INLA_THETA_MAXIT 1         /* max_iter reached                                       */
#define INLA_THETA_LINESEARCH 2    /* no step length of the line search decreased enough    */
#define INLA_THETA_EVAL_FAILED 3   /* an evaluation at the iterate failed (info != 0)        */
#define INLA_THETA_NOT_PD (-2000)  /* inla_ccd_points: the negative Hessian is not positive definite */
#define INLA_CCD_MAX_T 12
/* model: one model (its device arrays), t = number of theta components of its
 * prior kind plus one; theta0 (host [t]); log_prior may be NULL (flat).  Host
 * outputs: theta_star [t], f_star = log pi~(theta* | y) (may be NULL), grad =
 * gradient of log pi~ at theta* (may be NULL), iterations, evaluations, info
 * (INLA_THETA_*).  Returns -i for an invalid i-th argument (-3: t does not
 * match the prior kind), else the status of the Laplace evaluations. */
int inla_theta_mode(inla_handle *h, const inla_model *model, int32_t t, const double *theta0,
                    const inla_theta_opts *opts, inla_log_prior_fn log_prior, void *user, double *theta_star,
                    double *f_star, double *grad, int32_t *iters, int32_t *evals, int32_t *info);
/* Negative Hessian of log pi~(theta | y) at theta (host [t]) by central
 * differences with step `step` (<= 0: 5e-3): diagonal (f(+h) - 2 f(0) + f(-h)) / h^2,
 * off-diagonal four-point stencil, 1 + 2 t^2 evaluations, the last 2 t^2 in
 * one batch (the paper's bound is 2 (t^2 + t)).  Writes neg_hess (host t x t,
 * row-major) and log_post = log pi~(theta | y) (may be NULL); info (may be
 * NULL) is INLA_THETA_EVAL_FAILED if an evaluation failed. */
int inla_theta_hessian(inla_handle *h, const inla_model *model, int32_t t, const double *theta, double step,
                       const inla_opts *opts, inla_log_prior_fn log_prior, void *user, double *neg_hess,
                       double *log_post, int32_t *info);
/* Central composite design (section "Hyperparameter exploration": 45 points
 * at t = 6) in the standardised z scale: the centre, the 2t axial points
 * +-f0 sqrt(t) e_i, and the factorial points f0 (+-1, ..., +-1): all 2^t for
 * t <= 4, for t >= 5 the half fraction whose last coordinate is the product of
 * the others (1 + 2t + 2^(t-1) points: 27 at t = 5, 45 at t = 6); none at
 * t = 1.  Every point but the centre lies on the sphere |z| = f0 sqrt(t), f0 > 1.
 * delta: design weights relative to the density's value at each point, chosen
 * so that the rule is exact for the mass, mean and covariance of a standard
 * Gaussian: 1 - 1/f0^2 at the centre, exp(f0^2 t / 2) / (f0^2 (n - 1)) elsewhere.
 * With z and delta NULL only *n_points is written; otherwise *n_points is the
 * capacity on input (-3 and the needed count when too small), z is host
 * [n x t] row-major and delta host [n].  Host only, no handle. */
int inla_ccd_design(int32_t t, double f0, int32_t *n_points, double *z, double *delta);
/* The design mapped to theta: theta_k = theta* + V Lambda^{1/2} z_k with the
 * eigen-decomposition Sigma = neg_hess^{-1} = V Lambda V^T (the z-parameterisation
 * of the appendix on asymmetric Gaussian interpolation).  neg_hess host t x t
 * row-major (symmetrised); returns INLA_THETA_NOT_PD if it is not positive
 * definite.  *n_points: capacity in, count out; theta_k host [n x t], delta host [n]. */
int inla_ccd_points(int32_t t, const double *theta_star, const double *neg_hess, double f0, int32_t *n_points,
                    double *theta_k, double *delta);
/* Integration weights of the explored points: w_k proportional to
 * delta_k exp(log_post_k), normalised to sum 1 (host arrays of n_points; a
 * non-finite log_post_k gets weight 0). */
int inla_ccd_weights(int32_t n_points, const double *delta, const double *log_post, double *weights);

/* ------------------------------------- Moore-Penrose route (intrinsic priors) */
/* Section "Bypassing constraints complexity in disease mapping models using
 * dense matrices": a rank-deficient (intrinsic) prior precision is handled
 * through its Moore-Penrose inverse, whose null space identifies the field in
 * place of explicit constraints, and the posterior covariance follows the
 * Woodbury form of Eq. (woodeqn).
 *
 * inla_pinv: Q^+ of B symmetric matrices by a block Jacobi eigen-decomposition
 * Q = V diag(lambda) V^T: blocks of 32 indices, block pairs in round-robin
 * order, each pair's 64 x 64 principal submatrix reduced by one sweep of cyclic
 * Jacobi and the rotations applied to A and V as 64-wide tile products; sweeps
 * until the off-diagonal Frobenius norm is at most 4 eps ||A||_F, or below
 * 1e-14 ||A||_F and shrinking by less than 10% per sweep (at most 120 sweeps).
 * Q^+ = V diag(f) V^T with f_k = 1 / lambda_k where |lambda_k| > rtol *
 * max|lambda| and 0 otherwise.
 *   n        host [B] orders, 1 <= n[b] <= 16384
 *   Q        host array of B device pointers: column-major, lower triangle read
 *   ldq      host [B] leading dimensions (>= n[b])
 *   Qpinv    host array of B device pointers: output, full symmetric n x n
 *            (both triangles written), column-major, leading dimension ldp[b]
 *   rtol     relative rank threshold; <= 0: 1e-9
 *   rank     host [B] output: number of eigenvalues kept
 *   sweeps   host [B] output: outer sweeps taken.  An outer sweep is one
 *            round-robin sweep of the largest active matrix of the batch
 *            (nbk - 1 rounds, nbk = its order in 32-index blocks); a smaller
 *            matrix takes its own rounds in order meanwhile, so it completes
 *            more than one of its own sweeps per outer sweep and is checked
 *            for convergence at the outer sweep boundaries
 *   info     host [B] output: 0, INLA_INFO_EIG_MAXIT or INLA_INFO_NONFINITE
 * Uses the handle's workspace (2 ne^2 + O(ne) doubles per matrix, ne = n
 * rounded up to 64) and synchronises the handle's stream once per sweep.
 * Returns -i for an invalid i-th argument (a bad n[b] as -3), INLA_ERR_NOMEM
 * or INLA_ERR_HIP. */
int inla_pinv(inla_handle *h, int32_t B, const int32_t *n, const double *const *Q, const int32_t *ldq,
              double *const *Qpinv, const int32_t *ldp, double rtol, int32_t *rank, int32_t *sweeps, int32_t *info);

/* inla_woodbury_eval: log pi~(y | theta) with an intrinsic prior.  Each model
 * has prior INLA_PRIOR_PINV and k = 0; model.Qprior is the device
 * pseudo-inverse Q_prior(theta_b)^+ (full symmetric, ld model.ldq; the caller
 * scales it with theta), and theta row b holds the likelihood parameter only:
 * (lik), lik = log sigma^2 (Gaussian) or beta0 (Poisson).  Newton in covariance
 * form: b = g + W x, x_new = Sigma* b with Sigma* = Q^+ - Q^+ S M^{-1} S Q^+,
 * S = diag(sqrt(W)), M = I + S Q^+ S factored by the blocked Cholesky (FP64).
 * A general design matrix (model.m > 0, CSR as for inla_laplace_eval, checked
 * on the host) runs the same iteration on eta = A x with Q^+ replaced by
 * K = A Q^+ A^T (M is m x m) and maps back with x = Q^+ A^T z; the library
 * forms Q^+ A^T and K once per call (n m + m^2 doubles per theta).  The
 * stopping rule is that of inla_laplace_eval (Gaussian: one step), plus: a
 * step below 1e-7 of max(1, |x|_inf) that is larger than half the previous one
 * ends the iteration (the covariance form's rounding floor, which the condition
 * of M sets, can lie above tol).  The objective is the Laplace approximation on
 * range(Q_prior):
 *   objective = loglik - 1/2 x*^T Q_prior x* - 1/2 log|M|,
 * which equals 1/2 log pdet(Q_prior) + 1/2 log pdet(Sigma*) - 1/2 x*^T Q_prior x*
 * + loglik (pdet: product of the non-zero eigenvalues), and the kriging
 * objective with constraints spanning null(Q_prior).  M comes from the last
 * Newton step.  For A = I, x*^T Q_prior x* = z^T x*; for a general A, z^T A x*.
 *   x     host array of B device pointers [n]: start (opts->start = 1) and the mode
 *   opts  as for inla_laplace_eval; prec must be INLA_PREC_FP64
 *   res   host [B]: objective, xqx = x*^T Q_prior x*, loglik, logdet_qstar =
 *         log|M| (= log pdet(Q*) - log pdet(Q_prior) on range(Q_prior)), step,
 *         iters, info; the prior and constraint log-det fields are 0.
 * Returns -i for an invalid i-th argument (a model that is not of this form, or
 * a malformed CSR, as -3), INLA_ERR_UNSUPPORTED for another precision,
 * INLA_ERR_NOMEM, INLA_ERR_HIP. */
int inla_woodbury_eval(inla_handle *h, int32_t B, const inla_model *models, const double *theta, int32_t ldtheta,
                       double *const *x, const inla_opts *opts, inla_result *res);

/* inla_woodbury_var: marginal variances diag(Sigma*) of the Woodbury covariance
 * (Eq. (woodeqn)) at given modes, models and theta as for inla_woodbury_eval:
 * var_i = Q^+_ii - ||L^{-1} S A Q^+ e_i||^2 with S = diag(sqrt(W(A x_mode))) and
 * M = I + S A Q^+ A^T S = L L^T (A = I for m = 0), factored in FP64 with the n
 * border rows Q^+ A^T S (about n_o^3 / 3 + n n_o^2 flops, n_o = m or n, and
 * (n_o + n) n_o doubles of factor workspace per theta).
 *   x_mode  host array of B device pointers [n] (read)
 *   var     host array of B device pointers [n] (written)
 *   info    host [B]: 0 or the leading minor of M that is not positive definite
 * Returns -i for an invalid i-th argument (a model not of the form above as -3,
 * a non-finite likelihood parameter as -4), INLA_ERR_NOMEM or INLA_ERR_HIP. */
int inla_woodbury_var(inla_handle *h, int32_t B, const inla_model *models, const double *theta, int32_t ldtheta,
                      const double *const *x_mode, double *const *var, int32_t *info);

/* A prior given through the Moore-Penrose inverses of its diagonal blocks, for
 * Stage 1 on the Moore-Penrose route (section "Bypassing constraints
 * complexity ..."): Q_prior(theta) = blockdiag_k(tau_k R_k), so
 * Q_prior(theta)^+ = blockdiag_k(R_k^+ / tau_k) with tau_k = exp(theta[tau_index[k]]),
 * or a fixed 1 / tau_k = fixed_scale[k] where tau_index[k] < 0.  The blocks
 * tile [0, n) without gaps or overlaps (any order).  The likelihood parameter
 * is theta[lik_index], or lik_value where lik_index < 0.  All arrays are host
 * arrays; P[k] are device pointers to R_k^+ (column-major, ld[k] >= size[k]),
 * read only. */
typedef struct inla_pinv_prior {
  int32_t n_blocks;
  const int32_t *offset;
  const int32_t *size;
  const double *const *P;
  const int32_t *ld;
  const int32_t *tau_index;
  const double *fixed_scale;
  int32_t lik_index;
  int32_t reserved;
  double lik_value;
} inla_pinv_prior;

/* Q_prior(theta_b)^+ for B points (theta row-major, stride ldtheta), written
 * full n x n (column-major, ld n) to the device arrays out[b].  Returns -3 for
 * an invalid prior description (blocks not tiling [0, n), a null pointer, an
 * index outside theta), -i for another invalid i-th argument. */
int inla_pinv_prior_assemble(inla_handle *h, const inla_pinv_prior *prior, int32_t n, int32_t B, const double *theta,
                             int32_t ldtheta, double *const *out);
/* inla_theta_mode / inla_theta_hessian with every evaluation on the
 * Moore-Penrose route: each batch of points gets Q_prior(theta)^+ from `prior`
 * (device workspace of n^2 doubles per point) and is evaluated by
 * inla_woodbury_eval.  model: prior INLA_PRIOR_PINV, k = 0 (its Qprior and ldq
 * are ignored); t is the dimension of theta (every tau_index and lik_index
 * below t).  Other arguments and results as for inla_theta_mode and
 * inla_theta_hessian. */
int inla_theta_mode_pinv(inla_handle *h, const inla_model *model, const inla_pinv_prior *prior, int32_t t,
                         const double *theta0, const inla_theta_opts *opts, inla_log_prior_fn log_prior, void *user,
                         double *theta_star, double *f_star, double *grad, int32_t *iters, int32_t *evals,
                         int32_t *info);
int inla_theta_hessian_pinv(inla_handle *h, const inla_model *model, const inla_pinv_prior *prior, int32_t t,
                            const double *theta, double step, const inla_opts *opts, inla_log_prior_fn log_prior,
                            void *user, double *neg_hess, double *log_post, int32_t *info);

/* ------------------------------------------------------------ profiling */
/* Kernel classes timed when profiling is on. */
enum {
  INLA_K_TRAIL = 0,     /* MFMA trailing update of the blocked Cholesky (128 x 128 tiles) */
  INLA_K_PANEL = 1,     /* MFMA panel TRSM and in-panel updates (64 x 64 tiles)           */
  INLA_K_POTF2 = 2,     /* diagonal-block factorisation and inversion                     */
  INLA_K_ASSEMBLE = 3,  /* prior build, Q* / border assembly, likelihood                  */
  INLA_K_SOLVE = 4,     /* triangular solves, kriging system, reductions                  */
  INLA_K_BORDER = 5,    /* trailing update of the border rows when it runs apart from the
                           factored rows (FP32 operands beside a BF16 trailing update) */
  INLA_K_COUNT = 6
};
typedef struct inla_kstats {
  int64_t launches;  /* kernel launches recorded                              */
  double time_ms;    /* sum of launch durations (HIP events on the handle's stream) */
  double flops;      /* algorithmic flops of those launches (padding excluded) */
  double bytes;      /* algorithmic HBM bytes of those launches                */
} inla_kstats;
/* Turn per-launch event timing on (1) or off (0); turning it on clears the
 * counters.  Timing adds an event pair per launch. */
int inla_profile(inla_handle *h, int32_t enable);
/* Read the counters of kernel class `kclass` for the launches enqueued by
 * passes run at precision `prec` (an INLA_PREC_* value), collected
 * up to the last completed call.  A mixed-precision evaluation files its FP64
 * prior pass under INLA_PREC_FP64 and its Newton and final passes (including
 * their FP64 residual kernels) under INLA_PREC_FP32, except the BF16-trailing
 * factorisations of a BF16 evaluation, filed under INLA_PREC_BF16.  Returns -2 for an unknown
 * class, -3 for an unknown precision, -4 for a null `out`. */
int inla_profile_get(inla_handle *h, int32_t kclass, int32_t prec, inla_kstats *out);

/* ------------------------------------------------- graphs and autotuning */
/* The batched factorisation and the triangular solves are long chains of
 * dependent launches: per 64-wide diagonal block of a panel, the diagonal-block
 * factorisation, the panel TRSM and the in-panel update; per 64-row block of a
 * solve, one step.  With graphs enabled (the default) each such chain is
 * captured once into a hipGraph, keyed by the sizes that fix its grids, and
 * replayed; the per-theta pointers and parameters travel in a device argument
 * block that is refreshed before a replay when it changed.  The trailing
 * update and the other single launches are enqueued directly.  Results are
 * identical with and without graphs.  The handle owns the graphs (at most 1024,
 * least recently used dropped first) and releases them in inla_destroy or
 * when graphs are turned off.  Returns -1 for a null handle. */
int inla_set_graphs(inla_handle *h, int32_t enable);
/* Lookahead in the blocked Cholesky (allowed by default, used where the tuned
 * configuration asks for it): after each panel, the
 * trailing update of the next panel's columns runs first on the handle's
 * stream, the rest of the trailing update on a second stream owned by the
 * handle (created on first use, default priority), and the next panel is
 * factored on the handle's stream meanwhile; events order the two streams and
 * every call still returns with its work complete on the handle's stream.
 * Results are identical with and without lookahead.  Returns -1 for a null
 * handle. */
int inla_set_lookahead(inla_handle *h, int32_t enable);
/* Concurrent prior pass (off by default).  The prior's factorisation in
 * inla_laplace_eval and inla_constrained_mode (log|Q_prior|, C Q_prior^{-1} C^T
 * and their log-determinant, FP64 in every precision) depends on theta alone,
 * and the Newton iteration never reads it: with overlap on it runs on a third
 * stream owned by the handle (created on first use, default priority) while
 * the handle's stream runs the Newton iteration, in a workspace of its own
 * (one more FP64 bordered matrix of order n + k + 1, padded to 128, per
 * theta).  Events order the two streams; every call still returns with its
 * work complete on the handle's stream.  Results are identical with and
 * without overlap.  Returns -1 for a null handle. */
int inla_set_overlap(inla_handle *h, int32_t enable);
/* Graphs captured and replayed so far by this handle (host outputs; either may be NULL). */
int inla_graph_stats(inla_handle *h, int64_t *captured, int64_t *replays);
/* Whole-pass graphs (on by default; used while graphs are on and profiling is
 * off).  Each pass of inla_laplace_eval / inla_constrained_mode over a set of
 * theta (the bordered assembly at the current iterate, the factorisation of
 * Q* with the constraint and right-hand-side border rows, the kriging system's
 * build, factorisation and solve, and the Newton step: back-substitution and
 * acceptance, or the correction-form restart, or the final log-dets) and each
 * mixed-precision refinement step (FP64 KKT residual, the two triangular
 * solves, the kriging correction and the update) is one hipGraph, keyed by the
 * pass, the precision, the tuning table's state and every theta's sizes, and
 * launched with one copy of its argument block; the host reads back only the
 * per-theta results that decide the next pass.  A key's first pass runs
 * directly, its second is captured, later ones replay (after re-deriving the
 * arguments and checking the launch sequence against the captured one).  BF16
 * passes and the factorisation's lookahead stay outside these graphs.
 * Results are identical with and without them.  The handle keeps at most 64
 * pass keys (4 MB of device arguments per captured pass) and releases them as
 * inla_set_graphs(h, 0) does.  Returns -1 for a null handle. */
int inla_set_pass_graphs(inla_handle *h, int32_t enable);
/* Pass graphs captured and replayed so far by this handle (host outputs; either may be NULL). */
int inla_pass_graph_stats(inla_handle *h, int64_t *captured, int64_t *replays);
/* Autotuner of the blocked Cholesky.  A configuration is int32_t[3] =
 * {nb, tm, lookahead}: panel width nb in {128, 256, 512, 1024}, trailing tile
 * tm in {64, 128} (128 only for INLA_PREC_BF16) and lookahead 0 or 1 (see
 * inla_set_lookahead).  inla_autotune times the factorisation of a synthetic
 * symmetric positive definite batch shaped like B matrices of orders n[b]
 * with kb[b] border rows (host arrays; kb = k + 1 for the Newton and final
 * passes of a model with k constraints): every (nb, tm) without lookahead in
 * the order (128,64), (128,128), (256,64), ..., (1024,128) (BF16: the four nb
 * with tm = 128), then the fastest of them with lookahead (unless lookahead is
 * turned off), one untimed and `reps` timed runs each.  It records the fastest
 * for (prec, padded largest order, batch size rounded up to a power of two) in
 * the handle's table, which every later factorisation of such a batch uses
 * (the default pair unless another is at least 3% faster; the lookahead
 * variant only when it is at least 5% faster).
 * Outputs (host, each may be NULL): the chosen configuration, the mean time in
 * ms of each candidate in the order above (at most INLA_TUNE_MAX_CAND values)
 * and the candidate count.  Uses the handle's workspace; no caller data is
 * touched.  Without a table entry a batch factorises with the default:
 * {512, 64, 0} for FP64, {512, 128, 0} for FP32, and for BF16 {512, 128, 0}
 * below a padded order of 4096, {1024, 128, 0} from it (the BF16 trailing
 * update then passes over its FP32 trailing block once per 1024 of K).
 * Returns -2 for B < 1, -3 / -4 for a null or non-positive n / null or
 * negative kb, INLA_ERR_UNSUPPORTED for an unknown precision, -6 for reps < 1. */
#define INLA_TUNE_MAX_CAND 9
int inla_autotune(inla_handle *h, int32_t B, const int32_t *n, const int32_t *kb, int32_t prec, int32_t reps,
                  int32_t *config, double *ms, int32_t *n_cand);
/* Set the configuration for (prec, largest order n_max, batch size B)
 * directly, or erase the entry with config = NULL.  Returns -5 for an invalid
 * configuration. */
int inla_tune_set(inla_handle *h, int32_t prec, int32_t n_max, int32_t B, const int32_t *config);
/* The configuration a factorisation of such a batch uses (host output int32_t[3]). */
int inla_tune_get(inla_handle *h, int32_t prec, int32_t n_max, int32_t B, int32_t *config);

/* Library version string. */
const char *inla_version(void);

#ifdef __cplusplus
}
#endif
#endif /* INLA_DENSE_H */
