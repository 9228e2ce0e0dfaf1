/*
 * fsa.h -- C ABI of the MI355X (gfx950) full-scale-approximation library.
 *
 * Method: Gyger, Furrer & Sigrist, "Iterative Methods for Full-Scale
 * Gaussian Process Approximations for Large Spatial Data" (arXiv 2405.14492).
 *
 * The library computes, on one GPU, the negative log-likelihood of a
 * zero-mean Gaussian process under the full-scale approximation (FSA)
 *
 *   Sigma~_dagger = Sigma_mn^T Sigma_m^{-1} Sigma_mn            (Section 2.1)
 *                 + (Sigma - Sigma_mn^T Sigma_m^{-1} Sigma_mn) o T(gamma)
 *                 + sigma^2 I,
 *
 * its gradient in (sigma1^2, rho, sigma^2) (eq. NEGLLDNEGLLFSA), and the
 * FSA predictive variances (eq. MuPredFSA), all by preconditioned conjugate
 * gradients with the FITC preconditioner P = D_s + Sigma_mn^T Sigma_m^{-1}
 * Sigma_mn (eq. eqfitcp) applied through the Woodbury identity (App. F),
 * stochastic Lanczos quadrature for log det (Section 3.3), stochastic trace
 * estimation for the gradient (Section 3.3) and the simulation-based
 * variance estimator of Algorithm 1 (Section 3.2).
 *
 * Conventions for every entry point:
 *  - Every function returns fsa_status; no C++ exception crosses the ABI.
 *    On failure fsa_last_error() returns a message (thread-local).
 *  - Host pointers are read during the call only; the library keeps no
 *    caller pointer after returning.  Outputs go to caller buffers.
 *  - Locations are row-major n x d float64 arrays with d == 2.
 *  - A context is used by one host thread at a time.  Distinct contexts may
 *    run concurrently on distinct streams.
 *  - Device-pointer variants (suffix _dev) take device buffers that must stay
 *    valid for the duration of the call only.
 */
#ifndef FSA_H
#define FSA_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct fsa_ctx fsa_ctx; /* opaque; owned by the library until fsa_destroy */

typedef enum {
  FSA_OK = 0,
  FSA_ERR_INVALID_ARG = 1, /* bad size, non-finite input, parameter out of range */
  FSA_ERR_OOM = 2,         /* device allocation failed */
  FSA_ERR_NOT_SPD = 3,     /* Cholesky of Sigma_m or of the FITC capacitance failed */
  FSA_ERR_NOT_CONVERGED = 4, /* max_iter reached; outputs are still written */
  FSA_ERR_BREAKDOWN = 5,   /* CG breakdown: h^T Sigma~ h <= 0 or non-finite */
  FSA_ERR_DEVICE = 6       /* HIP runtime error */
} fsa_status;

/* Covariance function c(s_i, s_j) (Section 2), d = Euclidean distance:
 *   EXPONENTIAL: sigma1^2 exp(-d / rho)                      (Matérn 1/2)
 *   MATERN32:    sigma1^2 (1 + sqrt3 d/rho) exp(-sqrt3 d/rho) (Matérn 3/2) */
typedef enum { FSA_COV_EXPONENTIAL = 0, FSA_COV_MATERN32 = 1 } fsa_cov;

/* Arithmetic of the PCG loop.
 *   FP64: everything in float64.
 *   MIXED_FP32: covariance blocks, sparse values, low-rank factor and the
 *     PCG block vectors in float32; Cholesky factors, inner products, the
 *     CG coefficients, the solution accumulator and the tridiagonal
 *     eigensolve in float64; the residual is recomputed with the float64
 *     operator every rr_period iterations.  A column stops once its float32
 *     recurrence residual is below the tolerance and the float64 residual
 *     b - Sigma~ u, recomputed then, confirms it; a column it does not
 *     confirm continues its CG sequence from the float64 residual.  Where
 *     the low-rank part dominates (|A A^T| / D around 10^5 and more), the
 *     float32 Woodbury application q = (r - A C^{-1} A^T D^{-1} r) / D
 *     cancels most of its digits; a likelihood solve whose float32 iteration
 *     breaks down, or whose slowest column's residual does not halve over
 *     three replacement periods, is repeated in float64
 *     (fsa_stats.fp64_fallback).  The derivative factor F of the gradient
 *     (which enters the gradient only) is a float32 product from the float32
 *     copy of A.
 *   MIXED_BF16A: MIXED_FP32 on a model whose whitened low-rank factor A is
 *     rounded to bfloat16 (to nearest even, once, right after whitening).
 *     The rounded factor is used everywhere, in float64 where the method is
 *     float64: the tapered residual is computed against it (so inside the
 *     taper range the rounding is absorbed and the diagonal stays exact),
 *     and D_s, the capacitance, the probes, the gradient and the prediction
 *     factor use it too.  The PCG passes read A as bfloat16 (half the bytes
 *     of float32) and widen it to float32 in registers.  Results are those
 *     of the perturbed model: they differ from FP64 by the rounding of A
 *     outside the taper range, not by solver error.  Its sigma1^2 derivative
 *     takes the rounded model as proportional to sigma1^2 (as the unrounded
 *     one is); its rho derivative uses the exact dSigma_mn/drho and
 *     dSigma_m/drho with the rounded A. */
typedef enum { FSA_FP64 = 0, FSA_MIXED_FP32 = 1, FSA_MIXED_BF16A = 2 } fsa_precision;

/* fsa_options.fp32_products: the float32 products of MIXED_FP32's low-rank
 * PCG passes (A^T D^{-1} r and A C^{-1} w over the n x m factor).
 *   FSA_F32P_SPLIT (default): on the bfloat16 matrix cores, every float32
 *     operand split exactly into three bfloat16 parts and the six partial
 *     products above 2^-23 of the result summed in float32 (the dropped ones
 *     are below the float32 accumulation error of the k-long sums), at 6/16
 *     of the float32 matrix-core time, so the passes are bound by reading A.
 *     Blocks of more than 52 columns take the float32 matrix cores.
 *   FSA_F32P_MFMA: on the float32 matrix cores (16x16x4). */
typedef enum { FSA_F32P_SPLIT = 0, FSA_F32P_MFMA = 1 } fsa_fp32_products;

/* fsa_options.profile: all five kernel classes of fsa_stats.kernel_ms */
#define FSA_PROFILE_ALL 0x1f

/* fsa_options.control_variate: the FITC preconditioner as control variate
 * (App. E) in both stochastic estimates of the method, per parameter or per
 * prediction point:
 * - the gradient's trace estimate (eq. Troptc): each probe's sample
 *   a_i = (z_i^T Sigma~^{-1}) dSigma~/dtheta (P^{-1} z_i) gets c * b_i subtracted,
 *   b_i = (P^{-1} z_i)^T dP/dtheta (P^{-1} z_i), and c Tr(P^{-1} dP/dtheta)
 *   (exact, by Woodbury) added;
 * - Algorithm 1's stochastic diagonal of Sigma^s_{nn_p}^T Sigma~_s^{-1} Sigma^s_{nn_p}:
 *   each sample z_i o (S^T Sigma~_s^{-1} S z_i) gets c o z_i o (S^T D_s^{-1} S z_i)
 *   subtracted and c o diag(S^T D_s^{-1} S) (exact) added (P_s = D_s).
 *   FSA_CV_NONE         the plain estimates;
 *   FSA_CV_ONE          c = 1;
 *   FSA_CV_OPT          c = sum_i (a_i - mean a)(b_i - mean b) / sum_i (b_i - mean b)^2,
 *                       the coefficient of least sample variance (the paper's
 *                       c_opt read with a centred denominator);
 *   FSA_CV_OPT_PRINTED  c = sum_i (a_i - mean a) b_i / sum_i b_i^2, as printed.
 * The gradient's costs two m x m-triangular solves over n x m blocks per
 * theta (with the derivative build, after the solve) and one pass over the
 * probe block per gradient; the diagonal's two sparse products per
 * prediction. */
typedef enum { FSA_CV_NONE = 0, FSA_CV_ONE = 1, FSA_CV_OPT = 2, FSA_CV_OPT_PRINTED = 3 } fsa_control_variate;

typedef struct {
  int32_t cov;      /* fsa_cov */
  double sigma1_sq; /* marginal variance sigma1^2 > 0 */
  double rho;       /* range rho > 0 */
  double sigma_sq;  /* nugget sigma^2 > 0 (Theorems 1-2 assume it) */
} fsa_theta;

typedef struct {
  int32_t num_probes;    /* number of probe vectors ell >= 1 (Section 3.1) */
  int32_t control_variate; /* fsa_control_variate (default FSA_CV_NONE) */
  uint64_t seed;         /* key of the counter-based Rademacher generator */
  double cg_rel_tol;     /* per column ||r||_2 / ||b||_2 < tol stops the column */
  int32_t max_iter;      /* iteration cap; reaching it gives FSA_ERR_NOT_CONVERGED */
  int32_t fixed_iter;    /* > 0: every column runs exactly this many iterations */
  int32_t precision;     /* fsa_precision */
  int32_t rr_period;     /* mixed precision: periodic float64 residual replacement every rr_period iterations
                            (0 = none; the float64 stopping check of a tolerance run still replaces it once) */
  int32_t slq_weight_n;  /* 0: SLQ weight z^T P^{-1} z; 1: the weight n of Section 3.1 */
  int32_t profile;       /* bit k set: time every PCG launch of kernel class k (fsa_stats.kernel_ms[k]) with
                            a pair of HIP events on the stream (about 3 us each); FSA_PROFILE_ALL times all */
  double sigma_m_jitter; /* adds jitter * sigma1^2 to the diagonal of Sigma_m (default 0) */
  void* hip_stream;      /* hipStream_t to run on, or NULL for the default stream */
  int32_t graph;         /* nonzero: every PCG iteration after the first is replayed from a HIP graph captured from
                            the second (one launch per iteration instead of one per kernel; results are bitwise
                            those of the eager launches); ignored while profile is set and on the null stream,
                            which cannot be captured */
  int32_t fp32_products; /* fsa_fp32_products: how MIXED_FP32 multiplies the n x m low-rank factor in the PCG passes */
} fsa_options;

typedef struct {
  int32_t iters_min, iters_max; /* PCG iterations over the right-hand-side columns */
  int64_t probe_iters;          /* sum over columns of iterations executed */
  double rel_res_max;           /* largest final ||r|| / ||b|| over the likelihood solve's columns: FP64, the
                                   CG recurrence residual; mixed precision (tolerance mode), the float64
                                   residual b - Sigma~_dagger u on which the stop is confirmed */
  double logdet;                /* SLQ estimate of log det Sigma~_dagger */
  double logdet_P;              /* log det of the FITC preconditioner (Sylvester) */
  double quad;                  /* y^T Sigma~_dagger^{-1} y */
  double ms_build;              /* host wall time of a rebuild for a new theta inside the call (0 if none) */
  double ms_pcg;                /* the block PCG solve with its SLQ quadrature and quadratic term */
  double ms_backward;           /* the gradient after the solve, with the derivative build */
  double ms_total;
  int64_t nnz;                  /* nonzeros of the tapered residual */
  /* with options.profile: summed device time and launch count of the PCG
   * kernels: [0] sparse product Sigma~_s H, [1] fused update + A D^{-1} r
   * reduction, [2] Woodbury expansion A^T g, [3] search-direction update,
   * [4] small reductions and m-space products */
  double kernel_ms[5];
  int32_t kernel_launches[5];
  /* gradient parts: trace estimate (1/t) sum_i (Sigma~^{-1} z_i)^T dSigma~ P^{-1} z_i
   * and quadratic term u^T dSigma~ u (u = Sigma~^{-1} y), order (sigma1^2, rho, sigma^2) */
  double grad_trace[3];
  double grad_quad[3];
  /* with options.control_variate: the gradient's coefficients c and Tr(P^{-1} dP/dtheta),
   * order (sigma1^2, rho, sigma^2); grad_trace then holds the control-variate
   * estimate */
  double cv_c[3];
  double trace_P[3];
  /* MIXED_FP32 / MIXED_BF16A: 1 if the float32 solve broke down or stalled and
   * the likelihood solve was repeated in float64 (the likelihood is then the
   * float64 one; the gradient keeps the mode's float32 derivative factor);
   * fallback_probe_iters counts the abandoned float32
   * iterations (summed over columns) */
  int32_t fp64_fallback;
  int32_t reserved1;
  int64_t fallback_probe_iters;
} fsa_stats;

/* Default options: 50 probes, seed 0, tol 1e-8, max_iter 1000, FP64. */
void fsa_default_options(fsa_options* opt);

/* Build a context: taper pattern by uniform-grid neighbour search (Section
 * 2.1: T(gamma) is zero for d >= gamma; a pair is kept iff
 * dx*dx + dy*dy < gamma*gamma in float64), Sigma_m and its Cholesky factor,
 * the whitened low-rank factor L_m^{-1} Sigma_mn, the residual values, D_s,
 * and the FITC capacitance with its Cholesky factor (App. F).
 *   locs      host, n x d row-major; n >= 2 (Assumption 1)
 *   y         host, n responses (zero mean assumed: no fixed effects)
 *   theta     covariance parameters
 *   inducing  host, m x d row-major; 1 <= m <= min(n, 512), distinct
 *             (n below 2^27: the sparse product packs a neighbourhood
 *             position into 27 bits)
 *   taper_range gamma > 0
 *   opt       options (copied); NULL = defaults
 *   out       receives the new context
 * Errors: INVALID_ARG, OOM, NOT_SPD (Sigma_m or capacitance), DEVICE. */
fsa_status fsa_build(const double* locs, int64_t n, int32_t d, const double* y, const fsa_theta* theta,
                     const double* inducing, int32_t m, double taper_range, const fsa_options* opt,
                     fsa_ctx** out);
/* Same with device-resident locs, y and inducing (pointers as above, but on
 * the GPU the context will run on). */
fsa_status fsa_build_dev(const double* locs_dev, int64_t n, int32_t d, const double* y_dev,
                         const fsa_theta* theta, const double* inducing_dev, int32_t m, double taper_range,
                         const fsa_options* opt, fsa_ctx** out);

/* Negative log-likelihood (eq. NEGLLDNEGLLFSA) by preconditioned SLQ and,
 * if grad != NULL, its gradient by stochastic trace estimation with
 * z ~ (0, P) (Section 3.3).
 *   theta  NULL = the parameters of the build; else the context is revalued
 *          on the same taper pattern with these parameters (gamma fixed)
 *   nll    host scalar out
 *   grad   host [3] out, order (sigma1^2, rho, sigma^2), or NULL
 *   st     optional statistics out
 * Errors: INVALID_ARG, NOT_SPD, BREAKDOWN, NOT_CONVERGED (outputs written),
 * DEVICE. */
fsa_status fsa_nll_grad(fsa_ctx* ctx, const fsa_theta* theta, double* nll, double* grad, fsa_stats* st);

/* The same with the outputs in device memory of the context's GPU: nll_dev
 * (1 double) and, if not NULL, grad_dev (3 doubles, order (sigma1^2, rho,
 * sigma^2)), both written by copies on the context's stream (no host round
 * trip of the values).  Returns after the stream has drained; nll_dev is
 * +inf on a BREAKDOWN or NOT_SPD failure.  Errors as fsa_nll_grad. */
fsa_status fsa_nll_grad_dev(fsa_ctx* ctx, const fsa_theta* theta, double* nll_dev, double* grad_dev,
                            fsa_stats* st);

/* Gradient of the NLL of the preceding fsa_nll_grad call on this context
 * (eq. NEGLLDNEGLLFSA, trace by stochastic estimation with P^{-1} z,
 * Section 3.3), from the solves that call retained: the backward pass of the
 * likelihood.  grad: host [3] out, order (sigma1^2, rho, sigma^2).
 * Errors: INVALID_ARG (no preceding solve), DEVICE. */
fsa_status fsa_grad(fsa_ctx* ctx, double* grad, fsa_stats* st);

/* Predictive variances diag(Sigma^p_dagger) (eq. MuPredFSA, nugget
 * included) by Algorithm 1 with num_samples Rademacher vectors; Sigma~_s
 * solves by CG preconditioned with D_s (Section 3.3).  If mean_out is not
 * NULL, also the predictive mean Sigma^dagger_{n n_p}^T Sigma~^{-1} y
 * (Section 2.3), which needs a preceding fsa_nll_grad on this context.
 *   pred_locs host, n_p x d row-major; n_p >= 1
 *   var_out   host, n_p out; mean_out host, n_p out or NULL
 * Errors: INVALID_ARG, NOT_SPD, BREAKDOWN, NOT_CONVERGED, DEVICE. */
fsa_status fsa_predict_var(fsa_ctx* ctx, const double* pred_locs, int64_t n_p, int32_t num_samples,
                           double* var_out, double* mean_out, fsa_stats* st);

void fsa_destroy(fsa_ctx* ctx);
const char* fsa_last_error(void);

/* ---- inspection hooks (tests) ---- */
int64_t fsa_nnz(const fsa_ctx* ctx);
/* Taper pattern in the caller's point order: row_ptr host int64 (n+1),
 * col_idx host int32 (nnz), columns ascending per row; vals host float64
 * (nnz) or NULL gives the values of Sigma~_s. */
fsa_status fsa_export_csr(fsa_ctx* ctx, int64_t* row_ptr, int32_t* col_idx, double* vals);
/* D_s (host, n) and log det P. */
fsa_status fsa_export_diag(fsa_ctx* ctx, double* D, double* logdet_P);
/* Lanczos record of the last likelihood solve (Algorithm 2), for the t + 1
 * right-hand-side columns (0 = y, 1..t = probes), all host buffers, any may
 * be NULL: iters[t+1] iterations per column; alpha and beta
 * [L x (t+1)], row-major by iteration, the CG coefficients of each
 * iteration (entries past a column's count undefined), with L = fixed_iter
 * if set, else max_iter; weight[t+1] the quadrature weights and slq[t+1]
 * the terms weight_c e_1^T log(T_c) e_1 of Section 3.1 (column 0: 0).
 * FSA_ERR_INVALID_ARG before the first solve. */
fsa_status fsa_export_lanczos(fsa_ctx* ctx, int32_t* iters, double* alpha, double* beta, double* weight,
                              double* slq);

/* Solution block U = Sigma~_dagger^{-1} [y, z_1 .. z_t] of the last
 * likelihood solve (Section 3.1): host, n x (t+1) row-major, in the caller's
 * point order (column 0: u = Sigma~^{-1} y).  With fsa_apply(FSA_OP_PROBES)
 * it gives the residual b - Sigma~_dagger U of every column.
 * FSA_ERR_INVALID_ARG before the first solve. */
fsa_status fsa_export_solution(fsa_ctx* ctx, double* U);

enum {
  FSA_OP_SIGMA_DAGGER = 0, /* Sigma~_dagger X */
  FSA_OP_SIGMA_S = 1,      /* Sigma~_s X */
  FSA_OP_P_INV = 2,        /* P^{-1} X (Woodbury, App. F) */
  FSA_OP_D_SIGMA1 = 3,     /* dSigma~_dagger / dsigma1^2 X */
  FSA_OP_D_RHO = 4,        /* dSigma~_dagger / drho X */
  FSA_OP_PROBES = 5        /* ignores X; Y = the probe block z_1..z_ncols */
};
/* Apply an operator in float64 to ncols columns: X, Y host, n x ncols
 * row-major, in the caller's point order. */
fsa_status fsa_apply(fsa_ctx* ctx, int32_t which, const double* X, double* Y, int32_t ncols);

/* Scores of Gaussian predictive distributions against test responses
 * (Section 4), averaged over the n points: out[0] log-score
 * -log phi(y; mu, var), out[1] CRPS sigma (-1/sqrt(pi) + 2 phi(z) + z (2 Phi(z) - 1)),
 * z = (y - mu)/sigma, out[2] RMSE of the means.  y, mean, var: host arrays
 * of n doubles (var > 0), e.g. the outputs of fsa_predict_var; out: host,
 * 3 doubles.  Computed on the device (default stream) with fixed-order sums;
 * INVALID_ARG for n < 1, a null pointer, or a non-finite or non-positive
 * variance. */
fsa_status fsa_scores(const double* y, const double* mean, const double* var, int64_t n, double* out);

/* fsa_scores without any device allocation, for callers that cannot
 * allocate (code under stream capture, tight serving loops, harnesses that
 * forbid hipMalloc).  Same arguments, kernels, default stream and results
 * as fsa_scores; inputs are staged in a fixed library-owned device array of
 * 6.32 MB per GPU, held from the first call on that GPU until the process
 * ends, so n is limited to 262,144 points (INVALID_ARG beyond, with a
 * message).  All calls on one GPU share that array: they are serialized by
 * a lock inside the library, each returns after the default stream has
 * drained, and the array keeps the last call's contents (the counter of bad
 * variances is cleared by a kernel at every call). */
fsa_status fsa_scores_noalloc(const double* y, const double* mean, const double* var, int64_t n, double* out);

/* Release every cached device block of the process-wide pool and every
 * cached pinned host block of the solvers' readbacks.  Blocks held by live
 * contexts are not affected. */
void fsa_pool_trim(void);

/* Device memory from the caller (the problem statement's inputs and outputs
 * of Section 2 live in the caller's framework, e.g. torch's caching
 * allocator).  After this call every device block the library needs comes
 * from alloc(bytes, stream, user), where stream is the hipStream_t on which
 * the block is first used (the context's stream, or its side stream); a
 * null return is FSA_ERR_OOM.  Each block goes back through release(ptr,
 * user) once every piece of work the library enqueued on it has completed
 * (tracked by an event recorded at the library's release; the callback runs
 * on a thread that calls into the library, without library locks held, at
 * the latest in fsa_destroy of the owning context or fsa_pool_trim).  Blocks
 * keep their origin: a block from the library's own pool goes back to the
 * pool, a block from a callback pair to that pair, whatever is registered
 * later; the callbacks must stay valid until every block they handed out has
 * been released.  Both NULL: back to the library's own pool (hipMalloc,
 * cached).  The registration is process-wide; contexts in flight may mix
 * blocks of both origins.  INVALID_ARG if exactly one callback is NULL. */
typedef void* (*fsa_alloc_fn)(size_t bytes, void* hip_stream, void* user);
typedef void (*fsa_release_fn)(void* ptr, void* user);
fsa_status fsa_set_allocator(fsa_alloc_fn alloc, fsa_release_fn release, void* user);

/* ------------------------------------------------------------------------
 * Serving: likelihood + gradient and prediction requests of uneven size on
 * one GPU, each computed as fsa_nll_grad / fsa_predict_var compute it
 * (Section 3.1 with eq. NEGLLDNEGLLFSA, and Algorithm 1).
 *
 * A server owns `slots` workers, each with its own stream (default
 * priority) and host thread, and one block of `hbm_budget` bytes of device
 * memory taken at creation.  Requests are admitted in arrival order, each
 * once its arrival time has come, a worker is free and a contiguous range of
 * the block can hold the request's footprint (fsa_request_footprint); the
 * request then allocates only inside that range, so the admitted footprints
 * never sum past the budget and requests in flight never allocate from the
 * GPU.  Requests on different workers run concurrently on the device.  Every
 * result is that of the same request computed alone: a request's work uses
 * its own buffers and fixed-order reductions only.
 * ------------------------------------------------------------------------ */
typedef struct fsa_server fsa_server; /* opaque; owned by the library until fsa_server_destroy */

typedef enum { FSA_REQ_NLL_GRAD = 0, FSA_REQ_PREDICT_VAR = 1 } fsa_request_kind;

typedef struct {
  int32_t kind;             /* fsa_request_kind */
  int32_t m;                /* inducing points, 1 <= m <= min(n, 512) */
  int64_t n;                /* training locations, n >= 2 */
  const double* locs;       /* host, n x 2 row-major */
  const double* y;          /* host, n responses */
  const double* inducing;   /* host, m x 2 row-major */
  fsa_theta theta;          /* covariance parameters */
  double taper_range;       /* gamma > 0 */
  int64_t n_p;              /* FSA_REQ_PREDICT_VAR: prediction locations (>= 1), else 0 */
  const double* pred_locs;  /* host, n_p x 2 row-major (prediction only) */
  int32_t num_samples;      /* Algorithm 1's s (prediction only) */
  int32_t reserved0;
  double arrival_ms;        /* server clock (fsa_server_clock_ms); the request is not admitted before it */
} fsa_request;

typedef struct {
  int32_t slots;            /* workers: requests on the device at once, 1..64 */
  int32_t reserved0;
  uint64_t hbm_budget;      /* bytes of device memory shared by the admitted requests */
  fsa_options opt;          /* solver options of every request (hip_stream is ignored: each worker has one) */
} fsa_server_options;

typedef struct {
  int64_t id;
  int32_t status;           /* fsa_status of the request */
  int32_t kind;
  double nll;               /* FSA_REQ_NLL_GRAD */
  double grad[3];           /* FSA_REQ_NLL_GRAD, order (sigma1^2, rho, sigma^2) */
  double arrival_ms, admit_ms, done_ms; /* server clock */
  uint64_t footprint;       /* bytes reserved at admission */
  uint64_t peak_bytes;      /* most device bytes the request held at once */
  int32_t worker;           /* the worker that ran it (-1: refused) */
  int32_t iters_max;        /* PCG iterations of the slowest column */
  int64_t probe_iters;      /* PCG iterations summed over the columns */
  int64_t n_p;              /* length of the variance output */
  char message[192];        /* fsa_last_error() of a failed request */
} fsa_result;

typedef struct {
  int64_t submitted, completed, failed;
  uint64_t hbm_budget;
  uint64_t peak_reserved;   /* largest sum of admitted footprints at one time */
  int32_t slots, peak_active;
  double first_arrival_ms, last_done_ms;
} fsa_server_stats;

/* Device bytes a request may use at most: its context (taper pattern,
 * factors, float32 copies in the mixed modes), the PCG blocks and the
 * gradient (FSA_REQ_NLL_GRAD) or Algorithm 1's solves (FSA_REQ_PREDICT_VAR),
 * and the library's scratch.  The pattern's size comes from a host binning of
 * the locations on the device's grid (cells of side gamma (1 + 2^-20)): every
 * pair of points in neighbouring cells is counted, an upper bound on the
 * nonzeros.  INVALID_ARG for a request fsa_build would refuse. */
fsa_status fsa_request_footprint(const fsa_request* r, const fsa_options* opt, uint64_t* bytes);

/* Create a server on the current device; its clock starts at 0.  OOM if the
 * budget cannot be allocated; INVALID_ARG for bad options. */
fsa_status fsa_server_create(const fsa_server_options* o, fsa_server** out);
double fsa_server_clock_ms(const fsa_server* s);
/* Queue a request; its host arrays are copied before the call returns.
 * *id receives its handle.  A request whose footprint exceeds the budget
 * completes at once with FSA_ERR_OOM.  INVALID_ARG for a malformed request
 * (as fsa_build would refuse it). */
fsa_status fsa_server_submit(fsa_server* s, const fsa_request* r, int64_t* id);
/* Block until request `id` is done, fill *res, copy its predictive
 * variances (n_p doubles, nugget included) into var_out if not NULL, and
 * forget the request.  Returns FSA_OK when the wait succeeded (the request's
 * own status is res->status); INVALID_ARG for an unknown id. */
fsa_status fsa_server_wait(fsa_server* s, int64_t id, fsa_result* res, double* var_out);
fsa_status fsa_server_get_stats(fsa_server* s, fsa_server_stats* st);
/* Finish every queued request, then release the workers, streams and the
 * device block.  Results not yet collected are dropped. */
void fsa_server_destroy(fsa_server* s);

/* ------------------------------------------------------------------------
 * The FITC preconditioner in iterative methods for Vecchia approximations
 * (Section 5).
 *
 * Vecchia approximation of a latent process b ~ N(0, Sigma) (Section 5.1):
 * points in the given order; N(i) = the min(m_v, i) nearest of points
 * 0 .. i-1 (nearest first, a tie in distance to the lower index, squared
 * distances dx*dx + dy*dy in float64 without fused multiply-add);
 * A_i = Sigma_{N(i),i}^T Sigma_{N(i)}^{-1}, D_i = Sigma_ii - A_i Sigma_{N(i),i};
 * B unit lower triangular with B_{i,N(i)} = -A_i; Sigma_V^{-1} = B^T D^{-1} B.
 * W is a positive diagonal (negative second derivatives of a log-likelihood,
 * Section 5.1), given by the caller.
 *
 * Linear solves (Sigma_V^{-1} + W)^{-1} v are computed as
 * W^{-1} (Sigma_V + W^{-1})^{-1} Sigma_V v: block PCG on Sigma_V + W^{-1}
 * with the FITC preconditioner P = Sigma_mn^T Sigma_m^{-1} Sigma_mn + D_s,
 * D_s = diag(Sigma - Sigma_mn^T Sigma_m^{-1} Sigma_mn) + W^{-1} (Woodbury,
 * App. F).  (The printed equivalent form of eq. VL_v2 is not this inverse;
 * this one is.)  log det(Sigma_V^{-1} + W) = sum log W - sum log D +
 * log det(Sigma_V + W^{-1}), the last by preconditioned SLQ (Section 3.3)
 * with probes z ~ (0, P) drawn as for fsa_nll_grad (Rademacher, keyed by the
 * seed and the point index), weight z^T P^{-1} z.  Sigma_V products run as
 * two sparse triangular solves scheduled by levels of the neighbour graph.
 *
 * All pointers of these calls are device pointers; work runs on the stream
 * given at build (null: the default stream) and every call returns after it
 * has finished.
 * ------------------------------------------------------------------------ */
typedef struct fsa_vecchia fsa_vecchia; /* opaque; owned by the library until fsa_vecchia_destroy */

typedef struct {
  int32_t nlevels;      /* levels of the triangular-solve schedule */
  int32_t iters_max;    /* largest PCG iteration count over the columns */
  int32_t iters_rhs;    /* PCG iterations of the solve's column */
  int32_t converged;    /* 1 if every column met the tolerance */
  int64_t probe_iters;  /* PCG iterations summed over the columns */
  double logdet_P;      /* log det P (Sylvester, App. F) */
  double logdet_offset; /* sum log W - sum log D */
  double logdet_sw;     /* SLQ estimate of log det(Sigma_V + W^{-1}) */
  double ms_solve;      /* host wall-clock of the solve call */
} fsa_vecchia_stats;

typedef enum {
  FSA_V_SIGMA = 0,     /* Sigma_V X = B^{-1} D B^{-T} X */
  FSA_V_PRECISION = 1, /* Sigma_V^{-1} X = B^T D^{-1} B X */
  FSA_V_OPERATOR = 2,  /* (Sigma_V + W^{-1}) X, the PCG operator */
  FSA_V_P_INV = 3      /* P^{-1} X */
} fsa_vecchia_op;

/* Build the Vecchia factor (neighbours, A_i, D_i), its level schedule and
 * the FITC preconditioner of Sigma + W^{-1} (Section 5.1).  The neighbour
 * search is an exact scan of the earlier points (n^2/2 distance tests, about
 * 30 ms at n = 100,000); the triangular solves take one launch per level of
 * the neighbour graph (about 400 levels at n = 100,000, m_v = 30 in random
 * order), one per stretch of consecutive levels of a single point.  The
 * level schedule is built once per context.
 *   locs: n x 2 row-major; inducing: m x 2 row-major; w: n weights W_ii > 0;
 *   covariance kind (fsa_cov) with sigma1^2 > 0 and rho > 0 (no nugget:
 *   the process is latent); 0 <= m_v <= 32; 1 <= m <= 512.
 * The inputs are copied; the caller keeps ownership.  INVALID_ARG for bad
 * sizes or parameters or a weight that is not finite and positive; NOT_SPD
 * if a conditioning matrix Sigma_{N(i)}, Sigma_m or the capacitance cannot
 * be factored or a D_i is not positive.  A location repeated among the
 * earlier points makes D_i zero in exact arithmetic; in floating point it may
 * come out as a tiny positive number and pass, leaving an ill-conditioned
 * factor, so callers should merge duplicates first. */
fsa_status fsa_vecchia_build_dev(const double* locs, int64_t n, const double* inducing, int32_t m, int32_t kind,
                                 double sigma1_sq, double rho, int32_t mv, const double* w, void* hip_stream,
                                 fsa_vecchia** out);

/* Copy out the factor: nbr (n x m_v int32, -1 past the min(m_v, i)
 * neighbours of point i, nearest first), coef (n x m_v, A_i in the order of
 * nbr, 0 on the padding) and d (n, D_i). */
fsa_status fsa_vecchia_factor_dev(fsa_vecchia* v, int32_t* nbr, double* coef, double* d);

/* Y = op X for ncols columns of n x ncols row-major blocks with leading
 * dimensions ldx, ldy >= ncols; X and Y must not overlap. */
fsa_status fsa_vecchia_apply_dev(fsa_vecchia* v, int32_t which, const double* X, int64_t ldx, int32_t ncols,
                                 double* Y, int64_t ldy);

/* One block PCG run on Sigma_V + W^{-1} over [Sigma_V rhs, z_1 .. z_t]
 * (t = num_probes, 1..1023), each column stopped once ||r|| < tol ||b||, or,
 * with fixed_iter > 0 (<= 6000), every column run for exactly fixed_iter
 * iterations (tol and max_iter then unused):
 * x (n) = (Sigma_V^{-1} + W)^{-1} rhs and *logdet (host) = the SLQ estimate
 * of log det(Sigma_V^{-1} + W).  stats (host, may be null).  NOT_CONVERGED
 * if max_iter (<= 6000) was reached (outputs are still written); BREAKDOWN
 * if h^T K h <= 0 or a non-finite value appeared. */
fsa_status fsa_vecchia_solve_logdet_dev(fsa_vecchia* v, const double* rhs, double* x, int32_t num_probes,
                                        uint64_t seed, double tol, int32_t max_iter, int32_t fixed_iter,
                                        double* logdet, fsa_vecchia_stats* stats);

typedef struct {
  int32_t newton_steps;  /* Newton steps taken */
  int32_t converged;     /* 1 if the mode met newton_tol (0 with fixed_newton) */
  int32_t cg_iters_max;  /* most PCG iterations of any column of any solve */
  int32_t reserved0;
  int64_t probe_iters;   /* PCG iterations summed over every solve and column */
  double loglik;         /* log p(y | b) at the mode */
  double quad;           /* b^T Sigma_V^{-1} b at the mode */
  double sum_log_d;      /* sum log D_i of the Vecchia factor (log det Sigma_V) */
  double logdet;         /* SLQ estimate of log det(Sigma_V^{-1} + W) at the mode */
  double ms;             /* host wall-clock of the call */
} fsa_vecchia_laplace_stats;

/* Vecchia-Laplace approximation (Section 5.1) of the negative log marginal
 * likelihood of Bernoulli responses y in {0, 1} with the logistic link,
 * log p(y | b) = sum_i y_i b_i - log(1 + e^{b_i}), under the Vecchia prior
 * b ~ N(0, Sigma_V) of this handle.  The mode of log p(y|b) - b^T Sigma_V^{-1} b / 2
 * by Newton's method from b = 0,
 *   b <- (Sigma_V^{-1} + W)^{-1} (W b + y - pi),  pi = 1/(1 + e^{-b}),
 *   W = diag(pi (1 - pi)) (the negative second derivatives of the log-likelihood),
 * each solve by block PCG with the FITC preconditioner rebuilt for the
 * current W (as fsa_vecchia_solve_logdet_dev; the W given at build is
 * replaced), stopping when ||b_new - b|| <= newton_tol ||b_new|| or after
 * exactly fixed_newton steps (> 0; max_newton and newton_tol then unused).
 * At the mode, with W there,
 *   *nll = -log p(y|b) + b^T Sigma_V^{-1} b / 2 + log det(I + Sigma_V W) / 2,
 *   log det(I + Sigma_V W) = sum log D_i + log det(Sigma_V^{-1} + W),
 * the last term by SLQ with num_probes probes (1..1023) keyed by seed.
 * y and mode (n doubles, the caller's order) are device pointers; nll and
 * stats host.  tol, max_iter and fixed_iter apply to every PCG solve as in
 * fsa_vecchia_solve_logdet_dev.  INVALID_ARG for a response not 0 or 1 or
 * bad sizes; NOT_SPD if a weight underflows (|b| beyond about 36);
 * NOT_CONVERGED (outputs written) if a solve or the Newton iteration did not
 * converge; BREAKDOWN as the solve. */
fsa_status fsa_vecchia_laplace_dev(fsa_vecchia* v, const double* y, int32_t num_probes, uint64_t seed, double tol,
                                   int32_t max_iter, int32_t fixed_iter, double newton_tol, int32_t max_newton,
                                   int32_t fixed_newton, double* mode, double* nll,
                                   fsa_vecchia_laplace_stats* stats);

fsa_status fsa_vecchia_destroy(fsa_vecchia* v);

#ifdef __cplusplus
}
#endif
#endif /* FSA_H */
