/*
 * spa_smc.h -- C ABI of the MI355X (gfx950) sparsity-path SMC sampler.
 *
 * The library evaluates, on one GPU, the data-parallel hot path of Bayesian
 * sparsity-path analysis with generalized-t priors (Lee, Caron, Doucet & Holmes,
 * arXiv:1106.0322):
 *
 *   model (Section 2):  y_k ~ Bernoulli(logit^-1(x_k beta)), k = 1..n, no intercept,
 *                       x_k the column-standardised genotypes (Section 3: mean 0, unit
 *                       standard deviation; the population sd of the sample is used);
 *   prior (Section 2):  beta_j iid Gt(a, c): p(beta_j) = 1/(2c) (1 + |beta_j|/(a c))^-(a+1),
 *                       the double exponential DE(0, c) when a = +inf;
 *   sampler (Section 4): SMC over a strictly decreasing scale sequence c_1 > ... > c_T
 *                       (called lambda below): prior-ratio incremental weights, normalised
 *                       weights, effective sample size, the estimate of Z_t / Z_{t-1},
 *                       resampling before moving when the ESS is low, then MCMC moves
 *                       (joint random-walk or MALA proposals) invariant for pi_t.
 *
 * Conventions for every entry point:
 *  - Return value: SPA_OK (0) or an error code; nothing throws or aborts across the
 *    ABI.  A message for the last error is available from spa_smc_last_error.
 *  - Arguments are validated on the host before any device work, so invalid calls leave
 *    the device untouched.
 *  - "_dev" pointers are device memory on the handle's device, borrowed for the call and
 *    ordered on the handle's HIP stream; the library never frees them.  "_host" pointers
 *    are host memory, copied before the call returns.
 *  - Matrices are row-major: beta is M x p with the p coefficients of a particle
 *    contiguous; X is n x p with the p markers of an individual contiguous.
 *  - A handle is not thread-safe; distinct handles are independent.
 *  - Floating-point results that depend on GEMM precision are documented per call.
 */
#ifndef SPA_SMC_H
#define SPA_SMC_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct spa_smc spa_smc;   /* opaque; owns every internal device buffer */

typedef enum {
  SPA_OK = 0,
  SPA_ERR_ARG = 1,      /* invalid argument value (null pointer, range, enum)           */
  SPA_ERR_SHAPE = 2,    /* inconsistent sizes, or a zero-variance genotype column       */
  SPA_ERR_ALLOC = 3,    /* device or host allocation failed                             */
  SPA_ERR_HIP = 4,      /* a HIP runtime call failed (message kept in last_error)       */
  SPA_ERR_STATE = 5,    /* call not valid in the handle's state (e.g. step after t = T) */
  SPA_ERR_NUMERIC = 6   /* NaN/Inf or all-zero weights, non-finite log-likelihood       */
} spa_status;

/* Precision of the log-likelihood contraction eta = X_std beta and of its adjoint. */
typedef enum {
  SPA_PREC_FP64 = 0,    /* FP64 MFMA, FP64 elementwise: per-particle loglik rel. err ~1e-13 */
  SPA_PREC_FP32 = 1,    /* FP32 MFMA, FP32 elementwise, FP64 cross-tile sums: ~1e-6        */
  SPA_PREC_BF16X2 = 2,  /* genotypes exact in BF16 (or FP8 storage), beta/s split into BF16
                           hi + lo parts, residuals likewise, FP32 MFMA accumulation:
                           per-particle loglik rel. err < 1e-4                             */
  SPA_PREC_FP8X3 = 3,   /* forward log-likelihood only (spa_smc_loglik, random-walk sweeps):
                           genotypes exact in e4m3, beta/s split into 3 e4m3 terms with
                           per-particle power-of-two scales (the block scales of the FP8
                           MFMA), FP32 accumulation: per-particle loglik rel. err < 1e-4   */
  SPA_PREC_FP8X4 = 4    /* as SPA_PREC_FP8X3 with 4 terms: rel. err below the BF16X2 one    */
} spa_prec;

/* Storage of the 0/1/2 genotype operand on the BF16X2 path (exact in both formats);
 * SPA_X_AUTO selects BF16. */
typedef enum { SPA_X_AUTO = 0, SPA_X_FP8E4M3 = 1, SPA_X_BF16 = 2 } spa_xfmt;

/* Move kernels: joint random walk, preconditioned MALA, or the paper's cycles of
 * single-coordinate random-walk updates (Section 4.1; one "sweep" = one cycle over the
 * p coordinates, proposal standard deviation `step0` kept fixed; n <= 2048). */
typedef enum { SPA_MOVE_RWM = 0, SPA_MOVE_MALA = 1, SPA_MOVE_SINGLE = 2 } spa_move;

typedef struct {
  int32_t n, p, N;        /* individuals, markers, particles; n, p, N >= 1, p <= 511     */
  double a;               /* Gt degrees of freedom > 0; +INFINITY = double exponential   */
  int32_t T;              /* number of scales, >= 1                                      */
  const double *lambda;   /* host, length T, strictly decreasing, > 0 (the Gt scale c)   */
  spa_move move;          /* move kernel                                                 */
  int32_t sweeps;         /* joint proposals per particle per scale, >= 0                */
  int32_t init_sweeps;    /* burn-in sweeps targeting pi_1 from beta = 0, >= 0           */
  double ess_frac;        /* resample iff ESS < ess_frac * N; in (0, 1]                  */
  double step0;           /* initial random-walk kappa or MALA h, > 0                    */
  int32_t adapt;          /* 1: log step += clip(acceptance - target, -log 2, log 2) after
                             each burn-in sweep and each scale; 0: fixed step            */
  spa_prec prec;          /* GEMM precision of the moves (the FP8 multi-term ones with
                             SPA_MOVE_RWM only: they have no adjoint); particles are
                             stored in FP64 for SPA_PREC_FP64 and in FP32 otherwise       */
  spa_xfmt xfmt;          /* genotype storage for SPA_PREC_BF16X2                         */
  uint64_t seed;          /* Philox4x32-10 key (low word, high word)                      */
} spa_smc_config;

/* Per-scale record returned by spa_smc_step (and for t = 1 by spa_smc_get_stats). */
typedef struct {
  int32_t t;              /* 1-based scale index the particles now target                */
  int32_t resampled;      /* 1 if resampling happened at this scale                      */
  double lambda;          /* lambda_t                                                    */
  double ess;             /* 1 / sum W^2 after reweighting (before resampling)           */
  double log_z_inc;       /* log of sum_i W_{t-1,i} w_{t,i}  (estimate of log Z_t/Z_{t-1}) */
  double log_z;           /* cumulative log Z_t / Z_1                                    */
  double accept_rate;     /* acceptance rate of this scale's sweeps                      */
  double step;            /* kappa or h used for this scale's sweeps                     */
} spa_smc_stats;

/*
 * spa_smc_init -- create a sampler, prepare operands and draw the initial particles.
 *
 * X_host: n x p genotypes in {0,1,2}; y_host: n labels in {0,1}; both copied.
 * hip_stream: the hipStream_t all work is ordered on (NULL = the null stream).
 * Operand preparation: per-marker mean mu_j, population sd s_j and X_std^T y (FP64),
 * genotype copies in the GEMM formats.  Initial particles (Section 4.1): beta = 0, then
 * cfg->init_sweeps sweeps targeting pi_1 (first half preconditioned by 2/sqrt(n), the
 * inverse root of the diagonal Fisher information at beta = 0, second half by the
 * cloud's standard deviation), then equal weights.  Records the statistics of t = 1.
 * Errors: SPA_ERR_ARG / SPA_ERR_SHAPE for invalid configuration, genotype or label
 * values, or a zero-variance marker; SPA_ERR_ALLOC; SPA_ERR_HIP.  On error *out = NULL.
 */
spa_status spa_smc_init(const spa_smc_config *cfg, const uint8_t *X_host, const uint8_t *y_host,
                        void *hip_stream, spa_smc **out);

/*
 * spa_smc_step -- advance from scale t to t + 1 (Section 4): incremental weights
 * log Gt(beta | a, lambda_{t+1}) - log Gt(beta | a, lambda_t) at the pre-move particles
 * (FP64), normalisation and log Z increment by logsumexp (FP64), ESS = 1/sum W^2,
 * systematic resampling if ESS < ess_frac * N (offset from Philox, see
 * spa_smc_resample), then cfg->sweeps move sweeps targeting pi_{t+1}, then the weighted
 * mean/variance of every coefficient (FP64).  Blocks until the step's statistics are on
 * the host.  out may be NULL.  SPA_ERR_STATE once t = T.  SPA_ERR_NUMERIC if the weights
 * or log-likelihoods became non-finite.
 */
spa_status spa_smc_step(spa_smc *h, spa_smc_stats *out);

/*
 * spa_smc_loglik -- log f(y | X, beta_i) for M particles (Section 2 likelihood):
 * sum_k [y_k eta_ik - log(1 + exp(eta_ik))], eta_i = X_std beta_i.
 * beta_dev: M x p, FP64 if beta_is_fp64 else FP32.  loglik_dev: M doubles (output).
 * prec selects the contraction precision.  With the FP8 multi-term precisions
 * (SPA_PREC_FP8X3, SPA_PREC_FP8X4; the random-walk sweeps of a handle created with one of
 * them pack their proposals the same way) the coefficient row of each particle is written as
 * sum_t 2^E_t q_t with e4m3 entries q_t, term t taking the residual of the terms before it
 * scaled so that its largest entry lies in [128, 256) (Section 2 likelihood on the
 * represented coefficients, whose offsets and X_std^T y term are formed exactly in FP64).
 * A particle with a non-finite coefficient gets a NaN log-likelihood.  Asynchronous on the
 * handle's stream.
 * Errors: SPA_ERR_ARG (null pointers, M < 1, bad prec, p > 255 with SPA_PREC_FP64).
 */
spa_status spa_smc_loglik(spa_smc *h, const void *beta_dev, int32_t M, int32_t beta_is_fp64,
                          spa_prec prec, double *loglik_dev);

/*
 * spa_smc_loglik_noalloc -- spa_smc_loglik without any device allocation, for callers
 * that cannot allocate (code under HIP graph capture, tight serving loops, harnesses that
 * forbid hipMalloc).  Same arguments, kernels and results (bit-identical to
 * spa_smc_loglik at the same prec) for prec SPA_PREC_FP64, SPA_PREC_FP32 or
 * SPA_PREC_BF16X2; no host synchronisation.  The scaled-coefficient operand, its offsets
 * and the contraction's split partial sums live in one static device array of 32 MiB per
 * GPU (held until the process ends), whose address the library takes at spa_smc_init.
 * Every call on a GPU shares that GPU's array, so calls that overlap on one GPU (other
 * streams, other handles, other threads) race and must be ordered by the caller.  The
 * array needs, per particle row (M rounded up to 128), PP * 4 bytes (BF16X2: hi and lo),
 * PP * 4 (FP32) or PP * 8 (FP64) plus 16 bytes of offsets and 8 bytes per individual
 * split of the contraction, PP being p + 1 rounded up to the contraction's width (at
 * p = 200 in BF16X2 about 36000 particles fit).
 * Errors: as spa_smc_loglik; SPA_ERR_ARG also for the FP8 multi-term precisions and for
 * an M whose buffers exceed the array (the message gives the bytes needed);
 * SPA_ERR_STATE if the genotype copy of prec has not been prepared (the handle's own
 * precision always is; another one after one spa_smc_loglik call with it).
 */
spa_status spa_smc_loglik_noalloc(spa_smc *h, const void *beta_dev, int32_t M, int32_t beta_is_fp64,
                                  spa_prec prec, double *loglik_dev);

/*
 * spa_smc_grad -- gradient of the log posterior at scale lambda for M particles:
 * X_std^T (y - logit^-1(X_std beta_i)) + d/dbeta log Gt(beta_i | a, lambda), the prior part
 * being -(a+1) sign(beta_ij)/(a lambda + |beta_ij|) (-sign(beta_ij)/lambda when a = inf),
 * sign(0) = 0; its magnitude is the EM weight of Section 2.1.
 * grad_dev: M x p, same dtype as beta (output).  logpost_dev (nullable): M doubles,
 * log f(y | X, beta_i) + sum_j log Gt(beta_ij | a, lambda).  Asynchronous.
 * Errors: SPA_ERR_ARG (null pointers, M < 1, lambda <= 0, bad prec, p > 255 with
 * SPA_PREC_FP64).
 */
spa_status spa_smc_grad(spa_smc *h, const void *beta_dev, int32_t M, int32_t beta_is_fp64,
                        double lambda, spa_prec prec, void *grad_dev, double *logpost_dev);

/*
 * spa_smc_resample -- systematic resampling of M weights (Section 4, resampling step).
 * w_dev: M doubles >= 0 (need not sum to one).  Offset U = u32 * 2^-32.  The weights are
 * quantised to integers q_i = floor((w_i / max w) * 2^K), K = 53 - ceil(log2 M), so the
 * cumulative sums are exact; offspring i takes the smallest k with
 * C_k > ((i + U) / M) * C_{M-1}, clamped to M - 1.  ancestors_dev: M int32 (output,
 * non-decreasing).  Bit-exact with a sequential evaluation of the same definition.
 * Blocks until the result is written.  Errors: SPA_ERR_ARG; SPA_ERR_NUMERIC for a
 * negative, NaN or infinite weight or all-zero weights (ancestors_dev then untouched).
 */
spa_status spa_smc_resample(spa_smc *h, const double *w_dev, int32_t M, uint32_t u32,
                            int32_t *ancestors_dev);

/*
 * Sparsity-path summaries (Section 5: absolute-median paths, credible intervals,
 * concentration plots, the posterior over the scale and the c-marginal summaries of the
 * marginal plots, the mixture being eq. all_particles of Section 4).
 *
 * Definitions shared by the calls below.  The weights are quantised to integers
 * q_i = floor((w_i / max w) * 2^K), K = 63 - ceil(log2 M), so every cumulative sum is an
 * exact 64-bit integer.  For a level alpha in (0, 1] the weighted quantile of a column is
 * the smallest value whose cumulative q (values in ascending order, -0 = +0) reaches
 * ceil(alpha * C), C = sum q, with alpha taken as the exact rational its double denotes.
 * The concentration for a tolerance Delta > 0 is V = 1 - S / C, S = sum of q_i over
 * |value_i| < Delta (open interval), the division in FP64.  Both are bit-exact with a
 * sequential evaluation of the same definitions.  At most 8 levels and 8 tolerances.
 */

/*
 * spa_weighted_summaries -- quantiles and concentrations of every column of one weighted
 * set.  values_dev: M x p row-major (FP64 if values_are_fp64 else FP32), finite;
 * w_dev: M doubles (>= 0, finite, not all zero; need not sum to one).  levels (L) and
 * deltas (D) are host arrays.  quant_dev: L x p doubles, conc_dev: D x p doubles (device
 * outputs, either NULL when its count is 0).  Works on the handle's stream and blocks
 * until done.  Errors: SPA_ERR_ARG (null pointers, more than 8 levels/tolerances, a
 * level outside (0, 1], a tolerance <= 0), SPA_ERR_SHAPE (M or p < 1), SPA_ERR_NUMERIC
 * (invalid weights; outputs then undefined).
 */
spa_status spa_weighted_summaries(spa_smc *h, const void *values_dev, int32_t M, int32_t p,
                                  int32_t values_are_fp64, const double *w_dev, const double *levels,
                                  int32_t L, const double *deltas, int32_t D, double *quant_dev,
                                  double *conc_dev);

/*
 * spa_smc_set_summaries -- from now on, after the moves of every scale t (and at once
 * for the current scale) record the quantiles (levels, L) and concentrations (deltas, D)
 * of each coefficient under the particles' normalised weights W_t: row t-1 of a
 * T x L x p and a T x D x p device array.  keep_history != 0 also keeps every scale's
 * particles and log weights (T x N x p + T x N device memory) for
 * spa_smc_marginal_summaries; it must then be called at the first scale.  Once per
 * handle.  Errors: SPA_ERR_ARG (as above), SPA_ERR_STATE, SPA_ERR_ALLOC.
 */
spa_status spa_smc_set_summaries(spa_smc *h, const double *levels, int32_t L, const double *deltas,
                                 int32_t D, int32_t keep_history);

/* Borrow the per-scale summary paths (rows 0..t-1 filled); either pointer may be NULL. */
spa_status spa_smc_get_summaries(const spa_smc *h, const double **quant_path_dev,
                                 const double **conc_path_dev);

/*
 * spa_smc_marginal_summaries -- summaries of the c-marginal posterior over the scales
 * 1..t run so far: the mixture of the weighted sets with weights proportional to
 * (Z_s / Z_1) W_s,i (a uniform prior on log c over the geometric grid), evaluated as
 * exp(log Z_s - max log Z + log W_s,i).  quant_dev: L x p, conc_dev: D x p, and
 * scale_post_dev (nullable): t doubles, p(c = lambda_s | X, y, a) = Z_s / sum Z.
 * Blocks until done.  Errors: SPA_ERR_STATE without a kept history, SPA_ERR_ARG.
 */
spa_status spa_smc_marginal_summaries(spa_smc *h, double *quant_dev, double *conc_dev,
                                      double *scale_post_dev);

/*
 * MAP estimates (Section 2.1): EM on the scale-mixture representation.  E step:
 * w_j = (a+1)/(a lambda + |beta_j|) (1/lambda for the double exponential); M step: `inner`
 * sweeps of cyclic coordinate ascent (j = 1..p) of log f(y | X, beta) - sum_j w_j |beta_j|
 * with the curvature bound n/4: beta_j <- S(beta_j + 4 g_j / n, 4 w_j / n), S the
 * soft-threshold, g_j the likelihood gradient; `outer` E steps.  FP64 throughout.
 *
 * spa_map_em -- from M start points beta0_dev (M x p, FP64 if beta_is_fp64 else FP32) at
 * scale lambda: mode_dev (M x p doubles) and logpost_dev (M doubles, log f + sum log Gt at
 * the mode).  Asynchronous on the handle's stream.  Errors: SPA_ERR_ARG, SPA_ERR_SHAPE
 * (M < 1, n > 10240, p > 512).
 */
spa_status spa_map_em(spa_smc *h, const void *beta0_dev, int32_t M, int32_t beta_is_fp64, double lambda,
                      int32_t outer, int32_t inner, double *mode_dev, double *logpost_dev);

/*
 * spa_smc_set_map -- record the MAP path (Section 4.1): at the current scale and after the
 * moves of every later one, EM from the particle of highest posterior density and from
 * the previous scale's MAP; the mode of higher posterior density is kept (the first on a
 * tie).  Once per handle.  spa_smc_get_map borrows the T x p path (rows of the scales
 * recorded) and its T log posterior densities.  Errors: SPA_ERR_STATE, SPA_ERR_SHAPE.
 */
spa_status spa_smc_set_map(spa_smc *h, int32_t outer, int32_t inner);
spa_status spa_smc_get_map(const spa_smc *h, const double **map_path_dev, const double **logpost_path_dev);

/*
 * spa_smc_get -- borrow the current state: particles (N x p, FP64 for SPA_PREC_FP64
 * else FP32), normalised log weights (N doubles), the per-scale weighted mean and
 * variance of every coefficient (T x p doubles each, rows 0..t-1 filled) and the host
 * array of cumulative log Z_t / Z_1 (T doubles).  Any output pointer may be NULL.
 * Valid until the next call that mutates the handle.  The current scale index t is
 * returned in *t_out (nullable).
 */
spa_status spa_smc_get(const spa_smc *h, const void **beta_dev, const double **logw_dev,
                       const double **mean_path_dev, const double **var_path_dev,
                       const double **logz_path_host, int32_t *t_out);

/* Borrow the per-particle log-likelihoods of the current particles (N doubles, device;
 * valid until the next call that mutates the handle). */
spa_status spa_smc_get_loglik(const spa_smc *h, const double **loglik_dev);

/* Statistics of scale t (1 <= t <= current t) recorded by init/step. */
spa_status spa_smc_get_stats(const spa_smc *h, int32_t t, spa_smc_stats *out);

/*
 * spa_smc_set_state -- replace the particle system: beta_dev (N x p, the handle's
 * particle dtype), logw_dev (N doubles, normalised log weights), the current scale
 * index t (1..T), and the proposal step.  Log-likelihoods (and gradients for MALA) are
 * recomputed.  The next spa_smc_step moves to t + 1.  Used to run one step from a given
 * state.  Errors: SPA_ERR_ARG.
 */
spa_status spa_smc_set_state(spa_smc *h, const void *beta_dev, const double *logw_dev,
                             int32_t t, double step);

/*
 * spa_philox4x32_10 -- Philox4x32-10 (Salmon, Moraes, Dror & Shaw, SC'11) on the device:
 * out[4i..4i+3] = Philox(counter ctr[4i..4i+3], key (seed mod 2^32, seed >> 32)) for
 * i < M.  ctr_dev, out_dev: 4M uint32.  Asynchronous on the handle's stream.
 */
spa_status spa_philox4x32_10(spa_smc *h, const uint32_t *ctr_dev, int32_t M, uint64_t seed,
                             uint32_t *out_dev);

/*
 * Kernel timing.  spa_smc_set_timing(h, 1) resets the counters and brackets every
 * subsequent launch of spa_smc_step (and of the burn-in) with HIP events on the handle's
 * stream; spa_smc_get_timing synchronises that stream, collects every bracketed launch so
 * far and fills ms[c] (total milliseconds) and launches[c] for the SPA_TIMING_CLASSES
 * classes below (launches of the burn-in, spa_smc_step, spa_smc_loglik and spa_smc_grad).
 * Timing adds a few microseconds of event records per launch; it is off by default.
 * Errors: SPA_ERR_ARG (null pointers), SPA_ERR_HIP.
 */
enum {
  SPA_T_PROPOSE = 0,    /* proposal + scaled-coefficient operand (first sweep of a   */
                        /* step; burn-in sweeps; single-coordinate cycles)             */
  SPA_T_LOGLIK = 1,     /* MFMA log-likelihood contraction (+ adjoint for MALA)        */
  SPA_T_ACCEPT = 2,     /* Metropolis-Hastings decisions; within a step, every sweep */
                        /* but the last also draws the next sweep's proposal here      */
  SPA_T_REWEIGHT = 3,   /* prior-ratio incremental weights with the logsumexp / ESS    */
                        /* partials and their combination (one launch)                 */
  SPA_T_LSE = 4,        /* systematic resampling when triggered: quantised weights,    */
                        /* exact CDF scan, offspring search with the particle gather   */
  SPA_T_GATHER = 5,     /* (no launches: the gather is part of SPA_T_LSE)              */
  SPA_T_MOMENTS = 6,    /* weighted moments                                            */
  SPA_T_FINALIZE = 7,   /* ordered sum of the contraction's split partials             */
  SPA_T_SUMMARY = 8,    /* sparsity-path summaries (quantiles, concentrations)         */
  SPA_T_MAP = 9,        /* EM MAP estimates                                            */
  SPA_TIMING_CLASSES = 10
};
spa_status spa_smc_set_timing(spa_smc *h, int32_t enable);
spa_status spa_smc_get_timing(spa_smc *h, double *ms, int64_t *launches);

/*
 * Timing of chosen classes only: bit c of class_mask brackets the launches of class c
 * (spa_smc_set_timing(h, 1) is the mask of all classes, 0 turns timing off).  Like
 * spa_smc_set_timing it synchronises the stream and resets the counters.  Each bracketed
 * launch costs a pair of event records on the stream, so timing one class (say the
 * contraction) perturbs the measured run far less than timing all of them.
 * Errors: SPA_ERR_ARG (null handle, bits at or above SPA_TIMING_CLASSES).
 */
spa_status spa_smc_set_timing_classes(spa_smc *h, uint32_t class_mask);

/* Release every resource of the handle (NULL is a no-op). */
void spa_smc_destroy(spa_smc *h);

/* Message of the last error on this handle ("" if none); h == NULL gives the message of
 * the last failed spa_smc_init in this thread. */
const char *spa_smc_last_error(const spa_smc *h);

#ifdef __cplusplus
}
#endif

#endif /* SPA_SMC_H */
