// Launch interface of the bandwidth-bound kernels (see spa_kernels.hip).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <algorithm>

#include "spa_common.hpp"
#include "spa_internal.hpp"

namespace spa {

enum class XFormat { F64, F32, BF16, FP8 };

struct ProposeArgs {
  const void *beta;      // M x p current particles (PT)
  const void *gl;        // M x p log-likelihood gradient at beta (MALA)
  void *prop;            // M x p proposal (PT)
  void *Bhi, *Blo;       // M_pad x PP B operand of the proposal
  double *moff, *yb;     // M_pad
  double *lp_cur, *lp_prop, *lqf;   // M
  const void *mc;        // 4 x PP per-marker move constants (launch_move_consts), PT
  struct {
    const double *mu, *s, *inv_s, *ytil;   // PP-padded column constants
  } cc;
  Prior prior;
  double step, sqrt_step;
  int M, M_pad, p, PP;
  uint32_t k0, k1, sweep;
  int t;
  // Random-walk rows of a handle on the FP8 multi-term contraction (f8_terms = 3 or 4): the
  // operand is written as f8_terms e4m3 term rows (f8_terms x f8_Mp x f8_PP codes, f8_terms
  // x f8_Mp biased exponents) instead of BF16 hi/lo, and moff / yb describe those terms.
  uint8_t *f8_q;
  int32_t *f8_s;
  int f8_terms, f8_Mp, f8_PP;
};

struct AcceptArgs {
  void *beta, *gl;                  // M x p state (updated in place)
  const void *prop, *gl_prop;       // M x p proposal and its likelihood gradient
  double *ll;                       // M state log-likelihood (updated)
  const double *ll_prop, *lp_cur, *lp_prop, *lqf;
  // When the contraction ran in S > 1 individual ranges, its per-range partial sums are
  // combined here (same order and arithmetic as the finalize kernel) instead of reading
  // ll_prop / gl_prop: spl_part is S x Mp softplus sums, g_part S x Mp x PP adjoint sums.
  const double *spl_part;           // null: read ll_prop / gl_prop
  const void *g_part;
  int S, PP;
  size_t Mp;
  const double *yb, *mu, *inv_s, *ytil;
  const void *mc;                   // 4 x PP per-marker move constants, PT
  int *acc_cnt;
  Prior prior;
  double step;
  int M, p;
  uint32_t k0, k1, sweep;
  int t;
};

// Incremental weights with the normalisation and ESS partials (reweight_kernel).
struct ReweightArgs {
  const void *beta;            // M x p particles (FP64 or FP32)
  int M, p;
  double a;                    // Gt degrees of freedom (unused when a_inf)
  int a_inf;
  double lam_new, lam_old, ess_frac;
  double *logw;                // in: normalised log W_{t-1}; out: unnormalised log weights
  double *part;                // 3 x reweight_blocks(M, p) workgroup partials
  double *scalars;             // out: {ESS, L, resample flag, max log weight, non-finite, 0}
};

// Systematic resampling on the exact quantised CDF (quantise, scan, search [+ gather]).
struct ResampleArgs {
  int mode;                    // 0: from the reweighting pass's log weights; 1: linear weights w
  int M, K;                    // K = 53 - ceil(log2 M)
  uint32_t u32;                // offset U = u32 2^-32
  double *logw;                // mode 0: unnormalised log weights in; set to logw_eq when gathering
  double logw_eq;              // -log M
  const double *w;             // mode 1: weights >= 0
  double *cdf;                 // M scratch
  double *btot;                // 1024 scratch
  double *wpart;               // 2 x 1024 scratch (mode 1)
  double *scalars;             // [3] max log weight (mode 0), [5] invalid flag, [6] max w, [7] C
  int *anc;                    // M ancestors (out)
  // gather (null src: ancestors only): particle rows, gradient rows (nullable), loglik
  int p;
  const void *src;
  void *dst;
  const void *gsrc;
  void *gdst;
  const double *llsrc;
  double *lldst;
};

void launch_col_stats(const uint8_t *X, const uint8_t *y, int n, int p, double *mu, double *s,
                      double *inv_s, double *ytil, int *bad, hipStream_t st);
void launch_pack_x(XFormat f, Prec prec, const uint8_t *X, int n, int p, int n_pad, int PP, void *Xk,
                   void *Xt, hipStream_t st);
void launch_labels(const uint8_t *y, int n, int n_pad, bool f64, void *yv, hipStream_t st);
void launch_pack_b(Prec prec, bool in_f64, const void *beta, int M, int M_pad, int p, int PP,
                   const double *mu, const double *s, const double *inv_s, const double *ytil,
                   void *Bhi, void *Blo, double *moff, double *yb, hipStream_t st);
void launch_propose(Prec prec, bool mala, const ProposeArgs &a, hipStream_t st);
// next != null: the decision kernel also draws the next sweep's proposal (same buffers as
// a launch_propose with *next) from each row it has just decided.  PP: the padded row
// length of the contraction's operand (it sets the lanes per particle row).
hipError_t launch_accept(Prec prec, bool mala, int PP, const AcceptArgs &a, const ProposeArgs *next, hipStream_t st);
// Workgroups of the reweighting pass (its partials hold 3 doubles per workgroup); the
// launch is the pass and the one-workgroup combination of its partials.
int reweight_blocks(int M, int p);
void launch_reweight(bool f64, const ReweightArgs &a, hipStream_t st);
// Scratch of the resampling passes: at most this many workgroups per pass.
constexpr int kResampleBlocks = 1024;
void launch_resample(bool f64, const ResampleArgs &a, hipStream_t st);
int moments_chunks(int M);
// shift (nullable, device): the log weights are first normalised in place, logw -= *shift.
void launch_moments(bool f64, const void *beta, double *logw, const double *shift, int M, int p, double *part,
                    double *mean, double *var, double *sigma, double sigma_floor, hipStream_t st);
// out[0] = sum of the accept counts; out[1] = particles with a non-finite log-likelihood
// (ll may be null: 0).
void launch_count(const int *cnt, int M, const double *ll, long long *out, hipStream_t st);
void launch_fill(double *x, int n, double v, hipStream_t st);
void launch_zero_int(int *x, int n, hipStream_t st);
// Per-marker constants of the proposal and decision kernels for one step size and
// preconditioner, in the particle precision (double when f64, else float), written to mc
// (4 x PP): (0.5 step) sigma sigma; the MALA variance 2 step sigma sigma (in FP32 its
// hardware reciprocal); sqrt(step) sigma; step sigma (sigma = 0 in padded markers).  The
// kernel also zeroes the N acceptance counters acc.  sqrt_step is sqrt(step) in FP64.
void launch_move_consts(bool f64, const double *sigma, int p, int PP, double step, double sqrt_step, void *mc,
                        int *acc, int N, hipStream_t st);
void launch_convert(bool src_f64, const void *src, void *dst, size_t n, hipStream_t st);
void launch_add_prior(bool beta_f64, bool g_f64, const void *beta, int M, int p, const Prior &pr, void *g,
                      const double *ll, double *logpost, hipStream_t st);
void launch_philox(const uint32_t *ctr, int M, uint32_t k0, uint32_t k1, uint32_t *out, hipStream_t st);

}  // namespace spa
