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
  const double *sigma;   // p preconditioner
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
  const double *sigma;
  int *acc_cnt;
  Prior prior;
  double step;
  int M, p;
  uint32_t k0, k1, sweep;
  int t;
};

struct LseArgs {
  int mode;              // 0: log weights (normalise, ESS, maybe resample); 1: linear weights
  int M, K;
  double ess_frac;
  double *logw;          // mode 0: in/out
  const double *w;       // mode 1: input weights
  double *cdf;           // M scratch
  int *anc;              // M output ancestors
  double *scalars;       // {ess, log Z increment, resampled, max, nonfinite, invalid weights}
  uint32_t u32;
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
void launch_accept(Prec prec, bool mala, int PP, const AcceptArgs &a, const ProposeArgs *next, hipStream_t st);
void launch_reweight(bool f64, const void *beta, int M, int p, double a, int a_inf, double lam_new,
                     double lam_old, double *logw, hipStream_t st);
void launch_lse_resample(const LseArgs &a, hipStream_t st);
void launch_gather(bool f64, const int *anc, int M, int p, const void *src, void *dst, const void *gsrc,
                   void *gdst, const double *llsrc, double *lldst, hipStream_t st);
int moments_chunks(int M);
void launch_moments(bool f64, const void *beta, const double *logw, int M, int p, double *part,
                    double *mean, double *var, double *sigma, double sigma_floor, hipStream_t st);
// out[0] = sum of the accept counts; out[1] = particles with a non-finite log-likelihood
// (ll may be null: 0).
void launch_count(const int *cnt, int M, const double *ll, long long *out, hipStream_t st);
void launch_fill(double *x, int n, double v, hipStream_t st);
void launch_zero_int(int *x, int n, hipStream_t st);
void launch_convert(bool src_f64, const void *src, void *dst, size_t n, hipStream_t st);
void launch_add_prior(bool beta_f64, bool g_f64, const void *beta, int M, int p, const Prior &pr, void *g,
                      const double *ll, double *logpost, hipStream_t st);
void launch_philox(const uint32_t *ctr, int M, uint32_t k0, uint32_t k1, uint32_t *out, hipStream_t st);

}  // namespace spa
