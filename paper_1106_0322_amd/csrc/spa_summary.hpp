// Launch interface of the sparsity-path summary kernels (see spa_summary.hip).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace spa {

constexpr int kSqMaxLevels = 8;   // quantile levels and concentration tolerances per call

struct SqLevels {
  int L, D;                       // number of quantile levels / tolerances
  double alpha[kSqMaxLevels];     // levels in (0, 1]
  double delta[kSqMaxLevels];     // tolerances > 0
};

struct SqState {                  // device
  uint64_t total;                 // C = sum of the quantised weights
  uint64_t thr[kSqMaxLevels];     // ceil(alpha_l C)
  int flags;                      // bit 0: invalid weights
};

struct SqSel {                    // device, per (coefficient, level)
  uint64_t prefix;                // key digits chosen so far
  uint64_t below;                 // quantised weight of all values below the prefix's range
};

struct SqArgs {
  const void *values;             // M x p, FP64 if f64 else FP32
  bool f64;
  int M, p;
  const double *w;                // M weights (>= 0, finite, not all zero), or log weights
  bool log_weights;               // w holds log weights (-inf allowed): w_i = exp(w_i - max)
  SqLevels lv;
  // scratch (device)
  uint64_t *q;                    // M
  void *keys;                     // p x M keys (8 or 4 bytes each)
  SqState *st;
  SqSel *sel;                     // p x kSqMaxLevels
  unsigned long long *hist;       // p x kSqMaxLevels x 256, zero on entry, left zero
  unsigned long long *inside;     // kSqMaxLevels x p
  // outputs (device)
  double *quant;                  // L x p
  double *conc;                   // D x p
};

inline int ceil_log2_ll(long long m) {
  int k = 0;
  while ((1ll << k) < m) ++k;
  return k;
}

int sq_key_bytes(bool f64);
hipError_t launch_weighted_summaries(const SqArgs &a, hipStream_t s);
hipError_t launch_mixture_weights(const double *log_z, int T, int N, const double *logW, double *w,
                                  double *scale_post, hipStream_t s);

}  // namespace spa
