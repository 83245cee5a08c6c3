// Launch interface of the single-coordinate random-walk kernel (see spa_single.hip).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "spa_common.hpp"

namespace spa {

struct SingleSiteArgs {
  const void *xs;       // p x n_pad standardised genotypes, particle precision, zero padded
  const void *yv;       // n_pad labels, particle precision, zero padded
  // n_pad: single_site_rows(n), the kernel's register rows (its loads are unguarded)
  const float *cs;      // FP32 instance: p column coefficients c_j = sum_k (y_k - 1/2) xs_jk
  void *beta;           // M x p particles (updated in place)
  double *ll;           // M log-likelihoods (output, from the tracked linear predictor)
  int *acc_cnt;         // M accepted coordinate updates (accumulated)
  Prior prior;
  double step;          // proposal standard deviation
  int M, n, n_pad, p;
  int cycles, cycle0;   // cycles run in this launch; Philox cycle index of the first
  uint32_t k0, k1;
  int t;
};

// Largest n the kernel keeps in registers.
int single_site_max_n();
// Padded individual count of the kernel's columns for n individuals: 64 R with R the
// smallest of 4, 8, 16, 32 that holds n (-1 beyond single_site_max_n()).
int single_site_rows(int n);
hipError_t launch_single_site(bool f64, const SingleSiteArgs &a, hipStream_t st);
hipError_t launch_std_cols(bool f64, const uint8_t *X, int n, int p, int n_pad, const double *mu,
                           const double *s, void *xs, hipStream_t st);
// c_j = sum_{k < n} (y_k - 1/2) xs_jk from the FP32 columns and labels (FP64 sums, FP32 out).
hipError_t launch_lin_cols(const float *xs, const float *yv, int n, int p, int n_pad, float *cs, hipStream_t st);

}  // namespace spa
