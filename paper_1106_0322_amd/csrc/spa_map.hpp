// Launch interface of the EM MAP kernels (see spa_map.hip).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "spa_common.hpp"

namespace spa {

constexpr int kMapMaxP = 512;

struct MapArgs {
  const uint8_t *codes; // p x n_pad genotype codes 0/1/2, 3 in padded individuals
  const double *xv;     // p x 4 standardised value of each code ((c - mu_j)/s_j; 0 for code 3)
  const double *yv;     // n_pad labels (FP64), zero padded
  const void *beta0;    // M x p start points (FP32 or FP64)
  double *mode;         // M x p modes (output)
  double *logpost;      // M log posterior densities at the modes (output)
  Prior prior;
  int M, n, n_pad, p;
  int outer, inner;     // EM iterations; coordinate sweeps per iteration
};

// Largest n the EM kernel keeps in registers.
int map_max_n();
hipError_t launch_map_cols(const uint8_t *X, const uint8_t *y, int n, int p, int n_pad, const double *mu,
                           const double *sd, uint8_t *codes, double *xv, double *yv, hipStream_t st);
hipError_t launch_map_em(bool in_f64, const MapArgs &a, hipStream_t st);
hipError_t launch_best_particle(bool f64, const void *beta, const double *ll, int M, int p, const Prior &pr,
                                int *best, hipStream_t st);
hipError_t launch_map_starts(bool f64, const void *beta, const int *best, int p, const double *prev,
                             double *starts, hipStream_t st);
hipError_t launch_map_pick(const double *modes, const double *lp, int ns, int p, double *out, double *out_lp,
                           hipStream_t st);

}  // namespace spa
