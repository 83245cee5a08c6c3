// Host-side declarations shared by the C-ABI implementation and the kernel files.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/spa_smc.h"

namespace spa {

enum class Prec : int { F64 = 0, F32 = 1, BF16X2 = 2 };

// Padded marker count used by the GEMM operands: the smallest instantiated width that
// holds the p markers plus the all-ones column kept in the last padded column.
int gemm_pad_markers(int p, Prec prec);
// Individuals are padded to a multiple of this (largest tile of any precision).
constexpr int kIndPad = 64;
// Particle rows of every operand buffer are padded to a multiple of this.
constexpr int kPartPad = 64;

struct GemmArgs {
  Prec prec;
  int PP;              // padded markers (from gemm_pad_markers)
  bool grad;           // also compute the likelihood gradient
  bool x_fp8;          // BF16X2 only: genotypes stored as FP8 e4m3
  const void *Xk;      // n_pad x PP genotypes + ones column (storage format)
  const void *Xt;      // PP x n_pad, the transpose
  const void *yv;      // n_pad labels (double for F64, float otherwise), zero padded
  const void *Bhi;     // M_pad x PP scaled coefficients beta/s (BF16 hi part, or FP32/FP64)
  const void *Blo;     // M_pad x PP BF16 lo part (BF16X2 only)
  const double *moff;  // M_pad offsets m_i = sum_j mu_j beta_ij / s_j
  const double *yb;    // M: sum_j (X_std^T y)_j beta_ij
  const double *mu;    // PP (zero padded)
  const double *inv_s; // PP (zero padded)
  int n, n_pad, M, p;
  double *ll;          // M outputs: yb - sum_k softplus(eta_ik)
  void *g;             // M x p likelihood gradient (double for F64, float otherwise)
};

hipError_t launch_loglik(const GemmArgs &a, hipStream_t s);

}  // namespace spa
