// Host-side declarations shared by the C-ABI implementation and the kernel files.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/spa_smc.h"

namespace spa {

enum class Prec : int { F64 = 0, F32 = 1, BF16X2 = 2 };

// The reduced-precision contraction works in base 2: its coefficient operand holds
// (beta/s) log2(e) and its offsets m_i log2(e), so the kernel's exponentials and logarithms
// need no extra scaling.  FP64 keeps natural units.
constexpr double kLog2e = 1.44269504088896340736;
__host__ __device__ constexpr double operand_scale(Prec p) { return p == Prec::F64 ? 1.0 : kLog2e; }

// Padded marker count used by the GEMM operands: the smallest instantiated width that
// holds the p markers plus the all-ones column kept in the last padded column.
int gemm_pad_markers(int p, Prec prec);
// Particles per workgroup of the contraction kernel (operand rows are padded to it).
int gemm_particles_per_wg(Prec prec, int PP);
// Number of contiguous individual ranges the contraction is split into (1, 2, 4 or 8),
// chosen so that one range of both genotype copies fits an XCD's L2 and every CU has work.
int gemm_splits(Prec prec, int PP, int n_pad, int M, size_t x_bytes_both);
// Individuals are padded to a multiple of this (largest tile of any precision).
constexpr int kIndPad = 64;
// Particle rows of every operand buffer are padded to a multiple of this.
constexpr int kPartPad = 128;

struct GemmArgs {
  Prec prec;
  int PP;              // padded markers (from gemm_pad_markers)
  bool grad;           // also compute the likelihood gradient
  bool x_fp8;          // BF16X2 only: genotypes stored as FP8 e4m3
  const void *Xk;      // n_pad x PP genotypes + ones column (storage format)
  const void *Xt;      // PP x n_pad, the transpose
  const void *yv;      // n_pad labels (double for F64, float otherwise), zero padded
  const void *Bhi;     // M_pad x PP coefficients (beta/s) operand_scale (BF16 hi part, or FP32/FP64)
  const void *Blo;     // M_pad x PP BF16 lo part (BF16X2 only)
  const double *moff;  // M_pad offsets m_i = operand_scale sum_j mu_j beta_ij / s_j
  const double *yb;    // M: sum_j (X_std^T y)_j beta_ij
  const double *mu;    // PP (zero padded)
  const double *inv_s; // PP (zero padded)
  const double *ytil;  // PP: X_std^T y (zero padded)
  int n, n_pad, M, M_pad, p;
  int S;               // individual splits (1, 2, 4, 8)
  double *spl_part;    // S x M_pad partial softplus sums (S > 1)
  void *g_part;        // S x M_pad x PP partial adjoints (S > 1; double for F64, float otherwise)
  double *ll;          // M outputs: yb - sum_k softplus(eta_ik)
  void *g;             // M x p likelihood gradient (double for F64, float otherwise)
};

// The contraction kernel, then (when S > 1) the ordered combination of the split partials.
hipError_t launch_loglik(const GemmArgs &a, hipStream_t s);
hipError_t launch_gemm_finalize(const GemmArgs &a, hipStream_t s);

// Position of individual i (0 <= i < xt_group) inside a group of the marker-major genotype
// copy, chosen so that the K slots of a lane's adjoint MFMA fragment are contiguous in LDS:
// BF16 groups of 32 hold the lane-group pieces {4g..4g+3, 16+4g..16+4g+3} next to each
// other; FP64 groups of 16 hold {g, g+4, g+8, g+12} (the FP64 MFMA's output rows of lane
// group g) next to each other; FP32 keeps the natural order.
__host__ __device__ constexpr int xt_group(Prec p) { return p == Prec::BF16X2 ? 32 : 16; }
__host__ __device__ inline int xt_position(Prec p, int i) {
  if (p == Prec::BF16X2) {
    const int b = i / 16, r = i % 16;
    return (r / 4) * 8 + b * 4 + r % 4;
  }
  if (p == Prec::F64) return (i % 4) * 4 + i / 4;
  return i;
}

}  // namespace spa
