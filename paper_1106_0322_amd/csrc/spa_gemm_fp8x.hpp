// Forward log-likelihood contraction on the block-scaled FP8 MFMA, with the coefficients
// split into NTERM e4m3 terms (declarations shared by the C-ABI implementation).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace spa {

// Individuals per tile of the contraction; the genotype copy pads individuals to a multiple.
constexpr int kF8Tile = 128;
// Markers padded to whole 128-wide K steps of the FP8 MFMA: 128, 256, 384 or 512 (-1: p too large).
int fp8x_pad_markers(int p);
// Particles per workgroup for nterm terms (64, 128 or 256; operand rows are padded to it).
int fp8x_particles_per_wg(int PP, int nterm);

struct Fp8xArgs {
  int nterm;            // 3 or 4 coefficient terms
  int PP;               // padded markers (fp8x_pad_markers)
  const uint8_t *Xf;    // n_pad x PP genotype codes (e4m3), zero padded; n_pad % kF8Tile == 0
  const uint8_t *Bq;    // nterm x M_pad x PP e4m3 codes of the coefficient terms
  const int32_t *Bs;    // nterm x M_pad biased exponents (E8M0) of the terms' scales
  const double *moff;   // M_pad: log2(e) sum_j mu_j b_ij of the represented coefficients
  const double *yb;     // M_pad: sum_j (X_std^T y)_j beta_ij of the represented coefficients
  int n, n_pad, M, M_pad;
  int S;                // individual splits (1, 2, 4, 8)
  double *spl_part;     // S x M_pad partial softplus sums (S > 1)
  double *ll;           // M outputs
};

// Genotype codes (n x p bytes 0/1/2, row-major) -> Xf.
hipError_t launch_fp8x_pack_x(const uint8_t *X, int n, int p, int n_pad, int PP, uint8_t *Xf,
                              hipStream_t st);
// Particles (M x p, FP64 when in_f64 else FP32) -> the term codes, scales and offsets.
hipError_t launch_fp8x_pack_b(int nterm, bool in_f64, const void *beta, int M, int M_pad, int p, int PP,
                              const double *mu, const double *s, const double *inv_s, const double *ytil,
                              uint8_t *Bq, int32_t *Bs, double *moff, double *yb, hipStream_t st);
// Splits for a launch over M particles (same policy as the BF16 contraction).
int fp8x_splits(int PP, int nterm, int n_pad, int M);
// The contraction; with S > 1 it leaves split partials that launch_fp8x_finalize adds in
// split order into ll (a no-op for S = 1).
hipError_t launch_fp8x_loglik(const Fp8xArgs &a, hipStream_t st);
hipError_t launch_fp8x_finalize(const Fp8xArgs &a, hipStream_t st);

}  // namespace spa
