// Log-likelihood contraction of all particles against the genotype matrix, on MFMA.
//
// For a tile of particles i and all individuals k (Section 2 likelihood on standardised
// genotypes, Section 3):
//   eta_ik  = sum_j X_kj b_ij - m_i,     b_ij = beta_ij / s_j,  m_i = sum_j mu_j b_ij
//             (the standardisation folded into the coefficients, so X stays exact 0/1/2)
//   ll_i    = (X_std^T y) . beta_i - sum_k softplus(eta_ik)
//   g_ij    = (sum_k r_ik X_kj - mu_j rho_i) / s_j,   r_ik = y_k - logistic(eta_ik),
//             rho_i = sum_k r_ik  (the likelihood gradient X_std^T r_i)
//
// Structure (per workgroup of 4 wave64s): the particle tile's coefficients live in
// registers as MFMA B fragments for the whole sweep over individuals; genotype tiles
// (individual-major X and marker-major X^T) are staged through LDS; each wave computes
// eta^T blocks (individuals x particles) with MFMA, applies softplus/logistic in
// registers, and feeds the residuals -- already in the B-fragment layout of the MFMA
// output -- straight into the adjoint contraction G^T += X^T R^T, like the
// score-then-value chain of fused attention.  Neither eta nor the residuals touch HBM.
// On the BF16X2 path the coefficients and residuals are split into BF16 hi + lo parts
// (two MFMAs sharing the genotype fragment), with FP32 accumulation.  Softplus sums are
// accumulated per tile in the element type and across tiles in FP64, in a fixed order.
#include "spa_common.hpp"
#include "spa_internal.hpp"

namespace spa {

typedef __bf16 bf16x4 __attribute__((ext_vector_type(4)));

template <Prec P>
struct GT;

template <>
struct GT<Prec::BF16X2> {
  using LX = __bf16;   // genotype element in LDS
  using BT = __bf16;   // coefficient element in HBM
  using FR = bf16x8;   // MFMA A/B fragment (8 consecutive K values per lane)
  using AC = f32x4;
  using EL = float;    // elementwise type
  static constexpr int KS = 32, KV = 8, NT = 64, WP = 2, WN = 2;
  static __device__ __forceinline__ AC mfma(FR a, FR b, AC c) {
    return __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, c, 0, 0, 0);
  }
};

template <>
struct GT<Prec::F32> {
  using LX = float;
  using BT = float;
  using FR = float;
  using AC = f32x4;
  using EL = float;
  static constexpr int KS = 4, KV = 1, NT = 16, WP = 4, WN = 1;
  static __device__ __forceinline__ AC mfma(FR a, FR b, AC c) {
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
  }
};

template <>
struct GT<Prec::F64> {
  using LX = double;
  using BT = double;
  using FR = double;
  using AC = f64x4;
  using EL = double;
  static constexpr int KS = 4, KV = 1, NT = 16, WP = 4, WN = 1;
  static __device__ __forceinline__ AC mfma(FR a, FR b, AC c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
  }
};

template <Prec P, int PP>
struct Layout {
  using T = GT<P>;
  using LX = typename T::LX;
  using EL = typename T::EL;
  static constexpr int XS = PP + 16 / (int)sizeof(LX);     // sX row stride (elements)
  static constexpr int TS = T::NT + 16 / (int)sizeof(LX);  // sXt row stride
  static constexpr size_t tile_bytes =
      sizeof(LX) * ((size_t)T::NT * XS + (size_t)PP * TS) + sizeof(EL) * T::NT;
};

template <Prec P, int PP, int PB>
constexpr size_t lds_bytes() {
  using T = GT<P>;
  size_t red = 0;
  if (T::WN > 1) red = (size_t)T::WP * PB * (PP / 16) * 64 * 4 * sizeof(float) +
                       (size_t)T::WP * PB * 64 * sizeof(double);
  const size_t t = Layout<P, PP>::tile_bytes;
  return t > red ? t : red;
}

__device__ __forceinline__ float softplus_e(float eta, float e) {   // e = exp(-|eta|)
  return fmaxf(eta, 0.0f) + __logf(1.0f + e);
}
__device__ __forceinline__ double softplus_e(double eta, double e) {
  return fmax(eta, 0.0) + log1p(e);
}
__device__ __forceinline__ float exp_neg_abs(float eta) { return __expf(-fabsf(eta)); }
__device__ __forceinline__ double exp_neg_abs(double eta) { return exp(-fabs(eta)); }
__device__ __forceinline__ float logistic_e(float eta, float e) {
  const float r = __builtin_amdgcn_rcpf(1.0f + e);
  return eta >= 0.0f ? r : e * r;
}
__device__ __forceinline__ double logistic_e(double eta, double e) {
  return eta >= 0.0 ? 1.0 / (1.0 + e) : e / (1.0 + e);
}

template <Prec P, int PP, int PB, bool GRAD, bool FP8>
__global__ __launch_bounds__(256) void loglik_kernel(GemmArgs args) {
  using T = GT<P>;
  using LX = typename T::LX;
  using BT = typename T::BT;
  using FR = typename T::FR;
  using AC = typename T::AC;
  using EL = typename T::EL;
  constexpr int KS = T::KS, KV = T::KV, NT = T::NT, WP = T::WP, WN = T::WN;
  constexpr int IW = NT / WN;   // individuals per wave per tile
  constexpr int IB = IW / 16;   // 16-individual blocks per wave per tile
  constexpr int NKS = PP / KS;  // k-steps of the forward contraction
  constexpr int NMB = PP / 16;  // 16-marker blocks of the adjoint
  constexpr int XS = Layout<P, PP>::XS;
  constexpr int TS = Layout<P, PP>::TS;
  static_assert(IB >= 1, "a wave needs at least one 16-individual block");
  static_assert(P != Prec::BF16X2 || IB == 2, "BF16 adjoint k-step spans two blocks");
  static_assert(P == Prec::BF16X2 || IB == 1, "FP32/FP64 adjoint uses one block");

  extern __shared__ __align__(16) unsigned char smem[];
  LX *sX = reinterpret_cast<LX *>(smem);
  LX *sXt = sX + NT * XS;
  EL *sY = reinterpret_cast<EL *>(sXt + PP * TS);

  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int pg = wave / WN, nh = wave % WN;
  const int lr = lane & 15, lg = lane >> 4;
  const int wbase = blockIdx.x * (WP * 16 * PB) + pg * 16 * PB;

  // ---- coefficient fragments: register resident for the whole sweep over individuals
  FR bh[PB][NKS];
  FR bl[PB][(P == Prec::BF16X2) ? NKS : 1];
  EL moff[PB];
#pragma unroll
  for (int pb = 0; pb < PB; ++pb) {
    const size_t row = static_cast<size_t>(wbase + pb * 16 + lr);
    const BT *sh = reinterpret_cast<const BT *>(args.Bhi) + row * PP + lg * KV;
#pragma unroll
    for (int ks = 0; ks < NKS; ++ks) bh[pb][ks] = *reinterpret_cast<const FR *>(sh + ks * KS);
    if constexpr (P == Prec::BF16X2) {
      const BT *sl = reinterpret_cast<const BT *>(args.Blo) + row * PP + lg * KV;
#pragma unroll
      for (int ks = 0; ks < NKS; ++ks) bl[pb][ks] = *reinterpret_cast<const FR *>(sl + ks * KS);
    }
    moff[pb] = static_cast<EL>(args.moff[row]);
  }

  AC G[PB][GRAD ? NMB : 1];
  if constexpr (GRAD) {
#pragma unroll
    for (int pb = 0; pb < PB; ++pb)
#pragma unroll
      for (int mb = 0; mb < NMB; ++mb) G[pb][mb] = AC{0, 0, 0, 0};
  }
  double spl[PB];
#pragma unroll
  for (int pb = 0; pb < PB; ++pb) spl[pb] = 0.0;

  const int n = args.n, n_pad = args.n_pad;
  const EL *yv = reinterpret_cast<const EL *>(args.yv);

  for (int tile0 = 0; tile0 < n_pad; tile0 += NT) {
    __syncthreads();
    // ---- stage the genotype tile (individual-major) and its transpose (marker-major)
    if constexpr (FP8) {
      const uint8_t *gx = reinterpret_cast<const uint8_t *>(args.Xk) + (size_t)tile0 * PP;
      for (int idx = tid * 16; idx < NT * PP; idx += 256 * 16) {
        const uint4 v = *reinterpret_cast<const uint4 *>(gx + idx);
        const uint8_t *b = reinterpret_cast<const uint8_t *>(&v);
        LX *d = sX + (idx / PP) * XS + (idx % PP);
#pragma unroll
        for (int e = 0; e < 16; ++e) d[e] = static_cast<LX>(e4m3_to_float(b[e]));
      }
      const uint8_t *gt = reinterpret_cast<const uint8_t *>(args.Xt);
      for (int idx = tid * 16; idx < PP * NT; idx += 256 * 16) {
        const int r = idx / NT, c = idx % NT;
        const uint4 v = *reinterpret_cast<const uint4 *>(gt + (size_t)r * n_pad + tile0 + c);
        const uint8_t *b = reinterpret_cast<const uint8_t *>(&v);
        LX *d = sXt + r * TS + c;
#pragma unroll
        for (int e = 0; e < 16; ++e) d[e] = static_cast<LX>(e4m3_to_float(b[e]));
      }
    } else {
      constexpr int VG = 16 / (int)sizeof(LX);
      const LX *gx = reinterpret_cast<const LX *>(args.Xk) + (size_t)tile0 * PP;
      for (int idx = tid * VG; idx < NT * PP; idx += 256 * VG)
        *reinterpret_cast<uint4 *>(sX + (idx / PP) * XS + (idx % PP)) =
            *reinterpret_cast<const uint4 *>(gx + idx);
      const LX *gt = reinterpret_cast<const LX *>(args.Xt);
      for (int idx = tid * VG; idx < PP * NT; idx += 256 * VG) {
        const int r = idx / NT, c = idx % NT;
        *reinterpret_cast<uint4 *>(sXt + r * TS + c) =
            *reinterpret_cast<const uint4 *>(gt + (size_t)r * n_pad + tile0 + c);
      }
    }
    if (tid < NT) sY[tid] = yv[tile0 + tid];
    __syncthreads();

    // ---- forward: eta^T block (individuals x particles) = X_tile . b^T
    AC acc[IB][PB];
#pragma unroll
    for (int ib = 0; ib < IB; ++ib)
#pragma unroll
      for (int pb = 0; pb < PB; ++pb) acc[ib][pb] = AC{0, 0, 0, 0};
#pragma unroll
    for (int ks = 0; ks < NKS; ++ks) {
#pragma unroll
      for (int ib = 0; ib < IB; ++ib) {
        const FR a =
            *reinterpret_cast<const FR *>(sX + (nh * IW + ib * 16 + lr) * XS + ks * KS + lg * KV);
#pragma unroll
        for (int pb = 0; pb < PB; ++pb) {
          acc[ib][pb] = T::mfma(a, bh[pb][ks], acc[ib][pb]);
          if constexpr (P == Prec::BF16X2) acc[ib][pb] = T::mfma(a, bl[pb][ks], acc[ib][pb]);
        }
      }
    }

    // ---- elementwise: softplus row sums and residuals (lane: particle lr, 4 individuals)
    EL rv[IB][PB][4];
    EL sp[PB];
#pragma unroll
    for (int pb = 0; pb < PB; ++pb) sp[pb] = 0;
#pragma unroll
    for (int ib = 0; ib < IB; ++ib) {
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int kl = nh * IW + ib * 16 + lg * 4 + r;
        const bool valid = (tile0 + kl) < n;
        const EL yk = sY[kl];
#pragma unroll
        for (int pb = 0; pb < PB; ++pb) {
          const EL eta = static_cast<EL>(acc[ib][pb][r]) - moff[pb];
          const EL e = exp_neg_abs(eta);
          sp[pb] += valid ? softplus_e(eta, e) : EL(0);
          if constexpr (GRAD) rv[ib][pb][r] = valid ? yk - logistic_e(eta, e) : EL(0);
        }
      }
    }
#pragma unroll
    for (int pb = 0; pb < PB; ++pb) spl[pb] += static_cast<double>(sp[pb]);

    // ---- adjoint: G^T (markers x particles) += X_tile^T . R^T, residuals from registers
    if constexpr (GRAD) {
      if constexpr (P == Prec::BF16X2) {
        // K slot j of lane group lg maps to individual lg*4 + j (j < 4) of block 0 and
        // 16 + lg*4 + (j - 4) of block 1: exactly the rows this lane holds in acc.
        bf16x8 rh[PB], rl[PB];
#pragma unroll
        for (int pb = 0; pb < PB; ++pb) {
#pragma unroll
          for (int j = 0; j < 8; ++j) {
            const float v = rv[j >> 2][pb][j & 3];
            const __bf16 h = static_cast<__bf16>(v);
            rh[pb][j] = h;
            rl[pb][j] = static_cast<__bf16>(v - static_cast<float>(h));
          }
        }
#pragma unroll
        for (int mb = 0; mb < NMB; ++mb) {
          const LX *row = sXt + (mb * 16 + lr) * TS + nh * IW + lg * 4;
          const bf16x4 a0 = *reinterpret_cast<const bf16x4 *>(row);
          const bf16x4 a1 = *reinterpret_cast<const bf16x4 *>(row + 16);
          const bf16x8 a = __builtin_shufflevector(a0, a1, 0, 1, 2, 3, 4, 5, 6, 7);
#pragma unroll
          for (int pb = 0; pb < PB; ++pb) {
            G[pb][mb] = T::mfma(a, rh[pb], G[pb][mb]);
            G[pb][mb] = T::mfma(a, rl[pb], G[pb][mb]);
          }
        }
      } else {
        // 16x16x4: k-step i uses individual lg*4 + i, the lane's i-th row of acc.
#pragma unroll
        for (int mb = 0; mb < NMB; ++mb) {
          const LX *row = sXt + (mb * 16 + lr) * TS + nh * IW + lg * 4;
#pragma unroll
          for (int i = 0; i < 4; ++i) {
            const LX a = row[i];
#pragma unroll
            for (int pb = 0; pb < PB; ++pb) G[pb][mb] = T::mfma(a, rv[0][pb][i], G[pb][mb]);
          }
        }
      }
    }
  }

  // ---- reductions: over the 4 lane groups, then over the WN waves sharing particles
#pragma unroll
  for (int pb = 0; pb < PB; ++pb) {
    spl[pb] += __shfl_xor(spl[pb], 16, 64);
    spl[pb] += __shfl_xor(spl[pb], 32, 64);
  }
  if constexpr (WN > 1) {
    static_assert(WN == 2, "two waves share a particle group");
    __syncthreads();
    float *redG = reinterpret_cast<float *>(smem);
    double *redS = reinterpret_cast<double *>(smem + (size_t)WP * PB * NMB * 64 * 4 * sizeof(float));
    if (nh == 1) {
      if constexpr (GRAD) {
#pragma unroll
        for (int pb = 0; pb < PB; ++pb)
#pragma unroll
          for (int mb = 0; mb < NMB; ++mb)
            *reinterpret_cast<f32x4 *>(redG + (((pg * PB + pb) * NMB + mb) * 64 + lane) * 4) =
                G[pb][mb];
      }
#pragma unroll
      for (int pb = 0; pb < PB; ++pb) redS[(pg * PB + pb) * 64 + lane] = spl[pb];
    }
    __syncthreads();
    if (nh == 0) {
      if constexpr (GRAD) {
#pragma unroll
        for (int pb = 0; pb < PB; ++pb)
#pragma unroll
          for (int mb = 0; mb < NMB; ++mb)
            G[pb][mb] += *reinterpret_cast<const f32x4 *>(
                redG + (((pg * PB + pb) * NMB + mb) * 64 + lane) * 4);
      }
#pragma unroll
      for (int pb = 0; pb < PB; ++pb) spl[pb] += redS[(pg * PB + pb) * 64 + lane];
    }
  }
  if (nh != 0) return;

  // ---- epilogue: log-likelihood and standardised gradient
  const int M = args.M, p = args.p;
#pragma unroll
  for (int pb = 0; pb < PB; ++pb) {
    const int i = wbase + pb * 16 + lr;
    if (lg == 0 && i < M) args.ll[i] = args.yb[i] - spl[pb];
    if constexpr (GRAD) {
      // rho_i sits in the all-ones column PP-1: block NMB-1, lane group 3, element 3
      const double rho = static_cast<double>(__shfl(G[pb][NMB - 1][3], lr + 48, 64));
      if (i < M) {
        using GO = typename std::conditional<P == Prec::F64, double, float>::type;
        GO *g = reinterpret_cast<GO *>(args.g) + static_cast<size_t>(i) * p;
#pragma unroll
        for (int mb = 0; mb < NMB; ++mb) {
#pragma unroll
          for (int r = 0; r < 4; ++r) {
            const int j = mb * 16 + lg * 4 + r;
            if (j < p)
              g[j] = static_cast<GO>((static_cast<double>(G[pb][mb][r]) - args.mu[j] * rho) *
                                     args.inv_s[j]);
          }
        }
      }
    }
  }
}

// ------------------------------------------------------------------- dispatch

static const int kPadBF[] = {32, 64, 128, 224, 256, 384, 512};
static const int kPad64[] = {32, 64, 128, 224, 256};

int gemm_pad_markers(int p, Prec prec) {
  const int need = p + 1;   // + the all-ones column
  if (prec == Prec::F64) {
    for (int v : kPad64)
      if (v >= need) return v;
    return -1;
  }
  for (int v : kPadBF)
    if (v >= need) return v;
  return -1;
}

template <Prec P, int PP, int PB, bool GRAD, bool FP8>
static hipError_t launch_one(const GemmArgs &a, hipStream_t s) {
  constexpr size_t lds = lds_bytes<P, PP, PB>();
  static_assert(lds <= 160 * 1024, "LDS budget of one CU");
  auto kern = loglik_kernel<P, PP, PB, GRAD, FP8>;
  static bool attr_set = false;
  if (!attr_set) {
    hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void *>(kern),
                                       hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess) return e;
    attr_set = true;
  }
  constexpr int per_wg = GT<P>::WP * 16 * PB;
  const int grid = (a.M + per_wg - 1) / per_wg;
  hipLaunchKernelGGL(kern, dim3(grid), dim3(256), lds, s, a);
  return hipGetLastError();
}

template <Prec P, int PP, int PB>
static hipError_t launch_pp(const GemmArgs &a, hipStream_t s) {
  if (a.grad) {
    if (a.x_fp8) return launch_one<P, PP, PB, true, true>(a, s);
    return launch_one<P, PP, PB, true, false>(a, s);
  }
  if (a.x_fp8) return launch_one<P, PP, PB, false, true>(a, s);
  return launch_one<P, PP, PB, false, false>(a, s);
}

template <Prec P, int PP, int PB>
static hipError_t launch_pp_nofp8(const GemmArgs &a, hipStream_t s) {
  if (a.grad) return launch_one<P, PP, PB, true, false>(a, s);
  return launch_one<P, PP, PB, false, false>(a, s);
}

hipError_t launch_loglik(const GemmArgs &a, hipStream_t s) {
  switch (a.prec) {
    case Prec::BF16X2:
      switch (a.PP) {
        case 32: return launch_pp<Prec::BF16X2, 32, 2>(a, s);
        case 64: return launch_pp<Prec::BF16X2, 64, 2>(a, s);
        case 128: return launch_pp<Prec::BF16X2, 128, 2>(a, s);
        case 224: return launch_pp<Prec::BF16X2, 224, 2>(a, s);
        case 256: return launch_pp<Prec::BF16X2, 256, 2>(a, s);
        case 384: return launch_pp<Prec::BF16X2, 384, 1>(a, s);
        case 512: return launch_pp<Prec::BF16X2, 512, 1>(a, s);
      }
      break;
    case Prec::F32:
      switch (a.PP) {
        case 32: return launch_pp_nofp8<Prec::F32, 32, 1>(a, s);
        case 64: return launch_pp_nofp8<Prec::F32, 64, 1>(a, s);
        case 128: return launch_pp_nofp8<Prec::F32, 128, 1>(a, s);
        case 224: return launch_pp_nofp8<Prec::F32, 224, 1>(a, s);
        case 256: return launch_pp_nofp8<Prec::F32, 256, 1>(a, s);
        case 384: return launch_pp_nofp8<Prec::F32, 384, 1>(a, s);
        case 512: return launch_pp_nofp8<Prec::F32, 512, 1>(a, s);
      }
      break;
    case Prec::F64:
      switch (a.PP) {
        case 32: return launch_pp_nofp8<Prec::F64, 32, 1>(a, s);
        case 64: return launch_pp_nofp8<Prec::F64, 64, 1>(a, s);
        case 128: return launch_pp_nofp8<Prec::F64, 128, 1>(a, s);
        case 224: return launch_pp_nofp8<Prec::F64, 224, 1>(a, s);
        case 256: return launch_pp_nofp8<Prec::F64, 256, 1>(a, s);
      }
      break;
  }
  return hipErrorInvalidValue;
}

}  // namespace spa
