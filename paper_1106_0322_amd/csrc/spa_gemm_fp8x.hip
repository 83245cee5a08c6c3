// Forward log-likelihood contraction on the block-scaled FP8 MFMA (16x16x128, e4m3 x e4m3,
// FP32 accumulation), with the coefficients carried by several e4m3 terms.
//
// What is computed is the per-particle log-likelihood of Section 2 on standardised genotypes,
//   ll_i = (X_std^T y) . beta_i - sum_k softplus(eta_ik),   eta_ik = sum_j X_kj b_ij - m_i,
// with b_ij = beta_ij / s_j and m_i = sum_j mu_j b_ij (the standardisation folded into the
// coefficients, so the genotypes stay the exact codes 0/1/2, which e4m3 holds exactly).
//
// Coefficient split.  Per particle i, in units of log2(e), the row b_i is written as
//   b_i ~= sum_t 2^(E_it) q_it,   q_it in e4m3,
// term by term: E_it = floor(log2 max_j |r_ij|) - 7 puts the largest residual r of the row
// in [128, 256), each entry whose scaled residual is at least 1 is rounded to the nearest
// e4m3 value, smaller ones are left whole to the later terms, and what is not represented
// becomes the next term's residual.  Each term resolves at least 4 more bits of the row's
// largest entry; three terms meet a 1e-4 relative tolerance on the log-likelihood with
// margin and four are tighter than the BF16 hi+lo split.  The scale 2^(E_it) is the MFMA's
// per-column (per-particle) E8M0 block scale of the B operand, so one accumulator collects
// every term.  The offsets m_i and (X_std^T y) . beta_i are formed from the represented
// coefficients (exact in FP64), so eta is the linear predictor of exactly the coefficients
// the MFMA sees.
//
// Why entries below 1 wait: the MFMA adds the products of each group of 8 K values in a
// fixed-point window about 13 binades below the group's largest product (measured: with
// one product 2^8 and seven of 2^-6 in a group the small ones vanish, with 2^-5 they are
// kept; sums across groups and the accumulator are exact to FP32).  With |q| in [1, 256]
// and genotypes 0/1/2 every product lies in [1, 512] with its last bit at or above 2^-3,
// so each group sum is exact.
//
// Work decomposition as in the BF16 contraction: a wave owns 16 particles (their terms stay
// in registers for the whole pass), a workgroup of NW waves streams its range of
// individuals in tiles of 128 through double-buffered LDS filled by global -> LDS DMA, and
// the workgroup -> (split, particle tile) map follows the round-robin dispatch of
// workgroups to the 8 XCDs.  The genotype tile is one byte per entry, half the BF16 tile,
// and twice as many individuals per tile halve the tile barriers (measured: 68 -> 61 us for
// 3 terms at 5000 individuals, 200 markers, 16384 particles; a software pipeline that
// issues one half tile's MFMAs between the previous half's elementwise instructions was
// slower, 67 us).
//
// Operand layout of the 16x16x128 FP8 MFMA (measured): lane l holds row (A) or column (B)
// l % 16; within lane group g = l / 16 its 32 bytes are K = 16g..16g+15 and
// K = 64+16g..64+16g+15.  A and B use the same arrangement, so any fixed K order of the
// 128 markers of a step gives the same dot product; here bytes 0-15 and 16-31 of a lane are
// the row's 16-byte chunks 4*0+g and 4*1+g of the step.  The E8M0 scale of each operand is
// byte 0 of a per-lane register; every lane of a column carries the same exponent.
#include "spa_common.hpp"
#include "spa_lanes.hpp"
#include "spa_gemm_fp8x.hpp"
#include "spa_internal.hpp"

namespace spa {

namespace {

typedef int i32x8 __attribute__((ext_vector_type(8)));

constexpr int kF8Unit = 127;   // E8M0 code of 2^0

// Genotype codes (validated 0, 1 or 2 at init) in OCP e4m3: 0, 1.0 = 0x38, 2.0 = 0x40.
__device__ __forceinline__ uint8_t genotype_code(uint8_t v) { return v == 0 ? 0 : (v == 1 ? 0x38 : 0x40); }

// ---------------------------------------------------------------- packing
__global__ void fp8x_pack_x_kernel(const uint8_t *__restrict__ X, int n, int p, int n_pad, int PP,
                                   uint8_t *__restrict__ Xf) {
  const size_t total = (size_t)n_pad * PP;
  for (size_t idx = blockIdx.x * (size_t)blockDim.x + threadIdx.x; idx < total;
       idx += (size_t)gridDim.x * blockDim.x) {
    const int k = static_cast<int>(idx / PP), j = static_cast<int>(idx % PP);
    Xf[idx] = (k < n && j < p) ? genotype_code(X[(size_t)k * p + j]) : uint8_t(0);
  }
}

// Reductions over the LN lanes of a particle (fixed orders).
template <int LN>
__device__ __forceinline__ double f8_group_max(double v) {
#pragma unroll
  for (int o = LN / 2; o > 0; o >>= 1) v = fmax(v, __shfl_xor(v, o, 64));
  return v;
}
template <int LN>
__device__ __forceinline__ double f8_group_sum(double v) {
  return lane_group_sum<LN>(v);   // the order of the proposal step's sums (bit-identical operands)
}
template <int LN>
__device__ __forceinline__ int f8_group_or(int v) {
#pragma unroll
  for (int o = LN / 2; o > 0; o >>= 1) v |= __shfl_xor(v, o, 64);
  return v;
}

// LN lanes per particle row, in the layout of the sampler's move kernels: lane l holds
// markers 4l + 4 LN kb + k (kb = 0, 1; k = 0..3), LN = 32 (two rows per wave) when p + 1
// <= 256, else 64.  The sampler's proposal step packs its random-walk proposals with the
// same arithmetic in the same order, so both give identical codes, exponents and offsets.
template <int NTERM, int LN, typename IT>
__global__ __launch_bounds__(256) void fp8x_pack_b_kernel(const IT *__restrict__ beta, int M, int M_pad, int p,
                                                          int PP, const double *__restrict__ mu,
                                                          const double *__restrict__ s,
                                                          const double *__restrict__ inv_s,
                                                          const double *__restrict__ ytil, uint8_t *__restrict__ Bq,
                                                          int32_t *__restrict__ Bs, double *__restrict__ moff,
                                                          double *__restrict__ yb) {
  constexpr int KB = 2;
  const int lane = threadIdx.x & (LN - 1);
  const int i = static_cast<int>((blockIdx.x * blockDim.x + threadIdx.x) / LN);
  if (i >= M_pad) return;
  double v[KB][4], used[KB][4];
  int bad = 0;
#pragma unroll
  for (int kb = 0; kb < KB; ++kb)
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      const int j = 4 * lane + 4 * LN * kb + k;
      v[kb][k] = (i < M && j < p) ? static_cast<double>(beta[(size_t)i * p + j]) * inv_s[j] * kLog2e : 0.0;
      used[kb][k] = 0.0;
      bad |= !isfinite(v[kb][k]);
    }
  bad = f8_group_or<LN>(bad);
#pragma unroll
  for (int t = 0; t < NTERM; ++t) {
    double R = 0.0;
#pragma unroll
    for (int kb = 0; kb < KB; ++kb)
#pragma unroll
      for (int k = 0; k < 4; ++k) R = fmax(R, fabs(v[kb][k] - used[kb][k]));
    R = f8_group_max<LN>(R);
    int E = 0;
    if (R > 0.0 && isfinite(R)) {
      int e2;
      frexp(R, &e2);
      E = e2 - 1 - 7;                       // R 2^-E in [128, 256)
    }
    E = max(-kF8Unit, min(kF8Unit, E));
    uint8_t *q = Bq + ((size_t)t * M_pad + i) * PP;
#pragma unroll
    for (int kb = 0; kb < KB; ++kb) {
      const int b0 = 4 * lane + 4 * LN * kb;
      uint32_t packed = 0;
#pragma unroll
      for (int k = 0; k < 4; ++k) {
        // scaled residual below 256 in magnitude; the hardware conversion rounds it to the
        // nearest e4m3 value, and the decoded code (the value the MFMA uses) is what counts
        const float x = static_cast<float>(ldexp(v[kb][k] - used[kb][k], -E));
        const int c = fabsf(x) >= 1.0f ? (__builtin_amdgcn_cvt_pk_fp8_f32(x, 0.0f, 0, false) & 0xFF) : 0;
        used[kb][k] += ldexp(static_cast<double>(__builtin_amdgcn_cvt_f32_fp8(c, 0)), E);
        packed |= static_cast<uint32_t>(c) << (8 * k);
      }
      if (b0 < PP) *reinterpret_cast<uint32_t *>(q + b0) = packed;   // 4-byte aligned
    }
    if (lane == 0) Bs[(size_t)t * M_pad + i] = E + kF8Unit;
  }
  double m = 0.0, ybv = 0.0;
#pragma unroll
  for (int kb = 0; kb < KB; ++kb)
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      const int j = 4 * lane + 4 * LN * kb + k;
      const bool in = j < PP;
      m += (in ? mu[j] : 0.0) * used[kb][k];
      ybv += (in ? ytil[j] * s[j] : 0.0) * used[kb][k];
    }
  m = f8_group_sum<LN>(m);
  ybv = f8_group_sum<LN>(ybv);
  if (lane == 0) {
    const double nan = __builtin_nan("");
    moff[i] = bad ? nan : m;
    yb[i] = bad ? nan : ybv / kLog2e;
  }
}

// ---------------------------------------------------------------- contraction
// Waves per workgroup: with rows of up to 256 markers, 3 terms fit 4 waves per SIMD
// (120 VGPRs; measured 63 -> 59 us at 5000 individuals, 200 markers, 16384 particles),
// 4 terms 2 (at 4 they spill); wider rows 2 (at most 210 VGPRs).
__host__ __device__ constexpr int f8_waves(int PP, int nterm) { return PP <= 256 ? (nterm == 3 ? 16 : 8) : 8; }

template <int PP, int NTERM>
struct F8Shape {
  static constexpr int NT = kF8Tile;                // individuals per tile
  static constexpr int NW = f8_waves(PP, NTERM);
  static constexpr int NTHR = 64 * NW;
  static constexpr int WGP = 16 * NW;               // particles per workgroup
  static constexpr int CPR = PP / 16, CX = CPR + 1; // 16-byte chunks per row; odd LDS stride
  static constexpr int XSL = (NT * CX + NTHR - 1) / NTHR * NTHR;   // slots per stage
  static constexpr size_t bytes = 2 * (size_t)XSL * 16;
};

__device__ __forceinline__ void f8_lds_dma16(const void *g, uint4 *lds) {
  __builtin_amdgcn_global_load_lds(g, lds, 16, 0, 0);
}

template <int PP, int NTERM>
__global__ __attribute__((amdgpu_flat_work_group_size(64, (F8Shape<PP, NTERM>::NTHR))))
__attribute__((amdgpu_waves_per_eu((F8Shape<PP, NTERM>::NW / 4), (F8Shape<PP, NTERM>::NW / 4)))) void fp8x_loglik_kernel(Fp8xArgs args) {
  using SH = F8Shape<PP, NTERM>;
  constexpr int NT = SH::NT, IB = NT / 16, NKS = PP / 128, CX = SH::CX, CPR = SH::CPR;
  constexpr int XSL = SH::XSL, NTHR = SH::NTHR, WGP = SH::WGP, NQ = XSL / NTHR;
  extern __shared__ __align__(16) uint4 smem[];

  const int S = args.S, g8 = 8 / S;
  const int xcd = blockIdx.x & 7, slot = blockIdx.x >> 3;
  const int split = xcd / g8, ptile = slot * g8 + xcd % g8;
  if (ptile >= (args.M + WGP - 1) / WGP) return;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6, lr = lane & 15, lg = lane >> 4;
  const int n = args.n, n_pad = args.n_pad;
  const int chunk = ((n_pad + S - 1) / S + NT - 1) / NT * NT;
  const int i0 = min(n_pad, split * chunk);
  const int i1 = min(min(n_pad, i0 + chunk), (n + NT - 1) / NT * NT);
  const int ntiles = max(0, (i1 - i0) / NT);

  // ---- this lane's particle: its coefficient terms and scales, register resident
  const int row = ptile * WGP + wave * 16 + lr;
  i32x8 b[NTERM][NKS];
  int sc[NTERM];
#pragma unroll
  for (int t = 0; t < NTERM; ++t) {
    const uint8_t *q = args.Bq + ((size_t)t * args.M_pad + row) * PP + 16 * lg;
#pragma unroll
    for (int ks = 0; ks < NKS; ++ks) {
      const uint4 lo = *reinterpret_cast<const uint4 *>(q + ks * 128);
      const uint4 hi = *reinterpret_cast<const uint4 *>(q + ks * 128 + 64);
      b[t][ks] = i32x8{(int)lo.x, (int)lo.y, (int)lo.z, (int)lo.w, (int)hi.x, (int)hi.y, (int)hi.z, (int)hi.w};
    }
    sc[t] = args.Bs[(size_t)t * args.M_pad + row];
  }
  const float moff = static_cast<float>(args.moff[row]);
  double spl = 0.0;

  // ---- tile staging: slot q*NTHR + tid of a stage is this thread's q-th 16-byte copy
  int xoff[NQ];
#pragma unroll
  for (int q = 0; q < NQ; ++q) {
    const int sl = q * NTHR + tid, r = sl / CX, c = sl % CX;
    xoff[q] = (r < NT && c < CPR) ? r * PP + c * 16 : 0;   // padding slots copy chunk 0 (never read)
  }
  auto issue = [&](const int tile0, const int stage) {
    const uint8_t *bx = args.Xf + (size_t)tile0 * PP;
#pragma unroll
    for (int q = 0; q < NQ; ++q) f8_lds_dma16(bx + xoff[q], smem + stage * XSL + q * NTHR + wave * 64);
  };
  auto land = [&]() {
    asm volatile("s_waitcnt vmcnt(0)" ::: "memory");
    __syncthreads();
  };
  if (ntiles > 0) issue(i0, 0);
  land();

  auto tile_step = [&](const int it, auto masked_c) {
    constexpr bool MASKED = decltype(masked_c)::value;
    const int tile0 = i0 + it * NT, stage = it & 1;
    // next tile (the last one re-copies itself into the idle stage, never read)
    issue(i0 + min(it + 1, ntiles - 1) * NT, stage ^ 1);
    const uint4 *sX = smem + stage * XSL;
    // the tile in quarters of HB 16-individual blocks (bounds the fragment registers)
    constexpr int HB = 4;
#pragma unroll
    for (int h = 0; h < IB / HB; ++h) {
      f32x4 acc[HB];
#pragma unroll
      for (int ib = 0; ib < HB; ++ib) acc[ib] = f32x4{0, 0, 0, 0};
#pragma unroll
      for (int ks = 0; ks < NKS; ++ks) {
        i32x8 a[HB];
#pragma unroll
        for (int ib = 0; ib < HB; ++ib) {
          const uint4 *rp = sX + ((h * HB + ib) * 16 + lr) * CX + ks * 8 + lg;
          const uint4 lo = rp[0], hi = rp[4];
          a[ib] = i32x8{(int)lo.x, (int)lo.y, (int)lo.z, (int)lo.w, (int)hi.x, (int)hi.y, (int)hi.z, (int)hi.w};
        }
#pragma unroll
        for (int t = 0; t < NTERM; ++t)
#pragma unroll
          for (int ib = 0; ib < HB; ++ib)
            acc[ib] = __builtin_amdgcn_mfma_scale_f32_16x16x128_f8f6f4(a[ib], b[t][ks], acc[ib], 0, 0, 0,
                                                                       0x7F7F7F7F, 0, sc[t]);
      }
      // softplus sum, in base 2 (the operand carries log2(e)): lane holds particle lr and
      // individuals 16 (h HB + ib) + 4 lg + v; one log of the product of <= 16 factors in
      // (1, 2].
      float prod = 1.0f, mx = 0.0f;
#pragma unroll
      for (int ib = 0; ib < HB; ++ib)
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          const float z = acc[ib][v] - moff;
          const float e = __builtin_amdgcn_exp2f(-fabsf(z));
          if (!MASKED || tile0 + (h * HB + ib) * 16 + 4 * lg + v < n) {
            prod = fmaf(prod, e, prod);
            mx += fmaxf(z, 0.0f);
          }
        }
      spl += static_cast<double>(0.6931471805599453f * (mx + __builtin_amdgcn_logf(prod)));
    }
    land();
  };
  const bool has_tail = ntiles > 0 && i0 + ntiles * NT > n;
  const int nfull = ntiles - (has_tail ? 1 : 0);
  for (int it = 0; it < nfull; ++it) tile_step(it, std::false_type{});
  if (has_tail) tile_step(nfull, std::true_type{});

  spl += __shfl_xor(spl, 16, 64);
  spl += __shfl_xor(spl, 32, 64);
  if (lg == 0) {
    if (S == 1) {
      if (row < args.M) args.ll[row] = args.yb[row] - spl;
    } else {
      args.spl_part[(size_t)split * args.M_pad + row] = spl;
    }
  }
}

__global__ void fp8x_finalize_kernel(Fp8xArgs args) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= args.M) return;
  double spl = 0.0;
  for (int s = 0; s < args.S; ++s) spl += args.spl_part[(size_t)s * args.M_pad + i];
  args.ll[i] = args.yb[i] - spl;
}

template <int PP, int NTERM>
hipError_t launch_fp8x_one(const Fp8xArgs &a, hipStream_t st) {
  constexpr size_t lds = F8Shape<PP, NTERM>::bytes;
  static_assert(lds <= 160 * 1024, "LDS budget of one CU");
  auto kern = fp8x_loglik_kernel<PP, NTERM>;
  static bool attr_set = false;
  if (!attr_set) {
    const hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void *>(kern),
                                             hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess) return e;
    attr_set = true;
  }
  constexpr int per_wg = F8Shape<PP, NTERM>::WGP;
  const int tiles_p = (a.M + per_wg - 1) / per_wg;
  const int g8 = 8 / a.S;
  const int grid = 8 * ((tiles_p + g8 - 1) / g8);
  hipLaunchKernelGGL(kern, dim3(grid), dim3(F8Shape<PP, NTERM>::NTHR), lds, st, a);
  return hipGetLastError();
}

template <int NTERM>
hipError_t launch_fp8x_terms(const Fp8xArgs &a, hipStream_t st) {
  switch (a.PP) {
    case 128: return launch_fp8x_one<128, NTERM>(a, st);
    case 256: return launch_fp8x_one<256, NTERM>(a, st);
    case 384: return launch_fp8x_one<384, NTERM>(a, st);
    case 512: return launch_fp8x_one<512, NTERM>(a, st);
  }
  return hipErrorInvalidValue;
}

}  // namespace

int fp8x_pad_markers(int p) {
  const int PP = (p + 127) / 128 * 128;
  return (p >= 1 && PP <= 512) ? PP : -1;
}

int fp8x_particles_per_wg(int PP, int nterm) { return 16 * f8_waves(PP, nterm); }

int fp8x_splits(int PP, int nterm, int n_pad, int M) {
  const int NT = kF8Tile, per_wg = fp8x_particles_per_wg(PP, nterm);
  const int tiles_p = (M + per_wg - 1) / per_wg;
  const size_t x_bytes = (size_t)n_pad * PP;
  int S = 1;
  // keep one split's genotype slice within an XCD's L2 ...
  while (S < 8 && x_bytes / S > (size_t)3 * 1024 * 1024 && n_pad / (2 * S) >= NT) S *= 2;
  // ... and give every CU a workgroup
  while (S < 8 && (size_t)tiles_p * S < 256 && n_pad / (2 * S) >= NT) S *= 2;
  return S;
}

hipError_t launch_fp8x_pack_x(const uint8_t *X, int n, int p, int n_pad, int PP, uint8_t *Xf, hipStream_t st) {
  const size_t total = (size_t)n_pad * PP;
  const int grid = static_cast<int>(std::min<size_t>((total + 255) / 256, 65535));
  hipLaunchKernelGGL(fp8x_pack_x_kernel, dim3(grid), dim3(256), 0, st, X, n, p, n_pad, PP, Xf);
  return hipGetLastError();
}

hipError_t launch_fp8x_pack_b(int nterm, bool in_f64, const void *beta, int M, int M_pad, int p, int PP,
                              const double *mu, const double *s, const double *inv_s, const double *ytil,
                              uint8_t *Bq, int32_t *Bs, double *moff, double *yb, hipStream_t st) {
  if (PP > 512 || PP % 128 != 0 || M_pad % 8 != 0) return hipErrorInvalidValue;
  // lanes per row as in the sampler's move kernels: 32 when p + 1 <= 256
  const bool narrow = p + 1 <= 256;
#define SPA_F8PACK(NT_, LN_, IT_)                                                                         \
  hipLaunchKernelGGL((fp8x_pack_b_kernel<NT_, LN_, IT_>), dim3(M_pad / (256 / (LN_))), dim3(256), 0, st, \
                     (const IT_ *)beta, M, M_pad, p, PP, mu, s, inv_s, ytil, Bq, Bs, moff, yb)
#define SPA_F8PACK_LN(NT_, IT_)               \
  do {                                        \
    if (narrow) SPA_F8PACK(NT_, 32, IT_);     \
    else SPA_F8PACK(NT_, 64, IT_);            \
  } while (0)
  if (nterm == 3) {
    if (in_f64) SPA_F8PACK_LN(3, double); else SPA_F8PACK_LN(3, float);
  } else if (nterm == 4) {
    if (in_f64) SPA_F8PACK_LN(4, double); else SPA_F8PACK_LN(4, float);
  } else {
    return hipErrorInvalidValue;
  }
#undef SPA_F8PACK_LN
#undef SPA_F8PACK
  return hipGetLastError();
}

hipError_t launch_fp8x_loglik(const Fp8xArgs &a, hipStream_t st) {
  if (a.S != 1 && a.S != 2 && a.S != 4 && a.S != 8) return hipErrorInvalidValue;
  if (a.M_pad % fp8x_particles_per_wg(a.PP, a.nterm) != 0 || a.n_pad % kF8Tile != 0) return hipErrorInvalidValue;
  return a.nterm == 3 ? launch_fp8x_terms<3>(a, st)
         : a.nterm == 4 ? launch_fp8x_terms<4>(a, st) : hipErrorInvalidValue;
}

hipError_t launch_fp8x_finalize(const Fp8xArgs &a, hipStream_t st) {
  if (a.S == 1) return hipSuccess;
  hipLaunchKernelGGL(fp8x_finalize_kernel, dim3((a.M + 255) / 256), dim3(256), 0, st, a);
  return hipGetLastError();
}

}  // namespace spa
