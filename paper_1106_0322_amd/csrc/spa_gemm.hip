// Log-likelihood contraction of all particles against the genotype matrix, on MFMA.
//
// For particles i and individuals k (Section 2 likelihood on standardised genotypes,
// Section 3):
//   eta_ik = sum_j X_kj b_ij - m_i,    b_ij = beta_ij / s_j,   m_i = sum_j mu_j b_ij
//            (the standardisation folded into the coefficients: X stays exact 0/1/2)
//   ll_i   = (X_std^T y) . beta_i - sum_k softplus(eta_ik)
//   g_ij   = (X_std^T y)_j - (sum_k sigma_ik X_kj - mu_j sum_k sigma_ik) / s_j,
//            sigma_ik = logistic(eta_ik)   (the likelihood gradient X_std^T (y - sigma))
//
// Work decomposition.  A workgroup of 4 wave64s owns a tile of 64*PB particles; each wave
// keeps the BF16 hi/lo (or FP32/FP64) fragments of its 16*PB particles in registers for
// the whole pass.  Individuals are split into S contiguous ranges, one per workgroup of a
// "split"; the workgroup -> (split, particle tile) map follows the round-robin dispatch of
// workgroups to the 8 XCDs so that the XCDs of one split share its genotype slice in their
// L2.  A workgroup streams its slice in tiles of NT individuals through double-buffered
// LDS (the next tile is prefetched into registers while the current one is used): the
// individual-major tile feeds the forward MFMA (eta^T blocks, individuals x particles) and,
// for the gradient, the marker-major tile feeds the adjoint MFMA G^T += X^T sigma^T, whose
// B operand is the logistic of the forward output taken straight from the accumulator
// registers (a lane of an eta^T block holds four individuals of one particle, i.e. the K
// slots of an MFMA B fragment).  Softplus sums: per lane and tile, sum max(eta, 0) plus
// one log of prod (1 + exp(-|eta|)) (the product of at most 16 factors in (1, 2] cannot
// overflow), accumulated across tiles in FP64 in a fixed order; in reduced precision
// sum max(eta, 0) is taken as half of sum |eta| (the standardised genotypes are centred,
// so sum_k eta_ik = 0 over the real individuals).  With S > 1 each split
// writes partial sums that a finalize kernel adds in split order.
#include "spa_common.hpp"
#include "spa_internal.hpp"

namespace spa {

typedef __bf16 bf16x4 __attribute__((ext_vector_type(4)));
typedef float f32x2 __attribute__((ext_vector_type(2)));
typedef __bf16 bf16x2 __attribute__((ext_vector_type(2)));

template <Prec P>
struct GT;

template <>
struct GT<Prec::BF16X2> {
  using LX = __bf16;   // genotype element in LDS
  using BT = __bf16;   // coefficient element in HBM
  using FR = bf16x8;   // MFMA A/B fragment (8 consecutive K values per lane)
  using AC = f32x4;
  using EL = float;
  static constexpr int KS = 32, KV = 8;
  // rows of a 16x16 output block held by lane group g: 4g + v
  static __device__ __forceinline__ constexpr int crow(int g, int v) { return 4 * g + v; }
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
  static constexpr int KS = 4, KV = 1;
  static __device__ __forceinline__ constexpr int crow(int g, int v) { return 4 * g + v; }
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
  static constexpr int KS = 4, KV = 1;
  // the FP64 16x16x4 MFMA interleaves rows across lane groups: g + 4v
  static __device__ __forceinline__ constexpr int crow(int g, int v) { return g + 4 * v; }
  static __device__ __forceinline__ AC mfma(FR a, FR b, AC c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
  }
};

// LDS fragment reads kept in flight ahead of the MFMAs that consume them (BF16 path).
constexpr int kPrefetch = 4;

// Tile shape per precision and padded marker count.  Each wave owns 16 particles (one
// MFMA column block); a workgroup has NW waves.  With PP <= 256 the BF16 and FP32 variants
// fit two waves per SIMD (8 per workgroup), so one wave's elementwise VALU work overlaps
// the other's MFMAs; wider rows (and FP64) keep one wave per SIMD.
template <Prec P, int PP>
struct Shape {
  static constexpr int NT = (P == Prec::BF16X2) ? (PP <= 256 ? 64 : 32) : 16;   // individuals
  static constexpr int PB = 1;                                                   // 16-particle blocks per wave
  static constexpr int NW = (P != Prec::F64 && PP <= 256) ? 8 : 4;               // waves per workgroup
  static constexpr int NTHR = 64 * NW;
  static constexpr int WGP = NW * 16 * PB;                                       // particles per workgroup
};

// LDS stage layout in 16-byte chunks ("slots").  The individual-major tile has NT rows of
// CPR = PP*es/16 chunks and the marker-major tile PP rows of CPT = NT*es/16 chunks; each row
// is padded by one chunk (odd stride: the 16-byte fragment reads of 16 consecutive rows hit
// distinct banks), and each region is rounded up to a multiple of the thread count so that every thread moves
// exactly one chunk per copy instruction.  Two stages (double buffering).
template <Prec P, int PP, bool GRAD>
struct Lds {
  using LX = typename GT<P>::LX;
  static constexpr int NT = Shape<P, PP>::NT;
  static constexpr int CPR = PP * (int)sizeof(LX) / 16, CX = CPR + 1;
  static constexpr int CPT = NT * (int)sizeof(LX) / 16, CT = CPT + 1;
  static constexpr int NTHR = Shape<P, PP>::NTHR;
  static constexpr int XSL = (NT * CX + NTHR - 1) / NTHR * NTHR;
  static constexpr int TSL = GRAD ? (PP * CT + NTHR - 1) / NTHR * NTHR : 0;
  static constexpr int STG = XSL + TSL;
  static constexpr size_t bytes = 2 * (size_t)STG * 16;
};

// One 16-byte global -> LDS copy per lane; lane i writes lds[i] (wave-uniform base).
__device__ __forceinline__ void lds_dma16(const void *g, uint4 *lds) {
  __builtin_amdgcn_global_load_lds(g, lds, 16, 0, 0);
}

__device__ __forceinline__ float fast_exp2(float x) { return __builtin_amdgcn_exp2f(x); }
__device__ __forceinline__ float fast_log2(float x) { return __builtin_amdgcn_logf(x); }
__device__ __forceinline__ float fast_rcp(float x) { return __builtin_amdgcn_rcpf(x); }

// 16 FP8 (e4m3) codes -> 16 BF16 values in LDS (exact for finite codes).
__device__ __forceinline__ void store_fp8_as_bf16(__bf16 *dst, uint4 v) {
  const uint32_t w[4] = {v.x, v.y, v.z, v.w};
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    const f32x2 lo = __builtin_amdgcn_cvt_pk_f32_fp8(static_cast<int>(w[q]), false);
    const f32x2 hi = __builtin_amdgcn_cvt_pk_f32_fp8(static_cast<int>(w[q]), true);
    bf16x4 o;
    o[0] = static_cast<__bf16>(lo[0]);
    o[1] = static_cast<__bf16>(lo[1]);
    o[2] = static_cast<__bf16>(hi[0]);
    o[3] = static_cast<__bf16>(hi[1]);
    *reinterpret_cast<bf16x4 *>(dst + 4 * q) = o;
  }
}

// One workgroup per CU (the double-buffered tiles take most of the LDS): NW/4 waves per SIMD.
template <Prec P, int PP, bool GRAD, bool FP8>
__global__ __attribute__((amdgpu_flat_work_group_size(64, (Shape<P, PP>::NTHR))))
__attribute__((amdgpu_waves_per_eu((Shape<P, PP>::NW / 4), (Shape<P, PP>::NW / 4)))) void loglik_kernel(GemmArgs args) {
  using T = GT<P>;
  using LX = typename T::LX;
  using BT = typename T::BT;
  using FR = typename T::FR;
  using AC = typename T::AC;
  using EL = typename T::EL;
  using SH = Shape<P, PP>;
  using L = Lds<P, PP, GRAD>;
  using XG = typename std::conditional<FP8, uint8_t, LX>::type;   // genotype element in HBM
  constexpr int KS = T::KS, KV = T::KV, NT = SH::NT, PB = SH::PB, WGP = SH::WGP;
  constexpr int IB = NT / 16;    // 16-individual blocks per tile
  constexpr int QB = (P == Prec::BF16X2) ? 2 : 1;   // blocks per adjoint k-step
  constexpr int NKS = PP / KS;   // k-steps of the forward contraction
  constexpr int NMB = PP / 16;   // 16-marker blocks of the adjoint
  constexpr int CX = L::CX, CT = L::CT, CPR = L::CPR, CPT = L::CPT;
  constexpr int XSL = L::XSL, TSL = L::TSL, STG = L::STG;
  constexpr int NTHR = SH::NTHR;
  constexpr int NQX = XSL / NTHR, NQT = GRAD ? TSL / NTHR : 1;   // copy instructions per thread
  static_assert(P != Prec::BF16X2 || IB % 2 == 0, "BF16 adjoint k-step spans two blocks");
  static_assert(P == Prec::BF16X2 || IB == 1, "FP32/FP64 adjoint uses one block per tile");
  static_assert(!FP8 || P == Prec::BF16X2, "FP8 storage feeds the BF16 path");

  extern __shared__ __align__(16) uint4 smem[];   // STG 16-byte slots per stage

  // ---- workgroup -> (split, particle tile); XCD-aware (workgroups go round-robin to 8 XCDs)
  const int S = args.S;
  const int g8 = 8 / S;
  const int xcd = blockIdx.x & 7, slot = blockIdx.x >> 3;
  const int split = xcd / g8;
  const int ptile = slot * g8 + (xcd % g8);
  const int ntiles_p = (args.M + WGP - 1) / WGP;
  if (ptile >= ntiles_p) return;

  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int lr = lane & 15, lg = lane >> 4;
  const int wbase = ptile * WGP + wave * 16 * PB;
  const int n = args.n, n_pad = args.n_pad;
  const int chunk = ((n_pad + S - 1) / S + NT - 1) / NT * NT;
  const int i0 = min(n_pad, split * chunk);
  // tiles holding at least one real individual (n_pad may exceed n by more than a tile)
  const int i1 = min(min(n_pad, i0 + chunk), (n + NT - 1) / NT * NT);
  const int ntiles = max(0, (i1 - i0) / NT);

  // ---- coefficient fragments: register resident for the whole pass
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

  // ---- tile staging.  Slot q*NTHR + tid of a region is filled by this thread's q-th copy;
  // its source offset inside a tile does not depend on the tile and is computed once.
  // Padding slots copy the tile's first chunk (never read).
  int xoff[NQX], toff[NQT];
#pragma unroll
  for (int q = 0; q < NQX; ++q) {
    const int sl = q * NTHR + tid, r = sl / CX, c = sl % CX;
    xoff[q] = (r < NT && c < CPR) ? r * PP * (int)sizeof(XG) + c * 16 * (int)sizeof(XG) / (int)sizeof(LX) : 0;
  }
#pragma unroll
  for (int q = 0; q < NQT; ++q) {
    const int sl = q * NTHR + tid, r = sl / CT, c = sl % CT;
    toff[q] = (GRAD && r < PP && c < CPT) ? r * n_pad * (int)sizeof(XG) + c * 16 * (int)sizeof(XG) / (int)sizeof(LX) : 0;
  }
  const uint8_t *gxk = reinterpret_cast<const uint8_t *>(args.Xk);
  const uint8_t *gxt = reinterpret_cast<const uint8_t *>(args.Xt);

  // Asynchronous copy of one tile into a stage (global -> LDS DMA, 16 bytes per lane).
#define SPA_ISSUE(tile0_, stage_)                                                                        \
  do {                                                                                                   \
    const uint8_t *bx_ = gxk + (size_t)(tile0_) * PP * sizeof(XG);                                       \
    _Pragma("unroll") for (int q = 0; q < NQX; ++q)                                                      \
      lds_dma16(bx_ + xoff[q], smem + (stage_) * STG + q * NTHR + wave * 64);                           \
    if constexpr (GRAD) {                                                                                \
      const uint8_t *bt_ = gxt + (size_t)(tile0_) * sizeof(XG);                                          \
      _Pragma("unroll") for (int q = 0; q < NQT; ++q)                                                    \
        lds_dma16(bt_ + toff[q], smem + (stage_) * STG + XSL + q * NTHR + wave * 64);                   \
    }                                                                                                    \
  } while (0)
  // One of the NQX + NQT copy instructions of a tile (part < NQX: individual-major copy).
  auto issue_part = [&](const int tile0_, const int stage_, const int part) {
    if (part < NQX) {
      lds_dma16(gxk + (size_t)(tile0_) * PP * sizeof(XG) + xoff[part], smem + (stage_) * STG + part * NTHR + wave * 64);
    } else if constexpr (GRAD) {
      const int q = part - NQX;
      lds_dma16(gxt + (size_t)(tile0_) * sizeof(XG) + toff[q], smem + (stage_) * STG + XSL + q * NTHR + wave * 64);
    }
  };
  // FP8 storage: each 16-byte chunk of codes becomes two BF16 chunks, through registers.
#define SPA_COPY_FP8(tile0_, stage_)                                                                     \
  do {                                                                                                   \
    __bf16 *sx_ = reinterpret_cast<__bf16 *>(smem + (stage_) * STG);                                     \
    for (int c = tid; c < NT * PP / 16; c += NTHR) {                                                     \
      const int r = c / (PP / 16), cc = c % (PP / 16);                                                   \
      const uint4 v = *reinterpret_cast<const uint4 *>(gxk + (size_t)((tile0_) + r) * PP + cc * 16);     \
      store_fp8_as_bf16(sx_ + (r * CX + 2 * cc) * 8, v);                                                 \
    }                                                                                                    \
    if constexpr (GRAD) {                                                                                \
      __bf16 *st_ = reinterpret_cast<__bf16 *>(smem + (stage_) * STG + XSL);                             \
      for (int c = tid; c < PP * NT / 16; c += NTHR) {                                                   \
        const int r = c / (NT / 16), cc = c % (NT / 16);                                                 \
        const uint4 v = *reinterpret_cast<const uint4 *>(gxt + (size_t)r * n_pad + (tile0_) + cc * 16); \
        store_fp8_as_bf16(st_ + (r * CT + 2 * cc) * 8, v);                                               \
      }                                                                                                  \
    }                                                                                                    \
  } while (0)
  // FP8 storage, in two halves: the next tile's codes are loaded into registers at the
  // start of a tile (their latency hidden by the tile's MFMA work) and widened into the
  // idle stage at its end.
  constexpr int NFX = FP8 ? (NT * PP / 16 + NTHR - 1) / NTHR : 1;        // chunks per thread
  constexpr int NFT = (FP8 && GRAD) ? (PP * NT / 16 + NTHR - 1) / NTHR : 1;
  uint4 fx[NFX], ft[NFT];
  auto fp8_load = [&](const int tile0_) {
    if constexpr (FP8) {
#pragma unroll
      for (int u = 0; u < NFX; ++u) {
        const int c = tid + u * NTHR;
        if (c < NT * PP / 16) {
          const int r = c / (PP / 16), cc = c % (PP / 16);
          fx[u] = *reinterpret_cast<const uint4 *>(gxk + (size_t)(tile0_ + r) * PP + cc * 16);
        }
      }
      if constexpr (GRAD) {
#pragma unroll
        for (int u = 0; u < NFT; ++u) {
          const int c = tid + u * NTHR;
          if (c < PP * NT / 16) {
            const int r = c / (NT / 16), cc = c % (NT / 16);
            ft[u] = *reinterpret_cast<const uint4 *>(gxt + (size_t)r * n_pad + tile0_ + cc * 16);
          }
        }
      }
    }
  };
  auto fp8_store = [&](const int stage_) {
    if constexpr (FP8) {
      __bf16 *sx_ = reinterpret_cast<__bf16 *>(smem + (stage_) * STG);
#pragma unroll
      for (int u = 0; u < NFX; ++u) {
        const int c = tid + u * NTHR;
        if (c < NT * PP / 16) {
          const int r = c / (PP / 16), cc = c % (PP / 16);
          store_fp8_as_bf16(sx_ + (r * CX + 2 * cc) * 8, fx[u]);
        }
      }
      if constexpr (GRAD) {
        __bf16 *st_ = reinterpret_cast<__bf16 *>(smem + (stage_) * STG + XSL);
#pragma unroll
        for (int u = 0; u < NFT; ++u) {
          const int c = tid + u * NTHR;
          if (c < PP * NT / 16) {
            const int r = c / (NT / 16), cc = c % (NT / 16);
            store_fp8_as_bf16(st_ + (r * CT + 2 * cc) * 8, ft[u]);
          }
        }
      }
    }
  };
  // Wait for this thread's copies, then make every wave's copies visible.
#define SPA_LAND()                                  \
  do {                                              \
    asm volatile("s_waitcnt vmcnt(0)" ::: "memory"); \
    __syncthreads();                                \
  } while (0)

  if (ntiles > 0) {
    if constexpr (FP8) SPA_COPY_FP8(i0, 0);
    else SPA_ISSUE(i0, 0);
  }
  SPA_LAND();

  // One tile: forward -> elementwise -> adjoint per group of QB 16-individual blocks, while the
  // next tile's copy lands in the other stage.  MASKED: the tile holds padded individuals,
  // which happens only for the last tile holding real ones (peeled off the main loop, so the
  // main loop body is one straight block).
  auto tile_step = [&](const int it, auto masked_c) {
    constexpr bool MASKED = decltype(masked_c)::value;
    const int tile0 = i0 + it * NT;
    const int stage = it & 1;
    // the next tile's copy; unconditional: the last tile re-copies itself into the idle
    // stage (never read).  BF16: its instructions are spread over the first group's MFMA
    // loops (one per forward k-step, one per other adjoint block) rather than issued in
    // one burst, which stalls the wave's issue (measured: ~4 % of the kernel time).
    const int ntile0 = i0 + min(it + 1, ntiles - 1) * NT;
    if constexpr (FP8) {
      if (it + 1 < ntiles) fp8_load(ntile0);
    }
    constexpr bool SPREAD = (P == Prec::BF16X2) && !FP8 && (NKS >= NQX) && (NMB >= 2 * NQT);
    if constexpr (!FP8 && !SPREAD) SPA_ISSUE(ntile0, stage ^ 1);
    const uint4 *sX = smem + stage * STG;          // individual-major tile, row stride CX slots
    const uint4 *sXt = sX + XSL;                   // marker-major tile, row stride CT slots
    // ---- per group of QB 16-individual blocks: forward -> elementwise -> adjoint
#pragma unroll
    for (int q = 0; q < IB / QB; ++q) {
      // forward: eta^T blocks (individuals x particles)
      AC acc[QB][PB];
#pragma unroll
      for (int b = 0; b < QB; ++b)
#pragma unroll
        for (int pb = 0; pb < PB; ++pb) acc[b][pb] = AC{0, 0, 0, 0};
#pragma unroll
      for (int ks = 0; ks < NKS; ++ks) {
        if constexpr (SPREAD) {
          if (q == 0 && ks < NQX) issue_part(ntile0, stage ^ 1, ks);
        }
#pragma unroll
        for (int b = 0; b < QB; ++b) {
          const int ib = q * QB + b;
          const FR a = reinterpret_cast<const FR *>(sX + (ib * 16 + lr) * CX)[ks * KS / KV + lg];
#pragma unroll
          for (int pb = 0; pb < PB; ++pb) {
            acc[b][pb] = T::mfma(a, bh[pb][ks], acc[b][pb]);
            if constexpr (P == Prec::BF16X2) acc[b][pb] = T::mfma(a, bl[pb][ks], acc[b][pb]);
          }
        }
      }
      // Scheduling: keep D k-steps of fragment reads in flight ahead of their MFMAs (the
      // default schedule waits on every read right before its use).
      if constexpr (P == Prec::BF16X2) {
        constexpr int D = kPrefetch;
        __builtin_amdgcn_sched_group_barrier(0x100, QB * D, 0);
#pragma unroll
        for (int ks = 0; ks < NKS; ++ks) {
          __builtin_amdgcn_sched_group_barrier(0x008, QB * PB * 2, 0);
          if (ks + D < NKS) __builtin_amdgcn_sched_group_barrier(0x100, QB, 0);
        }
      }

      // elementwise (lane: particle lr of each block, individuals crow(lg, v) of each block).
      // Padded genotype rows, ones column included, are zero: only the softplus sum masks them.
      EL sig[GRAD ? QB : 1][PB][4];
#define SPA_ELEMENTWISE(MASKED)                                                                   \
  _Pragma("unroll") for (int pb = 0; pb < PB; ++pb) {                                             \
    if constexpr (P == Prec::F64) {                                                               \
      double sp = 0.0;                                                                            \
      _Pragma("unroll") for (int b = 0; b < QB; ++b) _Pragma("unroll") for (int v = 0; v < 4; ++v) { \
        const double eta = acc[b][pb][v] - moff[pb];                                              \
        const double e = exp(-fabs(eta));                                                         \
        const bool valid = !(MASKED) || (tile0 + (q * QB + b) * 16 + T::crow(lg, v)) < n;         \
        sp += valid ? fmax(eta, 0.0) + log1p(e) : 0.0;                                            \
        if constexpr (GRAD) sig[b][pb][v] = eta >= 0.0 ? 1.0 / (1.0 + e) : e / (1.0 + e);         \
      }                                                                                           \
      spl[pb] += sp;                                                                              \
    } else {                                                                                      \
      /* reduced precision: the operand carries log2(e), so z = eta log2(e); the genotypes  */    \
      /* are centred, so sum_k eta_ik = 0 over the real individuals and sum_k max(z, 0) is  */    \
      /* half of sum_k |z| (one add with an abs modifier per element instead of two ops)   */     \
      float prod = 1.0f, mx = 0.0f;                                                               \
      _Pragma("unroll") for (int b = 0; b < QB; ++b) _Pragma("unroll") for (int v = 0; v < 4; ++v) { \
        const float z = acc[b][pb][v] - moff[pb];                                                 \
        const float e = fast_exp2(-fabsf(z));                                                     \
        if (!(MASKED) || (tile0 + (q * QB + b) * 16 + T::crow(lg, v)) < n) {                      \
          prod = fmaf(prod, e, prod);                                                             \
          mx += fabsf(z);                                                                         \
        }                                                                                         \
        if constexpr (GRAD) {                                                                     \
          const float rc = fast_rcp(1.0f + e);                                                    \
          sig[b][pb][v] = z >= 0.0f ? rc : e * rc;                                                \
        }                                                                                         \
      }                                                                                           \
      spl[pb] += static_cast<double>(0.6931471805599453f * (0.5f * mx + fast_log2(prod)));       \
    }                                                                                             \
  }
      SPA_ELEMENTWISE(MASKED)
#undef SPA_ELEMENTWISE

      // adjoint: G^T (markers x particles) += X_tile^T . sigma^T
      if constexpr (GRAD) {
        if constexpr (P == Prec::BF16X2) {
          // K slot j of lane group lg: individual 4lg + j of block 2q (j < 4), of block 2q+1 (j >= 4)
          bf16x8 rh[PB], rl[PB];
#pragma unroll
          for (int pb = 0; pb < PB; ++pb)
#pragma unroll
            for (int j = 0; j < 8; j += 2) {
              const f32x2 v = {sig[j >> 2][pb][j & 3], sig[j >> 2][pb][(j & 3) + 1]};
              const bf16x2 h = __builtin_convertvector(v, bf16x2);
              const f32x2 r = v - __builtin_convertvector(h, f32x2);
              const bf16x2 l = __builtin_convertvector(r, bf16x2);
              rh[pb][j] = h[0];
              rh[pb][j + 1] = h[1];
              rl[pb][j] = l[0];
              rl[pb][j + 1] = l[1];
            }
#pragma unroll
          for (int mb = 0; mb < NMB; ++mb) {
            if constexpr (SPREAD) {
              if (q == 0 && (mb & 1) == 0 && mb / 2 < NQT) issue_part(ntile0, stage ^ 1, NQX + mb / 2);
            }
            // the marker-major copy holds this lane group's 8 K slots contiguously
            const bf16x8 a = *reinterpret_cast<const bf16x8 *>(sXt + (mb * 16 + lr) * CT + q * 4 + lg);
#pragma unroll
            for (int pb = 0; pb < PB; ++pb) {
              G[pb][mb] = T::mfma(a, rh[pb], G[pb][mb]);
              G[pb][mb] = T::mfma(a, rl[pb], G[pb][mb]);
            }
          }
          {
            constexpr int D = kPrefetch;
            __builtin_amdgcn_sched_group_barrier(0x100, D, 1);
#pragma unroll
            for (int mb = 0; mb < NMB; ++mb) {
              __builtin_amdgcn_sched_group_barrier(0x008, PB * 2, 1);
              if (mb + D < NMB) __builtin_amdgcn_sched_group_barrier(0x100, 1, 1);
            }
          }
        } else {
          // 16x16x4: k-step v feeds the lane's v-th row, individual crow(lg, v)
#pragma unroll
          for (int mb = 0; mb < NMB; ++mb) {
            // the marker-major copy holds individuals crow(lg, 0..3) at positions 4lg..4lg+3
            const LX *row = reinterpret_cast<const LX *>(sXt + (mb * 16 + lr) * CT);
#pragma unroll
            for (int v = 0; v < 4; ++v) {
              const LX a = row[4 * lg + v];
#pragma unroll
              for (int pb = 0; pb < PB; ++pb) G[pb][mb] = T::mfma(a, sig[0][pb][v], G[pb][mb]);
            }
          }
        }
      }
    }

    if constexpr (FP8) {
      if (it + 1 < ntiles) fp8_store(stage ^ 1);
    }
    SPA_LAND();
  };
  const bool has_tail = ntiles > 0 && i0 + ntiles * NT > n;
  const int nfull = ntiles - (has_tail ? 1 : 0);
  for (int it = 0; it < nfull; ++it) tile_step(it, std::false_type{});
  if (has_tail) tile_step(nfull, std::true_type{});
#undef SPA_ISSUE
#undef SPA_COPY_FP8
#undef SPA_LAND


  // ---- softplus sums over the 4 lane groups sharing a particle
#pragma unroll
  for (int pb = 0; pb < PB; ++pb) {
    spl[pb] += __shfl_xor(spl[pb], 16, 64);
    spl[pb] += __shfl_xor(spl[pb], 32, 64);
  }

  const int M = args.M, p = args.p;
  using GO = typename std::conditional<P == Prec::F64, double, float>::type;
  if (S == 1) {
    // ---- epilogue: log-likelihood and standardised gradient
#pragma unroll
    for (int pb = 0; pb < PB; ++pb) {
      const int i = wbase + pb * 16 + lr;
      if (lg == 0 && i < M) args.ll[i] = args.yb[i] - spl[pb];
      if constexpr (GRAD) {
        // rho_i = sum_k sigma_ik: the all-ones column PP-1 (block NMB-1, lane group 3, element 3)
        const double rho = static_cast<double>(__shfl(G[pb][NMB - 1][3], lr + 48, 64));
        if (i < M) {
          GO *g = reinterpret_cast<GO *>(args.g) + static_cast<size_t>(i) * p;
#pragma unroll
          for (int mb = 0; mb < NMB; ++mb)
#pragma unroll
            for (int v = 0; v < 4; ++v) {
              const int j = mb * 16 + T::crow(lg, v);
              if (j < p)
                g[j] = static_cast<GO>(args.ytil[j] -
                                       (static_cast<double>(G[pb][mb][v]) - args.mu[j] * rho) * args.inv_s[j]);
            }
        }
      }
    }
  } else {
    // ---- partial sums of this split (combined in split order by the finalize kernel)
    const size_t Mp = static_cast<size_t>(args.M_pad);
#pragma unroll
    for (int pb = 0; pb < PB; ++pb) {
      const int i = wbase + pb * 16 + lr;
      if (lg == 0) args.spl_part[split * Mp + i] = spl[pb];
      if constexpr (GRAD) {
        GO *gp = reinterpret_cast<GO *>(args.g_part) + (split * Mp + i) * PP;
#pragma unroll
        for (int mb = 0; mb < NMB; ++mb) {
          if constexpr (P == Prec::F64) {
#pragma unroll
            for (int v = 0; v < 4; ++v) gp[mb * 16 + T::crow(lg, v)] = G[pb][mb][v];
          } else {
            *reinterpret_cast<f32x4 *>(gp + mb * 16 + lg * 4) = G[pb][mb];
          }
        }
      }
    }
  }
}

// Split-marker form of the BF16 hi+lo contraction with the adjoint, for rows of 384 or 512
// markers.  There one wave's coefficient fragments (hi and lo, 8 k-steps of 32 markers per
// 256) and adjoint accumulators (16 blocks of 16 markers per 256) would take all of a
// SIMD's registers; here the two waves w and w+4 of a SIMD share a block of 16 particles
// and each holds one half of the markers: it computes the forward partial sums of its half,
// the two halves are added through LDS (float addition commutes, so both waves hold the
// same eta), both evaluate the same elementwise step, and each accumulates the adjoint of
// its half.  Two waves per SIMD (8 per workgroup, 64 particles).  Tiles of 32 individuals
// are staged through registers (the next tile's 16-byte chunks are loaded during a tile and
// written, FP8 codes widened to BF16, into the single LDS stage between two barriers),
// which leaves room in LDS for the exchange.  The same arithmetic per element as
// loglik_kernel; a forward sum is formed as the sum of two half sums.  (Splitting the
// elementwise step between the two waves, with a second exchange of the logistic values,
// was measured slower: one more barrier per tile costs more than half the vector work.)
template <int PP, bool FP8>
__global__ __attribute__((amdgpu_flat_work_group_size(64, 512))) __attribute__((amdgpu_waves_per_eu(2, 2)))
void loglik_wide_kernel(GemmArgs args) {
  constexpr Prec P = Prec::BF16X2;
  using T = GT<P>;
  using FR = bf16x8;
  using AC = f32x4;
  using LX = __bf16;
  using XG = typename std::conditional<FP8, uint8_t, LX>::type;
  constexpr int KS = 32, KV = 8, NT = 32, NTHR = 512, WGP = 64;
  constexpr int H = PP / 2;                      // markers per half
  constexpr int NKH = H / KS, NMH = H / 16;      // forward k-steps, adjoint blocks per half
  constexpr int CPR = PP * 2 / 16, CX = CPR + 1;  // individual-major rows (BF16 chunks)
  constexpr int CPT = NT * 2 / 16, CT = CPT + 1;  // marker-major rows
  constexpr int XS = NT * CX, TS = PP * CT;       // slots of the two regions
  // staged 16-byte chunks of the source (FP8: 16 codes; BF16: 8 values)
  constexpr int EPC = 16 / (int)sizeof(XG);      // elements per staged chunk
  constexpr int NCX = NT * PP / EPC, NCT = PP * NT / EPC;
  constexpr int RX = (NCX + NTHR - 1) / NTHR, RT = (NCT + NTHR - 1) / NTHR;
  static_assert(PP == 384 || PP == 512, "rows of 384 or 512 markers");

  extern __shared__ __align__(16) uint4 smem[];   // XS + TS slots, then the exchange
  float *xbuf = reinterpret_cast<float *>(smem + XS + TS);   // 8 waves x 64 lanes x 8 floats

  const int S = args.S;
  const int g8 = 8 / S;
  const int xcd = blockIdx.x & 7, slot = blockIdx.x >> 3;
  const int split = xcd / g8;
  const int ptile = slot * g8 + (xcd % g8);
  const int ntiles_p = (args.M + WGP - 1) / WGP;
  if (ptile >= ntiles_p) return;

  const int tid = threadIdx.x, lane = tid & 63;
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int lr = lane & 15, lg = lane >> 4;
  const int half = wave >> 2, pblk = wave & 3;
  const int wbase = ptile * WGP + pblk * 16;
  const int n = args.n, n_pad = args.n_pad;
  const int chunk = ((n_pad + S - 1) / S + NT - 1) / NT * NT;
  const int i0 = min(n_pad, split * chunk);
  const int i1 = min(min(n_pad, i0 + chunk), (n + NT - 1) / NT * NT);
  const int ntiles = max(0, (i1 - i0) / NT);
  const int tmask = (ntiles > 0 && i0 + ntiles * NT > n) ? ntiles - 1 : ntiles;   // tile with padding

  FR bh[NKH], bl[NKH];
  float moff;
  {
    const size_t row = static_cast<size_t>(wbase + lr);
    const __bf16 *sh = reinterpret_cast<const __bf16 *>(args.Bhi) + row * PP + half * H + lg * KV;
    const __bf16 *sl = reinterpret_cast<const __bf16 *>(args.Blo) + row * PP + half * H + lg * KV;
#pragma unroll
    for (int ks = 0; ks < NKH; ++ks) {
      bh[ks] = *reinterpret_cast<const FR *>(sh + ks * KS);
      bl[ks] = *reinterpret_cast<const FR *>(sl + ks * KS);
    }
    moff = static_cast<float>(args.moff[row]);
  }
  AC G[NMH];
#pragma unroll
  for (int mb = 0; mb < NMH; ++mb) G[mb] = AC{0, 0, 0, 0};
  double spl = 0.0;

  const uint8_t *gxk = reinterpret_cast<const uint8_t *>(args.Xk);
  const uint8_t *gxt = reinterpret_cast<const uint8_t *>(args.Xt);
  uint4 sx[RX], st[RT];
  auto load_tile = [&](const int tile0) {   // the tile's chunks into registers
#pragma unroll
    for (int u = 0; u < RX; ++u) {
      const int c = tid + u * NTHR;
      if (c < NCX) {
        const int r = c / (PP / EPC), cc = c % (PP / EPC);
        sx[u] = *reinterpret_cast<const uint4 *>(gxk + ((size_t)(tile0 + r) * PP + cc * EPC) * sizeof(XG));
      }
    }
#pragma unroll
    for (int u = 0; u < RT; ++u) {
      const int c = tid + u * NTHR;
      if (c < NCT) {
        const int r = c / (NT / EPC), cc = c % (NT / EPC);
        st[u] = *reinterpret_cast<const uint4 *>(gxt + ((size_t)r * n_pad + tile0 + cc * EPC) * sizeof(XG));
      }
    }
  };
  auto store_tile = [&]() {   // registers -> the LDS stage (FP8 widened to BF16)
#pragma unroll
    for (int u = 0; u < RX; ++u) {
      const int c = tid + u * NTHR;
      if (c < NCX) {
        const int r = c / (PP / EPC), cc = c % (PP / EPC);
        if constexpr (FP8) store_fp8_as_bf16(reinterpret_cast<__bf16 *>(smem + r * CX + 2 * cc), sx[u]);
        else smem[r * CX + cc] = sx[u];
      }
    }
#pragma unroll
    for (int u = 0; u < RT; ++u) {
      const int c = tid + u * NTHR;
      if (c < NCT) {
        const int r = c / (NT / EPC), cc = c % (NT / EPC);
        if constexpr (FP8) store_fp8_as_bf16(reinterpret_cast<__bf16 *>(smem + XS + r * CT + 2 * cc), st[u]);
        else smem[XS + r * CT + cc] = st[u];
      }
    }
  };

  if (ntiles > 0) load_tile(i0);
  for (int it = 0; it < ntiles; ++it) {
    const int tile0 = i0 + it * NT;
    __syncthreads();                             // every wave is done with the previous tile
    store_tile();
    __syncthreads();                             // this tile is in LDS
    if (it + 1 < ntiles) load_tile(tile0 + NT);  // the next tile in flight during this one
    const uint4 *sX = smem, *sXt = smem + XS;
    // forward partial sums of this half: eta^T blocks of the tile's two 16-individual blocks
    AC acc[2] = {AC{0, 0, 0, 0}, AC{0, 0, 0, 0}};
#pragma unroll
    for (int ks = 0; ks < NKH; ++ks) {
#pragma unroll
      for (int b = 0; b < 2; ++b) {
        const FR a = reinterpret_cast<const FR *>(sX + (b * 16 + lr) * CX)[(half * NKH + ks) * KS / KV + lg];
        acc[b] = T::mfma(a, bh[ks], acc[b]);
        acc[b] = T::mfma(a, bl[ks], acc[b]);
      }
    }
    {
      constexpr int D = kPrefetch;
      __builtin_amdgcn_sched_group_barrier(0x100, 2 * D, 0);
#pragma unroll
      for (int ks = 0; ks < NKH; ++ks) {
        __builtin_amdgcn_sched_group_barrier(0x008, 4, 0);
        if (ks + D < NKH) __builtin_amdgcn_sched_group_barrier(0x100, 2, 0);
      }
    }
    // exchange the half sums with the other wave of the particle block
    float *mine = xbuf + ((size_t)wave * 64 + lane) * 8;
    const float *other = xbuf + ((size_t)(wave ^ 4) * 64 + lane) * 8;
#pragma unroll
    for (int b = 0; b < 2; ++b) *reinterpret_cast<AC *>(mine + 4 * b) = acc[b];
    __syncthreads();
#pragma unroll
    for (int b = 0; b < 2; ++b) acc[b] += *reinterpret_cast<const AC *>(other + 4 * b);
    // elementwise (the same in both waves of the pair)
    float prod = 1.0f, mx = 0.0f, sig[2][4];
    const bool masked = it == tmask;
#pragma unroll
    for (int b = 0; b < 2; ++b)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const float z = acc[b][v] - moff;
        const float e = fast_exp2(-fabsf(z));
        if (!masked || (tile0 + b * 16 + T::crow(lg, v)) < n) {
          prod = fmaf(prod, e, prod);
          mx += fabsf(z);
        }
        const float rc = fast_rcp(1.0f + e);
        sig[b][v] = z >= 0.0f ? rc : e * rc;
      }
    spl += static_cast<double>(0.6931471805599453f * (0.5f * mx + fast_log2(prod)));
    bf16x8 rh, rl;
#pragma unroll
    for (int j = 0; j < 8; j += 2) {
      const f32x2 v = {sig[j >> 2][j & 3], sig[j >> 2][(j & 3) + 1]};
      const bf16x2 h = __builtin_convertvector(v, bf16x2);
      const f32x2 r = v - __builtin_convertvector(h, f32x2);
      const bf16x2 l = __builtin_convertvector(r, bf16x2);
      rh[j] = h[0];
      rh[j + 1] = h[1];
      rl[j] = l[0];
      rl[j + 1] = l[1];
    }
    // adjoint of this half: G^T (markers x particles) += X_tile^T . sigma^T
#pragma unroll
    for (int mb = 0; mb < NMH; ++mb) {
      const bf16x8 a = *reinterpret_cast<const bf16x8 *>(sXt + ((half * NMH + mb) * 16 + lr) * CT + lg);
      G[mb] = T::mfma(a, rh, G[mb]);
      G[mb] = T::mfma(a, rl, G[mb]);
    }
    {
      constexpr int D = kPrefetch;
      __builtin_amdgcn_sched_group_barrier(0x100, D, 1);
#pragma unroll
      for (int mb = 0; mb < NMH; ++mb) {
        __builtin_amdgcn_sched_group_barrier(0x008, 2, 1);
        if (mb + D < NMH) __builtin_amdgcn_sched_group_barrier(0x100, 1, 1);
      }
    }
  }

  spl += __shfl_xor(spl, 16, 64);
  spl += __shfl_xor(spl, 32, 64);
  const int M = args.M, p = args.p;
  const int i = wbase + lr;
  if (S == 1) {
    // rho_i = sum_k sigma_ik sits in the all-ones column PP-1 of the upper half
    __syncthreads();
    if (half == 1) xbuf[(size_t)pblk * 64 + lr] = __shfl(G[NMH - 1][3], lr + 48, 64);
    __syncthreads();
    const double rho = static_cast<double>(xbuf[(size_t)pblk * 64 + lr]);
    if (half == 0 && lg == 0 && i < M) args.ll[i] = args.yb[i] - spl;
    if (i < M) {
      float *g = reinterpret_cast<float *>(args.g) + static_cast<size_t>(i) * p;
#pragma unroll
      for (int mb = 0; mb < NMH; ++mb)
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          const int j = (half * NMH + mb) * 16 + T::crow(lg, v);
          if (j < p)
            g[j] = static_cast<float>(args.ytil[j] - (static_cast<double>(G[mb][v]) - args.mu[j] * rho) * args.inv_s[j]);
        }
    }
  } else {
    const size_t Mp = static_cast<size_t>(args.M_pad);
    if (half == 0 && lg == 0) args.spl_part[split * Mp + i] = spl;
    float *gp = reinterpret_cast<float *>(args.g_part) + (split * Mp + i) * PP + half * H;
#pragma unroll
    for (int mb = 0; mb < NMH; ++mb) *reinterpret_cast<f32x4 *>(gp + mb * 16 + lg * 4) = G[mb];
  }
}

// Sum the S partials of every particle in split order and apply the epilogue.
template <typename GO, bool GRAD>
__global__ void gemm_finalize_kernel(GemmArgs args, int PP) {
  const int lane = threadIdx.x & 63;
  const int i = blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6);
  if (i >= args.M) return;
  const size_t Mp = static_cast<size_t>(args.M_pad);
  const int S = args.S, p = args.p;
  if (lane == 0) {
    double spl = 0.0;
    for (int s = 0; s < S; ++s) spl += args.spl_part[s * Mp + i];
    args.ll[i] = args.yb[i] - spl;
  }
  if constexpr (GRAD) {
    const GO *gp = reinterpret_cast<const GO *>(args.g_part);
    double rho = 0.0;
    for (int s = 0; s < S; ++s) rho += static_cast<double>(gp[(s * Mp + i) * PP + PP - 1]);
    GO *g = reinterpret_cast<GO *>(args.g) + static_cast<size_t>(i) * p;
    for (int j = lane; j < p; j += 64) {
      double acc = 0.0;
      for (int s = 0; s < S; ++s) acc += static_cast<double>(gp[(s * Mp + i) * PP + j]);
      g[j] = static_cast<GO>(args.ytil[j] - (acc - args.mu[j] * rho) * args.inv_s[j]);
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

int gemm_tile_individuals(Prec prec, int PP) {
  return prec == Prec::BF16X2 ? (PP <= 256 ? 64 : 32) : 16;
}

int gemm_particles_per_wg(Prec prec, int PP) {
  return prec == Prec::F64 ? 64 : (PP <= 256 ? 128 : 64);
}

int gemm_splits(Prec prec, int PP, int n_pad, int M, size_t x_bytes_both) {
  const int NT = gemm_tile_individuals(prec, PP);
  const int tiles_p = (M + gemm_particles_per_wg(prec, PP) - 1) / gemm_particles_per_wg(prec, PP);
  int S = 1;
  // keep one split's genotype slice (both orientations) within an XCD's L2 ...
  while (S < 8 && x_bytes_both / S > (size_t)3 * 1024 * 1024 && n_pad / (2 * S) >= NT) S *= 2;
  // ... and give every CU a workgroup
  while (S < 8 && (size_t)tiles_p * S < 256 && n_pad / (2 * S) >= NT) S *= 2;
  return S;
}

template <Prec P, int PP, bool GRAD, bool FP8>
static hipError_t launch_one(const GemmArgs &a, hipStream_t s) {
  constexpr size_t lds = Lds<P, PP, GRAD>::bytes;
  static_assert(lds <= 160 * 1024, "LDS budget of one CU");
  auto kern = loglik_kernel<P, PP, GRAD, FP8>;
  static bool attr_set = false;
  if (!attr_set) {
    hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void *>(kern),
                                       hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess) return e;
    attr_set = true;
  }
  constexpr int per_wg = Shape<P, PP>::WGP;
  const int tiles_p = (a.M + per_wg - 1) / per_wg;
  const int g8 = 8 / a.S;
  const int grid = 8 * ((tiles_p + g8 - 1) / g8);
  hipLaunchKernelGGL(kern, dim3(grid), dim3(Shape<P, PP>::NTHR), lds, s, a);
  return hipGetLastError();
}

template <int PP, bool FP8>
static hipError_t launch_wide(const GemmArgs &a, hipStream_t s) {
  constexpr int XS = 32 * (PP * 2 / 16 + 1), TS = PP * (32 * 2 / 16 + 1);
  constexpr size_t lds = (size_t)(XS + TS) * 16 + 8 * 64 * 8 * sizeof(float);
  static_assert(lds <= 160 * 1024, "LDS budget of one CU");
  auto kern = loglik_wide_kernel<PP, FP8>;
  static bool attr_set = false;
  if (!attr_set) {
    hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void *>(kern),
                                       hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess) return e;
    attr_set = true;
  }
  const int tiles_p = (a.M + 63) / 64;
  const int g8 = 8 / a.S;
  const int grid = 8 * ((tiles_p + g8 - 1) / g8);
  hipLaunchKernelGGL(kern, dim3(grid), dim3(512), lds, s, a);
  return hipGetLastError();
}

template <Prec P, int PP>
static hipError_t launch_pp(const GemmArgs &a, hipStream_t s) {
  if constexpr (P == Prec::BF16X2 && (PP == 384 || PP == 512)) {
    if (a.grad) return a.x_fp8 ? launch_wide<PP, true>(a, s) : launch_wide<PP, false>(a, s);
  }
  if constexpr (P == Prec::BF16X2) {
    if (a.x_fp8) {
      if (a.grad) return launch_one<P, PP, true, true>(a, s);
      return launch_one<P, PP, false, true>(a, s);
    }
  }
  if (a.grad) return launch_one<P, PP, true, false>(a, s);
  return launch_one<P, PP, false, false>(a, s);
}

hipError_t launch_gemm_finalize(const GemmArgs &a, hipStream_t s) {
  if (a.S == 1) return hipSuccess;
  const int grid = (a.M + 3) / 4;
  if (a.prec == Prec::F64) {
    if (a.grad) hipLaunchKernelGGL((gemm_finalize_kernel<double, true>), dim3(grid), dim3(256), 0, s, a, a.PP);
    else hipLaunchKernelGGL((gemm_finalize_kernel<double, false>), dim3(grid), dim3(256), 0, s, a, a.PP);
  } else {
    if (a.grad) hipLaunchKernelGGL((gemm_finalize_kernel<float, true>), dim3(grid), dim3(256), 0, s, a, a.PP);
    else hipLaunchKernelGGL((gemm_finalize_kernel<float, false>), dim3(grid), dim3(256), 0, s, a, a.PP);
  }
  return hipGetLastError();
}

hipError_t launch_loglik(const GemmArgs &a, hipStream_t s) {
  if (a.S != 1 && a.S != 2 && a.S != 4 && a.S != 8) return hipErrorInvalidValue;
  if (a.M_pad % gemm_particles_per_wg(a.prec, a.PP) != 0) return hipErrorInvalidValue;
  switch (a.prec) {
    case Prec::BF16X2:
      switch (a.PP) {
        case 32: return launch_pp<Prec::BF16X2, 32>(a, s);
        case 64: return launch_pp<Prec::BF16X2, 64>(a, s);
        case 128: return launch_pp<Prec::BF16X2, 128>(a, s);
        case 224: return launch_pp<Prec::BF16X2, 224>(a, s);
        case 256: return launch_pp<Prec::BF16X2, 256>(a, s);
        case 384: return launch_pp<Prec::BF16X2, 384>(a, s);
        case 512: return launch_pp<Prec::BF16X2, 512>(a, s);
      }
      break;
    case Prec::F32:
      switch (a.PP) {
        case 32: return launch_pp<Prec::F32, 32>(a, s);
        case 64: return launch_pp<Prec::F32, 64>(a, s);
        case 128: return launch_pp<Prec::F32, 128>(a, s);
        case 224: return launch_pp<Prec::F32, 224>(a, s);
        case 256: return launch_pp<Prec::F32, 256>(a, s);
        case 384: return launch_pp<Prec::F32, 384>(a, s);
        case 512: return launch_pp<Prec::F32, 512>(a, s);
      }
      break;
    case Prec::F64:
      switch (a.PP) {
        case 32: return launch_pp<Prec::F64, 32>(a, s);
        case 64: return launch_pp<Prec::F64, 64>(a, s);
        case 128: return launch_pp<Prec::F64, 128>(a, s);
        case 224: return launch_pp<Prec::F64, 224>(a, s);
        case 256: return launch_pp<Prec::F64, 256>(a, s);
      }
      break;
  }
  return hipErrorInvalidValue;
}

}  // namespace spa
