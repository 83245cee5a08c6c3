// Bandwidth-bound kernels of the sampler: operand preparation, proposals, MH decisions,
// incremental weights, logsumexp/ESS and systematic resampling, gathers and weighted
// moments.  Row kernels map one wave64 to one particle (its p coefficients are contiguous,
// so a wave reads a row with 16-byte lanes); reductions use fixed butterfly/tree orders.
#include "spa_common.hpp"
#include "spa_lanes.hpp"
#include "spa_kernels.hpp"

namespace spa {

// ============================================================== operand preparation

// Per-marker integer sums give exact mean, population variance and X_std^T y numerators:
//   mu = S1/n, var = (n S2 - S1^2)/n^2, ytil = (n SY - S1 NY)/(n s).
__global__ void col_stats_kernel(const uint8_t *__restrict__ X, const uint8_t *__restrict__ y,
                                 int n, int p, double *mu, double *s, double *inv_s,
                                 double *ytil, int *bad) {
  const int j = blockIdx.x;
  long long s1 = 0, s2 = 0, sy = 0, ny = 0;
  for (int k = threadIdx.x; k < n; k += blockDim.x) {
    const long long v = X[(size_t)k * p + j];
    const long long yk = y[k];
    s1 += v;
    s2 += v * v;
    sy += v * yk;
    ny += yk;
  }
  __shared__ long long red[4][4];
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) {
    s1 += __shfl_xor(s1, o, 64);
    s2 += __shfl_xor(s2, o, 64);
    sy += __shfl_xor(sy, o, 64);
    ny += __shfl_xor(ny, o, 64);
  }
  if (lane == 0) {
    red[w][0] = s1;
    red[w][1] = s2;
    red[w][2] = sy;
    red[w][3] = ny;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    s1 = red[0][0];
    s2 = red[0][1];
    sy = red[0][2];
    ny = red[0][3];
    for (int q = 1; q < (int)(blockDim.x >> 6); ++q) {
      s1 += red[q][0];
      s2 += red[q][1];
      sy += red[q][2];
      ny += red[q][3];
    }
    const double dn = static_cast<double>(n);
    const long long num = (long long)n * s2 - s1 * s1;
    const double var = static_cast<double>(num) / (dn * dn);
    const double sd = sqrt(var);
    mu[j] = static_cast<double>(s1) / dn;
    s[j] = sd;
    inv_s[j] = num > 0 ? 1.0 / sd : 0.0;
    ytil[j] = num > 0 ? static_cast<double>((long long)n * sy - s1 * ny) / (dn * sd) : 0.0;
    if (num <= 0) bad[0] = 1;
  }
}

template <typename XT>
__device__ __forceinline__ XT code_of(int v);
template <>
__device__ __forceinline__ double code_of<double>(int v) { return static_cast<double>(v); }
template <>
__device__ __forceinline__ float code_of<float>(int v) { return static_cast<float>(v); }
template <>
__device__ __forceinline__ __bf16 code_of<__bf16>(int v) { return static_cast<__bf16>(static_cast<float>(v)); }
template <>
__device__ __forceinline__ uint8_t code_of<uint8_t>(int v) {   // OCP e4m3: 0, 1.0, 2.0
  return v == 0 ? 0x00 : (v == 1 ? 0x38 : 0x40);
}

// Genotypes in GEMM storage: Xk (n_pad x PP, individual-major) and Xt (PP x n_pad), with
// an all-ones column at PP-1 for real individuals and zeros elsewhere in the padding.
// Within each group of xt_group(prec) individuals, Xt holds individual i at xt_position.
template <typename XT>
__global__ void pack_x_kernel(const uint8_t *__restrict__ X, int n, int p, int n_pad, int PP, Prec prec,
                              XT *__restrict__ Xk, XT *__restrict__ Xt) {
  const int grp = xt_group(prec);
  const size_t total = (size_t)n_pad * PP;
  for (size_t idx = blockIdx.x * (size_t)blockDim.x + threadIdx.x; idx < total;
       idx += (size_t)gridDim.x * blockDim.x) {
    const int k = static_cast<int>(idx / PP), j = static_cast<int>(idx % PP);
    int v = 0;
    if (k < n) v = (j < p) ? X[(size_t)k * p + j] : (j == PP - 1 ? 1 : 0);
    const XT c = code_of<XT>(v);
    Xk[idx] = c;
    Xt[(size_t)j * n_pad + (k / grp) * grp + xt_position(prec, k % grp)] = c;
  }
}

template <typename ET>
__global__ void labels_kernel(const uint8_t *__restrict__ y, int n, int n_pad, ET *__restrict__ yv) {
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k < n_pad) yv[k] = (k < n) ? static_cast<ET>(y[k]) : ET(0);
}

// ------------------------------------------------- scaled-coefficient operand b = beta/s
// Writes one coefficient of the B operand of the contraction, scaled by operand_scale(P),
// and returns in `used` the value the operand actually represents (in the scaled units).
template <Prec P>
struct BPack;

template <>
struct BPack<Prec::BF16X2> {
  using BT = __bf16;
  static constexpr double scale = kLog2e;
  __device__ static void put(double bj, BT *hi, BT *lo, size_t off, double &used) {
    const float f = static_cast<float>(bj * scale);
    const __bf16 h = static_cast<__bf16>(f);
    const __bf16 l = static_cast<__bf16>(f - static_cast<float>(h));
    hi[off] = h;
    lo[off] = l;
    used = static_cast<double>(static_cast<float>(h)) + static_cast<double>(static_cast<float>(l));
  }
};
template <>
struct BPack<Prec::F32> {
  using BT = float;
  static constexpr double scale = kLog2e;
  __device__ static void put(double bj, BT *hi, BT *, size_t off, double &used) {
    const float f = static_cast<float>(bj * scale);
    hi[off] = f;
    used = static_cast<double>(f);
  }
};
template <>
struct BPack<Prec::F64> {
  using BT = double;
  static constexpr double scale = 1.0;
  __device__ static void put(double bj, BT *hi, BT *, size_t off, double &used) {
    hi[off] = bj;
    used = bj;
  }
};

// Store four consecutive B-operand entries (PP is a multiple of 32, so the block is aligned).
template <Prec P, typename BT>
__device__ __forceinline__ void store4_b(BT *hi, BT *lo, size_t off, const BT h[4], const BT l[4]) {
  if constexpr (P == Prec::BF16X2) {
    typedef __bf16 bf16x4_t __attribute__((ext_vector_type(4)));
    *reinterpret_cast<bf16x4_t *>(hi + off) = bf16x4_t{h[0], h[1], h[2], h[3]};
    *reinterpret_cast<bf16x4_t *>(lo + off) = bf16x4_t{l[0], l[1], l[2], l[3]};
  } else if constexpr (P == Prec::F32) {
    *reinterpret_cast<float4 *>(hi + off) = make_float4(h[0], h[1], h[2], h[3]);
  } else {
    *reinterpret_cast<f64x4 *>(hi + off) = f64x4{h[0], h[1], h[2], h[3]};
  }
}

struct ColConst {
  const double *mu, *s, *inv_s, *ytil;   // PP-padded
};

// Pack an arbitrary particle matrix (dtype IT) into the B operand of precision P.
template <Prec P, typename IT>
__global__ void pack_b_kernel(const IT *__restrict__ beta, int M, int M_pad, int p, int PP,
                              ColConst cc, void *Bhi_, void *Blo_, double *__restrict__ moff,
                              double *__restrict__ yb) {
  using BT = typename BPack<P>::BT;
  BT *Bhi = reinterpret_cast<BT *>(Bhi_);
  BT *Blo = reinterpret_cast<BT *>(Blo_);
  const int lane = threadIdx.x & 63;
  const int i = blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6);
  if (i >= M_pad) return;
  double m = 0.0, ybv = 0.0;
  for (int j = lane; j < PP; j += 64) {
    const double bj = (i < M && j < p) ? static_cast<double>(beta[(size_t)i * p + j]) * cc.inv_s[j] : 0.0;
    double used;
    BPack<P>::put(bj, Bhi, Blo, (size_t)i * PP + j, used);
    m += cc.mu[j] * used;
    ybv += cc.ytil[j] * cc.s[j] * used;
  }
  m = wave_sum(m);
  ybv = wave_sum(ybv);
  if (lane == 0) {
    moff[i] = m;
    yb[i] = ybv / BPack<P>::scale;
  }
}

// ================================================================ move kernels

// Standard normals for a Philox block: Box-Muller in the particle precision.  The FP32 form
// uses the hardware transcendentals (v_sin/v_cos take the angle in revolutions, which is
// exactly w * 2^-32 here); the FP64 form is the libm one.
__device__ __forceinline__ void block_normals(uint4 w, double z[4]) {
  box_muller(w.x, w.y, z[0], z[1]);
  box_muller(w.z, w.w, z[2], z[3]);
}
__device__ __forceinline__ void block_normals(uint4 w, float z[4]) {
  const float l0 = __builtin_amdgcn_logf((static_cast<float>(w.x) + 1.0f) * 0x1p-32f);   // log2 u
  const float l1 = __builtin_amdgcn_logf((static_cast<float>(w.z) + 1.0f) * 0x1p-32f);
  const float r0 = __builtin_amdgcn_sqrtf(-1.3862943611198906f * l0);                   // sqrt(-2 ln u)
  const float r1 = __builtin_amdgcn_sqrtf(-1.3862943611198906f * l1);
  const float t0 = static_cast<float>(w.y) * 0x1p-32f, t1 = static_cast<float>(w.w) * 0x1p-32f;
  z[0] = r0 * __builtin_amdgcn_cosf(t0);
  z[1] = r0 * __builtin_amdgcn_sinf(t0);
  z[2] = r1 * __builtin_amdgcn_cosf(t1);
  z[3] = r1 * __builtin_amdgcn_sinf(t1);
}

// Four consecutive values starting at a multiple of 4 (16/32-byte aligned when `vec`).
template <typename T>
__device__ __forceinline__ void load4(const T *src, bool vec, int j0, int lim, T out[4]) {
  if (vec && j0 + 4 <= lim) {
    if constexpr (sizeof(T) == 4) {
      const float4 v = *reinterpret_cast<const float4 *>(src + j0);
      out[0] = v.x; out[1] = v.y; out[2] = v.z; out[3] = v.w;
    } else {
      const f64x4 v = *reinterpret_cast<const f64x4 *>(src + j0);
      out[0] = v[0]; out[1] = v[1]; out[2] = v[2]; out[3] = v[3];
    }
  } else {
#pragma unroll
    for (int k = 0; k < 4; ++k) out[k] = (j0 + k < lim) ? src[j0 + k] : T(0);
  }
}
template <typename T>
__device__ __forceinline__ void store4(T *dst, bool vec, int j0, int lim, const T v[4]) {
  if (vec && j0 + 4 <= lim) {
    if constexpr (sizeof(T) == 4) {
      *reinterpret_cast<float4 *>(dst + j0) = make_float4(v[0], v[1], v[2], v[3]);
    } else {
      *reinterpret_cast<f64x4 *>(dst + j0) = f64x4{v[0], v[1], v[2], v[3]};
    }
  } else {
#pragma unroll
    for (int k = 0; k < 4; ++k)
      if (j0 + k < lim) dst[j0 + k] = v[k];
  }
}

// One aligned vector access of the block of four at j0.
template <typename T>
__device__ __forceinline__ void vload4(const T *src, int j0, T out[4]) {
  if constexpr (sizeof(T) == 4) {
    const float4 v = *reinterpret_cast<const float4 *>(src + j0);
    out[0] = v.x; out[1] = v.y; out[2] = v.z; out[3] = v.w;
  } else {
    const f64x4 v = *reinterpret_cast<const f64x4 *>(src + j0);
    out[0] = v[0]; out[1] = v[1]; out[2] = v[2]; out[3] = v[3];
  }
}
template <typename T>
__device__ __forceinline__ void vstore4(T *dst, int j0, const T v[4]) {
  if constexpr (sizeof(T) == 4) *reinterpret_cast<float4 *>(dst + j0) = make_float4(v[0], v[1], v[2], v[3]);
  else *reinterpret_cast<f64x4 *>(dst + j0) = f64x4{v[0], v[1], v[2], v[3]};
}
// load4 / store4 of a block that starts inside the array (j0 < lim, which the caller
// guarantees).  VR: lim is a multiple of 4 and the blocks are aligned, so the block is
// whole: one vector access with no checks (the checks' branches kept the compiler from
// issuing a row's loads together).
template <bool VR, typename T>
__device__ __forceinline__ void load4in(const T *src, bool vec, int j0, int lim, T out[4]) {
  if constexpr (VR) vload4(src, j0, out);
  else load4(src, vec, j0, lim, out);
}
template <bool VR, typename T>
__device__ __forceinline__ void store4in(T *dst, bool vec, int j0, int lim, const T v[4]) {
  if constexpr (VR) vstore4(dst, j0, v);
  else store4(dst, vec, j0, lim, v);
}

// x / v for a per-marker variance v stored by the move-constants kernel: FP32 stores the
// hardware reciprocal of v (so this is div_t(x, v)), FP64 stores v.
__device__ __forceinline__ float div_pre(float x, float stored) { return x * stored; }
__device__ __forceinline__ double div_pre(double x, double stored) { return x / stored; }
__device__ __forceinline__ float pre_div(float v) { return __builtin_amdgcn_rcpf(v); }
__device__ __forceinline__ double pre_div(double v) { return v; }

// Particle rows in registers: LP lanes per particle (64, or 32 for rows of at most 256
// markers, two particles per wave); sub-lane l holds markers 4l..4l+3 and
// 4LP+4l..4LP+4l+3 (one Philox block of four normals each), which covers p <= 8 LP - 1.
constexpr int kRowBlocks = 2;

// Sum over the LP lanes of a particle, the same value in every lane of the group (the
// butterfly of lane_group_sum; the FP8 operand packing sums in the same order).
template <int LP>
__device__ __forceinline__ double group_sum(double v) {
  return lane_group_sum<LP>(v);
}

template <int LP>
__device__ __forceinline__ double group_max(double v) {
#pragma unroll
  for (int o = LP / 2; o > 0; o >>= 1) v = fmax(v, __shfl_xor(v, o, kWave));
  return v;
}

// The FP8 multi-term operand of one random-walk proposal row from its scaled coefficients
// bv = (beta'/s) log2(e) in the row layout above (zero outside the row): term by term, the
// exponent puts the largest residual of the row in [128, 256), residual entries of at
// least 1 in that scale are rounded to e4m3 by the hardware conversion and smaller ones
// wait for the next term; the decoded codes are what the FP8 MFMA multiplies, and their
// sum is returned in used.  The standalone packing kernel of the contraction uses the same
// lane layout and order, so both give identical codes, exponents and offsets.
template <int LP>
__device__ __forceinline__ void f8_terms_row(const ProposeArgs &a, const int i, const int lane,
                                             const double (&bv)[kRowBlocks][4], double (&used)[kRowBlocks][4]) {
#pragma unroll
  for (int kb = 0; kb < kRowBlocks; ++kb)
#pragma unroll
    for (int k = 0; k < 4; ++k) used[kb][k] = 0.0;
  for (int t = 0; t < a.f8_terms; ++t) {
    double R = 0.0;
#pragma unroll
    for (int kb = 0; kb < kRowBlocks; ++kb)
#pragma unroll
      for (int k = 0; k < 4; ++k) R = fmax(R, fabs(bv[kb][k] - used[kb][k]));
    R = group_max<LP>(R);
    int E = 0;
    if (R > 0.0 && isfinite(R)) {
      int e2;
      frexp(R, &e2);
      E = e2 - 1 - 7;
    }
    E = max(-127, min(127, E));
    uint8_t *q = a.f8_q + ((size_t)t * a.f8_Mp + i) * a.f8_PP;
#pragma unroll
    for (int kb = 0; kb < kRowBlocks; ++kb) {
      const int b0 = lane * 4 + 4 * LP * kb;
      uint32_t packed = 0;
#pragma unroll
      for (int k = 0; k < 4; ++k) {
        const float x = static_cast<float>(ldexp(bv[kb][k] - used[kb][k], -E));
        const int c = fabsf(x) >= 1.0f ? (__builtin_amdgcn_cvt_pk_fp8_f32(x, 0.0f, 0, false) & 0xFF) : 0;
        used[kb][k] += ldexp(static_cast<double>(__builtin_amdgcn_cvt_f32_fp8(c, 0)), E);
        packed |= static_cast<uint32_t>(c) << (8 * k);
      }
      if (b0 < a.f8_PP) *reinterpret_cast<uint32_t *>(q + b0) = packed;   // 4-byte aligned
    }
    if (lane == 0) a.f8_s[(size_t)t * a.f8_Mp + i] = E + 127;
  }
}

// The proposal of one particle row (random walk or MALA) from its current coefficients
// and likelihood gradient (in registers, zero outside the row), the B operand of the
// proposal and the per-particle log prior terms.  The prior and proposal arithmetic runs
// in the particle precision PT; the log prior of a block of four coefficients is one log
// of the product of their factors.  `live` is false for padded particles (i >= M), which
// get a zero operand row.
// F8: the instance for random-walk rows of a handle on the FP8 multi-term contraction
// (compiled separately, so the other instances keep their register budget).
template <Prec P, typename PT, bool MALA, int LP, bool F8, bool VR>
__device__ __forceinline__ void propose_row(const ProposeArgs &a, const int i, const int lane, const bool live,
                                            const PT (&cur)[kRowBlocks][4], const PT (&gv)[kRowBlocks][4]) {
  using BT = typename BPack<P>::BT;
  const int p = a.p, PP = a.PP;
  PT *prop = reinterpret_cast<PT *>(a.prop) + (size_t)i * p;
  BT *Bhi = reinterpret_cast<BT *>(a.Bhi);
  BT *Blo = reinterpret_cast<BT *>(a.Blo);
  const bool vrow = (p & 3) == 0;   // particle rows keep 4-marker blocks aligned
  const Prior pr = a.prior;
  const PT inv_ac = pr.inf ? PT(0) : static_cast<PT>(1.0 / (pr.a * pr.lam));
  const PT a1 = static_cast<PT>(pr.a + 1.0), ac = static_cast<PT>(pr.a * pr.lam);
  const PT inv_c = static_cast<PT>(1.0 / pr.lam);
  const PT *mc = static_cast<const PT *>(a.mc);
  double m = 0.0, ybv = 0.0, lpc = 0.0, lpp = 0.0, lqf = 0.0;
  // FP8 multi-term operand (random-walk rows only): the scaled coefficients are kept until
  // the row is complete, then split into terms
  constexpr bool F8OK = F8 && (P == Prec::BF16X2) && !MALA;
  constexpr bool f8 = F8OK;
  double bv[F8OK ? kRowBlocks : 1][4], mu8[F8OK ? kRowBlocks : 1][4], yts8[F8OK ? kRowBlocks : 1][4];
  if constexpr (F8OK) {
#pragma unroll
    for (int kb = 0; kb < kRowBlocks; ++kb)
#pragma unroll
      for (int k = 0; k < 4; ++k) bv[kb][k] = mu8[kb][k] = yts8[kb][k] = 0.0;
  }
#pragma unroll
  for (int kb = 0; kb < kRowBlocks; ++kb) {
    const int b0 = lane * 4 + 4 * LP * kb;
    if (b0 >= PP) continue;
    PT z[4] = {0, 0, 0, 0}, nv[4] = {0, 0, 0, 0};
    // per-marker constants (PP-long rows): MALA drift, variance and noise scale, or the
    // random-walk scale
    PT hs[4], dv[4], ss[4];
    if constexpr (MALA) {
      load4in<true>(mc, true, b0, PP, hs);
      load4in<true>(mc + PP, true, b0, PP, dv);
      load4in<true>(mc + 2 * PP, true, b0, PP, ss);
    } else {
      load4in<true>(mc + 3 * PP, true, b0, PP, ss);
    }
    double invs[4], mu4[4], yt4[4], s4[4];
    load4in<true>(a.cc.inv_s, true, b0, PP, invs);   // PP is a multiple of 32 and b0 < PP
    load4in<true>(a.cc.mu, true, b0, PP, mu4);
    load4in<true>(a.cc.ytil, true, b0, PP, yt4);
    load4in<true>(a.cc.s, true, b0, PP, s4);
    const bool act = live && b0 < p;
    if (act)
      block_normals(philox4x32_10(make_uint4(static_cast<uint32_t>(i), static_cast<uint32_t>(b0 >> 2), a.sweep,
                                             word3(a.t, kTagNormal)),
                                  a.k0, a.k1),
                    z);
    PT fc = PT(1), fp = PT(1), lc = PT(0), lpn = PT(0), q = PT(0);
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      const int j = b0 + k;
      if (act && (VR || j < p)) {   // VR: the whole block is in the row
        const PT c = cur[kb][k];
        if constexpr (MALA) {
          const PT g = gv[kb][k] + gt_grad_t<PT>(c, a1, ac, pr.inf, inv_c);
          const PT meanf = c + hs[k] * g;
          nv[k] = meanf + ss[k] * z[k];
          const PT d = nv[k] - meanf;
          q += div_pre(d * d, dv[k]);
        } else {
          nv[k] = c + ss[k] * z[k];
        }
        if (pr.inf) {
          lc += fabs(c);
          lpn += fabs(nv[k]);
        } else {
          fc *= gt_factor<PT>(c, inv_ac);
          fp *= gt_factor<PT>(nv[k], inv_ac);
        }
      }
    }
    if (act) store4in<VR>(prop, vrow, b0, p, nv);
    // B operand of the proposal (zero in padded markers and padded particles)
    if (f8) {
      if constexpr (F8OK) {
#pragma unroll
        for (int k = 0; k < 4; ++k) {
          const int j = b0 + k;
          bv[kb][k] = (act && (VR || j < p)) ? static_cast<double>(nv[k]) * invs[k] * kLog2e : 0.0;
          mu8[kb][k] = mu4[k];
          yts8[kb][k] = yt4[k] * s4[k];
        }
      }
    } else {
      BT hb[4], lb[4];
#pragma unroll
      for (int k = 0; k < 4; ++k) {
        const int j = b0 + k;
        const double bj = (act && (VR || j < p)) ? static_cast<double>(nv[k]) * invs[k] : 0.0;
        double used;
        BPack<P>::put(bj, hb, lb, k, used);
        m += mu4[k] * used;
        ybv += yt4[k] * s4[k] * used;
      }
      store4_b<P>(Bhi, Blo, (size_t)i * PP + b0, hb, lb);
    }
    if (pr.inf) {
      lpc += static_cast<double>(lc);
      lpp += static_cast<double>(lpn);
    } else {
      lpc += static_cast<double>(fast_log(fc));
      lpp += static_cast<double>(fast_log(fp));
    }
    lqf -= static_cast<double>(q);
  }
  if constexpr (F8OK) {
    if (f8) {
      double used[kRowBlocks][4];
      f8_terms_row<LP>(a, i, lane, bv, used);
#pragma unroll
      for (int kb = 0; kb < kRowBlocks; ++kb)
#pragma unroll
        for (int k = 0; k < 4; ++k) {
          m += mu8[kb][k] * used[kb][k];
          ybv += yts8[kb][k] * used[kb][k];
        }
    }
  }
  m = group_sum<LP>(m);
  ybv = group_sum<LP>(ybv);
  lpc = group_sum<LP>(lpc);
  lpp = group_sum<LP>(lpp);
  if constexpr (MALA) lqf = group_sum<LP>(lqf);
  if (lane == 0) {
    a.moff[i] = m;
    a.yb[i] = ybv / BPack<P>::scale;
    if (live) {
      // sum_j log Gt = -p log(2c) - (a+1) sum log(factors)   (or - sum |b| / c)
      const double base = -static_cast<double>(p) * pr.log2lam;
      const double scale = pr.inf ? 1.0 / pr.lam : pr.a + 1.0;
      a.lp_cur[i] = base - scale * lpc;
      a.lp_prop[i] = base - scale * lpp;
      a.lqf[i] = lqf;
    }
  }
}

// Load a particle row into the register layout above (zero outside the row).
template <int LP, bool VR, typename PT>
__device__ __forceinline__ void load_row(const PT *row, const int lane, const int p, PT (&v)[kRowBlocks][4]) {
  const bool vrow = (p & 3) == 0;
#pragma unroll
  for (int kb = 0; kb < kRowBlocks; ++kb) {
    const int b0 = lane * 4 + 4 * LP * kb;
#pragma unroll
    for (int k = 0; k < 4; ++k) v[kb][k] = PT(0);
    if (b0 < p) load4in<VR>(row, vrow, b0, p, v[kb]);
  }
}

template <int LP, bool VR, typename PT>
__device__ __forceinline__ void store_row(PT *row, const int lane, const int p, const PT (&v)[kRowBlocks][4]) {
  const bool vrow = (p & 3) == 0;
#pragma unroll
  for (int kb = 0; kb < kRowBlocks; ++kb) {
    const int b0 = lane * 4 + 4 * LP * kb;
    if (b0 < p) store4in<VR>(row, vrow, b0, p, v[kb]);
  }
}

// One proposal sweep over all (padded) particle rows; LP lanes per particle.
template <Prec P, typename PT, bool MALA, int LP, bool F8, bool VR>
__global__ __launch_bounds__(256) void propose_kernel(ProposeArgs a) {
  const int lane = threadIdx.x & (LP - 1);
  const int i = static_cast<int>((blockIdx.x * blockDim.x + threadIdx.x) / LP);
  if (i >= a.M_pad) return;
  const bool live = i < a.M;
  PT cur[kRowBlocks][4], gv[kRowBlocks][4];
  const int p = live ? a.p : 0;   // padded particles: all-zero rows
  load_row<LP, VR>(reinterpret_cast<const PT *>(a.beta) + (size_t)i * a.p, lane, p, cur);
  if constexpr (MALA) load_row<LP, VR>(reinterpret_cast<const PT *>(a.gl) + (size_t)i * a.p, lane, p, gv);
  else load_row<LP, VR>(static_cast<const PT *>(nullptr), lane, 0, gv);
  propose_row<P, PT, MALA, LP, F8, VR>(a, i, lane, live, cur, gv);
}

// Metropolis-Hastings decision for every particle; accepted rows are copied into the state.
// SPL > 0: the proposal's log-likelihood and likelihood gradient are combined from the SPL
// partial sums of the split contraction (a compile-time count, so that every partial is
// loaded at once rather than one memory round trip per split).  NEXT: the wave then draws
// the next sweep's proposal from the row it has just decided (the state after this
// decision, still in registers), so the next sweep needs no separate proposal launch;
// valid while the proposal scale, the step size and the prior stay fixed between the two
// sweeps.  The current gradient row is read with the other rows at the start, for every
// particle (a rejected row needs it for its next proposal), so that no row load waits on
// the decision.
template <Prec P, typename PT, bool MALA, int SPL, bool NEXT, int LP, bool F8, bool VR>
__global__ __launch_bounds__(256) void accept_kernel(AcceptArgs a, ProposeArgs na) {
  constexpr bool PARTS = SPL > 0;
  const int lane = threadIdx.x & (LP - 1);
  const int i = static_cast<int>((blockIdx.x * blockDim.x + threadIdx.x) / LP);
  if (i >= a.M) return;
  const int p = a.p;
  PT *beta = reinterpret_cast<PT *>(a.beta) + (size_t)i * p;
  PT *gl = reinterpret_cast<PT *>(a.gl) + (size_t)i * p;
  const Prior pr = a.prior;
  PT nv[kRowBlocks][4], cur[kRowBlocks][4], gnew[kRowBlocks][4];
  PT gold[(MALA && NEXT) ? kRowBlocks : 1][4];
  load_row<LP, VR>(reinterpret_cast<const PT *>(a.prop) + (size_t)i * p, lane, p, nv);
  load_row<LP, VR>(const_cast<const PT *>(beta), lane, MALA || NEXT ? p : 0, cur);
  if constexpr (MALA && NEXT) load_row<LP, VR>(const_cast<const PT *>(gl), lane, p, gold);
  double llp;
  if constexpr (PARTS) {
    double spl = 0.0;
#pragma unroll
    for (int s = 0; s < SPL; ++s) spl += a.spl_part[s * a.Mp + i];
    llp = a.yb[i] - spl;
    if constexpr (MALA) {
      const PT *gp = reinterpret_cast<const PT *>(a.g_part);
      const int PP = a.PP;
      double rho = 0.0;
#pragma unroll
      for (int s = 0; s < SPL; ++s) rho += static_cast<double>(gp[(s * a.Mp + i) * PP + PP - 1]);
#pragma unroll
      for (int kb = 0; kb < kRowBlocks; ++kb) {
        const int b0 = lane * 4 + 4 * LP * kb;
#pragma unroll
        for (int k = 0; k < 4; ++k) gnew[kb][k] = PT(0);
        if (b0 >= p) continue;
        double acc[4] = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
        for (int s = 0; s < SPL; ++s) {   // rows are PP long, PP a multiple of 32: aligned blocks
          PT t4[4];
          load4in<true>(gp + (s * a.Mp + i) * PP, true, b0, PP, t4);   // b0 < p <= PP
#pragma unroll
          for (int k = 0; k < 4; ++k) acc[k] += static_cast<double>(t4[k]);
        }
        double yt4[4], mu4[4], is4[4];
        load4in<true>(a.ytil, true, b0, PP, yt4);
        load4in<true>(a.mu, true, b0, PP, mu4);
        load4in<true>(a.inv_s, true, b0, PP, is4);
#pragma unroll
        for (int k = 0; k < 4; ++k)
          if (VR || b0 + k < p) gnew[kb][k] = static_cast<PT>(yt4[k] - (acc[k] - mu4[k] * rho) * is4[k]);
      }
    }
  } else {
    llp = a.ll_prop[i];
    if constexpr (MALA) load_row<LP, VR>(reinterpret_cast<const PT *>(a.gl_prop) + (size_t)i * p, lane, p, gnew);
  }
  double lqr = 0.0;
  if constexpr (MALA) {
    const PT a1 = static_cast<PT>(pr.a + 1.0), ac = static_cast<PT>(pr.a * pr.lam);
    const PT inv_c = static_cast<PT>(1.0 / pr.lam);
    const PT *mc = static_cast<const PT *>(a.mc);
    PT q = PT(0);
#pragma unroll
    for (int kb = 0; kb < kRowBlocks; ++kb) {
      const int b0 = lane * 4 + 4 * LP * kb;
      if (b0 >= p) continue;
      PT hs[4], dv[4];
      load4in<true>(mc, true, b0, a.PP, hs);   // b0 < p <= PP
      load4in<true>(mc + a.PP, true, b0, a.PP, dv);
#pragma unroll
      for (int k = 0; k < 4; ++k) {
        if (VR || b0 + k < p) {
          const PT g = gnew[kb][k] + gt_grad_t<PT>(nv[kb][k], a1, ac, pr.inf, inv_c);
          const PT meanr = nv[kb][k] + hs[k] * g;
          const PT d = cur[kb][k] - meanr;
          q += div_pre(d * d, dv[k]);
        }
      }
    }
    lqr = -group_sum<LP>(static_cast<double>(q));
  }
  const double log_alpha = llp - a.ll[i] + a.lp_prop[i] - a.lp_cur[i] + lqr - a.lqf[i];
  const int cnt = a.acc_cnt[i];
  const uint4 w = philox4x32_10(make_uint4(static_cast<uint32_t>(i), 0u, a.sweep, word3(a.t, kTagUniform)),
                                a.k0, a.k1);
  const double u = (static_cast<double>(w.x) + 0.5) * 0x1p-32;
  const bool acc = log(u) < log_alpha;   // false for NaN; the same in every lane of the group
  if (acc) {
    store_row<LP, VR>(beta, lane, p, nv);
    if constexpr (MALA) store_row<LP, VR>(gl, lane, p, gnew);
    if (lane == 0) a.ll[i] = llp;
  }
  if (lane == 0) a.acc_cnt[i] = cnt + (acc ? 1 : 0);
  if constexpr (NEXT) {
    PT nc[kRowBlocks][4], gv[kRowBlocks][4];
#pragma unroll
    for (int kb = 0; kb < kRowBlocks; ++kb)
#pragma unroll
      for (int k = 0; k < 4; ++k) {
        nc[kb][k] = acc ? nv[kb][k] : cur[kb][k];
        if constexpr (MALA) gv[kb][k] = acc ? gnew[kb][k] : gold[kb][k];
        else gv[kb][k] = PT(0);
      }
    propose_row<P, PT, MALA, LP, F8, VR>(na, i, lane, true, nc, gv);
  }
}

// ================================================================ weights

// Lanes per particle row of the weight, resampling-gather and moment passes: the fewest
// (8, 16, 32 or 64) for which a lane holds at most two blocks of four coefficients.
static __host__ __device__ constexpr int bw_lanes(int p) { return p <= 64 ? 8 : p <= 128 ? 16 : p <= 256 ? 32 : 64; }
constexpr int kBW = 256;   // threads per workgroup of the bandwidth kernels

// Fixed-order workgroup reductions of one value per thread over WG threads (every thread
// gets the result); sh holds WG / kWave doubles.
template <int WG = kBW>
__device__ double wg_max(double v, double *sh) {
  v = wave_max(v);
  __syncthreads();
  if ((threadIdx.x & (kWave - 1)) == 0) sh[threadIdx.x / kWave] = v;
  __syncthreads();
  double r = sh[0];
  for (int q = 1; q < WG / kWave; ++q) r = fmax(r, sh[q]);
  return r;
}
template <int WG = kBW>
__device__ double wg_sum(double v, double *sh) {
  v = wave_sum(v);
  __syncthreads();
  if ((threadIdx.x & (kWave - 1)) == 0) sh[threadIdx.x / kWave] = v;
  __syncthreads();
  double r = sh[0];
  for (int q = 1; q < WG / kWave; ++q) r += sh[q];
  return r;
}

// Incremental weights, then the pieces of the normalisation and ESS (Section 4).
//   logw_i <- logw_i + sum_j [log Gt(b_ij | a, lam_new) - log Gt(b_ij | a, lam_old)]
//           = logw_i + p a log r - (a+1) sum_j log((a lam_new + |b_ij|)/(a lam_old + |b_ij|)),
// r = lam_new/lam_old (a lane multiplies its at most 8 ratios, all in (r, 1], before one
// log); the double exponential: p log(1/r) - (1/lam_new - 1/lam_old) sum_j |b_ij|.
// With logw_{t-1} normalised, L = log sum_i exp(logw_i) is the log Z increment, and
// ESS = (sum e^{logw})^2 / sum e^{2 logw}.  Each workgroup writes its maximum m_b and the
// sums of e^{logw - m_b} and e^{2(logw - m_b)} (lse_finalize_kernel combines them).  The
// log weights are left unnormalised (the next pass subtracts L).
// The reweighting pass: one particle row per LP lanes, rw_rows(LP) = kBW / LP rows per
// workgroup (larger workgroups, or several rows per lane with their loads issued together,
// measured slower at n = 5000, p = 200, N = 16384).
static __host__ __device__ constexpr int rw_rows(int LP) { return kBW / LP; }

template <typename PT, int LP>
__global__ __launch_bounds__(rw_rows(LP) * LP) void reweight_kernel(ReweightArgs a) {
  constexpr int NP = 1;
  constexpr int kRwRows = rw_rows(LP);
  constexpr int WG = kRwRows * LP;
  __shared__ double sh[WG / kWave];
  const int lane = threadIdx.x & (LP - 1);
  const int r0 = blockIdx.x * kRwRows + threadIdx.x / LP;
  const int p = a.p;
  const bool vec = (p & 3) == 0;
  PT v[NP][2][4];
  double lw0[NP];
#pragma unroll
  for (int q = 0; q < NP; ++q) {
    const int i = r0 + q * kRwRows;
    const bool live = i < a.M;
    lw0[q] = live ? a.logw[i] : 0.0;
    const PT *row = static_cast<const PT *>(a.beta) + (size_t)(live ? i : 0) * p;
#pragma unroll
    for (int kb = 0; kb < 2; ++kb) {
      const int j0 = 4 * (lane + LP * kb);
      if (live && j0 < p) load4(row, vec, j0, p, v[q][kb]);
      else v[q][kb][0] = v[q][kb][1] = v[q][kb][2] = v[q][kb][3] = PT(0);
    }
  }
  const double lr = log(a.lam_new / a.lam_old);
  const double an = a.a * a.lam_new, ao = a.a * a.lam_old;
  const double cst = static_cast<double>(p) * (a.a_inf ? -lr : a.a * lr);
  double lw[NP];
#pragma unroll
  for (int q = 0; q < NP; ++q) {
    double d;
    if (a.a_inf) {
      double sx = 0.0;
#pragma unroll
      for (int kb = 0; kb < 2; ++kb)
#pragma unroll
        for (int e = 0; e < 4; ++e) sx += fabs(static_cast<double>(v[q][kb][e]));
      d = -(1.0 / a.lam_new - 1.0 / a.lam_old) * sx;
    } else {
      // one division per lane: the products of the (at most 8) numerators and denominators;
      // if either leaves the finite positive range, the product of the ratios instead
      double num = 1.0, den = 1.0;
#pragma unroll
      for (int kb = 0; kb < 2; ++kb)
#pragma unroll
        for (int e = 0; e < 4; ++e) {
          const double x = fabs(static_cast<double>(v[q][kb][e]));
          if (4 * (lane + LP * kb) + e < p) {
            num *= an + x;
            den *= ao + x;
          }
        }
      double ratio = num / den;
      if (!(num > 0.0 && num < INFINITY && den > 0.0 && den < INFINITY)) {
        ratio = 1.0;
#pragma unroll
        for (int kb = 0; kb < 2; ++kb)
#pragma unroll
          for (int e = 0; e < 4; ++e) {
            const double x = fabs(static_cast<double>(v[q][kb][e]));
            if (4 * (lane + LP * kb) + e < p) ratio *= (an + x) / (ao + x);
          }
      }
      d = -(a.a + 1.0) * log(ratio);
    }
    d = group_sum<LP>(d);
    const int i = r0 + q * kRwRows;
    lw[q] = -INFINITY;   // rows past M carry no weight
    if (i < a.M) {
      lw[q] = lw0[q] + d + cst;
      if (lane == 0) a.logw[i] = lw[q];
    }
  }
  double m = lw[0];
#pragma unroll
  for (int q = 1; q < NP; ++q) m = fmax(m, lw[q]);
  m = wg_max<WG>(m, sh);
  double e1 = 0.0, e2 = 0.0;
  if (lane == 0 && m != -INFINITY)
#pragma unroll
    for (int q = 0; q < NP; ++q)
      if (r0 + q * kRwRows < a.M) {
        const double e = exp(lw[q] - m);
        e1 += e;
        e2 += e * e;
      }
  const double s1 = wg_sum<WG>(e1, sh);
  const double s2 = wg_sum<WG>(e2, sh);
  if (threadIdx.x == 0) {
    double *o = a.part + 3 * (size_t)blockIdx.x;
    o[0] = m;
    o[1] = s1;
    o[2] = s2;
  }
}

// Combination of the reweighting pass's G workgroup partials in workgroup order (one
// workgroup; the kernel boundary makes the partials visible):
//   L = m + log S1, ESS = S1^2 / S2, S1 = sum_b e^{m_b - m} s1_b, S2 = sum_b e^{2(m_b - m)} s2_b,
// m = max_b m_b; writes {ESS, L, resample flag, m, non-finite flag, 0} to scalars.
constexpr int kFin = 1024;   // threads of the combination kernel

__global__ __launch_bounds__(kFin) void lse_finalize_kernel(const double *__restrict__ part, int G, int M,
                                                            double ess_frac, double *__restrict__ scalars) {
  __shared__ double sh[kFin / kWave];
  constexpr int B = 4;   // partials per thread per batch, their loads issued together
  double gm = -INFINITY, t1 = 0.0, t2 = 0.0;
  // the batches run in order; within one, thread t holds partials b0 + t + kBW u
  double mb[B], p1[B], p2[B];
  for (int b0 = 0; b0 < G; b0 += B * kFin) {
#pragma unroll
    for (int u = 0; u < B; ++u) {
      const int b = b0 + threadIdx.x + u * kFin;
      mb[u] = b < G ? part[3 * (size_t)b] : -INFINITY;
      p1[u] = b < G ? part[3 * (size_t)b + 1] : 0.0;
      p2[u] = b < G ? part[3 * (size_t)b + 2] : 0.0;
    }
    double bm = mb[0];
#pragma unroll
    for (int u = 1; u < B; ++u) bm = fmax(bm, mb[u]);
    bm = wg_max<kFin>(bm, sh);
    const double nm = fmax(gm, bm);   // running maximum; earlier sums rescaled to it
    if (nm != -INFINITY) {
      if (gm != -INFINITY && nm != gm) {
        const double f = exp(gm - nm);
        t1 *= f;
        t2 *= f * f;
      }
#pragma unroll
      for (int u = 0; u < B; ++u)
        if (mb[u] != -INFINITY) {
          const double f = exp(mb[u] - nm);
          t1 += p1[u] * f;
          t2 += p2[u] * (f * f);
        }
    }
    gm = nm;
  }
  t1 = wg_sum<kFin>(t1, sh);
  t2 = wg_sum<kFin>(t2, sh);
  if (threadIdx.x == 0) {
    const double L = gm + log(t1);
    const double ess = t1 * t1 / t2;
    const bool ok = isfinite(L) && isfinite(ess);
    scalars[0] = ess;
    scalars[1] = L;
    scalars[2] = (ok && ess < ess_frac * static_cast<double>(M)) ? 1.0 : 0.0;
    scalars[3] = gm;
    scalars[4] = ok ? 0.0 : 1.0;
    scalars[5] = 0.0;   // no invalid-weight flag for the resampling passes that may follow
  }
}

// ---------------------------------------------------------------- systematic resampling
// On the quantised weights q_i = floor(x_i 2^K), K = 53 - ceil(log2 M), x_i in [0, 1] the
// weight relative to the largest: every partial sum C_k = q_0 + ... + q_k is an integer
// below 2^53, exact in FP64 in any summation order, so the multi-workgroup scan below is
// bit-exact.  Offspring i takes the first k with C_k > ((i + U) C) / M (the product first,
// no fused multiply-add), clamped to M - 1, C = C_{M-1}.

// Validation and maximum of linear weights (spa_smc_resample), per workgroup:
// part[2b] = max w, part[2b+1] = 1 if a weight is negative, NaN or infinite.
__global__ __launch_bounds__(kBW) void wmax_kernel(const double *__restrict__ w, int M, double *__restrict__ part) {
  __shared__ double sh[kBW / kWave];
  double m = -INFINITY, bad = 0.0;
  for (int i = blockIdx.x * kBW + threadIdx.x; i < M; i += gridDim.x * kBW) {
    const double v = w[i];
    if (!(v >= 0.0) || isinf(v)) bad = 1.0;
    m = fmax(m, v);
  }
  m = wg_max(m, sh);
  bad = wg_max(bad, sh);
  if (threadIdx.x == 0) {
    part[2 * (size_t)blockIdx.x] = m;
    part[2 * (size_t)blockIdx.x + 1] = bad;
  }
}

// q_i into cdf[i] and the sum of q over each workgroup's range of kBW * ept weights (ept
// per thread, coalesced).  mode 0: x_i = min(e^{logw_i - max logw}, 1) from the
// reweighting pass's unnormalised log weights (scalars[3] = their maximum); mode 1:
// x_i = w_i / max w, max w and validity from the G workgroup partials of wmax_kernel
// (workgroup 0 records them: scalars[6] = max w, scalars[5] = 1 for invalid weights, all
// zero included, and then nothing is quantised).
__global__ __launch_bounds__(kBW) void quantise_kernel(int mode, const double *__restrict__ logw,
                                                       const double *__restrict__ w, const double *__restrict__ wpart,
                                                       int M, int K, int ept, double *__restrict__ scalars,
                                                       double *__restrict__ cdf, double *__restrict__ btot) {
  __shared__ double sh[kBW / kWave];
  double ref;
  if (mode == 0) {
    ref = scalars[3];
  } else {
    double m = -INFINITY, bad = 0.0;
    for (int b = threadIdx.x; b < (int)gridDim.x; b += kBW) {
      m = fmax(m, wpart[2 * (size_t)b]);
      bad = fmax(bad, wpart[2 * (size_t)b + 1]);
    }
    m = wg_max(m, sh);
    bad = wg_max(bad, sh);
    const bool invalid = bad != 0.0 || !(m > 0.0);
    if (blockIdx.x == 0 && threadIdx.x == 0) {
      scalars[5] = invalid ? 1.0 : 0.0;
      scalars[6] = m;
    }
    if (invalid) return;
    ref = m;
  }
  const double scale = ldexp(1.0, K);
  const size_t base = (size_t)blockIdx.x * kBW * ept;
  double s = 0.0;
  for (int e = 0; e < ept; ++e) {
    const size_t i = base + (size_t)e * kBW + threadIdx.x;
    if (i < (size_t)M) {
      const double x = mode == 0 ? fmin(exp(logw[i] - ref), 1.0) : w[i] / ref;
      const double q = floor(x * scale);
      cdf[i] = q;
      s += q;
    }
  }
  s = wg_sum(s, sh);
  if (threadIdx.x == 0) btot[blockIdx.x] = s;
}

// Inclusive scan of q over the whole array: a workgroup adds the totals of the ranges
// before its own, then scans its range (ept consecutive values per thread, a wave scan of
// the thread totals, the wave totals in order).  scalars[7] = C.
__global__ __launch_bounds__(kBW) void cdf_scan_kernel(int M, int ept, const double *__restrict__ btot,
                                                       double *__restrict__ cdf, double *__restrict__ scalars) {
  __shared__ double sh[kBW / kWave];
  __shared__ double wtot[kBW / kWave];
  if (scalars[5] != 0.0) return;
  const int G = gridDim.x;
  double before = 0.0, all = 0.0;
  for (int b = threadIdx.x; b < G; b += kBW) {
    const double v = btot[b];
    all += v;
    if (b < (int)blockIdx.x) before += v;
  }
  before = wg_sum(before, sh);
  all = wg_sum(all, sh);
  const size_t lo = (size_t)blockIdx.x * kBW * ept + (size_t)threadIdx.x * ept;
  double run = 0.0;
  for (int e = 0; e < ept; ++e)
    if (lo + e < (size_t)M) run += cdf[lo + e];
  // inclusive wave scan of the thread totals
  const int ln = threadIdx.x & (kWave - 1), wv = threadIdx.x / kWave;
  double inc = run;
#pragma unroll
  for (int o = 1; o < kWave; o <<= 1) {
    const double v = __shfl_up(inc, o, kWave);
    if (ln >= o) inc += v;
  }
  if (ln == kWave - 1) wtot[wv] = inc;
  __syncthreads();
  double off = before;
  for (int q = 0; q < wv; ++q) off += wtot[q];
  off += inc - run;   // exclusive prefix of this thread
  for (int e = 0; e < ept; ++e)
    if (lo + e < (size_t)M) {
      off += cdf[lo + e];
      cdf[lo + e] = off;
    }
  if (blockIdx.x == 0 && threadIdx.x == 0) scalars[7] = all;
}

// Offspring search, LP lanes per offspring: each round the lanes probe the ends of LP
// equal segments of the remaining range [lo, hi] (hi = M or a position whose C exceeds
// the target) and keep the first segment whose end exceeds it, so M = 16384 takes three
// rounds of loads at LP = 32.  Optionally the offspring's rows are gathered from its
// ancestor (particles, gradients, log-likelihoods) and its log weight set to -log M.
template <typename PT, int LP>
__global__ __launch_bounds__(kBW) void search_gather_kernel(ResampleArgs a) {
  if (a.scalars[5] != 0.0) return;
  const int lane = threadIdx.x & (LP - 1);
  const int i = blockIdx.x * (kBW / LP) + threadIdx.x / LP;
  if (i >= a.M) return;   // whole groups leave together
  const double C = a.scalars[7];
  const double U = static_cast<double>(a.u32) * 0x1p-32;
  const double tpos = __ddiv_rn(__dmul_rn(__dadd_rn(static_cast<double>(i), U), C), static_cast<double>(a.M));
  const int gbase = (threadIdx.x & (kWave - 1)) & ~(LP - 1);   // first lane of the group in the wave
  int lo = 0, hi = a.M;
  while (lo < hi) {
    const int step = (hi - lo + LP - 1) / LP;
    const int pos = lo + (lane + 1) * step - 1;
    const bool gt = pos >= hi || a.cdf[pos] > tpos;
    const unsigned long long bal = __ballot(gt);
    const unsigned long long gm = (bal >> gbase) & (LP == 64 ? ~0ull : ((1ull << LP) - 1));
    if (gm == 0ull) {   // even C at hi - 1 does not exceed the target: the answer is hi
      lo = hi;
      break;
    }
    const int f = __builtin_ctzll(gm);   // first segment whose end exceeds the target
    const int flo = lo + f * step;
    const int fhi = min(lo + (f + 1) * step - 1, hi);
    lo = flo;
    hi = fhi;
    if (fhi == flo) break;
  }
  const int k = min(lo, a.M - 1);
  if (lane == 0) a.anc[i] = k;
  if (!a.src) return;
  const int p = a.p;
  const bool vec = (p & 3) == 0;
  const PT *s = static_cast<const PT *>(a.src) + (size_t)k * p;
  PT *d = static_cast<PT *>(a.dst) + (size_t)i * p;
  const PT *gs = a.gsrc ? static_cast<const PT *>(a.gsrc) + (size_t)k * p : nullptr;
  PT *gd = a.gsrc ? static_cast<PT *>(a.gdst) + (size_t)i * p : nullptr;
#pragma unroll
  for (int kb = 0; kb < 2; ++kb) {
    const int j0 = 4 * (lane + LP * kb);
    if (j0 < p) {
      PT v[4];
      load4(s, vec, j0, p, v);
      store4(d, vec, j0, p, v);
      if (gs) {
        load4(gs, vec, j0, p, v);
        store4(gd, vec, j0, p, v);
      }
    }
  }
  if (lane == 0) {
    a.lldst[i] = a.llsrc[k];
    a.logw[i] = a.logw_eq;
  }
}

// ---- weighted moments per coefficient (two kernels: chunk partials, ordered combine).
// Partial sums are shifted by the first particle's row (removes cancellation):
//   S0 = sum W, S1_j = sum W (b_ij - c_j), S2_j = sum W (b_ij - c_j)^2.
// A workgroup covers one chunk of kMomRows rows and every column: RG row groups of CP
// column threads (CP = p rounded up to 64, at most 256; RG = 256 / CP), whose partials are
// added in row-group order.  With `shift`, the chunk's log weights are first normalised
// in place (logw_i -= *shift); only this workgroup reads those rows' weights.
constexpr int kMomRows = 64;

template <typename PT>
__global__ __launch_bounds__(kBW) void moments_partial_kernel(const PT *__restrict__ beta, double *__restrict__ logw,
                                                              const double *__restrict__ shift, int M, int p,
                                                              double *__restrict__ part) {
  __shared__ double Wsh[kMomRows];
  __shared__ double sh[3][kBW];
  const int chunk = blockIdx.x;
  const int r0 = chunk * kMomRows, r1 = min(M, r0 + kMomRows);
  if ((int)threadIdx.x < r1 - r0) {
    double lw = logw[r0 + threadIdx.x];
    if (shift) {
      lw -= *shift;
      logw[r0 + threadIdx.x] = lw;
    }
    Wsh[threadIdx.x] = exp(lw);
  }
  __syncthreads();
  const int CP = min(kBW, (p + 63) / 64 * 64);
  const int RG = kBW / CP;
  const int rg = threadIdx.x / CP, cl = threadIdx.x % CP;
  for (int col0 = 0; col0 < p; col0 += CP) {   // one pass unless p > 256
    const int col = col0 + cl;
    double s0 = 0.0, s1 = 0.0, s2 = 0.0;
    if (rg < RG && col < p) {
      const double c = static_cast<double>(beta[col]);
      const PT *bp = beta + col;
      int i = r0 + rg;
      for (; i + 15 * RG < r1; i += 16 * RG) {   // sixteen rows' loads in flight, then in order
        PT v[16];
#pragma unroll
        for (int u = 0; u < 16; ++u) v[u] = bp[(size_t)(i + u * RG) * p];
#pragma unroll
        for (int u = 0; u < 16; ++u) {
          const double W = Wsh[i + u * RG - r0];
          const double dd = static_cast<double>(v[u]) - c;
          s0 += W;
          s1 += W * dd;
          s2 += W * dd * dd;
        }
      }
      for (; i < r1; i += RG) {
        const double W = Wsh[i - r0];
        const double dd = static_cast<double>(bp[(size_t)i * p]) - c;
        s0 += W;
        s1 += W * dd;
        s2 += W * dd * dd;
      }
    }
    if (RG > 1) {
      __syncthreads();
      sh[0][threadIdx.x] = s0;
      sh[1][threadIdx.x] = s1;
      sh[2][threadIdx.x] = s2;
      __syncthreads();
      if (rg == 0)
        for (int q = 1; q < RG; ++q) {
          s0 += sh[0][q * CP + cl];
          s1 += sh[1][q * CP + cl];
          s2 += sh[2][q * CP + cl];
        }
    }
    if (rg == 0 && col < p) {
      double *o = part + ((size_t)chunk * p + col) * 3;
      o[0] = s0;
      o[1] = s1;
      o[2] = s2;
    }
  }
}

// One wave per coefficient: lanes take the chunks (fixed tree order).
template <typename PT>
__global__ void moments_final_kernel(const PT *__restrict__ beta, const double *__restrict__ part,
                                     int nchunks, int p, double *__restrict__ mean,
                                     double *__restrict__ var, double *__restrict__ sigma,
                                     double sigma_floor) {
  const int lane = threadIdx.x & 63;
  const int j = blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6);
  if (j >= p) return;
  double t0 = 0.0, t1 = 0.0, t2 = 0.0;
  for (int c = lane; c < nchunks; c += 64) {
    const double *o = part + ((size_t)c * p + j) * 3;
    t0 += o[0];
    t1 += o[1];
    t2 += o[2];
  }
  t0 = wave_sum(t0);
  t1 = wave_sum(t1);
  t2 = wave_sum(t2);
  if (lane != 0) return;
  const double d1 = t1 / t0;
  const double m = static_cast<double>(beta[j]) + d1;
  const double v = fmax(t2 / t0 - d1 * d1, 0.0);
  if (mean) mean[j] = m;
  if (var) var[j] = v;
  if (sigma) sigma[j] = sqrt(fmax(v, sigma_floor * sigma_floor));
}

// Accept count of a step, and the number of particles whose log-likelihood is not finite.
__global__ void count_kernel(const int *__restrict__ cnt, int M, const double *__restrict__ ll,
                             long long *__restrict__ out) {
  __shared__ long long sh[2][16];
  long long s = 0, bad = 0;
  for (int i = threadIdx.x; i < M; i += blockDim.x) {
    s += cnt[i];
    if (ll && !isfinite(ll[i])) ++bad;
  }
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) {
    s += __shfl_xor(s, o, 64);
    bad += __shfl_xor(bad, o, 64);
  }
  if ((threadIdx.x & 63) == 0) {
    sh[0][threadIdx.x >> 6] = s;
    sh[1][threadIdx.x >> 6] = bad;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    long long r = 0, b = 0;
    for (int q = 0; q < (int)(blockDim.x >> 6); ++q) {
      r += sh[0][q];
      b += sh[1][q];
    }
    out[0] = r;
    out[1] = b;
  }
}

__global__ void fill_kernel(double *__restrict__ x, int n, double v) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) x[i] = v;
}
__global__ void zero_int_kernel(int *__restrict__ x, int n) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) x[i] = 0;
}

template <typename ST, typename DT>
__global__ void convert_kernel(const ST *__restrict__ src, DT *__restrict__ dst, size_t n) {
  for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x)
    dst[i] = static_cast<DT>(src[i]);
}

// log posterior = loglik + sum_j log Gt(beta_ij); gradient += prior gradient (in place, in
// the gradient's own dtype, so a later conversion rounds only once).
template <typename BT, typename GT>
__global__ void add_prior_kernel(const BT *__restrict__ beta, int M, int p, Prior pr,
                                 GT *__restrict__ g, const double *__restrict__ ll,
                                 double *__restrict__ logpost) {
  const int lane = threadIdx.x & 63;
  const int i = blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6);
  if (i >= M) return;
  double lp = 0.0;
  for (int j = lane; j < p; j += 64) {
    const size_t off = (size_t)i * p + j;
    const double b = static_cast<double>(beta[off]);
    if (g) g[off] = static_cast<GT>(static_cast<double>(g[off]) + gt_grad(b, pr));
    lp += gt_logpdf(b, pr);
  }
  lp = wave_sum(lp);
  if (lane == 0 && logpost) logpost[i] = ll[i] + lp;
}

__global__ void philox_kernel(const uint32_t *__restrict__ ctr, int M, uint32_t k0, uint32_t k1,
                              uint32_t *__restrict__ out) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= M) return;
  const uint4 c = make_uint4(ctr[4 * i], ctr[4 * i + 1], ctr[4 * i + 2], ctr[4 * i + 3]);
  const uint4 r = philox4x32_10(c, k0, k1);
  out[4 * i] = r.x;
  out[4 * i + 1] = r.y;
  out[4 * i + 2] = r.z;
  out[4 * i + 3] = r.w;
}

// ================================================================ host launchers

static inline int grid_rows(int rows, int rows_per_block) { return (rows + rows_per_block - 1) / rows_per_block; }

void launch_col_stats(const uint8_t *X, const uint8_t *y, int n, int p, double *mu, double *s,
                      double *inv_s, double *ytil, int *bad, hipStream_t st) {
  hipLaunchKernelGGL(col_stats_kernel, dim3(p), dim3(256), 0, st, X, y, n, p, mu, s, inv_s, ytil, bad);
}

void launch_pack_x(XFormat f, Prec prec, const uint8_t *X, int n, int p, int n_pad, int PP, void *Xk,
                   void *Xt, hipStream_t st) {
  const size_t total = (size_t)n_pad * PP;
  const int grid = static_cast<int>(std::min<size_t>((total + 255) / 256, 65535));
  switch (f) {
    case XFormat::F64:
      hipLaunchKernelGGL(pack_x_kernel<double>, dim3(grid), dim3(256), 0, st, X, n, p, n_pad, PP, prec,
                         (double *)Xk, (double *)Xt);
      break;
    case XFormat::F32:
      hipLaunchKernelGGL(pack_x_kernel<float>, dim3(grid), dim3(256), 0, st, X, n, p, n_pad, PP, prec,
                         (float *)Xk, (float *)Xt);
      break;
    case XFormat::BF16:
      hipLaunchKernelGGL(pack_x_kernel<__bf16>, dim3(grid), dim3(256), 0, st, X, n, p, n_pad, PP, prec,
                         (__bf16 *)Xk, (__bf16 *)Xt);
      break;
    case XFormat::FP8:
      hipLaunchKernelGGL(pack_x_kernel<uint8_t>, dim3(grid), dim3(256), 0, st, X, n, p, n_pad, PP, prec,
                         (uint8_t *)Xk, (uint8_t *)Xt);
      break;
  }
}

void launch_labels(const uint8_t *y, int n, int n_pad, bool f64, void *yv, hipStream_t st) {
  if (f64)
    hipLaunchKernelGGL(labels_kernel<double>, dim3((n_pad + 255) / 256), dim3(256), 0, st, y, n, n_pad, (double *)yv);
  else
    hipLaunchKernelGGL(labels_kernel<float>, dim3((n_pad + 255) / 256), dim3(256), 0, st, y, n, n_pad, (float *)yv);
}

void launch_pack_b(Prec prec, bool in_f64, const void *beta, int M, int M_pad, int p, int PP,
                   const double *mu, const double *s, const double *inv_s, const double *ytil,
                   void *Bhi, void *Blo, double *moff, double *yb, hipStream_t st) {
  ColConst cc{mu, s, inv_s, ytil};
  const int grid = grid_rows(M_pad, 4);
#define SPA_PACK(P, IT)                                                                       \
  hipLaunchKernelGGL((pack_b_kernel<P, IT>), dim3(grid), dim3(256), 0, st, (const IT *)beta, M, \
                     M_pad, p, PP, cc, Bhi, Blo, moff, yb)
  if (prec == Prec::BF16X2) {
    if (in_f64) SPA_PACK(Prec::BF16X2, double); else SPA_PACK(Prec::BF16X2, float);
  } else if (prec == Prec::F32) {
    if (in_f64) SPA_PACK(Prec::F32, double); else SPA_PACK(Prec::F32, float);
  } else {
    if (in_f64) SPA_PACK(Prec::F64, double); else SPA_PACK(Prec::F64, float);
  }
#undef SPA_PACK
}

// Lanes per particle row of the proposal and decision kernels: half a wave when the
// padded row fits in 256 markers.
static inline int row_lanes(int PP) { return PP <= 256 ? 32 : 64; }

template <Prec P, typename PT, bool MALA, bool F8 = false>
static void launch_propose_t(const ProposeArgs &a, hipStream_t st) {
  const bool vr = (a.p & 3) == 0;   // whole 4-marker blocks in every particle row
  if (row_lanes(a.PP) == 32) {
    const dim3 grid(grid_rows(a.M_pad, 8));
    if (vr) hipLaunchKernelGGL((propose_kernel<P, PT, MALA, 32, F8, true>), grid, dim3(256), 0, st, a);
    else hipLaunchKernelGGL((propose_kernel<P, PT, MALA, 32, F8, false>), grid, dim3(256), 0, st, a);
  } else {
    const dim3 grid(grid_rows(a.M_pad, 4));
    if (vr) hipLaunchKernelGGL((propose_kernel<P, PT, MALA, 64, F8, true>), grid, dim3(256), 0, st, a);
    else hipLaunchKernelGGL((propose_kernel<P, PT, MALA, 64, F8, false>), grid, dim3(256), 0, st, a);
  }
}

void launch_propose(Prec prec, bool mala, const ProposeArgs &a, hipStream_t st) {
  if (prec == Prec::F64) {
    if (mala) launch_propose_t<Prec::F64, double, true>(a, st);
    else launch_propose_t<Prec::F64, double, false>(a, st);
  } else if (prec == Prec::F32) {
    if (mala) launch_propose_t<Prec::F32, float, true>(a, st);
    else launch_propose_t<Prec::F32, float, false>(a, st);
  } else {
    if (mala) launch_propose_t<Prec::BF16X2, float, true>(a, st);
    else if (a.f8_terms > 0) launch_propose_t<Prec::BF16X2, float, false, true>(a, st);
    else launch_propose_t<Prec::BF16X2, float, false>(a, st);
  }
}

template <Prec P, typename PT, bool MALA, bool NEXT, int LP, bool F8, bool VR>
static void launch_accept_vr(int S, const AcceptArgs &a, const ProposeArgs &na, hipStream_t st) {
  const int grid = grid_rows(a.M, 256 / LP);
  switch (S) {
    case 1: hipLaunchKernelGGL((accept_kernel<P, PT, MALA, 0, NEXT, LP, F8, VR>), dim3(grid), dim3(256), 0, st, a, na); break;
    case 2: hipLaunchKernelGGL((accept_kernel<P, PT, MALA, 2, NEXT, LP, F8, VR>), dim3(grid), dim3(256), 0, st, a, na); break;
    case 4: hipLaunchKernelGGL((accept_kernel<P, PT, MALA, 4, NEXT, LP, F8, VR>), dim3(grid), dim3(256), 0, st, a, na); break;
    case 8: hipLaunchKernelGGL((accept_kernel<P, PT, MALA, 8, NEXT, LP, F8, VR>), dim3(grid), dim3(256), 0, st, a, na); break;
  }
}

template <Prec P, typename PT, bool MALA, bool NEXT, int LP, bool F8>
static void launch_accept_lp(int S, const AcceptArgs &a, const ProposeArgs &na, hipStream_t st) {
  if ((a.p & 3) == 0) launch_accept_vr<P, PT, MALA, NEXT, LP, F8, true>(S, a, na, st);   // whole blocks
  else launch_accept_vr<P, PT, MALA, NEXT, LP, F8, false>(S, a, na, st);
}

// S: the number of partial sums to combine (1: the contraction wrote whole results).
template <Prec P, typename PT, bool MALA, bool NEXT, bool F8 = false>
static void launch_accept_t(int S, int PP, const AcceptArgs &a, const ProposeArgs &na, hipStream_t st) {
  if (row_lanes(PP) == 32) launch_accept_lp<P, PT, MALA, NEXT, 32, F8>(S, a, na, st);
  else launch_accept_lp<P, PT, MALA, NEXT, 64, F8>(S, a, na, st);
}

template <Prec P, typename PT>
static void launch_accept_p(bool mala, int S, int PP, const AcceptArgs &a, const ProposeArgs *next,
                            hipStream_t st) {
  const ProposeArgs none{};
  if (next) {
    if constexpr (P == Prec::BF16X2) {
      if (!mala && next->f8_terms > 0) {
        launch_accept_t<P, PT, false, true, true>(S, PP, a, *next, st);
        return;
      }
    }
    if (mala) launch_accept_t<P, PT, true, true>(S, PP, a, *next, st);
    else launch_accept_t<P, PT, false, true>(S, PP, a, *next, st);
  } else {
    if (mala) launch_accept_t<P, PT, true, false>(S, PP, a, none, st);
    else launch_accept_t<P, PT, false, false>(S, PP, a, none, st);
  }
}

hipError_t launch_accept(Prec prec, bool mala, int PP, const AcceptArgs &a, const ProposeArgs *next, hipStream_t st) {
  const int S = a.spl_part != nullptr ? a.S : 1;
  if (S != 1 && S != 2 && S != 4 && S != 8) return hipErrorInvalidValue;   // split counts are powers of two <= 8
  if (prec == Prec::F64) launch_accept_p<Prec::F64, double>(mala, S, PP, a, next, st);
  else if (prec == Prec::F32 || !next) launch_accept_p<Prec::F32, float>(mala, S, PP, a, next, st);
  else launch_accept_p<Prec::BF16X2, float>(mala, S, PP, a, next, st);   // no operand written: one instance
  return hipSuccess;
}

int reweight_blocks(int M, int p) {
  const int rows = rw_rows(bw_lanes(p));
  return std::max(1, (M + rows - 1) / rows);
}

template <int LP>
static void launch_reweight_lp(bool f64, const ReweightArgs &a, hipStream_t st) {
  const dim3 grid(reweight_blocks(a.M, a.p));
  const dim3 block(rw_rows(LP) * LP);
  if (f64) hipLaunchKernelGGL((reweight_kernel<double, LP>), grid, block, 0, st, a);
  else hipLaunchKernelGGL((reweight_kernel<float, LP>), grid, block, 0, st, a);
}

void launch_reweight(bool f64, const ReweightArgs &a, hipStream_t st) {
  switch (bw_lanes(a.p)) {
    case 8: launch_reweight_lp<8>(f64, a, st); break;
    case 16: launch_reweight_lp<16>(f64, a, st); break;
    case 32: launch_reweight_lp<32>(f64, a, st); break;
    default: launch_reweight_lp<64>(f64, a, st); break;
  }
  hipLaunchKernelGGL(lse_finalize_kernel, dim3(1), dim3(kFin), 0, st, a.part, reweight_blocks(a.M, a.p), a.M,
                     a.ess_frac, a.scalars);
}

template <int LP>
static void launch_search_lp(bool f64, const ResampleArgs &a, hipStream_t st) {
  const dim3 grid((a.M + kBW / LP - 1) / (kBW / LP));
  if (f64) hipLaunchKernelGGL((search_gather_kernel<double, LP>), grid, dim3(kBW), 0, st, a);
  else hipLaunchKernelGGL((search_gather_kernel<float, LP>), grid, dim3(kBW), 0, st, a);
}

void launch_resample(bool f64, const ResampleArgs &a, hipStream_t st) {
  // ept weights per thread so that a pass has at most kResampleBlocks workgroups
  const int ept = std::max(1, (a.M + kBW * kResampleBlocks - 1) / (kBW * kResampleBlocks));
  const int G = (a.M + kBW * ept - 1) / (kBW * ept);
  if (a.mode == 1) hipLaunchKernelGGL(wmax_kernel, dim3(G), dim3(kBW), 0, st, a.w, a.M, a.wpart);
  hipLaunchKernelGGL(quantise_kernel, dim3(G), dim3(kBW), 0, st, a.mode, a.logw, a.w, a.wpart, a.M, a.K, ept,
                     a.scalars, a.cdf, a.btot);
  hipLaunchKernelGGL(cdf_scan_kernel, dim3(G), dim3(kBW), 0, st, a.M, ept, a.btot, a.cdf, a.scalars);
  switch (a.src ? bw_lanes(a.p) : 32) {
    case 8: launch_search_lp<8>(f64, a, st); break;
    case 16: launch_search_lp<16>(f64, a, st); break;
    case 32: launch_search_lp<32>(f64, a, st); break;
    default: launch_search_lp<64>(f64, a, st); break;
  }
}

// 64-row chunks, every column in one workgroup
int moments_chunks(int M) { return std::max(1, (M + kMomRows - 1) / kMomRows); }

void launch_moments(bool f64, const void *beta, double *logw, const double *shift, int M, int p, double *part,
                    double *mean, double *var, double *sigma, double sigma_floor, hipStream_t st) {
  const int nch = moments_chunks(M);
  if (f64) {
    hipLaunchKernelGGL(moments_partial_kernel<double>, dim3(nch), dim3(kBW), 0, st, (const double *)beta, logw,
                       shift, M, p, part);
    hipLaunchKernelGGL(moments_final_kernel<double>, dim3((p + 3) / 4), dim3(256), 0, st,
                       (const double *)beta, part, nch, p, mean, var, sigma, sigma_floor);
  } else {
    hipLaunchKernelGGL(moments_partial_kernel<float>, dim3(nch), dim3(kBW), 0, st, (const float *)beta, logw,
                       shift, M, p, part);
    hipLaunchKernelGGL(moments_final_kernel<float>, dim3((p + 3) / 4), dim3(256), 0, st,
                       (const float *)beta, part, nch, p, mean, var, sigma, sigma_floor);
  }
}

void launch_count(const int *cnt, int M, const double *ll, long long *out, hipStream_t st) {
  hipLaunchKernelGGL(count_kernel, dim3(1), dim3(1024), 0, st, cnt, M, ll, out);
}

void launch_fill(double *x, int n, double v, hipStream_t st) {
  hipLaunchKernelGGL(fill_kernel, dim3((n + 255) / 256), dim3(256), 0, st, x, n, v);
}
template <typename PT>
__global__ void move_consts_kernel(const double *__restrict__ sigma, int p, int PP, double step, double sqrt_step,
                                   PT *__restrict__ mc, int *__restrict__ acc, int N) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t < N) acc[t] = 0;
  if (t < PP) {
    // each product in the order the proposal and decision formulas take it per coefficient
    const PT st = static_cast<PT>(step), sst = static_cast<PT>(sqrt_step);
    const PT sg = t < p ? static_cast<PT>(sigma[t]) : PT(0);
    mc[t] = PT(0.5) * st * sg * sg;
    mc[PP + t] = pre_div(PT(2) * st * sg * sg);
    mc[2 * PP + t] = sst * sg;
    mc[3 * PP + t] = st * sg;
  }
}

void launch_move_consts(bool f64, const double *sigma, int p, int PP, double step, double sqrt_step, void *mc,
                        int *acc, int N, hipStream_t st) {
  const int n = std::max(N, PP);
  const dim3 grid((n + 255) / 256);
  if (f64)
    hipLaunchKernelGGL(move_consts_kernel<double>, grid, dim3(256), 0, st, sigma, p, PP, step, sqrt_step,
                       static_cast<double *>(mc), acc, N);
  else
    hipLaunchKernelGGL(move_consts_kernel<float>, grid, dim3(256), 0, st, sigma, p, PP, step, sqrt_step,
                       static_cast<float *>(mc), acc, N);
}

void launch_zero_int(int *x, int n, hipStream_t st) {
  hipLaunchKernelGGL(zero_int_kernel, dim3((n + 255) / 256), dim3(256), 0, st, x, n);
}

void launch_convert(bool src_f64, const void *src, void *dst, size_t n, hipStream_t st) {
  const int grid = static_cast<int>(std::min<size_t>((n + 255) / 256, 65535));
  if (src_f64)
    hipLaunchKernelGGL((convert_kernel<double, float>), dim3(grid), dim3(256), 0, st, (const double *)src,
                       (float *)dst, n);
  else
    hipLaunchKernelGGL((convert_kernel<float, double>), dim3(grid), dim3(256), 0, st, (const float *)src,
                       (double *)dst, n);
}

void launch_add_prior(bool beta_f64, bool g_f64, const void *beta, int M, int p, const Prior &pr, void *g,
                      const double *ll, double *logpost, hipStream_t st) {
  const int grid = grid_rows(M, 4);
#define SPA_ADDP(BT, GT)                                                                                 \
  hipLaunchKernelGGL((add_prior_kernel<BT, GT>), dim3(grid), dim3(256), 0, st, (const BT *)beta, M, p, pr, \
                     (GT *)g, ll, logpost)
  if (beta_f64) {
    if (g_f64) SPA_ADDP(double, double); else SPA_ADDP(double, float);
  } else {
    if (g_f64) SPA_ADDP(float, double); else SPA_ADDP(float, float);
  }
#undef SPA_ADDP
}

void launch_philox(const uint32_t *ctr, int M, uint32_t k0, uint32_t k1, uint32_t *out, hipStream_t st) {
  hipLaunchKernelGGL(philox_kernel, dim3((M + 255) / 256), dim3(256), 0, st, ctr, M, k0, k1, out);
}

}  // namespace spa
