// Device-side building blocks shared by the sampler's HIP kernels (gfx950, wave64).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace spa {

constexpr int kWave = 64;

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef double f64x4 __attribute__((ext_vector_type(4)));

// ----------------------------------------------------------------------------
// Philox4x32-10 (Salmon, Moraes, Dror & Shaw, SC'11): ten rounds of two 32x32->64
// multiplications by 0xD2511F53 / 0xCD9E8D57, the output words being
// (hi(c2*M1) ^ c1 ^ k0, lo(c2*M1), hi(c0*M0) ^ c3 ^ k1, lo(c0*M0)); the key is advanced
// by the Weyl increments 0x9E3779B9 / 0xBB67AE85 between rounds.
// ----------------------------------------------------------------------------
__device__ __forceinline__ uint4 philox4x32_10(uint4 c, uint32_t k0, uint32_t k1) {
#pragma unroll
  for (int r = 0; r < 10; ++r) {
    if (r) {
      k0 += 0x9E3779B9u;
      k1 += 0xBB67AE85u;
    }
    // each 64-bit product is one v_mad_u64_u32 (separate low and high 32-bit multiplies
    // took two; measured 27 % faster per Philox block, same outputs)
    const uint64_t p0 = static_cast<uint64_t>(0xD2511F53u) * c.x;
    const uint64_t p1 = static_cast<uint64_t>(0xCD9E8D57u) * c.z;
    c = make_uint4(static_cast<uint32_t>(p1 >> 32) ^ c.y ^ k0, static_cast<uint32_t>(p1),
                   static_cast<uint32_t>(p0 >> 32) ^ c.w ^ k1, static_cast<uint32_t>(p0));
  }
  return c;
}

// Stream layout: counter = (particle, block, sweep, (t << 4) | tag).
enum : uint32_t { kTagNormal = 0, kTagUniform = 1, kTagResample = 2, kTagSingleSite = 3 };

__device__ __forceinline__ uint32_t word3(int t, uint32_t tag) {
  return (static_cast<uint32_t>(t) << 4) | tag;
}

// Box-Muller on two 32-bit words: r = sqrt(-2 ln((w0 + 1) 2^-32)), theta = 2 pi w1 2^-32.
__device__ __forceinline__ void box_muller(uint32_t w0, uint32_t w1, double &z0, double &z1) {
  const double u = (static_cast<double>(w0) + 1.0) * 0x1p-32;
  const double th = 6.283185307179586476925286766559 * (static_cast<double>(w1) * 0x1p-32);
  const double r = sqrt(-2.0 * log(u));
  double s, c;
  sincos(th, &s, &c);
  z0 = r * c;
  z1 = r * s;
}

__device__ __forceinline__ void box_muller(uint32_t w0, uint32_t w1, float &z0, float &z1) {
  const float u = (static_cast<float>(w0) + 1.0f) * 0x1p-32f;
  const float th = 6.28318530717958647692f * (static_cast<float>(w1) * 0x1p-32f);
  const float r = sqrtf(-2.0f * logf(u));
  float s, c;
  sincosf(th, &s, &c);
  z0 = r * c;
  z1 = r * s;
}

// ----------------------------------------------------------------------------
// Wave-level reductions (fixed butterfly order: deterministic).
// ----------------------------------------------------------------------------
__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, kWave);
  return v;
}
__device__ __forceinline__ double wave_max(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v = fmax(v, __shfl_xor(v, o, kWave));
  return v;
}
__device__ __forceinline__ int wave_sum_int(int v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, kWave);
  return v;
}

// ----------------------------------------------------------------------------
// Generalized-t prior Gt(a, c) (L1 form, centred): log p = -log(2c) - (a+1) log1p(|b|/(a c));
// a = inf: the double exponential -log(2c) - |b|/c.  inv_a = 1/a (0 encodes a = inf).
// ----------------------------------------------------------------------------
struct Prior {
  double a;      // degrees of freedom (unused when inf)
  double lam;    // scale c
  int inf;       // 1: double-exponential limit
  double log2lam;
};

__device__ __forceinline__ double gt_logpdf(double b, const Prior &pr) {
  const double x = fabs(b);
  if (pr.inf) return -pr.log2lam - x / pr.lam;
  return -pr.log2lam - (pr.a + 1.0) * log1p(x / (pr.a * pr.lam));
}

// d/db log Gt(b | a, c) = -(a+1) sign(b) / (a c + |b|), sign(0) = 0.
__device__ __forceinline__ double gt_grad(double b, const Prior &pr) {
  const double sg = (b > 0.0) ? 1.0 : ((b < 0.0) ? -1.0 : 0.0);
  if (pr.inf) return -sg / pr.lam;
  return -(pr.a + 1.0) * sg / (pr.a * pr.lam + fabs(b));
}

// Precision-generic pieces of the prior, for products of a few factors (one log per lane
// instead of one per coefficient): log Gt(b) = -log(2c) - (a+1) log(1 + |b|/(a c)).
template <typename T>
__device__ __forceinline__ T gt_factor(T b, T inv_ac) { return T(1) + fabs(b) * inv_ac; }
// x / y in the particle precision: FP64 divides; FP32 multiplies by the hardware
// reciprocal (1 ulp), the proposal and decision arithmetic of the reduced-precision
// sampler (deterministic, so the forward and reverse MALA densities use the same function).
__device__ __forceinline__ double div_t(double x, double y) { return x / y; }
__device__ __forceinline__ float div_t(float x, float y) { return x * __builtin_amdgcn_rcpf(y); }
// d/db log Gt(b) = -(a+1) sign(b) / (a c + |b|); -sign(b)/c for the double exponential.
template <typename T>
__device__ __forceinline__ T gt_grad_t(T b, T a1, T ac, int inf, T inv_c) {
  const T sg = (b > T(0)) ? T(1) : ((b < T(0)) ? T(-1) : T(0));
  if (inf) return -sg * inv_c;
  return div_t(-a1 * sg, ac + fabs(b));
}
__device__ __forceinline__ float fast_log(float x) { return __logf(x); }
__device__ __forceinline__ double fast_log(double x) { return log(x); }

// FP8 (OCP e4m3) -> float for finite normal/zero codes (the genotype codes 0/1/2 and 1
// of the ones column are all exact).
__device__ __forceinline__ float e4m3_to_float(uint8_t v) {
  const uint32_t s = v >> 7, e = (v >> 3) & 0xF, m = v & 7;
  if (e == 0 && m == 0) return s ? -0.0f : 0.0f;
  float f;
  if (e == 0) f = ldexpf(static_cast<float>(m), -9);           // subnormal: m * 2^-9
  else f = ldexpf(1.0f + static_cast<float>(m) * 0.125f, static_cast<int>(e) - 7);
  return s ? -f : f;
}

}  // namespace spa
