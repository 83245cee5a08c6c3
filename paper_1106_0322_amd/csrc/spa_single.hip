// The paper's own move kernel (Section 4.1): cycles of single-coordinate random-walk
// Metropolis-Hastings updates, beta'_j = beta_j + step z for j = 1..p in order, each
// costing O(n) through the incrementally updated linear predictor eta = X_std beta.
//
// One wave64 per particle.  The particle's eta (and e^{-|eta|}) live in registers for
// the whole launch: lane l holds individuals l, l+64, ..., so an update reads one
// standardised genotype column (contiguous bytes per lane group), forms the likelihood
// difference with one exponential per individual (the cached e^{-|eta|} gives the other
// softplus term) and one logarithm per lane (the ratio terms are multiplied first), and
// reduces it across the wave.
//
// The FP32 instance uses softplus(z) = z/2 + |z|/2 + log(1 + e^{-|z|}): with d_k = delta x_k
// the likelihood difference of a move is
//   delta c_j + (1/2) sum_k (|eta_k| - |eta_k + d_k|) + log(prod_k (1 + e^{-|eta_k|}) / prod_k (1 + e^{-|eta_k + d_k|})),
// c_j = sum_k (y_k - 1/2) x_kj one number per column; sum_k |eta_k| and the product over the
// current state are kept per lane (replaced on acceptance by the proposal's), the proposal's
// product accumulated with FMAs and the two divided once per lane; eta is kept in log2
// units so that e^{-|eta|} is one exp2.  Per individual and move: one FMA for the new eta,
// one exponential, one FMA for the product and one add.  The particle's coefficients are held by lane j mod 64 and
// broadcast with readlane; the cycle's normals and uniforms are drawn up front, one
// Philox block per coordinate, by the lane holding that coordinate.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <type_traits>

#include "spa_common.hpp"
#include "spa_lanes.hpp"
#include "spa_single.hpp"

namespace spa {

namespace {

constexpr int kMaxCoordBlocks = 8;   // p <= 512

__device__ __forceinline__ float bcast(float v, int lane) {
  return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), lane));
}
__device__ __forceinline__ double bcast(double v, int lane) {
  const long long b = __double_as_longlong(v);
  const int lo = __builtin_amdgcn_readlane(static_cast<int>(b & 0xffffffffll), lane);
  const int hi = __builtin_amdgcn_readlane(static_cast<int>(b >> 32), lane);
  return __longlong_as_double((static_cast<long long>(hi) << 32) | static_cast<unsigned int>(lo));
}

__device__ __forceinline__ float exp_neg(float x) { return __builtin_amdgcn_exp2f(-1.4426950408889634f * x); }
__device__ __forceinline__ double exp_neg(double x) { return exp(-x); }
__device__ __forceinline__ float log_t(float x) { return 0.6931471805599453f * __builtin_amdgcn_logf(x); }
__device__ __forceinline__ double log_t(double x) { return log(x); }
__device__ __forceinline__ float ratio(float num, float den) { return num * __builtin_amdgcn_rcpf(den); }
__device__ __forceinline__ double ratio(double num, double den) { return num / den; }

// Lane-identical wave sums (xor butterfly: every lane adds the same pairs, commutatively).
__device__ __forceinline__ float wave_sum_t(float v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, kWave);
  return v;
}
__device__ __forceinline__ double wave_sum_t(double v) { return wave_sum(v); }

// log u and log Gt(b') - log Gt(b) in the particle precision (FP64: the oracle's
// arithmetic, so the decisions match it; FP32: one logarithm of a ratio each).
__device__ __forceinline__ double log_uniform(uint32_t w, double) {
  return log((static_cast<double>(w) + 0.5) * 0x1p-32);
}
__device__ __forceinline__ float log_uniform(uint32_t w, float) {
  return log_t((static_cast<float>(w) + 0.5f) * 0x1p-32f);
}
__device__ __forceinline__ double prior_diff(double bn, double b, const Prior &pr) {
  return gt_logpdf(bn, pr) - gt_logpdf(b, pr);
}
__device__ __forceinline__ float prior_diff(float bn, float b, const Prior &pr) {
  if (pr.inf) return -(fabsf(bn) - fabsf(b)) * static_cast<float>(1.0 / pr.lam);
  const float ac = static_cast<float>(pr.a * pr.lam);
  return -static_cast<float>(pr.a + 1.0) * log_t(ratio(ac + fabsf(bn), ac + fabsf(b)));
}

// Box-Muller cosine normal from (w0, w1), in the particle precision.
__device__ __forceinline__ double draw_normal(uint4 w, double) {
  const double r = sqrt(-2.0 * log((static_cast<double>(w.x) + 1.0) * 0x1p-32));
  return r * cos(6.283185307179586476925286766559 * (static_cast<double>(w.y) * 0x1p-32));
}
__device__ __forceinline__ float draw_normal(uint4 w, float) {
  const float l = __builtin_amdgcn_logf((static_cast<float>(w.x) + 1.0f) * 0x1p-32f);
  return __builtin_amdgcn_sqrtf(-1.3862943611198906f * l) * __builtin_amdgcn_cosf(static_cast<float>(w.y) * 0x1p-32f);
}

template <typename PT, int R>
__global__ __launch_bounds__(256) void single_site_kernel(SingleSiteArgs a) {
  const int lane = threadIdx.x & 63;
  const int i = blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6);
  if (i >= a.M) return;
  const int n = a.n, n_pad = a.n_pad, p = a.p;
  const PT *xs = reinterpret_cast<const PT *>(a.xs);   // p x n_pad, zero padded; n_pad = 64 R
  const PT *yv = reinterpret_cast<const PT *>(a.yv);
  PT *beta = reinterpret_cast<PT *>(a.beta) + (size_t)i * p;
  const Prior pr = a.prior;
  const PT step = static_cast<PT>(a.step);

  // coefficients: lane l holds beta_j for j = l + 64 m
  PT bv[kMaxCoordBlocks];
#pragma unroll
  for (int m = 0; m < kMaxCoordBlocks; ++m) {
    const int j = lane + 64 * m;
    bv[m] = j < p ? beta[j] : PT(0);
  }
  // linear predictor of this particle
  PT eta[R], em[R], yk[R];
#pragma unroll
  for (int r = 0; r < R; ++r) {
    eta[r] = PT(0);
    const int k = lane + 64 * r;
    yk[r] = yv[k];
  }
#pragma unroll
  for (int m = 0; m < kMaxCoordBlocks; ++m) {
    if (64 * m >= p) break;
    for (int jl = 0; jl < 64 && 64 * m + jl < p; ++jl) {
      const int j = 64 * m + jl;
      const PT bj = bcast(bv[m], jl);
      const PT *col = xs + (size_t)j * n_pad;
#pragma unroll
      for (int r = 0; r < R; ++r) {
        const int k = lane + 64 * r;
        eta[r] += bj * col[k];
      }
    }
  }
  int cnt = 0;
  if constexpr (std::is_same<PT, float>::value) {
    constexpr float kL2e = 1.4426950408889634f, kLn2 = 0.6931471805599453f;
    float sa = 0.0f;   // this lane's sum of |eta| (log2 units)
#pragma unroll
    for (int r = 0; r < R; ++r) {
      eta[r] *= kL2e;
      em[r] = __builtin_amdgcn_exp2f(-fabsf(eta[r]));
      sa += fabsf(eta[r]);
    }
    // this lane's product of (1 + e^-|eta|), formed in the same order as a proposal's (so an
    // accepted proposal's product is exactly the product of the new state)
    float pm = 1.0f;
#pragma unroll
    for (int r = 0; r < R; ++r) pm = fmaf(pm, em[r], pm);
    for (int c = 0; c < a.cycles; ++c) {
      const uint32_t cyc = static_cast<uint32_t>(a.cycle0 + c);
      // per coordinate, by the lane holding it: the move delta, log Gt(b + delta) - log Gt(b)
      // and log u (a coordinate changes only at its own update, so these are the values its
      // update needs)
      float dz[kMaxCoordBlocks], dp[kMaxCoordBlocks], lu[kMaxCoordBlocks];
#pragma unroll
      for (int m = 0; m < kMaxCoordBlocks; ++m) {
        const int j = lane + 64 * m;
        dz[m] = dp[m] = lu[m] = 0.0f;
        if (64 * m < p && j < p) {
          const uint4 w = philox4x32_10(make_uint4(static_cast<uint32_t>(i), static_cast<uint32_t>(j), cyc,
                                                   word3(a.t, kTagSingleSite)),
                                        a.k0, a.k1);
          dz[m] = step * draw_normal(w, 0.0f);
          dp[m] = prior_diff(bv[m] + dz[m], bv[m], pr);
          lu[m] = log_uniform(w.z, 0.0f);
        }
      }
#pragma unroll
      for (int m = 0; m < kMaxCoordBlocks; ++m) {
        if (64 * m >= p) break;
        for (int jl = 0; jl < 64 && 64 * m + jl < p; ++jl) {
          const int j = 64 * m + jl;
          const float delta = bcast(dz[m], jl);
          const float dl = delta * kL2e;
          const PT *col = xs + (size_t)j * n_pad;
          float e1[R], en[R];
          float den = 1.0f, sn = 0.0f;
#pragma unroll
          for (int r = 0; r < R; ++r) {
            const int k = lane + 64 * r;
            const float x = col[k];
            e1[r] = fmaf(dl, x, eta[r]);
            en[r] = __builtin_amdgcn_exp2f(-fabsf(e1[r]));
            den = fmaf(den, en[r], den);
            sn += fabsf(e1[r]);
          }
          const float part = kLn2 * (0.5f * (sa - sn) + __builtin_amdgcn_logf(pm * __builtin_amdgcn_rcpf(den)));
          const float dll = wave_total_f32(part) + delta * a.cs[j];
          if (bcast(lu[m], jl) < dll + bcast(dp[m], jl)) {   // uniform across the wave (lane-identical sums)
#pragma unroll
            for (int r = 0; r < R; ++r) eta[r] = e1[r];
            sa = sn;
            pm = den;
            if (lane == jl) bv[m] += dz[m];
            ++cnt;
          }
        }
      }
    }
#pragma unroll
    for (int r = 0; r < R; ++r) eta[r] *= kLn2;   // back to natural units for the write-back
  } else {
#pragma unroll
  for (int r = 0; r < R; ++r) em[r] = exp_neg(fabs(eta[r]));

  for (int c = 0; c < a.cycles; ++c) {
    const uint32_t cyc = static_cast<uint32_t>(a.cycle0 + c);
    // per coordinate, by the lane holding it: the move, the prior difference and log u
    PT dz[kMaxCoordBlocks], dp[kMaxCoordBlocks], lu[kMaxCoordBlocks];
#pragma unroll
    for (int m = 0; m < kMaxCoordBlocks; ++m) {
      const int j = lane + 64 * m;
      dz[m] = dp[m] = lu[m] = PT(0);
      if (64 * m < p && j < p) {
        const uint4 w = philox4x32_10(make_uint4(static_cast<uint32_t>(i), static_cast<uint32_t>(j), cyc,
                                                 word3(a.t, kTagSingleSite)),
                                      a.k0, a.k1);
        dz[m] = step * draw_normal(w, PT(0));
        dp[m] = prior_diff(bv[m] + dz[m], bv[m], pr);
        lu[m] = log_uniform(w.z, PT(0));
      }
    }
#pragma unroll
    for (int m = 0; m < kMaxCoordBlocks; ++m) {
      if (64 * m >= p) break;
      for (int jl = 0; jl < 64 && 64 * m + jl < p; ++jl) {
        const int j = 64 * m + jl;
        const PT delta = bcast(dz[m], jl);
        const PT *col = xs + (size_t)j * n_pad;
        PT d[R], en[R];
        PT prod = PT(1), lin = PT(0);
#pragma unroll
        for (int r = 0; r < R; ++r) {
          const int k = lane + 64 * r;
          const PT x = col[k];
          d[r] = delta * x;
          const PT e1 = eta[r] + d[r];
          en[r] = exp_neg(fabs(e1));
          // softplus(eta) - softplus(eta + d) = max(eta,0) - max(eta+d,0) + log((1+em)/(1+en))
          prod *= ratio(PT(1) + em[r], PT(1) + en[r]);
          lin += yk[r] * d[r] + (fmax(eta[r], PT(0)) - fmax(e1, PT(0)));
        }
        const PT dll = wave_sum_t(lin + log_t(prod));
        if (bcast(lu[m], jl) < dll + bcast(dp[m], jl)) {   // uniform across the wave (lane-identical sums)
#pragma unroll
          for (int r = 0; r < R; ++r) {
            eta[r] += d[r];
            em[r] = en[r];
          }
          if (lane == jl) bv[m] += dz[m];
          ++cnt;
        }
      }
    }
  }
  }

  // write back: coefficients, log-likelihood from the tracked predictor, accept count
#pragma unroll
  for (int m = 0; m < kMaxCoordBlocks; ++m) {
    const int j = lane + 64 * m;
    if (j < p) beta[j] = bv[m];
  }
  double ll = 0.0;
#pragma unroll
  for (int r = 0; r < R; ++r) {
    const int k = lane + 64 * r;
    if (k < n) {
      const double e = static_cast<double>(eta[r]);
      ll += static_cast<double>(yk[r]) * e - (fmax(e, 0.0) + log1p(exp(-fabs(e))));
    }
  }
  ll = wave_sum(ll);
  if (lane == 0) {
    a.ll[i] = ll;
    a.acc_cnt[i] += cnt;
  }
}

// Standardised genotype columns for the single-site kernel: xs[j][k] = (X_kj - mu_j) / s_j
// in the particle precision (rounded once from FP64), zero for padded individuals.
template <typename PT>
__global__ void std_cols_kernel(const uint8_t *__restrict__ X, int n, int p, int n_pad,
                                const double *__restrict__ mu, const double *__restrict__ s,
                                PT *__restrict__ xs) {
  const size_t total = (size_t)p * n_pad;
  for (size_t idx = blockIdx.x * (size_t)blockDim.x + threadIdx.x; idx < total;
       idx += (size_t)gridDim.x * blockDim.x) {
    const int j = static_cast<int>(idx / n_pad), k = static_cast<int>(idx % n_pad);
    xs[idx] = k < n ? static_cast<PT>((static_cast<double>(X[(size_t)k * p + j]) - mu[j]) / s[j]) : PT(0);
  }
}

// c_j = sum_{k < n} (y_k - 1/2) xs_jk: one wave per column, FP64 sums of the FP32 values.
__global__ __launch_bounds__(64) void lin_cols_kernel(const float *__restrict__ xs, const float *__restrict__ yv,
                                                     int n, int n_pad, float *__restrict__ cs) {
  const int j = blockIdx.x, lane = threadIdx.x;
  double acc = 0.0;
  for (int k = lane; k < n; k += 64)
    acc += (static_cast<double>(yv[k]) - 0.5) * static_cast<double>(xs[(size_t)j * n_pad + k]);
  acc = wave_sum(acc);
  if (lane == 0) cs[j] = static_cast<float>(acc);
}

template <typename PT, int R>
static void launch_r(const SingleSiteArgs &a, hipStream_t st) {
  hipLaunchKernelGGL((single_site_kernel<PT, R>), dim3((a.M + 3) / 4), dim3(256), 0, st, a);
}

template <typename PT>
static hipError_t launch_t(const SingleSiteArgs &a, hipStream_t st) {
  switch (a.n_pad) {   // the columns are padded to exactly 64 R individuals
    case 64 * 4: launch_r<PT, 4>(a, st); break;
    case 64 * 8: launch_r<PT, 8>(a, st); break;
    case 64 * 16: launch_r<PT, 16>(a, st); break;
    case 64 * 32: launch_r<PT, 32>(a, st); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

}  // namespace

int single_site_max_n() { return 64 * 32; }

int single_site_rows(int n) {
  for (int R = 4; R <= 32; R *= 2)
    if (n <= 64 * R) return 64 * R;
  return -1;
}

hipError_t launch_single_site(bool f64, const SingleSiteArgs &a, hipStream_t st) {
  if (a.p > 64 * kMaxCoordBlocks) return hipErrorInvalidValue;
  return f64 ? launch_t<double>(a, st) : launch_t<float>(a, st);
}

hipError_t launch_std_cols(bool f64, const uint8_t *X, int n, int p, int n_pad, const double *mu,
                           const double *s, void *xs, hipStream_t st) {
  const size_t total = (size_t)p * n_pad;
  const int grid = static_cast<int>((total + 255) / 256 < 4096 ? (total + 255) / 256 : 4096);
  if (f64)
    hipLaunchKernelGGL(std_cols_kernel<double>, dim3(grid), dim3(256), 0, st, X, n, p, n_pad, mu, s,
                       reinterpret_cast<double *>(xs));
  else
    hipLaunchKernelGGL(std_cols_kernel<float>, dim3(grid), dim3(256), 0, st, X, n, p, n_pad, mu, s,
                       reinterpret_cast<float *>(xs));
  return hipGetLastError();
}

hipError_t launch_lin_cols(const float *xs, const float *yv, int n, int p, int n_pad, float *cs, hipStream_t st) {
  hipLaunchKernelGGL(lin_cols_kernel, dim3(p), dim3(64), 0, st, xs, yv, n, n_pad, cs);
  return hipGetLastError();
}

}  // namespace spa
