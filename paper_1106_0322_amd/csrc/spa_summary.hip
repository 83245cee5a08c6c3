// Sparsity-path summaries of a weighted particle set (Section 5): weighted quantiles
// F^-1(alpha) per coefficient (absolute medians, credible intervals) and concentrations
// V(Delta) = 1 - Pr(|beta_j| < Delta), on the GPU.
//
// Exactness: the weights are quantised to integers q_i = floor((w_i / max w) 2^K),
// K = 63 - ceil(log2 M), so every partial sum is an exact 64-bit integer and no result
// depends on summation order.  The alpha-quantile is the smallest value whose cumulative
// q reaches ceil(alpha * C) (C = sum q, the product taken exactly in 128 bits).
//
// Selection is a most-significant-digit radix select on order-preserving integer keys of
// the values (8-bit digits: 4 passes for FP32 values, 8 for FP64): each pass builds, per
// coefficient and level, the weighted histogram of the next digit over the values that
// still match the level's prefix, then picks the bucket where the cumulative weight
// crosses the threshold.  The values are first transposed into per-coefficient key
// columns so that every pass reads contiguous memory.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <algorithm>

#include "spa_common.hpp"
#include "spa_summary.hpp"

namespace spa {

namespace {

constexpr int kPrepThreads = 1024;
constexpr int kHistThreads = 256;
constexpr int kChunk = 4096;         // values per histogram workgroup
constexpr int kBuckets = 256;

__device__ __forceinline__ uint32_t key_of(float v) {
  uint32_t u = __float_as_uint(v);
  if (u == 0x80000000u) u = 0u;      // -0 and +0 are one value
  return (u & 0x80000000u) ? ~u : (u | 0x80000000u);
}
__device__ __forceinline__ uint64_t key_of(double v) {
  uint64_t u = static_cast<uint64_t>(__double_as_longlong(v));
  if (u == 0x8000000000000000ull) u = 0ull;
  return (u & 0x8000000000000000ull) ? ~u : (u | 0x8000000000000000ull);
}
__device__ __forceinline__ double value_of_key(uint32_t k) {
  const uint32_t u = (k & 0x80000000u) ? (k & 0x7fffffffu) : ~k;
  return static_cast<double>(__uint_as_float(u));
}
__device__ __forceinline__ double value_of_key(uint64_t k) {
  const uint64_t u = (k & 0x8000000000000000ull) ? (k & 0x7fffffffffffffffull) : ~k;
  return __longlong_as_double(static_cast<long long>(u));
}

// ceil(alpha * C) exactly: alpha = m 2^(e - 1075) from its bit pattern (alpha in (0, 1]).
__device__ __forceinline__ uint64_t exact_threshold(double alpha, uint64_t C) {
  const uint64_t bits = static_cast<uint64_t>(__double_as_longlong(alpha));
  const int e = static_cast<int>((bits >> 52) & 0x7ff);
  uint64_t m = bits & ((1ull << 52) - 1);
  int shift;
  if (e == 0) {
    shift = 1074;                     // subnormal: m 2^-1074
  } else {
    m |= (1ull << 52);
    shift = 1075 - e;
  }
  const unsigned __int128 prod = static_cast<unsigned __int128>(m) * C;
  if (shift >= 128) return prod != 0 ? 1ull : 0ull;
  uint64_t t = static_cast<uint64_t>(prod >> shift);
  const unsigned __int128 rem = prod & ((static_cast<unsigned __int128>(1) << shift) - 1);
  if (rem != 0) ++t;
  return t;
}

__device__ __forceinline__ uint64_t wave_sum_u64(uint64_t v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, kWave);
  return v;
}

// One workgroup: max weight, validation, quantised weights, their total and the exact
// thresholds of every level.  st->flags bit 0: invalid weights.
__global__ __launch_bounds__(kPrepThreads) void sq_prepare_kernel(const double *__restrict__ w, int M,
                                                                   bool logw, int K, SqLevels lv,
                                                                   uint64_t *__restrict__ q,
                                                                   SqState *__restrict__ st) {
  __shared__ double smax[kPrepThreads / 64];
  __shared__ uint64_t ssum[kPrepThreads / 64];
  __shared__ int sbad[kPrepThreads / 64];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  double mx = logw ? -INFINITY : 0.0;
  int bad = 0;
  for (int i = tid; i < M; i += kPrepThreads) {
    const double v = w[i];
    if (logw ? (isnan(v) || v == INFINITY) : (!(v >= 0.0) || !isfinite(v))) bad = 1;
    else mx = fmax(mx, v);
  }
  mx = wave_max(mx);
  bad = wave_sum_int(bad);
  if (lane == 0) {
    smax[wave] = mx;
    sbad[wave] = bad;
  }
  __syncthreads();
  mx = logw ? -INFINITY : 0.0;
  bad = 0;
  for (int k = 0; k < kPrepThreads / 64; ++k) {
    mx = fmax(mx, smax[k]);
    bad += sbad[k];
  }
  if (bad > 0 || (logw ? mx == -INFINITY : !(mx > 0.0))) {
    if (tid == 0) st->flags = 1;
    return;
  }
  uint64_t acc = 0;
  for (int i = tid; i < M; i += kPrepThreads) {
    const double r = logw ? exp(w[i] - mx) : __ddiv_rn(w[i], mx);   // correctly rounded division
    const uint64_t qi = static_cast<uint64_t>(floor(ldexp(r, K)));
    q[i] = qi;
    acc += qi;
  }
  acc = wave_sum_u64(acc);
  if (lane == 0) ssum[wave] = acc;
  __syncthreads();
  if (tid == 0) {
    uint64_t C = 0;
    for (int k = 0; k < kPrepThreads / 64; ++k) C += ssum[k];
    st->flags = 0;
    st->total = C;
    for (int l = 0; l < lv.L; ++l) st->thr[l] = exact_threshold(lv.alpha[l], C);
  }
}

// Transpose values (M x p row-major) into key columns (p x M), and count the quantised
// weight of |v| < Delta_d per coefficient (exact integer sums, any order).
template <typename VT, typename KT>
__global__ void sq_keys_kernel(const VT *__restrict__ vals, int M, int p, const uint64_t *__restrict__ q,
                               SqLevels lv, KT *__restrict__ keys, unsigned long long *__restrict__ inside) {
  __shared__ VT tile[32][33];
  const int i0 = blockIdx.x * 32, j0 = blockIdx.y * 32;
  const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;   // 32 x 8 threads
  for (int r = ty; r < 32; r += 8) {
    const int i = i0 + r, j = j0 + tx;
    tile[r][tx] = (i < M && j < p) ? vals[(size_t)i * p + j] : VT(0);
  }
  __syncthreads();
  for (int r = ty; r < 32; r += 8) {
    const int j = j0 + r, i = i0 + tx;
    const bool ok = i < M && j < p;
    const VT v = tile[tx][r];
    if (ok) keys[(size_t)j * M + i] = key_of(v);
    // concentrations: lanes tx of one row r share coefficient j
    for (int d = 0; d < lv.D; ++d) {
      uint64_t s = (ok && fabs(static_cast<double>(v)) < lv.delta[d]) ? q[i] : 0ull;
#pragma unroll
      for (int o = 16; o > 0; o >>= 1) s += __shfl_xor(s, o, 32);
      if (tx == 0 && s != 0 && j < p)
        atomicAdd(&inside[(size_t)d * p + j], static_cast<unsigned long long>(s));
    }
  }
}

// Weighted digit histograms of one pass.  grid = (chunks of kChunk values, p).
template <typename KT>
__global__ __launch_bounds__(kHistThreads) void sq_hist_kernel(const KT *__restrict__ keys, int M, int p,
                                                               const uint64_t *__restrict__ q, int L,
                                                               int shift, const SqSel *__restrict__ sel,
                                                               unsigned long long *__restrict__ hist) {
  __shared__ unsigned long long h[kSqMaxLevels][kBuckets];
  const int j = blockIdx.y;
  const int tid = threadIdx.x;
  for (int k = tid; k < L * kBuckets; k += kHistThreads) h[k / kBuckets][k % kBuckets] = 0ull;
  __syncthreads();
  KT pre[kSqMaxLevels];
  for (int l = 0; l < L; ++l) pre[l] = static_cast<KT>(sel[(size_t)j * kSqMaxLevels + l].prefix);
  const int hi_shift = shift + 8;   // bits above the current digit
  const KT *kc = keys + (size_t)j * M;
  const int b0 = blockIdx.x * kChunk, b1 = min(M, b0 + kChunk);
  for (int i = b0 + tid; i < b1; i += kHistThreads) {
    const KT k = kc[i];
    const uint64_t w = q[i];
    if (w == 0) continue;
    const int dig = static_cast<int>((k >> shift) & 0xff);
    const KT hi = (hi_shift >= static_cast<int>(8 * sizeof(KT))) ? KT(0) : (k >> hi_shift);
    for (int l = 0; l < L; ++l)
      if (hi == pre[l]) atomicAdd(&h[l][dig], static_cast<unsigned long long>(w));
  }
  __syncthreads();
  for (int k = tid; k < L * kBuckets; k += kHistThreads) {
    const unsigned long long v = h[k / kBuckets][k % kBuckets];
    if (v) atomicAdd(&hist[((size_t)j * kSqMaxLevels + k / kBuckets) * kBuckets + k % kBuckets], v);
  }
}

// Pick each (coefficient, level)'s digit: the bucket where below + cumulative weight
// reaches the threshold; clears the histogram for the next pass.  One wave per pair.
template <typename KT>
__global__ void sq_select_kernel(int p, int L, int last, const SqState *__restrict__ st,
                                 SqSel *__restrict__ sel, unsigned long long *__restrict__ hist,
                                 double *__restrict__ quant) {
  const int lane = threadIdx.x & 63;
  const int pair = blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6);
  if (pair >= p * L) return;
  const int j = pair / L, l = pair % L;
  SqSel &s = sel[(size_t)j * kSqMaxLevels + l];
  unsigned long long *hb = hist + ((size_t)j * kSqMaxLevels + l) * kBuckets;
  // 4 buckets per lane, in bucket order
  uint64_t c[4], loc = 0;
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    c[k] = hb[lane * 4 + k];
    loc += c[k];
  }
  // exclusive scan of the lanes' sums
  uint64_t incl = loc;
#pragma unroll
  for (int o = 1; o < 64; o <<= 1) {
    const uint64_t v = __shfl_up(incl, o, kWave);
    if (lane >= o) incl += v;
  }
  const uint64_t excl = incl - loc;
  const uint64_t need = st->thr[l] - s.below;   // > 0 and <= the weight still in range
  int found = -1;
  uint64_t below_b = 0;
  uint64_t run = excl;
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    if (found < 0 && run + c[k] >= need) {
      found = lane * 4 + k;
      below_b = run;
    }
    run += c[k];
  }
  // the first lane holding the crossing bucket decides
  const unsigned long long ball = __ballot(found >= 0);
  const int src = ball ? __ffsll(static_cast<long long>(ball)) - 1 : 63;
  int b = __shfl(found, src, kWave);
  const uint64_t bb = __shfl(below_b, src, kWave);
  if (b < 0) b = kBuckets - 1;   // unreachable for valid weights (the range holds the target)
#pragma unroll
  for (int k = 0; k < 4; ++k) hb[lane * 4 + k] = 0ull;
  if (lane == 0) {
    s.prefix = (s.prefix << 8) | static_cast<uint64_t>(b);
    s.below += bb;
    if (last) quant[(size_t)l * p + j] = value_of_key(static_cast<KT>(s.prefix));
  }
}

__global__ void sq_conc_kernel(int p, int D, const SqState *__restrict__ st,
                               const unsigned long long *__restrict__ inside, double *__restrict__ conc) {
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= p * D) return;
  conc[k] = 1.0 - static_cast<double>(inside[k]) / static_cast<double>(st->total);
}

__global__ void sq_init_kernel(int p, SqSel *__restrict__ sel, unsigned long long *__restrict__ inside, int D) {
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k < p * kSqMaxLevels) {
    sel[k].prefix = 0;
    sel[k].below = 0;
  }
  if (k < p * D) inside[k] = 0ull;
}

// Pooled weights of the c-marginal mixture: w_ti = exp(log_z_t - max_s log_z_s + logW_ti),
// and the posterior over the scale p_t = exp(log_z_t - logsumexp(log_z)).
__global__ void sq_mixture_weights_kernel(const double *__restrict__ log_z, int T, int N,
                                          const double *__restrict__ logW, double *__restrict__ w,
                                          double *__restrict__ scale_post) {
  __shared__ double s_m, s_l;
  if (threadIdx.x == 0) {
    double m = -INFINITY;
    for (int t = 0; t < T; ++t) m = fmax(m, log_z[t]);
    double e = 0.0;
    for (int t = 0; t < T; ++t) e += exp(log_z[t] - m);
    s_m = m;
    s_l = m + log(e);
  }
  __syncthreads();
  const size_t tot = (size_t)T * N;
  for (size_t k = blockIdx.x * (size_t)blockDim.x + threadIdx.x; k < tot; k += (size_t)gridDim.x * blockDim.x) {
    const int t = static_cast<int>(k / N);
    w[k] = exp((log_z[t] - s_m) + logW[k]);
  }
  if (blockIdx.x == 0 && scale_post)
    for (int t = threadIdx.x; t < T; t += blockDim.x) scale_post[t] = exp(log_z[t] - s_l);
}

}  // namespace

int sq_key_bytes(bool f64) { return f64 ? 8 : 4; }

hipError_t launch_weighted_summaries(const SqArgs &a, hipStream_t s) {
  const int M = a.M, p = a.p, L = a.lv.L, D = a.lv.D;
  const int K = 63 - ceil_log2_ll(M);
  hipLaunchKernelGGL(sq_init_kernel, dim3((p * kSqMaxLevels + 255) / 256), dim3(256), 0, s, p, a.sel,
                     a.inside, D);
  hipLaunchKernelGGL(sq_prepare_kernel, dim3(1), dim3(kPrepThreads), 0, s, a.w, M, a.log_weights, K, a.lv, a.q,
                     a.st);
  const dim3 tg((M + 31) / 32, (p + 31) / 32);
  if (a.f64)
    hipLaunchKernelGGL((sq_keys_kernel<double, uint64_t>), tg, dim3(256), 0, s,
                       reinterpret_cast<const double *>(a.values), M, p, a.q, a.lv,
                       reinterpret_cast<uint64_t *>(a.keys), a.inside);
  else
    hipLaunchKernelGGL((sq_keys_kernel<float, uint32_t>), tg, dim3(256), 0, s,
                       reinterpret_cast<const float *>(a.values), M, p, a.q, a.lv,
                       reinterpret_cast<uint32_t *>(a.keys), a.inside);
  if (L > 0) {
    const int bits = a.f64 ? 64 : 32;
    const dim3 hg((M + kChunk - 1) / kChunk, p);
    const int sgrid = (p * L + 3) / 4;
    for (int shift = bits - 8; shift >= 0; shift -= 8) {
      const int last = shift == 0;
      if (a.f64) {
        hipLaunchKernelGGL((sq_hist_kernel<uint64_t>), hg, dim3(kHistThreads), 0, s,
                           reinterpret_cast<const uint64_t *>(a.keys), M, p, a.q, L, shift, a.sel, a.hist);
        hipLaunchKernelGGL((sq_select_kernel<uint64_t>), dim3(sgrid), dim3(256), 0, s, p, L, last, a.st, a.sel,
                           a.hist, a.quant);
      } else {
        hipLaunchKernelGGL((sq_hist_kernel<uint32_t>), hg, dim3(kHistThreads), 0, s,
                           reinterpret_cast<const uint32_t *>(a.keys), M, p, a.q, L, shift, a.sel, a.hist);
        hipLaunchKernelGGL((sq_select_kernel<uint32_t>), dim3(sgrid), dim3(256), 0, s, p, L, last, a.st, a.sel,
                           a.hist, a.quant);
      }
    }
  }
  if (D > 0)
    hipLaunchKernelGGL(sq_conc_kernel, dim3((p * D + 255) / 256), dim3(256), 0, s, p, D, a.st, a.inside, a.conc);
  return hipGetLastError();
}

hipError_t launch_mixture_weights(const double *log_z, int T, int N, const double *logW, double *w,
                                  double *scale_post, hipStream_t s) {
  const size_t tot = (size_t)T * N;
  const int grid = static_cast<int>(std::min<size_t>((tot + 255) / 256, 4096));
  hipLaunchKernelGGL(sq_mixture_weights_kernel, dim3(grid), dim3(256), 0, s, log_z, T, N, logW, w, scale_post);
  return hipGetLastError();
}

}  // namespace spa
