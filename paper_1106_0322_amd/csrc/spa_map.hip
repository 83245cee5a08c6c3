// MAP estimates under the Gt(a, c) prior by EM (Section 2.1) and the MAP path of
// Section 4.1, on the GPU, in FP64.
//
// EM: E step w_j = (a+1)/(a c + |beta_j|) (1/c for the double exponential); M step: the
// weighted-L1 logistic problem by cyclic coordinate ascent with the curvature bound n/4,
// beta_j <- S(beta_j + 4 g_j / n, 4 w_j / n), g_j = sum_k (y_k - sigma(eta_k)) X_std,kj.
//
// One workgroup (8 wave64s, two per SIMD) per start point.  Thread t keeps E_k = exp(-eta_k)
// and sigma(eta_k) = 1/(1 + E_k) of individuals t, t+512, ... in registers; the
// coefficients, the weights and the standardised values of the genotype codes live in LDS.
// A column of standardised genotypes takes only three values x_c = (c - mu_j)/s_j, c = 0,
// 1, 2, so a move beta_j += delta multiplies every E_k by one of the three constants
// exp(-delta x_c): lanes 0..3 of each wave put them (and 1 for code 3, padded individuals)
// in a four-entry table in LDS, then per individual one table read, one multiply and a
// reciprocal (hardware estimate refined by one Newton step).  The columns are read as
// one-byte codes.  As in the oracle, eta is recomputed from the coefficients at the start
// of every coordinate sweep, which also bounds the rounding of the products to one sweep.
// Each coordinate update is one block-wide reduction of g_j (a DPP sum inside each wave,
// then the 8 wave partials added as a fixed tree by every thread, so all threads take the
// same value).  A coordinate update is latency-bound: at n = 5000 it is ~4000 cycles, most
// of it the per-individual FP64 work of the waves sharing a SIMD and the barrier.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "spa_common.hpp"
#include "spa_lanes.hpp"
#include "spa_map.hpp"

namespace spa {

namespace {

constexpr int kMapThreads = 512;
constexpr int kMapWaves = kMapThreads / 64;

// 1 / (1 + e) for e >= 0 (e = +inf gives 0): hardware reciprocal (relative error near
// 2^-23) and one Newton step (error near 2^-46, squared by the step).
__device__ __forceinline__ double inv1p(double e) {
  const double d = 1.0 + e;
  if (!(d < INFINITY)) return 0.0;
  double r = __builtin_amdgcn_rcp(d);
  const double q = fma(-d, r, 1.0);
  return fma(r, q, r);
}

template <typename IT, int R>
__global__ __launch_bounds__(kMapThreads) void map_em_kernel(MapArgs a) {
  __shared__ double bl[kMapMaxP], wl[kMapMaxP], xv[kMapMaxP][4];
  __shared__ __align__(16) double part[2][kMapWaves];
  __shared__ double red[kMapWaves];
  __shared__ double cltab[kMapWaves][4];   // per wave: exp(-delta x_c) of codes 0..3
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int s = blockIdx.x;                      // start point
  const int n = a.n, n_pad = a.n_pad, p = a.p;
  const uint8_t *codes = a.codes;                // p x n_pad, 3 in padded individuals
  const IT *b0 = reinterpret_cast<const IT *>(a.beta0) + (size_t)s * p;
  const Prior pr = a.prior;
  const double inv_n4 = 4.0 / static_cast<double>(n);

  for (int j = tid; j < p; j += kMapThreads) {
    bl[j] = static_cast<double>(b0[j]);
#pragma unroll
    for (int c = 0; c < 4; ++c) xv[j][c] = a.xv[4 * j + c];
  }
  __syncthreads();
  double E[R], sg[R], yk[R];
#pragma unroll
  for (int r = 0; r < R; ++r) {
    const int k = tid + kMapThreads * r;
    yk[r] = k < n_pad ? a.yv[k] : 0.0;
  }
  auto load_codes = [&](const int j, int (&c)[R]) {
    const uint8_t *col = codes + (size_t)j * n_pad;
#pragma unroll
    for (int r = 0; r < R; ++r) {
      const int k = tid + kMapThreads * r;
      c[r] = k < n_pad ? static_cast<int>(col[k]) : 3;
    }
  };
  // eta from the coefficients (the sweep's fresh linear predictor), then E and sigma
  auto refresh = [&](double (&eta)[R]) {
#pragma unroll
    for (int r = 0; r < R; ++r) eta[r] = 0.0;
    for (int j = 0; j < p; ++j) {
      int c[R];
      load_codes(j, c);
      const double bj = bl[j];
#pragma unroll
      for (int r = 0; r < R; ++r) eta[r] += bj * xv[j][c[r]];
    }
#pragma unroll
    for (int r = 0; r < R; ++r) {
      E[r] = exp(-eta[r]);
      sg[r] = inv1p(E[r]);
    }
  };

  int parity = 0;
  for (int it = 0; it < a.outer; ++it) {
    __syncthreads();                             // bl final for this E step
    for (int j = tid; j < p; j += kMapThreads)
      wl[j] = pr.inf ? 1.0 / pr.lam : (pr.a + 1.0) / (pr.a * pr.lam + fabs(bl[j]));
    __syncthreads();
    for (int sw = 0; sw < a.inner; ++sw) {
      __syncthreads();                           // the previous sweep's last coefficient
      {
        double eta[R];
        refresh(eta);
      }
      int cn[R];
      load_codes(0, cn);
      for (int j = 0; j < p; ++j) {
        // read beta_j before the barrier: thread 0 overwrites it after the barrier
        const double bj = bl[j], wj = wl[j];
        int c[R];
#pragma unroll
        for (int r = 0; r < R; ++r) c[r] = cn[r];
        if (j + 1 < p) load_codes(j + 1, cn);   // next column's codes in flight
        double g = 0.0;
#pragma unroll
        for (int r = 0; r < R; ++r) g += (yk[r] - sg[r]) * xv[j][c[r]];   // padded: x = 0
        g = wave_total_f64(g);
        if (lane == 0) part[parity][wave] = g;
        __syncthreads();
        {
          // the wave sums, added as a balanced tree (the same order in every thread)
          static_assert(kMapWaves == 8, "tree of 8 wave sums");
          const double2 *pp = reinterpret_cast<const double2 *>(part[parity]);
          double t[4];
#pragma unroll
          for (int i = 0; i < 4; ++i) {
            const double2 q = pp[i];
            t[i] = q.x + q.y;
          }
          g = (t[0] + t[1]) + (t[2] + t[3]);
        }
        parity ^= 1;
        const double z = bj + inv_n4 * g, thr = inv_n4 * wj;
        const double nb = z > thr ? z - thr : (z < -thr ? z + thr : 0.0);
        const double delta = nb - bj;
        if (delta != 0.0) {                      // uniform: every thread holds the same values
          // lanes 0..3 put the factor of codes 0..3 in the wave's table (x_3 = 0: factor 1);
          // a wave's LDS accesses are processed in order, and the wave barrier keeps the
          // compiler from moving the table reads above the write
          if (lane < 4) cltab[wave][lane] = exp(-delta * xv[j][lane]);
          __builtin_amdgcn_wave_barrier();
#pragma unroll
          for (int r = 0; r < R; ++r) {
            E[r] *= cltab[wave][c[r]];
            sg[r] = inv1p(E[r]);
          }
        }
        if (tid == 0) bl[j] = nb;
      }
    }
  }
  __syncthreads();
  // log posterior at the mode: sum_k [y eta - softplus(eta)] + sum_j log Gt(beta_j)
  double eta[R];
  refresh(eta);
  double acc = 0.0;
#pragma unroll
  for (int r = 0; r < R; ++r) {
    const int k = tid + kMapThreads * r;
    if (k < n) acc += yk[r] * eta[r] - (fmax(eta[r], 0.0) + log1p(exp(-fabs(eta[r]))));
  }
  for (int j = tid; j < p; j += kMapThreads) acc += gt_logpdf(bl[j], pr);
  acc = wave_sum(acc);
  if (lane == 0) red[wave] = acc;
  __syncthreads();
  if (tid == 0) {
    double lp = red[0];
    for (int w = 1; w < kMapWaves; ++w) lp += red[w];
    a.logpost[s] = lp;
  }
  for (int j = tid; j < p; j += kMapThreads) a.mode[(size_t)s * p + j] = bl[j];
}

// Genotype codes per column (3 in padded individuals), the standardised value of each code
// (x_c = (c - mu_j)/s_j, 0 for code 3) and the labels in FP64, for the EM kernel.
__global__ void map_cols_kernel(const uint8_t *__restrict__ X, int n, int p, int n_pad,
                                const double *__restrict__ mu, const double *__restrict__ sd,
                                uint8_t *__restrict__ codes, double *__restrict__ xv, double *__restrict__ yv,
                                const uint8_t *__restrict__ y) {
  const size_t total = (size_t)p * n_pad;
  for (size_t idx = blockIdx.x * (size_t)blockDim.x + threadIdx.x; idx < total;
       idx += (size_t)gridDim.x * blockDim.x) {
    const int j = static_cast<int>(idx / n_pad), k = static_cast<int>(idx % n_pad);
    codes[idx] = k < n ? X[(size_t)k * p + j] : uint8_t(3);
    if (j == 0) yv[k] = k < n ? static_cast<double>(y[k]) : 0.0;
    if (k < 4) xv[4 * j + k] = k < 3 ? (static_cast<double>(k) - mu[j]) / sd[j] : 0.0;
  }
}

// Log posterior of every particle at scale lam and the first index of its maximum.
// One workgroup of 1024 threads; a wave per particle, particles strided.
template <typename IT>
__global__ __launch_bounds__(1024) void best_particle_kernel(const IT *__restrict__ beta, const double *__restrict__ ll,
                                                             int M, int p, Prior pr, int *__restrict__ best) {
  __shared__ double sv[16];
  __shared__ int si[16];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  double bv = -INFINITY;
  int bi = 0x7fffffff;
  for (int i = wave; i < M; i += 16) {
    double lp = 0.0;
    for (int j = lane; j < p; j += 64) lp += gt_logpdf(static_cast<double>(beta[(size_t)i * p + j]), pr);
    lp = wave_sum(lp) + ll[i];
    if (lp > bv) {                               // strictly: keeps the first index of a tie
      bv = lp;
      bi = i;
    }
  }
  if (lane == 0) {
    sv[wave] = bv;
    si[wave] = bi;
  }
  __syncthreads();
  if (tid == 0) {
    double v = sv[0];
    int idx = si[0];
    for (int w = 1; w < 16; ++w)
      if (sv[w] > v || (sv[w] == v && si[w] < idx)) {
        v = sv[w];
        idx = si[w];
      }
    best[0] = idx == 0x7fffffff ? 0 : idx;     // no finite density: the first particle
  }
}

// Gather the EM starts of one scale: the best particle, then (if any) the previous MAP.
template <typename IT>
__global__ void map_starts_kernel(const IT *__restrict__ beta, const int *__restrict__ best, int p,
                                  const double *__restrict__ prev, double *__restrict__ starts) {
  for (int j = threadIdx.x; j < p; j += blockDim.x) {
    starts[j] = static_cast<double>(beta[(size_t)best[0] * p + j]);
    if (prev) starts[p + j] = prev[j];
  }
}

// Keep the start whose mode has the higher posterior density (the first on ties).
__global__ void map_pick_kernel(const double *__restrict__ modes, const double *__restrict__ lp, int ns, int p,
                                double *__restrict__ out, double *__restrict__ out_lp) {
  int k = 0;
  for (int s = 1; s < ns; ++s)
    if (lp[s] > lp[k]) k = s;
  for (int j = threadIdx.x; j < p; j += blockDim.x) out[j] = modes[(size_t)k * p + j];
  if (threadIdx.x == 0) out_lp[0] = lp[k];
}

template <typename IT, int R>
void launch_em_r(const MapArgs &a, hipStream_t st) {
  hipLaunchKernelGGL((map_em_kernel<IT, R>), dim3(a.M), dim3(kMapThreads), 0, st, a);
}

template <typename IT>
hipError_t launch_em_t(const MapArgs &a, hipStream_t st) {
  const int R = (a.n_pad + kMapThreads - 1) / kMapThreads;
  if (R <= 1) launch_em_r<IT, 1>(a, st);
  else if (R <= 2) launch_em_r<IT, 2>(a, st);
  else if (R <= 3) launch_em_r<IT, 3>(a, st);
  else if (R <= 4) launch_em_r<IT, 4>(a, st);
  else if (R <= 5) launch_em_r<IT, 5>(a, st);
  else if (R <= 6) launch_em_r<IT, 6>(a, st);
  else if (R <= 8) launch_em_r<IT, 8>(a, st);
  else if (R <= 10) launch_em_r<IT, 10>(a, st);
  else if (R <= 12) launch_em_r<IT, 12>(a, st);
  else if (R <= 16) launch_em_r<IT, 16>(a, st);
  else if (R <= 20) launch_em_r<IT, 20>(a, st);
  else return hipErrorInvalidValue;
  return hipGetLastError();
}

}  // namespace

int map_max_n() { return kMapThreads * 20; }

hipError_t launch_map_cols(const uint8_t *X, const uint8_t *y, int n, int p, int n_pad, const double *mu,
                           const double *sd, uint8_t *codes, double *xv, double *yv, hipStream_t st) {
  const size_t total = (size_t)p * n_pad;
  const int grid = static_cast<int>((total + 255) / 256 < 4096 ? (total + 255) / 256 : 4096);
  hipLaunchKernelGGL(map_cols_kernel, dim3(grid), dim3(256), 0, st, X, n, p, n_pad, mu, sd, codes, xv, yv, y);
  return hipGetLastError();
}

hipError_t launch_map_em(bool in_f64, const MapArgs &a, hipStream_t st) {
  if (a.p > kMapMaxP || a.M < 1) return hipErrorInvalidValue;
  return in_f64 ? launch_em_t<double>(a, st) : launch_em_t<float>(a, st);
}

hipError_t launch_best_particle(bool f64, const void *beta, const double *ll, int M, int p, const Prior &pr,
                                int *best, hipStream_t st) {
  if (f64)
    hipLaunchKernelGGL(best_particle_kernel<double>, dim3(1), dim3(1024), 0, st,
                       reinterpret_cast<const double *>(beta), ll, M, p, pr, best);
  else
    hipLaunchKernelGGL(best_particle_kernel<float>, dim3(1), dim3(1024), 0, st,
                       reinterpret_cast<const float *>(beta), ll, M, p, pr, best);
  return hipGetLastError();
}

hipError_t launch_map_starts(bool f64, const void *beta, const int *best, int p, const double *prev,
                             double *starts, hipStream_t st) {
  if (f64)
    hipLaunchKernelGGL(map_starts_kernel<double>, dim3(1), dim3(256), 0, st,
                       reinterpret_cast<const double *>(beta), best, p, prev, starts);
  else
    hipLaunchKernelGGL(map_starts_kernel<float>, dim3(1), dim3(256), 0, st,
                       reinterpret_cast<const float *>(beta), best, p, prev, starts);
  return hipGetLastError();
}

hipError_t launch_map_pick(const double *modes, const double *lp, int ns, int p, double *out, double *out_lp,
                           hipStream_t st) {
  hipLaunchKernelGGL(map_pick_kernel, dim3(1), dim3(256), 0, st, modes, lp, ns, p, out, out_lp);
  return hipGetLastError();
}

}  // namespace spa
