// C-ABI implementation: handle, validation, buffers and the per-scale orchestration of the
// sampler (Section 4): reweight -> normalise/ESS -> [resample] -> sweeps -> moments.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <string>
#include <utility>
#include <vector>

#include "../../include/spa_smc.h"
#include "spa_gemm_fp8x.hpp"
#include "spa_internal.hpp"
#include "spa_kernels.hpp"
#include "spa_map.hpp"
#include "spa_single.hpp"
#include "spa_summary.hpp"

using namespace spa;

// Device scratch of spa_smc_loglik_noalloc (operand rows, offsets and split partials).
// Each GPU the library runs on holds its own copy until the process ends.  Host code never
// passes the array's name to a kernel: it uses the device address taken per device with
// hipGetSymbolAddress at handle creation (noalloc_setup).
constexpr size_t kNoAllocBytes = size_t(32) << 20;
static __device__ __align__(256) unsigned char scratch[kNoAllocBytes];

namespace {

thread_local std::string g_init_error;

constexpr int kMaxPP = 512;
constexpr double kSigmaFloor = 1e-12;

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void *g_scratch_ptr[kMaxDevices] = {};

int round_up(int v, int m) { return (v + m - 1) / m * m; }
int ceil_log2(long long m) {
  int k = 0;
  while ((1LL << k) < m) ++k;
  return k;
}

// Host copy of Philox4x32-10 for the resampling offsets (same definition as the device one).
uint32_t philox_w0(uint32_t c0, uint32_t c1, uint32_t c2, uint32_t c3, uint32_t k0, uint32_t k1) {
  for (int r = 0; r < 10; ++r) {
    if (r) {
      k0 += 0x9E3779B9u;
      k1 += 0xBB67AE85u;
    }
    const uint64_t p0 = 0xD2511F53ull * c0, p1 = 0xCD9E8D57ull * c2;
    const uint32_t hi0 = static_cast<uint32_t>(p0 >> 32), lo0 = static_cast<uint32_t>(p0);
    const uint32_t hi1 = static_cast<uint32_t>(p1 >> 32), lo1 = static_cast<uint32_t>(p1);
    const uint32_t n0 = hi1 ^ c1 ^ k0, n2 = hi0 ^ c3 ^ k1;
    c0 = n0;
    c1 = lo1;
    c2 = n2;
    c3 = lo0;
  }
  return c0;
}

struct XPack {
  void *Xk = nullptr, *Xt = nullptr, *yv = nullptr;
  int PP = 0;
  bool fp8 = false;
  bool ready = false;
};

struct OpScratch {
  void *Bhi = nullptr, *Blo = nullptr;
  double *moff = nullptr, *yb = nullptr;
  size_t cap = 0;   // rows
  int PP = 0;
};

}  // namespace

struct spa_smc {
  // configuration
  int n = 0, p = 0, N = 0, T = 0;
  double a = 1.0;
  int a_inf = 0;
  spa_move move = SPA_MOVE_RWM;
  int sweeps = 0, init_sweeps = 0, adapt = 1;
  double ess_frac = 0.5, step = 1.0;
  Prec prec = Prec::F64;
  spa_xfmt xfmt = SPA_X_AUTO;
  uint32_t k0 = 0, k1 = 0;
  std::vector<double> lambda;
  hipStream_t stream = nullptr;
  int device = 0;
  int n_pad = 0, Npad = 0, PP = 0;
  bool f64 = true;
  size_t psz = 8;
  // device data
  uint8_t *dX = nullptr, *dy = nullptr;
  double *mu = nullptr, *s = nullptr, *inv_s = nullptr, *ytil = nullptr;
  int *dbad = nullptr;
  XPack xp[3];
  void *beta = nullptr, *prop = nullptr, *tmp = nullptr;
  void *gl = nullptr, *glp = nullptr, *gltmp = nullptr;
  double *ll = nullptr, *llp = nullptr, *lltmp = nullptr, *logw = nullptr;
  double *lpc = nullptr, *lpp = nullptr, *lqf = nullptr;
  int *acc = nullptr, *anc = nullptr;
  OpScratch op;                  // operand of the sampler's own sweeps
  double *sigma = nullptr, *mean_path = nullptr, *var_path = nullptr, *part = nullptr;
  void *mc = nullptr;            // per-marker move constants of the current step size (4 x PP)
  double *cdf = nullptr, *scal = nullptr;
  size_t cdf_cap = 0;
  double *rw_part = nullptr;     // workgroup partials of the reweighting pass
  double *btot = nullptr, *wpart = nullptr;   // resampling pass scratch
  long long *dcount = nullptr;
  double *hscal = nullptr;       // pinned host
  long long *hcount = nullptr;   // pinned host
  OpScratch scr[3];              // operands of loglik/grad calls, per precision
  void *gscr = nullptr;
  size_t gscr_cap = 0;
  double *spl_part = nullptr;    // split partials of the contraction
  size_t spl_part_cap = 0;
  void *g_part = nullptr;
  size_t g_part_cap = 0;
  double *llscr = nullptr;
  size_t llscr_cap = 0;
  void *noalloc = nullptr;       // this device's address of the static scratch array
  // FP8 multi-term forward contraction (loglik calls, and the contraction of random-walk
  // sweeps when the handle's precision is one of the FP8 ones)
  int f8_terms = 0;              // 3 or 4 when the sampler contracts on the FP8 MFMA
  uint8_t *f8_X = nullptr;       // (n rounded up to kF8Tile) x PP8 genotype codes, PP8 = fp8x_pad_markers(p)
  uint8_t *f8_Bq = nullptr;      // 4 x f8_cap x PP8 term codes
  int32_t *f8_Bs = nullptr;      // 4 x f8_cap term exponents
  double *f8_moff = nullptr, *f8_yb = nullptr, *f8_part = nullptr;
  size_t f8_cap = 0;             // particle rows of the buffers above
  std::vector<void *> allocs;
  // optional per-kernel-class timing with HIP events on the handle's stream
  bool timing = false;
  uint32_t tmask = 0;              // bit c: launches of class c are bracketed
  bool topen = false;              // a tbeg of a timed class awaits its tend
  std::vector<hipEvent_t> ev;      // pool, used in (start, stop) pairs
  std::vector<int> ev_cat;         // category of each recorded pair
  double t_ms[SPA_TIMING_CLASSES] = {0};
  long long t_cnt[SPA_TIMING_CLASSES] = {0};
  // EM MAP estimates (FP64 standardised columns and labels) and the MAP path
  uint8_t *map_codes = nullptr;                       // p x n_pad genotype codes (EM)
  double *map_xv = nullptr, *map_yv = nullptr;        // p x 4 code values, n_pad labels
  bool map_on = false;
  int map_outer = 0, map_inner = 0, map_last_row = -1;
  double *map_path = nullptr, *map_lp = nullptr;        // T x p, T
  int *map_best = nullptr;
  double *map_starts = nullptr, *map_modes = nullptr, *map_mlp = nullptr;
  // single-coordinate kernel operands (standardised genotype columns, labels)
  void *xs_ss = nullptr, *yv_ss = nullptr;
  int ss_rows = 0;          // padded individuals of xs_ss / yv_ss (single_site_rows(n))
  float *cs_ss = nullptr;   // FP32: column coefficients sum_k (y_k - 1/2) xs_jk
  // sparsity-path summaries (per scale, and the c-marginal mixture)
  SqLevels sq_lv{};
  bool sq_on = false, sq_keep = false;
  double *quant_path = nullptr, *conc_path = nullptr;   // T x L x p, T x D x p
  void *hist_beta = nullptr;                            // T x N x p particles after the moves
  double *hist_logw = nullptr;                          // T x N normalised log weights
  uint64_t *sq_q = nullptr;
  size_t sq_q_cap = 0;
  void *sq_keys = nullptr;
  size_t sq_keys_cap = 0;                               // bytes
  SqState *sq_st = nullptr;
  SqSel *sq_sel = nullptr;
  unsigned long long *sq_hist = nullptr, *sq_inside = nullptr;
  int sq_p_cap = 0;
  double *sq_w = nullptr, *sq_logz = nullptr;
  size_t sq_w_cap = 0;
  SqState *hsq_st = nullptr;                            // pinned host
  // path
  int t = 0;
  double log_z = 0.0;
  std::vector<spa_smc_stats> stats;
  std::vector<double> logz_path;
  std::string err;
};

namespace {

spa_status set_err(spa_smc *h, spa_status st, const std::string &msg) {
  if (h) h->err = msg;
  else g_init_error = msg;
  return st;
}

spa_status hip_fail(spa_smc *h, hipError_t e, const char *what) {
  std::string m = std::string(what) + ": " + hipGetErrorString(e);
  return set_err(h, SPA_ERR_HIP, m);
}

#define SPA_CK(h, expr)                                   \
  do {                                                    \
    hipError_t e_ = (expr);                               \
    if (e_ != hipSuccess) return hip_fail((h), e_, #expr); \
  } while (0)

template <typename P>
spa_status dalloc(spa_smc *h, P **ptr, size_t bytes) {
  void *v = nullptr;
  if (bytes == 0) bytes = 16;
  hipError_t e = hipMalloc(&v, bytes);
  if (e != hipSuccess) return set_err(h, SPA_ERR_ALLOC, std::string("hipMalloc: ") + hipGetErrorString(e));
  h->allocs.push_back(v);
  e = hipMemsetAsync(v, 0, bytes, h->stream);
  if (e != hipSuccess) return hip_fail(h, e, "hipMemsetAsync");
  *ptr = static_cast<P *>(v);
  return SPA_OK;
}

void dfree(spa_smc *h, void *v) {
  if (!v) return;
  for (auto it = h->allocs.begin(); it != h->allocs.end(); ++it)
    if (*it == v) {
      h->allocs.erase(it);
      break;
    }
  (void)hipFree(v);
}

Prec to_prec(spa_prec p) {
  return p == SPA_PREC_FP64 ? Prec::F64 : (p == SPA_PREC_FP32 ? Prec::F32 : Prec::BF16X2);
}

Prior make_prior(const spa_smc *h, double lam) {
  Prior pr;
  pr.a = h->a;
  pr.lam = lam;
  pr.inf = h->a_inf;
  pr.log2lam = std::log(2.0 * lam);
  return pr;
}

// ---- timing: tbeg/tend bracket one launch; flush after a synchronisation point
void tbeg(spa_smc *h, int cat) {
  h->topen = false;
  if (!h->timing || !((h->tmask >> cat) & 1u)) return;
  const size_t k = 2 * h->ev_cat.size();
  while (h->ev.size() < k + 2) {
    hipEvent_t e;
    // timing only, read after a stream synchronisation: no system-scope fence (its cache
    // write-back and invalidation would land on the bracketed kernels)
    if (hipEventCreateWithFlags(&e, hipEventDisableSystemFence) != hipSuccess) {
      h->timing = false;
      return;
    }
    h->ev.push_back(e);
  }
  h->ev_cat.push_back(cat);
  (void)hipEventRecord(h->ev[k], h->stream);
  h->topen = true;
}
void tend(spa_smc *h) {
  if (!h->topen) return;
  h->topen = false;
  (void)hipEventRecord(h->ev[2 * h->ev_cat.size() - 1], h->stream);
}
void tflush(spa_smc *h) {   // the stream must be synchronised
  for (size_t i = 0; i < h->ev_cat.size(); ++i) {
    float ms = 0.f;
    if (hipEventElapsedTime(&ms, h->ev[2 * i], h->ev[2 * i + 1]) == hipSuccess) {
      h->t_ms[h->ev_cat[i]] += ms;
      h->t_cnt[h->ev_cat[i]] += 1;
    }
  }
  h->ev_cat.clear();
}

size_t bt_size(Prec p) { return p == Prec::F64 ? 8 : (p == Prec::F32 ? 4 : 2); }

spa_status ensure_xpack(spa_smc *h, Prec prec) {
  XPack &x = h->xp[static_cast<int>(prec)];
  if (x.ready) return SPA_OK;
  const int PP = gemm_pad_markers(h->p, prec);
  if (PP < 0) return set_err(h, SPA_ERR_ARG, "p too large for this precision");
  x.PP = PP;
  x.fp8 = (prec == Prec::BF16X2) && (h->xfmt == SPA_X_FP8E4M3);
  XFormat f = prec == Prec::F64 ? XFormat::F64
              : prec == Prec::F32 ? XFormat::F32
              : (x.fp8 ? XFormat::FP8 : XFormat::BF16);
  const size_t es = prec == Prec::F64 ? 8 : prec == Prec::F32 ? 4 : (x.fp8 ? 1 : 2);
  spa_status st;
  if ((st = dalloc(h, &x.Xk, es * (size_t)h->n_pad * PP)) != SPA_OK) return st;
  if ((st = dalloc(h, &x.Xt, es * (size_t)h->n_pad * PP)) != SPA_OK) return st;
  const bool yf64 = prec == Prec::F64;
  if ((st = dalloc(h, &x.yv, (yf64 ? 8 : 4) * (size_t)h->n_pad)) != SPA_OK) return st;
  launch_pack_x(f, prec, h->dX, h->n, h->p, h->n_pad, PP, x.Xk, x.Xt, h->stream);
  launch_labels(h->dy, h->n, h->n_pad, yf64, x.yv, h->stream);
  SPA_CK(h, hipGetLastError());
  x.ready = true;
  return SPA_OK;
}

spa_status ensure_op(spa_smc *h, OpScratch &o, Prec prec, int PP, size_t rows) {
  if (o.cap >= rows && o.PP == PP) return SPA_OK;
  dfree(h, o.Bhi);
  dfree(h, o.Blo);
  dfree(h, o.moff);
  dfree(h, o.yb);
  o = OpScratch{};
  spa_status st;
  const size_t bs = bt_size(prec);
  if ((st = dalloc(h, &o.Bhi, bs * rows * PP)) != SPA_OK) return st;
  if ((st = dalloc(h, &o.Blo, prec == Prec::BF16X2 ? bs * rows * PP : 16)) != SPA_OK) return st;
  if ((st = dalloc(h, &o.moff, 8 * rows)) != SPA_OK) return st;
  if ((st = dalloc(h, &o.yb, 8 * rows)) != SPA_OK) return st;
  o.cap = rows;
  o.PP = PP;
  return SPA_OK;
}

// Arguments of one contraction launch without its partial-sum buffers (a.S tells whether
// they are needed: S x M_pad softplus sums, and for the gradient S x M_pad x PP adjoints).
GemmArgs gemm_args_core(const spa_smc *h, Prec prec, const OpScratch &o, int M, bool grad, double *ll, void *g) {
  const XPack &x = h->xp[static_cast<int>(prec)];
  GemmArgs a{};
  a.prec = prec;
  a.PP = x.PP;
  a.grad = grad;
  a.x_fp8 = x.fp8;
  a.Xk = x.Xk;
  a.Xt = x.Xt;
  a.yv = x.yv;
  a.Bhi = o.Bhi;
  a.Blo = o.Blo;
  a.moff = o.moff;
  a.yb = o.yb;
  a.mu = h->mu;
  a.inv_s = h->inv_s;
  a.ytil = h->ytil;
  a.n = h->n;
  a.n_pad = h->n_pad;
  a.M = M;
  a.M_pad = round_up(M, gemm_particles_per_wg(prec, x.PP));
  a.p = h->p;
  a.ll = ll;
  a.g = g;
  const size_t es = prec == Prec::F64 ? 8 : prec == Prec::F32 ? 4 : (x.fp8 ? 1 : 2);
  a.S = gemm_splits(prec, x.PP, h->n_pad, M, 2 * es * (size_t)h->n_pad * x.PP);
  return a;
}

// Arguments of one contraction launch; allocates the split partials on first need.
spa_status gemm_args(spa_smc *h, Prec prec, const OpScratch &o, int M, bool grad, double *ll, void *g,
                     GemmArgs *out) {
  const XPack &x = h->xp[static_cast<int>(prec)];
  GemmArgs a = gemm_args_core(h, prec, o, M, grad, ll, g);
  if ((size_t)a.M_pad > o.cap) return set_err(h, SPA_ERR_ARG, "operand rows not padded");
  if (a.S > 1) {
    spa_status st;
    const size_t ns = (size_t)a.S * a.M_pad;
    if (h->spl_part_cap < ns) {
      dfree(h, h->spl_part);
      h->spl_part = nullptr;
      if ((st = dalloc(h, &h->spl_part, 8 * ns)) != SPA_OK) return st;
      h->spl_part_cap = ns;
    }
    const size_t ng = grad ? ns * x.PP * (prec == Prec::F64 ? 8 : 4) : 0;
    if (ng && h->g_part_cap < ng) {
      dfree(h, h->g_part);
      h->g_part = nullptr;
      if ((st = dalloc(h, &h->g_part, ng)) != SPA_OK) return st;
      h->g_part_cap = ng;
    }
    a.spl_part = h->spl_part;
    a.g_part = h->g_part;
  }
  *out = a;
  return SPA_OK;
}

// The contraction; with finalize = false and S > 1 the partial sums are left for the caller
// (the MH decision combines them), and *used describes them.
spa_status run_gemm(spa_smc *h, Prec prec, const OpScratch &o, int M, bool grad, double *ll, void *g,
                    bool finalize = true, GemmArgs *used = nullptr) {
  GemmArgs a;
  spa_status st = gemm_args(h, prec, o, M, grad, ll, g, &a);
  if (st != SPA_OK) return st;
  tbeg(h, SPA_T_LOGLIK);
  SPA_CK(h, launch_loglik(a, h->stream));
  tend(h);
  if (a.S > 1 && finalize) {
    tbeg(h, SPA_T_FINALIZE);
    SPA_CK(h, launch_gemm_finalize(a, h->stream));
    tend(h);
  }
  if (used) *used = a;
  return SPA_OK;
}

// Buffers of the FP8 multi-term contraction for M particles (grown on demand; the genotype
// copy is packed once); *PPo / *Mpado receive the padded marker and particle counts.
spa_status ensure_f8(spa_smc *h, int M, int nterm, int *PPo, int *Mpado) {
  spa_status st;
  const int PP = fp8x_pad_markers(h->p);
  if (PP < 0) return set_err(h, SPA_ERR_ARG, "FP8 multi-term path needs p <= 512");
  const int n_pad = round_up(h->n, kF8Tile);
  if (!h->f8_X) {
    if ((st = dalloc(h, &h->f8_X, (size_t)n_pad * PP)) != SPA_OK) return st;
    SPA_CK(h, launch_fp8x_pack_x(h->dX, h->n, h->p, n_pad, PP, h->f8_X, h->stream));
  }
  const int Mpad = round_up(M, std::max(kPartPad, fp8x_particles_per_wg(PP, nterm)));
  if (h->f8_cap < (size_t)Mpad) {
    dfree(h, h->f8_Bq);
    dfree(h, h->f8_Bs);
    dfree(h, h->f8_moff);
    dfree(h, h->f8_yb);
    dfree(h, h->f8_part);
    h->f8_Bq = nullptr;
    h->f8_Bs = nullptr;
    h->f8_moff = h->f8_yb = h->f8_part = nullptr;
    h->f8_cap = 0;
    if ((st = dalloc(h, &h->f8_Bq, 4 * (size_t)Mpad * PP)) != SPA_OK) return st;
    if ((st = dalloc(h, &h->f8_Bs, 4 * 4 * (size_t)Mpad)) != SPA_OK) return st;
    if ((st = dalloc(h, &h->f8_moff, 8 * (size_t)Mpad)) != SPA_OK) return st;
    if ((st = dalloc(h, &h->f8_yb, 8 * (size_t)Mpad)) != SPA_OK) return st;
    if ((st = dalloc(h, &h->f8_part, 8 * 8 * (size_t)Mpad)) != SPA_OK) return st;
    h->f8_cap = Mpad;
  }
  *PPo = PP;
  *Mpado = Mpad;
  return SPA_OK;
}

// Forward log-likelihood on the FP8 MFMA with the coefficients split into nterm e4m3 terms.
// With finalize = false and more than one individual split the partial sums are left for
// the caller (the MH decision combines them), and *used describes them.  pack = false: the
// term rows, exponents and offsets of `beta` are already in the buffers (written by the
// sampler's proposal step).
spa_status fp8x_contract(spa_smc *h, const void *beta, int M, int is_f64, int nterm, double *out,
                         bool finalize, Fp8xArgs *used, bool pack = true) {
  spa_status st;
  int PP = 0, Mpad = 0;
  if ((st = ensure_f8(h, M, nterm, &PP, &Mpad)) != SPA_OK) return st;
  const int n_pad = round_up(h->n, kF8Tile);
  const int S = fp8x_splits(PP, nterm, n_pad, M);
  if (pack)
    SPA_CK(h, launch_fp8x_pack_b(nterm, is_f64 != 0, beta, M, Mpad, h->p, PP, h->mu, h->s, h->inv_s, h->ytil,
                                 h->f8_Bq, h->f8_Bs, h->f8_moff, h->f8_yb, h->stream));
  Fp8xArgs a{};
  a.nterm = nterm;
  a.PP = PP;
  a.Xf = h->f8_X;
  a.Bq = h->f8_Bq;
  a.Bs = h->f8_Bs;
  a.moff = h->f8_moff;
  a.yb = h->f8_yb;
  a.n = h->n;
  a.n_pad = n_pad;
  a.M = M;
  a.M_pad = Mpad;
  a.S = S;
  a.spl_part = h->f8_part;
  a.ll = out;
  tbeg(h, SPA_T_LOGLIK);
  SPA_CK(h, launch_fp8x_loglik(a, h->stream));
  tend(h);
  if (S > 1 && finalize) {
    tbeg(h, SPA_T_FINALIZE);
    SPA_CK(h, launch_fp8x_finalize(a, h->stream));
    tend(h);
  }
  if (used) *used = a;
  return SPA_OK;
}

// Log-likelihood (and gradient) of the handle's own particle buffer `beta` into ll/g.
spa_status eval_state(spa_smc *h, const void *beta, double *ll, void *g) {
  if (h->f8_terms) return fp8x_contract(h, beta, h->N, 0, h->f8_terms, ll, true, nullptr);
  launch_pack_b(h->prec, h->f64, beta, h->N, h->Npad, h->p, h->PP, h->mu, h->s, h->inv_s, h->ytil,
                h->op.Bhi, h->op.Blo, h->op.moff, h->op.yb, h->stream);
  const bool grad = h->move == SPA_MOVE_MALA;
  return run_gemm(h, h->prec, h->op, h->N, grad, ll, grad ? g : nullptr);
}

// One sweep targeting pi(. | lam): propose -> contraction (+ adjoint) -> MH decision.
// have_prop: the previous sweep's decision kernel already drew this sweep's proposal;
// make_next: this sweep's decision kernel draws the proposal of sweep s + 1 (the caller
// keeps the step size, the preconditioner and lam fixed until that sweep).
spa_status sweep(spa_smc *h, int t, int s, double lam, bool have_prop = false, bool make_next = false) {
  const bool mala = h->move == SPA_MOVE_MALA;
  const Prior pr = make_prior(h, lam);
  ProposeArgs pa{};
  pa.beta = h->beta;
  pa.gl = h->gl;
  pa.prop = h->prop;
  pa.Bhi = h->op.Bhi;
  pa.Blo = h->op.Blo;
  pa.moff = h->op.moff;
  pa.yb = h->op.yb;
  pa.lp_cur = h->lpc;
  pa.lp_prop = h->lpp;
  pa.lqf = h->lqf;
  pa.mc = h->mc;
  pa.cc.mu = h->mu;
  pa.cc.s = h->s;
  pa.cc.inv_s = h->inv_s;
  pa.cc.ytil = h->ytil;
  pa.prior = pr;
  pa.step = h->step;
  pa.sqrt_step = std::sqrt(h->step);
  pa.M = h->N;
  pa.M_pad = h->Npad;
  pa.p = h->p;
  pa.PP = h->PP;
  pa.k0 = h->k0;
  pa.k1 = h->k1;
  pa.sweep = static_cast<uint32_t>(s);
  pa.t = t;
  if (h->f8_terms) {   // random-walk rows write the FP8 term operand instead of BF16 hi/lo
    int PP8 = 0, Mp8 = 0;
    spa_status st = ensure_f8(h, h->N, h->f8_terms, &PP8, &Mp8);
    if (st != SPA_OK) return st;
    pa.f8_q = h->f8_Bq;
    pa.f8_s = h->f8_Bs;
    pa.f8_terms = h->f8_terms;
    pa.f8_Mp = Mp8;
    pa.f8_PP = PP8;
    pa.moff = h->f8_moff;
    pa.yb = h->f8_yb;
  }
  if (!have_prop) {
    // the step size and the preconditioner hold for this sweep and the ones chained to it
    launch_move_consts(h->f64, h->sigma, h->p, h->PP, h->step, pa.sqrt_step, h->mc, h->acc, h->N, h->stream);
    tbeg(h, SPA_T_PROPOSE);
    launch_propose(h->prec, mala, pa, h->stream);
    tend(h);
  }
  AcceptArgs aa{};
  aa.PP = h->PP;   // row length of the move constants (and of the split adjoints below)
  if (h->f8_terms) {   // random-walk moves on the FP8 MFMA: the proposal is packed into terms
    Fp8xArgs fa;
    spa_status st = fp8x_contract(h, h->prop, h->N, 0, h->f8_terms, h->llp, false, &fa, false);
    if (st != SPA_OK) return st;
    if (fa.S > 1) {
      aa.spl_part = fa.spl_part;
      aa.S = fa.S;
      aa.Mp = static_cast<size_t>(fa.M_pad);
      aa.yb = fa.yb;
    }
  }
  GemmArgs ga{};
  if (!h->f8_terms) {
    spa_status st = run_gemm(h, h->prec, h->op, h->N, mala, h->llp, mala ? h->glp : nullptr, false, &ga);
    if (st != SPA_OK) return st;
  }
  if (!h->f8_terms && ga.S > 1) {   // the MH decision combines the contraction's partial sums itself
    aa.spl_part = ga.spl_part;
    aa.g_part = ga.g_part;
    aa.S = ga.S;
    aa.PP = ga.PP;
    aa.Mp = static_cast<size_t>(ga.M_pad);
    aa.yb = ga.yb;
    aa.mu = ga.mu;
    aa.inv_s = ga.inv_s;
    aa.ytil = ga.ytil;
  }
  aa.beta = h->beta;
  aa.gl = h->gl;
  aa.prop = h->prop;
  aa.gl_prop = h->glp;
  aa.ll = h->ll;
  aa.ll_prop = h->llp;
  aa.lp_cur = h->lpc;
  aa.lp_prop = h->lpp;
  aa.lqf = h->lqf;
  aa.mc = h->mc;
  aa.acc_cnt = h->acc;
  aa.prior = pr;
  aa.step = h->step;
  aa.M = h->N;
  aa.p = h->p;
  aa.k0 = h->k0;
  aa.k1 = h->k1;
  aa.sweep = static_cast<uint32_t>(s);
  aa.t = t;
  ProposeArgs na = pa;
  na.sweep = static_cast<uint32_t>(s + 1);
  tbeg(h, SPA_T_ACCEPT);
  SPA_CK(h, launch_accept(h->prec, mala, h->PP, aa, make_next ? &na : nullptr, h->stream));
  tend(h);
  SPA_CK(h, hipGetLastError());
  return SPA_OK;
}

// Accept count of the sweeps since the counters were zeroed; *nonfinite (nullable) receives
// the number of particles whose log-likelihood is not finite.
spa_status read_count(spa_smc *h, long long *out, long long *nonfinite = nullptr) {
  launch_count(h->acc, h->N, nonfinite ? h->ll : nullptr, h->dcount, h->stream);
  SPA_CK(h, hipMemcpyAsync(h->hcount, h->dcount, 2 * sizeof(long long), hipMemcpyDeviceToHost, h->stream));
  SPA_CK(h, hipStreamSynchronize(h->stream));
  tflush(h);
  *out = h->hcount[0];
  if (nonfinite) *nonfinite = h->hcount[1];
  return SPA_OK;
}

void adapt_step(spa_smc *h, double acc_rate) {
  if (!h->adapt || h->move == SPA_MOVE_SINGLE) return;   // the single-coordinate variance is fixed
  const double target = h->move == SPA_MOVE_MALA ? 0.574 : 0.234;
  double d = acc_rate - target;
  const double l2 = std::log(2.0);
  d = std::min(std::max(d, -l2), l2);
  h->step *= std::exp(d);
}

spa_status record_moments(spa_smc *h, int row) {
  tbeg(h, SPA_T_MOMENTS);
  launch_moments(h->f64, h->beta, h->logw, nullptr, h->N, h->p, h->part, h->mean_path + (size_t)row * h->p,
                 h->var_path + (size_t)row * h->p, nullptr, kSigmaFloor, h->stream);
  tend(h);
  SPA_CK(h, hipGetLastError());
  return SPA_OK;
}

// Cycles of the single-coordinate kernel (Section 4.1) at scale lam, Philox index t.
spa_status single_site_cycles(spa_smc *h, int t, int cycles, double lam) {
  SingleSiteArgs a{};
  a.xs = h->xs_ss;
  a.yv = h->yv_ss;
  a.cs = h->cs_ss;
  a.beta = h->beta;
  a.ll = h->ll;
  a.acc_cnt = h->acc;
  a.prior = make_prior(h, lam);
  a.step = h->step;
  a.M = h->N;
  a.n = h->n;
  a.n_pad = h->ss_rows;
  a.p = h->p;
  a.cycles = cycles;
  a.cycle0 = 0;
  a.k0 = h->k0;
  a.k1 = h->k1;
  a.t = t;
  tbeg(h, SPA_T_PROPOSE);
  SPA_CK(h, launch_single_site(h->f64, a, h->stream));
  tend(h);
  return SPA_OK;
}

spa_status ensure_map_cols(spa_smc *h) {
  if (h->map_codes) return SPA_OK;
  spa_status st;
  if ((st = dalloc(h, &h->map_codes, (size_t)h->p * h->n_pad)) != SPA_OK) return st;
  if ((st = dalloc(h, &h->map_xv, 8 * 4 * (size_t)h->p)) != SPA_OK) return st;
  if ((st = dalloc(h, &h->map_yv, 8 * (size_t)h->n_pad)) != SPA_OK) return st;
  SPA_CK(h, launch_map_cols(h->dX, h->dy, h->n, h->p, h->n_pad, h->mu, h->s, h->map_codes, h->map_xv, h->map_yv,
                            h->stream));
  return SPA_OK;
}

spa_status run_map_em(spa_smc *h, const void *beta0, bool in_f64, int M, double lam, int outer, int inner,
                      double *mode, double *logpost) {
  spa_status st;
  if ((st = ensure_map_cols(h)) != SPA_OK) return st;
  MapArgs a{};
  a.codes = h->map_codes;
  a.xv = h->map_xv;
  a.yv = h->map_yv;
  a.beta0 = beta0;
  a.mode = mode;
  a.logpost = logpost;
  a.prior = make_prior(h, lam);
  a.M = M;
  a.n = h->n;
  a.n_pad = h->n_pad;
  a.p = h->p;
  a.outer = outer;
  a.inner = inner;
  tbeg(h, SPA_T_MAP);
  SPA_CK(h, launch_map_em(in_f64, a, h->stream));
  tend(h);
  return SPA_OK;
}

// MAP path row `row` (Section 4.1): EM from the particle of highest posterior density at
// this scale and from the previous row's MAP; the better mode is kept.
spa_status record_map(spa_smc *h, int row) {
  if (!h->map_on) return SPA_OK;
  const double lam = h->lambda[row];
  const Prior pr = make_prior(h, lam);
  const int p = h->p;
  const bool prev = h->map_last_row == row - 1 && row > 0;
  tbeg(h, SPA_T_MAP);
  SPA_CK(h, launch_best_particle(h->f64, h->beta, h->ll, h->N, p, pr, h->map_best, h->stream));
  SPA_CK(h, launch_map_starts(h->f64, h->beta, h->map_best, p, prev ? h->map_path + (size_t)(row - 1) * p : nullptr,
                              h->map_starts, h->stream));
  tend(h);
  const int ns = prev ? 2 : 1;
  spa_status st = run_map_em(h, h->map_starts, true, ns, lam, h->map_outer, h->map_inner, h->map_modes, h->map_mlp);
  if (st != SPA_OK) return st;
  SPA_CK(h, launch_map_pick(h->map_modes, h->map_mlp, ns, p, h->map_path + (size_t)row * p, h->map_lp + row,
                            h->stream));
  h->map_last_row = row;
  return SPA_OK;
}

// Summary scratch for M values of p coefficients.
spa_status ensure_sq(spa_smc *h, size_t M, int p, bool f64) {
  spa_status st;
  if (h->sq_q_cap < M) {
    dfree(h, h->sq_q);
    h->sq_q = nullptr;
    if ((st = dalloc(h, &h->sq_q, 8 * M)) != SPA_OK) return st;
    h->sq_q_cap = M;
  }
  const size_t kb = M * (size_t)p * sq_key_bytes(f64);
  if (h->sq_keys_cap < kb) {
    dfree(h, h->sq_keys);
    h->sq_keys = nullptr;
    if ((st = dalloc(h, &h->sq_keys, kb)) != SPA_OK) return st;
    h->sq_keys_cap = kb;
  }
  if (h->sq_p_cap < p) {
    dfree(h, h->sq_sel);
    dfree(h, h->sq_hist);
    dfree(h, h->sq_inside);
    h->sq_sel = nullptr;
    h->sq_hist = nullptr;
    h->sq_inside = nullptr;
    if ((st = dalloc(h, &h->sq_sel, sizeof(SqSel) * (size_t)p * kSqMaxLevels)) != SPA_OK) return st;
    if ((st = dalloc(h, &h->sq_hist, 8 * (size_t)p * kSqMaxLevels * 256)) != SPA_OK) return st;
    if ((st = dalloc(h, &h->sq_inside, 8 * (size_t)p * kSqMaxLevels)) != SPA_OK) return st;
    h->sq_p_cap = p;
  }
  if (!h->sq_st && (st = dalloc(h, &h->sq_st, sizeof(SqState))) != SPA_OK) return st;
  return SPA_OK;
}

spa_status run_summaries(spa_smc *h, const void *values, bool f64, int M, int p, const double *w, bool logw,
                         const SqLevels &lv, double *quant, double *conc) {
  spa_status st;
  if ((st = ensure_sq(h, (size_t)M, p, f64)) != SPA_OK) return st;
  SqArgs a{};
  a.values = values;
  a.f64 = f64;
  a.M = M;
  a.p = p;
  a.w = w;
  a.log_weights = logw;
  a.lv = lv;
  a.q = h->sq_q;
  a.keys = h->sq_keys;
  a.st = h->sq_st;
  a.sel = h->sq_sel;
  a.hist = h->sq_hist;
  a.inside = h->sq_inside;
  a.quant = quant;
  a.conc = conc;
  tbeg(h, SPA_T_SUMMARY);
  SPA_CK(h, launch_weighted_summaries(a, h->stream));
  tend(h);
  return SPA_OK;
}

// Per-scale summaries of the current particles into row `row` of the paths, and the
// history copy used by the c-marginal mixture.
spa_status record_summaries(spa_smc *h, int row) {
  if (!h->sq_on) return SPA_OK;
  const int L = h->sq_lv.L, D = h->sq_lv.D, p = h->p;
  spa_status st = run_summaries(h, h->beta, h->f64, h->N, p, h->logw, true, h->sq_lv,
                                L ? h->quant_path + (size_t)row * L * p : nullptr,
                                D ? h->conc_path + (size_t)row * D * p : nullptr);
  if (st != SPA_OK) return st;
  if (h->sq_keep) {
    const size_t rb = h->psz * (size_t)h->N * p;
    SPA_CK(h, hipMemcpyAsync(static_cast<char *>(h->hist_beta) + rb * row, h->beta, rb, hipMemcpyDeviceToDevice,
                             h->stream));
    SPA_CK(h, hipMemcpyAsync(h->hist_logw + (size_t)row * h->N, h->logw, 8 * (size_t)h->N,
                             hipMemcpyDeviceToDevice, h->stream));
  }
  return SPA_OK;
}

spa_status parse_levels(spa_smc *h, const double *levels, int32_t L, const double *deltas, int32_t D,
                        SqLevels *out) {
  if (L < 0 || D < 0 || L > kSqMaxLevels || D > kSqMaxLevels)
    return set_err(h, SPA_ERR_ARG, "between 0 and 8 quantile levels and tolerances");
  if ((L > 0 && !levels) || (D > 0 && !deltas)) return set_err(h, SPA_ERR_ARG, "levels/deltas is NULL");
  SqLevels lv{};
  lv.L = L;
  lv.D = D;
  for (int l = 0; l < L; ++l) {
    if (!(levels[l] > 0.0 && levels[l] <= 1.0)) return set_err(h, SPA_ERR_ARG, "quantile levels must lie in (0, 1]");
    lv.alpha[l] = levels[l];
  }
  for (int d = 0; d < D; ++d) {
    if (!(deltas[d] > 0.0) || !std::isfinite(deltas[d])) return set_err(h, SPA_ERR_ARG, "tolerances must be > 0");
    lv.delta[d] = deltas[d];
  }
  *out = lv;
  return SPA_OK;
}

// This device's address of the static scratch array, taken once per device (with that
// device current) and kept for the rest of the process.
spa_status noalloc_setup(spa_smc *h) {
  if (h->device < 0 || h->device >= kMaxDevices) return set_err(h, SPA_ERR_STATE, "device index out of range");
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (!g_scratch_ptr[h->device]) {
    void *ptr = nullptr;
    hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return hip_fail(h, e, "hipGetSymbolAddress(scratch)");
    if (!ptr) return set_err(h, SPA_ERR_HIP, "hipGetSymbolAddress(scratch) returned NULL");
    g_scratch_ptr[h->device] = ptr;
  }
  h->noalloc = g_scratch_ptr[h->device];
  return SPA_OK;
}

size_t align256(size_t v) { return (v + 255) / 256 * 256; }

// Byte offsets, inside the static scratch, of the operand and partial sums of an
// M-particle contraction at precision prec: Bhi, Blo, moff, yb, spl_part; returns the total.
size_t noalloc_layout(const spa_smc *h, Prec prec, int M, size_t off[5]) {
  const int PP = h->xp[static_cast<int>(prec)].PP;
  const size_t Mpad = static_cast<size_t>(round_up(M, kPartPad));
  const size_t bs = bt_size(prec);
  OpScratch probe{};
  probe.PP = PP;
  probe.cap = Mpad;
  const GemmArgs a = gemm_args_core(h, prec, probe, M, false, nullptr, nullptr);
  size_t at = 0;
  off[0] = at;
  at = align256(at + bs * Mpad * PP);
  off[1] = at;
  at = align256(at + (prec == Prec::BF16X2 ? bs * Mpad * PP : 0));
  off[2] = at;
  at = align256(at + 8 * Mpad);
  off[3] = at;
  at = align256(at + 8 * Mpad);
  off[4] = at;
  at = align256(at + (a.S > 1 ? 8 * (size_t)a.S * a.M_pad : 0));
  return at;
}

spa_status validate_cfg(const spa_smc_config *c) {
  if (!c) return set_err(nullptr, SPA_ERR_ARG, "cfg is NULL");
  if (c->n < 1 || c->p < 1 || c->N < 1) return set_err(nullptr, SPA_ERR_SHAPE, "n, p and N must be >= 1");
  if (c->p > kMaxPP - 1) return set_err(nullptr, SPA_ERR_SHAPE, "p must be <= 511");
  if ((long long)c->n * c->p > (1LL << 31) || (long long)c->N * c->p > (1LL << 31))
    return set_err(nullptr, SPA_ERR_SHAPE, "problem too large for 32-bit indices");
  if (!(c->a > 0.0)) return set_err(nullptr, SPA_ERR_ARG, "a must be > 0");
  if (c->T < 1 || !c->lambda) return set_err(nullptr, SPA_ERR_ARG, "T >= 1 and lambda required");
  for (int i = 0; i < c->T; ++i) {
    if (!(c->lambda[i] > 0.0) || !std::isfinite(c->lambda[i]))
      return set_err(nullptr, SPA_ERR_ARG, "lambda must be finite and > 0");
    if (i && !(c->lambda[i] < c->lambda[i - 1]))
      return set_err(nullptr, SPA_ERR_ARG, "lambda must be strictly decreasing");
  }
  if (c->move != SPA_MOVE_RWM && c->move != SPA_MOVE_MALA && c->move != SPA_MOVE_SINGLE)
    return set_err(nullptr, SPA_ERR_ARG, "bad move");
  if (c->move == SPA_MOVE_SINGLE && c->n > single_site_max_n())
    return set_err(nullptr, SPA_ERR_SHAPE, "the single-coordinate kernel holds at most 2048 individuals");
  if (c->sweeps < 0 || c->init_sweeps < 0) return set_err(nullptr, SPA_ERR_ARG, "sweeps must be >= 0");
  if (!(c->ess_frac > 0.0 && c->ess_frac <= 1.0)) return set_err(nullptr, SPA_ERR_ARG, "ess_frac in (0, 1]");
  if (!(c->step0 > 0.0) || !std::isfinite(c->step0)) return set_err(nullptr, SPA_ERR_ARG, "step0 must be > 0");
  if (c->adapt != 0 && c->adapt != 1) return set_err(nullptr, SPA_ERR_ARG, "adapt must be 0 or 1");
  const bool f8 = c->prec == SPA_PREC_FP8X3 || c->prec == SPA_PREC_FP8X4;
  if (c->prec != SPA_PREC_FP64 && c->prec != SPA_PREC_FP32 && c->prec != SPA_PREC_BF16X2 && !f8)
    return set_err(nullptr, SPA_ERR_ARG, "bad prec");
  if (f8 && c->move != SPA_MOVE_RWM)
    return set_err(nullptr, SPA_ERR_ARG, "the FP8 multi-term contraction has no adjoint: random-walk moves only");
  if (c->xfmt != SPA_X_AUTO && c->xfmt != SPA_X_FP8E4M3 && c->xfmt != SPA_X_BF16)
    return set_err(nullptr, SPA_ERR_ARG, "bad xfmt");
  if (c->prec == SPA_PREC_FP64 && c->p > 255) return set_err(nullptr, SPA_ERR_SHAPE, "FP64 path needs p <= 255");
  return SPA_OK;
}

}  // namespace

// =====================================================================================

extern "C" spa_status spa_smc_init(const spa_smc_config *cfg, const uint8_t *X_host, const uint8_t *y_host,
                                   void *hip_stream, spa_smc **out) {
  g_init_error.clear();
  if (!out) return set_err(nullptr, SPA_ERR_ARG, "out is NULL");
  *out = nullptr;
  spa_status st = validate_cfg(cfg);
  if (st != SPA_OK) return st;
  if (!X_host || !y_host) return set_err(nullptr, SPA_ERR_ARG, "X and y are required");
  const int n = cfg->n, p = cfg->p;
  for (size_t i = 0; i < (size_t)n * p; ++i)
    if (X_host[i] > 2) return set_err(nullptr, SPA_ERR_ARG, "genotypes must be 0, 1 or 2");
  for (int k = 0; k < n; ++k)
    if (y_host[k] > 1) return set_err(nullptr, SPA_ERR_ARG, "labels must be 0 or 1");
  for (int j = 0; j < p; ++j) {
    uint8_t lo = 255, hi = 0;
    for (int k = 0; k < n; ++k) {
      lo = std::min(lo, X_host[(size_t)k * p + j]);
      hi = std::max(hi, X_host[(size_t)k * p + j]);
    }
    if (lo == hi) return set_err(nullptr, SPA_ERR_SHAPE, "marker " + std::to_string(j) + " has zero variance");
  }

  spa_smc *h = new (std::nothrow) spa_smc();
  if (!h) return set_err(nullptr, SPA_ERR_ALLOC, "handle allocation failed");
  h->n = n;
  h->p = p;
  h->N = cfg->N;
  h->T = cfg->T;
  h->a = cfg->a;
  h->a_inf = std::isinf(cfg->a) ? 1 : 0;
  h->move = cfg->move;
  h->sweeps = cfg->sweeps;
  h->init_sweeps = cfg->init_sweeps;
  h->ess_frac = cfg->ess_frac;
  h->step = cfg->step0;
  h->adapt = cfg->adapt;
  h->prec = to_prec(cfg->prec);   // the FP8 precisions run the BF16 move kernels (FP32 particles)
  h->f8_terms = cfg->prec == SPA_PREC_FP8X3 ? 3 : (cfg->prec == SPA_PREC_FP8X4 ? 4 : 0);
  h->xfmt = cfg->xfmt;
  h->k0 = static_cast<uint32_t>(cfg->seed & 0xFFFFFFFFull);
  h->k1 = static_cast<uint32_t>(cfg->seed >> 32);
  h->lambda.assign(cfg->lambda, cfg->lambda + cfg->T);
  h->stream = static_cast<hipStream_t>(hip_stream);
  h->f64 = h->prec == Prec::F64;
  h->psz = h->f64 ? 8 : 4;
  h->n_pad = round_up(n, kIndPad);
  h->Npad = round_up(h->N, kPartPad);
  h->PP = gemm_pad_markers(p, h->prec);

  auto fail = [&](spa_status s) {
    g_init_error = h->err;
    spa_smc_destroy(h);
    return s;
  };
  hipError_t he = hipGetDevice(&h->device);
  if (he != hipSuccess) {
    hip_fail(h, he, "hipGetDevice");
    return fail(SPA_ERR_HIP);
  }
  if ((st = noalloc_setup(h)) != SPA_OK) return fail(st);
  const size_t NP = (size_t)h->Npad * p;
  const bool mala = h->move == SPA_MOVE_MALA;
#define SPA_AL(ptr, bytes) \
  if ((st = dalloc(h, &(ptr), (bytes))) != SPA_OK) return fail(st)
  SPA_AL(h->dX, (size_t)n * p);
  SPA_AL(h->dy, (size_t)n);
  SPA_AL(h->mu, 8 * kMaxPP);
  SPA_AL(h->s, 8 * kMaxPP);
  SPA_AL(h->inv_s, 8 * kMaxPP);
  SPA_AL(h->ytil, 8 * kMaxPP);
  SPA_AL(h->dbad, 16);
  SPA_AL(h->beta, h->psz * NP);
  SPA_AL(h->prop, h->psz * NP);
  SPA_AL(h->tmp, h->psz * NP);
  SPA_AL(h->gl, mala ? h->psz * NP : 16);
  SPA_AL(h->glp, mala ? h->psz * NP : 16);
  SPA_AL(h->gltmp, mala ? h->psz * NP : 16);
  SPA_AL(h->ll, 8 * (size_t)h->Npad);
  SPA_AL(h->llp, 8 * (size_t)h->Npad);
  SPA_AL(h->lltmp, 8 * (size_t)h->Npad);
  SPA_AL(h->logw, 8 * (size_t)h->Npad);
  SPA_AL(h->lpc, 8 * (size_t)h->Npad);
  SPA_AL(h->lpp, 8 * (size_t)h->Npad);
  SPA_AL(h->lqf, 8 * (size_t)h->Npad);
  SPA_AL(h->acc, 4 * (size_t)h->Npad);
  SPA_AL(h->anc, 4 * (size_t)h->Npad);
  SPA_AL(h->sigma, 8 * kMaxPP);
  SPA_AL(h->mc, 8 * 4 * kMaxPP);
  SPA_AL(h->mean_path, 8 * (size_t)h->T * p);
  SPA_AL(h->var_path, 8 * (size_t)h->T * p);
  SPA_AL(h->part, 8 * 3 * (size_t)moments_chunks(h->N) * p);
  SPA_AL(h->cdf, 8 * (size_t)h->Npad);
  h->cdf_cap = h->Npad;
  SPA_AL(h->rw_part, 8 * 3 * (size_t)reweight_blocks(h->Npad, p));
  SPA_AL(h->btot, 8 * (size_t)kResampleBlocks);
  SPA_AL(h->wpart, 8 * 2 * (size_t)kResampleBlocks);
  SPA_AL(h->scal, 8 * 16);
  SPA_AL(h->dcount, 16);
#undef SPA_AL
  if (hipHostMalloc(reinterpret_cast<void **>(&h->hscal), 16 * sizeof(double)) != hipSuccess ||
      hipHostMalloc(reinterpret_cast<void **>(&h->hcount), 2 * sizeof(long long)) != hipSuccess) {
    set_err(h, SPA_ERR_ALLOC, "hipHostMalloc failed");
    return fail(SPA_ERR_ALLOC);
  }
  // the FP8 multi-term sampler packs its proposals into FP8 terms and contracts the FP8
  // genotype copy: the BF16 operand and genotype copies are made only if a BF16 call asks
  if (!h->f8_terms && (st = ensure_op(h, h->op, h->prec, h->PP, h->Npad)) != SPA_OK) return fail(st);

  // ---- operand preparation (once)
  he = hipMemcpyAsync(h->dX, X_host, (size_t)n * p, hipMemcpyHostToDevice, h->stream);
  if (he == hipSuccess) he = hipMemcpyAsync(h->dy, y_host, (size_t)n, hipMemcpyHostToDevice, h->stream);
  if (he != hipSuccess) {
    hip_fail(h, he, "hipMemcpyAsync");
    return fail(SPA_ERR_HIP);
  }
  launch_col_stats(h->dX, h->dy, n, p, h->mu, h->s, h->inv_s, h->ytil, h->dbad, h->stream);
  if (!h->f8_terms && (st = ensure_xpack(h, h->prec)) != SPA_OK) return fail(st);
  if (h->move == SPA_MOVE_SINGLE) {
    h->ss_rows = single_site_rows(n);   // n <= single_site_max_n() was checked above
    if ((st = dalloc(h, &h->xs_ss, h->psz * (size_t)p * h->ss_rows)) != SPA_OK) return fail(st);
    if ((st = dalloc(h, &h->yv_ss, h->psz * (size_t)h->ss_rows)) != SPA_OK) return fail(st);
    he = launch_std_cols(h->f64, h->dX, n, p, h->ss_rows, h->mu, h->s, h->xs_ss, h->stream);
    if (he != hipSuccess) {
      hip_fail(h, he, "std_cols");
      return fail(SPA_ERR_HIP);
    }
    launch_labels(h->dy, n, h->ss_rows, h->f64, h->yv_ss, h->stream);
    if (!h->f64) {
      if ((st = dalloc(h, &h->cs_ss, sizeof(float) * (size_t)p)) != SPA_OK) return fail(st);
      he = launch_lin_cols(static_cast<const float *>(h->xs_ss), static_cast<const float *>(h->yv_ss), n, p,
                           h->ss_rows, h->cs_ss, h->stream);
      if (he != hipSuccess) {
        hip_fail(h, he, "lin_cols");
        return fail(SPA_ERR_HIP);
      }
    }
  }

  // ---- initial particles: beta = 0, burn-in targeting pi_1, equal weights
  launch_fill(h->logw, h->N, -std::log(static_cast<double>(h->N)), h->stream);
  launch_fill(h->sigma, p, 2.0 / std::sqrt(static_cast<double>(n)), h->stream);
  if ((st = eval_state(h, h->beta, h->ll, h->gl)) != SPA_OK) return fail(st);
  if (h->move == SPA_MOVE_SINGLE && h->init_sweeps > 0) {   // one launch: fixed variance, no adaptation
    launch_zero_int(h->acc, h->N, h->stream);
    if ((st = single_site_cycles(h, 0, h->init_sweeps, h->lambda[0])) != SPA_OK) return fail(st);
  }
  for (int s = 0; s < (h->move == SPA_MOVE_SINGLE ? 0 : h->init_sweeps); ++s) {
    if (s == h->init_sweeps / 2) {
      launch_moments(h->f64, h->beta, h->logw, nullptr, h->N, p, h->part, nullptr, nullptr, h->sigma, kSigmaFloor,
                     h->stream);
    }
    if ((st = sweep(h, 0, s, h->lambda[0])) != SPA_OK) return fail(st);   // zeroes the accept counters
    long long cnt = 0;
    if ((st = read_count(h, &cnt)) != SPA_OK) return fail(st);
    adapt_step(h, static_cast<double>(cnt) / h->N);
  }
  if ((st = record_moments(h, 0)) != SPA_OK) return fail(st);
  he = hipStreamSynchronize(h->stream);
  if (he != hipSuccess) {
    hip_fail(h, he, "init");
    return fail(SPA_ERR_HIP);
  }
  h->t = 1;
  h->log_z = 0.0;
  spa_smc_stats s0{};
  s0.t = 1;
  s0.resampled = 0;
  s0.lambda = h->lambda[0];
  s0.ess = h->N;
  s0.log_z_inc = 0.0;
  s0.log_z = 0.0;
  s0.accept_rate = NAN;
  s0.step = h->step;
  h->stats.assign(1, s0);
  h->logz_path.assign(h->T, 0.0);
  *out = h;
  return SPA_OK;
}

extern "C" spa_status spa_smc_step(spa_smc *h, spa_smc_stats *out) {
  if (!h) return set_err(nullptr, SPA_ERR_ARG, "handle is NULL");
  if (h->t < 1) return set_err(h, SPA_ERR_STATE, "handle not initialised");
  if (h->t >= h->T) return set_err(h, SPA_ERR_STATE, "already at the last scale");
  const int t_new = h->t + 1;                // 1-based index of the new target
  const double lam_new = h->lambda[t_new - 1], lam_old = h->lambda[t_new - 2];
  const bool mala = h->move == SPA_MOVE_MALA;
  spa_status st;

  // ---- incremental weights, normalisation, ESS, resampling decision (Section 4)
  ReweightArgs ra{};
  ra.beta = h->beta;
  ra.M = h->N;
  ra.p = h->p;
  ra.a = h->a;
  ra.a_inf = h->a_inf;
  ra.lam_new = lam_new;
  ra.lam_old = lam_old;
  ra.ess_frac = h->ess_frac;
  ra.logw = h->logw;
  ra.part = h->rw_part;
  ra.scalars = h->scal;
  tbeg(h, SPA_T_REWEIGHT);
  launch_reweight(h->f64, ra, h->stream);
  tend(h);
  SPA_CK(h, hipGetLastError());
  SPA_CK(h, hipMemcpyAsync(h->hscal, h->scal, 8 * sizeof(double), hipMemcpyDeviceToHost, h->stream));
  SPA_CK(h, hipStreamSynchronize(h->stream));
  tflush(h);
  const double ess = h->hscal[0], L = h->hscal[1];
  const bool resampled = h->hscal[2] != 0.0;
  if (h->hscal[4] != 0.0) return set_err(h, SPA_ERR_NUMERIC, "non-finite weights");
  if (resampled) {   // systematic resampling and the gather; log weights become -log N
    ResampleArgs rs{};
    rs.mode = 0;
    rs.M = h->N;
    rs.K = 53 - ceil_log2(h->N);
    rs.u32 = philox_w0(0, 0, 0, (static_cast<uint32_t>(t_new) << 4) | 2u, h->k0, h->k1);
    rs.logw = h->logw;
    rs.logw_eq = -std::log(static_cast<double>(h->N));
    rs.cdf = h->cdf;
    rs.btot = h->btot;
    rs.wpart = h->wpart;
    rs.scalars = h->scal;
    rs.anc = h->anc;
    rs.p = h->p;
    rs.src = h->beta;
    rs.dst = h->tmp;
    rs.gsrc = mala ? h->gl : nullptr;
    rs.gdst = mala ? h->gltmp : nullptr;
    rs.llsrc = h->ll;
    rs.lldst = h->lltmp;
    tbeg(h, SPA_T_LSE);
    launch_resample(h->f64, rs, h->stream);
    tend(h);
    SPA_CK(h, hipGetLastError());
    std::swap(h->beta, h->tmp);
    if (mala) std::swap(h->gl, h->gltmp);
    std::swap(h->ll, h->lltmp);
  }
  // ---- preconditioner from the reweighted cloud (normalising the log weights by L
  // unless resampling reset them), then the moves targeting pi_t
  tbeg(h, SPA_T_MOMENTS);
  launch_moments(h->f64, h->beta, h->logw, resampled ? nullptr : h->scal + 1, h->N, h->p, h->part, nullptr, nullptr,
                 h->sigma, kSigmaFloor, h->stream);
  tend(h);
  const double step_used = h->step;
  if (h->move == SPA_MOVE_SINGLE) {
    launch_zero_int(h->acc, h->N, h->stream);
    if (h->sweeps > 0 && (st = single_site_cycles(h, t_new, h->sweeps, lam_new)) != SPA_OK) return st;
  } else {   // the first sweep's move-constants launch zeroes the accept counters
    for (int s = 0; s < h->sweeps; ++s)
      if ((st = sweep(h, t_new, s, lam_new, s > 0, s + 1 < h->sweeps)) != SPA_OK) return st;
  }
  // accept count and non-finite log-likelihoods, read back with the step's one final
  // synchronisation (after the per-scale records are enqueued)
  launch_count(h->acc, h->N, h->ll, h->dcount, h->stream);
  SPA_CK(h, hipMemcpyAsync(h->hcount, h->dcount, 2 * sizeof(long long), hipMemcpyDeviceToHost, h->stream));
  if ((st = record_moments(h, t_new - 1)) != SPA_OK) return st;
  if ((st = record_summaries(h, t_new - 1)) != SPA_OK) return st;
  if ((st = record_map(h, t_new - 1)) != SPA_OK) return st;
  SPA_CK(h, hipStreamSynchronize(h->stream));
  tflush(h);
  const long long cnt = h->hcount[0], bad_ll = h->hcount[1];
  if (bad_ll) return set_err(h, SPA_ERR_NUMERIC, std::to_string(bad_ll) + " particle(s) with a non-finite log-likelihood");
  const double upd = static_cast<double>(h->N) * (h->move == SPA_MOVE_SINGLE ? h->p : 1);   // MH decisions per sweep
  const double acc_rate = h->sweeps > 0 ? static_cast<double>(cnt) / (upd * h->sweeps) : NAN;
  if (h->sweeps > 0) adapt_step(h, acc_rate);
  h->log_z += L;
  h->t = t_new;
  h->logz_path[t_new - 1] = h->log_z;
  spa_smc_stats s{};
  s.t = t_new;
  s.resampled = resampled ? 1 : 0;
  s.lambda = lam_new;
  s.ess = ess;
  s.log_z_inc = L;
  s.log_z = h->log_z;
  s.accept_rate = acc_rate;
  s.step = step_used;
  h->stats.push_back(s);
  if (out) *out = s;
  return SPA_OK;
}

static spa_status prep_operand(spa_smc *h, const void *beta, int M, int is_f64, Prec prec) {
  spa_status st;
  if ((st = ensure_xpack(h, prec)) != SPA_OK) return st;
  const int PP = h->xp[static_cast<int>(prec)].PP;
  const int Mpad = round_up(M, kPartPad);
  OpScratch &o = h->scr[static_cast<int>(prec)];
  if ((st = ensure_op(h, o, prec, PP, Mpad)) != SPA_OK) return st;
  launch_pack_b(prec, is_f64 != 0, beta, M, Mpad, h->p, PP, h->mu, h->s, h->inv_s, h->ytil, o.Bhi, o.Blo,
                o.moff, o.yb, h->stream);
  SPA_CK(h, hipGetLastError());
  return SPA_OK;
}

static bool valid_prec(spa_prec p) { return p == SPA_PREC_FP64 || p == SPA_PREC_FP32 || p == SPA_PREC_BF16X2; }


extern "C" spa_status spa_smc_loglik(spa_smc *h, const void *beta_dev, int32_t M, int32_t beta_is_fp64,
                                     spa_prec prec, double *loglik_dev) {
  if (!h) return set_err(nullptr, SPA_ERR_ARG, "handle is NULL");
  if (!beta_dev || !loglik_dev || M < 1) return set_err(h, SPA_ERR_ARG, "null pointer or M < 1");
  if (prec == SPA_PREC_FP8X3 || prec == SPA_PREC_FP8X4)
    return fp8x_contract(h, beta_dev, M, beta_is_fp64, prec == SPA_PREC_FP8X3 ? 3 : 4, loglik_dev, true, nullptr);
  if (!valid_prec(prec)) return set_err(h, SPA_ERR_ARG, "bad prec");
  if (prec == SPA_PREC_FP64 && h->p > 255) return set_err(h, SPA_ERR_ARG, "FP64 path needs p <= 255");
  const Prec P = to_prec(prec);
  spa_status st;
  if ((st = prep_operand(h, beta_dev, M, beta_is_fp64, P)) != SPA_OK) return st;
  return run_gemm(h, P, h->scr[static_cast<int>(P)], M, false, loglik_dev, nullptr);
}

extern "C" spa_status spa_smc_loglik_noalloc(spa_smc *h, const void *beta_dev, int32_t M, int32_t beta_is_fp64,
                                             spa_prec prec, double *loglik_dev) {
  if (!h) return set_err(nullptr, SPA_ERR_ARG, "handle is NULL");
  if (!beta_dev || !loglik_dev || M < 1) return set_err(h, SPA_ERR_ARG, "null pointer or M < 1");
  if (!valid_prec(prec)) return set_err(h, SPA_ERR_ARG, "bad prec (FP64, FP32 or BF16X2 without allocation)");
  if (prec == SPA_PREC_FP64 && h->p > 255) return set_err(h, SPA_ERR_ARG, "FP64 path needs p <= 255");
  const Prec P = to_prec(prec);
  const XPack &x = h->xp[static_cast<int>(P)];
  if (!x.ready)
    return set_err(h, SPA_ERR_STATE, "genotype copy of this precision not prepared (call spa_smc_loglik with it once)");
  if (!h->noalloc) return set_err(h, SPA_ERR_STATE, "no scratch address for this device");
  size_t off[5];
  const size_t need = noalloc_layout(h, P, M, off);
  if (need > kNoAllocBytes)
    return set_err(h, SPA_ERR_ARG, "M too large for the static scratch (" + std::to_string(need) + " bytes needed, " +
                                       std::to_string(kNoAllocBytes) + " available)");
  char *base = static_cast<char *>(h->noalloc);
  OpScratch o{};
  o.Bhi = base + off[0];
  o.Blo = base + (P == Prec::BF16X2 ? off[1] : off[0]);
  o.moff = reinterpret_cast<double *>(base + off[2]);
  o.yb = reinterpret_cast<double *>(base + off[3]);
  o.cap = static_cast<size_t>(round_up(M, kPartPad));
  o.PP = x.PP;
  // every padded row and column of the operand is written here, and the contraction writes
  // every partial it reads, so nothing left by an earlier call is read
  launch_pack_b(P, beta_is_fp64 != 0, beta_dev, M, static_cast<int>(o.cap), h->p, o.PP, h->mu, h->s, h->inv_s,
                h->ytil, o.Bhi, o.Blo, o.moff, o.yb, h->stream);
  SPA_CK(h, hipGetLastError());
  GemmArgs a = gemm_args_core(h, P, o, M, false, loglik_dev, nullptr);
  if ((size_t)a.M_pad > o.cap) return set_err(h, SPA_ERR_ARG, "operand rows not padded");
  if (a.S > 1) a.spl_part = reinterpret_cast<double *>(base + off[4]);
  SPA_CK(h, launch_loglik(a, h->stream));
  if (a.S > 1) SPA_CK(h, launch_gemm_finalize(a, h->stream));
  return SPA_OK;
}

extern "C" spa_status spa_smc_grad(spa_smc *h, const void *beta_dev, int32_t M, int32_t beta_is_fp64,
                                   double lambda, spa_prec prec, void *grad_dev, double *logpost_dev) {
  if (!h) return set_err(nullptr, SPA_ERR_ARG, "handle is NULL");
  if (!beta_dev || !grad_dev || M < 1) return set_err(h, SPA_ERR_ARG, "null pointer or M < 1");
  if (!(lambda > 0.0) || !std::isfinite(lambda)) return set_err(h, SPA_ERR_ARG, "lambda must be > 0");
  if (!valid_prec(prec)) return set_err(h, SPA_ERR_ARG, "bad prec");
  if (prec == SPA_PREC_FP64 && h->p > 255) return set_err(h, SPA_ERR_ARG, "FP64 path needs p <= 255");
  const Prec P = to_prec(prec);
  spa_status st;
  if ((st = prep_operand(h, beta_dev, M, beta_is_fp64, P)) != SPA_OK) return st;
  if (h->llscr_cap < (size_t)M) {
    dfree(h, h->llscr);
    h->llscr = nullptr;
    if ((st = dalloc(h, &h->llscr, 8 * (size_t)M)) != SPA_OK) return st;
    h->llscr_cap = M;
  }
  const bool native_f64 = P == Prec::F64;
  void *gout = grad_dev;
  if (native_f64 != (beta_is_fp64 != 0)) {   // contraction dtype differs from the caller's
    const size_t need = (native_f64 ? 8 : 4) * (size_t)M * h->p;
    if (h->gscr_cap < need) {
      dfree(h, h->gscr);
      h->gscr = nullptr;
      if ((st = dalloc(h, &h->gscr, need)) != SPA_OK) return st;
      h->gscr_cap = need;
    }
    gout = h->gscr;
  }
  if ((st = run_gemm(h, P, h->scr[static_cast<int>(P)], M, true, h->llscr, gout)) != SPA_OK) return st;
  launch_add_prior(beta_is_fp64 != 0, native_f64, beta_dev, M, h->p, make_prior(h, lambda), gout, h->llscr,
                   logpost_dev, h->stream);
  if (gout != grad_dev) launch_convert(native_f64, gout, grad_dev, (size_t)M * h->p, h->stream);
  SPA_CK(h, hipGetLastError());
  return SPA_OK;
}

extern "C" spa_status spa_smc_resample(spa_smc *h, const double *w_dev, int32_t M, uint32_t u32,
                                       int32_t *ancestors_dev) {
  if (!h) return set_err(nullptr, SPA_ERR_ARG, "handle is NULL");
  if (!w_dev || !ancestors_dev || M < 1) return set_err(h, SPA_ERR_ARG, "null pointer or M < 1");
  if (M > (1 << 24)) return set_err(h, SPA_ERR_ARG, "M must be <= 2^24");
  spa_status st;
  if (h->cdf_cap < (size_t)M) {
    dfree(h, h->cdf);
    h->cdf = nullptr;
    if ((st = dalloc(h, &h->cdf, 8 * (size_t)M)) != SPA_OK) return st;
    h->cdf_cap = M;
  }
  ResampleArgs rs{};
  rs.mode = 1;
  rs.M = M;
  rs.K = 53 - ceil_log2(M);
  rs.u32 = u32;
  rs.w = w_dev;
  rs.cdf = h->cdf;
  rs.btot = h->btot;
  rs.wpart = h->wpart;
  rs.scalars = h->scal;
  rs.anc = ancestors_dev;
  launch_resample(false, rs, h->stream);
  SPA_CK(h, hipGetLastError());
  SPA_CK(h, hipMemcpyAsync(h->hscal, h->scal, 8 * sizeof(double), hipMemcpyDeviceToHost, h->stream));
  SPA_CK(h, hipStreamSynchronize(h->stream));
  if (h->hscal[5] != 0.0) return set_err(h, SPA_ERR_NUMERIC, "weights must be finite, >= 0 and not all zero");
  return SPA_OK;
}

extern "C" spa_status spa_weighted_summaries(spa_smc *h, const void *values_dev, int32_t M, int32_t p,
                                             int32_t values_are_fp64, const double *w_dev, const double *levels,
                                             int32_t L, const double *deltas, int32_t D, double *quant_dev,
                                             double *conc_dev) {
  if (!h) return set_err(nullptr, SPA_ERR_ARG, "handle is NULL");
  if (!values_dev || !w_dev) return set_err(h, SPA_ERR_ARG, "values/weights is NULL");
  if (M < 1 || p < 1) return set_err(h, SPA_ERR_SHAPE, "M and p must be >= 1");
  SqLevels lv;
  spa_status st = parse_levels(h, levels, L, deltas, D, &lv);
  if (st != SPA_OK) return st;
  if ((L > 0 && !quant_dev) || (D > 0 && !conc_dev)) return set_err(h, SPA_ERR_ARG, "output is NULL");
  if ((st = run_summaries(h, values_dev, values_are_fp64 != 0, M, p, w_dev, false, lv, quant_dev, conc_dev)) !=
      SPA_OK)
    return st;
  SPA_CK(h, hipMemcpyAsync(h->hscal + 8, &h->sq_st->flags, sizeof(int), hipMemcpyDeviceToHost, h->stream));
  SPA_CK(h, hipStreamSynchronize(h->stream));
  tflush(h);
  int flags = 0;
  std::memcpy(&flags, h->hscal + 8, sizeof(int));
  if (flags & 1) return set_err(h, SPA_ERR_NUMERIC, "weights must be finite, >= 0 and not all zero");
  return SPA_OK;
}

extern "C" spa_status spa_smc_set_summaries(spa_smc *h, const double *levels, int32_t L, const double *deltas,
                                            int32_t D, int32_t keep_history) {
  if (!h) return set_err(nullptr, SPA_ERR_ARG, "handle is NULL");
  if (h->t < 1) return set_err(h, SPA_ERR_STATE, "handle not initialised");
  if (h->sq_on) return set_err(h, SPA_ERR_STATE, "summaries already configured");
  if (keep_history && h->t != 1) return set_err(h, SPA_ERR_STATE, "the history must start at the first scale");
  SqLevels lv;
  spa_status st = parse_levels(h, levels, L, deltas, D, &lv);
  if (st != SPA_OK) return st;
  const size_t T = h->T, p = h->p, N = h->N;
  if (L && (st = dalloc(h, &h->quant_path, 8 * T * L * p)) != SPA_OK) return st;
  if (D && (st = dalloc(h, &h->conc_path, 8 * T * D * p)) != SPA_OK) return st;
  if (keep_history) {
    if ((st = dalloc(h, &h->hist_beta, h->psz * T * N * p)) != SPA_OK) return st;
    if ((st = dalloc(h, &h->hist_logw, 8 * T * N)) != SPA_OK) return st;
  }
  h->sq_lv = lv;
  h->sq_on = true;
  h->sq_keep = keep_history != 0;
  for (int row = 0; row < h->t; ++row) {   // the current scale (rows before it are not kept)
    if (row != h->t - 1) continue;
    if ((st = record_summaries(h, row)) != SPA_OK) return st;
  }
  SPA_CK(h, hipStreamSynchronize(h->stream));
  tflush(h);
  return SPA_OK;
}

extern "C" spa_status spa_smc_get_summaries(const spa_smc *h, const double **quant_path_dev,
                                            const double **conc_path_dev) {
  if (!h) return set_err(nullptr, SPA_ERR_ARG, "handle is NULL");
  if (!h->sq_on) return SPA_ERR_STATE;
  if (quant_path_dev) *quant_path_dev = h->quant_path;
  if (conc_path_dev) *conc_path_dev = h->conc_path;
  return SPA_OK;
}

extern "C" spa_status spa_smc_marginal_summaries(spa_smc *h, double *quant_dev, double *conc_dev,
                                                 double *scale_post_dev) {
  if (!h) return set_err(nullptr, SPA_ERR_ARG, "handle is NULL");
  if (!h->sq_on || !h->sq_keep) return set_err(h, SPA_ERR_STATE, "no particle history (spa_smc_set_summaries)");
  const SqLevels &lv = h->sq_lv;
  if ((lv.L > 0 && !quant_dev) || (lv.D > 0 && !conc_dev)) return set_err(h, SPA_ERR_ARG, "output is NULL");
  const int T = h->t, N = h->N;
  const size_t M = (size_t)T * N;
  if (M > 0x7fffffff) return set_err(h, SPA_ERR_SHAPE, "history too large");
  spa_status st;
  if (h->sq_w_cap < M) {
    dfree(h, h->sq_w);
    h->sq_w = nullptr;
    if ((st = dalloc(h, &h->sq_w, 8 * M)) != SPA_OK) return st;
    h->sq_w_cap = M;
  }
  if (!h->sq_logz && (st = dalloc(h, &h->sq_logz, 8 * (size_t)h->T)) != SPA_OK) return st;
  SPA_CK(h, hipMemcpyAsync(h->sq_logz, h->logz_path.data(), 8 * (size_t)T, hipMemcpyHostToDevice, h->stream));
  tbeg(h, SPA_T_SUMMARY);
  SPA_CK(h, launch_mixture_weights(h->sq_logz, T, N, h->hist_logw, h->sq_w, scale_post_dev, h->stream));
  tend(h);
  if ((st = run_summaries(h, h->hist_beta, h->f64, static_cast<int>(M), h->p, h->sq_w, false, lv, quant_dev,
                          conc_dev)) != SPA_OK)
    return st;
  SPA_CK(h, hipStreamSynchronize(h->stream));
  tflush(h);
  return SPA_OK;
}

extern "C" spa_status spa_smc_get(const spa_smc *h, const void **beta_dev, const double **logw_dev,
                                  const double **mean_path_dev, const double **var_path_dev,
                                  const double **logz_path_host, int32_t *t_out) {
  if (!h) return SPA_ERR_ARG;
  if (beta_dev) *beta_dev = h->beta;
  if (logw_dev) *logw_dev = h->logw;
  if (mean_path_dev) *mean_path_dev = h->mean_path;
  if (var_path_dev) *var_path_dev = h->var_path;
  if (logz_path_host) *logz_path_host = h->logz_path.data();
  if (t_out) *t_out = h->t;
  return SPA_OK;
}

extern "C" spa_status spa_map_em(spa_smc *h, const void *beta0_dev, int32_t M, int32_t beta_is_fp64,
                                 double lambda, int32_t outer, int32_t inner, double *mode_dev,
                                 double *logpost_dev) {
  if (!h) return set_err(nullptr, SPA_ERR_ARG, "handle is NULL");
  if (!beta0_dev || !mode_dev || !logpost_dev) return set_err(h, SPA_ERR_ARG, "NULL pointer");
  if (M < 1) return set_err(h, SPA_ERR_SHAPE, "M must be >= 1");
  if (!(lambda > 0.0) || !std::isfinite(lambda)) return set_err(h, SPA_ERR_ARG, "lambda must be > 0");
  if (outer < 0 || inner < 0) return set_err(h, SPA_ERR_ARG, "iteration counts must be >= 0");
  if (h->n > map_max_n() || h->p > kMapMaxP) return set_err(h, SPA_ERR_SHAPE, "n > 10240 or p > 512");
  return run_map_em(h, beta0_dev, beta_is_fp64 != 0, M, lambda, outer, inner, mode_dev, logpost_dev);
}

extern "C" spa_status spa_smc_set_map(spa_smc *h, int32_t outer, int32_t inner) {
  if (!h) return set_err(nullptr, SPA_ERR_ARG, "handle is NULL");
  if (h->t < 1) return set_err(h, SPA_ERR_STATE, "handle not initialised");
  if (h->map_on) return set_err(h, SPA_ERR_STATE, "MAP path already configured");
  if (outer < 0 || inner < 0) return set_err(h, SPA_ERR_ARG, "iteration counts must be >= 0");
  if (h->n > map_max_n() || h->p > kMapMaxP) return set_err(h, SPA_ERR_SHAPE, "n > 10240 or p > 512");
  spa_status st;
  const size_t T = h->T, p = h->p;
  if ((st = dalloc(h, &h->map_path, 8 * T * p)) != SPA_OK) return st;
  if ((st = dalloc(h, &h->map_lp, 8 * T)) != SPA_OK) return st;
  if ((st = dalloc(h, &h->map_best, 16)) != SPA_OK) return st;
  if ((st = dalloc(h, &h->map_starts, 8 * 2 * p)) != SPA_OK) return st;
  if ((st = dalloc(h, &h->map_modes, 8 * 2 * p)) != SPA_OK) return st;
  if ((st = dalloc(h, &h->map_mlp, 16)) != SPA_OK) return st;
  h->map_on = true;
  h->map_outer = outer;
  h->map_inner = inner;
  if ((st = record_map(h, h->t - 1)) != SPA_OK) return st;
  SPA_CK(h, hipStreamSynchronize(h->stream));
  tflush(h);
  return SPA_OK;
}

extern "C" spa_status spa_smc_get_map(const spa_smc *h, const double **map_path_dev, const double **logpost_path_dev) {
  if (!h) return set_err(nullptr, SPA_ERR_ARG, "handle is NULL");
  if (!h->map_on) return SPA_ERR_STATE;
  if (map_path_dev) *map_path_dev = h->map_path;
  if (logpost_path_dev) *logpost_path_dev = h->map_lp;
  return SPA_OK;
}

extern "C" spa_status spa_smc_get_loglik(const spa_smc *h, const double **loglik_dev) {
  if (!h || !loglik_dev) return set_err(const_cast<spa_smc *>(h), SPA_ERR_ARG, "NULL argument");
  *loglik_dev = h->ll;
  return SPA_OK;
}

extern "C" spa_status spa_smc_get_stats(const spa_smc *h, int32_t t, spa_smc_stats *out) {
  if (!h || !out) return SPA_ERR_ARG;
  if (t < 1 || t > (int)h->stats.size()) return SPA_ERR_ARG;
  *out = h->stats[t - 1];
  return SPA_OK;
}

extern "C" spa_status spa_smc_set_state(spa_smc *h, const void *beta_dev, const double *logw_dev, int32_t t,
                                        double step) {
  if (!h) return set_err(nullptr, SPA_ERR_ARG, "handle is NULL");
  if (!beta_dev || !logw_dev) return set_err(h, SPA_ERR_ARG, "null pointer");
  if (t < 1 || t > h->T) return set_err(h, SPA_ERR_ARG, "t out of range");
  if (!(step > 0.0) || !std::isfinite(step)) return set_err(h, SPA_ERR_ARG, "step must be > 0");
  SPA_CK(h, hipMemcpyAsync(h->beta, beta_dev, h->psz * (size_t)h->N * h->p, hipMemcpyDeviceToDevice, h->stream));
  SPA_CK(h, hipMemcpyAsync(h->logw, logw_dev, 8 * (size_t)h->N, hipMemcpyDeviceToDevice, h->stream));
  spa_status st;
  if ((st = eval_state(h, h->beta, h->ll, h->gl)) != SPA_OK) return st;
  // the log Z path before t is unknown for an injected state: restart the record at t
  h->t = t;
  h->step = step;
  h->log_z = 0.0;
  std::fill(h->logz_path.begin(), h->logz_path.end(), 0.0);
  spa_smc_stats s{};
  s.t = t;
  s.lambda = h->lambda[t - 1];
  s.ess = NAN;
  s.accept_rate = NAN;
  s.step = step;
  h->stats.assign(t, s);
  SPA_CK(h, hipStreamSynchronize(h->stream));
  return SPA_OK;
}

extern "C" spa_status spa_philox4x32_10(spa_smc *h, const uint32_t *ctr_dev, int32_t M, uint64_t seed,
                                        uint32_t *out_dev) {
  if (!h) return set_err(nullptr, SPA_ERR_ARG, "handle is NULL");
  if (!ctr_dev || !out_dev || M < 1) return set_err(h, SPA_ERR_ARG, "null pointer or M < 1");
  launch_philox(ctr_dev, M, static_cast<uint32_t>(seed & 0xFFFFFFFFull), static_cast<uint32_t>(seed >> 32),
                out_dev, h->stream);
  SPA_CK(h, hipGetLastError());
  return SPA_OK;
}

extern "C" spa_status spa_smc_set_timing(spa_smc *h, int32_t enable) {
  return spa_smc_set_timing_classes(h, enable ? (1u << SPA_TIMING_CLASSES) - 1u : 0u);
}

extern "C" spa_status spa_smc_set_timing_classes(spa_smc *h, uint32_t class_mask) {
  if (!h) return set_err(nullptr, SPA_ERR_ARG, "handle is NULL");
  if (class_mask >> SPA_TIMING_CLASSES) return set_err(h, SPA_ERR_ARG, "timing class mask has unknown bits");
  SPA_CK(h, hipStreamSynchronize(h->stream));
  tflush(h);
  h->tmask = class_mask;
  h->timing = class_mask != 0;
  h->topen = false;
  for (int c = 0; c < SPA_TIMING_CLASSES; ++c) {
    h->t_ms[c] = 0.0;
    h->t_cnt[c] = 0;
  }
  return SPA_OK;
}

extern "C" spa_status spa_smc_get_timing(spa_smc *h, double *ms, int64_t *launches) {
  if (!h || !ms || !launches) return SPA_ERR_ARG;
  SPA_CK(h, hipStreamSynchronize(h->stream));
  tflush(h);
  for (int c = 0; c < SPA_TIMING_CLASSES; ++c) {
    ms[c] = h->t_ms[c];
    launches[c] = h->t_cnt[c];
  }
  return SPA_OK;
}

extern "C" void spa_smc_destroy(spa_smc *h) {
  if (!h) return;
  (void)hipStreamSynchronize(h->stream);
  for (void *v : h->allocs) (void)hipFree(v);
  for (hipEvent_t e : h->ev) (void)hipEventDestroy(e);
  if (h->hscal) (void)hipHostFree(h->hscal);
  if (h->hcount) (void)hipHostFree(h->hcount);
  delete h;
}

extern "C" const char *spa_smc_last_error(const spa_smc *h) {
  if (!h) return g_init_error.c_str();
  return h->err.c_str();
}
