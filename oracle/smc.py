"""SMC sampler indexed on the generalized-t scale, oracle side (Section 4, Section 4.1).

Test infrastructure only (see the package docstring).

Targets pi_t(beta) proportional to f(y | X, beta) Gt(beta | a, lam_t) for a strictly
decreasing scale sequence lam_1 > ... > lam_T.  With an MCMC kernel K_t invariant for
pi_t and its reversal as backward kernel, the incremental weight of a particle is the
ratio gamma_t / gamma_{t-1} evaluated at its pre-move position, which here is the
prior ratio (the likelihood cancels).  The weights are normalised, the ratio
Z_t / Z_{t-1} is estimated by sum_i W_{t-1,i} w_{t,i}, the particles are resampled
before moving when the effective sample size falls below a threshold, and then moved
by K_t.

Readings taken where the paper is silent (each also listed in the design notes):
* ESS = 1 / sum W^2 (Liu & Chen);
* resampling is systematic, given a quantised CDF (``systematic_resample``), triggered
  iff ESS < ess_frac * N (strict);
* one "sweep" is one joint p-dimensional proposal and one MH decision per particle;
  K_t is ``sweeps`` sweeps of a random walk (scale kappa * sigma_j) or of MALA with
  diagonal preconditioner M = diag(sigma^2) and step h;
* the paper's own kernel (Section 4.1, further details): one "sweep" is a cycle over
  j = 1..p of single-coordinate random-walk MH updates with proposal standard deviation
  ``step`` (the paper's variance 0.25: step 0.5, kept fixed), the linear predictor being
  updated incrementally, eta += delta X_std[:, j]; K_t is ``sweeps`` such cycles (5);
* sigma_j is the weighted standard deviation of the current particles under W_t
  before the moves (floored at 1e-12); the first half of the burn-in uses
  2 / sqrt(n), the inverse square root of the diagonal Fisher information at beta = 0,
  and the second half the standard deviation of the cloud at its midpoint;
* the proposal scale adapts after every step (every burn-in sweep):
  log s += clip(acceptance - target, -log 2, log 2), targets 0.234 (RW), 0.574 (MALA);
* initial particles: N chains from beta = 0 run for ``init_sweeps`` sweeps targeting
  pi_1 (with adaptation), then W = 1/N;
* the normalised Gt density (with its -log(2 lam) term) is used in the weights, so the
  accumulated log Z_t / Z_1 is the log marginal-likelihood ratio.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

from . import gt_prior, likelihood, philox

TARGET_ACC = {"rwm": 0.234, "mala": 0.574, "single": None}   # single-site: fixed variance
SIGMA_FLOOR = 1e-12
LOG2 = math.log(2.0)


# ---------------------------------------------------------------- weights (Section 4)

def reweight_delta(beta, a: float, lam_new: float, lam_old: float):
    """Incremental log weight sum_j [log Gt(beta_j | a, lam_new) - log Gt(beta_j | a, lam_old)]."""
    return gt_prior.log_prior(beta, a, lam_new) - gt_prior.log_prior(beta, a, lam_old)


def logsumexp(v):
    v = np.asarray(v, dtype=np.float64)
    m = np.max(v)
    if not np.isfinite(m):
        return m
    return m + math.log(np.sum(np.exp(v - m)))


def normalise(logw):
    """Normalised log weights and log of their sum: logW = logw - LSE(logw)."""
    L = logsumexp(logw)
    return logw - L, L


def ess(logW):
    """Effective sample size 1 / sum_i W_i^2 of normalised log weights."""
    W = np.exp(np.asarray(logW, dtype=np.float64))
    return 1.0 / np.sum(W * W)


def weighted_moments(beta, logW):
    """Weighted mean and variance per coordinate: E[beta_j], E[(beta_j - E beta_j)^2]."""
    W = np.exp(np.asarray(logW, dtype=np.float64))
    W = W / np.sum(W)
    mean = W @ beta
    var = W @ (beta - mean) ** 2
    return mean, var


# ------------------------------------------------------------ systematic resampling

def ceil_log2(m: int) -> int:
    return (int(m) - 1).bit_length()


def systematic_resample(w, u32: int):
    """Systematic resampling of M weights w_i >= 0 with offset U = u32 * 2^-32.

    The weights are first quantised to integers q_i = floor((w_i / max w) 2^K), with
    K = 53 - ceil(log2 M), so that every partial sum C_k = q_0 + ... + q_k is an integer
    below 2^53 (exact in FP64 in any order).  Offspring i takes the smallest k with
    C_k > ((i + U) / M) C_{M-1}, clamped to M - 1."""
    w = np.asarray(w, dtype=np.float64)
    M = w.shape[0]
    if M < 1:
        raise ValueError("empty weight vector")
    if not np.all(np.isfinite(w)) or np.any(w < 0.0):
        raise ValueError("weights must be finite and non-negative")
    wmax = np.max(w)
    if not wmax > 0.0:
        raise ValueError("all weights are zero")
    K = 53 - ceil_log2(M)
    q = np.floor((w / wmax) * (2.0 ** K))
    C = np.cumsum(q)
    U = float(u32) * 2.0 ** -32
    tpos = ((np.arange(M, dtype=np.float64) + U) * C[-1]) / float(M)
    anc = np.searchsorted(C, tpos, side="right")
    return np.minimum(anc, M - 1).astype(np.int32)


# --------------------------------------------------------------------- the sampler

@dataclass
class Problem:
    """Data of one run: standardised genotypes, labels and the prior's a."""
    Xs: np.ndarray
    y: np.ndarray
    a: float
    likelihood_off: bool = False   # loglik == 0 (the sampler then targets the prior)

    @property
    def n(self):
        return self.Xs.shape[0]

    @property
    def p(self):
        return self.Xs.shape[1]

    def loglik(self, beta):
        if self.likelihood_off:
            return np.zeros(beta.shape[0])
        return likelihood.loglik(beta, self.Xs, self.y)

    def loglik_and_grad(self, beta):
        if self.likelihood_off:
            return np.zeros(beta.shape[0]), np.zeros_like(beta)
        return likelihood.loglik_and_grad(beta, self.Xs, self.y)


@dataclass
class State:
    beta: np.ndarray      # (N, p)
    ll: np.ndarray        # (N,) log-likelihood at beta
    gl: np.ndarray        # (N, p) log-likelihood gradient at beta (MALA only)
    logW: np.ndarray      # (N,) normalised log weights


def rwm_sweep(prob: Problem, st: State, lam: float, kappa: float, sigma, seed: int,
              sweep: int, t: int) -> int:
    """One joint random-walk MH sweep targeting pi(. | lam); returns the accept count."""
    N, p = st.beta.shape
    xi = philox.proposal_normals(seed, N, p, sweep, t)
    prop = st.beta + kappa * sigma * xi
    ll_p = prob.loglik(prop)
    log_alpha = (ll_p - st.ll + gt_prior.log_prior(prop, prob.a, lam)
                 - gt_prior.log_prior(st.beta, prob.a, lam))
    u = philox.mh_uniforms(seed, N, sweep, t)
    acc = np.log(u) < log_alpha
    st.beta[acc] = prop[acc]
    st.ll[acc] = ll_p[acc]
    return int(np.count_nonzero(acc))


def mala_sweep(prob: Problem, st: State, lam: float, h: float, sigma, seed: int,
               sweep: int, t: int) -> int:
    """One preconditioned MALA sweep targeting pi(. | lam): proposal
    N(beta + (h/2) M grad log pi(beta), h M), M = diag(sigma^2); returns the accept count."""
    N, p = st.beta.shape
    s2 = sigma * sigma
    g = st.gl + gt_prior.gt_grad(st.beta, prob.a, lam)
    mean_f = st.beta + 0.5 * h * s2 * g
    xi = philox.proposal_normals(seed, N, p, sweep, t)
    prop = mean_f + math.sqrt(h) * sigma * xi
    ll_p, gl_p = prob.loglik_and_grad(prop)
    g_p = gl_p + gt_prior.gt_grad(prop, prob.a, lam)
    mean_r = prop + 0.5 * h * s2 * g_p
    lq_fwd = -np.sum((prop - mean_f) ** 2 / (2.0 * h * s2), axis=1)
    lq_rev = -np.sum((st.beta - mean_r) ** 2 / (2.0 * h * s2), axis=1)
    log_alpha = (ll_p - st.ll + gt_prior.log_prior(prop, prob.a, lam)
                 - gt_prior.log_prior(st.beta, prob.a, lam) + lq_rev - lq_fwd)
    u = philox.mh_uniforms(seed, N, sweep, t)
    acc = np.log(u) < log_alpha
    st.beta[acc] = prop[acc]
    st.ll[acc] = ll_p[acc]
    st.gl[acc] = gl_p[acc]
    return int(np.count_nonzero(acc))


def single_site_sweep(prob: Problem, st: State, lam: float, step: float, sigma, seed: int,
                      cycle: int, t: int) -> int:
    """One cycle of single-coordinate random-walk MH updates, j = 1..p in order, for every
    particle (Section 4.1): beta'_j = beta_j + step z, accepted iff
    log u < [l(beta') - l(beta)] + log Gt(beta'_j) - log Gt(beta_j), where the likelihood
    difference comes from the incrementally updated linear predictor eta = X_std beta.
    Returns the number of accepted coordinate updates."""
    N, p = st.beta.shape
    z, u = philox.single_site_draws(seed, N, p, cycle, t)
    eta = st.beta @ prob.Xs.T                        # (N, n)
    acc = 0
    for j in range(p):
        x = prob.Xs[:, j]
        delta = step * z[:, j]
        eta_p = eta + delta[:, None] * x[None, :]
        if prob.likelihood_off:
            dll = np.zeros(N)
        else:
            dll = (delta * (prob.y @ x)
                   - np.sum(likelihood.softplus(eta_p) - likelihood.softplus(eta), axis=1))
        b, bp = st.beta[:, j], st.beta[:, j] + delta
        dlp = gt_prior.gt_logpdf(bp, prob.a, lam) - gt_prior.gt_logpdf(b, prob.a, lam)
        ok = np.log(u[:, j]) < dll + dlp
        st.beta[ok, j] = bp[ok]
        eta[ok] = eta_p[ok]
        acc += int(np.count_nonzero(ok))
    st.ll = prob.loglik(st.beta)
    return acc


def adapt_step(step: float, acc_rate: float, move: str) -> float:
    """log step += clip(acceptance - target, -log 2, log 2); the single-site kernel keeps
    its proposal variance fixed."""
    if TARGET_ACC[move] is None:
        return step
    d = min(max(acc_rate - TARGET_ACC[move], -LOG2), LOG2)
    return step * math.exp(d)


@dataclass
class Result:
    lambdas: np.ndarray
    mean: np.ndarray          # (T, p) posterior means after the moves at each scale
    var: np.ndarray           # (T, p)
    ess: np.ndarray           # (T,) ESS after reweighting (N at t = 1)
    resampled: np.ndarray     # (T,) bool
    log_z_inc: np.ndarray     # (T,) log Z_t / Z_{t-1} (0 at t = 1)
    log_z: np.ndarray         # (T,) log Z_t / Z_1
    accept: np.ndarray        # (T,) acceptance rate of the moves at each scale
    step: np.ndarray          # (T,) proposal scale used at each scale
    state: State = None
    snapshots: dict = field(default_factory=dict)


def run_smc(prob: Problem, lambdas, N: int, move: str, sweeps: int, init_sweeps: int,
            ess_frac: float, step0: float, seed: int, adapt: bool = True,
            snapshot_at=(), T_stop: int | None = None) -> Result:
    """The full sweep over the scale grid; returns the per-scale summaries."""
    lam = np.asarray(lambdas, dtype=np.float64)
    T = lam.shape[0] if T_stop is None else T_stop
    n, p = prob.Xs.shape
    if move not in TARGET_ACC:
        raise ValueError(move)
    sweep_fn = {"rwm": rwm_sweep, "mala": mala_sweep, "single": single_site_sweep}[move]
    upd = N * (p if move == "single" else 1)         # MH decisions per sweep

    beta = np.zeros((N, p))
    if move == "mala":
        ll, gl = prob.loglik_and_grad(beta)
    else:
        ll, gl = prob.loglik(beta), np.zeros((N, p))
    st = State(beta=beta, ll=ll, gl=gl, logW=np.full(N, -math.log(N)))

    # burn-in targeting pi_1 from beta = 0 (Section 4.1, initial particles)
    step = float(step0)
    sigma = np.full(p, 2.0 / math.sqrt(n))
    for s in range(init_sweeps):
        if s == init_sweeps // 2:
            sigma = _preconditioner(st)
        acc = sweep_fn(prob, st, lam[0], step, sigma, seed, s, 0)
        if adapt:
            step = adapt_step(step, acc / upd, move)

    out = Result(lambdas=lam[:T], mean=np.zeros((T, p)), var=np.zeros((T, p)),
                 ess=np.zeros(T), resampled=np.zeros(T, bool), log_z_inc=np.zeros(T),
                 log_z=np.zeros(T), accept=np.zeros(T), step=np.zeros(T))
    out.mean[0], out.var[0] = weighted_moments(st.beta, st.logW)
    out.ess[0] = N
    out.step[0] = step
    out.accept[0] = np.nan
    if 1 in snapshot_at:
        out.snapshots[1] = _snap(st)

    log_z = 0.0
    for ti in range(1, T):
        t = ti + 1                                   # 1-based scale index
        delta = reweight_delta(st.beta, prob.a, lam[ti], lam[ti - 1])
        logw = st.logW + delta
        st.logW, L = normalise(logw)                 # L = log sum_i W_{t-1,i} w_{t,i}
        log_z += L
        e = ess(st.logW)
        out.ess[ti], out.log_z_inc[ti], out.log_z[ti] = e, L, log_z
        if e < ess_frac * N:
            anc = systematic_resample(np.exp(st.logW), philox.resample_u32(seed, t))
            st.beta, st.ll, st.gl = st.beta[anc], st.ll[anc], st.gl[anc]
            st.logW = np.full(N, -math.log(N))
            out.resampled[ti] = True
        sigma = _preconditioner(st)
        acc = 0
        for s in range(sweeps):
            acc += sweep_fn(prob, st, lam[ti], step, sigma, seed, s, t)
        out.accept[ti] = acc / (upd * sweeps)
        out.step[ti] = step
        if adapt:
            step = adapt_step(step, acc / (upd * sweeps), move)
        out.mean[ti], out.var[ti] = weighted_moments(st.beta, st.logW)
        if t in snapshot_at:
            out.snapshots[t] = _snap(st)
    out.state = st
    return out


def _preconditioner(st: State):
    """sigma_j: weighted standard deviation of the current particles, floored."""
    _, var = weighted_moments(st.beta, st.logW)
    return np.sqrt(np.maximum(var, SIGMA_FLOOR ** 2))


def _snap(st: State) -> State:
    return State(beta=st.beta.copy(), ll=st.ll.copy(), gl=st.gl.copy(), logW=st.logW.copy())


def run_config(cfg, X, y, seed: int | None = None, N: int | None = None,
               T_stop: int | None = None, **kw) -> Result:
    """Convenience wrapper: run the sampler for a workload configuration."""
    Xs, _, _ = likelihood.standardise(X)
    prob = Problem(Xs=Xs, y=np.asarray(y, dtype=np.float64), a=cfg.a)
    return run_smc(prob, cfg.grid(), N or cfg.N, cfg.move, cfg.sweeps, cfg.init_sweeps,
                   cfg.ess_frac, cfg.step0(), cfg.seed if seed is None else seed,
                   T_stop=T_stop, **kw)
