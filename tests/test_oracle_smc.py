"""Statistical pins of the oracle's SMC sampler (Section 4 and 4.1).

* prior only (likelihood switched off): the particles at every scale follow
  Gt(a, lam_t) (closed-form CDF) and log Z_t / Z_1 = 0;
* p = 1, 2: posterior means and log Z_t / Z_1 along the scale path agree with brute-force
  quadrature within Monte Carlo error, for both move kernels;
* p = 10: the SMC posterior mean at an intermediate scale agrees with long fixed-scale
  MCMC runs (the validation recipe of Section 4.2);
* planted mistakes in the oracle are caught by these pins.
"""
import math

import numpy as np
import pytest
from scipy import stats

from oracle import gt_prior, likelihood, quadrature, smc
from synth import CONFIGS, lambda_grid, make_dataset


def weighted_ks(x, w, cdf):
    o = np.argsort(x)
    x, w = x[o], w[o] / w.sum()
    Fw = np.cumsum(w)
    F = cdf(x)
    return max(np.max(np.abs(Fw - F)), np.max(np.abs(Fw - w - F)))


def test_prior_only_targets_are_gt():
    a, N, p = 4.0, 4096, 3
    T = 16
    lam = lambda_grid(1.0, 1e-2, T)
    prob = smc.Problem(Xs=np.zeros((10, p)), y=np.zeros(10), a=a, likelihood_off=True)
    res = smc.run_smc(prob, lam, N, "rwm", sweeps=20, init_sweeps=300, ess_frac=0.5,
                      step0=2.38 / math.sqrt(p), seed=21, snapshot_at=range(1, T + 1))
    for t in range(1, T + 1):
        st = res.snapshots[t]
        W = np.exp(st.logW)
        x = st.beta.ravel()
        w = np.repeat(W, p)
        D = weighted_ks(x, w, lambda v: gt_prior.gt_cdf(v, a, lam[t - 1]))
        assert D < 0.03, (t, D)
        # a wrong scale (b = a c instead of c) is far away
        D_wrong = weighted_ks(x, w, lambda v: gt_prior.gt_cdf(v, a, a * lam[t - 1]))
        assert D_wrong > 0.15
    assert np.all(np.abs(res.log_z) < 0.15), res.log_z


def _tiny_dataset(p, seed):
    cfg = CONFIGS["n500_p10_rwm_fp64"].replace(k_causal=1, beta_sd=1.0, rho=0.5)
    d = make_dataset(cfg, n=60, p=p, seed=seed)
    Xs, _, _ = likelihood.standardise(d.X)
    return Xs, d.y.astype(np.float64)


@pytest.mark.parametrize("p,move", [(1, "rwm"), (2, "rwm"), (2, "mala"), (1, "single"), (2, "single")])
def test_small_p_against_quadrature(p, move):
    Xs, y = _tiny_dataset(p, seed=10 + p)
    a, T, N, R = 1.0, 12, 2000, 6
    lam = lambda_grid(1e3, 1e-2, T)
    prob = smc.Problem(Xs=Xs, y=y, a=a)
    step0 = {"rwm": 2.38 / math.sqrt(p), "mala": 1.65 ** 2 / p ** (1 / 3), "single": 0.5}[move]
    runs = [smc.run_smc(prob, lam, N, move, sweeps=5, init_sweeps=150, ess_frac=0.5,
                        step0=step0, seed=100 + r) for r in range(R)]
    means = np.stack([r.mean for r in runs])           # (R, T, p)
    logz = np.stack([r.log_z for r in runs])           # (R, T)
    q = [quadrature.posterior_summary(Xs, y, a, l, bound=8.0, lo=1e-7,
                                      panels_per_decade=2, order=16) for l in lam]
    q_logz = np.array([v[0] for v in q]) - q[0][0]
    q_mean = np.stack([v[1] for v in q])
    q_sd = np.sqrt(np.stack([v[2] for v in q]))
    se = means.std(axis=0, ddof=1) / math.sqrt(R)
    tcrit = stats.t.ppf(1 - 0.001 / (2 * T * p), R - 1)
    err = np.abs(means.mean(axis=0) - q_mean)
    assert np.all(err <= tcrit * se + 0.02 * q_sd + 1e-4), (err, se)
    se_z = logz.std(axis=0, ddof=1) / math.sqrt(R)
    err_z = np.abs(logz.mean(axis=0) - q_logz)
    assert np.all(err_z <= tcrit * se_z + 0.02), (err_z, se_z)


def test_fixed_scale_mcmc_agrees_with_smc():
    """Section 4.2's check: run MCMC at a fixed intermediate scale and compare."""
    cfg = CONFIGS["n500_p10_rwm_fp64"]
    d = make_dataset(cfg)
    Xs, _, _ = likelihood.standardise(d.X)
    prob = smc.Problem(Xs=Xs, y=d.y.astype(np.float64), a=cfg.a)
    lam = cfg.grid()
    t_stop, N = 14, 512
    smc_means = np.stack([smc.run_smc(prob, lam, N, "rwm", 5, 150, 0.5, cfg.step0(),
                                      seed=300 + r, T_stop=t_stop).mean[-1] for r in range(3)])
    mc_means = []
    for r in range(3):
        st = smc.State(beta=np.zeros((N, Xs.shape[1])), ll=prob.loglik(np.zeros((N, Xs.shape[1]))),
                       gl=np.zeros((N, Xs.shape[1])), logW=np.full(N, -math.log(N)))
        step, sigma = cfg.step0(), np.full(Xs.shape[1], 2 / math.sqrt(Xs.shape[0]))
        for s in range(300):
            acc = smc.rwm_sweep(prob, st, lam[t_stop - 1], step, sigma, 500 + r, s, 0)
            if s < 150:
                step = smc.adapt_step(step, acc / N, "rwm")
            if s == 149:
                sigma = np.sqrt(np.maximum(st.beta.var(axis=0), 1e-24))
        mc_means.append(st.beta.mean(axis=0))
    mc_means = np.stack(mc_means)
    diff = smc_means.mean(0) - mc_means.mean(0)
    se = np.sqrt(smc_means.var(0, ddof=1) / 3 + mc_means.var(0, ddof=1) / 3)
    sd = np.sqrt(smc.weighted_moments(st.beta, st.logW)[1])
    assert np.all(np.abs(diff) <= 6 * se + 0.1 * sd + 2e-3), (diff, se, sd)


def test_single_site_increment_is_the_likelihood_difference():
    """The incremental eta update gives l(beta') - l(beta) of the full likelihood, and an
    accepted coordinate update changes only that coordinate."""
    Xs, y = _tiny_dataset(5, seed=3)
    prob = smc.Problem(Xs=Xs, y=y, a=1.0)
    rng = np.random.default_rng(0)
    N = 64
    beta = rng.normal(0, 0.3, size=(N, 5))
    st = smc.State(beta=beta.copy(), ll=prob.loglik(beta), gl=np.zeros_like(beta),
                   logW=np.full(N, -math.log(N)))
    acc = smc.single_site_sweep(prob, st, 0.5, 0.5, None, seed=7, cycle=0, t=3)
    # replay the cycle with full likelihood evaluations
    z, u = smc.philox.single_site_draws(7, N, 5, 0, 3)
    b = beta.copy()
    n_acc = 0
    for j in range(5):
        bp = b.copy()
        bp[:, j] += 0.5 * z[:, j]
        la = (prob.loglik(bp) - prob.loglik(b) + gt_prior.gt_logpdf(bp[:, j], 1.0, 0.5)
              - gt_prior.gt_logpdf(b[:, j], 1.0, 0.5))
        ok = np.log(u[:, j]) < la
        b[ok] = bp[ok]
        n_acc += int(ok.sum())
    assert n_acc == acc
    assert np.allclose(st.beta, b, rtol=0, atol=1e-14)
    assert np.allclose(st.ll, prob.loglik(b), rtol=1e-13)


def test_single_site_prior_only_targets_are_gt():
    # scales within reach of the fixed 0.5 proposal (a heavy-tailed Gt(1, 1) target needs
    # far longer random-walk runs than a test affords)
    a, N, p, T = 4.0, 4096, 2, 6
    lam = lambda_grid(0.3, 0.03, T)
    prob = smc.Problem(Xs=np.zeros((10, p)), y=np.zeros(10), a=a, likelihood_off=True)
    res = smc.run_smc(prob, lam, N, "single", sweeps=20, init_sweeps=200, ess_frac=0.5,
                      step0=0.5, seed=22, snapshot_at=range(1, T + 1))
    for t in range(1, T + 1):
        st = res.snapshots[t]
        D = weighted_ks(st.beta.ravel(), np.repeat(np.exp(st.logW), p),
                        lambda v: gt_prior.gt_cdf(v, a, lam[t - 1]))
        assert D < 0.03, (t, D)


def test_single_site_draws_are_the_stream():
    from oracle import philox
    z, u = philox.single_site_draws(5, 3, 4, 2, 7)
    w = philox.philox4x32_10(np.array([[1, 2, 2, (7 << 4) | 3]], dtype=np.uint64), philox.key_of(5))[0]
    assert u[1, 2] == (float(w[2]) + 0.5) * 2.0 ** -32
    r = math.sqrt(-2.0 * math.log((float(w[0]) + 1.0) * 2.0 ** -32))
    assert math.isclose(z[1, 2], r * math.cos(2.0 * math.pi * float(w[1]) * 2.0 ** -32), rel_tol=1e-15)
    zz, uu = philox.single_site_draws(9, 2000, 50, 0, 1)
    assert abs(zz.mean()) < 0.01 and abs(zz.var() - 1.0) < 0.01
    assert abs(uu.mean() - 0.5) < 0.005 and uu.min() > 0.0 and uu.max() < 1.0


# ----------------------------------------------------------- planted mistakes

def test_planted_mistakes_are_caught(monkeypatch):
    """Mutations of the oracle that the pins above must reject."""
    rng = np.random.default_rng(0)
    b = rng.normal(size=100)
    good = gt_prior.gt_logpdf(b, 1.0, 0.5)
    # 1. dropped normalising term: the density no longer integrates to one
    x, w = quadrature.line_nodes(1e4)
    assert abs(np.sum(w * np.exp(gt_prior.gt_logpdf(x, 1.0, 0.2) + math.log(2 * 0.2))) - 1) > 0.5
    # 2. wrong sign in the prior gradient: finite differences disagree
    h = 1e-6
    fd = (gt_prior.gt_logpdf(b + h, 1.0, 0.5) - gt_prior.gt_logpdf(b - h, 1.0, 0.5)) / (2 * h)
    assert not np.allclose(-gt_prior.gt_grad(b, 1.0, 0.5), fd, rtol=1e-3)
    # 3. resampler searching with C_k >= t instead of C_k > t differs from the definition
    q = np.array([0.0, 3.0, 0.0, 1.0])
    C = np.cumsum(q)
    tpos = (np.arange(4) + 0.0) / 4 * C[-1]
    assert not np.array_equal(np.searchsorted(C, tpos, side="left"),
                              smc.systematic_resample(q, 0))
    # 4. incremental weight with the scales swapped: prior-only Z ratio no longer 1
    lo, lt, N = 0.2, 0.1, 200000
    draws = gt_prior.gt_ppf(rng.uniform(size=(N, 2)), 1.0, lo)
    bad = smc.reweight_delta(draws, 1.0, lo, lt)          # swapped
    assert abs(math.exp(smc.normalise(np.full(N, -math.log(N)) + bad)[1]) - 1) > 0.05
    assert np.array_equal(good, gt_prior.gt_logpdf(b, 1.0, 0.5))
