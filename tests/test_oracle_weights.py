"""Pins of the oracle's incremental weights, normalisation, ESS and marginal-likelihood
ratio (Section 4: prior-ratio weights under the reversal backward kernel, normalised
weights, Z_t/Z_{t-1} estimate)."""
import math

import numpy as np
from scipy import stats

from oracle import gt_prior, smc


def test_equal_scales_give_zero_increment():
    b = np.random.default_rng(0).normal(size=(50, 7))
    assert np.array_equal(smc.reweight_delta(b, 1.0, 0.3, 0.3), np.zeros(50))


def test_increment_is_lomax_log_ratio():
    rng = np.random.default_rng(1)
    b = rng.normal(0, 0.5, size=(20, 5))
    for a in (0.5, 1.0, 4.0):
        lt, lo = 0.1, 0.15
        ref = (stats.lomax(c=a, scale=a * lt).logpdf(np.abs(b))
               - stats.lomax(c=a, scale=a * lo).logpdf(np.abs(b))).sum(axis=1)
        assert np.allclose(smc.reweight_delta(b, a, lt, lo), ref, rtol=1e-12, atol=1e-12)
    ref = (stats.laplace(scale=0.1).logpdf(b) - stats.laplace(scale=0.15).logpdf(b)).sum(axis=1)
    assert np.allclose(smc.reweight_delta(b, math.inf, 0.1, 0.15), ref, rtol=1e-12, atol=1e-12)


def test_normalise_and_ess():
    rng = np.random.default_rng(2)
    logw = rng.normal(0, 3, size=1000) - 700.0
    logW, L = smc.normalise(logw)
    assert abs(np.exp(logW).sum() - 1.0) < 1e-12
    assert abs(L - math.log(np.exp(logw + 700.0).sum()) + 700.0) < 1e-10
    assert abs(smc.ess(np.full(64, -math.log(64))) - 64) < 1e-10
    one_hot = np.full(64, -np.inf); one_hot[5] = 0.0
    assert smc.ess(one_hot) == 1.0
    W = np.exp(logW)
    assert abs(smc.ess(logW) - W.sum() ** 2 / (W * W).sum()) < 1e-9


def test_prior_only_z_ratio_is_one():
    """With the likelihood switched off Z_t = 1 for every t (the prior is normalised), so
    sum_i W_{t-1,i} w_{t,i} estimates 1: exact prior draws at lam_{t-1} reweighted to lam_t."""
    rng = np.random.default_rng(3)
    a, lo, lt, N = 1.0, 0.2, 0.17, 200000
    b = gt_prior.gt_ppf(rng.uniform(size=(N, 3)), a, lo)
    logW = np.full(N, -math.log(N))
    _, L = smc.normalise(logW + smc.reweight_delta(b, a, lt, lo))
    w = np.exp(smc.reweight_delta(b, a, lt, lo))
    se = w.std() / math.sqrt(N)
    assert abs(math.exp(L) - 1.0) < 5 * se


def test_weighted_moments():
    rng = np.random.default_rng(4)
    b = rng.normal(size=(300, 4))
    logW, _ = smc.normalise(rng.normal(size=300))
    m, v = smc.weighted_moments(b, logW)
    W = np.exp(logW)
    for j in range(4):
        mj = sum(W[i] * b[i, j] for i in range(300))
        vj = sum(W[i] * (b[i, j] - mj) ** 2 for i in range(300))
        assert abs(m[j] - mj) < 1e-12 and abs(v[j] - vj) < 1e-12


def test_adaptation_rule():
    assert smc.adapt_step(1.0, 0.234, "rwm") == 1.0
    assert abs(smc.adapt_step(1.0, 0.0, "rwm") - math.exp(-0.234)) < 1e-15
    assert abs(smc.adapt_step(1.0, 1.0, "mala") - math.exp(0.426)) < 1e-15
    assert abs(smc.adapt_step(1.0, 1.0, "rwm") - 2.0) < 1e-15        # clipped at log 2
