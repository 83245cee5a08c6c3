"""Pins of the oracle's brute-force quadrature (used to pin the SMC at p = 1, 2)."""
import math

import numpy as np
import pytest
from scipy import integrate

from oracle import gt_prior, likelihood, quadrature


def test_normal_prior_closed_form():
    """Under a N(0, tau^2) prior and y ~ N(beta, 1) the posterior mean is y tau^2/(1 + tau^2)."""
    y = np.linspace(-6, 6, 13)
    for tau in (0.3, 1.0, 4.0):
        got = quadrature.normal_obs_posterior_mean(y, 0, 0, prior="normal", tau=tau)
        assert np.allclose(got, y * tau ** 2 / (1 + tau ** 2), rtol=1e-10, atol=1e-12)


@pytest.mark.parametrize("a", [1.0, 4.0])
def test_normal_observation_shrinkage_curve(a):
    """Shape of the posterior mean under one normal observation and a Gt(a, 0.1) prior:
    odd, monotone, shrinks towards zero, strongly near y = 0 (sparsity) and
    less and less as |y| grows (approximate unbiasedness)."""
    y = np.linspace(0.0, 12.0, 49)
    m = quadrature.normal_obs_posterior_mean(y, a, 0.1)
    assert abs(m[0]) < 1e-12
    assert np.allclose(quadrature.normal_obs_posterior_mean(-y, a, 0.1), -m, atol=1e-12)
    assert np.all(np.diff(m) > 0)
    assert np.all(m[1:] < y[1:])
    assert m[4] / y[4] < 0.2                         # y = 1: shrunk by more than 80 %
    assert (y[-1] - m[-1]) / y[-1] < 0.05            # y = 12: within 5 %
    # far from zero the shrinkage approaches the prior score (a+1)/(a c + |y|)
    assert abs((y[-1] - m[-1]) - (a + 1) / (a * 0.1 + y[-1])) < 0.05


def test_nodes_integrate_known_functions():
    x, w = quadrature.line_nodes(30.0)
    for lam in (1e-2, 1.0, 10.0):
        for a in (0.5, 1.0):
            f = np.exp(gt_prior.gt_logpdf(x, a, lam))
            # mass of Gt on (-30, 30) is 1 - 2 * tail
            mass = 1.0 - 2.0 * (1.0 - gt_prior.gt_cdf(30.0, a, lam))
            assert abs(np.sum(w * f) - mass) < 1e-10


def test_one_dim_log_evidence_vs_adaptive_quad():
    rng = np.random.default_rng(0)
    X = rng.integers(0, 3, size=(40, 1)).astype(np.uint8)
    y = (rng.uniform(size=40) < 0.5).astype(np.uint8)
    Xs, _, _ = likelihood.standardise(X)
    for a, lam in [(1.0, 1e3), (0.5, 0.3), (1.0, 1e-2)]:
        logZ, mean, var = quadrature.posterior_summary(Xs, y, a, lam)

        def f(b, k=0):
            return (b ** k) * math.exp(likelihood.loglik(np.array([[b]]), Xs, y)[0]
                                       + gt_prior.gt_logpdf(b, a, lam) + 40 * math.log(2))
        pts = sorted({-a * lam, a * lam, -1.0, 1.0})
        Z = sum(integrate.quad(f, lo, hi, limit=500, epsabs=0, epsrel=1e-11)[0]
                for lo, hi in [(-30, -max(pts)), (-max(pts), 0), (0, max(pts)), (max(pts), 30)])
        M1 = sum(integrate.quad(lambda b: f(b, 1), lo, hi, limit=500, epsabs=0, epsrel=1e-11)[0]
                 for lo, hi in [(-30, -max(pts)), (-max(pts), 0), (0, max(pts)), (max(pts), 30)])
        assert abs(logZ - (math.log(Z) - 40 * math.log(2))) < 1e-8
        assert abs(mean[0] - M1 / Z) < 1e-8


def test_two_dim_resolution_converged():
    rng = np.random.default_rng(1)
    X = rng.integers(0, 3, size=(50, 2)).astype(np.uint8)
    y = (rng.uniform(size=50) < 0.5).astype(np.uint8)
    Xs, _, _ = likelihood.standardise(X)
    for lam in (1e2, 0.05):
        z1, m1, v1 = quadrature.posterior_summary(Xs, y, 1.0, lam, bound=8.0, lo=1e-7,
                                                  panels_per_decade=2, order=16)
        z2, m2, v2 = quadrature.posterior_summary(Xs, y, 1.0, lam, bound=8.0, lo=1e-8,
                                                  panels_per_decade=3, order=24)
        assert abs(z1 - z2) < 1e-8 and np.allclose(m1, m2, atol=1e-8)
