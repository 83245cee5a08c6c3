"""Pins of the oracle's EM MAP estimates (Section 2.1) and MAP path (Section 4.1)."""
import math

import numpy as np
import pytest
from scipy import optimize

from oracle import em, gt_prior, likelihood
from synth import CONFIGS, make_dataset


def _data(n=200, p=8, seed=1):
    cfg = CONFIGS["n500_p10_rwm_fp64"].replace(k_causal=3, beta_sd=0.8)
    d = make_dataset(cfg, n=n, p=p, seed=seed)
    Xs, _, _ = likelihood.standardise(d.X)
    return Xs, d.y.astype(np.float64)


def _grad(beta, Xs, y):
    return likelihood.grad_loglik(beta[None, :], Xs, y)[0]


def test_double_exponential_limit_is_the_weighted_lasso_optimum():
    """a = inf: every EM weight is 1/lam and one EM iteration is the convex L1-penalised
    logistic regression; compare with L-BFGS-B on the split form beta = u - v, u, v >= 0."""
    Xs, y = _data()
    p = Xs.shape[1]
    lam = 0.05
    b, lp = em.map_em(Xs, y, np.zeros(p), math.inf, lam, outer=1, inner=3000)

    def f(z):
        u, v = z[:p], z[p:]
        beta = u - v
        g = _grad(beta, Xs, y)
        val = -likelihood.loglik(beta[None, :], Xs, y)[0] + np.sum(u + v) / lam
        return val, np.concatenate([-g + 1.0 / lam, g + 1.0 / lam])

    r = optimize.minimize(f, np.zeros(2 * p), jac=True, method="L-BFGS-B",
                          bounds=[(0, None)] * (2 * p), options={"ftol": 1e-15, "gtol": 1e-12, "maxiter": 20000})
    ref = r.x[:p] - r.x[p:]
    obj = lambda beta: likelihood.loglik(beta[None, :], Xs, y)[0] - np.sum(np.abs(beta)) / lam
    assert obj(b[0]) >= obj(ref) - 1e-7
    assert np.allclose(b[0], ref, atol=1e-4)
    assert np.count_nonzero(b[0]) < p            # the L1 penalty zeroes some coefficients


@pytest.mark.parametrize("a,lam", [(1.0, 0.05), (4.0, 0.02), (0.5, 0.2)])
def test_em_fixed_point_is_a_stationary_point_of_the_posterior(a, lam):
    Xs, y = _data(seed=2)
    p = Xs.shape[1]
    b, _ = em.map_em(Xs, y, 0.1 * np.ones(p), a, lam, outer=300, inner=20)
    b = b[0]
    g = _grad(b, Xs, y)
    w = gt_prior.em_weight(b, a, lam)
    nz = b != 0.0
    assert np.all(np.abs(g[nz] - w[nz] * np.sign(b[nz])) <= 1e-6), (g, w, b)
    assert np.all(np.abs(g[~nz]) <= w[~nz] + 1e-9)
    # the prior's gradient at a nonzero coefficient is -w sign(b): the posterior gradient vanishes
    assert np.all(np.abs(g[nz] + gt_prior.gt_grad(b[nz], a, lam)) <= 1e-6)


def test_em_never_decreases_the_posterior():
    Xs, y = _data(seed=3)
    p = Xs.shape[1]
    rng = np.random.default_rng(0)
    b0 = rng.normal(0, 0.5, size=(5, p))
    prev = em.log_posterior(b0, Xs, y, 1.0, 0.03)
    b = b0
    for _ in range(15):
        b, lp = em.map_em(Xs, y, b, 1.0, 0.03, outer=1, inner=2)
        assert np.all(lp >= prev - 1e-10)
        prev = lp


def test_one_coefficient_matches_the_grid_argmax():
    Xs, y = _data(n=300, p=1, seed=4)
    for a, lam in ((1.0, 0.5), (4.0, 0.1), (1.0, 1e-4)):
        grid = np.linspace(-3, 3, 600001)
        lp = em.log_posterior(grid[:, None], Xs, y, a, lam)
        best = grid[np.argmax(lp)]
        b, _ = em.map_em(Xs, y, np.array([best]), a, lam, outer=200, inner=5)
        assert abs(b[0, 0] - best) <= 2e-5, (a, lam, b, best)
    # a tiny scale with a weak signal: the mode is exactly zero
    b, _ = em.map_em(Xs, y, np.array([0.3]), 1.0, 1e-6, outer=50, inner=5)
    assert b[0, 0] == 0.0


def test_map_step_keeps_the_better_mode():
    Xs, y = _data(seed=5)
    p = Xs.shape[1]
    rng = np.random.default_rng(1)
    beta = rng.normal(0, 0.3, size=(64, p))
    ll = likelihood.loglik(beta, Xs, y)
    i = em.best_particle(beta, ll, 1.0, 0.05)
    lp = ll + gt_prior.log_prior(beta, 1.0, 0.05)
    assert i == int(np.argmax(lp))
    m1, v1 = em.map_step(Xs, y, beta, ll, 1.0, 0.05, None, 20, 5)
    bad = np.full(p, 2.0)
    m2, v2 = em.map_step(Xs, y, beta, ll, 1.0, 0.05, bad, 20, 5)
    mb, vb = em.map_em(Xs, y, bad, 1.0, 0.05, 20, 5)
    assert v2 == max(v1, float(vb[0]))
