"""Pins of the oracle's logistic likelihood and gradient (Section 2: Bernoulli likelihood
with p_i = logit^-1(x_i beta), no intercept; Section 3: column-standardised genotypes)."""
import math

import numpy as np
import pytest

from oracle import likelihood
from synth import CONFIGS, make_dataset


@pytest.fixture(scope="module")
def small():
    rng = np.random.default_rng(7)
    X = rng.integers(0, 3, size=(12, 3)).astype(np.uint8)
    y = rng.integers(0, 2, size=12).astype(np.uint8)
    Xs, mu, s = likelihood.standardise(X)
    return X, y, Xs


def test_standardise_moments():
    d = make_dataset(CONFIGS["n500_p10_rwm_fp64"])
    Xs, mu, s = likelihood.standardise(d.X)
    assert np.allclose(Xs.mean(axis=0), 0.0, atol=1e-14)
    assert np.allclose((Xs ** 2).mean(axis=0), 1.0, rtol=1e-13)     # population sd
    assert np.allclose(mu, d.X.mean(axis=0))


def test_zero_variance_column_rejected():
    X = np.array([[0, 1], [0, 2], [0, 0]], dtype=np.uint8)
    with pytest.raises(ValueError):
        likelihood.standardise(X)


def test_beta_zero_is_minus_n_log2():
    d = make_dataset(CONFIGS["n500_p10_rwm_fp64"])
    Xs, _, _ = likelihood.standardise(d.X)
    ll = likelihood.loglik(np.zeros((3, Xs.shape[1])), Xs, d.y)
    assert np.allclose(ll, -d.X.shape[0] * math.log(2.0), rtol=1e-15)


def test_bernoulli_product_brute_force(small):
    """The softplus form equals the log of prod p_k^y_k (1 - p_k)^(1 - y_k), computed
    element by element with scalar math."""
    X, y, Xs = small
    rng = np.random.default_rng(3)
    for _ in range(5):
        b = rng.normal(0, 0.8, size=3)
        prod = 1.0
        for k in range(X.shape[0]):
            e = sum(Xs[k, j] * b[j] for j in range(3))
            pk = 1.0 / (1.0 + math.exp(-e))
            prod *= pk if y[k] == 1 else (1.0 - pk)
        assert abs(likelihood.loglik(b[None], Xs, y)[0] - math.log(prod)) < 1e-12


def test_label_flip_symmetry():
    d = make_dataset(CONFIGS["n500_p10_rwm_fp64"])
    Xs, _, _ = likelihood.standardise(d.X)
    b = np.random.default_rng(4).normal(0, 0.3, size=(5, Xs.shape[1]))
    assert np.allclose(likelihood.loglik(-b, Xs, 1 - d.y), likelihood.loglik(b, Xs, d.y),
                       rtol=1e-13)


def test_gradient_at_zero_closed_form():
    d = make_dataset(CONFIGS["n500_p10_rwm_fp64"])
    Xs, _, _ = likelihood.standardise(d.X)
    g = likelihood.grad_loglik(np.zeros((1, Xs.shape[1])), Xs, d.y)[0]
    ref = np.array([sum(Xs[k, j] * (d.y[k] - 0.5) for k in range(Xs.shape[0]))
                    for j in range(Xs.shape[1])])
    assert np.allclose(g, ref, rtol=1e-12, atol=1e-12)


def test_gradient_finite_differences():
    d = make_dataset(CONFIGS["n500_p10_rwm_fp64"])
    Xs, _, _ = likelihood.standardise(d.X)
    rng = np.random.default_rng(5)
    b = rng.normal(0, 0.2, size=(4, Xs.shape[1]))
    g = likelihood.grad_loglik(b, Xs, d.y)
    h = 1e-6
    for j in range(Xs.shape[1]):
        e = np.zeros(Xs.shape[1]); e[j] = h
        fd = (likelihood.loglik(b + e, Xs, d.y) - likelihood.loglik(b - e, Xs, d.y)) / (2 * h)
        assert np.allclose(g[:, j], fd, rtol=1e-6, atol=1e-5)
    ll2, g2 = likelihood.loglik_and_grad(b, Xs, d.y)
    assert np.array_equal(g2, g) and np.array_equal(ll2, likelihood.loglik(b, Xs, d.y))
