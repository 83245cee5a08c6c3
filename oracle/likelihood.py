"""Logistic likelihood without intercept on standardised genotypes, oracle side.

Test infrastructure only (see the package docstring).

Section 2: f(y | X, beta) = prod_k p_k^y_k (1 - p_k)^(1 - y_k), p_k = logit^-1(x_k beta),
so log f = sum_k [y_k eta_k - log(1 + exp(eta_k))] with eta = X beta.  Section 3 fixes
X to column-standardised genotypes (mean 0, unit standard deviation); the population
standard deviation (ddof = 0) of the sample is used.
"""
from __future__ import annotations

import numpy as np
from scipy.special import expit

_CHUNK = 1024   # particles per block: bounds the (chunk x n) eta buffer, not the arithmetic


def standardise(X):
    """Column-standardised design: (X - mean) / population sd, FP64; also returns (mu, s)."""
    X = np.asarray(X, dtype=np.float64)
    mu = X.mean(axis=0)
    s = np.sqrt(((X - mu) ** 2).mean(axis=0))
    if np.any(s == 0.0):
        raise ValueError("zero-variance marker column")
    return (X - mu) / s, mu, s


def softplus(eta):
    """log(1 + exp(eta)), evaluated without overflow."""
    return np.logaddexp(0.0, eta)


def loglik(beta, Xs, y):
    """Per-particle log-likelihood sum_k [y_k eta_k - softplus(eta_k)], eta = Xs beta_i.

    beta: (M, p); Xs: (n, p) standardised; y: (n,) 0/1.  Returns (M,) FP64."""
    beta = np.atleast_2d(np.asarray(beta, dtype=np.float64))
    y = np.asarray(y, dtype=np.float64)
    out = np.empty(beta.shape[0])
    for lo in range(0, beta.shape[0], _CHUNK):
        eta = beta[lo:lo + _CHUNK] @ Xs.T
        out[lo:lo + _CHUNK] = np.sum(y * eta - softplus(eta), axis=1)
    return out


def grad_loglik(beta, Xs, y):
    """Per-particle gradient Xs^T (y - logistic(eta)); returns (M, p) FP64."""
    beta = np.atleast_2d(np.asarray(beta, dtype=np.float64))
    y = np.asarray(y, dtype=np.float64)
    out = np.empty_like(beta)
    for lo in range(0, beta.shape[0], _CHUNK):
        eta = beta[lo:lo + _CHUNK] @ Xs.T
        out[lo:lo + _CHUNK] = (y - expit(eta)) @ Xs
    return out


def loglik_and_grad(beta, Xs, y):
    beta = np.atleast_2d(np.asarray(beta, dtype=np.float64))
    y = np.asarray(y, dtype=np.float64)
    ll = np.empty(beta.shape[0])
    g = np.empty_like(beta)
    for lo in range(0, beta.shape[0], _CHUNK):
        eta = beta[lo:lo + _CHUNK] @ Xs.T
        ll[lo:lo + _CHUNK] = np.sum(y * eta - softplus(eta), axis=1)
        g[lo:lo + _CHUNK] = (y - expit(eta)) @ Xs
    return ll, g
