"""Generalized-t prior, oracle side (Section 2).

Test infrastructure only (see the package docstring).

The general generalized-t density with location mu, degrees of freedom a, scale c
and norm q is

    p(beta) = q / (2 c a^(1/q) B(1/q, a)) * (1 + |beta - mu|^q / (a c^q))^-(a + 1/q),

and the sampler uses its centred L1 member (q = 1, mu = 0), written Gt(a, c):

    p(beta) = 1/(2c) * (1 + |beta|/(a c))^-(a+1).

The double-exponential DE(0, c) with density exp(-|beta|/c)/(2c) is its a -> inf limit.
The scale ``lam`` of every function below is the paper's c (the scale indexed by the
SMC sweep; b = a c in the scale-mixture form).
"""
from __future__ import annotations

import math

import numpy as np
from scipy.special import betaln


def gt_general_pdf(beta, mu: float, a: float, c: float, q: float):
    """The general generalized-t density (Section 2, general form)."""
    beta = np.asarray(beta, dtype=np.float64)
    log_norm = math.log(q) - math.log(2.0 * c) - math.log(a) / q - betaln(1.0 / q, a)
    z = np.abs(beta - mu) ** q / (a * c ** q)
    return np.exp(log_norm - (a + 1.0 / q) * np.log1p(z))


def gt_logpdf(beta, a: float, lam: float):
    """log Gt(beta | a, lam), elementwise; a = inf gives the double exponential."""
    beta = np.asarray(beta, dtype=np.float64)
    x = np.abs(beta)
    if math.isinf(a):
        return -math.log(2.0 * lam) - x / lam
    return -math.log(2.0 * lam) - (a + 1.0) * np.log1p(x / (a * lam))


def de_logpdf(beta, lam: float):
    """log DE(beta | 0, lam) = -log(2 lam) - |beta|/lam."""
    beta = np.asarray(beta, dtype=np.float64)
    return -math.log(2.0 * lam) - np.abs(beta) / lam


def gt_cdf(beta, a: float, lam: float):
    """CDF of Gt(a, lam): 1/2 (1 + |beta|/(a lam))^-a below zero, its complement above."""
    beta = np.asarray(beta, dtype=np.float64)
    x = np.abs(beta)
    if math.isinf(a):
        tail = 0.5 * np.exp(-x / lam)
    else:
        tail = 0.5 * (1.0 + x / (a * lam)) ** (-a)
    return np.where(beta < 0.0, tail, 1.0 - tail)


def gt_ppf(u, a: float, lam: float):
    """Inverse CDF of Gt(a, lam) (used to draw exact prior samples in tests)."""
    u = np.asarray(u, dtype=np.float64)
    tail = np.minimum(u, 1.0 - u)
    if math.isinf(a):
        mag = -lam * np.log(2.0 * tail)
    else:
        mag = a * lam * ((2.0 * tail) ** (-1.0 / a) - 1.0)
    return np.where(u < 0.5, -mag, mag)


def gt_grad(beta, a: float, lam: float):
    """d/dbeta log Gt(beta | a, lam) = -(a+1) sign(beta) / (a lam + |beta|), sign(0) = 0.

    Its magnitude is the EM weight (a+1)/(a c + |beta|) of Section 2.1; as a -> inf it
    tends to sign(beta)/c, the Lasso penalty."""
    beta = np.asarray(beta, dtype=np.float64)
    if math.isinf(a):
        return -np.sign(beta) / lam
    return -(a + 1.0) * np.sign(beta) / (a * lam + np.abs(beta))


def em_weight(beta, a: float, c: float):
    """EM weight w_j = (a+1) / (a c + |beta_j|) (Section 2.1, adaptive-weight equation)."""
    beta = np.asarray(beta, dtype=np.float64)
    return (a + 1.0) / (a * c + np.abs(beta))


def log_prior(beta, a: float, lam: float):
    """Sum over markers of log Gt(beta_j | a, lam); beta is (..., p)."""
    return np.sum(gt_logpdf(beta, a, lam), axis=-1)
