"""MAP estimates under the Gt(a, c) prior by the EM algorithm of Section 2.1, and the MAP
path of Section 4.1 (further details), oracle side.

Test infrastructure only (see the package docstring).

With the scale-mixture representation (Laplace given tau_j, tau_j inverse gamma), the E
step gives the expected precision E[1/tau_j | beta_j] = (a+1)/(a c + |beta_j|) (its a = inf
limit 1/c), so one EM iteration solves the convex problem

    beta^(t+1) = argmax  l(beta) - sum_j w_j |beta_j|,   w_j = (a+1)/(a c + |beta_j^(t)|).

The paper leaves the inner solver to "standard techniques"; the reading taken here (also in
the design notes) is cyclic coordinate ascent with a quadratic minoriser: along
coordinate j the logistic log-likelihood of standardised genotypes has curvature at most
sum_k X_std,kj^2 / 4 = n / 4, so the update

    beta_j <- S(beta_j + 4 g_j / n, 4 w_j / n),   g_j = sum_k (y_k - sigma(eta_k)) X_std,kj,

with S the soft-threshold, never decreases the inner objective.  Each EM iteration runs a
fixed number of such sweeps (j = 1..p in order); iteration counts are fixed, so the
result is a deterministic function of the start point.

MAP path (Section 4.1): at each scale, EM is started from the particle with the highest
posterior density and from the previous scale's MAP; the result with the higher posterior
density is kept.
"""
from __future__ import annotations

import math

import numpy as np
from scipy.special import expit

from . import gt_prior, likelihood


def em_weights(beta, a: float, lam: float):
    """E[1/tau_j | beta_j] = (a+1)/(a lam + |beta_j|); 1/lam for the double exponential."""
    beta = np.asarray(beta, dtype=np.float64)
    if math.isinf(a):
        return np.full_like(beta, 1.0 / lam)
    return gt_prior.em_weight(beta, a, lam)


def soft_threshold(z, thr):
    return np.sign(z) * np.maximum(np.abs(z) - thr, 0.0)


def log_posterior(beta, Xs, y, a: float, lam: float):
    """log f(y | X, beta) + sum_j log Gt(beta_j | a, lam), per row of beta."""
    beta = np.atleast_2d(beta)
    return likelihood.loglik(beta, Xs, y) + gt_prior.log_prior(beta, a, lam)


def cd_sweep(Xs, y, beta, w):
    """One cyclic coordinate-ascent sweep of the weighted-L1 logistic problem for every row
    of beta (in place), with the curvature bound n/4; returns beta."""
    n = Xs.shape[0]
    eta = beta @ Xs.T                                   # (M, n)
    for j in range(Xs.shape[1]):
        x = Xs[:, j]
        r = y[None, :] - expit(eta)
        g = r @ x
        new = soft_threshold(beta[:, j] + 4.0 * g / n, 4.0 * w[:, j] / n)
        delta = new - beta[:, j]
        beta[:, j] = new
        eta += delta[:, None] * x[None, :]
    return beta


def map_em(Xs, y, beta0, a: float, lam: float, outer: int, inner: int):
    """EM from each row of beta0 (M x p): `outer` E steps, each followed by `inner`
    coordinate sweeps.  Returns (modes M x p, log posterior at the modes)."""
    beta = np.array(beta0, dtype=np.float64, copy=True)
    if beta.ndim == 1:
        beta = beta[None, :]
    y = np.asarray(y, dtype=np.float64)
    for _ in range(outer):
        w = em_weights(beta, a, lam)
        for _ in range(inner):
            cd_sweep(Xs, y, beta, w)
    return beta, log_posterior(beta, Xs, y, a, lam)


def best_particle(beta, ll, a: float, lam: float) -> int:
    """Index of the particle with the highest posterior density at scale lam (the first
    one on ties)."""
    lp = np.asarray(ll) + gt_prior.log_prior(beta, a, lam)
    return int(np.argmax(lp))


def map_step(Xs, y, beta, ll, a: float, lam: float, prev_map, outer: int, inner: int):
    """One scale of the MAP path: EM from the best particle and from the previous MAP
    (if any); the mode with the higher posterior density (the first on ties)."""
    starts = [beta[best_particle(beta, ll, a, lam)]]
    if prev_map is not None:
        starts.append(prev_map)
    modes, lp = map_em(Xs, y, np.stack(starts), a, lam, outer, inner)
    k = int(np.argmax(lp))
    return modes[k], float(lp[k])
