"""Brute-force quadrature of small posteriors (p = 1, 2), oracle side.

Test infrastructure only (see the package docstring).

For one or two coefficients the SMC targets can be integrated directly:
Z(lam) = integral of f(y | X, beta) Gt(beta | a, lam) d beta, and the posterior mean is
integral of beta f Gt / Z.  The Gt density has a cusp at beta_j = 0 and, for small lam,
a scale a*lam far below the likelihood's; the nodes are therefore composite
Gauss-Legendre panels on each half-line, with geometrically graded breakpoints from
1e-9 up to ``bound`` so that every scale between them is resolved.
"""
from __future__ import annotations

import math

import numpy as np

from . import gt_prior, likelihood


def half_line_nodes(bound: float, lo: float = 1e-9, panels_per_decade: int = 3,
                    order: int = 24):
    """Nodes/weights on (0, bound): panels [0, lo], then geometric panels up to bound."""
    x, w = np.polynomial.legendre.leggauss(order)
    decades = max(1, math.ceil(math.log10(bound / lo)))
    edges = np.concatenate([[0.0], np.geomspace(lo, bound, decades * panels_per_decade + 1)])
    nodes, weights = [], []
    for a, b in zip(edges[:-1], edges[1:]):
        nodes.append(0.5 * (b - a) * x + 0.5 * (b + a))
        weights.append(0.5 * (b - a) * w)
    return np.concatenate(nodes), np.concatenate(weights)


def line_nodes(bound: float, **kw):
    """Symmetric nodes on (-bound, bound), split at the cusp beta = 0."""
    x, w = half_line_nodes(bound, **kw)
    return np.concatenate([-x[::-1], x]), np.concatenate([w[::-1], w])


def _log_target(beta, Xs, y, a, lam):
    return likelihood.loglik(beta, Xs, y) + gt_prior.log_prior(beta, a, lam)


def posterior_summary(Xs, y, a: float, lam: float, bound: float = 30.0, **kw):
    """(log Z, posterior mean (p,), posterior variance (p,)) for p = 1 or 2."""
    Xs = np.asarray(Xs, dtype=np.float64)
    p = Xs.shape[1]
    x, w = line_nodes(bound, **kw)
    if p == 1:
        B = x[:, None]
        W = w
    elif p == 2:
        g0, g1 = np.meshgrid(x, x, indexing="ij")
        B = np.stack([g0.ravel(), g1.ravel()], axis=1)
        W = np.outer(w, w).ravel()
    else:
        raise ValueError("quadrature is for p = 1 or 2")
    lt = _log_target(B, Xs, y, a, lam)
    m = np.max(lt)
    f = W * np.exp(lt - m)
    Z = np.sum(f)
    mean = f @ B / Z
    var = f @ (B - mean) ** 2 / Z
    return m + math.log(Z), mean, var


def normal_obs_posterior_mean(yobs, a: float, lam: float, bound: float = 60.0,
                              prior: str = "gt", tau: float = 1.0, **kw):
    """Posterior mean of beta given one observation yobs ~ N(beta, 1) under a Gt(a, lam)
    prior (the shrinkage curve of the normal-observation figure), or under a N(0, tau^2)
    prior with prior="normal" (a closed-form check of the same routine)."""
    x, w = line_nodes(bound, **kw)
    yobs = np.atleast_1d(np.asarray(yobs, dtype=np.float64))
    out = np.empty_like(yobs)
    for i, yo in enumerate(yobs):
        if prior == "gt":
            lp = gt_prior.gt_logpdf(x, a, lam)
        else:
            lp = -0.5 * (x / tau) ** 2
        lt = -0.5 * (yo - x) ** 2 + lp
        f = w * np.exp(lt - np.max(lt))
        out[i] = np.sum(f * x) / np.sum(f)
    return out
