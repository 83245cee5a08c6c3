"""Sparsity-path summaries of weighted particle sets, oracle side (Section 5, and the
c-marginal mixture of Section 4, eq. all_particles).

Test infrastructure only (see the package docstring).

For every scale c = lam_t the SMC run leaves a weighted particle set {W_t,i, beta_t,i}.
The SPA plots summarise, per coefficient j:

* the inverse weighted empirical CDF F^-1(alpha | c): the absolute median
  z_j(c) = |F^-1(0.5 | c)| (Section 5, item (b)) and 90 % credible intervals
  [F^-1(0.05), F^-1(0.95)] (Section 5, individual coefficient plots);
* the concentration away from zero V_j(c) = 1 - Pr(|beta_j| < Delta | c)
  (Section 5, item (d); Delta in {0.05, 0.1});
* the posterior over the scale p(c | X, y, a) (Section 5, item (c)): with a uniform prior
  on log c and the geometric grid (uniform in log c), the mass at lam_t is proportional
  to Z_t / Z_1, whose estimate the SMC run accumulates (Section 4);
* the c-marginal posterior (Section 5, marginal plots): the mixture over t of the
  weighted sets with mixture weights Z_t/Z_1 normalised over t (eq. all_particles), and
  its quantiles and concentrations.

Readings (also listed in the design notes):
* Weighted quantile: F^-1(alpha) = min{x : F(x) >= alpha}, the generalised inverse of
  the weighted empirical CDF, for alpha in (0, 1].
* So that the choice of the order statistic is exact (no dependence on summation order),
  the weights are first quantised to integers q_i = floor((w_i / max w) 2^K) with
  K = 63 - ceil(log2 M): every partial sum of q is an integer below 2^63.  The
  alpha-quantile is then the smallest sorted value whose cumulative q reaches
  ceil(alpha * sum q), evaluated exactly (alpha is the given double, an exact rational).
  The quantised CDF differs from the exact one by at most M 2^-K.
* V uses the same quantised weights: V = 1 - S / C with S = sum of q_i over
  |beta_ij| < Delta (open interval, as in the paper) and C = sum q_i, the final division
  in FP64.
"""
from __future__ import annotations

import math
from fractions import Fraction

import numpy as np


def quantise_weights(w):
    """Integer weights q_i = floor((w_i / max w) 2^K), K = 63 - ceil(log2 M), as uint64
    (exact; every partial sum stays below 2^63).  w: non-negative finite, not all zero."""
    w = np.asarray(w, dtype=np.float64)
    M = w.shape[0]
    if M < 1:
        raise ValueError("empty weight vector")
    if not np.all(np.isfinite(w)) or np.any(w < 0.0):
        raise ValueError("weights must be finite and non-negative")
    wmax = float(np.max(w))
    if not wmax > 0.0:
        raise ValueError("all weights are zero")
    K = 63 - (M - 1).bit_length()
    ratio = w / wmax                                  # one correctly rounded division each
    # ratio * 2^K is exact (a power-of-two scaling) and so is the floor of a double
    return np.floor(np.ldexp(ratio, K)).astype(np.uint64), K


def _threshold(alpha: float, C: int) -> int:
    """ceil(alpha * C) in exact arithmetic (alpha the given double)."""
    a = Fraction(float(alpha))
    if not (0 < a <= 1):
        raise ValueError("quantile level must lie in (0, 1]")
    v = a * C
    return -((-v.numerator) // v.denominator)


def _columns(values):
    values = np.asarray(values, dtype=np.float64)
    return values[:, None] if values.ndim == 1 else values


def weighted_quantiles(values, w, levels):
    """F^-1(alpha) per column of values (M x p) under weights w (M), for each alpha in
    levels: returns an array (len(levels), p).  Per column: sort, cumulative quantised
    weight, first position reaching ceil(alpha C)."""
    values = _columns(values)
    M, p = values.shape
    q, _ = quantise_weights(w)
    C = int(q.sum(dtype=np.uint64))
    thr = [_threshold(alpha, C) for alpha in levels]
    out = np.empty((len(levels), p))
    for j in range(p):
        order = np.argsort(values[:, j], kind="stable")
        cum = np.cumsum(q[order], dtype=np.uint64)
        for li, t in enumerate(thr):
            k = int(np.searchsorted(cum, np.uint64(t), side="left"))
            out[li, j] = values[order[k], j]
    return out


def concentration(values, w, deltas):
    """V_j = 1 - Pr(|beta_j| < Delta) under the quantised weights: (len(deltas), p)."""
    values = _columns(values)
    q, _ = quantise_weights(w)
    C = int(q.sum(dtype=np.uint64))
    out = np.empty((len(deltas), values.shape[1]))
    for di, d in enumerate(deltas):
        inside = np.abs(values) < d
        S = (q[:, None] * inside).sum(axis=0, dtype=np.uint64)
        out[di] = 1.0 - S.astype(np.float64) / float(C)
    return out


def concentration_plain(values, w, deltas):
    """The plain definition with the real weights: 1 - sum_i W_i 1[|beta_ij| < Delta]."""
    values = _columns(values)
    W = np.asarray(w, dtype=np.float64)
    W = W / W.sum()
    return np.array([1.0 - (W[:, None] * (np.abs(values) < d)).sum(axis=0) for d in deltas])


def abs_median(values, w):
    """z_j = |F^-1(0.5)| (Section 5, item (b))."""
    return np.abs(weighted_quantiles(values, w, [0.5])[0])


def credible_interval(values, w, mass: float = 0.9):
    """Equal-tailed interval [F^-1((1-mass)/2), F^-1((1+mass)/2)]: (2, p)."""
    lo = 0.5 * (1.0 - mass)
    return weighted_quantiles(values, w, [lo, 1.0 - lo])


def scale_posterior(log_z):
    """p(c = lam_t | X, y, a) on a grid uniform in log c: Z_t/Z_1 normalised over t."""
    lz = np.asarray(log_z, dtype=np.float64)
    m = np.max(lz)
    e = np.exp(lz - m)
    return e / e.sum()


def scale_mode(lambdas, log_z):
    """The grid scale maximising p(c | X, y, a)."""
    return float(np.asarray(lambdas)[int(np.argmax(log_z))])


def mixture_weights(log_z, logW):
    """Weights of the c-marginal mixture (eq. all_particles): p_t W_t,i, as a flat (T N)
    array in (t, i) order.  logW: (T, N) normalised log weights per scale."""
    pt = scale_posterior(log_z)
    W = np.exp(np.asarray(logW, dtype=np.float64))
    return (pt[:, None] * W).reshape(-1)


def marginal_summaries(beta_path, logW_path, log_z, levels, deltas):
    """Quantiles and concentrations of the c-marginal mixture: beta_path (T, N, p),
    logW_path (T, N), log_z (T,)."""
    beta_path = np.asarray(beta_path, dtype=np.float64)
    T, N, p = beta_path.shape
    w = mixture_weights(log_z, logW_path)
    flat = beta_path.reshape(T * N, p)
    return weighted_quantiles(flat, w, levels), concentration(flat, w, deltas)
