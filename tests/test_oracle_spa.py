"""Pins of the oracle's sparsity-path summaries (Section 5; eq. all_particles of Section 4)
against closed forms, library routines and brute force."""
import math
from fractions import Fraction

import numpy as np
import pytest

from oracle import gt_prior, spa


def _inverted_cdf(x, alpha):
    """NumPy's inverse-empirical-CDF quantile (Hyndman & Fan type 1)."""
    return np.quantile(x, alpha, axis=0, method="inverted_cdf")


@pytest.mark.parametrize("M", [1, 7, 997, 4099])
def test_equal_weights_match_the_inverse_empirical_cdf(M):
    rng = np.random.default_rng(M)
    v = rng.standard_t(2, size=(M, 3))
    levels = [0.05, 0.3, 0.5, 0.95]
    # keep alpha * M away from integers, where the two conventions for rounding the
    # level differ (exact rational alpha here, a float product in NumPy)
    levels = [a for a in levels if M == 1 or abs(a * M - round(a * M)) > 1e-6]
    got = spa.weighted_quantiles(v, np.full(M, 0.37), levels)
    for li, a in enumerate(levels):
        assert np.array_equal(got[li], _inverted_cdf(v, a).reshape(-1)), a


def test_integer_weights_match_the_repeated_sample():
    """Weight m_i / 8 counts a value m_i times (the quantisation is exact here)."""
    rng = np.random.default_rng(5)
    v = rng.normal(size=(301, 4))
    m = rng.integers(0, 9, size=301)
    m[0] = 8
    levels = [0.05, 0.25, 0.5, 0.9, 0.95, 1.0]
    got = spa.weighted_quantiles(v, m / 8.0, levels)
    tot = int(m.sum())
    for li, a in enumerate(levels):
        if a < 1.0 and abs(a * tot - round(a * tot)) < 1e-6:
            continue
        for j in range(v.shape[1]):
            assert got[li, j] == _inverted_cdf(np.repeat(v[:, j], m), a)


def test_stratified_prior_draws_give_the_closed_form_quantiles():
    """x_i = F^-1((i + 1/2)/N) of the Gt prior with equal weights: the alpha-quantile is
    x_(ceil(alpha N)) exactly, and V(Delta) is within 1/N of the closed-form mass."""
    N, a, lam = 4000, 1.0, 0.2
    x = gt_prior.gt_ppf((np.arange(N) + 0.5) / N, a, lam)
    perm = np.random.default_rng(0).permutation(N)
    v = x[perm]
    for alpha in (0.05, 0.123, 0.5, 0.95):
        k = math.ceil(Fraction(alpha) * N)
        want = gt_prior.gt_ppf((k - 0.5) / N, a, lam)
        assert spa.weighted_quantiles(v, np.ones(N), [alpha])[0, 0] == want
    for d in (0.05, 0.1):
        mass = gt_prior.gt_cdf(d, a, lam) - gt_prior.gt_cdf(-d, a, lam)
        V = spa.concentration(v, np.ones(N), [d])[0, 0]
        assert abs(V - (1.0 - mass)) <= 1.0 / N


def _brute_force_quantile(v, w, alpha):
    """min{x in v : sum_{v_i <= x} q_i / C >= alpha}, every candidate checked in exact
    rational arithmetic (no sorting, no cumulative sums)."""
    q, _ = spa.quantise_weights(w)
    q = [int(t) for t in q]
    C = sum(q)
    best = None
    for x in v:
        F = Fraction(sum(qi for vi, qi in zip(v, q) if vi <= x), C)
        if F >= Fraction(alpha) and (best is None or x < best):
            best = x
    return best


def test_brute_force_definition_with_real_weights_and_ties():
    rng = np.random.default_rng(11)
    for trial in range(25):
        M = int(rng.integers(1, 40))
        v = np.round(rng.normal(size=M), 1)          # many ties
        w = rng.exponential(size=M) ** 3
        w[rng.uniform(size=M) < 0.2] = 0.0
        if not w.any():
            w[0] = 1.0
        for alpha in (0.05, 0.5, 0.95, 1.0, float(rng.uniform(0.01, 1.0))):
            got = spa.weighted_quantiles(v, w, [alpha])[0, 0]
            assert got == _brute_force_quantile(list(v), w, alpha), (trial, alpha)


def test_zero_weight_values_are_never_returned_and_alpha_one_is_the_weighted_max():
    v = np.array([-9.0, 1.0, 2.0, 3.0, 99.0])
    w = np.array([0.0, 1.0, 1.0, 1.0, 0.0])
    q = spa.weighted_quantiles(v, w, [1e-300, 0.5, 1.0])[:, 0]
    assert list(q) == [1.0, 2.0, 3.0]


def test_invariances():
    rng = np.random.default_rng(2)
    v = rng.normal(size=(500, 2))
    w = rng.exponential(size=500)
    base = spa.weighted_quantiles(v, w, [0.05, 0.5, 0.95])
    perm = rng.permutation(500)
    assert np.array_equal(spa.weighted_quantiles(v[perm], w[perm], [0.05, 0.5, 0.95]), base)
    assert np.array_equal(spa.weighted_quantiles(v, w * 2.0 ** -40, [0.05, 0.5, 0.95]), base)
    # monotone in alpha; the median of a sign-flipped sample is the negated median's partner
    qs = spa.weighted_quantiles(v, w, np.linspace(0.01, 1.0, 40))
    assert np.all(np.diff(qs, axis=0) >= 0.0)


def test_quantisation_error_bound():
    rng = np.random.default_rng(4)
    for M in (3, 100, 5000):
        w = rng.exponential(size=M) ** 4
        q, K = spa.quantise_weights(w)
        Cq = float(q.sum(dtype=np.uint64))
        Fq = np.cumsum(q.astype(np.float64)) / Cq
        Fw = np.cumsum(w) / w.sum()
        assert np.max(np.abs(Fq - Fw)) <= M * 2.0 ** -K + 1e-15
        assert K == 63 - (M - 1).bit_length()


def test_concentration_matches_the_plain_definition():
    rng = np.random.default_rng(8)
    v = rng.laplace(scale=0.1, size=(3000, 5))
    w = rng.exponential(size=3000)
    for d in (0.05, 0.1):
        a = spa.concentration(v, w, [d])[0]
        b = spa.concentration_plain(v, w, [d])[0]
        assert np.max(np.abs(a - b)) <= 3000 * 2.0 ** -(63 - 12) + 1e-14
    # open interval: a value exactly at Delta counts as away from zero
    assert spa.concentration(np.array([0.1, -0.1, 0.0]), np.ones(3), [0.1])[0, 0] == 1.0 - 1.0 / 3.0


def test_scale_posterior_closed_form():
    lz = np.log([1.0, 2.0, 3.0, 4.0]) + 123.0
    assert np.allclose(spa.scale_posterior(lz), [0.1, 0.2, 0.3, 0.4], rtol=1e-13, atol=0)
    assert spa.scale_mode([8.0, 4.0, 2.0, 1.0], lz) == 1.0


def test_mixture_reduces_and_matches_the_repeated_sample():
    rng = np.random.default_rng(9)
    T, N, p = 3, 40, 2
    beta = rng.normal(size=(T, N, p))
    # one scale: the mixture is that scale's weighted set
    logW = np.log(np.full((1, N), 1.0 / N))
    qm, cm = spa.marginal_summaries(beta[:1], logW, [0.0], [0.05, 0.5], [0.1])
    assert np.array_equal(qm, spa.weighted_quantiles(beta[0], np.ones(N), [0.05, 0.5]))
    assert np.array_equal(cm, spa.concentration(beta[0], np.ones(N), [0.1]))
    # p_t in ratio 1:2:1 with equal W: scale t's particles count 1, 2, 1 times
    log_z = np.log([1.0, 2.0, 1.0])
    logW = np.full((T, N), -math.log(N))
    qm, _ = spa.marginal_summaries(beta, logW, log_z, [0.05, 0.5, 0.95], [0.1])
    reps = np.concatenate([beta[0], beta[1], beta[1], beta[2]])
    tot = 4 * N
    for li, a in enumerate([0.05, 0.5, 0.95]):
        if abs(a * tot - round(a * tot)) < 1e-6:
            continue
        for j in range(p):
            assert qm[li, j] == _inverted_cdf(reps[:, j], a)


def test_rejects_invalid_inputs():
    with pytest.raises(ValueError):
        spa.quantise_weights(np.zeros(3))
    with pytest.raises(ValueError):
        spa.quantise_weights(np.array([1.0, -1.0]))
    with pytest.raises(ValueError):
        spa.weighted_quantiles(np.ones(3), np.ones(3), [0.0])
