"""Pins of the oracle's generalized-t prior against what the paper and mathematics fix
(Section 2: the general generalized-t density and its centred L1 form, the
scale-mixture representation, the double-exponential limit; Section 2.1: EM weight)."""
import math

import numpy as np
import pytest
from scipy import integrate, stats

from oracle import gt_prior

CASES = [(1.0, 1.0), (0.5, 0.01), (4.0, 1e3), (1.0, 1e-2), (0.5, 3.0), (4.0, 0.2)]


def _quad_line(f, scale):
    """Integral over the real line, split at the cusp and at the density's scale."""
    tot = 0.0
    for lo, hi in [(-np.inf, -scale), (-scale, 0.0), (0.0, scale), (scale, np.inf)]:
        v, _ = integrate.quad(f, lo, hi, limit=400, epsabs=0, epsrel=1e-12)
        tot += v
    return tot


@pytest.mark.parametrize("a,c", CASES)
def test_normalised(a, c):
    """The density integrates to one (normaliser 1/(2c) of the L1 form)."""
    tot = _quad_line(lambda b: math.exp(gt_prior.gt_logpdf(b, a, c)), a * c)
    assert abs(tot - 1.0) < 1e-9


@pytest.mark.parametrize("a,c", CASES)
def test_l1_form_is_general_form_q1(a, c):
    """q = 1, mu = 0 in the general density (B(1, a) = 1/a) gives the L1 form."""
    b = np.linspace(-5 * c, 5 * c, 101)
    ref = gt_prior.gt_general_pdf(b, 0.0, a, c, 1.0)
    got = np.exp(gt_prior.gt_logpdf(b, a, c))
    assert np.allclose(got, ref, rtol=1e-13, atol=0)


@pytest.mark.parametrize("a", [0.5, 1.0, 2.5, 10.0])
def test_general_form_student_special_case(a):
    """q = 2, c = sqrt(2) gives Student's t with 2a degrees of freedom."""
    b = np.linspace(-8, 8, 161)
    got = gt_prior.gt_general_pdf(b, 0.0, a, math.sqrt(2.0), 2.0)
    assert np.allclose(got, stats.t(df=2 * a).pdf(b), rtol=1e-12)


@pytest.mark.parametrize("a,c", CASES)
def test_lomax_special_case(a, c):
    """|beta| under Gt(a, c) is Lomax (Pareto II) with shape a and scale a c."""
    b = np.concatenate([-np.geomspace(1e-4, 1e4, 40) * c, np.geomspace(1e-4, 1e4, 40) * c])
    ref = np.log(0.5) + stats.lomax(c=a, scale=a * c).logpdf(np.abs(b))
    assert np.allclose(gt_prior.gt_logpdf(b, a, c), ref, rtol=1e-12, atol=1e-12)


@pytest.mark.parametrize("a,c", CASES)
def test_cdf_and_ppf(a, c):
    """Closed-form CDF equals the integral of the density; the inverse CDF inverts it."""
    def dens(x):
        return math.exp(gt_prior.gt_logpdf(x, a, c))

    left_half = _quad_line(lambda x: dens(x) if x < 0 else 0.0, a * c)
    assert abs(left_half - 0.5) < 1e-9
    for bi in np.geomspace(1e-3, 1e3, 13) * c:
        mid, _ = integrate.quad(dens, 0.0, bi, epsabs=0, epsrel=1e-12, limit=400)
        assert abs(gt_prior.gt_cdf(bi, a, c) - (0.5 + mid)) < 1e-9
        assert abs(gt_prior.gt_cdf(-bi, a, c) - (0.5 - mid)) < 1e-9
    u = np.linspace(0.001, 0.999, 99)
    assert np.allclose(gt_prior.gt_cdf(gt_prior.gt_ppf(u, a, c), a, c), u, rtol=0, atol=1e-12)


@pytest.mark.parametrize("a,c,beta", [(1.5, 0.2, 0.3), (0.5, 1.0, -2.0), (4.0, 0.05, 0.01),
                                      (1.0, 1.0, 0.0)])
def test_scale_mixture(a, c, beta):
    """beta | tau ~ DE(tau), tau ~ IG(a, b) has marginal Gt(a, b/a); with b = a c it is Gt(a, c)."""
    b = a * c
    ig = stats.invgamma(a, scale=b)

    def integrand(tau):
        return math.exp(-abs(beta) / tau) / (2.0 * tau) * ig.pdf(tau)

    v = 0.0
    for lo, hi in [(0, b / 100), (b / 100, b), (b, 100 * b), (100 * b, np.inf)]:
        v += integrate.quad(integrand, lo, hi, epsabs=0, epsrel=1e-12, limit=400)[0]
    assert abs(v - math.exp(gt_prior.gt_logpdf(beta, a, c))) < 1e-10 * max(1.0, v)


@pytest.mark.parametrize("a", [1e4, 1e6])
def test_double_exponential_limit(a):
    """log Gt - log DE = (x^2/2 - x)/a + O(a^-2), x = |beta|/c, as a -> inf."""
    c = 0.7
    b = np.linspace(-3, 3, 61)
    x = np.abs(b) / c
    gap = gt_prior.gt_logpdf(b, a, c) - gt_prior.de_logpdf(b, c)
    assert np.allclose(gap, (0.5 * x * x - x) / a, rtol=0, atol=20.0 / a ** 2)
    # the a = inf branch is the double exponential itself (library Laplace density)
    assert np.allclose(gt_prior.gt_logpdf(b, math.inf, c), stats.laplace(scale=c).logpdf(b),
                       rtol=1e-14, atol=1e-14)
    assert np.allclose(gt_prior.gt_cdf(b, math.inf, c), stats.laplace(scale=c).cdf(b),
                       rtol=1e-13, atol=1e-14)


def test_table1_log_density_shape():
    """Up to a constant, log Gt(a, c) is -(a+1) log(1 + |beta|/(a c)) (Table 1)."""
    a, c = 2.0, 0.3
    b = np.array([-1.0, -0.1, 0.0, 0.2, 3.0])
    d = gt_prior.gt_logpdf(b, a, c) - gt_prior.gt_logpdf(0.0, a, c)
    assert np.allclose(d, -(a + 1) * np.log(1 + np.abs(b) / (a * c)), rtol=1e-14, atol=1e-15)


@pytest.mark.parametrize("a,c", CASES + [(math.inf, 0.5)])
def test_gradient(a, c):
    """Central finite differences, EM-weight magnitude, sign(0) = 0."""
    rng = np.random.default_rng(1)
    b = rng.standard_t(2, size=200) * c
    b = b[np.abs(b) > 1e-3 * c]
    h = 1e-6 * c
    fd = (gt_prior.gt_logpdf(b + h, a, c) - gt_prior.gt_logpdf(b - h, a, c)) / (2 * h)
    g = gt_prior.gt_grad(b, a, c)
    assert np.allclose(g, fd, rtol=1e-6, atol=1e-6 / c)
    assert gt_prior.gt_grad(0.0, a, c) == 0.0
    if not math.isinf(a):
        assert np.allclose(np.abs(g), gt_prior.em_weight(b, a, c), rtol=1e-14)


def test_em_weight_lasso_limit():
    """As a -> inf the EM weight tends to 1/c (the Lasso penalty lambda = 1/c)."""
    c = 0.25
    b = np.array([0.0, 0.1, 1.0, 5.0])
    for a in [1e6, 1e8]:
        assert np.allclose(gt_prior.em_weight(b, a, c), 1.0 / c, rtol=10 * (1 + 5 / c) / a)
