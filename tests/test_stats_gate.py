"""CPU checks of the replicate-parity rules (tests/stats_gate.py)."""
import math

import numpy as np
from scipy import stats

from tests.stats_gate import permutation_gate, welch_gate, welch_t


def _paths(rng, R, shape, sd):
    base = np.cumsum(rng.normal(size=shape), axis=0) * 0.01
    return base, base + rng.normal(scale=sd, size=(R,) + shape)


def test_welch_matches_scipy():
    """Per-cell Welch t and its Satterthwaite p-value equal scipy's unequal-variance t test."""
    rng = np.random.default_rng(0)
    g = rng.normal(0.0, 1.0, size=(8, 25))
    o = rng.normal(0.3, 2.0, size=(6, 25))
    t, nu, _, _ = welch_t(g, o)
    ref = stats.ttest_ind(g, o, equal_var=False, axis=0)
    assert np.allclose(t, ref.statistic, rtol=1e-12)
    assert np.allclose(2.0 * stats.t.sf(np.abs(t), nu), ref.pvalue, rtol=1e-9)


def test_null_passes_both_rules():
    rng = np.random.default_rng(1)
    base, g = _paths(rng, 8, (40, 30), 0.01)
    o = base + rng.normal(scale=0.02, size=(8, 40, 30))
    w = welch_gate(g, o)
    pm = permutation_gate(g, o)
    assert w["passed"] and pm["passed"]
    assert pm["splits"] == math.comb(16, 8)
    assert 1.0 / pm["splits"] <= pm["p_value"] <= 1.0


def test_local_departure_fails():
    """One cell 15 standard errors away fails the Bonferroni rule and the max-|t| permutation
    rule."""
    rng = np.random.default_rng(2)
    base, g = _paths(rng, 8, (40, 30), 0.01)
    o = base + rng.normal(scale=0.01, size=(8, 40, 30))
    se = math.sqrt(2 * 0.01 ** 2 / 8)
    g[:, 17, 4] += 15 * se
    assert not welch_gate(g, o)["passed"]
    pm = permutation_gate(g, o)
    assert not pm["passed"] and pm["p_value"] < 1e-3


def test_systematic_departure_fails_rms_rule():
    """A shift of 0.8 standard errors in every cell is invisible to max |t| but not to the
    rms permutation rule."""
    rng = np.random.default_rng(3)
    base, g = _paths(rng, 8, (40, 30), 0.01)
    o = base + rng.normal(scale=0.01, size=(8, 40, 30))
    g = g + 0.8 * math.sqrt(2 * 0.01 ** 2 / 8)
    assert welch_gate(g, o)["passed"]
    pm = permutation_gate(g, o)
    assert pm["p_value_rms"] < 5e-4 and not pm["passed"]


def test_constant_cells():
    """Cells equal on every replicate of both sides are left out; a zero-variance cell that
    differs between the sides fails."""
    rng = np.random.default_rng(4)
    g = rng.normal(size=(8, 10))
    o = rng.normal(size=(8, 10))
    g[:, 0] = o[:, 0] = 0.0
    w = welch_gate(g, o)
    assert w["cells"] == 9 and w["passed"]
    g[:, 1] = 1.0
    o[:, 1] = 2.0
    assert not welch_gate(g, o)["passed"] and not permutation_gate(g, o)["passed"]
