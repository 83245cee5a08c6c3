"""Pins of the oracle's systematic resampler: the textbook definition in exact rational
arithmetic, the offspring-count property, special cases and error paths."""
from fractions import Fraction

import numpy as np
import pytest

from oracle import smc


def exact_systematic(q, u32):
    """Systematic resampling of integer weights q with offset U = u32/2^32, in exact
    rational arithmetic: offspring i takes the first k with C_k > (i + U) C / M."""
    M = len(q)
    C = np.cumsum([int(v) for v in q]).tolist()
    U = Fraction(int(u32), 2 ** 32)
    out = []
    k = 0
    for i in range(M):
        t = (i + U) * C[-1] / M     # exact; the FP64 version rounds (i+U)*C, then /M
        while k < M - 1 and not C[k] > t:
            k += 1
        out.append(k)
    return np.array(out)


def quantise(w):
    M = len(w)
    K = 53 - smc.ceil_log2(M)
    return np.floor((np.asarray(w) / np.max(w)) * 2.0 ** K)


@pytest.mark.parametrize("M", [1, 2, 7, 64, 1000, 1024])
def test_matches_exact_definition(M):
    rng = np.random.default_rng(M)
    for trial in range(5):
        w = rng.exponential(size=M) ** 3
        if trial == 1:
            w[rng.integers(0, M, size=max(1, M // 3))] = 0.0
            w[0] = max(w[0], 1e-3)
        u32 = int(rng.integers(0, 2 ** 32))
        got = smc.systematic_resample(w, u32)
        ref = exact_systematic(quantise(w), u32)
        assert np.array_equal(got, ref)
        assert np.all(np.diff(got) >= 0)
        assert got.min() >= 0 and got.max() < M


def test_identity_on_equal_weights():
    for M in (1, 5, 1000, 1024, 32768, 100000):
        assert np.array_equal(smc.systematic_resample(np.ones(M), 0), np.arange(M))


@pytest.mark.parametrize("M", [8, 256, 4096])
def test_offspring_counts_floor_ceil(M):
    """o_k is floor(M W_k) or ceil(M W_k) and sum o_k = M (dyadic weights, so the
    quantisation is exact)."""
    rng = np.random.default_rng(M + 1)
    for _ in range(10):
        w = rng.integers(0, 2 ** 20, size=M).astype(np.float64)
        w[0] = 2.0 ** 20
        W = w / w.sum()
        anc = smc.systematic_resample(w, int(rng.integers(0, 2 ** 32)))
        o = np.bincount(anc, minlength=M)
        assert o.sum() == M
        assert np.all(o >= np.floor(M * W) - 1e-9) and np.all(o <= np.ceil(M * W) + 1e-9)


def test_zero_weight_never_selected():
    w = np.array([0.0, 1.0, 0.0, 2.0, 0.0])
    for u in (0, 2 ** 31, 2 ** 32 - 1):
        anc = smc.systematic_resample(w, u)
        assert set(anc.tolist()) <= {1, 3}


def test_power_of_two_scale_invariance():
    """Only w / max w enters, so scaling by a power of two changes nothing."""
    rng = np.random.default_rng(9)
    w = rng.exponential(size=500)
    ref = smc.systematic_resample(w, 12345)
    for s in (2.0 ** -600, 2.0 ** -30, 2.0 ** 500):
        assert np.array_equal(smc.systematic_resample(w * s, 12345), ref)


@pytest.mark.parametrize("bad", [np.array([]), np.array([0.0, 0.0]), np.array([1.0, -1.0]),
                                 np.array([1.0, np.nan]), np.array([np.inf, 1.0])])
def test_rejects_bad_weights(bad):
    with pytest.raises(ValueError):
        smc.systematic_resample(bad, 0)
