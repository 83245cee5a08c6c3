"""Pins of the oracle's Philox4x32-10 (published known-answer vectors) and of the
normals and uniforms derived from it."""
import os

import numpy as np
from scipy import stats

from oracle import philox


def _kat(golden_dir):
    rows = []
    with open(os.path.join(golden_dir, "philox4x32_10_kat.txt")) as f:
        for line in f:
            if line.strip() and not line.startswith("#"):
                rows.append([int(v, 16) for v in line.split()])
    return rows


def test_known_answer_vectors(golden_dir):
    rows = _kat(golden_dir)
    assert len(rows) == 3
    for r in rows:
        out = philox.philox4x32_10(np.array(r[0:4], dtype=np.uint64), (r[4], r[5]))
        assert [int(v) for v in out] == r[6:10]


def test_vectorised_matches_scalar():
    ctr = np.array([[i, 7, 3, 0x55] for i in range(10)], dtype=np.uint64)
    out = philox.philox4x32_10(ctr, (123, 456))
    for i in range(10):
        assert np.array_equal(out[i], philox.philox4x32_10(ctr[i], (123, 456)))


def test_normals_distribution():
    z = philox.proposal_normals(seed=11, N=4096, p=64, sweep=3, t=5).ravel()
    n = z.size
    assert abs(z.mean()) < 5.0 / np.sqrt(n)
    assert abs(z.var() - 1.0) < 5.0 * np.sqrt(2.0 / n)
    assert stats.kstest(z, "norm").pvalue > 1e-4


def test_uniforms_open_interval_and_streams_distinct():
    u = philox.mh_uniforms(seed=2, N=100000, sweep=0, t=1)
    assert u.min() > 0.0 and u.max() < 1.0
    assert stats.kstest(u, "uniform").pvalue > 1e-4
    z0 = philox.proposal_normals(2, 8, 8, 0, 1)
    z1 = philox.proposal_normals(2, 8, 8, 1, 1)
    z2 = philox.proposal_normals(2, 8, 8, 0, 2)
    z3 = philox.proposal_normals(3, 8, 8, 0, 1)
    for other in (z1, z2, z3):
        assert not np.any(np.isclose(z0, other))
    # the first p normals of a longer row are the same draws
    assert np.array_equal(philox.proposal_normals(2, 8, 6, 0, 1), z0[:, :6])


def test_resample_word_layout():
    w = philox.philox4x32_10(np.array([0, 0, 0, (9 << 4) | 2], dtype=np.uint64),
                             philox.key_of(0x1234_5678_9ABC))
    assert philox.resample_u32(0x1234_5678_9ABC, 9) == int(w[0])
    assert philox.key_of(0x1234_5678_9ABC) == (0x5678_9ABC, 0x1234)
