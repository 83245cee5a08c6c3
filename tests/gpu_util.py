"""Shared helpers of the GPU parity tests: seeded inputs and particle sets."""
import functools

import numpy as np

from oracle import likelihood
from synth import CONFIGS, make_dataset


@functools.lru_cache(maxsize=None)
def dataset(name: str, n: int = None, p: int = None, seed: int = None):
    cfg = CONFIGS[name]
    d = make_dataset(cfg, n=n, p=p, seed=seed)
    Xs, mu, s = likelihood.standardise(d.X)
    return cfg, d.X, d.y, Xs


def particles(M: int, p: int, seed: int, scale: float = 0.15):
    """A mix of posterior-like draws, exact zeros, tight clusters and heavy tails."""
    rng = np.random.default_rng(seed)
    b = rng.normal(0.0, scale, size=(M, p))
    kind = rng.integers(0, 4, size=M)
    b[kind == 1] *= 0.05
    b[kind == 2] = rng.standard_t(1.5, size=(int((kind == 2).sum()), p)) * scale
    mask = rng.uniform(size=(M, p)) < 0.3
    b[(kind == 3)[:, None] & mask] = 0.0
    b = np.clip(b, -3.0, 3.0)
    return b


def rel_err(got, ref):
    return np.abs(got - ref) / np.maximum(np.abs(ref), 1e-300)
