"""Helpers of the replicate parity tests: stored oracle replicates, GPU replicates and the
statistical rules of ``tests/stats_gate.py``."""
import hashlib
import os

import numpy as np

from tests.stats_gate import describe, permutation_gate, welch_gate

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")
GPU_SEED0 = 1000      # GPU replicate r uses Philox key 1000 + r (the oracle's are 2000 + r)


def load_fixture(name: str):
    """Oracle replicates written by tests/golden/make_replicates.py."""
    return np.load(os.path.join(GOLDEN, f"replicates_{name}.npz"), allow_pickle=False)


def data_digest(X, y) -> str:
    h = hashlib.sha256()
    h.update(np.ascontiguousarray(X, dtype=np.uint8).tobytes())
    h.update(np.ascontiguousarray(y, dtype=np.uint8).tobytes())
    return h.hexdigest()


def check_fixture(fx, cfg, X, y):
    """The fixture was written for this data set and this sampler (up to precision and N)."""
    assert str(fx["data_sha256"]) == data_digest(X, y), "fixture was written for other data"
    assert (int(fx["n"]), int(fx["p"])) == X.shape
    assert int(fx["T"]) == cfg.T and int(fx["sweeps"]) == cfg.sweeps
    assert int(fx["init_sweeps"]) == cfg.init_sweeps and str(fx["move"]) == cfg.move
    assert float(fx["a"]) == cfg.a
    assert np.array_equal(fx["lambdas"], cfg.grid())


def gpu_replicates(cfg, X, y, R: int):
    """R runs of the HIP sampler over the whole grid, Philox keys GPU_SEED0 + r."""
    from paper_1106_0322_amd import SamplerConfig, SpaSMC
    means, logz = [], []
    for r in range(R):
        g = SpaSMC(SamplerConfig.from_workload(cfg, n=X.shape[0], p=X.shape[1], seed=GPU_SEED0 + r), X, y)
        g.run()
        m, _, lz = g.paths()
        means.append(m)
        logz.append(lz)
        g.close()
    return np.stack(means), np.stack(logz)


def compare(case, gm, om, gz, oz, exchangeable: bool) -> dict:
    """Welch rule always; the permutation rule too when both sides run at the same N."""
    om = np.asarray(om, np.float64)
    results = {"means, Welch": welch_gate(gm, om), "log Z, Welch": welch_gate(gz, oz)}
    if exchangeable:
        results["means, permutation"] = permutation_gate(gm, om)
        results["log Z, permutation"] = permutation_gate(gz, oz)
    for name, res in results.items():
        print(describe(f"{case} {name}", res))
    return results


def failed(results: dict):
    return [k for k, v in results.items() if not v["passed"]]
