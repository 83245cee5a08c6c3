"""Whole-sweep statistical parity at the workloads' stated sizes (Section 4, Section 4.2).

Each workload's full scale grid (T scales, S sweeps per scale, the stated burn-in) runs on
the GPU from 8 independent Philox keys.  Its posterior-mean path (T x p cells) and its
log Z_t / Z_1 path are compared with 8 FP64 oracle replicates stored in
``tests/golden/replicates_<workload>_N<N>.npz``.  ``tests/golden/make_replicates.py`` wrote
those from ``oracle`` and ``synth`` only.  ``tests/stats_gate.py`` holds the rules:
* the family-wise Welch-t rule applies at any pair of particle counts;
* the exact permutation rule is added when the GPU runs at the oracle's particle count.
The GPU runs in the precision the workload names: FP32 random walk, BF16 hi+lo from FP8
storage, the FP8 three-term random walk, BF16 hi+lo MALA, and MALA on FP8 storage; one
case runs MALA with 20 sweeps per scale in FP64 (the ESS/s reference of bench.py).
"""
import numpy as np
import pytest

from synth import CONFIGS, make_dataset
from tests.replicate_util import check_fixture, compare, failed, gpu_replicates, load_fixture

pytestmark = pytest.mark.gpu

# (case id, workload whose data are used, fixture name, sampler overrides of the fixture
# (both sides), GPU-only overrides, oracle N, GPU N)
CASES = [
    ("n2000_p50_rwm_fp32", "n2000_p50_rwm_fp32", None, {}, {}, 8192, 8192),
    ("n2000_p50_rwm_bf16x2_fp8storage", "n2000_p50_rwm_fp32", None, {}, dict(prec="bf16x2", xfmt="fp8"), 8192, 8192),
    ("n2000_p50_rwm_fp8x3", "n2000_p50_rwm_fp32", None, {}, dict(prec="fp8x3"), 8192, 8192),
    ("n5000_p200_mala_bf16_full", "n5000_p200_mala_bf16", None, {}, {}, 4096, 16384),
    ("n5000_p200_mala_bf16_N4096", "n5000_p200_mala_bf16", None, {}, {}, 4096, 4096),
    # 20 sweeps per scale (the ESS/s reference of bench.py), FP64 on both sides
    ("n5000_p200_mala_fp64_S20_N2048", "n5000_p200_mala_bf16", "n5000_p200_mala_S20_N2048", dict(sweeps=20),
     dict(prec="fp64"), 2048, 2048),
    ("n10000_p500_mala_fp8_full", "n10000_p500_mala_fp8", None, {}, {}, 1024, 32768),
    ("n10000_p500_mala_fp8_N1024", "n10000_p500_mala_fp8", None, {}, {}, 1024, 1024),
]


@pytest.mark.parametrize("case,workload,fixture,over,gpu_over,N_orc,N_gpu", CASES, ids=[c[0] for c in CASES])
def test_sweep_parity(case, workload, fixture, over, gpu_over, N_orc, N_gpu):
    import os
    from tests.replicate_util import GOLDEN
    name = fixture or f"{workload}_N{N_orc}"
    if not os.path.exists(os.path.join(GOLDEN, f"replicates_{name}.npz")):
        pytest.skip(f"oracle fixture replicates_{name}.npz not written yet (tests/golden/make_replicates.py)")
    fx = load_fixture(name)
    base = CONFIGS[workload].replace(**over)
    d = make_dataset(base)
    check_fixture(fx, base, d.X, d.y)
    assert int(fx["N"]) == N_orc
    cfg = base.replace(N=N_gpu, **gpu_over)
    om, oz = fx["mean"], fx["log_z"]
    gm, gz = gpu_replicates(cfg, d.X, d.y, om.shape[0])
    assert gm.shape == om.shape and gz.shape == oz.shape
    assert np.all(np.isfinite(gm)) and np.all(np.isfinite(gz))
    res = compare(case, gm, om, gz, oz, exchangeable=N_gpu == N_orc)
    assert not failed(res), failed(res)
