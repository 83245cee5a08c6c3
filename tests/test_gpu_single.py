"""GPU parity of the paper's single-coordinate random-walk kernel (Section 4.1) against
the FP64 oracle.

* FP64 end to end: the Philox streams are shared, so the GPU trajectory (every accept
  decision of every coordinate update) tracks the oracle's to round-off;
* FP32: posterior-mean and log Z paths within Monte Carlo error over independent seeds;
* the log-likelihood the kernel leaves (from its incrementally updated predictor) equals
  the likelihood of the particles it leaves."""
import dataclasses
import math

import numpy as np
import pytest

from oracle import likelihood, smc
from synth import CONFIGS, make_dataset
from tests.gpu_util import rel_err

pytestmark = pytest.mark.gpu


def _torch():
    import torch
    return torch


def _setup(n, p, seed, **over):
    from paper_1106_0322_amd import SamplerConfig, SpaSMC
    cfg = CONFIGS["paper_small"].replace(**over)
    d = make_dataset(cfg, n=n, p=p, seed=seed)
    sc = SamplerConfig.from_workload(cfg, n=n, p=p)
    return cfg, d.X, d.y, sc, SpaSMC


@pytest.mark.parametrize("n,p,N,T,S,init", [
    (500, 10, 256, 6, 2, 6),      # one coordinate block, 8 individuals per lane
    (130, 150, 64, 4, 1, 2),      # three coordinate blocks, padded individuals
    (2048, 5, 32, 3, 1, 1),       # the largest n the kernel holds in registers
])
def test_fp64_trajectory_tracks_oracle(n, p, N, T, S, init):
    cfg, X, y, sc, SpaSMC = _setup(n, p, seed=n + p, N=N, T=T, sweeps=S, init_sweeps=init,
                                   prec="fp64", lambdas=tuple(0.5 * 0.8 ** np.arange(T)))
    Xs, _, _ = likelihood.standardise(X)
    prob = smc.Problem(Xs=Xs, y=y.astype(np.float64), a=cfg.a)
    r = smc.run_smc(prob, cfg.grid(), N, "single", S, init, cfg.ess_frac, 0.5, cfg.seed)
    g = SpaSMC(sc, X, y)
    print(f"single-site fp64 n={n} p={p} N={N}", flush=True)
    stats = g.run()
    mean, var, logz = g.paths()
    beta, _ = g.particles()
    d = np.abs(mean - r.mean).max()
    db = np.abs(beta.cpu().numpy() - r.state.beta).max()
    print(f"mean path max diff {d:.3e}; particles max diff {db:.3e}")
    assert d <= 1e-8 and db <= 1e-8
    assert np.allclose(logz, r.log_z, rtol=1e-10, atol=1e-9)
    assert [s["resampled"] for s in stats] == list(r.resampled)
    acc = np.array([s["accept_rate"] for s in stats[1:]])
    assert np.allclose(acc, r.accept[1:], rtol=0, atol=1e-12)


def test_loglik_left_by_the_kernel_is_the_likelihood_of_its_particles():
    torch = _torch()
    for prec, tol in (("fp64", 1e-10), ("fp32", 1e-4)):
        cfg, X, y, sc, SpaSMC = _setup(500, 50, seed=3, N=512, T=4, sweeps=5, init_sweeps=10, prec=prec)
        g = SpaSMC(sc, X, y)
        g.step()
        beta, _ = g.particles()
        Xs, _, _ = likelihood.standardise(X)
        ll_gpu = g.state_loglik().cpu().numpy()
        ref = likelihood.loglik(beta.double().cpu().numpy(), Xs, y.astype(np.float64))
        e = rel_err(ll_gpu, ref).max()
        print(f"{prec}: loglik of the particles, max rel err {e:.3e}")
        assert e <= tol


def test_fp32_statistical_parity():
    """8 GPU seeds against 8 stored FP64 oracle replicates of the same configuration:
    posterior means and log Z within Monte Carlo error (family-wise Welch and exact
    permutation rules)."""
    from tests.replicate_util import check_fixture, compare, failed, gpu_replicates, load_fixture
    fx = load_fixture("single_n500_p12_T8")
    cfg = CONFIGS["paper_small"].replace(n=500, p=12, data_seed=9, N=512, T=8, sweeps=2, init_sweeps=20,
                                         lam_hi=1.0, lam_lo=0.2097152, lambdas=None)
    d = make_dataset(cfg)
    check_fixture(fx, cfg, d.X, d.y)
    gm, gz = gpu_replicates(cfg, d.X, d.y, fx["mean"].shape[0])
    res = compare("single-coordinate fp32", gm, fx["mean"], gz, fx["log_z"], exchangeable=int(fx["N"]) == cfg.N)
    assert not failed(res), failed(res)


def test_rejects_too_many_individuals():
    from paper_1106_0322_amd import SpaError
    cfg, X, y, sc, SpaSMC = _setup(2050, 5, seed=1, N=16, T=2, sweeps=1, init_sweeps=0, prec="fp32")
    with pytest.raises(SpaError) as ei:
        SpaSMC(sc, X, y)
    assert ei.value.status == 2


def test_fp32_decisions_follow_fp64():
    """The FP32 kernel forms each move's likelihood difference as delta c_j + half the change
    of sum |eta| + the log of two products (a rearrangement of the FP64 kernel's
    softplus differences).  From the same data and Philox draws its accept decisions must be
    those of the FP64 kernel, which follows the oracle decision for decision, except where
    a difference of rounding falls between log u and the acceptance log ratio: a handful of
    particles at most, and the same acceptance rates."""
    torch = _torch()
    runs = {}
    for prec in ("fp64", "fp32"):
        # scales close together: no resampling, so the particles stay in step
        cfg, X, y, sc, SpaSMC = _setup(500, 10, seed=5, N=512, T=3, sweeps=3, init_sweeps=5, prec=prec,
                                       lambdas=(0.5, 0.495, 0.49))
        g = SpaSMC(sc, X, y)
        stats = [g.step() for _ in range(2)]
        assert not any(s["resampled"] for s in stats)
        beta, _ = g.particles()
        runs[prec] = (beta.double().cpu().numpy(), [s["accept_rate"] for s in stats])
    b64, a64 = runs["fp64"]
    b32, a32 = runs["fp32"]
    dev = np.abs(b32 - b64).max(axis=1)
    diverged = float(np.mean(dev > 1e-4))
    print(f"fp32 vs fp64: particles apart {diverged:.4f}, largest kept deviation "
          f"{dev[dev <= 1e-4].max():.2e}, accept rates {a32} vs {a64}")
    assert diverged <= 0.02
    assert np.allclose(a32, a64, rtol=0, atol=0.01)
