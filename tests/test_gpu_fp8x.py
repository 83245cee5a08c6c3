"""GPU parity of the FP8 multi-term forward contraction (SPA_PREC_FP8X3 / SPA_PREC_FP8X4)
against the FP64 oracle's log-likelihood of the same coefficients.

The coefficients are carried by 3 or 4 e4m3 terms with per-particle power-of-two scales;
each term resolves at least 4 more bits of the row's largest entry, so 3 terms meet the
1e-4 relative tolerance of the reduced-precision paths and 4 terms sit below the BF16
hi+lo error on the same inputs."""
import math

import numpy as np
import pytest

from oracle import likelihood
from tests.gpu_util import dataset, particles, rel_err

pytestmark = pytest.mark.gpu


def _torch():
    import torch
    return torch


def _sampler(name, n=None, p=None):
    from paper_1106_0322_amd import SamplerConfig, SpaSMC
    cfg, X, y, Xs = dataset(name, n, p)
    sc = SamplerConfig(n=X.shape[0], p=X.shape[1], N=64, a=cfg.a, lambdas=np.geomspace(10, 1, 2),
                       move="rwm", sweeps=0, init_sweeps=0, prec="bf16x2", seed=0)
    return SpaSMC(sc, X, y), cfg, X, y, Xs


@pytest.mark.parametrize("name,M", [("n5000_p200_mala_bf16", 300), ("n2000_p50_rwm_fp32", 700)])
def test_fp8x_loglik_parity(name, M):
    torch = _torch()
    s, cfg, X, y, Xs = _sampler(name)
    b = particles(M, X.shape[1], seed=M)
    errs = {}
    for dt in (torch.float64, torch.float32):
        bt = torch.from_numpy(b).to("cuda", dt)
        ref = likelihood.loglik(bt.double().cpu().numpy(), Xs, y)   # oracle at the stored values
        for prec in ("fp8x3", "fp8x4", "bf16x2"):
            got = s.loglik(bt, prec).cpu().numpy()
            errs[prec, dt] = rel_err(got, ref).max()
            print(f"{name} {prec} {dt}: max rel {errs[prec, dt]:.3e}")
        assert errs["fp8x3", dt] <= 1e-4
        assert errs["fp8x4", dt] <= 1e-4
        assert errs["fp8x4", dt] <= errs["bf16x2", dt]
    s.close()


@pytest.mark.parametrize("n,p,M", [
    (130, 1, 65), (70, 7, 129), (66, 127, 3), (200, 128, 128), (100, 129, 1), (64, 255, 64),
    (300, 256, 200), (34, 257, 130), (200, 383, 33), (200, 511, 40), (4000, 200, 5),
])
@pytest.mark.parametrize("prec", ["fp8x3", "fp8x4"])
def test_fp8x_loglik_edge_shapes(n, p, M, prec):
    """Rows of 128..512 padded markers, ragged marker, individual and particle counts, one
    and several individual splits."""
    torch = _torch()
    s, cfg, X, y, Xs = _sampler("n5000_p200_mala_bf16", n=n, p=p)
    b = particles(M, p, seed=n + p)
    got = s.loglik(torch.from_numpy(b).to("cuda", torch.float64), prec).cpu().numpy()
    ref = likelihood.loglik(b, Xs, y)
    assert rel_err(got, ref).max() <= 1e-4
    # beta = 0 gives -n log 2 up to rounding of the softplus sum
    z = s.loglik(torch.zeros(3, p, dtype=torch.float64, device="cuda"), prec).cpu().numpy()
    assert np.allclose(z, -n * math.log(2.0), rtol=1e-6)
    s.close()


@pytest.mark.parametrize("name,M", [("n5000_p200_mala_bf16", 16384), ("n10000_p500_mala_fp8", 32768)])
def test_fp8x_full_size_sampled(name, M):
    """At the particle counts of the timed comparison on the 5000 x 200 and 10000 x 500
    data sets (two individual splits each; 256 and 512 padded markers), sampled particles
    against the oracle one by one."""
    torch = _torch()
    s, cfg, X, y, Xs = _sampler(name)
    b = particles(M, X.shape[1], seed=7, scale=0.15)
    bt = torch.from_numpy(b).to("cuda", torch.float32)
    idx = np.random.default_rng(1).choice(M, size=256, replace=False)
    ref = likelihood.loglik(bt.double().cpu().numpy()[idx], Xs, y)
    for prec in ("fp8x3", "fp8x4"):
        got = s.loglik(bt, prec).cpu().numpy()
        assert np.all(np.isfinite(got))
        e = rel_err(got[idx], ref)
        print(f"{name} {prec} M={M}: sampled max rel {e.max():.3e}")
        assert e.max() <= 1e-4
    s.close()


def test_fp8x_nonfinite_coefficient_gives_nan_for_that_particle_only():
    torch = _torch()
    s, cfg, X, y, Xs = _sampler("n2000_p50_rwm_fp32")
    b = particles(130, X.shape[1], seed=2)
    b[5, 3] = np.nan
    b[77, 0] = np.inf
    got = s.loglik(torch.from_numpy(b).to("cuda", torch.float64), "fp8x4").cpu().numpy()
    bad = np.zeros(130, dtype=bool)
    bad[[5, 77]] = True
    assert np.all(np.isnan(got[bad]))
    ref = likelihood.loglik(b[~bad], Xs, y)
    assert rel_err(got[~bad], ref).max() <= 1e-4
    s.close()


def test_fp8x_is_refused_for_mala_and_the_gradient():
    from paper_1106_0322_amd import SamplerConfig, SpaSMC, SpaError
    torch = _torch()
    s, cfg, X, y, Xs = _sampler("n500_p10_rwm_fp64")
    with pytest.raises(SpaError):
        s.grad(torch.zeros(4, X.shape[1], dtype=torch.float64, device="cuda"), 1.0, "fp8x4")
    s.close()
    sc = SamplerConfig(n=X.shape[0], p=X.shape[1], N=64, a=cfg.a, lambdas=np.geomspace(10, 1, 2),
                       move="mala", sweeps=0, init_sweeps=0, prec="fp8x3", seed=0)
    with pytest.raises(SpaError):
        SpaSMC(sc, X, y)


@pytest.mark.parametrize("name,n,p,N,init,prec", [
    ("n5000_p200_rwm_fp32", None, None, None, 4, "fp8x3"),
    ("n5000_p200_rwm_fp32", None, None, None, 4, "fp8x4"),
    ("n10000_p500_mala_fp8", None, None, None, 2, "fp8x3"),   # 64 lanes per row
    ("n2000_p50_rwm_fp32", 2000, 256, 1024, 4, "fp8x3"),       # 64 lanes, 256-marker FP8 rows
])
def test_fp8x_random_walk_sampler(name, n, p, N, init, prec):
    """Random-walk sweeps contracting on the FP8 MFMA (the full 5000 x 200 / 16384 and
    10000 x 500 / 32768 shapes, and the p = 256 boundary where the move kernels switch to 64
    lanes per row while the FP8 rows stay 256 wide): the log-likelihoods the sampler keeps
    (its proposal step writes the term operand) are bit-identical to a fresh evaluation
    through the standalone packing (same layout, codes, exponents and summation order), and
    sampled rows are within 1e-4 of the oracle."""
    from paper_1106_0322_amd import SamplerConfig, SpaSMC
    cfg, X, y, Xs = dataset(name, n, p)
    w = cfg.replace(prec=prec, move="rwm", **({"N": N} if N else {}))
    s = SpaSMC(SamplerConfig.from_workload(w, n=X.shape[0], p=X.shape[1], init_sweeps=init), X, y)
    out = s.step()
    assert math.isfinite(out["ess"]) and 0.0 < out["accept_rate"] < 1.0
    beta, logw = s.particles()
    kept = s.state_loglik().cpu().numpy()
    fresh = s.loglik(beta, prec).cpu().numpy()
    assert np.array_equal(kept, fresh)
    idx = np.random.default_rng(0).choice(w.N, size=48, replace=False)
    ref = likelihood.loglik(beta[idx].double().cpu().numpy(), Xs, y)
    e = rel_err(kept[idx], ref)
    print(f"{name} p={X.shape[1]} {prec} sampler: sampled loglik max rel err {e.max():.3e}, "
          f"accept {out['accept_rate']:.3f}")
    assert e.max() <= 1e-4
    assert np.all(np.isfinite(logw.cpu().numpy()))
    s.close()
