"""spa_smc_loglik_noalloc: the log-likelihood entry point that allocates nothing.

Its operand and split partial sums live in the library's static per-GPU scratch array.
Its output is checked against spa_smc_loglik's on the same particles (same kernels, so
bit-identical), over two calls in a row, the second with a smaller input, and against the
FP64 oracle on sampled rows (1e-10 relative in FP64, 1e-4 in FP32 and BF16 hi+lo)."""
import numpy as np
import pytest

from oracle import likelihood
from tests.gpu_util import dataset, particles, rel_err

pytestmark = pytest.mark.gpu


def _handle(name, prec, N=256):
    from paper_1106_0322_amd import SamplerConfig, SpaSMC
    cfg, X, y, Xs = dataset(name)
    sc = SamplerConfig(n=X.shape[0], p=X.shape[1], N=N, a=cfg.a, lambdas=np.geomspace(10, 1, 2),
                       move="rwm", sweeps=0, init_sweeps=0, prec=prec, seed=0)
    return SpaSMC(sc, X, y), X, y, Xs


def _both(s, b, prec, dtype):
    import torch
    bt = torch.from_numpy(b).to("cuda", dtype).contiguous()
    ref = s.loglik(bt, prec)
    out = torch.full((b.shape[0],), float("nan"), dtype=torch.float64, device="cuda")
    s.loglik_noalloc(bt, out, prec)
    torch.cuda.synchronize()
    return out.cpu().numpy(), ref.cpu().numpy(), bt.double().cpu().numpy()


# (workload, precision, first M, second M, oracle tolerance); the BF16 case's first call
# is the bench workload's particle count at p = 200
CASES = [
    ("n5000_p200_mala_bf16", "bf16x2", 16384, 1000, 1e-4),
    ("n5000_p200_mala_bf16", "fp32", 3000, 129, 1e-4),
    ("n2000_p50_rwm_fp32", "fp64", 2000, 77, 1e-10),
    ("n500_p10_rwm_fp64", "fp64", 1000, 1, 1e-10),
]


@pytest.mark.parametrize("name,prec,M1,M2,tol", CASES, ids=[f"{c[0]}-{c[1]}" for c in CASES])
def test_noalloc_matches_loglik(name, prec, M1, M2, tol):
    import torch
    s, X, y, Xs = _handle(name, prec)
    dt = torch.float64 if prec == "fp64" else torch.float32
    for call, M in enumerate((M1, M2)):
        b = particles(M, X.shape[1], seed=100 + call)
        got, ref, bstored = _both(s, b, prec, dt)
        assert np.array_equal(got, ref), f"call {call}: differs from spa_smc_loglik"
        idx = np.unique(np.random.default_rng(call).choice(M, size=min(M, 64), replace=False))
        r = likelihood.loglik(bstored[idx], Xs, y)
        assert rel_err(got[idx], r).max() <= tol
    s.close()


def test_noalloc_shares_the_array_across_handles():
    """Two handles on one GPU use the same array in turn (ordered on one stream)."""
    import torch
    s1, X1, y1, Xs1 = _handle("n5000_p200_mala_bf16", "bf16x2")
    s2, X2, y2, Xs2 = _handle("n2000_p50_rwm_fp32", "bf16x2")
    b1 = particles(4096, X1.shape[1], seed=7)
    b2 = particles(500, X2.shape[1], seed=8)
    for _ in range(2):
        g1, r1, _ = _both(s1, b1, "bf16x2", torch.float32)
        g2, r2, _ = _both(s2, b2, "bf16x2", torch.float32)
        assert np.array_equal(g1, r1) and np.array_equal(g2, r2)
    s1.close()
    s2.close()


def test_noalloc_refusals():
    import torch
    from paper_1106_0322_amd import SpaError
    s, X, y, Xs = _handle("n5000_p200_mala_bf16", "bf16x2")
    out = torch.empty(200000, dtype=torch.float64, device="cuda")
    big = torch.zeros(200000, X.shape[1], dtype=torch.float32, device="cuda")
    with pytest.raises(SpaError) as ei:      # buffers beyond the static array
        s.loglik_noalloc(big, out, "bf16x2")
    assert ei.value.status == 1 and "too large" in str(ei.value)
    small = big[:64].contiguous()
    with pytest.raises(SpaError) as ei:      # no FP8 multi-term form
        s.loglik_noalloc(small, out, "fp8x3")
    assert ei.value.status == 1
    with pytest.raises(SpaError) as ei:      # FP32 genotype copy not prepared yet
        s.loglik_noalloc(small, out, "fp32")
    assert ei.value.status == 5
    s.loglik(small, "fp32")                  # prepares it
    s.loglik_noalloc(small, out, "fp32")
    torch.cuda.synchronize()
    assert np.allclose(out[:64].cpu().numpy(), s.loglik(small, "fp32").cpu().numpy(), rtol=0, atol=0)
    s.close()
