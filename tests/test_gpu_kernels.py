"""GPU parity of the C-ABI entry points against the FP64 oracle, element by element.

Tolerances: per-particle log-likelihood relative error 1e-10 (FP64) and 1e-4 (FP32 and
BF16 hi+lo); gradients see the per-test derivation; resampling and Philox bit-exact."""
import math

import numpy as np
import pytest

from oracle import gt_prior, likelihood, philox, smc
from tests.gpu_util import dataset, particles, rel_err

pytestmark = pytest.mark.gpu


def _torch():
    import torch
    return torch


def _sampler(name, prec, n=None, p=None, N=64, xfmt="auto", move="rwm", T=2, **kw):
    from paper_1106_0322_amd import SamplerConfig, SpaSMC
    cfg, X, y, Xs = dataset(name, n, p)
    sc = SamplerConfig(n=X.shape[0], p=X.shape[1], N=N, a=cfg.a, lambdas=np.geomspace(10, 1, T),
                       move=move, sweeps=0, init_sweeps=0, prec=prec, xfmt=xfmt, seed=0, **kw)
    return SpaSMC(sc, X, y), cfg, X, y, Xs


def test_philox_bit_exact():
    torch = _torch()
    s, *_ = _sampler("n500_p10_rwm_fp64", "fp64")
    rng = np.random.default_rng(0)
    ctr = rng.integers(0, 2 ** 32, size=(4096, 4), dtype=np.uint64)
    ctr[:3] = [[0, 0, 0, 0], [2 ** 32 - 1] * 4, [0x243f6a88, 0x85a308d3, 0x13198a2e, 0x03707344]]
    for seed in (0, 0x299f31d0a4093822, 0xFFFFFFFFFFFFFFFF, 12345):
        got = s.philox(torch.from_numpy(ctr.astype(np.uint32).view(np.int32)), seed)
        got = got.cpu().numpy().view(np.uint32).reshape(-1, 4)
        ref = philox.philox4x32_10(ctr, philox.key_of(seed))
        assert np.array_equal(got, ref)


@pytest.mark.parametrize("name,prec,M,tol", [
    ("n500_p10_rwm_fp64", "fp64", 1000, 1e-10),
    ("n2000_p50_rwm_fp32", "fp64", 333, 1e-10),
    ("n2000_p50_rwm_fp32", "fp32", 700, 1e-4),
    ("n2000_p50_rwm_fp32", "bf16x2", 700, 1e-4),
    ("n5000_p200_mala_bf16", "bf16x2", 300, 1e-4),
    ("n5000_p200_mala_bf16", "fp32", 200, 1e-4),
    ("n5000_p200_mala_bf16", "fp64", 100, 1e-10),
])
def test_loglik_parity(name, prec, M, tol):
    torch = _torch()
    s, cfg, X, y, Xs = _sampler(name, prec)
    b = particles(M, X.shape[1], seed=M)
    ref = likelihood.loglik(b, Xs, y)
    for dt in (torch.float64, torch.float32):
        bt = torch.from_numpy(b).to("cuda", dt)
        got = s.loglik(bt, prec).cpu().numpy()
        r = likelihood.loglik(bt.double().cpu().numpy(), Xs, y)   # oracle at the stored values
        e = rel_err(got, r)
        print(f"{name} {prec} {dt}: max rel {e.max():.3e}, max abs {np.abs(got - r).max():.3e}")
        assert e.max() <= tol
    assert np.allclose(ref, likelihood.loglik(b, Xs, y))


@pytest.mark.parametrize("n,p", [(2000, 50), (2000, 300)])
def test_loglik_fp8_storage_equals_bf16_storage(n, p):
    """The 0/1/2 genotypes are exact in FP8 and in BF16, and both storages feed the same
    BF16 contraction (rows of up to 256 and of more markers): identical results."""
    torch = _torch()
    s8, cfg, X, y, Xs = _sampler("n2000_p50_rwm_fp32", "bf16x2", n=n, p=p, xfmt="fp8")
    s16, *_ = _sampler("n2000_p50_rwm_fp32", "bf16x2", n=n, p=p, xfmt="bf16")
    b = torch.from_numpy(particles(257, X.shape[1], seed=3)).to("cuda", torch.float32)
    assert torch.equal(s8.loglik(b), s16.loglik(b))


@pytest.mark.parametrize("n,p,M", [(2000, 50, 257), (5000, 200, 1000), (334, 127, 130), (1000, 255, 64),
                                   (130, 63, 129), (64, 100, 200), (400, 300, 130), (1000, 511, 65)])
def test_grad_fp8_storage_equals_bf16_storage(n, p, M):
    """The BF16 hi+lo log-likelihood with the adjoint from FP8 and from BF16 genotype
    storage (FP8 codes widened to BF16 through registers, BF16 copied straight into LDS):
    the same arithmetic in the same order, so log-likelihoods and gradients are identical
    (ragged individual counts, one or more individual splits, padded particle rows)."""
    torch = _torch()
    s8, cfg, X, y, Xs = _sampler("n5000_p200_mala_bf16", "bf16x2", n=n, p=p, xfmt="fp8", move="mala")
    s16, *_ = _sampler("n5000_p200_mala_bf16", "bf16x2", n=n, p=p, xfmt="bf16", move="mala")
    b = torch.from_numpy(particles(M, X.shape[1], seed=p)).to("cuda", torch.float32)
    g8, lp8 = s8.grad(b, 0.3)
    g16, lp16 = s16.grad(b, 0.3)
    assert torch.equal(g8, g16) and torch.equal(lp8, lp16)
    bs = b.double().cpu().numpy()
    ll_ref = likelihood.loglik(bs, Xs, y) + gt_prior.log_prior(bs, cfg.a, 0.3)
    assert rel_err(lp16.cpu().numpy(), ll_ref).max() <= 1e-4


@pytest.mark.parametrize("n,p,prec,M", [
    (130, 1, "fp64", 1), (130, 1, "bf16x2", 65), (70, 7, "fp32", 129), (200, 255, "fp64", 17),
    (200, 511, "bf16x2", 33), (200, 511, "fp32", 40), (64, 31, "bf16x2", 64), (66, 32, "bf16x2", 3),
    # BF16 rows of PP = 64, 128, 224, 256; one split (n <= 64) and ragged tails
    (60, 100, "bf16x2", 50), (200, 63, "bf16x2", 129), (100, 127, "bf16x2", 5), (34, 200, "bf16x2", 130),
    (300, 255, "bf16x2", 200),
])
def test_loglik_edge_shapes(n, p, prec, M):
    torch = _torch()
    s, cfg, X, y, Xs = _sampler("n5000_p200_mala_bf16", prec, n=n, p=p)
    b = particles(M, p, seed=n + p)
    bt = torch.from_numpy(b).to("cuda", torch.float64)
    got = s.loglik(bt, prec).cpu().numpy()
    ref = likelihood.loglik(b, Xs, y)
    tol = 1e-10 if prec == "fp64" else 1e-4
    assert rel_err(got, ref).max() <= tol
    # beta = 0 gives exactly -n log 2 up to rounding of the softplus sum
    z = s.loglik(torch.zeros(3, p, dtype=torch.float64, device="cuda"), prec).cpu().numpy()
    assert np.allclose(z, -n * math.log(2.0), rtol=1e-12 if prec == "fp64" else 1e-6)


@pytest.mark.parametrize("name,prec", [("n5000_p200_mala_bf16", "bf16x2"), ("n5000_p200_mala_bf16", "fp32"), ("n2000_p50_rwm_fp32", "bf16x2"), ("n500_p10_rwm_fp64", "fp64")])
def test_loglik_difference_of_a_move(name, prec):
    """The MH decision uses l(beta') - l(beta): its absolute error for proposal-sized moves
    (the sum of the two evaluations' errors bounds it; both are checked to 1e-4 or 1e-10
    relative), reported beside the per-particle errors."""
    torch = _torch()
    s, cfg, X, y, Xs = _sampler(name, prec)
    M = 256
    b = particles(M, X.shape[1], seed=11)
    rng = np.random.default_rng(5)
    b2 = b + 0.01 * rng.standard_normal(b.shape)
    dt = torch.float64 if prec == "fp64" else torch.float32
    bt, bt2 = (torch.from_numpy(v).to("cuda", dt) for v in (b, b2))
    l1, l2 = s.loglik(bt, prec).cpu().numpy(), s.loglik(bt2, prec).cpu().numpy()
    r1 = likelihood.loglik(bt.double().cpu().numpy(), Xs, y)
    r2 = likelihood.loglik(bt2.double().cpu().numpy(), Xs, y)
    err = np.abs((l2 - l1) - (r2 - r1))
    rel = 1e-10 if prec == "fp64" else 1e-4
    print(f"{name} {prec}: |d(l'-l)| max {err.max():.3e}, median {np.median(err):.3e}; "
          f"|l'-l| median {np.median(np.abs(r2 - r1)):.3e}")
    assert np.all(err <= rel * (np.abs(r1) + np.abs(r2)))


def _grad_tol(prec, Xs):
    # FP64: round-off only.  Reduced precision: the coefficients enter as b~ = b (1 + d),
    # |d| <= 2^-16 (BF16 hi+lo) or 2^-24 (FP32), the residuals likewise, and the FP32
    # accumulation over n terms adds n 2^-24 |X| per term; bounded by
    # c * sum_k |X_std,kj| with c = 1e-4 (BF16 hi+lo) and 1e-5 (FP32).
    col = np.abs(Xs).sum(axis=0)
    return {"fp64": 1e-10 * col, "fp32": 1e-5 * col, "bf16x2": 1e-4 * col}[prec]


@pytest.mark.parametrize("name,prec,M,lam", [
    ("n500_p10_rwm_fp64", "fp64", 300, 0.5), ("n5000_p200_mala_bf16", "fp64", 64, 0.05), ("n5000_p200_mala_bf16", "bf16x2", 256, 0.05),
    ("n2000_p50_rwm_fp32", "fp32", 200, 2.0), ("n2000_p50_rwm_fp32", "bf16x2", 200, 1e-2),
])
def test_grad_parity(name, prec, M, lam):
    torch = _torch()
    s, cfg, X, y, Xs = _sampler(name, prec)
    b = particles(M, X.shape[1], seed=7 * M)
    for dt in (torch.float64, torch.float32):
        bt = torch.from_numpy(b).to("cuda", dt)
        bs = bt.double().cpu().numpy()
        g, lp = s.grad(bt, lam, prec)
        g = g.double().cpu().numpy()
        ll_ref, gl_ref = likelihood.loglik_and_grad(bs, Xs, y)
        g_ref = gl_ref + gt_prior.gt_grad(bs, cfg.a, lam)
        lp_ref = ll_ref + gt_prior.log_prior(bs, cfg.a, lam)
        err = np.abs(g - g_ref)
        tol = _grad_tol(prec, Xs)
        if dt == torch.float32:   # the gradient itself is returned in FP32 (one rounding)
            tol = tol + 2.0 ** -24 * np.abs(g_ref)
        print(f"{name} {prec} {dt}: grad max abs err {err.max():.3e} (tol min {tol.min():.3e})")
        assert np.all(err <= tol)
        ltol = 1e-10 if prec == "fp64" else 1e-4
        assert rel_err(lp.cpu().numpy(), lp_ref).max() <= ltol


@pytest.mark.parametrize("n,p,xfmt,M", [(400, 300, "bf16", 130), (1000, 500, "fp8", 200), (2000, 383, "fp8", 64),
                                        (64, 511, "bf16", 70), (130, 450, "bf16", 257), (10000, 500, "fp8", 96)])
def test_grad_parity_wide_rows(n, p, xfmt, M):
    """Rows of 384 and 512 markers (the split-marker contraction: two waves per particle
    block, each with one half of the markers, the forward halves added through LDS), BF16
    and FP8 genotype storage, ragged individual and particle counts, one and several
    individual splits: log posterior and gradient against the oracle."""
    torch = _torch()
    s, cfg, X, y, Xs = _sampler("n10000_p500_mala_fp8", "bf16x2", n=n, p=p, xfmt=xfmt, move="mala")
    lam = 0.05
    b = particles(M, X.shape[1], seed=n + p)
    bt = torch.from_numpy(b).to("cuda", torch.float32)
    bs = bt.double().cpu().numpy()
    g, lp = s.grad(bt, lam)
    g = g.double().cpu().numpy()
    ll_ref, gl_ref = likelihood.loglik_and_grad(bs, Xs, y)
    g_ref = gl_ref + gt_prior.gt_grad(bs, cfg.a, lam)
    lp_ref = ll_ref + gt_prior.log_prior(bs, cfg.a, lam)
    tol = _grad_tol("bf16x2", Xs) + 2.0 ** -24 * np.abs(g_ref)
    err = np.abs(g - g_ref)
    print(f"n={n} p={p} {xfmt}: grad max abs err {err.max():.3e}, lp max rel err "
          f"{rel_err(lp.cpu().numpy(), lp_ref).max():.3e}")
    assert np.all(err <= tol)
    assert rel_err(lp.cpu().numpy(), lp_ref).max() <= 1e-4


@pytest.mark.parametrize("prec", ["fp64", "fp32", "bf16x2"])
def test_grad_parity_double_exponential(prec):
    """a = inf (the double-exponential prior, Section 2): prior gradient -sign(b)/lam and
    log prior -log(2 lam) - |b|/lam, with exact zeros in the coefficients (sign(0) = 0)."""
    torch = _torch()
    from paper_1106_0322_amd import SamplerConfig, SpaSMC
    cfg, X, y, Xs = dataset("n2000_p50_rwm_fp32")
    sc = SamplerConfig(n=X.shape[0], p=X.shape[1], N=64, a=math.inf, lambdas=np.geomspace(10, 1, 2),
                       move="mala", sweeps=0, init_sweeps=0, prec=prec, seed=0)
    s = SpaSMC(sc, X, y)
    b = particles(150, X.shape[1], seed=41)
    lam = 0.2
    dt = torch.float64 if prec == "fp64" else torch.float32
    bt = torch.from_numpy(b).to("cuda", dt)
    bs = bt.double().cpu().numpy()
    g, lp = s.grad(bt, lam, prec)
    ll_ref, gl_ref = likelihood.loglik_and_grad(bs, Xs, y)
    g_ref = gl_ref + gt_prior.gt_grad(bs, math.inf, lam)
    tol = _grad_tol(prec, Xs) + (2.0 ** -24 * np.abs(g_ref) if dt == torch.float32 else 0.0)
    err = np.abs(g.double().cpu().numpy() - g_ref)
    print(f"a=inf {prec}: grad max abs err {err.max():.3e}")
    assert np.all(err <= tol)
    lp_ref = ll_ref + gt_prior.log_prior(bs, math.inf, lam)
    assert rel_err(lp.cpu().numpy(), lp_ref).max() <= (1e-10 if prec == "fp64" else 1e-4)
    s.close()


@pytest.mark.parametrize("n,p,M", [(60, 100, 70), (66, 32, 3), (300, 255, 130), (1000, 200, 257)])
def test_grad_parity_edge_shapes_bf16(n, p, M):
    """The BF16 adjoint at one split (n <= 64), ragged tails, PP = 64, 224 and 256, and
    particle counts that leave partial workgroups."""
    torch = _torch()
    s, cfg, X, y, Xs = _sampler("n5000_p200_mala_bf16", "bf16x2", n=n, p=p)
    b = particles(M, p, seed=n + 3 * p)
    bt = torch.from_numpy(b).to("cuda", torch.float32)
    bs = bt.double().cpu().numpy()
    lam = 0.05
    g, lp = s.grad(bt, lam, "bf16x2")
    ll_ref, gl_ref = likelihood.loglik_and_grad(bs, Xs, y)
    g_ref = gl_ref + gt_prior.gt_grad(bs, cfg.a, lam)
    err = np.abs(g.double().cpu().numpy() - g_ref)
    tol = _grad_tol("bf16x2", Xs) + 2.0 ** -24 * np.abs(g_ref)
    print(f"n={n} p={p} M={M}: grad max abs err {err.max():.3e}")
    assert np.all(err <= tol)
    assert rel_err(lp.cpu().numpy(), ll_ref + gt_prior.log_prior(bs, cfg.a, lam)).max() <= 1e-4


def test_grad_central_differences_fp64():
    """The adjoint against central differences (h = 1e-6, FP64) on 64 particles of the
    n=5000, p=200 data, coefficients kept away from the prior's cusp."""
    torch = _torch()
    s, cfg, X, y, Xs = _sampler("n5000_p200_mala_bf16", "fp64")
    rng = np.random.default_rng(11)
    b = rng.normal(0, 0.1, size=(64, X.shape[1]))
    b = np.where(np.abs(b) < 1e-4, 1e-4, b)
    lam, h = 0.3, 1e-6
    bt = torch.from_numpy(b).cuda()
    g, lp = s.grad(bt, lam, "fp64")
    g = g.cpu().numpy()
    cols = rng.choice(X.shape[1], size=12, replace=False)
    for j in cols:
        e = torch.zeros_like(bt)
        e[:, j] = h
        up = s.grad(bt + e, lam, "fp64")[1].cpu().numpy()
        dn = s.grad(bt - e, lam, "fp64")[1].cpu().numpy()
        fd = (up - dn) / (2 * h)
        assert np.allclose(g[:, j], fd, rtol=1e-5, atol=1e-4), (j, np.abs(g[:, j] - fd).max())


def test_autograd_function_backward_is_the_adjoint():
    torch = _torch()
    from paper_1106_0322_amd import log_posterior
    s, cfg, X, y, Xs = _sampler("n500_p10_rwm_fp64", "fp64")
    b = torch.from_numpy(particles(50, X.shape[1], seed=5)).cuda().requires_grad_(True)
    lp = log_posterior(b, 0.7, s, "fp64")
    w = torch.linspace(0.5, 2.0, 50, dtype=torch.float64, device="cuda")
    (lp * w).sum().backward()
    bs = b.detach().cpu().numpy()
    g_ref = likelihood.grad_loglik(bs, Xs, y) + gt_prior.gt_grad(bs, cfg.a, 0.7)
    assert np.allclose(b.grad.cpu().numpy(), w.cpu().numpy()[:, None] * g_ref, rtol=1e-9, atol=1e-9)


# M spans one workgroup, ragged multi-workgroup ranges, and (M > 2^18) several weights per
# thread in the quantisation and scan passes
@pytest.mark.parametrize("M", [1, 2, 7, 64, 255, 257, 1000, 1024, 4097, 16384, 32768, 100000, 1000003])
def test_resample_bit_exact(M):
    torch = _torch()
    s, *_ = _sampler("n500_p10_rwm_fp64", "fp64")
    rng = np.random.default_rng(M)
    for trial in range(4):
        w = rng.exponential(size=M) ** (1 + 3 * trial)
        if trial == 2:
            w[rng.uniform(size=M) < 0.5] = 0.0
            w[M // 2] = 1.0
        if trial == 3:
            w = np.ones(M)
        u32 = int(rng.integers(0, 2 ** 32)) if trial != 3 else 0
        got = s.resample(torch.from_numpy(w), u32).cpu().numpy()
        ref = smc.systematic_resample(w, u32)
        assert np.array_equal(got, ref)
        if trial == 3:   # equal weights, U = 0: the identity map for every M
            assert np.array_equal(got, np.arange(M))


def test_resample_rejects_invalid_weights():
    torch = _torch()
    from paper_1106_0322_amd import SpaError
    s, *_ = _sampler("n500_p10_rwm_fp64", "fp64")
    for w in ([0.0, 0.0], [1.0, -1.0], [1.0, float("nan")], [float("inf"), 1.0]):
        with pytest.raises(SpaError) as ei:
            s.resample(torch.tensor(w, dtype=torch.float64), 0)
        assert ei.value.status == 6
