"""GPU parity of the sparsity-path summaries (Section 5) against the FP64 oracle.

* spa_weighted_summaries on given values and weights: quantiles and concentrations are
  bit-exact (the weights are quantised to integers on both sides, so the order statistic
  chosen does not depend on summation order);
* per-scale summaries recorded by the sampler and the c-marginal mixture of the FP64
  path (which tracks the oracle's trajectory to round-off): equal to the oracle's
  summaries of its own snapshots, to round-off of the particle values."""
import math

import numpy as np
import pytest

from oracle import smc, spa
from tests.gpu_util import dataset, particles

pytestmark = pytest.mark.gpu

LEVELS = [0.05, 0.5, 0.95]
DELTAS = [0.05, 0.1]


def _torch():
    import torch
    return torch


def _handle(name="n500_p10_rwm_fp64", **over):
    from paper_1106_0322_amd import SamplerConfig, SpaSMC
    cfg, X, y, Xs = dataset(name)
    sc = SamplerConfig.from_workload(cfg, n=X.shape[0], p=X.shape[1], **over)
    return SpaSMC(sc, X, y), cfg, X, y


def _weights(rng, M, kind):
    if kind == "equal":
        return np.ones(M)
    w = rng.exponential(size=M) ** (1 + 3 * (kind == "skewed"))
    if kind == "sparse":
        w[rng.uniform(size=M) < 0.6] = 0.0
        w[rng.integers(0, M)] = 1.0
    return w


@pytest.mark.parametrize("M,p,f64", [
    (1, 1, True), (7, 3, False), (1000, 5, True), (4097, 33, False), (4097, 33, True),
    (16384, 200, False), (9000, 64, True),
])
@pytest.mark.parametrize("kind", ["equal", "skewed", "sparse"])
def test_weighted_summaries_bit_exact(M, p, f64, kind):
    torch = _torch()
    s, *_ = _handle(N=64, lambdas=np.geomspace(10.0, 1.0, 3), init_sweeps=0, sweeps=0)
    rng = np.random.default_rng(M * 7 + p)
    v = particles(M, p, seed=M + p)
    if kind == "sparse":
        v = np.round(v, 2)                       # many ties, exact zeros
    if not f64:
        v = v.astype(np.float32)
    w = _weights(rng, M, kind)
    levels = LEVELS + [1.0, float(rng.uniform(0.01, 0.99))]
    print(f"summaries M={M} p={p} f64={f64} kind={kind}", flush=True)
    q, c = s.weighted_summaries(torch.from_numpy(v).cuda(), torch.from_numpy(w), levels, DELTAS)
    q_ref = spa.weighted_quantiles(v.astype(np.float64), w, levels)
    c_ref = spa.concentration(v.astype(np.float64), w, DELTAS)
    assert np.array_equal(q.cpu().numpy(), q_ref)
    assert np.array_equal(c.cpu().numpy(), c_ref)


def test_weighted_summaries_edge_values_and_errors():
    torch = _torch()
    from paper_1106_0322_amd import SpaError
    s, *_ = _handle(N=64, lambdas=np.geomspace(10.0, 1.0, 3), init_sweeps=0, sweeps=0)
    # signed zeros, equal values, extreme magnitudes
    v = np.array([[-0.0], [0.0], [1e-300], [-1e-300], [1e300], [-1e300], [5.0], [5.0]])
    w = np.array([1.0, 2.0, 1.0, 1.0, 0.5, 0.5, 3.0, 0.0])
    levels = [1e-300, 0.1, 0.25, 0.5, 0.75, 1.0]
    q, c = s.weighted_summaries(torch.from_numpy(v).cuda(), torch.from_numpy(w), levels, [1e-300, 1.0])
    assert np.array_equal(q.cpu().numpy(), spa.weighted_quantiles(v, w, levels))
    assert np.array_equal(c.cpu().numpy(), spa.concentration(v, w, [1e-300, 1.0]))
    for bad in ([0.0, 0.0], [1.0, -1.0], [1.0, float("nan")], [float("inf"), 1.0]):
        with pytest.raises(SpaError) as ei:
            s.weighted_summaries(torch.zeros(2, 1, dtype=torch.float64).cuda(),
                                 torch.tensor(bad, dtype=torch.float64), LEVELS, DELTAS)
        assert ei.value.status == 6
    for lv in ([0.0], [1.5], [0.5] * 9):
        with pytest.raises(SpaError) as ei:
            s.weighted_summaries(torch.zeros(2, 1).cuda(), torch.ones(2), lv, DELTAS)
        assert ei.value.status == 1


def test_sampler_summaries_and_marginal_fp64_track_oracle():
    """n500_p10_rwm_fp64 FP64 for 10 scales: the per-scale summaries and the c-marginal mixture equal
    the oracle's summaries of its own particle snapshots."""
    cfg, X, y, Xs = dataset("n500_p10_rwm_fp64")
    T = 10
    r = smc.run_config(cfg, X, y, T_stop=T, snapshot_at=tuple(range(1, T + 1)))
    s, *_ = _handle()
    s.set_summaries(LEVELS, DELTAS, keep_history=True)
    for _ in range(T - 1):
        s.step()
    q, c = s.summaries()
    assert q.shape == (T, len(LEVELS), X.shape[1]) and c.shape == (T, len(DELTAS), X.shape[1])
    qm, cm, sp = s.marginal_summaries()
    worst_q = worst_c = 0.0
    for t in range(1, T + 1):
        snap = r.snapshots[t]
        W = np.exp(snap.logW)
        qr = spa.weighted_quantiles(snap.beta, W, LEVELS)
        cr = spa.concentration(snap.beta, W, DELTAS)
        worst_q = max(worst_q, np.abs(q[t - 1] - qr).max())
        worst_c = max(worst_c, np.abs(c[t - 1] - cr).max())
    print(f"per-scale summaries: max |dq| {worst_q:.3e}, max |dV| {worst_c:.3e}")
    assert worst_q <= 1e-10 and worst_c <= 1e-12
    beta_path = np.stack([r.snapshots[t].beta for t in range(1, T + 1)])
    logW_path = np.stack([r.snapshots[t].logW for t in range(1, T + 1)])
    qmr, cmr = spa.marginal_summaries(beta_path, logW_path, r.log_z, LEVELS, DELTAS)
    print(f"marginal: max |dq| {np.abs(qm - qmr).max():.3e}, max |dV| {np.abs(cm - cmr).max():.3e}")
    assert np.abs(qm - qmr).max() <= 1e-10 and np.abs(cm - cmr).max() <= 1e-12
    assert np.allclose(sp, spa.scale_posterior(r.log_z), rtol=1e-10, atol=1e-300)
    assert math.isclose(sp.sum(), 1.0, rel_tol=1e-12)


def test_sampler_summaries_full_size_bf16():
    """n=5000, p=200, N=16384 MALA (one scale step).
    * The summaries of the GPU's own particles under given linear weights W equal the
      oracle's summaries of the same values and weights bit for bit (both sides quantise
      W / max W by one correctly rounded division).
    * The per-scale record exponentiates the log weights on the device, so each W may
      differ from the host's exp by an ulp or two.  That moves each quantised weight
      floor((W / max W) 2^K) by at most 1 (K = 49 at M = 16384), so the quantised CDF
      moves by at most M / C <= M 2^-K = 2^-35 anywhere.  Each recorded quantile must
      then lie between the oracle's quantiles at the levels alpha -/+ 2^-30, and each
      recorded concentration within 1e-12 of the oracle's."""
    torch = _torch()
    s, cfg, X, y = _handle("n5000_p200_mala_bf16", init_sweeps=20)
    s.set_summaries(LEVELS, DELTAS)
    s.step()
    q, c = s.summaries()
    beta, logw = s.particles()
    b = beta.double().cpu().numpy()
    lw = logw.cpu().numpy()
    W = np.exp(lw - lw.max())
    qr = spa.weighted_quantiles(b, W, LEVELS)
    cr = spa.concentration(b, W, DELTAS)
    # bit-exact on the same linear weights
    qg, cg = s.weighted_summaries(beta, torch.from_numpy(W), LEVELS, DELTAS)
    assert np.array_equal(qg.cpu().numpy(), qr) and np.array_equal(cg.cpu().numpy(), cr)
    # the recorded summaries: within a 2^-30 perturbation of the level
    eps = 2.0 ** -30
    lo = spa.weighted_quantiles(b, W, [max(a - eps, 2.0 ** -60) for a in LEVELS])
    hi = spa.weighted_quantiles(b, W, [min(a + eps, 1.0) for a in LEVELS])
    rec = q[-1]
    within = (rec >= np.minimum(lo, hi)) & (rec <= np.maximum(lo, hi))
    print(f"n5000_p200_mala_bf16 summaries: {np.mean(rec != qr):.4f} of recorded quantiles differ from the "
          f"host-weight ones, all within the level band: {bool(within.all())}; "
          f"max |dV| {np.abs(c[-1] - cr).max():.3e}")
    assert within.all()
    assert np.abs(c[-1] - cr).max() <= 1e-12
