"""GPU parity of the EM MAP estimates (Section 2.1) and the MAP path (Section 4.1) against
the FP64 oracle.  Both sides run the same iteration (E step, then fixed coordinate-ascent
sweeps in marker order) in FP64; they differ only in summation order, so the modes agree
to round-off."""
import math

import numpy as np
import pytest

from oracle import em, smc
from tests.gpu_util import dataset, particles

pytestmark = pytest.mark.gpu


def _torch():
    import torch
    return torch


def _handle(name, n=None, p=None, **over):
    from paper_1106_0322_amd import SamplerConfig, SpaSMC
    cfg, X, y, Xs = dataset(name, n, p)
    sc = SamplerConfig.from_workload(cfg, n=X.shape[0], p=X.shape[1], **over)
    return SpaSMC(sc, X, y), cfg, X, y, Xs


@pytest.mark.parametrize("name,n,p,M,a,lam,outer,inner", [
    ("n500_p10_rwm_fp64", None, None, 7, 1.0, 0.05, 30, 5),
    ("n500_p10_rwm_fp64", None, None, 5, math.inf, 0.02, 10, 20),
    ("n2000_p50_rwm_fp32", None, None, 6, 0.5, 0.1, 20, 4),
    ("n5000_p200_mala_bf16", 130, 150, 3, 4.0, 0.01, 10, 3),
    ("n5000_p200_mala_bf16", None, None, 2, 1.0, 0.02, 3, 2),
])
def test_map_em_matches_oracle(name, n, p, M, a, lam, outer, inner):
    torch = _torch()
    s, cfg, X, y, Xs = _handle(name, n, p, N=64, lambdas=np.geomspace(10.0, 1.0, 3), init_sweeps=0, sweeps=0,
                               a=a)
    b0 = particles(M, X.shape[1], seed=M + X.shape[1], scale=0.3)
    for dt in (torch.float64, torch.float32):
        bt = torch.from_numpy(b0).to("cuda", dt)
        print(f"map_em {name} n={X.shape[0]} p={X.shape[1]} a={a} dtype={dt}", flush=True)
        mode, lp = s.map_em(bt, lam, outer, inner)
        ref, lref = em.map_em(Xs, y.astype(np.float64), bt.double().cpu().numpy(), a, lam, outer, inner)
        d = np.abs(mode.cpu().numpy() - ref).max()
        dl = np.abs(lp.cpu().numpy() - lref).max() / np.abs(lref).max()
        print(f"  max |d mode| {d:.3e}, rel d logpost {dl:.3e}")
        assert d <= 1e-9 and dl <= 1e-12
        # exact zeros agree: the soft-threshold sets the same coordinates to zero
        assert np.array_equal(mode.cpu().numpy() == 0.0, ref == 0.0)


def test_map_path_fp64_tracks_oracle():
    # enough iterations that the two EM runs of a scale, when they climb to the same mode,
    # agree far below the tolerance (their choice is then a tie decided by round-off)
    T, outer, inner = 8, 40, 10
    s, cfg, X, y, Xs = _handle("n500_p10_rwm_fp64")
    r = smc.run_config(cfg, X, y, T_stop=T, snapshot_at=tuple(range(1, T + 1)))
    s.set_map(outer, inner)
    for _ in range(T - 1):
        s.step()
    mp, mlp = s.map_path()
    prev = None
    worst = 0.0
    for t in range(1, T + 1):
        snap = r.snapshots[t]
        m, v = em.map_step(Xs, y.astype(np.float64), snap.beta, snap.ll, cfg.a, cfg.grid()[t - 1], prev,
                           outer, inner)
        worst = max(worst, np.abs(mp[t - 1] - m).max())
        assert math.isclose(mlp[t - 1], v, rel_tol=1e-12, abs_tol=1e-9), (t, mlp[t - 1], v)
        prev = m
    print(f"MAP path max |diff| {worst:.3e}")
    assert worst <= 1e-9


def test_map_rejects_bad_arguments():
    torch = _torch()
    from paper_1106_0322_amd import SpaError
    s, *_ = _handle("n500_p10_rwm_fp64", N=64, lambdas=np.geomspace(10.0, 1.0, 3), init_sweeps=0, sweeps=0)
    b = torch.zeros(2, 10, dtype=torch.float64, device="cuda")
    for lam, outer in ((0.0, 1), (-1.0, 1), (1.0, -1)):
        with pytest.raises(SpaError) as ei:
            s.map_em(b, lam, outer, 1)
        assert ei.value.status == 1
