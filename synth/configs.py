"""The five workload configurations of the sparsity-path sampler, plus the scale grid.

Sizes and distributions follow the workloads named for this hot path: individuals n
(balanced cases/controls), markers p, latent AR(1) linkage disequilibrium with
correlation rho (optionally restarted in blocks), a handful of causal markers, N
particles, T scales on a geometric grid from 1e3 down to 1e-2, a generalized-t prior
with ``a`` degrees of freedom, and S move sweeps per scale.  The paper's own runs
(Section 4.1) used n=500, p=50, N=8192 and b_t = 2 * 0.98^(t-1); those shapes are
available as ``paper_small`` / ``paper_large`` for context runs.
"""
from __future__ import annotations

import dataclasses
import math
from typing import Optional

import numpy as np


@dataclasses.dataclass(frozen=True)
class WorkloadConfig:
    name: str
    n: int                 # individuals (cases + controls, balanced)
    p: int                 # markers
    rho: float             # AR(1) latent correlation between adjacent markers
    block: int             # restart the latent chain every `block` markers (0 = one chain)
    k_causal: int          # number of markers with a non-zero effect
    beta_sd: float         # effect sizes ~ N(0, beta_sd^2)
    N: int                 # particles
    T: int                 # number of prior scales
    a: float               # generalized-t degrees of freedom (math.inf = double exponential)
    move: str              # "rwm" or "mala"
    sweeps: int            # joint proposals per particle per scale
    init_sweeps: int       # burn-in sweeps targeting the first scale
    prec: str              # GEMM precision: "fp64", "fp32", "bf16x2", or "fp8x3" / "fp8x4" (RWM)
    xfmt: str = "auto"     # genotype storage for bf16x2: "auto", "bf16" or "fp8"
    ess_frac: float = 0.5  # resample iff ESS < ess_frac * N
    seed: int = 0          # Philox key of the sampler
    data_seed: int = 0     # NumPy seed of the genotype/label generator
    lam_hi: float = 1e3
    lam_lo: float = 1e-2
    lambdas: Optional[tuple] = None   # explicit scale grid (overrides the geometric one)

    def grid(self) -> np.ndarray:
        if self.lambdas is not None:
            return np.asarray(self.lambdas, dtype=np.float64)
        return lambda_grid(self.lam_hi, self.lam_lo, self.T)

    def step0(self) -> float:
        """Initial proposal scale: 2.38/sqrt(p) for the random walk, 1.65^2/p^(1/3) for MALA
        (optimal-scaling constants of Roberts, Gelman & Gilks 1997 and Roberts & Rosenthal 1998);
        0.5 for the single-coordinate kernel (the proposal variance 0.25 of Section 4.1)."""
        if self.move == "rwm":
            return 2.38 / math.sqrt(self.p)
        if self.move == "single":
            return 0.5                      # single-coordinate random walk, variance 0.25
        return 1.65 ** 2 / self.p ** (1.0 / 3.0)

    def replace(self, **kw) -> "WorkloadConfig":
        return dataclasses.replace(self, **kw)


def lambda_grid(hi: float, lo: float, T: int) -> np.ndarray:
    """Inclusive geometric grid hi -> lo with T points (strictly decreasing)."""
    if T == 1:
        return np.array([hi], dtype=np.float64)
    t = np.arange(T, dtype=np.float64)
    return hi * (lo / hi) ** (t / (T - 1))


CONFIGS = {
    "n500_p10_rwm_fp64": WorkloadConfig("n500_p10_rwm_fp64", n=500, p=10, rho=0.90, block=0, k_causal=2, beta_sd=0.5,
                           N=1024, T=20, a=1.0, move="rwm", sweeps=5, init_sweeps=200,
                           prec="fp64", seed=0, data_seed=0),
    "n2000_p50_rwm_fp32": WorkloadConfig("n2000_p50_rwm_fp32", n=2000, p=50, rho=0.95, block=0, k_causal=3, beta_sd=0.3,
                           N=8192, T=100, a=0.5, move="rwm", sweeps=10, init_sweeps=200,
                           prec="fp32", seed=1, data_seed=1),
    "n2000_p50_rwm_fp8": WorkloadConfig("n2000_p50_rwm_fp8", n=2000, p=50, rho=0.95, block=0, k_causal=3, beta_sd=0.3,
                           N=8192, T=100, a=0.5, move="rwm", sweeps=10, init_sweeps=200,
                           prec="bf16x2", xfmt="fp8", seed=1, data_seed=1),
    "n5000_p200_mala_bf16": WorkloadConfig("n5000_p200_mala_bf16", n=5000, p=200, rho=0.97, block=20, k_causal=5, beta_sd=0.2,
                           N=16384, T=100, a=1.0, move="mala", sweeps=10, init_sweeps=500,
                           prec="bf16x2", xfmt="bf16", seed=3, data_seed=3),
    "n10000_p500_mala_fp8": WorkloadConfig("n10000_p500_mala_fp8", n=10000, p=500, rho=0.97, block=25, k_causal=8, beta_sd=0.2,
                           N=32768, T=200, a=0.5, move="mala", sweeps=10, init_sweeps=500,
                           prec="bf16x2", xfmt="fp8", seed=4, data_seed=4),
    # plain FP32 random-walk SMC on the n=5000, p=200 data (the comparison form)
    "n5000_p200_rwm_fp32": WorkloadConfig("n5000_p200_rwm_fp32", n=5000, p=200, rho=0.97, block=20, k_causal=5,
                                 beta_sd=0.2, N=16384, T=100, a=1.0, move="rwm", sweeps=10,
                                 init_sweeps=500, prec="fp32", seed=3, data_seed=3),
    # the paper's own shapes and kernel (Section 4.1: 5 cycles of single-coordinate random-walk
    # updates per scale): context runs on synthetic LD genotypes
    "paper_small": WorkloadConfig("paper_small", n=500, p=50, rho=0.95, block=0, k_causal=5,
                                  beta_sd=math.sqrt(0.2), N=8192, T=450, a=1.0, move="single",
                                  sweeps=5, init_sweeps=200, prec="fp32", ess_frac=0.75,
                                  seed=5, data_seed=5,
                                  lambdas=tuple(2.0 * 0.98 ** np.arange(450))),
    "paper_large": WorkloadConfig("paper_large", n=1859, p=184, rho=0.95, block=0, k_causal=5,
                                  beta_sd=math.sqrt(0.2), N=8192, T=250, a=4.0, move="single",
                                  sweeps=5, init_sweeps=200, prec="fp32", ess_frac=0.75,
                                  seed=6, data_seed=6,
                                  # the paper indexes on b = a*c; the sampler's scale is c = b/a
                                  lambdas=tuple(0.98 ** np.arange(250) / 4.0)),
}


def get_config(name: str, **overrides) -> WorkloadConfig:
    cfg = CONFIGS[name]
    return cfg.replace(**overrides) if overrides else cfg
