"""Synthetic linkage-disequilibrium genotypes and retrospective case-control labels.

Stands in for the paper's private genotype data (Section 3: a high-LD hit region
with block-like correlation, a few causal loci with GWAS-sized effects and binary
phenotypes drawn from a logistic model).  Recipe:

1. minor-allele frequencies MAF_j ~ U(0.05, 0.5) and thresholds tau_j = Phi^-1(1 - MAF_j);
2. per individual, two haplotypes of an AR(1) latent Gaussian chain
   Z_j = rho * Z_{j-1} + sqrt(1 - rho^2) * eps_j (restarted at each block start);
   allele = [Z_j > tau_j], genotype = sum of the two alleles (exact Binomial(2, MAF_j)
   marginals, values 0/1/2);
3. k causal markers chosen without replacement, effects ~ N(0, beta_sd^2);
4. P(case) = logistic(x_pop . beta) with the Hardy-Weinberg standardisation
   x_pop = (g - 2 MAF) / sqrt(2 MAF (1 - MAF)) and no intercept (Section 2, Section 3);
5. individuals are drawn in sequence and admitted to the case or the control group
   until each holds n/2 (retrospective case-control sampling);
6. a sample with a monomorphic column is redrawn from the next sub-seed.

The NumPy generator here is the host input stream; it is independent of the
sampler's counter-based Philox stream.
"""
from __future__ import annotations

import dataclasses

import numpy as np
from scipy.special import ndtri

from .configs import WorkloadConfig


@dataclasses.dataclass
class Dataset:
    X: np.ndarray          # (n, p) uint8 in {0, 1, 2}, row-major (individual-major)
    y: np.ndarray          # (n,) uint8 in {0, 1}
    maf: np.ndarray        # (p,) float64
    causal: np.ndarray     # (k,) int64 marker indices
    beta_true: np.ndarray  # (p,) float64


def _haplotypes(rng: np.random.Generator, m: int, tau: np.ndarray, rho: float,
                block: int) -> np.ndarray:
    """m haplotypes over p markers: thresholded AR(1) latent chains (uint8 alleles)."""
    p = tau.shape[0]
    out = np.empty((m, p), dtype=np.uint8)
    innov = np.sqrt(1.0 - rho * rho)
    z = rng.standard_normal(m)
    out[:, 0] = z > tau[0]
    for j in range(1, p):
        e = rng.standard_normal(m)
        if block and j % block == 0:
            z = e
        else:
            z = rho * z + innov * e
        out[:, j] = z > tau[j]
    return out


def make_dataset(cfg: WorkloadConfig, n: int | None = None, p: int | None = None,
                 seed: int | None = None) -> Dataset:
    n = cfg.n if n is None else n
    p = cfg.p if p is None else p
    seed = cfg.data_seed if seed is None else seed
    if n < 2 or n % 2:
        raise ValueError("n must be even and >= 2 (balanced cases/controls)")
    k = min(cfg.k_causal, p)
    for attempt in range(64):
        rng = np.random.default_rng([seed, attempt])
        maf = rng.uniform(0.05, 0.5, size=p)
        tau = ndtri(1.0 - maf)
        causal = np.sort(rng.choice(p, size=k, replace=False))
        beta = np.zeros(p)
        beta[causal] = rng.normal(0.0, cfg.beta_sd, size=k)
        mu_pop = 2.0 * maf
        sd_pop = np.sqrt(2.0 * maf * (1.0 - maf))
        half = n // 2
        cases, controls = [], []
        n_case = n_ctrl = 0
        while n_case < half or n_ctrl < half:
            m = max(256, n)
            g = (_haplotypes(rng, m, tau, cfg.rho, cfg.block)
                 + _haplotypes(rng, m, tau, cfg.rho, cfg.block))
            eta = ((g - mu_pop) / sd_pop) @ beta
            prob = 1.0 / (1.0 + np.exp(-eta))
            lab = rng.uniform(size=m) < prob
            for i in range(m):
                if lab[i] and n_case < half:
                    cases.append(g[i]); n_case += 1
                elif not lab[i] and n_ctrl < half:
                    controls.append(g[i]); n_ctrl += 1
                if n_case >= half and n_ctrl >= half:
                    break
        X = np.concatenate([np.stack(cases), np.stack(controls)]).astype(np.uint8)
        y = np.concatenate([np.ones(half, np.uint8), np.zeros(half, np.uint8)])
        # interleave cases and controls deterministically so that tiles see both labels
        perm = rng.permutation(n)
        X, y = np.ascontiguousarray(X[perm]), np.ascontiguousarray(y[perm])
        if np.all(X.max(axis=0) > X.min(axis=0)):
            return Dataset(X=X, y=y, maf=maf, causal=causal, beta_true=beta)
    raise RuntimeError("could not draw a sample without monomorphic markers")
