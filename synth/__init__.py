"""Seeded synthetic inputs shared by the HIP path, the oracle and the benchmarks.

This package holds none of the sampler's arithmetic: it only draws genotype
matrices and case-control labels (host-side NumPy stream, independent of the
sampler's Philox stream) and describes the five workload configurations.
"""
from .configs import CONFIGS, WorkloadConfig, lambda_grid, get_config  # noqa: F401
from .genotypes import make_dataset, Dataset  # noqa: F401
