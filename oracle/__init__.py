"""Plain FP64 CPU oracle for the sparsity-path SMC sampler -- TEST INFRASTRUCTURE.

This package is the checker, not the product.  Only the test-suite, the smoke check
and the benchmark's CPU-baseline leg may import it; the HIP library never routes
through it and it shares no code with the HIP path (the only common dependency is
the seeded input generator in ``synth``).

Every function is written from the paper's definitions in FP64 NumPy (SciPy only for
quadrature and special functions), without blocking, fusion or reordering beyond the
definition it cites:

* ``gt_prior``   -- the centred L1 generalized-t density Gt(a, c) (Section 2, eq. of the
                    general generalized-t and its q=1, mu=0 form), its CDF, inverse CDF,
                    gradient, the double-exponential limit and the EM weight (Section 2.1).
* ``likelihood`` -- the logistic likelihood without intercept on column-standardised
                    genotypes (Section 2 and Section 3), its gradient.
* ``philox``     -- Philox4x32-10 (Salmon, Moraes, Dror & Shaw, SC'11) and the sampler's
                    stream layout (Box-Muller normals, MH uniforms, resampling offset).
* ``smc``        -- the SMC sampler indexed on the prior scale (Section 4 and 4.1):
                    prior-ratio incremental weights, normalisation, ESS, marginal-
                    likelihood ratios, systematic resampling, random-walk and MALA moves,
                    weighted moments and the scale-adaptation rule.
* ``quadrature`` -- brute-force posterior means and log marginal likelihoods for p = 1, 2.
* ``em``         -- MAP estimates by the EM algorithm of Section 2.1 (weighted-L1 logistic
                    inner problems by coordinate ascent) and the MAP path of Section 4.1.
* ``spa``        -- the sparsity-path summaries (Section 5): weighted quantiles (absolute
                    medians, credible intervals), concentrations, the posterior over the
                    scale and the c-marginal mixture (Section 4, eq. all_particles).

Parity status: every function here is pinned by the CPU tests (closed forms,
library special cases, invariants, brute force, published known-answer vectors).  The
sampler's posterior-mean and log-Z paths at p >= 10 have no closed form: there they are
parity unpinned beyond the pins of the same code at p = 1, 2 and prior-only targets, and
the GPU is compared with them statistically (replicate seeds), see the test-suite.
"""
from . import gt_prior, likelihood, philox, smc, quadrature, spa, em  # noqa: F401
