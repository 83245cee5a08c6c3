"""MI355X-native sparsity-path SMC sampler (generalized-t priors, logistic likelihood).

The computation lives in the HIP library ``libspa_smc.so`` (C ABI in include/spa_smc.h);
this package only builds it and marshals arguments to it.
"""
from .binding import (  # noqa: F401
    EXPORTS, SamplerConfig, SpaError, SpaSMC, SpaLogPost, load_library, log_posterior,
    LIB_PATH,
)
