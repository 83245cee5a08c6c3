"""CPU checks of the C-ABI library: it loads, exports every entry point the header
declares, and rejects invalid calls on the host before any device work."""
import ctypes
import os
import re

import numpy as np
import pytest

from paper_1106_0322_amd import binding

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "spa_smc.h")


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(binding.LIB_PATH):
        from paper_1106_0322_amd import build
        build.build()
    return binding.load_library()


def declared_functions():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"^\s*(?:spa_status|void|const char \*)\s*(\w+)\s*\(", src, flags=re.M)))


def test_header_declares_the_path_entry_points():
    names = declared_functions()
    for required in ("spa_smc_init", "spa_smc_step", "spa_smc_loglik", "spa_smc_grad",
                     "spa_smc_resample"):
        assert required in names
    assert sorted(binding.EXPORTS) == names


def test_binding_precision_names_match_the_header_enum():
    src = open(HEADER).read()
    enum = dict((m.group(1).lower(), int(m.group(2)))
                for m in re.finditer(r"SPA_PREC_(\w+)\s*=\s*(\d+)", src))
    assert enum == binding.PREC


def test_library_exports_every_declared_symbol(lib):
    for name in declared_functions():
        assert hasattr(lib, name), name


def _cfg(lam, **kw):
    base = dict(n=10, p=3, N=8, a=1.0, T=len(lam),
                lam=lam.ctypes.data_as(ctypes.POINTER(ctypes.c_double)), move=0, sweeps=1,
                init_sweeps=0, ess_frac=0.5, step0=1.0, adapt=1, prec=0, xfmt=0, seed=0)
    base.update(kw)
    return binding._Config(**base)


def _init(lib, cfg, X, y):
    h = ctypes.c_void_p()
    st = lib.spa_smc_init(ctypes.byref(cfg) if cfg is not None else None,
                          X.ctypes.data_as(ctypes.c_void_p) if X is not None else None,
                          y.ctypes.data_as(ctypes.c_void_p) if y is not None else None,
                          None, ctypes.byref(h))
    return st, h, lib.spa_smc_last_error(None).decode()


def _good_data(n=10, p=3):
    X = (np.arange(n * p).reshape(n, p) % 3).astype(np.uint8)
    y = (np.arange(n) % 2).astype(np.uint8)
    return X, y


CASES = [
    ("null config", None, binding.SPA_ERR_ARG),
    ("increasing scales", dict(lam=[1.0, 2.0]), binding.SPA_ERR_ARG),
    ("equal scales", dict(lam=[1.0, 1.0]), binding.SPA_ERR_ARG),
    ("negative scale", dict(lam=[1.0, -1.0]), binding.SPA_ERR_ARG),
    ("a <= 0", dict(a=0.0), binding.SPA_ERR_ARG),
    ("N = 0", dict(N=0), binding.SPA_ERR_SHAPE),
    ("p too large", dict(p=512), binding.SPA_ERR_SHAPE),
    ("fp64 with p = 300", dict(p=300, prec=0), binding.SPA_ERR_SHAPE),
    ("ess_frac = 0", dict(ess_frac=0.0), binding.SPA_ERR_ARG),
    ("ess_frac > 1", dict(ess_frac=1.5), binding.SPA_ERR_ARG),
    ("bad move", dict(move=7), binding.SPA_ERR_ARG),
    ("bad prec", dict(prec=9), binding.SPA_ERR_ARG),
    ("FP8 3-term prec with MALA (no adjoint)", dict(prec=3, move=1), binding.SPA_ERR_ARG),
    ("FP8 4-term prec with single-coordinate moves", dict(prec=4, move=2), binding.SPA_ERR_ARG),
    ("negative sweeps", dict(sweeps=-1), binding.SPA_ERR_ARG),
    ("step0 = 0", dict(step0=0.0), binding.SPA_ERR_ARG),
]


@pytest.mark.parametrize("name,over,code", CASES, ids=[c[0] for c in CASES])
def test_invalid_configurations_rejected_on_host(lib, name, over, code):
    X, y = _good_data()
    if over is None:
        st, h, msg = _init(lib, None, X, y)
    else:
        over = dict(over)
        lam = np.array(over.pop("lam", [2.0, 1.0]), dtype=np.float64)
        p = over.get("p", 3)
        X, y = _good_data(p=p)
        st, h, msg = _init(lib, _cfg(lam, **over), X, y)
    assert st == code, (st, msg)
    assert msg
    assert not h.value


def test_invalid_data_rejected_on_host(lib):
    lam = np.array([2.0, 1.0])
    X, y = _good_data()
    Xb = X.copy(); Xb[0, 0] = 3
    assert _init(lib, _cfg(lam), Xb, y)[0] == binding.SPA_ERR_ARG
    yb = y.copy(); yb[1] = 2
    assert _init(lib, _cfg(lam), X, yb)[0] == binding.SPA_ERR_ARG
    Xc = X.copy(); Xc[:, 1] = 1
    st, _, msg = _init(lib, _cfg(lam), Xc, y)
    assert st == binding.SPA_ERR_SHAPE and "zero variance" in msg
    assert _init(lib, _cfg(lam), None, y)[0] == binding.SPA_ERR_ARG


def test_null_handle_calls(lib):
    assert lib.spa_smc_step(None, None) == binding.SPA_ERR_ARG
    assert lib.spa_smc_loglik(None, None, 1, 0, 0, None) == binding.SPA_ERR_ARG
    assert lib.spa_smc_loglik_noalloc(None, None, 1, 0, 0, None) == binding.SPA_ERR_ARG
    assert lib.spa_smc_grad(None, None, 1, 0, 1.0, 0, None, None) == binding.SPA_ERR_ARG
    assert lib.spa_smc_resample(None, None, 1, 0, None) == binding.SPA_ERR_ARG
    assert lib.spa_smc_set_state(None, None, None, 1, 1.0) == binding.SPA_ERR_ARG
    assert lib.spa_philox4x32_10(None, None, 1, 0, None) == binding.SPA_ERR_ARG
    assert lib.spa_weighted_summaries(None, None, 1, 1, 0, None, None, 0, None, 0, None, None) == binding.SPA_ERR_ARG
    assert lib.spa_smc_set_summaries(None, None, 0, None, 0, 0) == binding.SPA_ERR_ARG
    assert lib.spa_smc_get_summaries(None, None, None) == binding.SPA_ERR_ARG
    assert lib.spa_smc_marginal_summaries(None, None, None, None) == binding.SPA_ERR_ARG
    assert lib.spa_map_em(None, None, 1, 0, 1.0, 1, 1, None, None) == binding.SPA_ERR_ARG
    assert lib.spa_smc_set_map(None, 1, 1) == binding.SPA_ERR_ARG
    assert lib.spa_smc_get_map(None, None, None) == binding.SPA_ERR_ARG
    assert lib.spa_smc_get_loglik(None, None) == binding.SPA_ERR_ARG
    assert lib.spa_smc_set_timing(None, 1) == binding.SPA_ERR_ARG
    assert lib.spa_smc_set_timing_classes(None, 2) == binding.SPA_ERR_ARG
    lib.spa_smc_destroy(None)


def test_product_path_has_no_cpu_fallback():
    """The binding never imports the oracle and refuses to run without a GPU."""
    src = open(os.path.join(ROOT, "paper_1106_0322_amd", "binding.py")).read()
    assert "oracle" not in src
    import torch
    if not torch.cuda.is_available():
        with pytest.raises(RuntimeError):
            binding._torch()
