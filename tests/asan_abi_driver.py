"""Drives the host-side validation paths of the C ABI in the host-AddressSanitizer build of
the library (run by tests/test_abi_asan.py in a child process with the sanitizer runtime
preloaded; no GPU and no torch).  Every call here is rejected on the host before device
work; the sanitizer reports any out-of-bounds or use-after-free access on the way."""
import ctypes
import os
import sys

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)
from paper_1106_0322_amd.binding import _Config  # noqa: E402  (ctypes structure only)

lib = ctypes.CDLL(sys.argv[1])
vp, i32, dbl = ctypes.c_void_p, ctypes.c_int32, ctypes.c_double
lib.spa_smc_init.argtypes = [ctypes.POINTER(_Config), vp, vp, vp, ctypes.POINTER(vp)]
lib.spa_smc_last_error.argtypes = [vp]
lib.spa_smc_last_error.restype = ctypes.c_char_p
lib.spa_smc_destroy.argtypes = [vp]
lib.spa_smc_destroy.restype = None


def cfg(lam, **kw):
    base = dict(n=10, p=3, N=8, a=1.0, T=len(lam), lam=lam.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
                move=0, sweeps=1, init_sweeps=0, ess_frac=0.5, step0=1.0, adapt=1, prec=0, xfmt=0, seed=0)
    base.update(kw)
    return _Config(**base)


def init(c, X, y):
    h = ctypes.c_void_p()
    st = lib.spa_smc_init(ctypes.byref(c) if c is not None else None,
                          X.ctypes.data_as(vp) if X is not None else None,
                          y.ctypes.data_as(vp) if y is not None else None, None, ctypes.byref(h))
    msg = lib.spa_smc_last_error(None).decode()
    assert not h.value and st != 0 and msg, (st, msg)
    return st


def data(n=10, p=3):
    return (np.arange(n * p).reshape(n, p) % 3).astype(np.uint8), (np.arange(n) % 2).astype(np.uint8)


count = 0
for n, p in ((10, 3), (64, 40), (300, 511)):
    X, y = data(n, p)
    lam = np.array([2.0, 1.0])
    for over in (dict(a=0.0), dict(N=0), dict(p=512), dict(ess_frac=0.0), dict(move=7), dict(prec=9),
                 dict(prec=3, move=1), dict(sweeps=-1), dict(step0=0.0), dict(p=300, prec=0)):
        Xo, yo = data(n, over.get("p", p)) if "p" in over else (X, y)
        init(cfg(lam, n=n, p=over.get("p", p), **{k: v for k, v in over.items() if k != "p"}), Xo, yo)
        count += 1
    for bad in (np.array([1.0, 2.0]), np.array([1.0, 1.0]), np.array([1.0, -1.0]), np.array([np.nan, 1.0])):
        init(cfg(bad, n=n, p=p), X, y)
        count += 1
    Xb = X.copy(); Xb[-1, -1] = 3
    init(cfg(lam, n=n, p=p), Xb, y)
    yb = y.copy(); yb[-1] = 2
    init(cfg(lam, n=n, p=p), X, yb)
    Xc = X.copy(); Xc[:, -1] = 1
    init(cfg(lam, n=n, p=p), Xc, y)
    init(None, X, y)
    init(cfg(lam, n=n, p=p), None, y)
    count += 5
# null-handle calls of every entry point
calls = [("spa_smc_step", (None, None)), ("spa_smc_loglik", (None, None, 1, 0, 0, None)),
         ("spa_smc_loglik_noalloc", (None, None, 1, 0, 0, None)),
         ("spa_smc_grad", (None, None, 1, 0, dbl(1.0), 0, None, None)),
         ("spa_smc_resample", (None, None, 1, 0, None)), ("spa_smc_set_state", (None, None, None, 1, dbl(1.0))),
         ("spa_philox4x32_10", (None, None, 1, ctypes.c_uint64(0), None)),
         ("spa_smc_set_timing", (None, 1)), ("spa_smc_get_loglik", (None, None)),
         ("spa_map_em", (None, None, 1, 0, dbl(1.0), 1, 1, None, None)), ("spa_smc_set_map", (None, 1, 1))]
for name, args in calls:
    assert getattr(lib, name)(*args) != 0, name
    count += 1
lib.spa_smc_destroy(None)
print(f"asan driver: {count} rejected calls, no sanitizer report")
