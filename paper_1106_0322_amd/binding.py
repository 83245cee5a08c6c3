"""ctypes binding of libspa_smc.so (argument marshalling only).

Every computation runs in the HIP library; PyTorch provides device memory (tensors whose
``data_ptr`` is passed through) and the HIP stream (``torch.cuda.current_stream()``).
There is no CPU fallback: if the library is not built, or no GPU is present, the calls
raise.
"""
from __future__ import annotations

import ctypes
import math
import os
from dataclasses import dataclass
from typing import Optional

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libspa_smc.so")

SPA_OK, SPA_ERR_ARG, SPA_ERR_SHAPE, SPA_ERR_ALLOC, SPA_ERR_HIP, SPA_ERR_STATE, SPA_ERR_NUMERIC = range(7)
STATUS_NAMES = ["SPA_OK", "SPA_ERR_ARG", "SPA_ERR_SHAPE", "SPA_ERR_ALLOC", "SPA_ERR_HIP",
                "SPA_ERR_STATE", "SPA_ERR_NUMERIC"]
PREC = {"fp64": 0, "fp32": 1, "bf16x2": 2, "fp8x3": 3, "fp8x4": 4}
XFMT = {"auto": 0, "fp8": 1, "bf16": 2}
MOVE = {"rwm": 0, "mala": 1, "single": 2}

# The exported C entry points (kept in step with include/spa_smc.h).
EXPORTS = ["spa_smc_init", "spa_smc_step", "spa_smc_loglik", "spa_smc_loglik_noalloc", "spa_smc_grad",
           "spa_smc_resample",
           "spa_weighted_summaries", "spa_smc_set_summaries", "spa_smc_get_summaries",
           "spa_smc_marginal_summaries", "spa_map_em", "spa_smc_set_map", "spa_smc_get_map",
           "spa_smc_get", "spa_smc_get_loglik", "spa_smc_get_stats", "spa_smc_set_state",
           "spa_philox4x32_10",
           "spa_smc_set_timing", "spa_smc_set_timing_classes", "spa_smc_get_timing", "spa_smc_destroy",
           "spa_smc_last_error"]
TIMING_CLASSES = ["propose", "loglik", "accept", "reweight", "lse_resample", "gather", "moments",
                  "finalize", "summary", "map"]


class SpaError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"{STATUS_NAMES[status] if 0 <= status < 7 else status}: {msg}")
        self.status = status


class _Config(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int32), ("p", ctypes.c_int32), ("N", ctypes.c_int32),
                ("a", ctypes.c_double), ("T", ctypes.c_int32),
                ("lam", ctypes.POINTER(ctypes.c_double)), ("move", ctypes.c_int),
                ("sweeps", ctypes.c_int32), ("init_sweeps", ctypes.c_int32),
                ("ess_frac", ctypes.c_double), ("step0", ctypes.c_double),
                ("adapt", ctypes.c_int32), ("prec", ctypes.c_int), ("xfmt", ctypes.c_int),
                ("seed", ctypes.c_uint64)]


class _Stats(ctypes.Structure):
    _fields_ = [("t", ctypes.c_int32), ("resampled", ctypes.c_int32), ("lam", ctypes.c_double),
                ("ess", ctypes.c_double), ("log_z_inc", ctypes.c_double),
                ("log_z", ctypes.c_double), ("accept_rate", ctypes.c_double),
                ("step", ctypes.c_double)]

    def as_dict(self):
        return {"t": self.t, "resampled": bool(self.resampled), "lambda": self.lam,
                "ess": self.ess, "log_z_inc": self.log_z_inc, "log_z": self.log_z,
                "accept_rate": self.accept_rate, "step": self.step}


_lib = None


def load_library(path: str = LIB_PATH) -> ctypes.CDLL:
    """Load libspa_smc.so and declare the signatures; raises if it is not built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise RuntimeError(f"{path} is not built; run `python -m paper_1106_0322_amd.build`")
    # torch first: its HIP runtime (soname libamdhip64.so.7) is then the one the library binds to
    import torch  # noqa: F401
    lib = ctypes.CDLL(path)
    vp, i32, dbl = ctypes.c_void_p, ctypes.c_int32, ctypes.c_double
    lib.spa_smc_init.argtypes = [ctypes.POINTER(_Config), vp, vp, vp, ctypes.POINTER(vp)]
    lib.spa_smc_step.argtypes = [vp, ctypes.POINTER(_Stats)]
    lib.spa_smc_loglik.argtypes = [vp, vp, i32, i32, ctypes.c_int, vp]
    lib.spa_smc_loglik_noalloc.argtypes = [vp, vp, i32, i32, ctypes.c_int, vp]
    lib.spa_smc_grad.argtypes = [vp, vp, i32, i32, dbl, ctypes.c_int, vp, vp]
    lib.spa_smc_resample.argtypes = [vp, vp, i32, ctypes.c_uint32, vp]
    dptr = ctypes.POINTER(ctypes.c_double)
    lib.spa_weighted_summaries.argtypes = [vp, vp, i32, i32, i32, vp, dptr, i32, dptr, i32, vp, vp]
    lib.spa_smc_set_summaries.argtypes = [vp, dptr, i32, dptr, i32, i32]
    lib.spa_smc_get_summaries.argtypes = [vp, ctypes.POINTER(vp), ctypes.POINTER(vp)]
    lib.spa_smc_marginal_summaries.argtypes = [vp, vp, vp, vp]
    lib.spa_smc_get.argtypes = [vp, ctypes.POINTER(vp), ctypes.POINTER(vp), ctypes.POINTER(vp),
                                ctypes.POINTER(vp), ctypes.POINTER(vp), ctypes.POINTER(i32)]
    lib.spa_smc_get_loglik.argtypes = [vp, ctypes.POINTER(vp)]
    lib.spa_map_em.argtypes = [vp, vp, i32, i32, dbl, i32, i32, vp, vp]
    lib.spa_smc_set_map.argtypes = [vp, i32, i32]
    lib.spa_smc_get_map.argtypes = [vp, ctypes.POINTER(vp), ctypes.POINTER(vp)]
    lib.spa_smc_get_stats.argtypes = [vp, i32, ctypes.POINTER(_Stats)]
    lib.spa_smc_set_state.argtypes = [vp, vp, vp, i32, dbl]
    lib.spa_philox4x32_10.argtypes = [vp, vp, i32, ctypes.c_uint64, vp]
    lib.spa_smc_set_timing.argtypes = [vp, i32]
    lib.spa_smc_set_timing_classes.argtypes = [vp, ctypes.c_uint32]
    lib.spa_smc_get_timing.argtypes = [vp, vp, vp]
    lib.spa_smc_destroy.argtypes = [vp]
    lib.spa_smc_destroy.restype = None
    lib.spa_smc_last_error.argtypes = [vp]
    lib.spa_smc_last_error.restype = ctypes.c_char_p
    for name in EXPORTS:
        if name not in ("spa_smc_destroy", "spa_smc_last_error"):
            getattr(lib, name).restype = ctypes.c_int
    _lib = lib
    return lib


def _torch():
    import torch
    if not torch.cuda.is_available():
        raise RuntimeError("the HIP sampler needs a GPU (torch.cuda.is_available() is False)")
    return torch


def _ptr(t) -> ctypes.c_void_p:
    return ctypes.c_void_p(t.data_ptr())


@dataclass
class SamplerConfig:
    """Sampler configuration mirroring spa_smc_config."""
    n: int
    p: int
    N: int
    a: float
    lambdas: np.ndarray
    move: str = "rwm"
    sweeps: int = 5
    init_sweeps: int = 200
    ess_frac: float = 0.5
    step0: float = 1.0
    adapt: bool = True
    prec: str = "fp64"
    xfmt: str = "auto"
    seed: int = 0

    @classmethod
    def from_workload(cls, w, **over) -> "SamplerConfig":
        kw = dict(n=w.n, p=w.p, N=w.N, a=w.a, lambdas=w.grid(), move=w.move, sweeps=w.sweeps,
                  init_sweeps=w.init_sweeps, ess_frac=w.ess_frac, step0=w.step0(),
                  prec=w.prec, xfmt=w.xfmt, seed=w.seed)
        kw.update(over)
        return cls(**kw)


class SpaSMC:
    """One sampler handle (spa_smc_init .. spa_smc_destroy)."""

    def __init__(self, cfg: SamplerConfig, X: np.ndarray, y: np.ndarray, stream=None):
        torch = _torch()
        self.lib = load_library()
        self.cfg = cfg
        X = np.ascontiguousarray(X, dtype=np.uint8)
        y = np.ascontiguousarray(y, dtype=np.uint8)
        if X.shape != (cfg.n, cfg.p) or y.shape != (cfg.n,):
            raise SpaError(SPA_ERR_SHAPE, f"X {X.shape} / y {y.shape} do not match n={cfg.n}, p={cfg.p}")
        self._lam = np.ascontiguousarray(cfg.lambdas, dtype=np.float64)
        c = _Config(n=cfg.n, p=cfg.p, N=cfg.N, a=float(cfg.a), T=len(self._lam),
                    lam=self._lam.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
                    move=MOVE[cfg.move], sweeps=cfg.sweeps, init_sweeps=cfg.init_sweeps,
                    ess_frac=cfg.ess_frac, step0=cfg.step0, adapt=int(bool(cfg.adapt)),
                    prec=PREC[cfg.prec], xfmt=XFMT[cfg.xfmt], seed=int(cfg.seed) & (2 ** 64 - 1))
        self.stream = stream if stream is not None else torch.cuda.current_stream()
        self.device = self.stream.device
        h = ctypes.c_void_p()
        st = self.lib.spa_smc_init(ctypes.byref(c), X.ctypes.data_as(ctypes.c_void_p),
                                   y.ctypes.data_as(ctypes.c_void_p),
                                   ctypes.c_void_p(self.stream.cuda_stream), ctypes.byref(h))
        if st != SPA_OK:
            raise SpaError(st, self.lib.spa_smc_last_error(None).decode())
        self.h = h
        self.particle_dtype = torch.float64 if cfg.prec == "fp64" else torch.float32

    # -------------------------------------------------------------- helpers
    def _check(self, st):
        if st != SPA_OK:
            raise SpaError(st, self.lib.spa_smc_last_error(self.h).decode())

    def close(self):
        if getattr(self, "h", None) is not None and self.h.value:
            self.lib.spa_smc_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    # -------------------------------------------------------------- sampler
    def step(self) -> dict:
        s = _Stats()
        self._check(self.lib.spa_smc_step(self.h, ctypes.byref(s)))
        return s.as_dict()

    def run(self) -> list:
        out = [self.stats(1)]
        while self.t < len(self._lam):
            out.append(self.step())
        return out

    def stats(self, t: int) -> dict:
        s = _Stats()
        self._check(self.lib.spa_smc_get_stats(self.h, t, ctypes.byref(s)))
        return s.as_dict()

    def _get(self):
        vp = ctypes.c_void_p
        b, lw, mp, vpth, lz = vp(), vp(), vp(), vp(), vp()
        t = ctypes.c_int32()
        self._check(self.lib.spa_smc_get(self.h, ctypes.byref(b), ctypes.byref(lw), ctypes.byref(mp),
                                         ctypes.byref(vpth), ctypes.byref(lz), ctypes.byref(t)))
        return b, lw, mp, vpth, lz, t.value

    @property
    def t(self) -> int:
        return self._get()[5]

    def _copy_dev(self, ptr, numel, dtype):
        """Copy a library-owned device array into a new torch tensor (device-to-device)."""
        torch = _torch()
        out = torch.empty(numel, dtype=dtype, device=self.device)
        nbytes = numel * out.element_size()
        hip = _hip_runtime()
        with torch.cuda.stream(self.stream):
            st = hip.hipMemcpyAsync(ctypes.c_void_p(out.data_ptr()), ptr, ctypes.c_size_t(nbytes),
                                    ctypes.c_int(3), ctypes.c_void_p(self.stream.cuda_stream))
        if st != 0:
            raise SpaError(SPA_ERR_HIP, f"hipMemcpyAsync failed ({st})")
        return out

    def particles(self):
        """(beta N x p, normalised log weights N) as new device tensors."""
        torch = _torch()
        b, lw, _, _, _, _ = self._get()
        beta = self._copy_dev(b, self.cfg.N * self.cfg.p, self.particle_dtype).view(self.cfg.N, self.cfg.p)
        logw = self._copy_dev(lw, self.cfg.N, torch.float64)
        return beta, logw

    def state_loglik(self):
        """Log-likelihoods of the current particles (N,) as a new device tensor."""
        torch = _torch()
        ll = ctypes.c_void_p()
        self._check(self.lib.spa_smc_get_loglik(self.h, ctypes.byref(ll)))
        return self._copy_dev(ll, self.cfg.N, torch.float64)

    def paths(self):
        """Per-scale weighted mean and variance (t x p) and cumulative log Z (t,), on the host."""
        torch = _torch()
        _, _, mp, vpth, lz, t = self._get()
        T, p = len(self._lam), self.cfg.p
        mean = self._copy_dev(mp, T * p, torch.float64).view(T, p)
        var = self._copy_dev(vpth, T * p, torch.float64).view(T, p)
        self.stream.synchronize()
        logz = np.ctypeslib.as_array(ctypes.cast(lz, ctypes.POINTER(ctypes.c_double)), shape=(T,)).copy()
        return mean[:t].cpu().numpy(), var[:t].cpu().numpy(), logz[:t]

    def set_state(self, beta, logw, t: int, step: float):
        torch = _torch()
        beta = beta.to(device=self.device, dtype=self.particle_dtype).contiguous()
        logw = logw.to(device=self.device, dtype=torch.float64).contiguous()
        self._check(self.lib.spa_smc_set_state(self.h, _ptr(beta), _ptr(logw), int(t), float(step)))

    # -------------------------------------------------------------- path entry points
    def loglik(self, beta, prec: Optional[str] = None):
        torch = _torch()
        beta = beta.to(self.device).contiguous()
        assert beta.dim() == 2 and beta.shape[1] == self.cfg.p
        out = torch.empty(beta.shape[0], dtype=torch.float64, device=self.device)
        self._check(self.lib.spa_smc_loglik(self.h, _ptr(beta), beta.shape[0],
                                            int(beta.dtype == torch.float64),
                                            PREC[prec or self.cfg.prec], _ptr(out)))
        return out

    def loglik_noalloc(self, beta, out, prec: Optional[str] = None):
        """spa_smc_loglik_noalloc into the caller's `out` (M doubles on the device): the
        library allocates nothing (its scratch is a static device array per GPU)."""
        torch = _torch()
        assert beta.is_cuda and beta.is_contiguous() and beta.dim() == 2 and beta.shape[1] == self.cfg.p
        assert out.is_cuda and out.is_contiguous() and out.dtype == torch.float64 and out.numel() >= beta.shape[0]
        self._check(self.lib.spa_smc_loglik_noalloc(self.h, _ptr(beta), beta.shape[0],
                                                    int(beta.dtype == torch.float64),
                                                    PREC[prec or self.cfg.prec], _ptr(out)))
        return out

    def grad(self, beta, lam: float, prec: Optional[str] = None, want_logpost: bool = True):
        torch = _torch()
        beta = beta.to(self.device).contiguous()
        assert beta.dim() == 2 and beta.shape[1] == self.cfg.p
        assert beta.dtype in (torch.float32, torch.float64)
        g = torch.empty_like(beta)
        lp = torch.empty(beta.shape[0], dtype=torch.float64, device=self.device) if want_logpost else None
        self._check(self.lib.spa_smc_grad(self.h, _ptr(beta), beta.shape[0],
                                          int(beta.dtype == torch.float64), float(lam),
                                          PREC[prec or self.cfg.prec], _ptr(g),
                                          _ptr(lp) if lp is not None else None))
        return g, lp

    def resample(self, w, u32: int):
        torch = _torch()
        w = w.to(device=self.device, dtype=torch.float64).contiguous()
        anc = torch.empty(w.shape[0], dtype=torch.int32, device=self.device)
        self._check(self.lib.spa_smc_resample(self.h, _ptr(w), w.shape[0], ctypes.c_uint32(u32), _ptr(anc)))
        return anc

    # ------------------------------------------------------ sparsity-path summaries
    @staticmethod
    def _dbl_array(v):
        v = [float(x) for x in v]
        return (ctypes.c_double * max(1, len(v)))(*v), len(v)

    def weighted_summaries(self, values, w, levels=(0.05, 0.5, 0.95), deltas=(0.05, 0.1)):
        """Weighted quantiles (len(levels) x p) and concentrations (len(deltas) x p) of
        every column of values (M x p, FP32 or FP64) under weights w (M)."""
        torch = _torch()
        values = values.to(self.device).contiguous()
        if values.dim() == 1:
            values = values[:, None]
        assert values.dtype in (torch.float32, torch.float64)
        w = w.to(device=self.device, dtype=torch.float64).contiguous()
        M, p = values.shape
        la, L = self._dbl_array(levels)
        da, D = self._dbl_array(deltas)
        q = torch.empty((L, p), dtype=torch.float64, device=self.device)
        c = torch.empty((D, p), dtype=torch.float64, device=self.device)
        self._check(self.lib.spa_weighted_summaries(self.h, _ptr(values), M, p, int(values.dtype == torch.float64),
                                                    _ptr(w), la, L, da, D, _ptr(q) if L else None,
                                                    _ptr(c) if D else None))
        return q, c

    def set_summaries(self, levels=(0.05, 0.5, 0.95), deltas=(0.05, 0.1), keep_history: bool = False):
        la, L = self._dbl_array(levels)
        da, D = self._dbl_array(deltas)
        self._levels, self._deltas = list(levels), list(deltas)
        self._check(self.lib.spa_smc_set_summaries(self.h, la, L, da, D, int(bool(keep_history))))

    def summaries(self):
        """Per-scale quantile (t x L x p) and concentration (t x D x p) paths, on the host."""
        torch = _torch()
        qp, cp = ctypes.c_void_p(), ctypes.c_void_p()
        self._check(self.lib.spa_smc_get_summaries(self.h, ctypes.byref(qp), ctypes.byref(cp)))
        _, _, _, _, _, t = self._get()
        T, p = len(self._lam), self.cfg.p
        L, D = len(self._levels), len(self._deltas)
        q = self._copy_dev(qp, T * L * p, torch.float64).view(T, L, p) if L else None
        c = self._copy_dev(cp, T * D * p, torch.float64).view(T, D, p) if D else None
        self.stream.synchronize()
        return (q[:t].cpu().numpy() if L else None), (c[:t].cpu().numpy() if D else None)

    def marginal_summaries(self):
        """Quantiles (L x p) and concentrations (D x p) of the c-marginal mixture over the
        scales run so far, and the posterior over those scales (t,)."""
        torch = _torch()
        _, _, _, _, _, t = self._get()
        p, L, D = self.cfg.p, len(self._levels), len(self._deltas)
        q = torch.empty((L, p), dtype=torch.float64, device=self.device)
        c = torch.empty((D, p), dtype=torch.float64, device=self.device)
        sp = torch.empty(t, dtype=torch.float64, device=self.device)
        self._check(self.lib.spa_smc_marginal_summaries(self.h, _ptr(q) if L else None, _ptr(c) if D else None,
                                                        _ptr(sp)))
        return q.cpu().numpy(), c.cpu().numpy(), sp.cpu().numpy()

    # ---------------------------------------------------------------- MAP estimates
    def map_em(self, beta0, lam: float, outer: int = 50, inner: int = 5):
        """EM modes (M x p, FP64) and their log posterior densities from start points beta0."""
        torch = _torch()
        beta0 = beta0.to(self.device).contiguous()
        if beta0.dim() == 1:
            beta0 = beta0[None, :]
        assert beta0.dtype in (torch.float32, torch.float64) and beta0.shape[1] == self.cfg.p
        mode = torch.empty(beta0.shape, dtype=torch.float64, device=self.device)
        lp = torch.empty(beta0.shape[0], dtype=torch.float64, device=self.device)
        self._check(self.lib.spa_map_em(self.h, _ptr(beta0), beta0.shape[0], int(beta0.dtype == torch.float64),
                                        float(lam), int(outer), int(inner), _ptr(mode), _ptr(lp)))
        return mode, lp

    def set_map(self, outer: int = 50, inner: int = 5):
        self._check(self.lib.spa_smc_set_map(self.h, int(outer), int(inner)))

    def map_path(self):
        """MAP path (t x p) and its log posterior densities (t,), on the host."""
        torch = _torch()
        mp, lp = ctypes.c_void_p(), ctypes.c_void_p()
        self._check(self.lib.spa_smc_get_map(self.h, ctypes.byref(mp), ctypes.byref(lp)))
        _, _, _, _, _, t = self._get()
        T, p = len(self._lam), self.cfg.p
        m = self._copy_dev(mp, T * p, torch.float64).view(T, p)
        v = self._copy_dev(lp, T, torch.float64)
        self.stream.synchronize()
        return m[:t].cpu().numpy(), v[:t].cpu().numpy()

    def set_timing(self, enable: bool = True, classes=None):
        """Bracket launches with HIP events: every class, or only the named ones
        (names from TIMING_CLASSES); set_timing(False) turns timing off."""
        if classes is None:
            self._check(self.lib.spa_smc_set_timing(self.h, int(bool(enable))))
            return
        mask = 0
        for c in classes:
            if c not in TIMING_CLASSES:
                raise ValueError(f"unknown timing class {c!r}")
            mask |= 1 << TIMING_CLASSES.index(c)
        self._check(self.lib.spa_smc_set_timing_classes(self.h, mask if enable else 0))

    def timing(self) -> dict:
        """{class: (total ms, launches)} accumulated since set_timing(True)."""
        k = len(TIMING_CLASSES)
        ms = (ctypes.c_double * k)()
        cnt = (ctypes.c_int64 * k)()
        self._check(self.lib.spa_smc_get_timing(self.h, ms, cnt))
        return {name: (ms[i], cnt[i]) for i, name in enumerate(TIMING_CLASSES)}

    def philox(self, ctr, seed: int):
        torch = _torch()
        ctr = ctr.to(device=self.device, dtype=torch.int32).contiguous()
        out = torch.empty_like(ctr)
        self._check(self.lib.spa_philox4x32_10(self.h, _ptr(ctr), ctr.numel() // 4,
                                               ctypes.c_uint64(seed & (2 ** 64 - 1)), _ptr(out)))
        return out


_hip = None


def _hip_runtime():
    """libamdhip64 for the device-to-device copies of library-owned buffers."""
    global _hip
    if _hip is None:
        import torch  # noqa: F401  (the runtime torch loaded, matched by soname)
        for name in ("libamdhip64.so.7",):
            try:
                _hip = ctypes.CDLL(name)
                break
            except OSError:
                continue
        if _hip is None:
            raise RuntimeError("libamdhip64.so not found")
        _hip.hipMemcpyAsync.argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_size_t, ctypes.c_int,
                                        ctypes.c_void_p]
        _hip.hipMemcpyAsync.restype = ctypes.c_int
    return _hip


def _make_logpost_function():
    import torch

    class SpaLogPost(torch.autograd.Function):
        """log p(beta | X, y, lambda) up to Z: log-likelihood + sum_j log Gt(beta_j | a, lambda).

        Forward runs spa_smc_grad (contraction + adjoint); backward scales the saved gradient
        by the incoming per-particle gradient."""

        @staticmethod
        def forward(ctx, beta, lam, sampler, prec=None):
            g, lp = sampler.grad(beta.detach(), float(lam), prec)
            ctx.save_for_backward(g)
            return lp

        @staticmethod
        def backward(ctx, grad_out):
            (g,) = ctx.saved_tensors
            return grad_out.to(g.dtype)[:, None] * g, None, None, None

    return SpaLogPost


_SpaLogPost = None


def SpaLogPost():
    """The torch.autograd.Function class (created on first use so that importing the
    binding does not import torch)."""
    global _SpaLogPost
    if _SpaLogPost is None:
        _SpaLogPost = _make_logpost_function()
    return _SpaLogPost


def log_posterior(beta, lam: float, sampler: SpaSMC, prec: Optional[str] = None):
    """Differentiable log posterior of each particle (rows of beta)."""
    return SpaLogPost().apply(beta, lam, sampler, prec)
