"""Benchmark of the sparsity-path SMC hot path on one MI355X.

One "step" is one pass of the whole hot path at one prior scale: prior-ratio reweight,
logsumexp/ESS, (systematic resampling), S move sweeps (proposal -> MFMA log-likelihood
contraction (+ adjoint for MALA) -> MH decisions) and weighted moments, over the N
particles of the workload.  The workload is the n=5000 / p=200 / N=16384 MALA run with
BF16 hi+lo contractions (LD blocks of 20, a = 1, 100 scales, 10 sweeps per scale).

    python bench.py [--steps K] [--warmup W] [--workload n5000_p200_mala_bf16] [--no-cpu]

Prints one JSON line.  `value` is whole-job algorithmic contraction throughput
(2 N n p flops per log-likelihood evaluation plus 2 N n p per gradient evaluation)
over the K timed steps, inputs resident in HBM.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

PEAK = {"bf16x2": 2500.0, "fp32": 157.3, "fp64": 78.6}     # dense MFMA TFLOP/s of MI355X
PEAK_FP8 = 5000.0                                            # dense FP8 MFMA TFLOP/s of MI355X
HBM_PEAK_GBS = 8000.0
KERNEL_SOURCES = ["paper_1106_0322_amd/csrc/spa_gemm.hip", "paper_1106_0322_amd/csrc/spa_common.hpp",
                  "paper_1106_0322_amd/csrc/spa_internal.hpp"]
BREAKDOWN_STEPS = 2       # untimed steps after the timed ones, every kernel class bracketed
TRAFFIC_PROFILE = {"n5000_p200_mala_bf16": "profiles/loglik_kernel_n5000_p200_N16384_mala_bf16x2_traffic.txt"}
MFMA_PROFILE = {"n5000_p200_mala_bf16": "profiles/loglik_kernel_n5000_p200_N16384_mala_bf16x2_mfma.txt"}


def profile_values(table: dict, workload: str):
    """key=value lines of a committed counter summary for this workload, or None when there
    is none or the contraction kernel's sources have changed since it was taken."""
    import hashlib
    path = table.get(workload)
    if path is None or not os.path.exists(os.path.join(ROOT, path)):
        return None
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        with open(os.path.join(ROOT, f), "rb") as fh:
            h.update(fh.read())
    kv = {}
    for line in open(os.path.join(ROOT, path)):
        if "=" in line and not line.startswith("#"):
            k, v = line.strip().split("=", 1)
            kv[k] = v
    if kv.get("kernel_source_sha256_16") != h.hexdigest()[:16]:
        return None
    return kv


def profiled_traffic(workload: str):
    """HBM bytes per launch of the contraction kernel from the committed FETCH_SIZE /
    WRITE_SIZE summary (copy-calibrated), or None (no summary, or stale)."""
    kv = profile_values(TRAFFIC_PROFILE, workload)
    return None if kv is None else int(kv["hbm_bytes_per_launch"])


def copy_calibration():
    """A plain device copy of known size: 64 Mi float32 (256 MiB read, 256 MiB written),
    three times.  Its FETCH_SIZE / WRITE_SIZE readings scale the contraction's counters."""
    import torch
    n = 64 * 1024 * 1024
    x = torch.ones(n, device="cuda")
    y = torch.empty_like(x)
    for _ in range(3):
        y.copy_(x)
    torch.cuda.synchronize()
    print(f"copied 3 x {n * 4} bytes", flush=True)


# The single-coordinate kernel's roofline is taken on the method's own work per
# eta-element update (particle i, coordinate j, individual k), not on the kernel's
# instructions: the update eta' = eta + delta x (one FMA), the new e^-|eta'| (one
# exponential, a quarter-rate instruction: four lane-slots), its factor in the
# likelihood-ratio product (one multiply-add) and the linear term y delta x (one
# multiply-add): 3 + 4 = 7 VALU lane-slots.  The chip's VALU lane-slot rate is
# 256 CUs x 4 SIMDs x 16 lanes x 2.4 GHz (the 157.3 TFLOP/s FP32 vector peak counts an FMA
# as two flops and packed FP32 as two lanes).  For comparison the FP32 kernel itself issues
# 50 VALU + 10 transcendental instructions per coordinate update of 8 individuals per lane
# on the path without acceptance (its ISA: the update loop minus the acceptance block; the
# transcendentals are the 8 exponentials and the reciprocal and logarithm of the likelihood
# ratio; the move, the prior difference and log u are formed once per coordinate and cycle
# by the lane holding the coordinate; an accepted move adds 9 vector instructions), about
# 11.3 lane-slots per element update; the ratio of the two is its overhead.
SINGLE_SITE_ALG_SLOTS = 3 + 4 * 1
SINGLE_SITE_SLOTS = (50 + 4 * 10) / 8.0
VALU_LANE_SLOTS_PER_S = 256 * 4 * 16 * 2.4e9


def single_site_leg(steps: int = 10):
    """The paper's kernel (Section 4.1) at the paper's small shape: n=500, p=50, N=8192,
    5 cycles of single-coordinate updates per scale, FP32.  Throughput in eta-element
    updates per second (5 N p n per scale)."""
    import torch
    from paper_1106_0322_amd import SamplerConfig, SpaSMC
    from synth import CONFIGS, make_dataset

    cfg = CONFIGS["paper_small"]
    d = make_dataset(cfg)
    s = SpaSMC(SamplerConfig.from_workload(cfg, init_sweeps=5), d.X, d.y)
    for _ in range(2):
        s.step()
    s.set_timing(True, classes=["propose"])    # the single-coordinate launches
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        s.step()
    torch.cuda.synchronize()
    el = (time.perf_counter() - t0) / steps
    ms_k, cnt = s.timing()["propose"]
    s.close()
    k_s = ms_k / max(cnt, 1) * 1e-3
    units = cfg.sweeps * cfg.N * cfg.p * cfg.n
    rate_k = units / k_s
    return {"workload": f"n={cfg.n} p={cfg.p} N={cfg.N} a={cfg.a} 5 single-coordinate cycles per scale, fp32",
            "ms_per_step": round(el * 1e3, 4), "kernel_ms_per_step": round(k_s * 1e3, 4),
            "eta_updates_per_s": round(units / el, 1), "kernel_eta_updates_per_s": round(rate_k, 1),
            "est_full_run_s_T450": round(el * (cfg.T - 1), 2),
            "roofline": {"bound": "alu", "achieved": round(rate_k * SINGLE_SITE_ALG_SLOTS / 1e12, 3),
                         "peak": round(VALU_LANE_SLOTS_PER_S / 1e12, 3), "unit": "T VALU lane-slots/s",
                         "frac": round(rate_k * SINGLE_SITE_ALG_SLOTS / VALU_LANE_SLOTS_PER_S, 4),
                         "slots_per_update": SINGLE_SITE_ALG_SLOTS,
                         "kernel_slots_per_update": round(SINGLE_SITE_SLOTS, 2),
                         "issue_frac": round(rate_k * SINGLE_SITE_SLOTS / VALU_LANE_SLOTS_PER_S, 4)}}


def analysis_legs(torch, s, cfg):
    """Timings of the sparsity-path analysis on the bench workload's live particles:
    per-scale summaries (3 quantile levels, 2 tolerances) and one MAP-path scale (EM from
    two start points, 50 E steps x 5 coordinate sweeps)."""
    beta, logw = s.particles()
    w = torch.exp(logw - logw.max())
    s.weighted_summaries(beta, w)                 # warm-up (allocates its scratch)
    torch.cuda.synchronize()
    K = 5
    t0 = time.perf_counter()
    for _ in range(K):
        s.weighted_summaries(beta, w)
    torch.cuda.synchronize()
    t_sum = (time.perf_counter() - t0) / K
    starts = beta[:2].double()
    s.map_em(starts, float(cfg.grid()[min(10, cfg.T - 1)]), 1, 1)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    s.map_em(starts, float(cfg.grid()[min(10, cfg.T - 1)]), 50, 5)
    torch.cuda.synchronize()
    t_map = time.perf_counter() - t0
    vbytes = cfg.N * cfg.p * beta.element_size()
    return {"summaries": {"ms": round(t_sum * 1e3, 3), "values_GBps": round(vbytes / t_sum / 1e9, 1),
                          "what": f"quantiles (0.05, 0.5, 0.95) and V(0.05), V(0.1) of {cfg.p} coefficients "
                                  f"over N={cfg.N} weighted particles"},
            "map_em": {"ms": round(t_map * 1e3, 3),
                       "what": f"EM from 2 start points, 50 E steps x 5 coordinate sweeps, n={cfg.n} p={cfg.p}"}}


def precision_legs(torch, s, cfg, reps: int = 20):
    """The forward contraction (log-likelihood only) on the workload's live particles at
    each reduced precision: BF16 hi+lo MFMA against the FP8 MFMA with the coefficients in 3
    and 4 e4m3 terms.  Kernel time per call from the HIP events of the contraction and the
    split combination (the operand packing is not bracketed); the deviation is the largest
    relative difference from the FP64 contraction on the same particles."""
    beta, _ = s.particles()
    ref = s.loglik(beta.double(), "fp64").cpu().numpy() if cfg.p <= 255 else None
    flops = 2.0 * beta.shape[0] * cfg.n * cfg.p
    pp8 = -(-cfg.p // 128) * 128
    out = {"what": f"forward contraction, N={beta.shape[0]} live particles, n={cfg.n} p={cfg.p}"}
    for prec in ("bf16x2", "fp8x3", "fp8x4"):
        ll = s.loglik(beta, prec).cpu().numpy()
        s.set_timing(True, classes=["loglik", "finalize"])
        for _ in range(reps):
            s.loglik(beta, prec)
        t = s.timing()
        s.set_timing(False)
        k_s = (t["loglik"][0] + t["finalize"][0]) / reps * 1e-3
        rec = {"kernel_us": round(k_s * 1e6, 2),
               "algorithmic_TFLOPs": round(flops / k_s / 1e12, 2),
               "max_rel_dev_vs_fp64": None if ref is None else float(f"{np.max(np.abs(ll - ref) / np.abs(ref)):.3e}")}
        if prec.startswith("fp8x"):
            terms = int(prec[-1])
            n_pad = -(-cfg.n // 128) * 128
            executed = 2.0 * beta.shape[0] * n_pad * pp8 * terms
            rec["executed_TFLOPs"] = round(executed / k_s / 1e12, 2)
            rec["executed_frac_of_fp8_peak"] = round(executed / k_s / 1e12 / PEAK_FP8, 4)
        out[prec] = rec
    return out


def bandwidth_leg(cfg, X, y, reps: int = 10):
    """The weight, resampling and moment kernels at the workload's N and p, timed with HIP
    events per class: steps without moves from given states, alternately with spread
    log weights (ESS below the threshold: the resampling passes and the gather run) and
    with nearly equal ones (no resampling: the moment pass also normalises the weights).
    Rates are algorithmic bytes per launch over the class's average launch time (the
    reweighting pass and its one-workgroup combination count as one launch, and so do the
    quantisation, scan and search + gather passes; the moments are two launches per step,
    the partial sums and their ordered combination)."""
    import torch
    from paper_1106_0322_amd import SamplerConfig, SpaSMC

    N, p = cfg.N, cfg.p
    es = 8 if cfg.prec == "fp64" else 4
    g = SpaSMC(SamplerConfig.from_workload(cfg, sweeps=0, init_sweeps=0), X, y)
    rng = np.random.default_rng(0)
    beta = torch.from_numpy(np.clip(rng.normal(0, 0.1, size=(N, p)), -2, 2)).to(
        torch.float64 if es == 8 else torch.float32)
    states = []
    for k in range(2):
        lw = rng.normal(0, 2.0 if k == 0 else 0.05, size=N)
        lw -= np.log(np.exp(lw - lw.max()).sum()) + lw.max()
        states.append(torch.from_numpy(lw))
    g.set_timing(True, classes=["reweight", "lse_resample", "moments"])
    resampled = 0
    t0 = min(40, cfg.T - 1)
    for r in range(2 * reps):
        g.set_state(beta, states[r % 2], t0, 0.1)
        resampled += int(g.step()["resampled"])
    t = g.timing()
    g.close()
    mala = cfg.move == "mala"
    rows = N * p * es
    by = {"reweight": rows + 16 * N,                                  # beta, log w read + written
          "lse_resample": 2 * rows * (2 if mala else 1) + 8 * N * 6,  # rows (+ gradients) read and written;
                                                                      # log w, q/C written and read, ll moved
          "moments": rows + 16 * N}                                   # beta, log w (+ normalised write)
    out = {"what": f"N={N} p={p} {cfg.prec} particles, {2 * reps} steps without moves, {resampled} resampling"}
    for k, b in by.items():
        ms, n = t[k]
        if not n:
            continue
        us = ms / n * 1e3
        out[k] = {"us_per_launch": round(us, 2), "launches": n, "algorithmic_bytes": b,
                  "GBps": round(b / (us * 1e-6) / 1e9, 1), "frac_of_hbm": round(b / (us * 1e-6) / 1e9 / HBM_PEAK_GBS, 4)}
    return out


def gemm_flops(cfg) -> float:
    """Algorithmic flops of one sweep's contraction: loglik 2Nnp, + adjoint 2Nnp for MALA."""
    f = 2.0 * cfg.N * cfg.n * cfg.p
    return f * (2.0 if cfg.move == "mala" else 1.0)


def cpu_leg(workload: str, N: int = 1024, init_sweeps: int = 4, steps: int = 8) -> dict:
    """The oracle (FP64 NumPy, untuned) running the sampler itself on the workload's data:
    burn-in and the first scale steps of a whole SMC sweep at N particles, timed on this
    process's threads.  Returns the algorithmic contraction throughput (the GPU line's
    unit) and the full sweep's time extrapolated to the workload's particle count and
    sweep count (the cost is linear in both)."""
    from oracle import smc
    from synth import CONFIGS, make_dataset

    cfg = CONFIGS[workload]
    d = make_dataset(cfg)
    run = cfg.replace(N=N, init_sweeps=init_sweeps)
    t0 = time.perf_counter()
    smc.run_config(run, d.X, d.y, T_stop=steps + 1)
    el = time.perf_counter() - t0
    sweeps = init_sweeps + steps * cfg.sweeps
    flops = gemm_flops(run) * sweeps
    full_sweeps = cfg.init_sweeps + (cfg.T - 1) * cfg.sweeps
    return {"value": flops / el / 1e12, "seconds": round(el, 2), "sweeps": sweeps, "N": N,
            "full_sweep_s_extrapolated": round(el / sweeps * full_sweeps * cfg.N / N, 1)}


def cpu_baseline(cfg) -> dict:
    """The oracle timed on the host cores, all threads and one thread (BLAS and OpenMP
    pinned to 1 in a child process), each on a bounded sample of whole sweeps (about 10 s)."""
    import subprocess
    try:
        threads = len(os.sched_getaffinity(0))
    except AttributeError:
        threads = os.cpu_count()
    allc = cpu_leg(cfg.name)
    env = dict(os.environ, OMP_NUM_THREADS="1", OPENBLAS_NUM_THREADS="1", MKL_NUM_THREADS="1")
    r = subprocess.run([sys.executable, os.path.abspath(__file__), "--cpu-leg", cfg.name], env=env,
                       capture_output=True, text=True, timeout=600)
    one = json.loads(r.stdout.strip().splitlines()[-1]) if r.returncode == 0 else {"error": r.stderr[-400:]}
    sample = (f"oracle SMC on the {cfg.name} data (n={cfg.n}, p={cfg.p}, {cfg.move.upper()}): "
              f"{allc['sweeps']} whole sweeps (burn-in + first scale steps) of {allc['N']} particles, "
              f"FP64 NumPy, {allc['seconds']} s; throughput scaled per contraction flop")
    out = {"value": round(allc["value"], 5), "unit": "TFLOP/s", "cores": threads, "kind": "oracle",
           "sample": sample,
           "full_sweep_s_extrapolated": allc["full_sweep_s_extrapolated"],
           "single_thread": {"value": round(one["value"], 6) if "value" in one else None, "unit": "TFLOP/s",
                             "cores": 1, "seconds": one.get("seconds"),
                             "full_sweep_s_extrapolated": one.get("full_sweep_s_extrapolated"),
                             "error": one.get("error")}}
    try:
        out["cpu_model"] = next(l.split(":", 1)[1].strip() for l in open("/proc/cpuinfo") if l.startswith("model name"))
    except (OSError, StopIteration):
        pass
    return out


def full_sweep(cfg, X, y, seed, **over):
    """One full sweep over the scale grid (init + T-1 steps); returns (mean, var, log Z, s)."""
    import torch
    from paper_1106_0322_amd import SamplerConfig, SpaSMC

    torch.cuda.synchronize()
    t0 = time.perf_counter()
    s = SpaSMC(SamplerConfig.from_workload(cfg, seed=seed, **over), X, y)
    s.run()
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    mean, var, logz = s.paths()
    s.close()
    return mean, var, logz, el


def ess_protocol(R: int = 8, boot: int = 2000):
    """SPA sweep ESS/s on the n=5000, p=200 data: mixed-precision MALA (BF16 hi+lo, the
    workload) vs plain FP32 random walk, R independent seeds each.

    Reference: the pooled posterior-mean path of stored FP64 oracle replicates (tests/golden,
    8 oracle sweeps of the same data and grid with 2S = 20 MALA sweeps per scale at N=2048,
    written by the oracle alone): at finite N the path depends on the sweeps per scale, so
    a reference with twice the sweeps of the compared runs does not share their mixing
    error; its own Monte Carlo variance var_ref (replicate variance / 8) is subtracted from
    each method's MSE.  ESS_{t,j} = Var_t(beta_j) / (MSE_{t,j} - var_ref),
    the posterior variance from the runs' variance paths, summarised by the median over
    scales t >= 2 and coefficients j and divided by the wall-clock of one full sweep
    (init + T-1 steps).  At equal posterior-mean error the ratio of the two methods' ESS/s
    is the ratio of the times they need.  The interval is a bootstrap over the GPU seeds
    of both methods (the reference fixed).  A GPU FP64 MALA run with 4N
    particles and 2S sweeps is checked against that pool and against the S = 10 oracle pool
    (N=4096) of the sweep-parity test (z per cell)."""
    from synth import CONFIGS, make_dataset

    mala, rwm = CONFIGS["n5000_p200_mala_bf16"], CONFIGS["n5000_p200_rwm_fp32"]
    d = make_dataset(mala)
    golden = os.path.join(ROOT, "tests", "golden")
    fx = np.load(os.path.join(golden, "replicates_n5000_p200_mala_S20_N2048.npz"), allow_pickle=False)
    fx10 = np.load(os.path.join(golden, "replicates_n5000_p200_mala_bf16_N4096.npz"), allow_pickle=False)
    orc = fx["mean"].astype(np.float64)                      # (R_o, T, p)
    Ro, No = orc.shape[0], int(fx["N"])
    g_mean, g_var, _, g_s = full_sweep(mala, d.X, d.y, seed=9999, N=4 * mala.N, sweeps=2 * mala.sweeps,
                                       prec="fp64")

    def zcheck(pool, n_pool):
        """z per cell of the GPU FP64 4N/2S path against an oracle pool (variance of one
        4N run scaled from the pool's particle count)."""
        vs = pool.var(axis=0, ddof=1)
        z = (g_mean - pool.mean(axis=0)) / np.sqrt(vs / pool.shape[0] + vs * n_pool / (4 * mala.N))
        zc = z[1:].ravel()
        return {"max_abs_z": round(float(np.max(np.abs(zc))), 3), "rms_z": round(float(np.sqrt(np.mean(zc * zc))), 3),
                "frac_abs_z_gt_3": round(float(np.mean(np.abs(zc) > 3)), 5), "cells": int(zc.size)}

    out = {"reference": {"kind": "oracle replicate pool", "replicates": Ro, "N": No, "sweeps": int(fx["sweeps"]),
                         "prec": "fp64",
                         "check_gpu_fp64_mala_4N_2S": {"N": 4 * mala.N, "sweeps": 2 * mala.sweeps,
                                                       "seconds": round(g_s, 2),
                                                       "vs_reference_pool_S20": zcheck(orc, No),
                                                       "vs_oracle_pool_S10_N4096": zcheck(
                                                           fx10["mean"].astype(np.float64), int(fx10["N"]))}}}
    runs = {}
    for tag, cfg in (("mala_bf16x2", mala), ("rwm_fp32", rwm)):
        means, vars_, secs = [], [], []
        for r in range(R):
            m, v, _, el = full_sweep(cfg, d.X, d.y, seed=100 + r)
            means.append(m)
            vars_.append(v)
            secs.append(el)
        runs[tag] = (np.stack(means), np.stack(vars_), float(np.median(secs)), cfg)
    post_var = np.mean(np.concatenate([runs[k][1] for k in runs]), axis=0)   # Var_t(beta_j)

    def summary(means, wall, orc_s):
        rf = orc_s.mean(axis=0)
        vr = orc_s.var(axis=0, ddof=1) / orc_s.shape[0]
        mse_raw = np.mean((means - rf[None]) ** 2, axis=0)[1:]
        mse = np.maximum(mse_raw - vr[1:], 1e-300)
        ess = post_var[1:] / mse
        return float(np.median(ess)), float(np.median(ess)) / wall, mse, mse_raw

    for tag, (means, _, wall, cfg) in runs.items():
        ess_med, ess_s, mse, mse_raw = summary(means, wall, orc)
        out[tag] = {"ess_median": round(ess_med, 2), "sweep_seconds": round(wall, 4), "ess_per_sec": round(ess_s, 2),
                    "rmse_mean_path": float(f"{np.sqrt(np.mean(mse)):.4e}"),
                    "rmse_mean_path_uncorrected": float(f"{np.sqrt(np.mean(mse_raw)):.4e}"),
                    "sweeps_per_scale": cfg.sweeps, "N": cfg.N, "seeds": R}
    ratio = out["mala_bf16x2"]["ess_per_sec"] / max(out["rwm_fp32"]["ess_per_sec"], 1e-300)
    rng = np.random.default_rng(0)
    bs = []
    for _ in range(boot):
        e = {}
        for tag, (means, _, wall, _c) in runs.items():
            e[tag] = summary(means[rng.integers(0, R, R)], wall, orc)[1]
        bs.append(e["mala_bf16x2"] / max(e["rwm_fp32"], 1e-300))
    out["mala_over_rwm_ess_per_sec"] = round(ratio, 3)
    out["mala_over_rwm_ess_per_sec_ci95"] = [round(float(np.quantile(bs, 0.025)), 3),
                                             round(float(np.quantile(bs, 0.975)), 3)]
    out["bootstrap"] = boot
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="n5000_p200_mala_bf16")
    ap.add_argument("--init-sweeps", type=int, default=None)
    ap.add_argument("--prec", default=None, choices=["fp64", "fp32", "bf16x2", "fp8x3", "fp8x4"],
                    help="override the workload's contraction precision (fp8x*: random-walk moves)")
    ap.add_argument("--move", default=None, choices=["rwm", "mala"], help="override the workload's move")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-ess", action="store_true", help="skip the ESS/s protocol")
    ap.add_argument("--ess-seeds", type=int, default=8)
    ap.add_argument("--no-single", action="store_true", help="skip the single-coordinate kernel leg")
    ap.add_argument("--no-precision", action="store_true",
                    help="skip the forward-contraction comparison of BF16 hi+lo and the FP8 splits")
    ap.add_argument("--no-bandwidth", action="store_true", help="skip the weight / resampling / moment kernel leg")
    ap.add_argument("--bandwidth-only", action="store_true",
                    help="only run the weight / resampling / moment kernel leg and print its JSON")
    ap.add_argument("--cpu-leg", default=None, metavar="WORKLOAD",
                    help="only time the oracle leg of the CPU baseline on this process's threads (JSON)")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="only run a plain 256 MiB device copy three times (the reference "
                         "launch for scaling FETCH_SIZE / WRITE_SIZE counters)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for --gpus {args.gpus}); sharding the "
              "particles across GPUs is not implemented", file=sys.stderr)
        sys.exit(2)
    if args.copy_calibration:
        copy_calibration()
        return
    if args.cpu_leg:
        print(json.dumps(cpu_leg(args.cpu_leg)))
        return

    import torch
    from paper_1106_0322_amd import SamplerConfig, SpaSMC
    from synth import CONFIGS, make_dataset

    cfg = CONFIGS[args.workload]
    # the committed counter summaries describe the workload as configured
    prof_key = args.workload
    if args.prec is not None or args.move is not None:
        cfg = cfg.replace(prec=args.prec or cfg.prec, move=args.move or cfg.move)
        prof_key = None
    if args.bandwidth_only:
        d = make_dataset(cfg)
        torch.cuda.set_device(0)
        print(json.dumps(bandwidth_leg(cfg, d.X, d.y)))
        return
    if args.steps + args.warmup + BREAKDOWN_STEPS > cfg.T - 1:
        sys.exit(f"steps + warmup must be <= {cfg.T - 1 - BREAKDOWN_STEPS} scales")
    d = make_dataset(cfg)
    torch.cuda.set_device(0)
    over = {}
    if args.init_sweeps is not None:
        over["init_sweeps"] = args.init_sweeps
    s = SpaSMC(SamplerConfig.from_workload(cfg, **over), d.X, d.y)
    for _ in range(args.warmup):
        s.step()
    # the timed steps bracket only the contraction's launches with events (each bracketed
    # launch costs an event pair on the stream); the per-kernel breakdown comes from a
    # few further steps with every class bracketed
    s.set_timing(True, classes=["loglik"])
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    stats = [s.step() for _ in range(args.steps)]
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    tim = s.timing()
    s.set_timing(True)
    for _ in range(BREAKDOWN_STEPS):
        s.step()
    brk = s.timing()
    ms_step = el * 1e3 / args.steps
    flops_step = gemm_flops(cfg) * cfg.sweeps
    value = flops_step / (ms_step * 1e-3) / 1e12
    gemm_ms, gemm_n = tim["loglik"]
    gemm_avg_ms = gemm_ms / max(gemm_n, 1)
    achieved = gemm_flops(cfg) / (gemm_avg_ms * 1e-3) / 1e12
    # executed matrix work (hi and lo products over the padded shapes) from the committed
    # counter summary, over this run's live launch time; and the counters' pipe-busy share
    mf = profile_values(MFMA_PROFILE, prof_key)
    executed = None if mf is None else float(mf["mfma_flops_per_launch"]) / (gemm_avg_ms * 1e-3) / 1e12
    dtype = {"bf16x2": "bf16", "fp32": "f32", "fp64": "f64", "fp8x3": "fp8", "fp8x4": "fp8"}[cfg.prec]
    peak = PEAK_FP8 if cfg.prec.startswith("fp8x") else PEAK[cfg.prec]
    out = {
        "metric": "loglik TFLOP/s + SPA sweep ESS/sec: plain FP32 RWM vs mixed-prec MALA",
        "value": round(value, 3),
        "unit": "TFLOP/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_step, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": dtype,
        "data": "synthetic",
        "config": {"workload": f"{cfg.name}: n={cfg.n} p={cfg.p} N={cfg.N} a={cfg.a} "
                               f"{cfg.move.upper()} S={cfg.sweeps} {cfg.prec}"
                               + (f"/{cfg.xfmt}" if cfg.prec == "bf16x2" else ""),
                   "n": cfg.n, "p": cfg.p, "N": cfg.N, "sweeps_per_step": cfg.sweeps,
                   "move": cfg.move, "prec": cfg.prec},
        "roofline": {"bound": "mfma", "achieved": round(achieved, 2), "peak": peak,
                     "unit": "TFLOP/s", "frac": round(achieved / peak, 4),
                     "traffic": profiled_traffic(prof_key),
                     "kernel": "loglik_kernel (fused log-likelihood + adjoint)" if cfg.move == "mala"
                     else ("fp8x_loglik_kernel" if cfg.prec.startswith("fp8x") else "loglik_kernel"),
                     "avg_launch_us": round(gemm_avg_ms * 1e3, 2),
                     "executed_TFLOPs": None if executed is None else round(executed, 2),
                     "executed_frac": None if executed is None else round(executed / peak, 4),
                     "mfma_busy_frac": None if mf is None else float(mf["mfma_busy_frac"])},
        "kernel_ms_per_step": {k: round(v[0] / BREAKDOWN_STEPS, 4) for k, v in brk.items()},
        "accept_rate": round(float(np.mean([x["accept_rate"] for x in stats])), 4),
    }
    out["analysis"] = analysis_legs(torch, s, cfg)
    if not args.no_bandwidth:
        out["bandwidth_kernels"] = bandwidth_leg(cfg, d.X, d.y)
    if not args.no_precision:
        out["precision_variants"] = precision_legs(torch, s, cfg)
    s.close()
    if not args.no_single:
        out["single_site"] = single_site_leg()
    if not args.no_ess:
        out["ess"] = ess_protocol(args.ess_seeds)
    if not args.no_cpu:
        out["cpu_baseline"] = cpu_baseline(cfg)
    print(json.dumps(out))


if __name__ == "__main__":
    main()
