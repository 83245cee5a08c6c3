"""Write oracle replicate fixtures for the sweep-level statistical parity tests.

Runs the FP64 oracle sampler (``oracle.smc``) over a workload's full scale grid from R
independent Philox seeds and stores, per replicate, the posterior-mean path (T x p), the
log Z_t / Z_1 path, the ESS after reweighting, the resampling flags and the acceptance
rates.  Only ``oracle`` and ``synth`` are imported: no value here comes from the HIP
path.  The GPU tests compare their own replicates (independent seeds) with these, cell
by cell, with the Welch-t rule of ``tests/stats_gate.py``.

    python tests/golden/make_replicates.py --workload n5000_p200_mala_bf16 --N 4096 --R 8 --jobs 8
    python tests/golden/make_replicates.py --workload n5000_p200_mala_bf16 --name mala_n2000_p50_T12 \
        --set n=2000 p=50 N=1024 T=12 sweeps=5 init_sweeps=100

``--set`` overrides fields of the workload configuration (n and p also resize the
generated data set).  The fixture records the overrides; the tests check them.

The particle count of the oracle may be reduced from the workload's (it is stored in
the fixture); the comparison is between replicate means, each side with its own Monte
Carlo error.  The per-replicate mean paths are stored in float32 (relative rounding
6e-8, far below the Monte Carlo error of any cell); everything else in float64.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

# one BLAS thread per replicate process; replicates run side by side
for _v in ("OMP_NUM_THREADS", "OPENBLAS_NUM_THREADS", "MKL_NUM_THREADS"):
    os.environ.setdefault(_v, "1")

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

import numpy as np  # noqa: E402

from oracle import smc  # noqa: E402
from synth import CONFIGS, make_dataset  # noqa: E402

HERE = os.path.dirname(os.path.abspath(__file__))
ORACLE_SEED0 = 2000          # oracle replicate r uses Philox key 2000 + r


def fixture_path(name: str) -> str:
    return os.path.join(HERE, f"replicates_{name}.npz")


def parse_overrides(items) -> dict:
    """key=value pairs; integers, floats and names."""
    out = {}
    for it in items or []:
        k, v = it.split("=", 1)
        for conv in (int, float):
            try:
                out[k] = conv(v)
                break
            except ValueError:
                continue
        else:
            out[k] = None if v == "None" else v
    return out


def case_config(workload: str, over: dict):
    """The configuration and data set of a fixture case."""
    cfg = CONFIGS[workload].replace(**over)
    return cfg, make_dataset(cfg)


def data_digest(X, y) -> str:
    h = hashlib.sha256()
    h.update(np.ascontiguousarray(X, dtype=np.uint8).tobytes())
    h.update(np.ascontiguousarray(y, dtype=np.uint8).tobytes())
    return h.hexdigest()


def _one(args):
    workload, seed, over = args
    cfg, d = case_config(workload, over)
    t0 = time.time()
    r = smc.run_config(cfg, d.X, d.y, seed=seed)
    return dict(seed=seed, mean=r.mean, log_z=r.log_z, ess=r.ess, resampled=r.resampled,
                accept=r.accept, step=r.step, seconds=time.time() - t0)


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("--workload", required=True, choices=sorted(CONFIGS))
    ap.add_argument("--N", type=int, default=None, help="oracle particle count (default: the workload's)")
    ap.add_argument("--R", type=int, default=8)
    ap.add_argument("--jobs", type=int, default=8)
    ap.add_argument("--name", default=None, help="fixture name (default: <workload>_N<N>)")
    ap.add_argument("--set", nargs="*", default=[], help="configuration overrides key=value")
    args = ap.parse_args(argv)
    over = parse_overrides(args.set)
    if args.N:
        over["N"] = args.N
    cfg, d = case_config(args.workload, over)
    N = cfg.N
    name = args.name or f"{args.workload}_N{N}"
    seeds = [ORACLE_SEED0 + r for r in range(args.R)]
    print(f"{name}: n={cfg.n} p={cfg.p} T={cfg.T} S={cfg.sweeps} init={cfg.init_sweeps} "
          f"move={cfg.move} a={cfg.a}; oracle N={N}, R={args.R}", flush=True)
    from concurrent.futures import ProcessPoolExecutor
    out = {}
    with ProcessPoolExecutor(max_workers=args.jobs) as ex:
        futs = {ex.submit(_one, (args.workload, s, over)): s for s in seeds}
        from concurrent.futures import as_completed
        for f in as_completed(futs):
            res = f.result()
            out[res["seed"]] = res
            print(f"  seed {res['seed']} done in {res['seconds']:.0f} s", flush=True)
    rs = [out[s] for s in seeds]
    np.savez_compressed(
        fixture_path(name),
        workload=args.workload, overrides=json.dumps(over, sort_keys=True), N=N, seeds=np.array(seeds),
        data_sha256=data_digest(d.X, d.y),
        n=cfg.n, p=cfg.p, T=cfg.T, sweeps=cfg.sweeps, init_sweeps=cfg.init_sweeps, a=cfg.a,
        move=cfg.move, lambdas=cfg.grid(),
        mean=np.stack([r["mean"] for r in rs]).astype(np.float32),
        log_z=np.stack([r["log_z"] for r in rs]),
        ess=np.stack([r["ess"] for r in rs]),
        resampled=np.stack([r["resampled"] for r in rs]),
        accept=np.stack([r["accept"] for r in rs]),
        step=np.stack([r["step"] for r in rs]),
        seconds=np.array([r["seconds"] for r in rs]))
    print(f"wrote {fixture_path(name)}", flush=True)


if __name__ == "__main__":
    main()
