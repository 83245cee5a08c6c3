"""Sweep-level statistical parity of replicate paths (GPU seeds against oracle seeds).

A sampler run is one draw of a random path: the posterior means E_t[beta_j] over the
scale grid (T x p cells), or the log Z_t / Z_1 path (T cells).  Different Philox keys give
independent draws.  Each cell is an average over N weighted particles, so across seeds
it is approximately normal (the SMC central limit theorem).  Both samplers target the same
posterior, so under the null hypothesis every cell has the same expectation on both sides.

Two tests are used.  Both fix the family-wise false-alarm rate at alpha = 0.001 over all
the cells of a path.

* ``welch_gate``: Welch's t per cell, t = (mean_g - mean_o) / sqrt(s_g^2/R_g + s_o^2/R_o),
  with Welch-Satterthwaite degrees of freedom
  nu = (s_g^2/R_g + s_o^2/R_o)^2 / ((s_g^2/R_g)^2/(R_g-1) + (s_o^2/R_o)^2/(R_o-1)).
  The two-sided p-value is p = 2 sf_t(|t|, nu).  The path passes iff min_c p_c >= alpha/C over
  its C cells.  That is a per-tail level of alpha/(2C), i.e. 0.001/(2 T p) for a mean path.
  By Bonferroni the family-wise rate stays <= alpha however the cells are correlated.  The
  test allows different particle counts and variances on the two sides.  With 8 replicates a
  side its critical |t| is large (nu ~ 7-14 gives 10-24 at C = 20000), so its power is low.
* ``permutation_gate``: when both sides run the same sampler at the same particle count,
  the pooled replicates are exchangeable under the null.  Two statistics are used: max_c |t_c|
  (a local departure) and the root mean square of t_c over the cells (a small departure shared
  by many cells, the signature of a systematic error).  Their null distributions come from
  every split of the pooled replicates into groups of R_g and R_o (12870 splits for 8 + 8).
  Each is tested at alpha/2, so the pair is exact at level alpha and allows any correlation
  between cells.  The tests use the empirical tails, not the Student ones.

Cells whose values are identical across every replicate on both sides carry no
information (log Z at t = 1 is 0 by definition).  They are left out.  A zero-variance cell
whose two sides differ fails.
"""
from __future__ import annotations

import itertools
import math

import numpy as np
from scipy import stats

ALPHA = 1e-3


def welch_t(g, o):
    """Per-cell Welch t and Satterthwaite degrees of freedom of replicate arrays (R, ...)."""
    g = np.asarray(g, dtype=np.float64)
    o = np.asarray(o, dtype=np.float64)
    Rg, Ro = g.shape[0], o.shape[0]
    vg = g.var(axis=0, ddof=1) / Rg
    vo = o.var(axis=0, ddof=1) / Ro
    se2 = vg + vo
    d = g.mean(axis=0) - o.mean(axis=0)
    with np.errstate(divide="ignore", invalid="ignore"):
        t = d / np.sqrt(se2)
        nu = se2 * se2 / (vg * vg / (Rg - 1) + vo * vo / (Ro - 1))
    return t, nu, d, se2


def _informative(g, o):
    """Mask of cells whose replicate values are not all identical on both sides, and
    whether a degenerate cell has different values on the two sides."""
    allv = np.concatenate([np.asarray(g, np.float64), np.asarray(o, np.float64)], axis=0)
    const = np.all(allv == allv[:1], axis=0)
    g = np.asarray(g, np.float64)
    o = np.asarray(o, np.float64)
    zero_var = (g.var(axis=0) == 0) & (o.var(axis=0) == 0)
    bad = zero_var & ~const
    return ~const, bool(np.any(bad))


def welch_gate(g, o, alpha: float = ALPHA) -> dict:
    """Family-wise Welch-t rule (Bonferroni over the informative cells)."""
    keep, bad = _informative(g, o)
    t, nu, d, se2 = welch_t(g, o)
    t, nu = t[keep], nu[keep]
    C = int(t.size)
    pv = 2.0 * stats.t.sf(np.abs(t), nu) if C else np.ones(0)
    level = alpha / max(C, 1)
    out = dict(cells=C, max_abs_t=float(np.max(np.abs(t))) if C else 0.0,
               min_p=float(np.min(pv)) if C else 1.0, level=level,
               frac_p_below_3sigma=float(np.mean(pv < 2.0 * stats.norm.sf(3.0))) if C else 0.0,
               rms_t=float(np.sqrt(np.mean(t * t))) if C else 0.0,
               min_nu=float(np.min(nu)) if C else math.inf,
               degenerate_mismatch=bad)
    out["passed"] = (not bad) and (C == 0 or out["min_p"] >= level)
    return out


def permutation_gate(g, o, alpha: float = ALPHA, max_splits: int = 20000, seed: int = 0) -> dict:
    """Exact permutation tests of max_c |Welch t_c| and of rms_c t_c, each at alpha/2, over
    every split of the pooled replicates (a seeded random subset of splits when there are
    more than max_splits)."""
    g = np.asarray(g, np.float64)
    o = np.asarray(o, np.float64)
    keep, bad = _informative(g, o)
    Rg, Ro = g.shape[0], o.shape[0]
    R = Rg + Ro
    pool = np.concatenate([g, o], axis=0)[:, keep]
    pool = pool - pool.mean(axis=0)          # centred per cell: no cancellation in the sums
    total = math.comb(R, Rg)
    if total <= max_splits:
        idx = np.array(list(itertools.combinations(range(R), Rg)))
    else:
        rng = np.random.default_rng(seed)
        idx = np.stack([np.sort(rng.choice(R, size=Rg, replace=False)) for _ in range(max_splits)])
        idx = np.concatenate([np.arange(Rg)[None, :], idx])
    A = np.zeros((idx.shape[0], R))
    np.put_along_axis(A, idx, 1.0, axis=1)
    t1, t2 = pool.sum(axis=0), (pool * pool).sum(axis=0)
    sq = pool * pool
    stat = np.empty(A.shape[0])
    stat_rms = np.empty(A.shape[0])
    for lo in range(0, A.shape[0], 64):
        a = A[lo:lo + 64]
        s1g, s2g = a @ pool, a @ sq
        s1o, s2o = t1 - s1g, t2 - s2g
        vg = np.maximum(s2g - s1g * s1g / Rg, 0.0) / (Rg - 1) / Rg
        vo = np.maximum(s2o - s1o * s1o / Ro, 0.0) / (Ro - 1) / Ro
        with np.errstate(divide="ignore", invalid="ignore"):
            t = (s1g / Rg - s1o / Ro) / np.sqrt(vg + vo)
        t = np.where(np.isfinite(t), np.abs(t), 0.0)
        stat[lo:lo + 64] = t.max(axis=1) if t.shape[1] else 0.0
        stat_rms[lo:lo + 64] = np.sqrt(np.mean(t * t, axis=1)) if t.shape[1] else 0.0
    # the first split is (0..Rg-1): the observed one; it is among the splits, and ties count
    # against the test
    obs, obs_rms = float(stat[0]), float(stat_rms[0])
    pval = float(np.mean(stat >= obs * (1.0 - 1e-12)))
    pval_rms = float(np.mean(stat_rms >= obs_rms * (1.0 - 1e-12)))
    return dict(cells=int(pool.shape[1]), max_abs_t=obs, p_value=pval, rms_t=obs_rms, p_value_rms=pval_rms,
                splits=int(stat.size), null_max_q=float(np.quantile(stat, 1.0 - alpha / 2)),
                null_rms_q=float(np.quantile(stat_rms, 1.0 - alpha / 2)), degenerate_mismatch=bad,
                passed=(not bad) and pval >= alpha / 2 and pval_rms >= alpha / 2)


def describe(name: str, res: dict) -> str:
    if "p_value" in res:
        return (f"{name}: permutation max|t| {res['max_abs_t']:.2f} (critical {res['null_max_q']:.2f}, "
                f"p {res['p_value']:.4f}), rms t {res['rms_t']:.3f} (critical {res['null_rms_q']:.3f}, "
                f"p {res['p_value_rms']:.4f}) over {res['splits']} splits, {res['cells']} cells")
    return (f"{name}: Welch max|t| {res['max_abs_t']:.2f}, min p {res['min_p']:.2e} vs level "
            f"{res['level']:.2e} ({res['cells']} cells, min nu {res['min_nu']:.1f}), "
            f"frac p<0.0027 {res['frac_p_below_3sigma']:.4f}, rms t {res['rms_t']:.2f}")
