"""Statistical agreement of two sets of annealed <E_pot>(T) curves.

Each side runs M independently seeded annealing runs and records one
population mean per temperature: arrays g [M_g, n_T] and o [M_o, n_T].  The
question is whether both sides sample the same process (the annealed
<E>(T) "within 2 sigma").  The means of one run are correlated from one
temperature to the next (every temperature inherits the run's population
history), so per-temperature z-scores are not independent and a plain count of
|z| > 2 has no fixed null distribution.  The rule used here takes the
correlation from the runs themselves:

* Hotelling's two-sample T^2 on the n_T-vector of mean differences with the
  pooled across-run covariance: F = (n - p - 1) / (p (n - 2)) T^2 follows
  F(p, n - p - 1) under equal means (n = M_g + M_o runs, p = the rank of the
  pooled covariance);
* the per-temperature Welch z-scores, their count beyond 2 and their largest
  modulus, each compared with its null distribution under the estimated
  covariance by a parametric bootstrap (whole experiments of M_g and M_o
  Gaussian runs with the pooled covariance, the same statistics recomputed),
  which corrects the 2-sigma count for multiplicity and correlation.

All three p-values must exceed alpha (0.01 each in the tests).
"""
from __future__ import annotations

import numpy as np
from scipy import stats


def _welch_z(g: np.ndarray, o: np.ndarray) -> np.ndarray:
    se = np.sqrt(g.var(0, ddof=1) / len(g) + o.var(0, ddof=1) / len(o))
    return (g.mean(0) - o.mean(0)) / se


def hotelling_two_sample(g: np.ndarray, o: np.ndarray, rel_cut: float = 1e-10):
    """Two-sample Hotelling T^2 with pooled covariance.  Returns (T2, F, p,
    dim); directions of the pooled covariance with eigenvalue below
    rel_cut x the largest are dropped (dim counts the kept ones)."""
    g = np.asarray(g, np.float64)
    o = np.asarray(o, np.float64)
    mg, mo = len(g), len(o)
    n = mg + mo
    d = g.mean(0) - o.mean(0)
    sp = ((mg - 1) * np.cov(g, rowvar=False, ddof=1).reshape(d.size, d.size)
          + (mo - 1) * np.cov(o, rowvar=False, ddof=1).reshape(d.size, d.size)) / (n - 2)
    w, V = np.linalg.eigh(sp)
    keep = w > rel_cut * w.max()
    p = int(keep.sum())
    if n - p - 1 < 1:
        raise ValueError(f"{n} runs cannot estimate a {p}-dimensional covariance")
    y = V[:, keep].T @ d
    T2 = mg * mo / n * float(np.sum(y * y / w[keep]))
    F = (n - p - 1) / (p * (n - 2)) * T2
    return T2, F, float(stats.f.sf(F, p, n - p - 1)), p


def compare_energy_curves(g, o, n_boot: int = 4000, seed: int = 12345) -> dict:
    """The three statistics of the module docstring with their p-values."""
    g = np.asarray(g, np.float64)
    o = np.asarray(o, np.float64)
    mg, mo = len(g), len(o)
    z = _welch_z(g, o)
    count = int(np.sum(np.abs(z) > 2.0))
    zmax = float(np.max(np.abs(z)))
    T2, F, p_hot, dim = hotelling_two_sample(g, o)
    # parametric bootstrap of the per-temperature statistics under equal means
    sp = ((mg - 1) * np.cov(g, rowvar=False) + (mo - 1) * np.cov(o, rowvar=False)) / (mg + mo - 2)
    w, V = np.linalg.eigh(sp)
    L = V * np.sqrt(np.clip(w, 0.0, None))
    rng = np.random.default_rng(seed)
    nt = g.shape[1]
    cnt = np.empty(n_boot, np.int64)
    mx = np.empty(n_boot)
    for b in range(n_boot):
        gs = rng.standard_normal((mg, nt)) @ L.T
        os_ = rng.standard_normal((mo, nt)) @ L.T
        zb = _welch_z(gs, os_)
        cnt[b] = np.sum(np.abs(zb) > 2.0)
        mx[b] = np.max(np.abs(zb))
    p_count = float((np.sum(cnt >= count) + 1) / (n_boot + 1))
    p_max = float((np.sum(mx >= zmax) + 1) / (n_boot + 1))
    return dict(z=z, count2=count, zmax=zmax, T2=T2, F=F, dim=dim, p_hotelling=p_hot, p_count=p_count,
                p_max=p_max, count2_null_mean=float(cnt.mean()))


def report(res: dict) -> str:
    return (f"z = {np.round(res['z'], 2).tolist()}; beyond 2 sigma: {res['count2']} "
            f"(null mean {res['count2_null_mean']:.2f}, p = {res['p_count']:.3f}); max |z| = {res['zmax']:.2f} "
            f"(p = {res['p_max']:.3f}); Hotelling T^2 = {res['T2']:.2f} in {res['dim']} dims "
            f"(p = {res['p_hotelling']:.3f})")
