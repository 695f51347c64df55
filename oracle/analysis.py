"""FP64 reference of the population analysis -- TEST INFRASTRUCTURE ONLY.

Only ``tests/`` may import this module; it shares no code with the library.

Paper: Christiansen, Weigel & Janke, arXiv:1806.06016.
* Correlations after resampling (the paragraph after the thermostat
  discussion): copies of one configuration are correlated, which the errors of
  population averages must respect; the paper assesses this by binning over
  the population.  Here: the family (cluster) error, where a family is all
  copies of one initial replica (same ancestor), the consecutive-slot binning
  error, and the family statistics rho_t = R sum_f nu_f^2 and the family
  entropy S_f = -sum_f nu_f ln nu_f (nu_f = n_f / R).
* Free energies (the paragraph on the recorded normalisers): sum ln Q gives
  ln Z(T_i) - ln Z(T_0) directly and serves as the starting point of the
  multiple-histogram (WHAM) self-consistency iterations, here in their
  per-sample form (no energy bins).
"""
from __future__ import annotations

from typing import Dict, Sequence

import numpy as np
from scipy.special import logsumexp


def family_error(O: np.ndarray, ancestor: np.ndarray) -> Dict[str, float]:
    """Mean of O over the population and its standard errors.

    naive_se^2  = sum_j (O_j - mean)^2 / (R (R - 1))
    family_se^2 = sum_f (sum_{j in f} (O_j - mean))^2 / (R (R - 1))
    (singleton families reduce the second to the first)."""
    O = np.asarray(O, np.float64)
    R = len(O)
    mean = O.mean()
    d = O - mean
    _, inv, n_f = np.unique(np.asarray(ancestor), return_inverse=True, return_counts=True)
    S_f = np.bincount(inv, weights=d)
    nu = n_f / R
    denom = R * (R - 1) if R > 1 else np.inf
    return dict(mean=float(mean), naive_se=float(np.sqrt((d * d).sum() / denom)),
                family_se=float(np.sqrt((S_f * S_f).sum() / denom)), families=int(len(n_f)),
                rho_t=float(R * (nu * nu).sum()), family_entropy=float(-(nu * np.log(nu)).sum()))


def binning_error(O: np.ndarray, b: int) -> float:
    """Standard error of the mean from bins of b consecutive slots: the
    first floor(R / b) complete bins, se^2 = var(bin means, ddof 1) / n_bins."""
    O = np.asarray(O, np.float64)
    nb = len(O) // b
    if nb < 2:
        return float("nan")
    m = O[:nb * b].reshape(nb, b).mean(1)
    return float(np.sqrt(m.var(ddof=1) / nb))


def wham(beta: Sequence[float], samples: Sequence[np.ndarray], lnZ0: Sequence[float], iters: int = 1000,
         tol: float = 1e-10):
    """Multiple-histogram self-consistency in per-sample form.

    With N_l samples E_{l,n} at inverse temperature beta_l and ln Z_l the
    current estimates, every sample's mixture denominator is
        ln D(E) = logsumexp_l (ln N_l - beta_l E - ln Z_l),
    and the update is ln Z_k = logsumexp_{all samples} (-beta_k E - ln D(E)),
    shifted so that ln Z_0 keeps its starting value.  Iterates until the
    largest change is below tol.  Returns (ln Z [L], iterations)."""
    beta = np.asarray(beta, np.float64)
    E = np.concatenate([np.asarray(s, np.float64) for s in samples])
    lnN = np.log(np.array([len(s) for s in samples], np.float64))
    lnZ = np.asarray(lnZ0, np.float64).copy()
    for it in range(1, iters + 1):
        lnD = logsumexp(lnN[None, :] - np.outer(E, beta) - lnZ[None, :], axis=1)
        new = logsumexp(-np.outer(E, beta) - lnD[:, None], axis=0)
        new += lnZ[0] - new[0]
        delta = np.abs(new - lnZ).max()
        lnZ = new
        if delta < tol:
            return lnZ, it
    return lnZ, iters


def wham_average(beta_q: float, beta: Sequence[float], samples: Sequence[np.ndarray], lnZ: Sequence[float]):
    """<E> and <E^2> at inverse temperature beta_q from all samples, weights
    exp(-beta_q E) / D(E) with D from the (converged) ln Z."""
    beta = np.asarray(beta, np.float64)
    E = np.concatenate([np.asarray(s, np.float64) for s in samples])
    lnN = np.log(np.array([len(s) for s in samples], np.float64))
    lnD = logsumexp(lnN[None, :] - np.outer(E, beta) - np.asarray(lnZ)[None, :], axis=1)
    lw = -beta_q * E - lnD
    w = np.exp(lw - lw.max())
    w /= w.sum()
    return float((w * E).sum()), float((w * E * E).sum())
