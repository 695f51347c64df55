"""Pins of the oracle's two further resampling modes (CPU only).

* Multinomial resampling, the rule the paper states after the PAMD scheme: R
  independent draws from the categorical distribution p_j = tau_j / R, so the
  population size stays R.  Pins: deterministic stratified draws, the exact
  multinomial law on a tiny case (scipy's pmf), E[c_j] = R p_j and
  Cov(c_j, c_k) = R (p_j delta_jk - p_j p_k), zero-weight copies never drawn,
  the rounding tail u W == W.
* "none": resampling switched off (the paper's "anneal" ablation): every copy
  is kept once, so the run is R independent annealing runs.
"""
import itertools
import math

import numpy as np
from scipy import stats

from oracle import oracle as O
from pamd_inputs import systems as S


def test_equal_weights_with_stratified_draws_give_one_copy_each():
    R = 257
    E = np.random.default_rng(1).normal(0, 3, R)
    u = (np.arange(R) + 0.5) / R
    c, W = O.multinomial_counts(E, 0.0, u)
    assert (W == np.arange(1, R + 1)).all()
    assert (c == 1).all()


def test_draws_on_interval_edges_belong_to_the_interval_they_open():
    """Draw k selects j when u_k lies in [W_{j-1}, W_j) / W (half-open
    intervals of length p_j).  Equal weights, R a power of two, u_k = k / R:
    every u_k sits exactly on the left edge of interval k."""
    R = 256
    u = np.arange(R) / R
    c, W = O.multinomial_counts(np.zeros(R), 1.0, u)
    assert (u * W[-1] == np.arange(R)).all()
    assert (c == 1).all()


def test_dominant_weight_takes_every_draw():
    E = np.array([5.0, -400.0, 3.0, 7.0])
    u = O.multinomial_uniforms(100, 1, seed=3)
    c, _ = O.multinomial_counts(E, 1.0, u)
    assert c.tolist() == [0, 100, 0, 0]


def test_zero_weights_are_never_drawn_and_the_tail_rule():
    # w = exp(-(E - min)) underflows to 0 for the last two entries
    E = np.array([0.0, 1.0, 2000.0, 0.5, 3000.0, 4000.0])
    w = np.exp(-(E - E.min()))
    assert (w[[2, 4, 5]] == 0).all()
    u = np.array([0.0, 1.0 - 2.0 ** -53, 0.5, 0.999999])
    c, W = O.multinomial_counts(E, 1.0, u)
    assert c[[2, 4, 5]].sum() == 0 and c.sum() == 4
    # u = 0 picks the first entry; u -> 1 picks the last one with positive weight
    assert O.multinomial_counts(E, 1.0, np.array([0.0]))[0][0] == 1
    assert O.multinomial_counts(E, 1.0, np.array([1.0 - 2.0 ** -53]))[0][3] == 1


def test_tiny_case_follows_the_multinomial_law():
    """Three sources, three draws: frequencies of all 10 compositions over
    30000 independent resamplings (temperature index = trial) against scipy's
    multinomial pmf, chi-square p-value > 1e-4."""
    E = np.array([0.0, 0.7, 1.6])
    db = 1.3
    w = np.exp(-db * (E - E.min()))
    p = w / w.sum()
    n, trials = 3, 30000
    counts = {}
    for t in range(trials):
        c, _ = O.multinomial_counts(E, db, O.multinomial_uniforms(n, t + 1, seed=11))
        counts[tuple(c)] = counts.get(tuple(c), 0) + 1
    comps = [c for c in itertools.product(range(n + 1), repeat=3) if sum(c) == n]
    obs = np.array([counts.get(c, 0) for c in comps], float)
    exp = np.array([stats.multinomial.pmf(c, n, p) for c in comps]) * trials
    assert obs.sum() == trials
    chi2 = ((obs - exp) ** 2 / exp).sum()
    assert stats.chi2.sf(chi2, len(comps) - 1) > 1e-4, (obs, exp)


def test_mean_and_covariance_of_the_counts():
    """R = 6 sources, R draws, 20000 trials: every mean within 5 standard
    errors of R p_j; the covariance matrix within 0.06 of R (p_j delta_jk -
    p_j p_k) (its entries are O(1), their standard errors ~0.01)."""
    rng = np.random.default_rng(7)
    R, trials = 6, 20000
    E = rng.normal(0, 1.0, R)
    db = 0.9
    w = np.exp(-db * (E - E.min()))
    p = w / w.sum()
    C = np.array([O.multinomial_counts(E, db, O.multinomial_uniforms(R, t + 1, seed=5, run=2))[0]
                  for t in range(trials)], float)
    assert (C.sum(1) == R).all()
    cov = R * (np.diag(p) - np.outer(p, p))
    se = np.sqrt(np.diag(cov) / trials)
    assert np.all(np.abs(C.mean(0) - R * p) < 5 * se)
    assert np.abs(np.cov(C.T) - cov).max() < 0.06


def test_population_size_is_the_number_of_draws():
    rng = np.random.default_rng(9)
    for R_cur, R_t in [(1, 1), (1, 17), (1000, 1000), (999, 1024), (1500, 700)]:
        E = rng.normal(0, 5, R_cur)
        c = O.resampling_counts("multinomial", E, 0.4, R_t, 3, seed=2)
        assert c.sum() == R_t and len(c) == R_cur and (c >= 0).all()


def test_streams_are_distinct_from_the_rounding_uniforms():
    a = O.multinomial_uniforms(64, 5, seed=1)
    b = O.resample_uniforms(64, 5, seed=1)
    assert not np.any(a == b)
    assert np.all((a >= 0) & (a < 1))


def test_no_resampling_keeps_every_copy_and_runs_are_independent():
    """With resampling off the population never changes size or ancestry, and
    each copy's trajectory is independent of the others: the first 4 copies of
    an R = 8 run equal an R = 4 run from the same start (Philox counters are
    per slot)."""
    sysd = S.c1_system()
    sched = S.geometric_schedule(2.0, 1.0, 5)
    rng = np.random.default_rng(4)
    x0 = np.ascontiguousarray(sysd.x_init[None] + rng.normal(0, 0.05, (8,) + sysd.x_init.shape))
    a = O.anneal(sysd, 8, 2.0, sched, theta=30, theta_eq=30, dt=0.002, nu=1.0, seed=6, x0=x0,
                 resampling="none")
    b = O.anneal(sysd, 4, 2.0, sched, theta=30, theta_eq=30, dt=0.002, nu=1.0, seed=6,
                 x0=np.ascontiguousarray(x0[:4]), resampling="none")
    assert a.R == [8] * len(sched) and all(o["families"] == 8 for o in a.obs)
    assert np.array_equal(a.x[:4], b.x) and np.array_equal(a.v[:4], b.v)


def test_multinomial_anneal_keeps_R_and_estimates_the_gaussian_chain_free_energy():
    """PA with multinomial resampling on the zero-rest-length chain (N = 10,
    k = 100): sum ln Q -> 13.5 ln(1/4) over T 2 -> 0.5, R constant."""
    sysd = S.gaussian_chain(10, 100.0, 0.0)
    sched = S.geometric_schedule(2.0, 0.5, 20)
    R, M = 600, 5
    sums = []
    for seed in range(1, M + 1):
        rng = np.random.default_rng(300 + seed)
        # exact Boltzmann start: bond vectors ~ N(0, T / k) per component
        b = rng.normal(0, math.sqrt(2.0 / 100.0), (R, 9, 3))
        x0 = np.zeros((R, 10, 3))
        x0[:, 1:] = np.cumsum(b, axis=1)
        res = O.anneal(sysd, R, 2.0, sched, theta=100, theta_eq=100, dt=0.002, nu=1.0, seed=seed,
                       x0=np.ascontiguousarray(x0), resampling="multinomial")
        assert res.R == [R] * len(sched)
        sums.append(res.sum_lnQ)
    exact = 13.5 * math.log(0.25)
    mean, se = np.mean(sums), np.std(sums, ddof=1) / math.sqrt(M)
    assert abs(mean - exact) < 3 * se + 0.01, (mean, se, exact)
