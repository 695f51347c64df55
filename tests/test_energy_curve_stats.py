"""CPU pins of the <E>(T) agreement rule (tests/energy_curve_stats.py) used by
the GPU-against-oracle annealing tests: a textbook special case, its false
alarm rate on strongly correlated curves, and its power."""
import numpy as np
from scipy import stats

from energy_curve_stats import compare_energy_curves, hotelling_two_sample


def _curves(rng, M, nt, rho, shift=None):
    """M runs of an AR(1) curve over nt temperatures (correlation rho between
    neighbours, unit variance), plus an optional mean shift."""
    e = rng.standard_normal((M, nt))
    x = np.empty_like(e)
    x[:, 0] = e[:, 0]
    for t in range(1, nt):
        x[:, t] = rho * x[:, t - 1] + np.sqrt(1 - rho * rho) * e[:, t]
    return x + (0 if shift is None else shift)


def test_hotelling_one_dimension_is_the_pooled_t_test():
    rng = np.random.default_rng(1)
    g = rng.normal(0.3, 1.0, (11, 1))
    o = rng.normal(0.0, 1.0, (9, 1))
    T2, F, p, dim = hotelling_two_sample(g, o)
    t, pt = stats.ttest_ind(g[:, 0], o[:, 0], equal_var=True)
    assert dim == 1
    assert np.isclose(T2, t * t, rtol=1e-12) and np.isclose(F, t * t, rtol=1e-12)
    assert np.isclose(p, pt, rtol=1e-9)


def test_false_alarm_rate_on_correlated_curves():
    """Equal means, neighbour correlation 0.95 over 21 temperatures, 16 runs
    per side: each p-value falls below 0.01 in about 1 % of experiments,
    while the old fixed rule (at most 10 % of temperatures beyond 2 sigma)
    fails far more often."""
    rng = np.random.default_rng(7)
    n_exp, bad = 200, np.zeros(3, int)
    naive = 0
    for _ in range(n_exp):
        g = _curves(rng, 16, 21, 0.95)
        o = _curves(rng, 16, 21, 0.95)
        r = compare_energy_curves(g, o, n_boot=400, seed=int(rng.integers(1 << 30)))
        bad += [r["p_hotelling"] < 0.01, r["p_count"] < 0.01, r["p_max"] < 0.01]
        naive += r["count2"] > 2
    print("false alarms (hotelling, count, max):", bad, "of", n_exp, "; naive 10 % rule:", naive)
    assert np.all(bad <= 8)       # binomial(200, 0.01): P(>= 9) < 1e-3
    assert naive > 8


def test_power_against_systematic_and_local_shifts():
    rng = np.random.default_rng(11)
    n_exp = 40
    hit_smooth = hit_local = 0
    for _ in range(n_exp):
        # a smooth offset growing to 1.5 run-standard-deviations (4.2 standard
        # errors of the difference) at the lowest temperature
        shift = 1.5 * np.linspace(0, 1, 21)
        g = _curves(rng, 16, 21, 0.95, shift)
        o = _curves(rng, 16, 21, 0.95)
        r = compare_energy_curves(g, o, n_boot=400, seed=1)
        hit_smooth += min(r["p_hotelling"], r["p_count"], r["p_max"]) < 0.01
        # one temperature off by 2 run-standard-deviations
        shift = np.zeros(21)
        shift[13] = 2.0
        g = _curves(rng, 16, 21, 0.95, shift)
        o = _curves(rng, 16, 21, 0.95)
        r = compare_energy_curves(g, o, n_boot=400, seed=1)
        hit_local += min(r["p_hotelling"], r["p_count"], r["p_max"]) < 0.01
    print("power: smooth", hit_smooth, "local", hit_local, "of", n_exp)
    assert hit_smooth >= 0.8 * n_exp and hit_local >= 0.8 * n_exp
