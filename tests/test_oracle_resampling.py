"""Pins of the oracle's resampling (PAMD step 2), observables, adaptive
temperature choice and free-energy estimator (CPU only).

tau_j = exp(-(beta_i - beta_{i-1}) E_j) / Q with Q = (1/R) sum_j exp(...)
(PAMD scheme, step 2); ln Q_i estimates ln Z(T_i) - ln Z(T_{i-1}) (paragraph
on the recorded normalisers).  Pins: special cases with no randomness,
exact sums, expectations and brute-force distributions, and closed-form
partition functions of harmonic chains.
"""
import itertools
import math

import numpy as np
import pytest
from scipy import special, stats

from oracle import oracle as O
from pamd_inputs import systems as S


def test_equal_energies_give_one_copy_each():
    E = np.full(1000, -12.5)
    u = np.random.default_rng(0).random(1000)
    c, tau = O.copy_counts(E, 0.37, 1000, u)
    assert (tau == 1.0).all() and (c == 1).all()


def test_same_temperature_is_identity():
    E = np.random.default_rng(1).normal(0, 50, 777)
    u = np.random.default_rng(2).random(777)
    m, S_, S2, lq = O.lse(E, 0.0)
    assert lq == 0.0
    c, tau = O.copy_counts(E, 0.0, 777, u)
    assert (c == 1).all()


def test_tau_sums_to_target_and_lse_matches_naive():
    rng = np.random.default_rng(3)
    E = rng.normal(3.0, 0.5, 5000)
    db = 0.8
    m, S_, S2, lq = O.lse(E, db)
    naive = math.log(np.mean(np.exp(-db * E)))
    assert abs(lq - naive) < 1e-14 * max(1.0, abs(naive))
    c, tau = O.copy_counts(E, db, 4321, rng.random(5000))
    assert abs(math.fsum(tau) - 4321) < 1e-9
    # shift invariance: E + C changes ln Q by -dbeta C, not the weights
    m2, S2_, _, lq2 = O.lse(E + 1e6, db)
    assert abs(lq2 - (lq - db * 1e6)) < 1e-8 * 1e6 * db
    c2, tau2 = O.copy_counts(E + 1e6, db, 4321, rng.random(5000))
    assert np.allclose(tau2, tau, rtol=1e-9)


def test_counts_expectation_and_total_bound():
    """E[c_j] = tau_j for every j, and |sum c - R| <= 5 sqrt(sum f(1-f)) + 1."""
    rng = np.random.default_rng(4)
    R = 300
    E = rng.normal(0, 2.0, R)
    db = 0.6
    trials = 4000
    acc = np.zeros(R)
    tau = None
    for t in range(trials):
        c, tau = O.copy_counts(E, db, R, rng.random(R))
        f = tau - np.floor(tau)
        assert abs(int(c.sum()) - R) <= 5 * math.sqrt((f * (1 - f)).sum()) + 1
        acc += c
    mean = acc / trials
    f = tau - np.floor(tau)
    se = np.sqrt(f * (1 - f) / trials) + 1e-12
    z = (mean - tau) / se
    assert np.abs(z[f > 0.01]).max() < 5.0


def test_brute_force_count_distribution_small_R():
    """R = 6: c_j is floor(tau_j) plus a Bernoulli(frac tau_j) bit.  Compare
    the empirical joint law of (c_1..c_6) under uniform draws with the exact
    product law enumerated over all 2^6 outcomes (chi^2)."""
    rng = np.random.default_rng(5)
    E = np.array([0.0, 0.3, -0.4, 1.2, 0.8, -0.1])
    db = 1.3
    _, tau = O.copy_counts(E, db, 6, np.zeros(6))
    fl = np.floor(tau).astype(int)
    fr = tau - fl
    probs = {}
    for bits in itertools.product([0, 1], repeat=6):
        p = np.prod([fr[j] if b else 1 - fr[j] for j, b in enumerate(bits)])
        probs[tuple(fl + np.array(bits))] = p
    n = 20000
    seen = {}
    for _ in range(n):
        c, _ = O.copy_counts(E, db, 6, rng.random(6))
        seen[tuple(c)] = seen.get(tuple(c), 0) + 1
    assert set(seen) <= set(probs)
    keys = [k for k in probs if probs[k] * n >= 5]
    obs = np.array([seen.get(k, 0) for k in keys], float)
    exp = np.array([probs[k] * n for k in keys])
    chi2 = ((obs - exp) ** 2 / exp).sum()
    assert stats.chi2.sf(chi2, len(keys) - 1) > 1e-3


def test_gather_canonical_order_and_rescale():
    counts = np.array([0, 2, 1, 0, 3], np.int32)
    x = np.arange(5 * 2 * 3, dtype=float).reshape(5, 2, 3)
    anc = np.arange(5) + 100
    xn, an = O.gather(counts, [x, anc])
    assert list(an) == [101, 101, 102, 104, 104, 104]
    assert (xn[0] == x[1]).all() and (xn[5] == x[4]).all()
    mass = np.array([1.0, 3.0])
    xr = O.recentre(xn, mass)
    com = np.einsum("rac,a->rc", xr, mass) / 4.0
    assert np.abs(com).max() < 1e-13


def test_nonfinite_energy_is_an_error():
    E = np.array([1.0, np.nan, 2.0])
    with pytest.raises(FloatingPointError):
        O.lse(E, 0.1)


def _gamma_variance(x, d):
    """Normalised weight variance for energies E ~ Gamma(d/2, kB T_prev) (a
    harmonic system with d quadratic degrees of freedom), x = T_prev/T_next - 1."""
    return (1 + x) ** d / (1 + 2 * x) ** (d / 2) - 1


def test_weight_variance_and_adaptive_step_closed_form():
    """With harmonic energies (Gamma distributed with shape d/2) the
    normalised weight variance has the closed form (1+x)^d / (1+2x)^(d/2) - 1;
    the bisection must land where that equals 0.1 (large R)."""
    d = 27
    T_prev = 1.3
    rng = np.random.default_rng(6)
    E = rng.gamma(d / 2, T_prev, 400000)
    for x in (0.02, 0.05):
        T_next = T_prev / (1 + x)
        db = 1 / T_next - 1 / T_prev
        assert abs(O.weight_variance(E, db) - _gamma_variance(x, d)) < 0.05 * _gamma_variance(x, d)
    # closed-form root of V(x) = 0.1
    from scipy.optimize import brentq
    xs = brentq(lambda x: _gamma_variance(x, d) - 0.1, 1e-6, 1.0)
    db_max = 1 / 0.5 - 1 / T_prev
    db = O.adaptive_dbeta(E, db_max, 0.1)
    T_next = 1 / (db + 1 / T_prev)
    assert abs((T_prev / T_next - 1) - xs) < 0.03 * xs
    assert abs(O.weight_variance(E, db) - 0.1) < 1e-9
    # V at the far end within target -> take the far end
    assert O.adaptive_dbeta(E, 1e-4, 0.1) == 1e-4


def _chain_boltzmann_start(n, k, T, R, rng):
    """Exact Boltzmann sample of a zero-rest-length bonds-only chain: bond
    vectors N(0, T/k) per component."""
    b = rng.normal(0, math.sqrt(T / k), size=(R, n - 1, 3))
    x = np.zeros((R, n, 3))
    x[:, 1:] = np.cumsum(b, axis=1)
    return np.ascontiguousarray(x)


@pytest.mark.slow
def test_gaussian_chain_free_energy_and_energies():
    """PA on the zero-rest-length chain (N = 10, k = 100, kB = 1) over the
    bead-chain schedule T 2 -> 0.5 (20 geometric steps): Z_conf ~ beta^(-27/2),
    so sum ln Q -> 13.5 ln(0.25) = -18.715; <U> = 13.5 T and <K> = 15 T at
    every T.  The estimator's bias is O(1/R); the test allows 3 sigma over M
    independent seeds.  U is a sum of 27 independent quadratic terms, i.e.
    Gamma(13.5, T) distributed: Var U = 13.5 T^2, so the heat-capacity
    observable Cv / kB = Var U / (kB T)^2 = 13.5 at every T, and
    <U^2> = Var U + <U>^2 = 13.5 T^2 (1 + 13.5).  Population variances are
    noisy (resampled copies are correlated): each temperature's Cv averaged over
    the seeds within 12 %, the mean over all temperatures within 3 %."""
    sysd = S.gaussian_chain(10, 100.0, 0.0)
    sched = S.geometric_schedule(2.0, 0.5, 20)
    R, M = 600, 6
    sums, U, Cv, U2 = [], [], [], []
    for seed in range(1, M + 1):
        rng = np.random.default_rng(100 + seed)
        x0 = _chain_boltzmann_start(10, 100.0, 2.0, R, rng)
        res = O.anneal(sysd, R, 2.0, sched, theta=100, theta_eq=100, dt=0.002, nu=1.0,
                       seed=seed, x0=x0)
        sums.append(res.sum_lnQ)
        U.append([o["E_mean"] for o in res.obs])
        Cv.append([o["Cv"] for o in res.obs])
        U2.append([o["E2_mean"] for o in res.obs])
        Km = np.array([o["K_mean"] for o in res.obs])
        assert np.all(np.abs(Km / (15 * np.array(res.T)) - 1) < 0.05)
    exact = 13.5 * math.log(0.25)
    mean, se = np.mean(sums), np.std(sums, ddof=1) / math.sqrt(M)
    assert abs(mean - exact) < 3 * se + 0.01, (mean, se, exact)
    Um = np.mean(U, axis=0) / (13.5 * sched)
    assert np.all(np.abs(Um - 1) < 0.03), Um
    cv = np.mean(Cv, axis=0) / 13.5
    print("Cv / 13.5 per temperature", np.round(cv, 3), "mean", cv.mean())
    assert np.all(np.abs(cv - 1) < 0.12), cv
    assert abs(cv.mean() - 1) < 0.03, cv.mean()
    u2 = np.mean(U2, axis=0) / (13.5 * sched ** 2 * 14.5)
    assert np.all(np.abs(u2 - 1) < 0.07), u2


@pytest.mark.slow
def test_bonded_chain_free_energy_r0_one():
    """Bonds-only chain with r0 = 1 (k = 100): each bond vector contributes
    z_b(beta)/4pi = (r0^2 + 1/(2a)) sqrt(pi)/(2 sqrt a) (1 + erf(r0 sqrt a))
    + r0/(2a) e^{-a r0^2}, a = beta k / 2, so ln Z(T_N)/Z(T_0) = 9 [ln z_b(2) -
    ln z_b(0.5)].  Start: exact samples of the bond-length law by rejection."""
    k, r0, n = 100.0, 1.0, 10

    def lnzb(beta):
        a = beta * k / 2
        return math.log((r0 ** 2 + 1 / (2 * a)) * math.sqrt(math.pi) / (2 * math.sqrt(a))
                        * (1 + special.erf(r0 * math.sqrt(a))) + r0 / (2 * a) * math.exp(-a * r0 ** 2))

    exact = (n - 1) * (lnzb(1 / 0.5) - lnzb(1 / 2.0))
    sysd = S.gaussian_chain(n, k, r0)
    sched = S.geometric_schedule(2.0, 0.5, 20)
    R, M = 600, 5
    sums = []
    for seed in range(1, M + 1):
        rng = np.random.default_rng(200 + seed)
        # bond length density ~ r^2 exp(-a (r - r0)^2) at T0 = 2, by rejection
        a = 0.5 * k / 2
        lens = []
        while len(lens) < R * (n - 1):
            r = rng.normal(r0, 1 / math.sqrt(2 * a), 20000)
            r = r[r > 0]
            keep = rng.random(len(r)) < (r / (r0 + 6 / math.sqrt(2 * a))) ** 2
            lens.extend(r[keep].tolist())
        lens = np.array(lens[:R * (n - 1)]).reshape(R, n - 1)
        dirs = rng.normal(size=(R, n - 1, 3))
        dirs /= np.linalg.norm(dirs, axis=2, keepdims=True)
        x0 = np.zeros((R, n, 3))
        x0[:, 1:] = np.cumsum(dirs * lens[..., None], axis=1)
        res = O.anneal(sysd, R, 2.0, sched, theta=100, theta_eq=100, dt=0.002, nu=1.0,
                       seed=seed, x0=np.ascontiguousarray(x0))
        sums.append(res.sum_lnQ)
    mean, se = np.mean(sums), np.std(sums, ddof=1) / math.sqrt(M)
    assert abs(mean - exact) < 3 * se + 0.01, (mean, se, exact)


def test_observables_definitions():
    E = np.array([1.0, 2.0, 4.0])
    K = np.array([3.0, 3.0, 6.0])
    o = O.observables(E, K, np.array([0, 0, 2]), n_atoms=2, kB=2.0, T=1.5)
    assert o["E_mean"] == pytest.approx(7 / 3)
    # <E^2> = (1 + 4 + 16) / 3 = 7; population variance 7 - 49/9 = 14/9;
    # Cv / kB = var / (kB T)^2 = (14/9) / 3^2 (step 4: population averages)
    assert o["E2_mean"] == pytest.approx(7.0)
    assert o["Cv"] == pytest.approx(14.0 / 81.0)
    assert o["K_mean"] == pytest.approx(4.0)
    assert o["T_measured"] == pytest.approx(2 * 4.0 / (3 * 2 * 2.0))
    assert o["families"] == 2
