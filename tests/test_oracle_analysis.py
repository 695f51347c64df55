"""Pins of the oracle's population analysis (CPU only): family and binning
errors over a resampled population, family statistics, and the
multiple-histogram (WHAM) refinement of the free energies.

Pins: hand-computed tiny cases, the singleton-family and bin-size-one
reductions to the naive error, the exact finite-sample relation between
family and binning errors for equal contiguous families, the expectation of
the family error over many synthetic populations with perfectly correlated
copies, and WHAM on exact Boltzmann samples of a harmonic system whose
partition function is known in closed form (ln Z = -(d/2) ln beta + const).
"""
import math

import numpy as np

from oracle import analysis as A


def test_tiny_case_by_hand():
    # O = 1, 2, 4, 9 with ancestors 5, 5, 5, 7: mean 4, deviations -3, -2, 0, 5,
    # family sums -5 and 5; R (R - 1) = 12
    r = A.family_error(np.array([1.0, 2.0, 4.0, 9.0]), np.array([5, 5, 5, 7]))
    assert r["mean"] == 4.0
    assert abs(r["naive_se"] - math.sqrt(38.0 / 12.0)) < 1e-15
    assert abs(r["family_se"] - math.sqrt(50.0 / 12.0)) < 1e-15
    assert r["families"] == 2
    # nu = 3/4, 1/4: rho_t = 4 (9/16 + 1/16) = 2.5
    assert abs(r["rho_t"] - 2.5) < 1e-15
    assert abs(r["family_entropy"] - (-(0.75 * math.log(0.75) + 0.25 * math.log(0.25)))) < 1e-15


def test_singleton_families_and_unit_bins_are_the_naive_error():
    O = np.random.default_rng(1).normal(3.0, 2.0, 999)
    r = A.family_error(O, np.arange(999))
    assert abs(r["family_se"] / r["naive_se"] - 1) < 1e-13
    assert abs(A.binning_error(O, 1) / r["naive_se"] - 1) < 1e-13
    assert abs(r["rho_t"] - 1.0) < 1e-13 and abs(math.exp(r["family_entropy"]) - 999) < 1e-9


def test_equal_contiguous_families_relate_family_and_binning_errors():
    """F families of n consecutive copies: family_se^2 / binning_se(n)^2 =
    n (F - 1) / (n F - 1), and rho_t = n, exp(S_f) = F."""
    F, n = 50, 8
    rng = np.random.default_rng(2)
    O = rng.normal(0, 1, F * n)
    anc = np.repeat(rng.permutation(1000)[:F], n)
    r = A.family_error(O, anc)
    ratio = r["family_se"] ** 2 / A.binning_error(O, n) ** 2
    assert abs(ratio - n * (F - 1) / (n * F - 1)) < 1e-12
    assert abs(r["rho_t"] - n) < 1e-12 and abs(math.exp(r["family_entropy"]) - F) < 1e-9


def test_family_error_has_the_right_expectation_for_correlated_copies():
    """Populations of F families, each n identical copies of an N(0, 1) value
    (the extreme correlation resampling can create): Var(mean) = 1 / F.  Over
    4000 populations the average family variance estimate is within 5 % of
    it, while the naive estimate is ~n times too small."""
    F, n, trials = 40, 6, 4000
    rng = np.random.default_rng(3)
    fam, nai = [], []
    for _ in range(trials):
        O = np.repeat(rng.normal(0, 1, F), n)
        r = A.family_error(O, np.repeat(np.arange(F), n))
        fam.append(r["family_se"] ** 2)
        nai.append(r["naive_se"] ** 2)
    # E[family_se^2] = (F - 1) / F * n F / (n F - 1) / F for this estimator
    expect = (F - 1) / F * (n * F) / (n * F - 1) / F
    assert abs(np.mean(fam) / expect - 1) < 0.05
    assert abs(expect * F - 1) < 0.03
    assert np.mean(nai) < 0.3 * np.mean(fam)


def _gamma_samples(betas, N, d, seed):
    """N samples per temperature, or N[l] at temperature l."""
    rng = np.random.default_rng(seed)
    Ns = [N] * len(betas) if np.isscalar(N) else N
    return [rng.gamma(d / 2, 1.0 / b, n) for b, n in zip(betas, Ns)]


def test_wham_recovers_the_harmonic_partition_function():
    """d = 27 quadratic degrees of freedom (the Gaussian chain's U): U ~
    Gamma(d/2, 1/beta), ln Z(beta) - ln Z(beta_0) = -(d/2) ln(beta/beta_0).
    From a flat start WHAM converges to it within 0.05 over a total change of
    18.7 (the spread over seeds is ~0.01).  Sample counts differ between
    temperatures (500 ... 3000), as population sizes do."""
    betas = 1.0 / (2.0 * 0.25 ** (np.arange(21) / 20))
    d = 27
    exact = -(d / 2) * np.log(betas / betas[0])
    counts = [500 + 125 * l for l in range(21)]
    for seed in (1, 2):
        S = _gamma_samples(betas, counts, d, seed)
        lnZ, it = A.wham(betas, S, np.zeros(21), tol=1e-9)
        assert it < 1000
        assert np.abs(lnZ - lnZ[0] - exact).max() < 0.05, np.abs(lnZ - exact).max()
        # a further iteration from the converged values moves nothing
        lnZ2, it2 = A.wham(betas, S, lnZ, tol=1e-9)
        assert it2 <= 2 and np.abs(lnZ2 - lnZ).max() < 1e-8
        # reweighting to temperatures between the grid points: <U> = d / (2 beta)
        for bq in (0.5 * (betas[3] + betas[4]), 0.5 * (betas[15] + betas[16])):
            Em, E2m = A.wham_average(bq, betas, S, lnZ)
            assert abs(Em * bq / (d / 2) - 1) < 0.01
            assert abs((E2m - Em * Em) * bq * bq / (d / 2) - 1) < 0.1


def test_wham_with_one_temperature_keeps_its_start():
    S = _gamma_samples([1.0], 500, 27, 4)
    lnZ, it = A.wham([1.0], S, [3.25])
    assert lnZ[0] == 3.25 and it == 1
