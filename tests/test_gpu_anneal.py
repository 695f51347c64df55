"""GPU: whole annealing runs against the oracle and against closed forms.

* <E_pot>(T) over whole anneals on the GPU and on the oracle, each side over
  M independently seeded runs, for the bead chain (FP64 end to end, 21
  temperatures) and for a reduced 75-atom peptide anneal on the FP32 path of
  the main workload (10 temperatures 700 -> 500 K).  The means of one run are
  correlated from one temperature to the next, so agreement "within 2 sigma"
  is tested with that correlation taken from the runs (energy_curve_stats):
  Hotelling's T^2 on the vector of mean differences, and the count of
  per-temperature z-scores beyond 2 and their largest modulus against their
  bootstrap null distributions; each p-value must exceed 0.01.
* Sum ln Q of the zero-rest-length Gaussian chain on the GPU against the exact
  13.5 ln(T_N / T_0), within 3 standard errors over M seeds, and its
  heat-capacity observable against the exact Cv / kB = 13.5.
"""
import math

import numpy as np
import pytest

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

from energy_curve_stats import compare_energy_curves, report  # noqa: E402
from oracle import oracle as O  # noqa: E402
from pamd_inputs import systems as S  # noqa: E402


@pytest.fixture(scope="module")
def B():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1806_06016_amd import pamd
    pamd.load_library()
    return pamd


def _gpu_anneal(B, sysd, R, sched, theta, theta_eq, dt, nu, seed, precision, x0=None, want_cv=False):
    p = B.Pamd([sysd], R_target=R, T0=sched[0], dt=dt, nu=nu, seed=seed, precision=precision)
    if x0 is not None:
        st = p.get_state(0)
        p.set_state(0, x0, st["v"], T=sched[0])
    p.md_steps(theta_eq)
    o = p.observables()[0]
    E, Cv, lnq = [o["E_mean"]], [o["Cv"]], 0.0
    for T in sched[1:]:
        p.resample([T])
        p.md_steps(theta)
        o = p.observables()[0]
        E.append(o["E_mean"])
        Cv.append(o["Cv"])
        lnq = o["sum_lnQ"]
    p.close()
    if want_cv:
        return np.array(E), lnq, np.array(Cv)
    return np.array(E), lnq


def test_bead_chain_energy_curve_matches_oracle(B):
    """Independent seeds on the two sides (GPU 1..16, oracle 101..116), 16 runs
    of 1500 replicas each, 21 temperatures."""
    sysd = S.c1_system()
    sched = S.geometric_schedule(2.0, 0.5, 20)
    M, R = 16, 1500
    print("bead chain anneal, 16 + 16 runs", flush=True)
    g = np.array([_gpu_anneal(B, sysd, R, sched, 100, 1000, 0.002, 1.0, s, 0)[0] for s in range(1, M + 1)])
    o = np.array([[ob["E_mean"] for ob in O.anneal(sysd, R, 2.0, sched, theta=100, theta_eq=1000, dt=0.002,
                                                     nu=1.0, seed=100 + s).obs] for s in range(1, M + 1)])
    res = compare_energy_curves(g, o)
    print(report(res))
    assert res["p_hotelling"] > 0.01 and res["p_count"] > 0.01 and res["p_max"] > 0.01


def test_peptide_fp32_energy_curve_matches_oracle(B):
    """The FP32 path of the main workload over a reduced anneal of the
    75-atom peptide: R = 300, 400 equilibration steps at 700 K, then 9
    geometric steps to 500 K (normalised weight variance ~0.2 per step, near
    the adaptive schedule's 0.1) with theta = 150 steps of 1 fs each
    (Andersen, nu = 1/ps); 10 runs per side with independent seeds (GPU
    1..10, oracle 201..210)."""
    sysd = S.c2_system()
    sched = S.geometric_schedule(700.0, 500.0, 9)
    M, R = 10, 300
    print("peptide FP32 anneal, 10 + 10 runs", flush=True)
    g = np.array([_gpu_anneal(B, sysd, R, sched, 150, 400, 0.001, 1.0, s, 1)[0] for s in range(1, M + 1)])
    o = []
    for s in range(1, M + 1):
        o.append([ob["E_mean"] for ob in O.anneal(sysd, R, 700.0, sched, theta=150, theta_eq=400, dt=0.001,
                                                   nu=1.0, seed=200 + s).obs])
        print("oracle run", s, "done", flush=True)
    res = compare_energy_curves(g, np.array(o))
    print(report(res))
    assert res["p_hotelling"] > 0.01 and res["p_count"] > 0.01 and res["p_max"] > 0.01


def test_bead_chain_full_anneal_identical_seeds(B):
    """Identical seeds: every run's <E_pot>(T) and sum ln Q over the whole
    21-temperature anneal equal the oracle's (FP64 on both sides).  Over 3100
    chaotic MD steps the two sides' rounding differences (fused multiply-adds,
    summation order) grow to ~1e-8 relative; a wrong copy number or step would
    move the energies by ~1e-2."""
    sysd = S.c1_system()
    sched = S.geometric_schedule(2.0, 0.5, 20)
    R = 256
    for seed in (1, 2, 3):
        E, lnq = _gpu_anneal(B, sysd, R, sched, 100, 1000, 0.002, 1.0, seed, 0)
        res = O.anneal(sysd, R, 2.0, sched, theta=100, theta_eq=1000, dt=0.002, nu=1.0, seed=seed)
        Eo = np.array([ob["E_mean"] for ob in res.obs])
        print("seed", seed, "max rel dE", np.max(np.abs(E - Eo) / np.abs(Eo)), "dlnQ", lnq - res.sum_lnQ)
        assert np.allclose(E, Eo, rtol=1e-6, atol=1e-8)
        assert abs(lnq - res.sum_lnQ) < 1e-7


def test_gaussian_chain_free_energy_on_gpu(B):
    sysd = S.gaussian_chain(10, 100.0, 0.0)
    sched = S.geometric_schedule(2.0, 0.5, 20)
    M, R = 6, 1000
    sums, cvs = [], []
    for seed in range(1, M + 1):
        rng = np.random.default_rng(300 + seed)
        b = rng.normal(0, math.sqrt(2.0 / 100.0), size=(R, 9, 3))
        x0 = np.zeros((R, 10, 3))
        x0[:, 1:] = np.cumsum(b, axis=1)
        _, lnq, cv = _gpu_anneal(B, sysd, R, sched, 100, 100, 0.002, 1.0, seed, 0, x0=x0, want_cv=True)
        sums.append(lnq)
        cvs.append(cv)
    exact = 13.5 * math.log(0.25)
    mean, se = np.mean(sums), np.std(sums, ddof=1) / math.sqrt(M)
    print("sum lnQ", mean, "+-", se, "exact", exact)
    assert abs(mean - exact) < 3 * se + 0.01
    # U ~ Gamma(13.5, T): Cv / kB = Var U / T^2 = 13.5 at every temperature
    cv = np.mean(cvs, axis=0) / 13.5
    print("Cv / 13.5", np.round(cv, 3))
    assert np.all(np.abs(cv - 1) < 0.12) and abs(cv.mean() - 1) < 0.03


@pytest.mark.parametrize("which", ["chain", "peptide"])
def test_anneal_identical_streams_matches_oracle(B, which):
    """Identical seeds: after equilibration and two temperature steps the GPU
    population equals the oracle's (same copy numbers, ancestors, positions)."""
    if which == "chain":
        sysd, prec, T = S.c1_system(), 0, [2.0, 1.9, 1.8]
        dt, theta, tol = 0.002, 50, 1e-7
    else:
        sysd, prec, T = S.c2_system(), 1, [700.0, 690.0, 680.0]
        dt, theta, tol = 0.001, 50, 2e-4
    R, seed = 200, 31
    p = B.Pamd([sysd], R_target=R, T0=T[0], dt=dt, nu=1.0, seed=seed, precision=prec)
    p.md_steps(theta)
    osys = O.OracleSystem(sysd)
    st = p.get_state(0)
    x = np.ascontiguousarray(np.broadcast_to(sysd.x_init, (R, sysd.n_atoms, 3)).astype(np.float64))
    v = O.init_velocities(osys, R, T[0], seed)
    Ep, Ek = O.md_steps(osys, x, v, theta, T[0], dt, 1.0, seed, 0)
    assert np.abs(st["x"] - x).max() < tol
    step = theta
    anc = np.arange(R)
    for i in (1, 2):
        p.resample([T[i]])
        p.md_steps(theta)
        g = p.get_state(0)
        kB = sysd.kB
        db = 1 / (kB * T[i]) - 1 / (kB * T[i - 1])
        u = O.resample_uniforms(len(Ep), i, seed)
        c, _ = O.copy_counts(Ep, db, R, u)
        assert (p.get_counts(0) == c).all()
        x, v, Ep, anc = O.gather(c, [x, v, Ep, anc])
        x = np.ascontiguousarray(O.recentre(x, osys.mass))
        v = np.ascontiguousarray(v * math.sqrt(T[i] / T[i - 1]))
        Ep, Ek = O.md_steps(osys, x, v, theta, T[i], dt, 1.0, seed, step)
        step += theta
        assert (g["ancestor"] == anc).all()
        err = np.abs(g["x"] - x).max()
        print(which, "temperature step", i, "max |dx|", err)
        assert err < tol
        assert np.abs(g["E_pot"] - Ep).max() < (1e-9 if prec == 0 else 1e-3) * np.abs(Ep).mean() + 1e-9
    p.close()
