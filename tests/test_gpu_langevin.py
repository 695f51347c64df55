"""GPU: the Langevin bath (B-A-O-A-B velocity Verlet, friction gamma, noise
from Philox stream 5 per replica slot) against the FP64 oracle, through the
C ABI.

Tolerances as for the Andersen bath: positions within 1e-4 nm after 100 steps
in FP32 (identical noise streams on both sides), 1e-8 in FP64; energies and
kinetic energies 1e-3 relative in FP32 and 1e-9 in FP64.  Properties that hold
at any size: exact configurational variance of the harmonic chain at a large
step, equal <E_pot>(T) along a whole anneal with the same seeds.
"""
import math

import numpy as np
import pytest

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

from oracle import oracle as O  # noqa: E402
from pamd_inputs import systems as S  # noqa: E402
from pamd_inputs.precision import as_stored  # noqa: E402


@pytest.fixture(scope="module")
def B():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1806_06016_amd import pamd
    pamd.load_library()
    return pamd


def _perturbed(sysd, R, scale, seed):
    rng = np.random.default_rng(seed)
    return np.ascontiguousarray(sysd.x_init[None] + rng.normal(0, scale, size=(R,) + sysd.x_init.shape))


@pytest.mark.parametrize("which,prec,tol", [("peptide", 1, 1e-4), ("chain", 0, 1e-8), ("chain", 1, 1e-4),
                                            ("wide120", 1, 1e-4)])
def test_langevin_trajectory_matches_oracle(B, which, prec, tol):
    if which == "chain":
        sysd, T, gamma, dt, scale = S.c1_system(), 1.3, 5.0, 0.002, 0.05
    elif which == "peptide":
        sysd, T, gamma, dt, scale = S.c2_system(), 700.0, 1.0, 0.001, 0.005
    else:
        sysd, T, gamma, dt, scale = S.make_peptide(1807, 120), 700.0, 1.0, 0.0005, 0.003
    R, n_steps = 29, 100
    print(f"langevin trajectory {which} prec={prec}", flush=True)
    p = B.Pamd([sysd], R_target=R, T0=T, dt=dt, nu=gamma, seed=91, precision=prec, thermostat="langevin")
    osys = O.OracleSystem(sysd)
    x = _perturbed(sysd, R, scale, 4)
    v = O.init_velocities(osys, R, T, seed=6)
    p.set_state(0, x, v, T=T, step=300)
    xo, vo = as_stored(x, prec), as_stored(v, prec)
    st = p.get_state(0)
    assert np.array_equal(st["x"], xo) and np.array_equal(st["v"], vo)
    p.md_steps(n_steps)
    g = p.get_state(0)
    Ep, Ek = O.md_steps(osys, xo, vo, n_steps, T, dt, gamma, 91, step0=300, thermostat="langevin")
    err = np.abs(g["x"] - xo).max()
    print(f"max |dx| {err:.2e}")
    assert err < tol
    assert g["step"] == 300 + n_steps
    assert np.abs(g["E_pot"] - Ep).max() <= (1e-3 if prec else 1e-9) * np.abs(Ep).mean()
    assert np.allclose(g["E_kin"], Ek, rtol=1e-3 if prec else 1e-9)
    p.close()


def test_langevin_harmonic_chain_samples_configurations_exactly(B):
    """FP64 zero-rest-length chain (k = 100, unit masses) at omega_max dt = 1.6:
    <|b|^2> = 3 kB T / k per bond within 1 %."""
    sysd = S.gaussian_chain(10, 100.0, 0.0)
    R, T, dt = 4000, 1.0, 0.08
    rng = np.random.default_rng(1)
    b = rng.normal(0, math.sqrt(T / 100.0), (R, 9, 3))
    x = np.zeros((R, 10, 3))
    x[:, 1:] = np.cumsum(b, axis=1)
    p = B.Pamd([sysd], R_target=R, T0=T, dt=dt, nu=5.0, seed=7, precision=0, thermostat="langevin")
    st = p.get_state(0)
    p.set_state(0, np.ascontiguousarray(x), st["v"], T=T)
    ratios = []
    for blk in range(16):
        p.md_steps(50)
        if blk >= 4:
            xx = p.get_state(0)["x"]
            ratios.append((np.diff(xx, axis=1) ** 2).sum(-1).mean() / (3 * T / 100.0))
    print("ratio", np.mean(ratios))
    assert abs(np.mean(ratios) - 1) < 0.01
    p.close()


def test_langevin_anneal_identical_seeds(B):
    """A whole FP64 PA run of the bead chain with the Langevin bath: <E_pot> at
    every temperature and sum ln Q equal the oracle's."""
    sysd = S.c1_system()
    sched = S.geometric_schedule(2.0, 0.5, 10)
    R = 200
    for seed in (1, 2):
        p = B.Pamd([sysd], R_target=R, T0=2.0, dt=0.002, nu=2.0, seed=seed, precision=0, thermostat="langevin")
        p.md_steps(300)
        E = [p.observables()[0]["E_mean"]]
        for T in sched[1:]:
            p.resample([T])
            p.md_steps(100)
            E.append(p.observables()[0]["E_mean"])
        lnq = p.observables()[0]["sum_lnQ"]
        p.close()
        res = O.anneal(sysd, R, 2.0, sched, theta=100, theta_eq=300, dt=0.002, nu=2.0, seed=seed,
                       thermostat="langevin")
        Eo = np.array([o["E_mean"] for o in res.obs])
        print("seed", seed, "max rel dE", np.max(np.abs(np.array(E) - Eo) / np.abs(Eo)))
        assert np.allclose(E, Eo, rtol=1e-6, atol=1e-8)
        assert abs(lnq - res.sum_lnQ) < 1e-7


def test_langevin_with_the_surrogate_is_rejected(B):
    sysd = S.c2_system()
    nn = B.PamdNN(sysd, sysd.atype)
    p = B.Pamd([sysd], R_target=16, T0=700.0, dt=0.001, nu=1.0, seed=1, precision=B.PAMD_FP32,
               thermostat="langevin")
    with pytest.raises(B.PamdError) as e:
        p.set_mts(nn, 4)
    assert e.value.code == B.PAMD_ERR_ARG
    p.md_steps(5)
    p.close()
    nn.close()
