"""GPU: the grouped bonded terms on a molecule that exercises every split of
the grouping (six-coordinated hubs: 15 angles per centre, more than four
outer atoms; 25 torsions around one bond, more than three outer atoms per
side; a second torsion term stacked on five quadruples), against the FP64
oracle through the C ABI, in the register-tile layout (FP64 and FP32) and in
the wide layout (batched with a 120-atom peptide); and the same molecule with
torsion multiplicities 1..6 (the derivative's recurrence path for n > 3).

Tolerances as for the other molecules: forces within 1e-9 (FP64) / 1e-4
(FP32) of (|F_a| + F_rms) per atom, energies within 1e-10 / 1e-5 of the sum of
|terms|, positions within 1e-8 / 1e-4 after 100 NVT steps.
"""
import dataclasses

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


def _check_forces(F, E, sysd, xs, prec):
    osys = O.OracleSystem(sysd)
    Eo, Fo, terms = O.energy_forces(osys, xs, want_terms=True)
    tolF, tolE = (1e-9, 1e-10) if prec == 0 else (1e-4, 1e-5)
    frms = np.sqrt((Fo ** 2).sum(-1).mean(-1))[:, None]
    ratio = (np.linalg.norm(F - Fo, axis=-1) / (tolF * (np.linalg.norm(Fo, axis=-1) + frms))).max()
    print("force error / bound", ratio)
    assert ratio <= 1.0
    assert np.all(np.abs(E - Eo) <= tolE * np.abs(terms).sum(1))


@pytest.mark.parametrize("prec", [0, 1])
def test_branched_forces_register_tiles(B, prec):
    sysd = S.branched_pair()
    R = 19
    p = B.Pamd([sysd], R_target=R, T0=1.0, dt=0.002, nu=1.0, seed=4, precision=prec)
    x = _perturbed(sysd, R, 0.05, 8)
    p.set_state(0, x, np.zeros_like(x), T=1.0)
    F, E = p.get_forces(0)
    _check_forces(F, E, sysd, as_stored(x, prec), prec)
    p.close()


def test_branched_forces_wide_layout(B):
    # one batched launch shares the dielectric model: the peptide's eps = 4r
    syss = [dataclasses.replace(S.branched_pair(), dielectric=S.DIELECTRIC_4R), S.make_peptide(1806 + 3, 120)]
    R = 11
    p = B.Pamd(syss, R_target=R, T0=1.0, dt=0.002, nu=1.0, seed=4, precision=B.PAMD_FP32)
    x = _perturbed(syss[0], R, 0.05, 9)
    p.set_state(0, x, np.zeros_like(x), T=1.0)
    F, E = p.get_forces(0)
    _check_forces(F, E, syss[0], as_stored(x, True), 1)
    p.close()


@pytest.mark.parametrize("prec,tol", [(0, 1e-8), (1, 1e-4)])
def test_branched_trajectory(B, prec, tol):
    sysd = S.branched_pair()
    R, T, nu, dt, n_steps = 23, 0.8, 2.0, 0.002, 100
    osys = O.OracleSystem(sysd)
    p = B.Pamd([sysd], R_target=R, T0=T, dt=dt, nu=nu, seed=12, precision=prec)
    x = _perturbed(sysd, R, 0.03, 3)
    v = O.init_velocities(osys, R, T, seed=5)
    p.set_state(0, x, v, T=T, step=40)
    xo, vo = as_stored(x, prec), as_stored(v, prec)
    p.md_steps(n_steps)
    Ep, Ek = O.md_steps(osys, xo, vo, n_steps, T, dt, nu, 12, step0=40)
    g = p.get_state(0)
    err = np.abs(g["x"] - xo).max()
    print("max |dx|", err)
    assert err < tol
    assert np.abs(g["E_pot"] - Ep).max() <= (1e-3 if prec else 1e-9) * max(1.0, np.abs(Ep).mean())
    p.close()


def _high_multiplicity(sysd):
    """The branched pair with torsion multiplicities cycling through 1..6 (the
    derivative's recurrence path for n > 3, the quadratic for n <= 3, in one
    molecule), phases alternating 0 / pi."""
    nd = len(sysd.dih_n)
    n = (np.arange(nd) % 6 + 1).astype(np.int32)
    delta = np.where(np.arange(nd) % 2 == 0, 0.0, np.pi)
    return dataclasses.replace(sysd, dih_n=n, dih_delta=delta)


@pytest.mark.parametrize("prec", [0, 1])
def test_high_multiplicity_torsions_register_tiles(B, prec):
    sysd = _high_multiplicity(S.branched_pair())
    assert sysd.dih_n.max() == 6
    R = 13
    p = B.Pamd([sysd], R_target=R, T0=1.0, dt=0.002, nu=1.0, seed=4, precision=prec)
    x = _perturbed(sysd, R, 0.05, 21)
    p.set_state(0, x, np.zeros_like(x), T=1.0)
    F, E = p.get_forces(0)
    _check_forces(F, E, sysd, as_stored(x, prec), prec)
    p.close()


def test_high_multiplicity_torsions_wide_layout(B):
    syss = [dataclasses.replace(_high_multiplicity(S.branched_pair()), dielectric=S.DIELECTRIC_4R),
            S.make_peptide(1806 + 3, 120)]
    R = 11
    p = B.Pamd(syss, R_target=R, T0=1.0, dt=0.002, nu=1.0, seed=4, precision=B.PAMD_FP32)
    x = _perturbed(syss[0], R, 0.05, 22)
    p.set_state(0, x, np.zeros_like(x), T=1.0)
    F, E = p.get_forces(0)
    _check_forces(F, E, syss[0], as_stored(x, True), 1)
    p.close()


def test_branched_vacuum_wide_layout_trajectory(B):
    """The branched pair (vacuum 1/r Coulomb) forced into the wide layout:
    forces, then 100 NVT steps with identical streams against the oracle (the
    wide kernel's vacuum instantiation)."""
    sysd = S.branched_pair()
    assert sysd.dielectric == S.DIELECTRIC_VACUUM
    R, T, nu, dt, n_steps = 17, 0.8, 2.0, 0.002, 100
    osys = O.OracleSystem(sysd)
    p = B.Pamd([sysd], R_target=R, T0=T, dt=dt, nu=nu, seed=12, precision=B.PAMD_FP32, layout="wide")
    assert p.run_launch(0)["layout"] == "wide"
    x = _perturbed(sysd, R, 0.03, 31)
    v = O.init_velocities(osys, R, T, seed=6)
    p.set_state(0, x, v, T=T, step=7)
    xo, vo = as_stored(x, True), as_stored(v, True)
    F, E = p.get_forces(0)
    _check_forces(F, E, sysd, xo, 1)
    p.md_steps(n_steps)
    Ep, Ek = O.md_steps(osys, xo, vo, n_steps, T, dt, nu, 12, step0=7)
    g = p.get_state(0)
    err = np.abs(g["x"] - xo).max()
    print("max |dx|", err)
    assert err < 1e-4
    assert np.abs(g["E_pot"] - Ep).max() <= 1e-3 * max(1.0, np.abs(Ep).mean())
    p.close()
