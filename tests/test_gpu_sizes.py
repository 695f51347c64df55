"""GPU: molecule sizes at the edges of both layouts, against the FP64 oracle,
through the C ABI.

The register tiles hold 16-atom blocks (1 to 5 of them, at most 80 atoms); a
context with a larger molecule switches to the wide layout (64 lanes per
replica, up to 320 atoms).  Sizes: a single atom (no interaction at all), one
pair, a full block, a full block plus one atom (a one-atom ragged block), the
FP64 limit of 32, the 48- and 64-atom boundaries, the register-tile maximum
of 80, the first wide size 81 and the wide maximum 320.  Bead chains (vacuum
1/r Coulomb, reduced units) cover the small sizes in FP64 and FP32, peptides
(distance-dependent dielectric) the larger ones.  Same tolerances as the other
parity tests: per-atom forces within tol (|F_a| + F_rms), energies within
tolE of sum |terms|, positions after 100 NVT steps with identical Philox
streams within 1e-8 (FP64) / 1e-4 (FP32, nm or reduced units).  Sizes out of
range are rejected on the host (test_abi).
"""
import functools

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


@functools.lru_cache(maxsize=None)
def _system(kind, n):
    if kind == "chain":
        return S.bead_chain(n, seed=n)
    return S.make_peptide(seed=2000 + n, n_atoms=n)


# (kind, n_atoms, precision)
CASES = [("chain", 1, 0), ("chain", 2, 0), ("chain", 16, 0), ("chain", 17, 0), ("chain", 32, 0),
         ("chain", 1, 1), ("chain", 2, 1), ("chain", 16, 1), ("chain", 17, 1),
         ("peptide", 33, 1), ("peptide", 48, 1), ("peptide", 64, 1), ("peptide", 80, 1),
         ("peptide", 81, 1), ("peptide", 320, 1)]


def _conditions(sysd):
    # (T, dt, collision frequency, start perturbation)
    if sysd.units == "reduced":
        return 1.3, 0.002, 5.0, 0.05
    return 700.0, 0.0005, 2.0, 0.003


def _perturbed(sysd, R, scale, seed):
    rng = np.random.default_rng(seed)
    return np.ascontiguousarray(sysd.x_init[None] + rng.normal(0, scale, size=(R,) + sysd.x_init.shape))


@pytest.mark.parametrize("kind,n,prec", CASES)
def test_forces_and_energies(B, kind, n, prec):
    sysd = _system(kind, n)
    R = 9                                   # ragged against the replicas per wave
    T, dt, nu, _ = _conditions(sysd)
    print(f"forces {kind} n={n} prec={prec}", flush=True)
    p = B.Pamd([sysd], R_target=R, T0=T, dt=dt, nu=nu, seed=5, precision=prec)
    print("launch", p.launch_info())
    x = _perturbed(sysd, R, 0.1 if kind == "chain" else 0.01, 11)
    p.set_state(0, x, np.zeros_like(x), T=T)
    xs = as_stored(x, prec)
    assert np.array_equal(p.get_state(0)["x"], xs)
    F, E = p.get_forces(0)
    Eo, Fo, terms = O.energy_forces(O.OracleSystem(sysd), xs, want_terms=True)
    tolF, tolE = (1e-9, 1e-10) if prec == 0 else (1e-4, 1e-5)
    if n == 1:
        assert np.all(F == 0) and np.all(E == 0)
    else:
        frms = np.sqrt((Fo ** 2).sum(-1).mean(-1))[:, None]
        ratio = (np.linalg.norm(F - Fo, axis=-1) / (tolF * (np.linalg.norm(Fo, axis=-1) + frms))).max()
        print(f"force error / bound {ratio:.3f}")
        assert ratio <= 1.0
        assert np.all(np.abs(E - Eo) <= tolE * np.abs(terms).sum(1))
    p.close()


@pytest.mark.parametrize("kind,n,prec", CASES)
def test_trajectory(B, kind, n, prec):
    sysd = _system(kind, n)
    R, n_steps, seed = 9, 100, 41
    T, dt, nu, scale = _conditions(sysd)
    print(f"trajectory {kind} n={n} prec={prec}", flush=True)
    p = B.Pamd([sysd], R_target=R, T0=T, dt=dt, nu=nu, seed=seed, precision=prec)
    osys = O.OracleSystem(sysd)
    x = _perturbed(sysd, R, scale, 13)
    v = O.init_velocities(osys, R, T, seed=17)
    p.set_state(0, x, v, T=T, step=200)
    xo, vo = as_stored(x, prec).copy(), as_stored(v, prec).copy()
    st = p.get_state(0)
    assert np.array_equal(st["x"], xo) and np.array_equal(st["v"], vo)
    p.md_steps(n_steps)
    g = p.get_state(0)
    Ep, Ek, col = O.md_steps(osys, xo, vo, n_steps, T, dt, nu, seed, step0=200, want_collisions=True)
    err = np.abs(g["x"] - xo).max()
    print(f"max |dx| {err:.2e}, collisions {int(col.sum())}")
    assert col.sum() > 0
    assert err < (1e-8 if prec == 0 else 1e-4)
    assert g["step"] == 200 + n_steps
    assert np.abs(g["E_pot"] - Ep).max() <= (1e-9 if prec == 0 else 1e-3) * max(1.0, np.abs(Ep).mean())
    assert np.allclose(g["E_kin"], Ek, rtol=1e-9 if prec == 0 else 1e-3)
    p.close()



def test_register_tile_runs_of_different_sizes(B):
    """One context, three runs of 33, 64 and 75 atoms (all within the register
    tiles, so each run launches its own block count): 100 NVT steps of every
    run against the oracle with that run's Philox key, then one resampling
    step per run with its own temperature from host-given energies (copy
    numbers bit-exact)."""
    syss = [_system("peptide", n) for n in (33, 64)] + [S.c2_system()]
    R, n_steps, seed = 9, 100, 43
    T, dt, nu, scale = 700.0, 0.0005, 2.0, 0.003
    p = B.Pamd(syss, R_target=R, T0=T, dt=dt, nu=nu, seed=seed, precision=B.PAMD_FP32)
    starts = []
    for r, sysd in enumerate(syss):
        osys = O.OracleSystem(sysd)
        x = _perturbed(sysd, R, scale, 50 + r)
        v = O.init_velocities(osys, R, T, seed=60 + r)
        p.set_state(r, x, v, T=T, step=200)
        starts.append((as_stored(x, True).copy(), as_stored(v, True).copy()))
    p.md_steps(n_steps)
    for r, sysd in enumerate(syss):
        xo, vo = starts[r]
        Ep, Ek = O.md_steps(O.OracleSystem(sysd), xo, vo, n_steps, T, dt, nu, seed, step0=200, run=r)
        g = p.get_state(r)
        err = np.abs(g["x"] - xo).max()
        print(f"run {r} n={sysd.n_atoms}: max |dx| {err:.2e}")
        assert err < 1e-4 and g["step"] == 200 + n_steps
        assert np.abs(g["E_pot"] - Ep).max() <= 1e-3 * np.abs(Ep).mean()
    # resampling from host-given energies (the oracle never takes device output)
    temps = [690.0, 680.0, 670.0]
    E = []
    for r, sysd in enumerate(syss):
        E.append(np.random.default_rng(70 + r).normal(-300.0, 15.0, R))
        xo, vo = starts[r]
        p.set_state(r, xo, vo, T=T, E_pot=E[r], ancestor=np.arange(R))
    p.resample(temps)
    for r, sysd in enumerate(syss):
        db = 1 / (sysd.kB * temps[r]) - 1 / (sysd.kB * T)
        u = O.resample_uniforms(R, 1, seed=seed, run=r)
        co, _ = O.copy_counts(E[r], db, R, u)
        assert (p.get_counts(r) == co).all()
    p.close()
