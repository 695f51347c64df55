"""GPU: the hot path at the size and launch shape of the headline workload
(75-atom peptide, R = 1e5 replicas, FP32, 16 waves per CU, one persistent
launch over every CU), against the FP64 oracle, through the C ABI.

The oracle cannot advance 1e5 replicas in seconds, so MD is compared on
sampled replicas (the first and last slots, slots at wave and work-item
boundaries, the slots of the partial last round of work items, random ones):
the oracle advances each from the same start with the Philox counters of its
own slot.  Work that is O(R) on the host is compared for every replica.

* PAMD step 1: initial velocities of sampled slots within 1e-6 relative
  (FP32 storage of the same Maxwell-Boltzmann draws);
* PAMD step 3: 100 NVT steps, positions within 1e-4 nm, E_pot / E_kin within
  1e-3 relative, for the sampled slots; for every slot: finite state, step
  counter, E_kin equal to 1/2 m v^2 of the returned velocities (1e-12
  relative: FP64 sums of the same FP32 values in another order), ancestors
  kept;
* PAMD step 2: the adaptive temperature within 1e-9 relative of the oracle's
  bisection; with the oracle's temperature requested explicitly, every copy
  number bit-exact, ancestors and energies of the gathered population exact,
  sampled positions recentred within 2e-6 nm, ln Q within 1e-12 relative;
* the batched workload (eight peptides, R = 4096 each, wide layout): 100 NVT
  steps of sampled slots of every run, same tolerances as above.
"""
import math

import numpy as np
import pytest

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

from oracle import oracle as O  # noqa: E402
from pamd_inputs import systems as S  # noqa: E402
from pamd_inputs.precision import as_stored  # noqa: E402

R = 100_000
T0, DT, NU, SEED = 700.0, 0.001, 1.0, 1806


@pytest.fixture(scope="module")
def B():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1806_06016_amd import pamd
    pamd.load_library()
    return pamd


@pytest.fixture(scope="module")
def sysd():
    return S.c2_system()


def _sample_slots():
    rng = np.random.default_rng(99)
    # 4 replicas per wave, 16 waves per CU: work items of 4 slots; R / 4 =
    # 25000 items over 4096 resident waves leaves a partial last round
    edges = [0, 1, 2, 3, 4, 63, 64, 4095, 4096, 4097, 16383, 16384, 50001, 98303, 98304]
    tail = list(range(R - 6, R))
    return np.unique(np.r_[edges, tail, rng.choice(R, 17, replace=False)]).astype(np.int64)


def _ctx(B, sysd, **kw):
    p = B.Pamd([sysd], R_target=R, T0=T0, dt=DT, nu=NU, seed=SEED, precision=B.PAMD_FP32, waves_per_block=16,
               **kw)
    info = p.launch_info()
    print("launch", info, flush=True)
    assert info["waves_per_block"] == 16
    return p


def test_initial_velocities_sampled(B, sysd):
    p = _ctx(B, sysd)
    st = p.get_state(0)
    slots = _sample_slots()
    vo = O.init_velocities(O.OracleSystem(sysd), len(slots), T0, seed=SEED, slots=slots)
    rel = np.abs(st["v"][slots] - vo).max() / np.abs(vo).max()
    print("max relative velocity difference", rel)
    assert rel < 1e-6
    assert st["R"] == R and np.isfinite(st["v"]).all()
    p.close()


def test_md_sampled_and_whole_population_properties(B, sysd):
    p = _ctx(B, sysd)
    rng = np.random.default_rng(11)
    x = np.ascontiguousarray(sysd.x_init[None] + rng.normal(0, 0.003, (R,) + sysd.x_init.shape))
    sd = np.sqrt(sysd.kB * T0 / sysd.mass)[None, :, None]
    v = np.ascontiguousarray(rng.normal(size=x.shape) * sd)
    p.set_state(0, x, v, T=T0, step=500, ancestor=np.arange(R))
    xo, vo = as_stored(x, True), as_stored(v, True)
    del x, v
    n_steps = 100
    print("MD at R = 1e5", flush=True)
    p.md_steps(n_steps)
    g = p.get_state(0)
    assert g["step"] == 500 + n_steps and g["R"] == R
    assert np.isfinite(g["x"]).all() and np.isfinite(g["v"]).all() and np.isfinite(g["E_pot"]).all()
    assert (g["ancestor"] == np.arange(R)).all()
    ek = 0.5 * (sysd.mass[None, :] * (g["v"].astype(np.float64) ** 2).sum(-1)).sum(-1)
    assert np.abs(g["E_kin"] - ek).max() <= 1e-12 * np.abs(ek).max()
    slots = _sample_slots()
    xs, vs = np.ascontiguousarray(xo[slots]), np.ascontiguousarray(vo[slots])
    Ep, Ek, col = O.md_steps(O.OracleSystem(sysd), xs, vs, n_steps, T0, DT, NU, SEED, step0=500, slots=slots,
                             want_collisions=True)
    err = np.abs(g["x"][slots] - xs).max()
    print(f"sampled slots {len(slots)}: max |dx| {err:.2e}, collisions {int(col.sum())}")
    assert col.sum() > 0
    assert err < 1e-4
    assert np.abs(g["E_pot"][slots] - Ep).max() <= 1e-3 * np.abs(Ep).mean()
    assert np.allclose(g["E_kin"][slots], Ek, rtol=1e-3)
    p.close()


def _energies(sysd):
    # thermal spread of the peptide's 219 quadratic degrees of freedom at T0
    return np.random.default_rng(5).gamma(219 / 2, sysd.kB * T0, R) - 800.0


def _population(p, sysd, E):
    rng = np.random.default_rng(6)
    x = np.ascontiguousarray(sysd.x_init[None] + rng.normal(0, 0.01, (R,) + sysd.x_init.shape))
    v = rng.normal(size=x.shape)
    p.set_state(0, x, v, T=T0, E_pot=E, ancestor=np.arange(R))
    return as_stored(x, True), as_stored(v, True)


def test_adaptive_temperature_at_full_population(B, sysd):
    E = _energies(sysd)
    p = _ctx(B, sysd, T_final=250.0, V_target=0.1)
    _population(p, sysd, E)
    p.resample(None)
    g = p.get_state(0, want_xv=False)
    kB = sysd.kB
    db = O.adaptive_dbeta(E, 1 / (kB * 250.0) - 1 / (kB * T0), 0.1)
    To = 1 / (kB * (db + 1 / (kB * T0)))
    print("adaptive T", g["T"], "oracle", To)
    assert abs(g["T"] - To) <= 1e-9 * To
    p.close()


def test_copy_numbers_and_gather_at_full_population(B, sysd):
    E = _energies(sysd)
    kB = sysd.kB
    db = O.adaptive_dbeta(E, 1 / (kB * 250.0) - 1 / (kB * T0), 0.1)
    T1 = 1 / (kB * (db + 1 / (kB * T0)))
    db = 1 / (kB * T1) - 1 / (kB * T0)
    p = _ctx(B, sysd)
    xo, vo = _population(p, sysd, E)
    p.resample([T1])
    c = p.get_counts(0)
    u = O.resample_uniforms(R, 1, seed=SEED)
    co, tau = O.copy_counts(E, db, R, u)
    mism = np.nonzero(c != co)[0]
    assert len(mism) == 0, (len(mism), mism[:5])
    g = p.get_state(0)
    assert g["R"] == co.sum()
    _, _, _, lq = O.lse(E, db)
    assert abs(g["lnQ_last"] - lq) <= 1e-12 * max(1.0, abs(lq))
    src, Eo = O.gather(co, [np.arange(R), E])  # the source slot of every new slot
    assert (g["ancestor"] == src).all() and (g["E_pot"] == Eo).all()
    rows = np.unique(np.r_[0, len(src) - 1, np.random.default_rng(7).choice(len(src), 20, replace=False)])
    xr = O.recentre(np.ascontiguousarray(xo[src[rows]]), sysd.mass)
    assert np.abs(g["x"][rows] - xr).max() < 2e-6
    assert np.abs(g["v"][rows] - vo[src[rows]] * math.sqrt(T1 / T0)).max() < 1e-6 * np.abs(vo).max()
    print("families", p.observables()[0]["families"], "R", g["R"])
    p.close()


def test_batched_workload_sampled(B):
    """The batched workload as timed (eight peptides of 40-300 atoms, R = 4096
    each, 0.5 fs, one persistent wide launch with the default launch shape):
    100 NVT steps, sampled slots of every run against the oracle (Philox key
    of that run), every slot's state checked by properties."""
    syss = S.c4_systems()
    Rb, dt = 4096, 0.0005
    p = B.Pamd(syss, R_target=Rb, T0=T0, dt=dt, nu=NU, seed=SEED, precision=B.PAMD_FP32)
    print("launch", p.launch_info(), flush=True)
    starts = []
    for r, sysd in enumerate(syss):
        rng = np.random.default_rng(40 + r)
        x = np.ascontiguousarray(sysd.x_init[None] + rng.normal(0, 0.003, (Rb,) + sysd.x_init.shape))
        v = np.ascontiguousarray(rng.normal(size=x.shape) * np.sqrt(sysd.kB * T0 / sysd.mass)[None, :, None])
        p.set_state(r, x, v, T=T0, step=500)
        starts.append((as_stored(x, True), as_stored(v, True)))
    n_steps = 100
    p.md_steps(n_steps)
    rng = np.random.default_rng(41)
    for r, sysd in enumerate(syss):
        g = p.get_state(r)
        assert g["step"] == 500 + n_steps and g["R"] == Rb
        assert np.isfinite(g["x"]).all() and np.isfinite(g["E_pot"]).all()
        ek = 0.5 * (sysd.mass[None, :] * (g["v"].astype(np.float64) ** 2).sum(-1)).sum(-1)
        assert np.abs(g["E_kin"] - ek).max() <= 1e-12 * np.abs(ek).max()
        slots = np.unique(np.r_[0, 1, 63, 64, Rb - 1, rng.choice(Rb, 5, replace=False)]).astype(np.int64)
        xo, vo = starts[r]
        xs, vs = np.ascontiguousarray(xo[slots]), np.ascontiguousarray(vo[slots])
        Ep, Ek = O.md_steps(O.OracleSystem(sysd), xs, vs, n_steps, T0, dt, NU, SEED, step0=500, run=r,
                            slots=slots)
        err = np.abs(g["x"][slots] - xs).max()
        print(f"run {r} n={sysd.n_atoms}: max |dx| {err:.2e}")
        assert err < 1e-4
        assert np.abs(g["E_pot"][slots] - Ep).max() <= 1e-3 * np.abs(Ep).mean()
        assert np.allclose(g["E_kin"][slots], Ek, rtol=1e-3)
    p.close()


def test_million_replica_population(B, sysd):
    """R = 2^20 + 7 (ten times the headline population, ragged): the
    multi-block reductions loop over more blocks than a pass launches and the
    slab offsets pass 2^31 bytes.  Sampled initial velocities and 20 NVT steps
    against the oracle; then resampling of host-built energies: the adaptive
    temperature against the oracle's bisection, and at the oracle's
    temperature every copy number bit-exact, the gathered ancestors and
    energies exact."""
    Rm = (1 << 20) + 7
    kB = sysd.kB
    p = B.Pamd([sysd], R_target=Rm, T0=T0, dt=DT, nu=NU, seed=SEED, precision=B.PAMD_FP32, waves_per_block=16,
               T_final=250.0, V_target=0.1)
    slots = np.unique(np.r_[0, 1, 4095, 4096, (1 << 19) + 3, Rm - 8, Rm - 1,
                            np.random.default_rng(3).choice(Rm, 9, replace=False)]).astype(np.int64)
    st = p.get_state(0)
    osys = O.OracleSystem(sysd)
    vo = O.init_velocities(osys, len(slots), T0, seed=SEED, slots=slots)
    assert np.abs(st["v"][slots] - vo).max() <= 1e-6 * np.abs(vo).max()
    x0 = np.ascontiguousarray(np.broadcast_to(sysd.x_init, (len(slots),) + sysd.x_init.shape))
    xs, vs = as_stored(x0, True), as_stored(vo, True)
    del st
    print("MD at R = 2^20 + 7", flush=True)
    p.md_steps(20)
    g = p.get_state(0)
    assert g["R"] == Rm and g["step"] == 20 and np.isfinite(g["x"]).all() and np.isfinite(g["E_pot"]).all()
    O.md_steps(osys, xs, vs, 20, T0, DT, NU, SEED, step0=0, slots=slots)
    err = np.abs(g["x"][slots] - xs).max()
    print("sampled max |dx|", err, flush=True)
    assert err < 1e-4
    # resampling of host-built energies (the thermal spread of the peptide at T0):
    # the adaptive temperature, then (population restored) the copy numbers at
    # the oracle's temperature requested explicitly
    E = np.random.default_rng(8).gamma(219 / 2, kB * T0, Rm) - 800.0
    db = O.adaptive_dbeta(E, 1 / (kB * 250.0) - 1 / (kB * T0), 0.1)
    To = 1 / (kB * (db + 1 / (kB * T0)))
    p.set_state(0, g["x"], g["v"], T=T0, E_pot=E, ancestor=np.arange(Rm))
    p.resample(None)
    h = p.get_state(0, want_xv=False)
    print("adaptive T", h["T"], "oracle", To, flush=True)
    assert abs(h["T"] - To) <= 1e-9 * To
    p.set_state(0, g["x"], g["v"], T=T0, E_pot=E, ancestor=np.arange(Rm))
    del g
    p.resample([To])
    h = p.get_state(0, want_xv=False)
    db = 1 / (kB * To) - 1 / (kB * T0)
    c = p.get_counts(0)
    co, _ = O.copy_counts(E, db, Rm, O.resample_uniforms(Rm, 1, seed=SEED))
    mism = np.nonzero(c != co)[0]
    assert len(mism) == 0, (len(mism), mism[:5])
    src, Eo = O.gather(co, [np.arange(Rm), E])
    assert h["R"] == co.sum() and (h["ancestor"] == src).all() and (h["E_pot"] == Eo).all()
    print("R after resampling", h["R"], "families", p.observables()[0]["families"])
    p.close()
