"""GPU parity of the HIP path against the FP64 oracle (needs an MI355X).

Every call goes through libpamd's C ABI.  Tolerances:
  * forces: per atom |F_gpu - F_ora| <= tol (|F_ora,a| + F_rms) with tol = 1e-4 in FP32
    (pair terms and force sums in FP32) and 1e-9 in FP64; energies within
    1e-5 (FP32) / 1e-10 (FP64) of sum |terms|;
  * trajectories: positions within 1e-4 nm after 100 steps (FP32, identical
    Philox streams), 1e-8 reduced units in FP64;
  * copy numbers: bit-exact given the same energies and uniforms;
  * log-sum-exp / ln Q: 1e-12 relative (FP64 on both sides, different
    summation order).
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
def gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1806_06016_amd import pamd as B
    B.load_library()
    return B


def _ctx(B, sysd, R, prec, T0=None, dt=None, nu=1.0, seed=1806, **kw):
    if T0 is None:
        T0 = 2.0 if sysd.units == "reduced" else 700.0
    if dt is None:
        dt = 0.002 if sysd.units == "reduced" else 0.001
    return B.Pamd([sysd], R_target=R, T0=T0, dt=dt, nu=nu, seed=seed, precision=prec, **kw)


def _force_check(F, Fo, tol):
    frms = np.sqrt((Fo ** 2).sum(-1).mean(-1))[:, None]
    err = np.linalg.norm(F - Fo, axis=-1)
    bound = tol * (np.linalg.norm(Fo, axis=-1) + frms)
    return float((err / bound).max())


def _perturbed(sysd, R, scale, seed):
    rng = np.random.default_rng(seed)
    return np.ascontiguousarray(sysd.x_init[None] + rng.normal(0, scale, size=(R,) + sysd.x_init.shape))


@pytest.mark.parametrize("which,prec", [("chain", 0), ("peptide", 1), ("chain", 1)])
def test_forces_and_energies(gpu, which, prec):
    sysd = S.c1_system() if which == "chain" else S.c2_system()
    R = 37                                 # ragged: not a multiple of the 4 replicas per wave
    print(f"forces {which} prec={prec}", flush=True)
    p = _ctx(gpu, sysd, R, prec)
    x = _perturbed(sysd, R, 0.1 if which == "chain" else 0.01, 5)
    v = np.zeros_like(x)
    p.set_state(0, x, v, T=700.0 if which == "peptide" else 2.0)
    xs = as_stored(x, prec)                # the positions as the context stores them
    assert np.array_equal(p.get_state(0)["x"], xs)
    F, E = p.get_forces(0)
    osys = O.OracleSystem(sysd)
    Eo, Fo, terms = O.energy_forces(osys, xs, want_terms=True)
    tolF = 1e-9 if prec == 0 else 1e-4
    tolE = 1e-10 if prec == 0 else 1e-5
    assert _force_check(F, Fo, tolF) <= 1.0
    assert np.all(np.abs(E - Eo) <= tolE * np.abs(terms).sum(1))
    p.close()


def test_init_velocities_match_oracle(gpu):
    for sysd, prec in [(S.c1_system(), 0), (S.c2_system(), 1)]:
        R = 21
        p = _ctx(gpu, sysd, R, prec)
        st = p.get_state(0)
        osys = O.OracleSystem(sysd)
        vo = O.init_velocities(osys, R, 2.0 if prec == 0 else 700.0, seed=1806)
        rel = np.abs(st["v"] - vo).max() / np.abs(vo).max()
        assert rel < (1e-14 if prec == 0 else 1e-6), rel
        assert np.abs(st["x"] - sysd.x_init[None]).max() < (1e-15 if prec == 0 else 1e-6)
        assert (st["ancestor"] == np.arange(R)).all() and st["R"] == R
        p.close()


@pytest.mark.parametrize("which,prec,nsteps,tol", [("peptide", 1, 100, 1e-4), ("chain", 0, 100, 1e-8),
                                                    ("chain", 1, 100, 1e-4)])
def test_trajectory_matches_oracle(gpu, which, prec, nsteps, tol):
    """Same start, same Philox streams: positions agree after 100 NVT steps
    (Andersen collisions happen at the same atoms and steps on both sides)."""
    sysd = S.c1_system() if which == "chain" else S.c2_system()
    R = 45
    T = 700.0 if which == "peptide" else 1.3
    nu = 1.0 if which == "peptide" else 5.0
    print(f"trajectory {which} prec={prec}", flush=True)
    p = _ctx(gpu, sysd, R, prec, T0=T, nu=nu, seed=77)
    osys = O.OracleSystem(sysd)
    x = _perturbed(sysd, R, 0.005 if which == "peptide" else 0.05, 8)
    v = O.init_velocities(osys, R, T, seed=3)
    p.set_state(0, x, v, T=T, step=500)
    xo, vo = as_stored(x, prec).copy(), as_stored(v, prec).copy()
    st = p.get_state(0)
    assert np.array_equal(st["x"], xo) and np.array_equal(st["v"], vo)
    p.md_steps(nsteps)
    g = p.get_state(0)
    Ep, Ek, col = O.md_steps(osys, xo, vo, nsteps, T, 0.001 if which == "peptide" else 0.002, nu, 77,
                             step0=500, want_collisions=True)
    assert col.sum() > 0                       # the thermostat actually acted
    err = np.abs(g["x"] - xo).max()
    assert err < tol, err
    assert g["step"] == 500 + nsteps
    scale = np.abs(Ep).mean()
    assert np.abs(g["E_pot"] - Ep).max() <= (1e-3 if prec else 1e-9) * scale
    assert np.allclose(g["E_kin"], Ek, rtol=1e-3 if prec else 1e-9)
    p.close()


def _synthetic_population(p, sysd, R, E, T, seed=0):
    """Sets a seeded population with energies E; returns it as the context
    stores it (rounded on the host), after checking the device holds exactly that."""
    rng = np.random.default_rng(seed)
    x = _perturbed(sysd, R, 0.01, seed)
    v = rng.normal(size=x.shape)
    p.set_state(0, x, v, T=T, E_pot=E, ancestor=np.arange(R) + 1000 * 0)
    fp32 = p.fp32
    st = dict(x=as_stored(x, fp32), v=as_stored(v, fp32), E_pot=np.asarray(E, np.float64).copy(),
              ancestor=np.arange(R))
    g = p.get_state(0)
    assert np.array_equal(g["x"], st["x"]) and np.array_equal(g["v"], st["v"])
    assert np.array_equal(g["E_pot"], st["E_pot"])
    return st


@pytest.mark.parametrize("R", [1, 7, 1000, 4099])
def test_resample_counts_bit_exact_given_uniforms(gpu, R):
    sysd = S.c2_system()
    rng = np.random.default_rng(R)
    E = rng.normal(-500.0, 25.0, R)
    T0, T1 = 700.0, 650.0
    p = _ctx(gpu, sysd, R, 1, R_cap=max(2 * R, R + 64))
    st = _synthetic_population(p, sysd, R, E, T0, seed=R)
    u = rng.random(p.R_cap)
    ut = torch.tensor(u, dtype=torch.float64, device="cuda")
    p.resample([T1], uniforms=ut)
    c = p.get_counts(0)
    dbeta = 1 / (sysd.kB * T1) - 1 / (sysd.kB * T0)
    co, tau = O.copy_counts(st["E_pot"], dbeta, R, u[:R])
    mism = np.nonzero(c != co)[0]
    if len(mism):
        margin = np.abs(u[mism] - (tau[mism] - np.floor(tau[mism])))
        pytest.fail(f"{len(mism)} copy numbers differ; margins {margin[:5]}")
    g = p.get_state(0)
    m, S_, S2, lq = O.lse(st["E_pot"], dbeta)
    assert abs(g["lnQ_last"] - lq) <= 1e-12 * max(1.0, abs(lq))
    assert abs(g["sum_lnQ"] - lq) <= 1e-12 * max(1.0, abs(lq))
    assert g["R"] == co.sum() and g["temp_index"] == 1
    assert abs(g["T"] - T1) < 1e-12 and abs(g["T_prev"] - T0) < 1e-12
    # gather: canonical order, ancestors, energies, recentred x, rescaled v
    xo, vo, Eo, ao = O.gather(co, [st["x"], st["v"], st["E_pot"], st["ancestor"]])
    assert (g["ancestor"] == ao).all()
    assert (g["E_pot"] == Eo).all()
    xo = O.recentre(xo, sysd.mass)
    assert np.abs(g["x"] - xo).max() < 2e-6
    assert np.abs(g["v"] - vo * math.sqrt(T1 / T0)).max() < 1e-6 * np.abs(vo).max()
    p.close()


def test_resample_philox_uniforms_match_oracle(gpu):
    sysd = S.c1_system()
    R = 3000
    rng = np.random.default_rng(2)
    E = rng.normal(10.0, 3.0, R)
    p = _ctx(gpu, sysd, R, 0, seed=4242)
    st = _synthetic_population(p, sysd, R, E, 2.0)
    p.resample([1.8])
    c = p.get_counts(0)
    u = O.resample_uniforms(R, 1, seed=4242)
    co, _ = O.copy_counts(st["E_pot"], 1 / 1.8 - 1 / 2.0, R, u)
    assert (c == co).all()
    p.close()


def test_adaptive_temperature_matches_oracle(gpu):
    """Adaptive step: largest T-decrement with normalised weight variance 0.1."""
    sysd = S.c2_system()
    R = 20000
    rng = np.random.default_rng(9)
    T0 = 700.0
    d = 219
    E = rng.gamma(d / 2, sysd.kB * T0, R) - 800.0
    p = _ctx(gpu, sysd, R, 1, T0=T0, T_final=250.0, V_target=0.1)
    st = _synthetic_population(p, sysd, R, E, T0)
    p.resample(None)
    g = p.get_state(0)
    kB = sysd.kB
    dmax = 1 / (kB * 250.0) - 1 / (kB * T0)
    db = O.adaptive_dbeta(st["E_pot"], dmax, 0.1)
    To = 1 / (kB * (db + 1 / (kB * T0)))
    assert abs(g["T"] - To) <= 1e-9 * To, (g["T"], To)
    V = O.weight_variance(st["E_pot"], 1 / (kB * To) - 1 / (kB * T0))
    assert abs(V - 0.1) < 1e-6
    obs = p.observables()[0]
    assert abs(obs["V_last"] - V) < 1e-9
    p.close()


def test_observables_match_oracle(gpu):
    """Population averages (PAMD step 4): exact FP64 reductions of host-given
    energies and ancestors; then, after an energy evaluation, the kinetic
    averages against the host's 1/2 m v^2 of the stored velocities."""
    sysd = S.c2_system()
    R = 333
    rng = np.random.default_rng(12)
    p = _ctx(gpu, sysd, R, 1)
    E = rng.normal(-300.0, 20.0, R)
    anc = rng.integers(0, 40, R).astype(np.int32)
    x = _perturbed(sysd, R, 0.01, 13)
    v = rng.normal(0, 0.5, x.shape)
    p.set_state(0, x, v, T=700.0, E_pot=E, ancestor=anc, step=10)
    obs = p.observables()[0]
    vs = as_stored(v, True)
    K = 0.5 * (sysd.mass[None, :, None] * vs * vs).sum((1, 2))
    o = O.observables(E, K, anc, sysd.n_atoms, sysd.kB, 700.0)
    for k in ("E_mean", "E2_mean", "Cv"):
        assert abs(obs[k] - o[k]) <= 1e-12 * abs(o[k]) + 1e-12, k
    assert obs["R"] == R and obs["families"] == o["families"] and obs["step"] == 10
    p.md_steps(0)                              # E_pot and E_kin of the stored state
    obs = p.observables()[0]
    for k in ("K_mean", "T_measured"):
        assert abs(obs[k] - o[k]) <= 1e-6 * abs(o[k]), k
    p.close()


def test_capacity_overflow_is_reported_and_state_kept(gpu):
    from paper_1806_06016_amd import PamdError, PAMD_ERR_CAPACITY
    sysd = S.c1_system()
    R = 200
    E = np.zeros(R)
    E[:100] = 0.0
    E[100:] = 50.0
    p = _ctx(gpu, sysd, R, 0, R_cap=220)
    st = _synthetic_population(p, sysd, R, E, 2.0)
    # half of the copies get ~2 copies each only if weights are flat; make them not:
    u = torch.zeros(p.R_cap, dtype=torch.float64, device="cuda")      # every fractional part rounds up
    p.resample([1.0], uniforms=u)
    with pytest.raises(PamdError) as ei:
        p.observables()
    assert ei.value.code in (PAMD_ERR_CAPACITY,)
    # the stopped context still hands out the population the failed step
    # started from, so a caller can recover (e.g. retry with a smaller step)
    g = p.get_state(0, after_error=True)
    assert g["error"] == PAMD_ERR_CAPACITY and g["R"] == R and g["T"] == 2.0
    assert np.array_equal(g["x"], st["x"]) and np.array_equal(g["v"], st["v"])
    assert np.array_equal(g["E_pot"], st["E_pot"]) and (g["ancestor"] == np.arange(R)).all()
    with pytest.raises(PamdError) as ei:
        p.md_steps(1)
    assert ei.value.code == gpu.PAMD_ERR_STATE
    p.close()
    # recovery: the rescued population in a new context, a smaller step
    q = _ctx(gpu, sysd, R, 0, R_cap=220)
    q.set_state(0, g["x"], g["v"], T=g["T"], E_pot=g["E_pot"], ancestor=g["ancestor"], step=g["step"])
    q.resample([1.9])                         # the context's own Philox uniforms
    o = q.observables()[0]
    dbeta = 1 / 1.9 - 1 / 2.0
    co, _ = O.copy_counts(st["E_pot"], dbeta, R, O.resample_uniforms(R, 1, seed=1806))
    assert (q.get_counts(0) == co).all()
    assert o["R"] == co.sum() <= 220 and o["T"] == 1.9
    q.close()


@pytest.mark.parametrize("which", ["chain_fp64", "peptide_fp32", "wide_two_runs"])
def test_capacity_overflow_then_md_steps_keeps_state(gpu, which):
    """The calls are asynchronous, so MD steps can be enqueued after a
    resampling that overflows the capacity on the device and before the error
    surfaces.  Those steps must leave the failed run exactly as the resampling
    found it (positions, velocities, E_pot and the step counter), in the
    register-tile kernels and in the batched wide launch; in the batched
    launch the other run still advances."""
    from paper_1806_06016_amd import PamdError, PAMD_ERR_CAPACITY
    R = 200
    E = np.zeros(R)
    E[100:] = 50.0
    if which == "chain_fp64":
        systems, prec, T0, T1 = [S.c1_system()], 0, 2.0, 1.0
    elif which == "peptide_fp32":
        systems, prec, T0, T1 = [S.c2_system()], 1, 700.0, 350.0
    else:
        systems, prec, T0, T1 = [S.c2_system(), S.make_peptide(1811, 120)], 1, 700.0, 350.0
    print("capacity overflow then MD:", which, flush=True)
    p = gpu.Pamd(systems, R_target=R, T0=T0, dt=0.002 if prec == 0 else 0.0005, nu=1.0, seed=7, precision=prec,
                 R_cap=220)
    st = []
    for run, sysd in enumerate(systems):
        rng = np.random.default_rng(40 + run)
        x = _perturbed(sysd, R, 0.01, 40 + run)
        v = rng.normal(0, 0.1, size=x.shape)
        p.set_state(run, x, v, T=T0, E_pot=E, step=17)
        st.append(dict(x=as_stored(x, prec == 1), v=as_stored(v, prec == 1)))
    # run 0 overflows (every fractional copy number rounds up); in the two-run
    # case run 1 is resampled at its own temperature without overflowing
    u = torch.zeros((p.n_runs, p.R_cap), dtype=torch.float64, device="cuda")
    if p.n_runs > 1:
        u[1] = 0.999999
    p.resample([T1] + [T0] * (p.n_runs - 1), uniforms=u)
    p.md_steps(5)
    with pytest.raises(PamdError) as ei:
        p.observables()
    assert ei.value.code == PAMD_ERR_CAPACITY
    g = p.get_state(0, after_error=True)
    assert g["error"] == PAMD_ERR_CAPACITY and g["R"] == R and g["T"] == T0 and g["step"] == 17
    assert np.array_equal(g["x"], st[0]["x"]) and np.array_equal(g["v"], st[0]["v"])
    assert np.array_equal(g["E_pot"], E)
    if p.n_runs > 1:
        h = p.get_state(1, after_error=True)
        assert h["step"] == 17 + 5 and h["R"] == R
        assert not np.array_equal(h["x"], st[1]["x"])
    p.close()


def test_nonfinite_energy_is_reported(gpu):
    from paper_1806_06016_amd import PamdError, PAMD_ERR_NONFINITE
    sysd = S.c2_system()
    R = 8
    p = _ctx(gpu, sysd, R, 1)
    x = _perturbed(sysd, R, 0.01, 1)
    x[3, 5, 0] = np.nan
    p.set_state(0, x, np.zeros_like(x), T=700.0)
    p.md_steps(0)
    with pytest.raises(PamdError) as ei:
        p.observables()
    assert ei.value.code == PAMD_ERR_NONFINITE
    # the population is still readable: the bad replica is the one with the NaN
    g = p.get_state(0, after_error=True)
    assert g["error"] == PAMD_ERR_NONFINITE
    bad = ~np.isfinite(g["E_pot"])
    assert bad.tolist() == [r == 3 for r in range(R)]
    assert np.isnan(g["x"][3, 5, 0]) and np.isfinite(np.delete(g["x"], 3, axis=0)).all()
    p.close()


def test_determinism_same_seed_same_state(gpu):
    sysd = S.c2_system()
    out = []
    for _ in range(2):
        p = _ctx(gpu, sysd, 130, 1, seed=99)
        p.md_steps(50)
        p.resample([650.0])
        p.md_steps(50)
        st = p.get_state(0)
        out.append((st["x"], st["v"], st["E_pot"]))
        p.close()
    for a, b in zip(out[0], out[1]):
        assert np.array_equal(a, b)


def test_copies_decorrelate(gpu):
    """Two copies of one configuration separate under the stochastic thermostat
    (their collision streams are keyed by distinct slots)."""
    sysd = S.c2_system()
    R = 16
    p = _ctx(gpu, sysd, R, 1)
    x = np.ascontiguousarray(np.broadcast_to(sysd.x_init, (R, sysd.n_atoms, 3)))
    v = np.zeros_like(x)
    p.set_state(0, x, v, T=700.0)
    p.md_steps(200)
    st = p.get_state(0)
    assert np.abs(st["x"][0] - st["x"][1]).max() > 1e-3
    p.close()


def _check_degenerate(p, sysd, st, T_from, T_to, n_copies, u):
    """Every replica copied n_copies times (all tau_j equal), by the oracle's
    rule too; canonical gather; ln Q = -dbeta E_min (S = R exactly)."""
    g = p.get_state(0)
    R = len(st["E_pot"])
    dbeta = 1 / (sysd.kB * T_to) - 1 / (sysd.kB * T_from)
    co, tau = O.copy_counts(st["E_pot"], dbeta, p.R_target, u)
    assert (co == n_copies).all() and (tau == n_copies).all()
    assert (p.get_counts(0)[:R] == n_copies).all() and g["R"] == n_copies * R
    assert abs(g["T"] - T_to) <= 1e-12 * T_to
    lq = -dbeta * st["E_pot"].min()
    assert abs(g["lnQ_last"] - lq) <= 1e-12 * max(1.0, abs(lq)), (g["lnQ_last"], lq)
    xo, vo, Eo, ao = O.gather(co, [st["x"], st["v"], st["E_pot"], st["ancestor"]])
    assert (g["ancestor"] == ao).all() and (g["E_pot"] == Eo).all()
    assert np.abs(g["x"] - O.recentre(xo, sysd.mass)).max() < (1e-12 if not p.fp32 else 2e-6)
    if T_to == T_from:
        assert np.array_equal(g["v"], vo)              # scale sqrt(T / T) = 1
    else:
        assert np.abs(g["v"] - vo * math.sqrt(T_to / T_from)).max() <= 1e-6 * np.abs(vo).max()
    return g


@pytest.mark.parametrize("which,prec", [("chain", 0), ("peptide", 1)])
def test_degenerate_resampling_cases(gpu, which, prec):
    """Resampling steps whose result is fixed in closed form (PAMD step 2):
    at the current temperature (dbeta = 0) every weight is 1, so each replica
    is kept once, in place, with ln Q = 0 and unscaled velocities; equal
    energies at a lower temperature give the same copy numbers and
    ln Q = -dbeta E; equal energies at half the target size give two copies
    each; the adaptive step with equal energies (weight variance 0 at any
    dbeta) jumps straight to T_final, and at T_final it stays there."""
    sysd = S.c1_system() if which == "chain" else S.c2_system()
    kB = sysd.kB
    R = 389
    T0, T1, Tf = (2.0, 1.8, 0.5) if which == "chain" else (700.0, 650.0, 250.0)
    rng = np.random.default_rng(31 + prec)
    E = rng.normal(10.0, 3.0, R) if which == "chain" else rng.normal(-400.0, 30.0, R)
    flat = np.full(R, -412.625)
    print(f"degenerate resampling {which} prec={prec}", flush=True)

    p = _ctx(gpu, sysd, R, prec, T0=T0, seed=505, T_final=Tf, V_target=0.1)
    # same temperature, Philox uniforms (irrelevant: every frac(tau) is 0)
    st = _synthetic_population(p, sysd, R, E, T0, seed=1)
    p.resample([T0])
    u = O.resample_uniforms(p.R_cap, 1, seed=505)
    g = _check_degenerate(p, sysd, st, T0, T0, 1, u)
    assert g["lnQ_last"] == 0.0 and g["sum_lnQ"] == 0.0
    # equal energies, explicit lower temperature
    st = _synthetic_population(p, sysd, R, flat, T0, seed=2)
    p.resample([T1])
    _check_degenerate(p, sysd, st, T0, T1, 1, u)
    # equal energies, adaptive: V(dbeta_max) = 0 <= V_target, so T_final at once
    st = _synthetic_population(p, sysd, R, flat, T0, seed=3)
    p.resample(None)
    _check_degenerate(p, sysd, st, T0, Tf, 1, u)
    assert p.observables()[0]["V_last"] == 0.0
    # adaptive at T_final: no step left, the population is kept at T_final
    st = _synthetic_population(p, sysd, R, E, Tf, seed=4)
    p.resample(None)
    g = _check_degenerate(p, sysd, st, Tf, Tf, 1, u)
    assert g["lnQ_last"] == 0.0
    p.close()

    # equal energies with half the target population: tau_j = 2 for every j
    p = _ctx(gpu, sysd, 2 * R, prec, T0=T0, seed=505)
    st = _synthetic_population(p, sysd, R, flat, T0, seed=5)
    p.resample([T1])
    u = O.resample_uniforms(p.R_cap, 1, seed=505)
    _check_degenerate(p, sysd, st, T0, T1, 2, u)
    assert 1 / (kB * T1) > 1 / (kB * T0)
    p.close()
