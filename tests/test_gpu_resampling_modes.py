"""GPU: the multinomial and switched-off resampling modes against the oracle,
through the C ABI.

Multinomial copy numbers are compared draw for draw: both sides build FP64
running weight sums W_j (left to right on the oracle, in chunk order on the
GPU), so they may round apart by a few R eps W_{R-1}.  A draw whose target
u_k W_{R-1} lies within 4 R eps W_{R-1} of a boundary W_j is ambiguous: it may
land on either side.  Counts must be equal except at the sources such draws
touch, and there by at most one copy per ambiguous draw (at the sizes here the
expected number of ambiguous draws is below 1e-3).  Energies, ancestors,
positions and velocities follow the parity tolerances of the nearest-integer
mode.
"""
import math

import numpy as np
import pytest

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

from oracle import oracle as O  # noqa: E402
from pamd_inputs import systems as S  # noqa: E402
from pamd_inputs.precision import as_stored  # noqa: E402

EPS = 2.0 ** -52


@pytest.fixture(scope="module")
def B():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1806_06016_amd import pamd
    pamd.load_library()
    return pamd


def _population(p, run, sysd, R, E, T, seed):
    """Sets a seeded population; returns it as the context stores it (rounded
    on the host), after checking that the device holds exactly that."""
    rng = np.random.default_rng(seed)
    x = np.ascontiguousarray(sysd.x_init[None] + rng.normal(0, 0.01, (R,) + sysd.x_init.shape))
    v = rng.normal(size=x.shape)
    p.set_state(run, x, v, T=T, E_pot=E, ancestor=np.arange(R))
    st = dict(x=as_stored(x, p.fp32), v=as_stored(v, p.fp32), E_pot=np.asarray(E, np.float64).copy(),
              ancestor=np.arange(R))
    g = p.get_state(run)
    assert np.array_equal(g["x"], st["x"]) and np.array_equal(g["v"], st["v"])
    assert np.array_equal(g["E_pot"], st["E_pot"])
    return st


def _assert_draws_match(c, E, dbeta, u):
    """GPU counts c against the oracle's, allowing only ambiguous draws to differ."""
    co, W = O.multinomial_counts(E, dbeta, u)
    R = len(E)
    tol = 4 * R * EPS * W[-1]
    t = u * W[-1]
    pos = np.searchsorted(W, t)
    near = np.zeros(len(u), bool)
    for off in (-1, 0, 1):
        q = np.clip(pos + off, 0, R - 1)
        near |= np.abs(W[q] - t) <= tol
    allowed = set()
    for k in np.nonzero(near)[0]:
        q = np.nonzero(np.abs(W - t[k]) <= tol)[0]
        for j in q:
            allowed.add(int(j))
            nxt = np.nonzero(W[j + 1:] > W[j])[0]
            if len(nxt):
                allowed.add(int(j + 1 + nxt[0]))
    diff = np.nonzero(c != co)[0]
    assert set(diff.tolist()) <= allowed, (diff[:10], int(near.sum()))
    assert np.abs(c - co).sum() <= 2 * int(near.sum())
    return co, int(near.sum())


@pytest.mark.parametrize("R_cur,R_target", [(1, 1), (7, 7), (1000, 1000), (4099, 4099), (999, 1024),
                                            (1500, 700), (1, 300)])
def test_multinomial_counts_given_uniforms(B, R_cur, R_target):
    """FP32 peptide context, caller uniforms: copy numbers draw for draw, the
    gather (canonical order, ancestors, recentred x, rescaled v), ln Q."""
    sysd = S.c2_system()
    R_cap = max(R_cur, R_target) + 64
    p = B.Pamd([sysd], R_target=R_target, R_cap=R_cap, T0=700.0, dt=0.001, nu=1.0, seed=3,
               precision=B.PAMD_FP32, resampling="multinomial")
    rng = np.random.default_rng(R_cur * 7 + R_target)
    E = rng.normal(-500.0, 25.0, R_cur)
    T0, T1 = 700.0, 620.0
    st = _population(p, 0, sysd, R_cur, E, T0, R_cur)
    u = rng.random(R_cap)
    p.resample([T1], uniforms=torch.tensor(u, dtype=torch.float64, device="cuda"))
    c = p.get_counts(0)
    db = 1 / (sysd.kB * T1) - 1 / (sysd.kB * T0)
    co, amb = _assert_draws_match(c, st["E_pot"], db, u[:R_target])
    print(f"R {R_cur} -> {R_target}: ambiguous draws {amb}")
    assert c.sum() == R_target
    g = p.get_state(0)
    assert g["R"] == R_target
    m, S_, S2, lq = O.lse(st["E_pot"], db)
    assert abs(g["lnQ_last"] - lq) <= 1e-12 * max(1.0, abs(lq))
    if amb == 0:
        xo, vo, Eo, ao = O.gather(co, [st["x"], st["v"], st["E_pot"], st["ancestor"]])
        assert (g["ancestor"] == ao).all() and (g["E_pot"] == Eo).all()
        assert np.abs(g["x"] - O.recentre(xo, sysd.mass)).max() < 2e-6
        assert np.abs(g["v"] - vo * math.sqrt(T1 / T0)).max() < 1e-6 * np.abs(vo).max()
    p.close()


def test_multinomial_philox_draws_match_oracle_per_run(B):
    """FP64 bead-chain context with two runs: each run's draws come from Philox
    stream 4 under its own key (seed_hi + run)."""
    sysd = S.c1_system()
    R = 3000
    p = B.Pamd([sysd, sysd], R_target=R, T0=2.0, dt=0.002, nu=1.0, seed=4242, precision=B.PAMD_FP64,
               resampling="multinomial")
    pops = []
    for r in range(2):
        E = np.random.default_rng(20 + r).normal(10.0, 3.0, R)
        pops.append(_population(p, r, sysd, R, E, 2.0, 30 + r))
    p.resample([1.8, 1.7])
    for r, T1 in enumerate((1.8, 1.7)):
        u = O.multinomial_uniforms(R, 1, seed=4242, run=r)
        _assert_draws_match(p.get_counts(r), pops[r]["E_pot"], 1 / T1 - 1 / 2.0, u)
    p.close()


def test_multinomial_at_the_full_population(B):
    """R = 1e5 FP32 peptide copies (the population of the headline workload),
    energies with the spread of a thermal 75-atom peptide, the oracle's
    adaptive step: every draw against the oracle, population size exactly R."""
    sysd = S.c2_system()
    R = 100_000
    p = B.Pamd([sysd], R_target=R, T0=700.0, dt=0.001, nu=1.0, seed=77, precision=B.PAMD_FP32,
               T_final=250.0, resampling="multinomial")
    E = np.random.default_rng(5).gamma(219 / 2, sysd.kB * 700.0, R) - 800.0
    st = _population(p, 0, sysd, R, E, 700.0, 6)
    # the oracle's adaptive step, requested explicitly so both sides use one T
    kB = sysd.kB
    db = O.adaptive_dbeta(st["E_pot"], 1 / (kB * 250.0) - 1 / (kB * 700.0), 0.1)
    T1 = 1 / (kB * (db + 1 / (kB * 700.0)))
    db = 1 / (kB * T1) - 1 / (kB * 700.0)
    p.resample([T1])
    g = p.get_state(0, want_xv=False)
    u = O.multinomial_uniforms(R, 1, seed=77)
    c = p.get_counts(0)
    _, amb = _assert_draws_match(c, st["E_pot"], db, u)
    print("ambiguous draws", amb, "T", g["T"], "families", p.observables()[0]["families"])
    assert g["R"] == R and c.sum() == R
    p.close()


@pytest.mark.parametrize("prec", [0, 1])
def test_resampling_off_keeps_every_copy(B, prec):
    """Mode none: c_j = 1, population size and ancestors unchanged (also when
    R differs from R_target), velocities rescaled, copies recentred, ln Q still
    recorded."""
    sysd = S.c1_system() if prec == 0 else S.c2_system()
    T0, T1 = (2.0, 1.6) if prec == 0 else (700.0, 600.0)
    R, R_cur = 500, 437
    p = B.Pamd([sysd], R_target=R, T0=T0, dt=0.002, nu=1.0, seed=5, precision=prec, resampling="none")
    E = np.random.default_rng(8).normal(0.0, 5.0, R_cur)
    st = _population(p, 0, sysd, R_cur, E, T0, 9)
    p.resample([T1])
    c = p.get_counts(0)
    assert len(c) == R_cur and (c == 1).all()
    g = p.get_state(0)
    assert g["R"] == R_cur and (g["ancestor"] == st["ancestor"]).all()
    assert (g["E_pot"] == st["E_pot"]).all()
    tol = 1e-12 if prec == 0 else 2e-6
    assert np.abs(g["x"] - O.recentre(st["x"], sysd.mass)).max() < tol
    assert np.abs(g["v"] - st["v"] * math.sqrt(T1 / T0)).max() < tol * max(1.0, np.abs(st["v"]).max())
    _, _, _, lq = O.lse(st["E_pot"], 1 / (sysd.kB * T1) - 1 / (sysd.kB * T0))
    assert abs(g["lnQ_last"] - lq) <= 1e-12 * max(1.0, abs(lq))
    assert p.observables()[0]["families"] == R_cur
    p.close()


@pytest.mark.parametrize("mode", ["multinomial", "none"])
def test_bead_chain_anneal_identical_seeds(B, mode):
    """A whole FP64 anneal of the bead chain in each mode (same seeds): every
    temperature's <E_pot> and the final sum ln Q equal the oracle's (rounding
    differences of the two sides grow to ~1e-8 over the chaotic MD)."""
    sysd = S.c1_system()
    sched = S.geometric_schedule(2.0, 0.5, 12)
    R = 256
    for seed in (1, 2):
        p = B.Pamd([sysd], R_target=R, T0=2.0, dt=0.002, nu=1.0, seed=seed, precision=0, resampling=mode)
        p.md_steps(300)
        E = [p.observables()[0]["E_mean"]]
        for T in sched[1:]:
            p.resample([T])
            p.md_steps(100)
            E.append(p.observables()[0]["E_mean"])
        o = p.observables()[0]
        p.close()
        res = O.anneal(sysd, R, 2.0, sched, theta=100, theta_eq=300, dt=0.002, nu=1.0, seed=seed,
                       resampling=mode)
        Eo = np.array([ob["E_mean"] for ob in res.obs])
        print(mode, "seed", seed, "max rel dE", np.max(np.abs(np.array(E) - Eo) / np.abs(Eo)))
        assert np.allclose(E, Eo, rtol=1e-6, atol=1e-8)
        assert abs(o["sum_lnQ"] - res.sum_lnQ) < 1e-7
        assert o["R"] == R
        if mode == "none":
            assert o["families"] == R


@pytest.mark.parametrize("mode", ["multinomial", "none"])
def test_graph_replay_matches_eager(B, mode):
    sysd = S.c2_system()
    R = 777

    def run(use_graph):
        p = B.Pamd([sysd], R_target=R, T0=700.0, dt=0.001, nu=1.0, seed=12, precision=B.PAMD_FP32,
                   T_final=500.0, resampling=mode)
        p.md_steps(30)
        if use_graph:
            p.graph_capture(30, mode="adaptive", slot=0, parts="both")
            for _ in range(3):
                p.graph_launch(0)
                torch.cuda.synchronize()
                p.observables()
        else:
            for _ in range(3):
                p.resample(None)
                p.md_steps(30)
                p.observables()
        out = p.get_state(0)
        obs = p.observables()[0]
        p.close()
        return out, obs

    a, oa = run(False)
    b, ob = run(True)
    assert np.array_equal(a["x"], b["x"]) and np.array_equal(a["ancestor"], b["ancestor"])
    assert oa["T"] == ob["T"] and oa["sum_lnQ"] == ob["sum_lnQ"] and oa["R"] == ob["R"]
