"""GPU: the wide layout (one replica per wavefront) and the batched launch of
several uneven runs, against the FP64 oracle, through the C ABI.

A context holding a molecule above the register-tile limit runs its wide runs
in one persistent launch (items handed out largest molecule first); its runs
of at most 80 atoms take that launch too (layout "auto") or register-tile
launches of their own (layout "tile", the mixed case the autotuner may
choose).  Every test runs both.  Same
tolerances as the register-tile parity tests: per-atom forces within
1e-4 (|F_a| + F_rms), energies within 1e-5 of sum |terms|, positions within
1e-4 nm after 100 NVT steps with identical Philox streams, copy numbers
bit-exact.
"""
import functools
import math

import numpy as np
import pytest

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

from oracle import oracle as O  # noqa: E402
from pamd_inputs import systems as S  # noqa: E402
from pamd_inputs.precision import as_stored  # noqa: E402

SIZES = (40, 120, 300)


@pytest.fixture(scope="module")
def B():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1806_06016_amd import pamd
    pamd.load_library()
    return pamd


@functools.lru_cache(maxsize=None)
def _peptide(seed, n):
    # the generator's clash repair takes seconds for the larger molecules
    return S.make_peptide(seed=seed, n_atoms=n)


def _systems():
    return [_peptide(1806 + k, n) for k, n in enumerate(SIZES)]


def _batched_systems():
    return [_peptide(1806 + k, n) for k, n in enumerate(S.C4_SIZES)]


def _layouts(syss, mode):
    """per-run layout: "auto" everywhere, or "tile" for the runs that fit the register tile"""
    return ["tile" if (mode == "mixed" and s.n_atoms <= 80) else "auto" for s in syss]


def _check_layouts(p, syss, mode):
    for r, sysd in enumerate(syss):
        want = "wide" if (sysd.n_atoms > 80 or mode == "auto") else "tile"
        assert p.run_launch(r)["layout"] == want


def _perturbed(sysd, R, scale, seed):
    rng = np.random.default_rng(seed)
    return np.ascontiguousarray(sysd.x_init[None] + rng.normal(0, scale, size=(R,) + sysd.x_init.shape))


def test_batched_context_uses_the_wide_layout(B):
    p = B.Pamd(_systems(), R_target=13, T0=700.0, dt=0.001, nu=1.0, seed=3, precision=B.PAMD_FP32)
    info = p.launch_info()
    print("launch", info)
    assert 1 <= info["waves_per_block"] <= 8
    p.close()


@pytest.mark.parametrize("mode", ["auto", "mixed"])
def test_wide_forces_and_energies(B, mode):
    """Every molecule size of the batched workload (40 ... 300 atoms), batched."""
    syss = _batched_systems()
    R = 13
    print("wide forces", S.C4_SIZES, mode, flush=True)
    p = B.Pamd(syss, R_target=R, T0=700.0, dt=0.001, nu=1.0, seed=3, precision=B.PAMD_FP32,
               layout=_layouts(syss, mode))
    _check_layouts(p, syss, mode)
    for r, sysd in enumerate(syss):
        x = _perturbed(sysd, R, 0.01, 5 + r)
        p.set_state(r, x, np.zeros_like(x), T=700.0)
        F, E = p.get_forces(r)
        osys = O.OracleSystem(sysd)
        xs = as_stored(x, True)
        assert np.array_equal(p.get_state(r)["x"], xs)
        Eo, Fo, terms = O.energy_forces(osys, xs, want_terms=True)
        frms = np.sqrt((Fo ** 2).sum(-1).mean(-1))[:, None]
        ratio = (np.linalg.norm(F - Fo, axis=-1) / (1e-4 * (np.linalg.norm(Fo, axis=-1) + frms))).max()
        print(f"n={sysd.n_atoms}: force error / bound {ratio:.3f}")
        assert ratio <= 1.0
        assert np.all(np.abs(E - Eo) <= 1e-5 * np.abs(terms).sum(1))
    p.close()


@pytest.mark.parametrize("mode", ["auto", "mixed"])
def test_wide_trajectories_match_oracle(B, mode):
    """All runs advance in one call; each matches its own oracle run
    (Philox key seed_hi + run)."""
    syss = _systems()
    R, T, nu, seed, n_steps = 11, 700.0, 1.0, 77, 100
    print("wide trajectories", SIZES, mode, flush=True)
    p = B.Pamd(syss, R_target=R, T0=T, dt=0.001, nu=nu, seed=seed, precision=B.PAMD_FP32,
               layout=_layouts(syss, mode))
    _check_layouts(p, syss, mode)
    starts = []
    for r, sysd in enumerate(syss):
        osys = O.OracleSystem(sysd)
        x = _perturbed(sysd, R, 0.003, 8 + r)
        v = O.init_velocities(osys, R, T, seed=3 + r)
        p.set_state(r, x, v, T=T, step=500)
        starts.append((as_stored(x, True), as_stored(v, True)))
        st = p.get_state(r)
        assert np.array_equal(st["x"], starts[-1][0]) and np.array_equal(st["v"], starts[-1][1])
    p.md_steps(n_steps)
    for r, sysd in enumerate(syss):
        osys = O.OracleSystem(sysd)
        xo, vo = starts[r]
        Ep, Ek, col = O.md_steps(osys, xo, vo, n_steps, T, 0.001, nu, seed, step0=500, run=r, want_collisions=True)
        g = p.get_state(r)
        err = np.abs(g["x"] - xo).max()
        print(f"n={sysd.n_atoms}: max |dx| {err:.2e}, collisions {int(col.sum())}")
        assert col.sum() > 0
        assert err < 1e-4
        assert g["step"] == 500 + n_steps
        assert np.abs(g["E_pot"] - Ep).max() <= 1e-3 * np.abs(Ep).mean()
        assert np.allclose(g["E_kin"], Ek, rtol=1e-3)
    p.close()


@pytest.mark.parametrize("mode", ["auto", "mixed"])
def test_batched_anneal_matches_oracle_per_run(B, mode):
    """Two temperature steps of every run: per-run resampling (counts bit-exact,
    ancestors) and MD in the shared launch."""
    syss = _systems()
    R, seed, theta = 64, 31, 40
    temps = [700.0, 690.0, 680.0]
    print("batched anneal", SIZES, mode, flush=True)
    p = B.Pamd(syss, R_target=R, T0=temps[0], dt=0.001, nu=1.0, seed=seed, precision=B.PAMD_FP32,
               layout=_layouts(syss, mode))
    p.md_steps(theta)
    ora = []
    for r, sysd in enumerate(syss):
        osys = O.OracleSystem(sysd)
        x = np.ascontiguousarray(np.broadcast_to(sysd.x_init, (R, sysd.n_atoms, 3)).astype(np.float64))
        v = O.init_velocities(osys, R, temps[0], seed, run=r)
        Ep, Ek = O.md_steps(osys, x, v, theta, temps[0], 0.001, 1.0, seed, 0, run=r)
        assert np.abs(p.get_state(r)["x"] - x).max() < 1e-4
        ora.append([osys, x, v, Ep, np.arange(R)])
    step = theta
    for i in (1, 2):
        p.resample([temps[i]] * len(syss))
        p.md_steps(theta)
        for r, sysd in enumerate(syss):
            osys, x, v, Ep, anc = ora[r]
            kB = sysd.kB
            db = 1 / (kB * temps[i]) - 1 / (kB * temps[i - 1])
            u = O.resample_uniforms(len(Ep), i, seed, run=r)
            c, _ = O.copy_counts(Ep, db, R, u)
            assert (p.get_counts(r) == c).all()
            x, v, Ep, anc = O.gather(c, [x, v, Ep, anc])
            x = np.ascontiguousarray(O.recentre(x, osys.mass))
            v = np.ascontiguousarray(v * math.sqrt(temps[i] / temps[i - 1]))
            Ep, Ek = O.md_steps(osys, x, v, theta, temps[i], 0.001, 1.0, seed, step, run=r)
            g = p.get_state(r)
            assert (g["ancestor"] == anc).all()
            err = np.abs(g["x"] - x).max()
            print(f"n={sysd.n_atoms} temperature step {i}: max |dx| {err:.2e}")
            assert err < 2e-4
            ora[r] = [osys, x, v, Ep, anc]
        step += theta
    p.close()


@pytest.mark.parametrize("mode", ["auto", "mixed"])
def test_batched_graph_replay_is_identical(B, mode):
    syss = _systems()
    R = 48

    def run(use_graph):
        p = B.Pamd(syss, R_target=R, T0=700.0, dt=0.001, nu=1.0, seed=9, precision=B.PAMD_FP32,
                   T_final=600.0, layout=_layouts(syss, mode))
        p.md_steps(20)
        if use_graph:
            p.graph_capture(20, mode="adaptive", slot=0, parts="both")
            for _ in range(3):
                p.graph_launch(0)
        else:
            for _ in range(3):
                p.resample(None)
                p.md_steps(20)
        out = [p.get_state(r) for r in range(len(syss))]
        obs = p.observables()
        p.close()
        return out, obs

    a, oa = run(False)
    b, ob = run(True)
    for r in range(len(syss)):
        assert np.array_equal(a[r]["x"], b[r]["x"])
        assert oa[r]["T"] == ob[r]["T"] and oa[r]["sum_lnQ"] == ob[r]["sum_lnQ"]


def test_forced_wide_layout_of_a_small_molecule(B):
    """The 75-atom peptide alone, forced into the wide layout: forces and a
    short trajectory as in the register-tile layout (both against the oracle)."""
    sysd = S.c2_system()
    R, T, nu, seed = 9, 700.0, 1.0, 5
    p = B.Pamd([sysd], R_target=R, T0=T, dt=0.001, nu=nu, seed=seed, precision=B.PAMD_FP32, layout="wide")
    assert p.run_launch(0)["layout"] == "wide"
    osys = O.OracleSystem(sysd)
    x = _perturbed(sysd, R, 0.003, 2)
    v = O.init_velocities(osys, R, T, seed=4)
    p.set_state(0, x, v, T=T)
    xo, vo = as_stored(x, True), as_stored(v, True)
    F, E = p.get_forces(0)
    Eo, Fo = O.energy_forces(osys, xo)[:2]
    frms = np.sqrt((Fo ** 2).sum(-1).mean(-1))[:, None]
    assert (np.linalg.norm(F - Fo, axis=-1) <= 1e-4 * (np.linalg.norm(Fo, axis=-1) + frms)).all()
    p.md_steps(50)
    O.md_steps(osys, xo, vo, 50, T, 0.001, nu, seed, step0=0)
    assert np.abs(p.get_state(0)["x"] - xo).max() < 1e-4
    p.close()


def test_autotuner_picks_a_layout_and_wide_launch_shape(B):
    """The batched autotuner times every candidate (all runs wide, or the
    small runs in register-tile launches; 4..1 waves per workgroup of the
    wide launch; when the split wins, its register-tile launches at 8 and 4
    waves per workgroup too) and the chosen shape builds a working context."""
    from paper_1806_06016_amd.autotune import autotune_batched, TILE_SMALL_CANDIDATES
    syss = [_peptide(1806, 40), _peptide(1807, 120)]
    t = autotune_batched(syss, 512, theta_probe=10, use_cache=False)
    print("autotune", t)
    first = {f"{l}/w{w}" for l in ("wide", "tile_small") for w in (4, 3, 2, 1)}
    assert first <= set(t["timings"])
    best_first = max(first, key=lambda c: t["timings"][c])
    if best_first.startswith("tile_small"):
        assert set(t["timings"]) - first == {f"{best_first}/t{tw}" for tw in TILE_SMALL_CANDIDATES}
    else:
        assert set(t["timings"]) == first
    assert all(v > 0 for v in t["timings"].values())
    assert t["timings"][t["choice"]] == max(t["timings"].values())
    p = B.Pamd(syss, R_target=64, T0=700.0, dt=0.0005, nu=1.0, seed=2, precision=B.PAMD_FP32,
               layout=t["layout"], wide_waves=t["wide_waves_per_block"], waves_per_block=t["waves_per_block"])
    assert [p.run_launch(r)["layout"] for r in range(2)] == t["layout"]
    assert p.run_launch(1)["waves_per_block"] == t["wide_waves_per_block"]
    if t["waves_per_block"] and t["layout"][0] == "tile":
        assert p.run_launch(0)["waves_per_block"] == t["waves_per_block"]
    p.md_steps(5)
    assert p.observables()[1]["step"] == 5
    p.close()


def _with_lj_classes(sysd, k):
    """A copy of `sysd` whose atoms carry exactly k distinct (sigma, epsilon)
    pairs: the atoms of its most common pair are split into sub-classes by
    relative sigma changes of 1e-4 j (the molecule's geometry stays valid)."""
    import collections
    import dataclasses
    pairs = list(zip(sysd.sigma.tolist(), sysd.epsilon.tolist()))
    n0 = len(set(pairs))
    top = collections.Counter(pairs).most_common(1)[0][0]
    idx = [a for a, q in enumerate(pairs) if q == top]
    m = k - n0 + 1
    assert 1 <= m <= len(idx)
    sig = sysd.sigma.copy()
    for j, a in enumerate(idx):
        sig[a] = top[0] * (1.0 + 1e-4 * (j % m))
    out = dataclasses.replace(sysd, sigma=sig)
    assert len(set(zip(out.sigma.tolist(), out.epsilon.tolist()))) == k
    return out


def test_lj_class_table_at_its_capacity(B):
    """A 120-atom molecule with 25 distinct LJ parameter pairs, the most the
    wide kernels' class table holds (one more class, all zero, serves the
    padding atoms): the launch's LDS holds the table after the position and
    force stages, and forces and a 50-step trajectory match the oracle."""
    sysd = _with_lj_classes(_peptide(1807, 120), 25)
    R, T, nu, seed = 9, 700.0, 1.0, 5
    print("LJ classes 25", flush=True)
    p = B.Pamd([sysd], R_target=R, T0=T, dt=0.001, nu=nu, seed=seed, precision=B.PAMD_FP32)
    info = p.run_launch(0)
    assert info["layout"] == "wide"
    assert info["lds_bytes"] == info["waves_per_block"] * (6 * sysd.n_atoms * 4 + 26 * 27 * 8)
    osys = O.OracleSystem(sysd)
    x = _perturbed(sysd, R, 0.003, 2)
    v = O.init_velocities(osys, R, T, seed=4)
    p.set_state(0, x, v, T=T)
    xo, vo = as_stored(x, True), as_stored(v, True)
    F, E = p.get_forces(0)
    Eo, Fo, terms = O.energy_forces(osys, xo, want_terms=True)
    frms = np.sqrt((Fo ** 2).sum(-1).mean(-1))[:, None]
    assert (np.linalg.norm(F - Fo, axis=-1) <= 1e-4 * (np.linalg.norm(Fo, axis=-1) + frms)).all()
    assert np.all(np.abs(E - Eo) <= 1e-5 * np.abs(terms).sum(1))
    p.md_steps(50)
    Ep, Ek = O.md_steps(osys, xo, vo, 50, T, 0.001, nu, seed, step0=0)
    g = p.get_state(0)
    assert np.abs(g["x"] - xo).max() < 1e-4
    assert np.abs(g["E_pot"] - Ep).max() <= 1e-3 * np.abs(Ep).mean()
    p.close()


@pytest.mark.parametrize("n", [1, 2, 17])
def test_forced_wide_layout_of_tiny_chains(B, n):
    """Bead chains of 1, 2 and 17 atoms forced into the wide layout (one LJ
    class, vacuum 1/r Coulomb, nearly every lane a padding atom): forces and a
    100-step trajectory against the oracle, as in the register-tile layout."""
    sysd = S.bead_chain(n, seed=n)
    R, T, nu, seed = 7, 1.3, 5.0, 11
    print(f"tiny wide chain n={n}", flush=True)
    p = B.Pamd([sysd], R_target=R, T0=T, dt=0.002, nu=nu, seed=seed, precision=B.PAMD_FP32, layout="wide")
    assert p.run_launch(0)["layout"] == "wide"
    osys = O.OracleSystem(sysd)
    x = _perturbed(sysd, R, 0.05, 3)
    v = O.init_velocities(osys, R, T, seed=6)
    p.set_state(0, x, v, T=T)
    xo, vo = as_stored(x, True), as_stored(v, True)
    F, E = p.get_forces(0)
    Eo, Fo, terms = O.energy_forces(osys, xo, want_terms=True)
    frms = np.sqrt((Fo ** 2).sum(-1).mean(-1))[:, None]
    assert (np.linalg.norm(F - Fo, axis=-1) <= 1e-4 * (np.linalg.norm(Fo, axis=-1) + frms) + 1e-12).all()
    assert np.all(np.abs(E - Eo) <= 1e-5 * np.abs(terms).sum(1) + 1e-12)
    p.md_steps(100)
    O.md_steps(osys, xo, vo, 100, T, 0.002, nu, seed, step0=0)
    assert np.abs(p.get_state(0)["x"] - xo).max() < 1e-4
    p.close()
