"""GPU parity of the learned multiple-time-step surrogate against the FP64
oracle in oracle/nn.py (every call through libpamd's C ABI).

Tolerances.  The GPU rounds the features, the weight copies and the hidden
activations / adjoints to BF16 (unit roundoff u = 2^-9 ~ 2e-3) and accumulates
in FP32; each of the 5-6 roundings on the path from positions to forces adds
a relative error of order u.  Every element is checked: the force on each
atom within 2e-2 (about 10 u) of (|F_a| + F_rms), F_rms the RMS atomic force
of that configuration (so nearly cancelled atomic forces are not failed on
their own magnitude); each energy within 2e-2 of (|E| + RMS energy); every loss-gradient
component g within 5e-2 of (|g_o| + rms of its parameter block) (two more BF16
roundings: the feature derivative and the adjoints).  Integrator tests use surrogate-independent bounds: with
F_NN = 0 the r-RESPA trajectory matches to the FP32 MD bound (1e-4 nm); with
a non-zero surrogate the position difference is bounded by the force
difference, |dx| <~ (n dt)^2 |dF| / m.
"""
import numpy as np
import pytest

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

from oracle import nn as NN  # noqa: E402
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


def _confs(sysd, n, scale, seed):
    rng = np.random.default_rng(seed)
    return np.ascontiguousarray(sysd.x_init[None] + rng.normal(0, scale, size=(n,) + sysd.x_init.shape))


def _rel(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


def _force_ratio(F, Fo, tol):
    """max over configurations and atoms of |F_a - F_o,a| / (tol (|F_o,a| + F_rms))"""
    F = F.reshape(-1, Fo.shape[-2], 3)
    Fo = Fo.reshape(-1, Fo.shape[-2], 3)
    frms = np.sqrt((Fo ** 2).sum(-1).mean(-1))[:, None]
    return float((np.linalg.norm(F - Fo, axis=-1) / (tol * (np.linalg.norm(Fo, axis=-1) + frms))).max())


def _grad_ratio(g, go, tol):
    """max over the components of a parameter block of |g - g_o| / (tol (|g_o| + rms(g_o)))"""
    rms = np.sqrt(np.mean(go ** 2))
    return float((np.abs(g - go) / (tol * (np.abs(go) + rms))).max())


def test_surrogate_energies_and_forces(B):
    sysd = S.c2_system()
    n = sysd.n_atoms
    nb = 37                               # 37 x 75 rows: ragged in the 64-row tiles and the 3-per-block layout
    print("surrogate forces, peptide, 37 configurations", flush=True)
    x = _confs(sysd, nb, 0.02, 11)
    w = NN.init_weights(3)
    pairs = NN.nn_pairs(sysd)
    Eo, Fo = NN.energy_forces(x, sysd.atype, pairs, w)
    nn = B.PamdNN(sysd, sysd.atype)
    nn.set_weights(w)
    E, F = nn.forces(torch.tensor(x, dtype=torch.float32, device="cuda"))
    E, F = E.cpu().numpy().astype(np.float64), F.cpu().numpy().astype(np.float64)
    ratio = _force_ratio(F, Fo, 2e-2)
    print("per-atom force error / bound", ratio, "L2", max(_rel(F[c], Fo[c]) for c in range(nb)),
          "energy", np.abs(E - Eo).max() / np.abs(Eo).max())
    assert ratio <= 1.0
    assert np.all(np.abs(E - Eo) <= 2e-2 * (np.abs(Eo) + np.sqrt(np.mean(Eo ** 2))))
    nn.close()


def test_surrogate_zero_weights_give_zero_force(B):
    sysd = S.c2_system()
    nn = B.PamdNN(sysd, sysd.atype)
    x = torch.tensor(_confs(sysd, 5, 0.02, 2), dtype=torch.float32, device="cuda")
    E, F = nn.forces(x)
    assert torch.count_nonzero(F).item() == 0 and torch.count_nonzero(E).item() == 0
    nn.close()


def test_surrogate_small_molecule_and_single_configuration(B):
    """n = 10 (25 configurations per block) and one configuration."""
    sysd = S.c1_system()
    atype = np.arange(sysd.n_atoms, dtype=np.int32) % 8
    x = _confs(sysd, 1, 0.05, 4) * 0.3        # reduced-unit chain scaled into the Gaussian range
    w = NN.init_weights(5)
    pairs = NN.nn_pairs(sysd)
    Eo, Fo = NN.energy_forces(x, atype, pairs, w)
    nn = B.PamdNN(sysd, atype)
    nn.set_weights(w)
    E, F = nn.forces(torch.tensor(x, dtype=torch.float32, device="cuda"))
    F = F.cpu().numpy().astype(np.float64)
    ratio = _force_ratio(F, Fo, 2e-2)
    print("chain per-atom force error / bound", ratio)
    assert ratio <= 1.0
    assert abs(float(E[0]) - Eo[0]) < 2e-2 * abs(Eo[0]) + 1e-3
    nn.close()


def test_loss_gradient_matches_oracle(B):
    sysd = S.c2_system()
    nb = 5
    print("loss gradient, peptide, 5 configurations", flush=True)
    x = _confs(sysd, nb, 0.02, 21)
    w = NN.init_weights(7)
    pairs = NN.nn_pairs(sysd)
    rng = np.random.default_rng(8)
    Ft = rng.normal(0, 20.0, size=x.shape)
    L, g = NN.loss_grad_torch(x, Ft, sysd.atype, pairs, w)
    nn = B.PamdNN(sysd, sysd.atype)
    nn.set_weights(w)
    lg, gg = nn.loss_grad(torch.tensor(x, dtype=torch.float32, device="cuda"),
                          torch.tensor(Ft, dtype=torch.float32, device="cuda"))
    lg = float(lg.item())
    gd = B.unpack_params(gg.cpu().numpy().astype(np.float64))
    print("loss", lg, L)
    assert abs(lg - L) < 2e-2 * L
    for k in ("W1", "b1", "W2", "b2", "w3"):
        r = _grad_ratio(gd[k], g[k], 5e-2)
        print("gradient block", k, "max element error / bound", r, "L2 relative", _rel(gd[k], g[k]))
        assert r <= 1.0, k
    assert float(gd["b3"][0]) == 0.0
    nn.close()


def test_training_reduces_the_loss(B):
    """Teacher-student: targets are the forces of another weight set, which
    the network can represent exactly."""
    sysd = S.c2_system()
    x = _confs(sysd, 64, 0.01, 31)
    Ft = NN.energy_forces(x, sysd.atype, NN.nn_pairs(sysd), NN.init_weights(10, 0.5))[1]
    nn = B.PamdNN(sysd, sysd.atype)
    nn.set_weights(NN.init_weights(9, 0.5))
    xt = torch.tensor(x, dtype=torch.float32, device="cuda")
    ft = torch.tensor(Ft, dtype=torch.float32, device="cuda")
    loss = torch.zeros(1, dtype=torch.float32, device="cuda")
    hist = []
    for it in range(60):
        nn.train_step(xt, ft, 1e-3, loss)
        hist.append(float(loss.item()))
    print("loss", hist[0], "->", hist[-1])
    assert hist[-1] < 0.5 * hist[0]
    nn.close()


def test_export_configs_nonbonded_forces(B):
    sysd = S.c2_system()
    R = 21
    p = B.Pamd([sysd], R_target=R, T0=700.0, dt=0.001, nu=1.0, seed=5, precision=B.PAMD_FP32)
    osys = O.OracleSystem(sysd)
    x = _confs(sysd, R, 0.01, 6)
    p.set_state(0, x, np.zeros_like(x), T=700.0)
    xg, fg = p.export_configs(0, 0, R)
    xg, fg = xg.cpu().numpy().astype(np.float64), fg.cpu().numpy().astype(np.float64)
    xs = as_stored(x, True)
    assert np.array_equal(xg, xs)
    Fo = O.energy_forces(osys, xs, O.T_LJ | O.T_COUL)[1]
    frms = np.sqrt((Fo ** 2).sum(-1).mean(-1))[:, None]
    bound = 1e-4 * (np.linalg.norm(Fo, axis=-1) + frms)
    assert (np.linalg.norm(fg - Fo, axis=-1) <= bound).all()
    p.close()


def _respa_case(B, w, n_outer, M, seed=41):
    """Both sides start from the same relaxed state: 300 plain MD steps of the
    oracle from the built conformation (a perturbed start has clashes whose
    repulsion a 4 fs outer impulse cannot integrate stably, and unstable
    trajectories diverge at rounding level), stored in FP32.  With an untrained
    or zero surrogate the outer impulse carries the whole stiff nonbonded
    force, so the parity cases use an outer step of 2 inner steps."""
    sysd = S.c2_system()
    R, T, dt, nu = 45, 700.0, 0.001, 1.0
    osys = O.OracleSystem(sysd)
    x0 = np.ascontiguousarray(np.broadcast_to(sysd.x_init, (R, sysd.n_atoms, 3)).astype(np.float64))
    v0 = O.init_velocities(osys, R, T, seed)
    O.md_steps(osys, x0, v0, 300, T, dt, nu, seed, 0)
    step0 = 300
    xo, vo = as_stored(x0, True), as_stored(v0, True)
    p = B.Pamd([sysd], R_target=R, T0=T, dt=dt, nu=nu, seed=seed, precision=B.PAMD_FP32)
    p.set_state(0, x0, v0, T=T, step=step0)
    st = p.get_state(0)
    assert np.array_equal(st["x"], xo) and np.array_equal(st["v"], vo)
    print("start: max |F_nb|", np.abs(O.energy_forces(osys, xo, O.T_LJ | O.T_COUL)[1]).max(), flush=True)
    nn = B.PamdNN(sysd, sysd.atype)
    if w is not None:
        nn.set_weights(w)
    p.set_mts(nn, M)
    p.md_steps(n_outer * M)
    g = p.get_state(0)
    pairs = NN.nn_pairs(sysd)
    if w is None:
        f = lambda xx: np.zeros_like(xx)  # noqa: E731
    else:
        f = lambda xx: NN.energy_forces(xx, sysd.atype, pairs, w)[1]  # noqa: E731
    Ep, Ek = NN.respa_steps(osys, sysd, xo, vo, n_outer, M, dt, T, nu, seed, step0, f)
    p.set_mts(None)
    p.close()
    nn.close()
    assert g["step"] == step0 + n_outer * M
    return g, xo, vo, Ep, Ek


def test_respa_without_surrogate_matches_oracle(B):
    """F_NN = 0: the whole nonbonded force acts in the outer impulses."""
    print("r-RESPA, zero surrogate, 5 outer steps of 2", flush=True)
    g, xo, vo, Ep, Ek = _respa_case(B, None, 5, 2)
    err = np.abs(g["x"] - xo).max()
    print("max |dx|", err, "max |dE_pot| / |E_pot|", np.max(np.abs(g["E_pot"] - Ep) / np.abs(Ep)))
    assert err < 1e-4
    assert np.all(np.abs(g["E_pot"] - Ep) <= 1e-3 * np.abs(Ep))
    assert np.allclose(g["E_kin"], Ek, rtol=1e-3)


def test_respa_with_surrogate_matches_oracle(B):
    print("r-RESPA, surrogate, 4 outer steps", flush=True)
    g, xo, vo, Ep, Ek = _respa_case(B, NN.init_weights(13), 4, 2)
    err = np.abs(g["x"] - xo).max()
    print("max |dx|", err)
    # 8 steps of 1 fs: (0.008 ps)^2 x |dF_NN| (<~ 2e-2 x 1e3) / 1 amu ~ 1e-3 nm at worst
    assert err < 1e-3
    assert np.all(np.abs(g["E_pot"] - Ep) <= 1e-2 * np.abs(Ep))
