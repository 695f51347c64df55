"""Pins of the oracle's learned-MTS pieces (CPU only): surrogate forces are
minus the FD gradient of its energy; the energy is invariant under rigid
motions and under swapping two atoms of one type; the force-matching loss
gradient (autograd, FP64) matches FD of the loss; two independent
derivations of the surrogate forces agree; r-RESPA is time reversible and,
with the surrogate replaced by the exact nonbonded force, reduces to plain
velocity Verlet."""
import math

import numpy as np
import pytest

from oracle import nn as NN
from oracle import oracle as O
from pamd_inputs import systems as S


@pytest.fixture(scope="module")
def pep():
    sysd = S.c2_system()
    return sysd, NN.nn_pairs(sysd), NN.init_weights(3)


def _xs(sysd, B, scale, seed):
    rng = np.random.default_rng(seed)
    return sysd.x_init[None] + rng.normal(0, scale, size=(B,) + sysd.x_init.shape)


def test_nn_forces_are_minus_energy_gradient(pep):
    sysd, pairs, w = pep
    x = _xs(sysd, 2, 0.01, 1)
    E, F = NN.energy_forces(x, sysd.atype, pairs, w)
    h = 1e-6
    for a in (0, 7, 40, 74):
        for c in range(3):
            xp = x.copy(); xp[:, a, c] += h
            xm = x.copy(); xm[:, a, c] -= h
            fd = -(NN.energy_forces(xp, sysd.atype, pairs, w)[0] - NN.energy_forces(xm, sysd.atype, pairs, w)[0]) / (2 * h)
            assert np.allclose(fd, F[:, a, c], rtol=1e-6, atol=1e-8 * np.abs(F).max())


def test_nn_energy_invariances(pep):
    sysd, pairs, w = pep
    x = _xs(sysd, 1, 0.01, 2)
    E = NN.energy_forces(x, sysd.atype, pairs, w)[0][0]
    th = 0.9
    Rm = np.array([[math.cos(th), 0, math.sin(th)], [0, 1, 0], [-math.sin(th), 0, math.cos(th)]])
    assert abs(NN.energy_forces(x @ Rm.T + 3.0, sysd.atype, pairs, w)[0][0] - E) < 1e-9 * abs(E)
    # a two-atom system: the features of each atom are phi_k(r) in the partner's type slot
    two = np.array([[[0.0, 0.0, 0.0], [0.31, 0.0, 0.0]]])
    G, r, d, phi = NN.features(two, np.array([2, 5]), np.array([[0, 1]]))
    assert np.allclose(G[0, 0, 5], np.exp(-(0.31 - NN.MU) ** 2 / (2 * NN.SIG ** 2)))
    assert np.allclose(G[0, 1, 2], G[0, 0, 5]) and G[0, 0, 2].sum() == 0 and G[0, 1, 5].sum() == 0


def test_nn_forces_two_derivations_agree(pep):
    """Manual backprop (numpy) vs autograd of the same energy (torch)."""
    import torch
    sysd, pairs, w = pep
    x = _xs(sysd, 2, 0.01, 3)
    E, F = NN.energy_forces(x, sysd.atype, pairs, w)
    # autograd forces by a zero target: dL/dF = 2 F / n, L = mean F^2
    L, _ = NN.loss_grad_torch(x, np.zeros_like(x), sysd.atype, pairs, w)
    assert abs(L - np.mean(F ** 2)) < 1e-10 * L


def test_force_loss_gradient_matches_finite_differences(pep):
    sysd, pairs, w = pep
    x = _xs(sysd, 2, 0.01, 4)
    Ft = np.random.default_rng(5).normal(0, 50, x.shape)
    L, g = NN.loss_grad_torch(x, Ft, sysd.atype, pairs, w)
    h = 1e-6
    rng = np.random.default_rng(6)
    for name in ("W1", "b1", "W2", "b2", "w3"):
        idx = tuple(rng.integers(0, s) for s in w[name].shape)
        wp = {k: v.copy() for k, v in w.items()}
        wm = {k: v.copy() for k, v in w.items()}
        wp[name][idx] += h
        wm[name][idx] -= h
        fd = (NN.force_loss(x, Ft, sysd.atype, pairs, wp) - NN.force_loss(x, Ft, sysd.atype, pairs, wm)) / (2 * h)
        assert abs(fd - g[name][idx]) <= 1e-5 * max(abs(fd), 1e-3), (name, fd, g[name][idx])
    assert np.all(g["b3"] == 0)        # a constant energy shift exerts no force


def test_respa_with_exact_surrogate_is_velocity_verlet(pep):
    sysd, pairs, w = pep
    osys = O.OracleSystem(sysd)
    x0 = _xs(sysd, 3, 0.005, 7)
    v0 = O.init_velocities(osys, 3, 300.0, seed=2)
    nb = O.T_LJ | O.T_COUL
    x1, v1 = x0.copy(), v0.copy()
    NN.respa_steps(osys, sysd, x1, v1, 5, 4, 0.001, 300.0, 0.0, 1, 0,
                   lambda xx: O.energy_forces(osys, xx, nb)[1])
    x2, v2 = x0.copy(), v0.copy()
    O.md_steps(osys, x2, v2, 20, 300.0, 0.001, 0.0, 1, 0)
    assert np.abs(x1 - x2).max() < 1e-10 and np.abs(v1 - v2).max() < 1e-8


def test_respa_is_time_reversible(pep):
    sysd, pairs, w = pep
    osys = O.OracleSystem(sysd)
    x = _xs(sysd, 2, 0.005, 8)
    v = O.init_velocities(osys, 2, 300.0, seed=4)
    x0, v0 = x.copy(), v.copy()
    f = lambda xx: NN.energy_forces(xx, sysd.atype, pairs, w)[1]
    NN.respa_steps(osys, sysd, x, v, 3, 4, 0.001, 300.0, 0.0, 1, 0, f)
    v *= -1
    NN.respa_steps(osys, sysd, x, v, 3, 4, 0.001, 300.0, 0.0, 1, 0, f)
    v *= -1
    assert np.abs(x - x0).max() < 1e-9 and np.abs(v - v0).max() < 1e-6
