"""Pins of the oracle's Langevin bath (CPU only).

The paper's runs use a stochastic Langevin thermostat (friction 1/ps, a
distinct random stream per replica) inside a velocity-Verlet variant.  The
oracle takes the B-A-O-A-B splitting (Leimkuhler & Matthews 2013): half kick,
half drift, exact Ornstein-Uhlenbeck velocity step, half drift, force, half
kick.  Pins:
* zero friction reduces it to plain velocity Verlet;
* on free particles one step is x1 = x0 + dt/2 (v0 + v1) with
  v1 = c1 v0 + c2 sqrt(kB T / m) xi: regression slope c1 = exp(-gamma dt) and
  residual variance (1 - c1^2) kB T / m;
* on a harmonic (zero-rest-length) chain B-A-O-A-B samples configurations
  exactly at any stable time step: <|b|^2> = 3 kB T / k per bond even where
  velocity Verlet is 25-60 % off;
* equipartition <K> = 3/2 N kB T at a small step;
* every replica draws its own noise.
"""
import math

import numpy as np

from oracle import oracle as O
from pamd_inputs import systems as S


def _chain_start(n, k, T, R, seed):
    rng = np.random.default_rng(seed)
    b = rng.normal(0, math.sqrt(T / k), (R, n - 1, 3))
    x = np.zeros((R, n, 3))
    x[:, 1:] = np.cumsum(b, axis=1)
    return np.ascontiguousarray(x)


def test_zero_friction_is_velocity_verlet():
    sysd = S.c1_system()
    osys = O.OracleSystem(sysd)
    x0 = np.ascontiguousarray(np.broadcast_to(sysd.x_init, (8, 10, 3)).astype(np.float64))
    v0 = O.init_velocities(osys, 8, 2.0, seed=4)
    xa, va = x0.copy(), v0.copy()
    xb, vb = x0.copy(), v0.copy()
    Ea, _ = O.md_steps(osys, xa, va, 100, 2.0, 0.002, 0.0, 9, 0, thermostat="langevin")
    Eb, _ = O.md_steps(osys, xb, vb, 100, 2.0, 0.002, 0.0, 9, 0, thermostat="andersen")
    assert np.abs(xa - xb).max() < 1e-10 and np.abs(va - vb).max() < 1e-9
    assert np.allclose(Ea, Eb, rtol=1e-10)


def test_free_particle_step_is_an_exact_ornstein_uhlenbeck_step():
    sysd = S.gaussian_chain(10, 0.0, 0.0)          # no forces at all
    sysd.mass = np.linspace(1.0, 16.0, 10)          # masses 1 .. 16
    osys = O.OracleSystem(sysd)
    R, T, dt, gamma = 4000, 1.5, 0.01, 50.0
    rng = np.random.default_rng(2)
    x0 = np.ascontiguousarray(rng.normal(0, 1, (R, 10, 3)))
    v0 = O.init_velocities(osys, R, T, seed=5)
    x, v = x0.copy(), v0.copy()
    O.md_steps(osys, x, v, 1, T, dt, gamma, 11, 0, thermostat="langevin")
    assert np.abs((x - x0) - 0.5 * dt * (v0 + v)).max() < 1e-14
    c1 = math.exp(-gamma * dt)
    # in units of the thermal speed sqrt(kB T / m) of each atom
    w = np.sqrt(sysd.mass)[None, :, None]
    a, b = (v0 * w).ravel(), (v * w).ravel()
    slope = (a * b).sum() / (a * a).sum()
    resid = b - slope * a
    assert abs(slope - c1) < 0.01, (slope, c1)
    assert abs(resid.var() / ((1 - c1 * c1) * T) - 1) < 0.02


def test_harmonic_chain_configurations_are_exact_at_a_large_step():
    """omega_max dt = 1.6 on the k = 100 chain (unit masses, kB T = 1)."""
    sysd = S.gaussian_chain(10, 100.0, 0.0)
    osys = O.OracleSystem(sysd)
    R, T, dt = 2000, 1.0, 0.08
    x = _chain_start(10, 100.0, T, R, 1)
    v = O.init_velocities(osys, R, T, seed=3)
    ratios = []
    step = 0
    for blk in range(16):
        O.md_steps(osys, x, v, 50, T, dt, 5.0, 7, step, thermostat="langevin")
        step += 50
        if blk >= 4:
            b = np.diff(x, axis=1)
            ratios.append((b ** 2).sum(-1).mean() / (3 * T / 100.0))
    assert abs(np.mean(ratios) - 1) < 0.01, np.mean(ratios)


def test_equipartition_at_a_small_step():
    sysd = S.gaussian_chain(10, 100.0, 0.0)
    osys = O.OracleSystem(sysd)
    R, T = 1000, 2.0
    x = _chain_start(10, 100.0, T, R, 4)
    v = O.init_velocities(osys, R, 0.5, seed=3)     # start cold: the bath must heat it
    O.md_steps(osys, x, v, 400, T, 0.002, 5.0, 7, 0, thermostat="langevin")
    K = []
    for blk in range(10):
        _, Ek = O.md_steps(osys, x, v, 20, T, 0.002, 5.0, 7, 400 + 20 * blk, thermostat="langevin")
        K.append(Ek.mean())
    assert abs(np.mean(K) / (15 * T) - 1) < 0.02


def test_every_replica_draws_its_own_noise():
    sysd = S.c1_system()
    osys = O.OracleSystem(sysd)
    x = np.ascontiguousarray(np.broadcast_to(sysd.x_init, (4, 10, 3)).astype(np.float64))
    v = np.zeros_like(x)
    O.md_steps(osys, x, v, 1, 2.0, 0.002, 1.0, 9, 0, thermostat="langevin")
    for i in range(1, 4):
        assert np.abs(v[i] - v[0]).max() > 1e-6
