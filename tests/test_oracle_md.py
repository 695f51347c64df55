"""Pins of the oracle's MD update (PAMD step 3) and random numbers (CPU only).

Pins: the exact discrete map of velocity Verlet for a harmonic spring, time
reversibility, the second-order energy error, momentum conservation, the
Maxwell-Boltzmann statistics of Andersen collisions, and statistical
properties of the counter-based generator.
"""
import math

import numpy as np
import pytest
from scipy import stats

from oracle import oracle as O
from pamd_inputs import systems as S


def test_velocity_verlet_harmonic_closed_form():
    """Two particles on a zero-rest-length spring: each component of the
    separation is an oscillator with w^2 = k (1/m1 + 1/m2).  Velocity Verlet's
    one-step map is a rotation with cos(w~ dt) = 1 - (w dt)^2 / 2 (for w dt < 2),
    so s_n = A cos(n w~ dt) + B sin(n w~ dt) holds to rounding; the centre of
    mass moves uniformly."""
    k, m1, m2 = 50.0, 1.0, 3.0
    sysd = S.spring_pair(k, m1, m2)
    osys = O.OracleSystem(sysd)
    x = sysd.x_init[None].copy()
    v = np.array([[[0.2, -0.1, 0.05], [-0.3, 0.15, 0.4]]])
    dt = 0.01
    w = math.sqrt(k * (1 / m1 + 1 / m2))
    wt = math.acos(1 - (w * dt) ** 2 / 2) / dt
    s0 = x[0, 0] - x[0, 1]
    u0 = v[0, 0] - v[0, 1]
    # the first half-step uses the force at s0: VV's discrete velocity at step 0 is u0;
    # with s_n = A cos + B sin, s_1 = s0 + dt u0 - dt^2/2 w^2 s0 fixes B.
    A = s0
    s1 = s0 + dt * u0 - 0.5 * dt * dt * w * w * s0
    B = (s1 - A * math.cos(wt * dt)) / math.sin(wt * dt)
    M = m1 + m2
    com0 = (m1 * x[0, 0] + m2 * x[0, 1]) / M
    vcom = (m1 * v[0, 0] + m2 * v[0, 1]) / M
    nsteps = 700
    O.md_steps(osys, x, v, nsteps, T=1.0, dt=dt, nu=0.0, seed=1, step0=0)
    sn = x[0, 0] - x[0, 1]
    exact = A * math.cos(nsteps * wt * dt) + B * math.sin(nsteps * wt * dt)
    assert np.abs(sn - exact).max() < 1e-10
    com = (m1 * x[0, 0] + m2 * x[0, 1]) / M
    assert np.abs(com - (com0 + nsteps * dt * vcom)).max() < 1e-12


def test_time_reversibility():
    """Without thermostat VV is time reversible: run n steps, flip v, run n
    steps, flip v -> the starting state."""
    sysd = S.c1_system()
    osys = O.OracleSystem(sysd)
    x = sysd.x_init[None].copy()
    v = O.init_velocities(osys, 1, 1.0, seed=5)
    x0, v0 = x.copy(), v.copy()
    O.md_steps(osys, x, v, 400, 1.0, 0.002, 0.0, 1, 0)
    v *= -1
    O.md_steps(osys, x, v, 400, 1.0, 0.002, 0.0, 1, 0)
    v *= -1
    assert np.abs(x - x0).max() < 1e-9
    assert np.abs(v - v0).max() < 1e-9


def _energy_error_rms(sysd, x0, v0, dt, t_window):
    osys = O.OracleSystem(sysd)
    x = x0.copy()
    v = v0.copy()
    n = int(round(t_window / dt))
    E0 = O.energy_forces(osys, x)[0] + 0.5 * np.einsum("rac,a->r", v * v, osys.mass)
    errs = []
    chunk = max(1, n // 20)
    for _ in range(n // chunk):
        Ep, Ek = O.md_steps(osys, x, v, chunk, 1.0, dt, 0.0, 1, 0)
        errs.append(Ep + Ek - E0)
    return float(np.sqrt(np.mean(np.square(errs))))


def test_nve_energy_error_scales_as_dt_squared():
    """Velocity Verlet's energy error is second order: the RMS of
    E_tot(t) - E_tot(0) over a fixed window shrinks as dt^2."""
    sysd = S.c1_system()
    osys = O.OracleSystem(sysd)
    R = 64
    x = np.ascontiguousarray(np.broadcast_to(sysd.x_init, (R, 10, 3)))
    v = O.init_velocities(osys, R, 1.0, seed=9)
    O.md_steps(osys, x, v, 1000, 1.0, 0.002, 1.0, 9, 0)       # thermalise
    dts = [0.004, 0.002, 0.001]
    errs = [_energy_error_rms(sysd, x, v, dt, 4.0) for dt in dts]
    slope = np.polyfit(np.log(dts), np.log(errs), 1)[0]
    assert 1.8 <= slope <= 2.2, (errs, slope)


def test_momentum_and_angular_momentum_conserved():
    sysd = S.c2_system()
    osys = O.OracleSystem(sysd)
    x = sysd.x_init[None].copy()
    v = O.init_velocities(osys, 1, 300.0, seed=4)
    m = osys.mass[:, None]
    P0 = (m * v[0]).sum(0)
    L0 = np.cross(x[0], m * v[0]).sum(0)
    O.md_steps(osys, x, v, 1000, 300.0, 0.0005, 0.0, 1, 0)
    P1 = (m * v[0]).sum(0)
    L1 = np.cross(x[0], m * v[0]).sum(0)
    scale = (m * np.abs(v[0])).sum()
    assert np.abs(P1 - P0).max() < 1e-12 * scale
    assert np.abs(L1 - L0).max() < 1e-10 * scale * np.abs(x).max()


def test_init_velocities_maxwell_boltzmann():
    """Stream-3 initial velocities: each component N(0, kB T / m)."""
    sysd = S.c2_system()
    osys = O.OracleSystem(sysd)
    v = O.init_velocities(osys, 400, 500.0, seed=3)
    z = (v / np.sqrt(osys.kB * 500.0 / osys.mass)[None, :, None]).ravel()
    assert stats.kstest(z, "norm").pvalue > 1e-3
    assert abs(z.mean()) < 4 / math.sqrt(z.size)


def test_andersen_collision_rate_and_distribution():
    """Per-atom collision probability p = 1 - exp(-nu dt) (integer threshold) and
    collided velocities drawn from N(0, kB T / m): with a large nu the
    velocities of a harmonic chain forget their start and the kinetic energy
    settles at (3N/2) kB T."""
    sysd = S.gaussian_chain(10)
    osys = O.OracleSystem(sysd)
    R = 200
    x = np.ascontiguousarray(np.broadcast_to(sysd.x_init, (R, 10, 3)))
    v = np.zeros((R, 10, 3))
    nu, dt, T = 5.0, 0.002, 0.7
    Ep, Ek, col = O.md_steps(osys, x, v, 2000, T, dt, nu, seed=21, step0=0, want_collisions=True)
    p = O.collision_p24(nu, dt) / 2 ** 24
    n = R * 10 * 2000
    assert abs(col.sum() / n - p) < 4 * math.sqrt(p * (1 - p) / n)
    # equilibrium kinetic energy per replica
    Ep, Ek = O.md_steps(osys, x, v, 500, T, dt, nu, seed=21, step0=2000)
    assert abs(Ek.mean() - 15 * T) < 4 * Ek.std() / math.sqrt(R) + 0.02 * 15 * T
    # a single-step velocity snapshot of atom components is Gaussian
    z = (v / math.sqrt(T)).ravel()
    assert stats.kstest(z, "norm").pvalue > 1e-4


def test_philox_statistics():
    """Uniformity of 24-bit outputs over 256 bins (chi^2), avalanche (a one-bit
    counter change flips about half of the 128 output bits), determinism and
    distinct key streams."""
    outs = np.array([O.philox([i, 7, 0, 0], [1806, 0]) for i in range(4096)], dtype=np.uint64)
    hist = np.bincount(((outs >> np.uint64(24)) & np.uint64(255)).astype(np.int64).ravel(),
                       minlength=256)
    chi2 = ((hist - hist.mean()) ** 2 / hist.mean()).sum()
    assert stats.chi2.sf(chi2, 255) > 1e-3
    flips = []
    for i in range(256):
        a = O.philox([i, 3, 5, 1], [99, 1])
        b = O.philox([i ^ 1, 3, 5, 1], [99, 1])
        flips.append(sum(bin(int(x) ^ int(y)).count("1") for x, y in zip(a, b)))
    assert abs(np.mean(flips) - 64) < 2.0
    assert (O.philox([1, 2, 3, 4], [5, 6]) == O.philox([1, 2, 3, 4], [5, 6])).all()
    assert not (O.philox([1, 2, 3, 4], [5, 6]) == O.philox([1, 2, 3, 4], [5, 7])).any()


def test_resampling_uniforms_are_uniform():
    u = O.resample_uniforms(20000, 3, seed=77)
    assert ((u >= 0) & (u < 1)).all()
    assert stats.kstest(u, "uniform").pvalue > 1e-3
    assert len(np.unique(u)) == len(u)


def test_philox_known_answers():
    """The oracle's Philox-4x32-10 reproduces the generator's published
    known-answer vectors (tests/golden/philox4x32_10_kat.txt)."""
    import os
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "philox4x32_10_kat.txt")
    n = 0
    for line in open(path):
        if line.startswith("#") or not line.strip():
            continue
        c, k, o = ([int(w, 16) for w in part.split()] for part in line.split("|"))
        assert [int(w) for w in O.philox(c, k)] == o, line
        n += 1
    assert n == 3
