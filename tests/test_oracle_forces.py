"""Pins of the oracle's energy / force field (CPU only).

The force field is the functional form of the paper's molecular model (AMBER
type: harmonic bonds and angles, Fourier dihedrals, LJ + Coulomb with 1-2 /
1-3 exclusions and scaled 1-4 pairs).  Pins used here are independent of the
oracle's own formulas: central finite differences of its energy, translation /
rotation invariance, textbook special cases with known minima or values, and
graph-theoretic counts of the pair list.
"""
import math

import numpy as np
import pytest

from oracle import oracle as O
from pamd_inputs import systems as S


def _fd_forces(osys, x, mask, h):
    G = np.zeros_like(x)
    for a in range(x.shape[0]):
        for c in range(3):
            xp = x.copy(); xp[a, c] += h
            xm = x.copy(); xm[a, c] -= h
            G[a, c] = -(O.energy_forces(osys, xp, mask)[0] - O.energy_forces(osys, xm, mask)[0]) / (2 * h)
    return G


@pytest.mark.parametrize("which", ["chain", "peptide", "branched"])
@pytest.mark.parametrize("mask", [O.T_BOND, O.T_ANGLE, O.T_DIHEDRAL, O.T_LJ, O.T_COUL, O.T_ALL])
def test_forces_are_minus_energy_gradient(which, mask):
    """Every term type on the bead chain, the peptide and the branched pair
    (six-coordinated hubs, stacked torsion terms on one quadruple)."""
    sysd = {"chain": S.c1_system, "peptide": S.c2_system, "branched": S.branched_pair}[which]()
    osys = O.OracleSystem(sysd)
    rng = np.random.default_rng(11)
    noise = 0.01 if which == "peptide" else 0.1
    x = sysd.x_init + rng.normal(0, noise, size=sysd.x_init.shape)
    E, F = O.energy_forces(osys, x, mask)
    G = _fd_forces(osys, x, mask, 1e-6)
    assert np.abs(G - F).max() <= 1e-6 * np.abs(F).max()


def _four_atoms(phi, b=(1.0, 1.2, 0.9), ang=(1.9, 2.0)):
    """Four atoms with bond lengths b, angles ang and dihedral phi (radians),
    built from explicit trigonometry (independent of the oracle)."""
    x = np.zeros((4, 3))
    x[1] = [b[0], 0, 0]
    x[2] = x[1] + b[1] * np.array([-math.cos(ang[0]), math.sin(ang[0]), 0.0])
    # fourth atom: rotate about the 1-2 axis by phi from the cis position
    e = (x[2] - x[1]) / np.linalg.norm(x[2] - x[1])
    w0 = x[0] - x[1]
    u0 = w0 - np.dot(w0, e) * e
    u0 /= np.linalg.norm(u0)                                # towards atom 0, normal to the 1-2 axis
    d_cis = -math.cos(ang[1]) * e + math.sin(ang[1]) * u0   # in plane with atom 0 (cis, phi = 0)
    ax = e
    # Rodrigues rotation of d_cis about ax by phi
    d = (d_cis * math.cos(phi) + np.cross(ax, d_cis) * math.sin(phi)
         + ax * np.dot(ax, d_cis) * (1 - math.cos(phi)))
    x[3] = x[2] + b[2] * d
    return x


def _dihedral_system(k, n, delta):
    return S.System(
        name="dih", n_atoms=4, mass=np.ones(4), charge=np.zeros(4), sigma=np.ones(4),
        epsilon=np.zeros(4), atype=np.zeros(4, np.int32),
        bonds=np.array([[0, 1], [1, 2], [2, 3]], np.int32), bond_k=np.zeros(3), bond_r0=np.ones(3),
        angles=np.zeros((0, 3), np.int32), angle_k=np.zeros(0), angle_theta0=np.zeros(0),
        dihedrals=np.array([[0, 1, 2, 3]], np.int32), dih_k=np.array([k]),
        dih_n=np.array([n], np.int32), dih_delta=np.array([delta]),
        scale14_lj=1.0, scale14_coul=1.0, coulomb_k=1.0, dielectric=0, kB=1.0,
        x_init=_four_atoms(0.3))


@pytest.mark.parametrize("phi", [0.4, 1.3, -2.2, 2.9])
@pytest.mark.parametrize("n,delta", [(1, 0.0), (2, 0.7), (3, math.pi), (2, -1.1)])
def test_dihedral_energy_at_constructed_angle(phi, n, delta):
    """U = k (1 + cos(n phi - delta)) at a geometry built with a known phi;
    a general delta fixes the sign convention of phi, and FD checks the
    gradient of the same term for a non-symmetric delta."""
    sysd = _dihedral_system(2.5, n, delta)
    osys = O.OracleSystem(sysd)
    x = _four_atoms(phi)
    E, F = O.energy_forces(osys, x, O.T_DIHEDRAL)
    # the pair (0, 3) is a 1-4 pair, kept out of this check by the mask
    Uplus = 2.5 * (1 + math.cos(n * phi - delta))
    Uminus = 2.5 * (1 + math.cos(-n * phi - delta))
    assert min(abs(E - Uplus), abs(E - Uminus)) < 1e-12
    if abs(math.sin(delta)) > 1e-6:
        # the two orientations differ: the convention must be consistent between
        # a geometry and its mirror image
        xm = x * np.array([1, 1, -1.0])
        Em = O.energy_forces(osys, xm, O.T_DIHEDRAL)[0]
        assert abs(Em - (Uminus if abs(E - Uplus) < 1e-12 else Uplus)) < 1e-12
    G = _fd_forces(osys, x, O.T_DIHEDRAL, 1e-6)
    assert np.abs(G - F).max() <= 1e-7 * max(1.0, np.abs(F).max())


def test_lj_pair_minimum_and_value():
    """Single LJ pair: minimum at r = 2^(1/6) sigma with U = -eps and zero force."""
    sig, eps = 0.31, 0.7
    x = np.array([[0.0, 0, 0], [2 ** (1 / 6) * sig, 0, 0]])
    sysd = S.System(name="lj", n_atoms=2, mass=np.ones(2), charge=np.zeros(2),
                    sigma=np.full(2, sig), epsilon=np.full(2, eps), atype=np.zeros(2, np.int32),
                    bonds=np.zeros((0, 2), np.int32), bond_k=np.zeros(0), bond_r0=np.zeros(0),
                    angles=np.zeros((0, 3), np.int32), angle_k=np.zeros(0), angle_theta0=np.zeros(0),
                    dihedrals=np.zeros((0, 4), np.int32), dih_k=np.zeros(0),
                    dih_n=np.zeros(0, np.int32), dih_delta=np.zeros(0),
                    scale14_lj=0.5, scale14_coul=0.5, coulomb_k=138.935458, dielectric=1, kB=1.0,
                    x_init=x)
    osys = O.OracleSystem(sysd)
    E, F = O.energy_forces(osys, x)
    assert abs(E + eps) < 1e-12
    assert np.abs(F).max() < 1e-10
    # at r = sigma the LJ energy is exactly zero
    x2 = np.array([[0.0, 0, 0], [0, sig, 0]])
    assert abs(O.energy_forces(osys, x2)[0]) < 1e-12


def test_coulomb_distance_dependent_dielectric():
    """Single pair with eps(r) = 4r: U = k_e q_i q_j / (4 r^2)."""
    q = np.array([0.37, -0.52])
    for r in (0.2, 0.45, 1.3):
        x = np.array([[0.1, 0.2, 0.3], [0.1 + r * 0.6, 0.2 + r * 0.8, 0.3]])
        sysd = S.System(name="c", n_atoms=2, mass=np.ones(2), charge=q, sigma=np.ones(2),
                        epsilon=np.zeros(2), atype=np.zeros(2, np.int32),
                        bonds=np.zeros((0, 2), np.int32), bond_k=np.zeros(0), bond_r0=np.zeros(0),
                        angles=np.zeros((0, 3), np.int32), angle_k=np.zeros(0),
                        angle_theta0=np.zeros(0), dihedrals=np.zeros((0, 4), np.int32),
                        dih_k=np.zeros(0), dih_n=np.zeros(0, np.int32), dih_delta=np.zeros(0),
                        scale14_lj=0.5, scale14_coul=0.5, coulomb_k=138.935458, dielectric=1,
                        kB=1.0, x_init=x)
        E = O.energy_forces(O.OracleSystem(sysd), x)[0]
        assert abs(E - 138.935458 * q[0] * q[1] / (4 * r * r)) < 1e-12 * abs(E)


def test_bonded_minima_have_zero_force():
    """A bond at r0, an angle at theta0 and a dihedral at a minimum of
    k (1 + cos(n phi - delta)) each exert no force."""
    # bond + angle: three atoms at r0 = 1.1 and theta0 = 1.9 rad
    th = 1.9
    x = np.array([[1.1, 0, 0], [0, 0, 0], [1.1 * math.cos(th), 1.1 * math.sin(th), 0]])
    sysd = S.System(name="ba", n_atoms=3, mass=np.ones(3), charge=np.zeros(3), sigma=np.ones(3),
                    epsilon=np.zeros(3), atype=np.zeros(3, np.int32),
                    bonds=np.array([[0, 1], [1, 2]], np.int32), bond_k=np.full(2, 300.0),
                    bond_r0=np.full(2, 1.1), angles=np.array([[0, 1, 2]], np.int32),
                    angle_k=np.array([50.0]), angle_theta0=np.array([th]),
                    dihedrals=np.zeros((0, 4), np.int32), dih_k=np.zeros(0),
                    dih_n=np.zeros(0, np.int32), dih_delta=np.zeros(0),
                    scale14_lj=1.0, scale14_coul=1.0, coulomb_k=1.0, dielectric=0, kB=1.0, x_init=x)
    E, F = O.energy_forces(O.OracleSystem(sysd), x)
    assert abs(E) < 1e-20 and np.abs(F).max() < 1e-12
    # dihedral: n = 3, delta = 0 has minima at phi = pi/3, pi, 5 pi/3
    sysd = _dihedral_system(3.0, 3, 0.0)
    osys = O.OracleSystem(sysd)
    for phi in (math.pi / 3, math.pi):
        E, F = O.energy_forces(osys, _four_atoms(phi), O.T_DIHEDRAL)
        assert abs(E) < 1e-12 and np.abs(F).max() < 1e-10


def test_net_force_and_torque_vanish():
    """Translation and rotation invariance of U: sum_a F_a = 0, sum_a r_a x F_a = 0."""
    sysd = S.c2_system()
    osys = O.OracleSystem(sysd)
    rng = np.random.default_rng(3)
    x = sysd.x_init + rng.normal(0, 0.01, size=sysd.x_init.shape) + np.array([0.4, -1.3, 2.2])
    E, F = O.energy_forces(osys, x)
    scale = np.abs(F).sum()
    assert np.abs(F.sum(0)).max() < 1e-12 * scale
    torque = np.cross(x, F).sum(0)
    assert np.abs(torque).max() < 1e-11 * scale * np.abs(x).max()
    # and the energy itself is invariant under a rigid rotation + translation
    th = 0.7
    Rm = np.array([[math.cos(th), -math.sin(th), 0], [math.sin(th), math.cos(th), 0], [0, 0, 1]])
    E2 = O.energy_forces(osys, x @ Rm.T - 5.0)[0]
    assert abs(E2 - E) < 1e-11 * abs(E)


@pytest.mark.parametrize("which", ["chain", "peptide"])
def test_pair_list_counts(which):
    """For a tree-shaped molecule (all generated ones are trees) every 1-3 pair
    is one angle and every 1-4 pair is one proper dihedral, so the number of
    non-excluded pairs is N(N-1)/2 - bonds - angles and the number of scaled
    pairs equals the number of dihedrals."""
    sysd = S.c1_system() if which == "chain" else S.c2_system()
    pidx, slj, sc = O.pair_list(sysd.n_atoms, sysd.bonds, 0.5, 0.5)
    n = sysd.n_atoms
    assert len(pidx) == n * (n - 1) // 2 - len(sysd.bonds) - len(sysd.angles)
    assert int((slj == 0.5).sum()) == len(sysd.dihedrals)
    assert int((sc == 0.5).sum()) == len(sysd.dihedrals)
    if which == "chain":
        assert len(pidx) == 28
