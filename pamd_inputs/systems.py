"""Seeded synthetic molecular systems for population-annealing MD.

This module only *builds inputs*: topology (bond, angle and proper-dihedral
lists), per-atom and per-term force-field parameters, masses, types, charges
and initial coordinates.  It evaluates no energy, no force, no integrator
step and no resampling weight; both the FP64 oracle and the GPU library
receive the arrays it produces and derive everything else (exclusion and
1-4 lists included) on their own.

Systems
-------
* ``bead_chain``     -- the reduced-unit 10-bead chain used as the small
  correctness case (harmonic bonds / angles, cosine dihedrals, LJ + Coulomb
  with alternating charges, 1-2 and 1-3 exclusions, no cutoff, vacuum).
* ``make_peptide``   -- a peptide-shaped molecule standing in for the
  paper's met-enkephalin in vacuo (AMBER-style functional form: harmonic
  bonds and angles, Fourier dihedrals, LJ + Coulomb with scaled 1-4 pairs).
  The paper's molecule and ff94 parameters are not reproduced; every
  parameter is drawn from stated ranges with a seeded generator.
* ``gaussian_chain`` / ``spring_pair`` -- tiny analytic systems used as pins.
"""
from __future__ import annotations

import dataclasses
import math
from typing import Dict, List, Optional, Tuple

import numpy as np

# physical constants in kJ/mol, nm, ps, amu, e units
KB_KJ = 0.0083144626          # Boltzmann constant, kJ mol^-1 K^-1
KE_KJ = 138.935458            # Coulomb constant, kJ mol^-1 nm e^-2

DIELECTRIC_VACUUM = 0         # U_C = k_e q_i q_j / r
DIELECTRIC_4R = 1             # distance-dependent dielectric eps(r) = 4 r


@dataclasses.dataclass
class System:
    """Plain-array description of one molecule (all float arrays are float64)."""
    name: str
    n_atoms: int
    mass: np.ndarray            # [N]
    charge: np.ndarray          # [N]
    sigma: np.ndarray           # [N] LJ sigma (Lorentz-Berthelot combined pairwise)
    epsilon: np.ndarray         # [N] LJ epsilon
    atype: np.ndarray           # [N] int32 atom type (0..7)
    bonds: np.ndarray           # [nb, 2] int32
    bond_k: np.ndarray          # [nb]   U = 1/2 k (r - r0)^2
    bond_r0: np.ndarray         # [nb]
    angles: np.ndarray          # [na, 3] int32 (i, centre, k)
    angle_k: np.ndarray         # [na]   U = 1/2 k (theta - theta0)^2
    angle_theta0: np.ndarray    # [na]   radians
    dihedrals: np.ndarray       # [nd, 4] int32
    dih_k: np.ndarray           # [nd]   U = k (1 + cos(n phi - delta))
    dih_n: np.ndarray           # [nd] int32 multiplicity
    dih_delta: np.ndarray       # [nd]   radians
    scale14_lj: float
    scale14_coul: float
    coulomb_k: float
    dielectric: int
    kB: float
    x_init: np.ndarray          # [N, 3]
    units: str = "kJ/mol-nm-ps-amu-e"

    def counts(self) -> Dict[str, int]:
        return dict(atoms=self.n_atoms, bonds=len(self.bonds), angles=len(self.angles),
                    dihedrals=len(self.dihedrals))

    def to_npz(self, path: str) -> None:
        np.savez(path, **{f.name: getattr(self, f.name) for f in dataclasses.fields(self)})

    @staticmethod
    def from_npz(path: str) -> "System":
        d = np.load(path, allow_pickle=False)
        kw = {}
        for f in dataclasses.fields(System):
            v = d[f.name]
            if f.type in ("int", int):
                v = int(v)
            elif f.type in ("float", float):
                v = float(v)
            elif f.type in ("str", str):
                v = str(v)
            kw[f.name] = v
        return System(**kw)


def _i32(a) -> np.ndarray:
    return np.ascontiguousarray(np.asarray(a, dtype=np.int32))


def _f64(a) -> np.ndarray:
    return np.ascontiguousarray(np.asarray(a, dtype=np.float64))


def angles_and_dihedrals_from_bonds(n: int, bonds: np.ndarray) -> Tuple[np.ndarray, np.ndarray]:
    """Enumerate every bond angle (i, centre, k) and every proper dihedral
    (a, b, c, d) of the bond graph.  This is topology enumeration of the
    molecule description, not an energy."""
    nbr: List[List[int]] = [[] for _ in range(n)]
    for a, b in bonds:
        nbr[a].append(int(b))
        nbr[b].append(int(a))
    for l in nbr:
        l.sort()
    ang = []
    for c in range(n):
        for x in range(len(nbr[c])):
            for y in range(x + 1, len(nbr[c])):
                ang.append((nbr[c][x], c, nbr[c][y]))
    dih = []
    for b, c in bonds:
        b, c = int(b), int(c)
        for a in nbr[b]:
            if a == c:
                continue
            for d in nbr[c]:
                if d == b or d == a:
                    continue
                dih.append((a, b, c, d))
    return (_i32(ang).reshape(-1, 3), _i32(dih).reshape(-1, 4))


# ----------------------------------------------------------------------------
# reduced-unit bead chain
# ----------------------------------------------------------------------------

def bead_chain(n: int = 10, seed: int = 1, jitter: float = 0.05) -> System:
    """Linear chain in reduced units (m = 1, k_B = 1, k_e = 1).

    Bonds k = 100, r0 = 1; angles k = 20, theta0 = 109.5 deg; dihedrals k = 1,
    n = 3, delta = 0; LJ sigma = eps = 1; charges +0.2 / -0.2 alternating
    (even atoms positive); 1-2 and 1-3 pairs excluded and 1-4 pairs kept at
    full strength; plain 1/r Coulomb in vacuum.  Start: straight chain along
    x with seeded N(0, jitter^2) per-component noise (a perfectly straight
    chain makes the angle and dihedral gradients singular)."""
    rng = np.random.default_rng(seed)
    bonds = _i32([(i, i + 1) for i in range(n - 1)]).reshape(-1, 2)
    ang, dih = angles_and_dihedrals_from_bonds(n, bonds)
    x = np.zeros((n, 3))
    x[:, 0] = np.arange(n, dtype=np.float64)
    x += rng.normal(0.0, jitter, size=(n, 3))
    q = np.where(np.arange(n) % 2 == 0, 0.2, -0.2)
    return System(
        name=f"bead_chain_{n}", n_atoms=n,
        mass=np.ones(n), charge=_f64(q), sigma=np.ones(n), epsilon=np.ones(n),
        atype=np.zeros(n, np.int32),
        bonds=bonds, bond_k=np.full(len(bonds), 100.0), bond_r0=np.ones(len(bonds)),
        angles=ang, angle_k=np.full(len(ang), 20.0),
        angle_theta0=np.full(len(ang), math.radians(109.5)),
        dihedrals=dih, dih_k=np.ones(len(dih)), dih_n=np.full(len(dih), 3, np.int32),
        dih_delta=np.zeros(len(dih)),
        scale14_lj=1.0, scale14_coul=1.0, coulomb_k=1.0, dielectric=DIELECTRIC_VACUUM,
        kB=1.0, x_init=_f64(x), units="reduced")


def branched_pair(seed: int = 3, jitter: float = 0.04) -> System:
    """Two six-coordinated hubs joined by one bond, in reduced units: hub 0 and
    hub 1 each carry five leaves (12 atoms, 11 bonds), so each hub is the centre
    of 15 angles and the hub-hub bond is the central bond of 25 torsions; the
    torsions with i = leaf 2 carry a second term (n = 1, delta = pi) besides
    the n = 3 one, as force fields often stack terms on one quadruple.  Masses
    1..3, charges +-0.2, LJ sigma 0.6, epsilon 0.5; 1-4 pairs scaled by 0.5
    (LJ) and 0.8 (Coulomb).  Start: leaves on two cones about the hub axis,
    with seeded N(0, jitter^2) noise."""
    rng = np.random.default_rng(seed)
    n = 12
    bonds = [(0, 1)] + [(0, a) for a in range(2, 7)] + [(1, a) for a in range(7, 12)]
    bonds = _i32(bonds).reshape(-1, 2)
    ang, dih = angles_and_dihedrals_from_bonds(n, bonds)
    dih = np.asarray(dih, np.int32).reshape(-1, 4)
    extra = [d for d in dih if 2 in (d[0], d[3])]
    dih_all = np.concatenate([dih, np.asarray(extra, np.int32).reshape(-1, 4)])
    dk = np.concatenate([np.full(len(dih), 1.5), np.full(len(extra), 0.7)])
    dn = np.concatenate([np.full(len(dih), 3), np.full(len(extra), 1)]).astype(np.int32)
    dd = np.concatenate([np.zeros(len(dih)), np.full(len(extra), math.pi)])
    x = np.zeros((n, 3))
    x[1] = (1.0, 0.0, 0.0)
    for q in range(5):
        phi = 2 * math.pi * q / 5
        x[2 + q] = (-0.45, 0.9 * math.cos(phi), 0.9 * math.sin(phi))
        x[7 + q] = (1.45, 0.9 * math.cos(phi + 0.3), 0.9 * math.sin(phi + 0.3))
    x += rng.normal(0.0, jitter, size=(n, 3))
    q = np.where(np.arange(n) % 2 == 0, 0.2, -0.2)
    return System(
        name="branched_pair", n_atoms=n,
        mass=1.0 + (np.arange(n) % 3).astype(np.float64), charge=_f64(q), sigma=np.full(n, 0.6),
        epsilon=np.full(n, 0.5), atype=(np.arange(n) % 8).astype(np.int32),
        bonds=bonds, bond_k=np.full(len(bonds), 100.0), bond_r0=np.ones(len(bonds)),
        angles=np.asarray(ang, np.int32).reshape(-1, 3), angle_k=np.full(len(ang), 20.0),
        angle_theta0=np.full(len(ang), math.radians(100.0)),
        dihedrals=dih_all, dih_k=dk, dih_n=dn, dih_delta=dd,
        scale14_lj=0.5, scale14_coul=0.8, coulomb_k=1.0, dielectric=DIELECTRIC_VACUUM,
        kB=1.0, x_init=_f64(x), units="reduced")


def gaussian_chain(n: int = 10, k: float = 100.0, r0: float = 0.0) -> System:
    """Bonds-only chain in reduced units: no angles, dihedrals or nonbonded
    interactions (epsilon = charge = 0).  With r0 = 0 every bond vector is an
    independent 3-D Gaussian, which gives closed forms for the partition
    function and the mean energy."""
    bonds = _i32([(i, i + 1) for i in range(n - 1)]).reshape(-1, 2)
    x = np.zeros((n, 3))
    x[:, 0] = np.arange(n, dtype=np.float64) * max(r0, 0.1)
    return System(
        name=f"gaussian_chain_{n}_r0_{r0}", n_atoms=n,
        mass=np.ones(n), charge=np.zeros(n), sigma=np.ones(n), epsilon=np.zeros(n),
        atype=np.zeros(n, np.int32),
        bonds=bonds, bond_k=np.full(n - 1, float(k)), bond_r0=np.full(n - 1, float(r0)),
        angles=np.zeros((0, 3), np.int32), angle_k=np.zeros(0), angle_theta0=np.zeros(0),
        dihedrals=np.zeros((0, 4), np.int32), dih_k=np.zeros(0), dih_n=np.zeros(0, np.int32),
        dih_delta=np.zeros(0),
        scale14_lj=1.0, scale14_coul=1.0, coulomb_k=1.0, dielectric=DIELECTRIC_VACUUM,
        kB=1.0, x_init=_f64(x), units="reduced")


def spring_pair(k: float = 50.0, m1: float = 1.0, m2: float = 3.0) -> System:
    """Two particles joined by a zero-rest-length spring, nothing else."""
    x = np.array([[0.3, -0.2, 0.1], [-0.1, 0.4, 0.25]])
    return System(
        name="spring_pair", n_atoms=2,
        mass=_f64([m1, m2]), charge=np.zeros(2), sigma=np.ones(2), epsilon=np.zeros(2),
        atype=np.zeros(2, np.int32),
        bonds=_i32([[0, 1]]), bond_k=_f64([k]), bond_r0=_f64([0.0]),
        angles=np.zeros((0, 3), np.int32), angle_k=np.zeros(0), angle_theta0=np.zeros(0),
        dihedrals=np.zeros((0, 4), np.int32), dih_k=np.zeros(0), dih_n=np.zeros(0, np.int32),
        dih_delta=np.zeros(0),
        scale14_lj=1.0, scale14_coul=1.0, coulomb_k=1.0, dielectric=DIELECTRIC_VACUUM,
        kB=1.0, x_init=x, units="reduced")


# ----------------------------------------------------------------------------
# peptide-shaped molecule
# ----------------------------------------------------------------------------

# atom types: (name, element mass)
ATOM_TYPES = [
    ("H_apolar", 1.008),   # 0: H bonded to carbon
    ("H_polar", 1.008),    # 1: H bonded to N / O / S
    ("C_sp3", 12.011),     # 2
    ("C_sp2", 12.011),     # 3
    ("N", 14.007),         # 4
    ("O_carbonyl", 15.999),  # 5
    ("O_hydroxyl", 15.999),  # 6
    ("S", 32.06),          # 7
]
N_TYPES = len(ATOM_TYPES)

TETRA = math.acos(-1.0 / 3.0)   # ideal sp3 angle, 109.47 deg
TRIG = 2.0 * math.pi / 3.0      # ideal sp2 angle, 120 deg

# heavy atom kinds: element, hybridisation ('sp3' | 'sp2' | 'term'), valence, type
_HEAVY = {
    "C3": ("C", "sp3", 4, 2),
    "C2": ("C", "sp2", 3, 3),     # carbonyl / amide carbon (one double bond)
    "N2": ("N", "sp2", 3, 4),     # amide nitrogen
    "N3": ("N", "sp3", 4, 4),     # amine nitrogen (protonated)
    "O=": ("O", "term", 1, 5),    # carbonyl oxygen (double bond: no H)
    "OH": ("O", "sp3", 2, 6),
    "S2": ("S", "sp3", 2, 7),
}

# acyclic side chains: list of (kind, parent index; -1 = CA)
_SIDECHAINS = {
    "GLY": [],
    "ALA": [("C3", -1)],
    "SER": [("C3", -1), ("OH", 0)],
    "CYS": [("C3", -1), ("S2", 0)],
    "ABU": [("C3", -1), ("C3", 0)],
    "VAL": [("C3", -1), ("C3", 0), ("C3", 0)],
    "THR": [("C3", -1), ("OH", 0), ("C3", 0)],
    "ASN": [("C3", -1), ("C2", 0), ("O=", 1), ("N2", 1)],
    "LEU": [("C3", -1), ("C3", 0), ("C3", 1), ("C3", 1)],
    "ILE": [("C3", -1), ("C3", 0), ("C3", 0), ("C3", 1)],
    "MET": [("C3", -1), ("C3", 0), ("S2", 1), ("C3", 2)],
    "LYS": [("C3", -1), ("C3", 0), ("C3", 1), ("C3", 2), ("N3", 3)],
}


class _Mol:
    def __init__(self):
        self.kind: List[str] = []      # heavy kind or 'H'
        self.parent: List[int] = []
        self.children: List[List[int]] = []
        self.role: List[str] = []      # backbone role for dihedral choice

    def add(self, kind: str, parent: int, role: str = "") -> int:
        i = len(self.kind)
        self.kind.append(kind)
        self.parent.append(parent)
        self.children.append([])
        self.role.append(role)
        if parent >= 0:
            self.children[parent].append(i)
        return i

    def valence(self, i: int) -> int:
        return 1 if self.kind[i] == "H" else _HEAVY[self.kind[i]][2]

    def degree(self, i: int) -> int:
        return len(self.children[i]) + (1 if self.parent[i] >= 0 else 0)

    def saturate(self, i: int) -> None:
        while self.degree(i) < self.valence(i):
            self.add("H", i)


def _residue_atoms(name: str) -> int:
    sc = _SIDECHAINS[name]
    m = _Mol()
    ca = m.add("C3", -1)
    idx = []
    for kind, p in sc:
        idx.append(m.add(kind, ca if p < 0 else idx[p]))
    # CA keeps N, C neighbours + side chain + H; side chain atoms saturated
    n_sc_heavy = len(sc)
    n_h = 0
    for j, (kind, p) in enumerate(sc):
        deg = 1 + sum(1 for (_, pp) in sc if pp == j)
        n_h += _HEAVY[kind][2] - deg
    n_ca_h = 4 - 2 - (1 if sc else 0)     # CA: N, C, (CB) + H's
    return 6 - 1 + n_ca_h + n_sc_heavy + n_h   # N H CA C O + HA's + side chain


_RES_SIZE = {k: _residue_atoms(k) for k in _SIDECHAINS}


def _choose_residues(n_atoms: int, rng: np.random.Generator) -> List[str]:
    caps = 12                       # acetyl (6 atoms) + N-methylamide (6 atoms)
    target = n_atoms - caps
    names = sorted(_SIDECHAINS)
    sizes = sorted(set(_RES_SIZE.values()))
    n_res = max(1, int(round(target / 12.6)))   # 5 residues for 75 atoms
    for _ in range(100000):
        res = [names[rng.integers(len(names))] for _ in range(n_res - 1)]
        rest = target - sum(_RES_SIZE[r] for r in res)
        fits = [r for r in names if _RES_SIZE[r] == rest]
        if fits:
            res.append(fits[rng.integers(len(fits))])
            return res
    raise ValueError(f"cannot compose a peptide with {n_atoms} atoms from sizes {sizes}")


def _build_topology(res_names: List[str]) -> _Mol:
    m = _Mol()
    # acetyl cap: H-CH2-C(=O)-  ; the tree is rooted at one methyl hydrogen
    h0 = m.add("H", -1)
    cm = m.add("C3", h0)
    cc = m.add("C2", cm, role="C")
    prev_c = cc
    for r in res_names:
        n = m.add("N2", prev_c, role="N")
        m.add("H", n)
        ca = m.add("C3", n, role="CA")
        c = m.add("C2", ca, role="C")
        sc_idx = []
        for kind, p in _SIDECHAINS[r]:
            sc_idx.append(m.add(kind, ca if p < 0 else sc_idx[p], role="SC"))
        for j in sc_idx:
            m.saturate(j)
        m.saturate(ca)
        prev_c_old = prev_c
        # carbonyl O of the previous C is added when that C is closed below
        m.add("O=", prev_c_old)
        prev_c = c
    # N-methylamide cap
    n = m.add("N2", prev_c, role="N")
    m.add("H", n)
    m.add("O=", prev_c)
    cme = m.add("C3", n, role="SC")
    m.saturate(cme)
    m.saturate(cm)
    return m


def _nerf(a, b, c, bond, angle, torsion):
    bc = c - b
    bc /= np.linalg.norm(bc)
    nrm = np.cross(b - a, bc)
    nrm /= np.linalg.norm(nrm)
    mm = np.cross(nrm, bc)
    d2 = np.array([-bond * math.cos(angle),
                   bond * math.sin(angle) * math.cos(torsion),
                   bond * math.sin(angle) * math.sin(torsion)])
    return c + d2[0] * bc + d2[1] * mm + d2[2] * nrm


def _graph_dist(n: int, bonds: np.ndarray, maxd: int = 3) -> np.ndarray:
    nbr = [[] for _ in range(n)]
    for a, b in bonds:
        nbr[a].append(b)
        nbr[b].append(a)
    dist = np.full((n, n), 99, np.int32)
    for s in range(n):
        dist[s, s] = 0
        frontier = [s]
        for d in range(1, maxd + 1):
            nxt = []
            for u in frontier:
                for w in nbr[u]:
                    if dist[s, w] > d:
                        dist[s, w] = d
                        nxt.append(w)
            frontier = nxt
    return dist


def make_peptide(seed: int = 1806, n_atoms: int = 75) -> System:
    """Seeded peptide-shaped molecule of exactly ``n_atoms`` atoms.

    Acetyl cap + residues drawn from a library of acyclic side chains + an
    N-methylamide cap, so the bond graph is a tree (N - 1 bonds).  Parameters:
    bond k = 2e5 kJ mol^-1 nm^-2 with r0 drawn in [0.100, 0.110] nm for X-H and
    [0.130, 0.150] nm for heavy-heavy bonds; angle k = 400 kJ mol^-1 rad^-2 with
    theta0 the ideal sp3 / sp2 angle of the centre (so the built geometry sits
    at the bond and angle minima); dihedrals k in [0, 10] kJ/mol, n in
    {1, 2, 3}, delta in {0, pi}; 8 atom types with element masses and
    per-type sigma in [0.25, 0.37] nm, epsilon in [0.1, 0.8] kJ/mol; charges
    N(0, 0.3^2) e per atom, shifted to zero net charge (the two hydrogen
    types draw sigma from [0.25, 0.27] nm, heavy types from [0.29, 0.37] nm); 1-4 pairs scaled by
    0.5 (LJ and Coulomb); distance-dependent dielectric 4r.  Coordinates come
    from internal coordinates (backbone phi/psi in the extended / helical
    basins, trans amides, staggered side chains), redrawn until no
    non-excluded pair is closer than a clash threshold."""
    rng = np.random.default_rng(seed)
    res = _choose_residues(n_atoms, rng)
    m = _build_topology(res)
    n = len(m.kind)
    assert n == n_atoms, (n, n_atoms, res)
    bonds = _i32([(m.parent[i], i) for i in range(n) if m.parent[i] >= 0])
    ang, dih = angles_and_dihedrals_from_bonds(n, bonds)

    # types and masses
    atype = np.zeros(n, np.int32)
    for i, k in enumerate(m.kind):
        if k == "H":
            p = m.parent[i]
            atype[i] = 0 if m.kind[p] in ("C3", "C2") else 1
        else:
            atype[i] = _HEAVY[k][3]
    mass = _f64([ATOM_TYPES[t][1] for t in atype])

    # hybridisation of each centre -> ideal angle
    def ideal_angle(c: int) -> float:
        k = m.kind[c]
        if k == "H":
            return TETRA
        hyb = _HEAVY[k][1]
        return TRIG if hyb == "sp2" else TETRA

    # bond lengths
    r0 = np.zeros(len(bonds))
    for b, (p, c) in enumerate(bonds):
        is_h = m.kind[p] == "H" or m.kind[c] == "H"
        r0[b] = rng.uniform(0.100, 0.110) if is_h else rng.uniform(0.130, 0.150)
    bond_len = {int(c): r0[b] for b, (p, c) in enumerate(bonds)}

    theta0 = _f64([ideal_angle(int(c)) for (_, c, _) in ang])

    # per-type LJ (hydrogen types from the low end of the sigma range), per-atom charge
    sig_t = np.concatenate([rng.uniform(0.25, 0.27, size=2), rng.uniform(0.29, 0.37, size=N_TYPES - 2)])
    eps_t = rng.uniform(0.1, 0.8, size=N_TYPES)
    q = rng.normal(0.0, 0.3, size=n)
    q -= q.mean()

    # dihedral parameters
    nd = len(dih)
    dih_k = rng.uniform(0.0, 10.0, size=nd)
    dih_n = rng.integers(1, 4, size=nd).astype(np.int32)
    dih_delta = np.where(rng.integers(0, 2, size=nd) == 1, math.pi, 0.0)

    gd = _graph_dist(n, bonds, 3)
    geo_rng = np.random.default_rng(seed * 7919 + 13)
    x = _place(m, bond_len, ideal_angle, geo_rng, gd, sig_t[atype])
    x -= x.mean(axis=0)

    return System(
        name=f"peptide_{n}_s{seed}", n_atoms=n, mass=mass, charge=_f64(q),
        sigma=_f64(sig_t[atype]), epsilon=_f64(eps_t[atype]), atype=atype,
        bonds=bonds, bond_k=np.full(len(bonds), 2.0e5), bond_r0=_f64(r0),
        angles=ang, angle_k=np.full(len(ang), 400.0), angle_theta0=theta0,
        dihedrals=dih, dih_k=_f64(dih_k), dih_n=dih_n, dih_delta=_f64(dih_delta),
        scale14_lj=0.5, scale14_coul=0.5, coulomb_k=KE_KJ, dielectric=DIELECTRIC_4R,
        kB=KB_KJ, x_init=_f64(x))


def _draw_torsion(role: str, rng) -> float:
    if role == "N":              # omega about C-N: trans amide
        return math.pi
    if role == "CA":             # backbone phi
        return math.radians(rng.choice([-65.0, -120.0]) + rng.normal(0, 12))
    if role == "C":              # backbone psi
        return math.radians(rng.choice([-40.0, 130.0]) + rng.normal(0, 12))
    return math.radians(rng.choice([60.0, 180.0, 300.0]) + rng.normal(0, 10))


def _build_xyz(m: _Mol, bond_len, ideal_angle, tors: Dict[int, float]) -> np.ndarray:
    """Internal coordinates -> Cartesian: each centre's children get bond
    length r0, the centre's ideal angle and torsions tors[c] + t * (120 deg at
    sp3 / 180 deg at sp2 centres)."""
    n = len(m.kind)
    x = np.zeros((n, 3))
    anc = {-1: np.array([-0.10, 0.0, 0.0]), -2: np.array([-0.15, 0.10, 0.0])}
    par = m.parent

    def pos(i):
        return anc[i] if i < 0 else x[i]

    order = [0]
    k = 0
    while k < len(order):
        c = order[k]
        k += 1
        kids = m.children[c]
        if not kids:
            continue
        if c == 0:
            b, a = -1, -2
        else:
            b = par[c]
            a = par[b] if par[b] >= 0 else -1
        kind = m.kind[c]
        hyb = "sp3" if kind == "H" else _HEAVY[kind][1]
        step = math.pi if hyb == "sp2" else 2.0 * math.pi / 3.0
        for t, d in enumerate(sorted(kids, key=lambda j: (m.kind[j] == "H", j))):
            x[d] = _nerf(pos(a), pos(b), x[c], bond_len[d], ideal_angle(c), tors[c] + t * step)
            order.append(d)
    return x


def _place(m: _Mol, bond_len, ideal_angle, rng, gd, sig: np.ndarray,
           max_iter: int = 1500) -> np.ndarray:
    """Torsion-space clash repair: start from peptide-like torsions, then
    repeatedly redraw one rotatable torsion on the tree path between the
    worst-clashing pair, keeping the change when the smallest distance ratio
    does not drop.  Only pairs four or more bonds apart are repaired (1-4
    distances follow from bond lengths, angles and torsions of one bond);
    the reference distance is 0.75 sigma_ij (sigma_ij the arithmetic mean)."""
    n = len(m.kind)
    centres = [c for c in range(n) if m.children[c]]
    tors = {c: _draw_torsion(m.role[c], rng) for c in centres}
    iu = np.triu_indices(n, 1)
    g = gd[iu]
    far = g >= 4
    sij = 0.5 * (sig[iu[0]] + sig[iu[1]])
    thr = 0.75 * sij[far]
    ia, ja = iu[0][far], iu[1][far]

    def score(x):
        r = np.linalg.norm(x[ia] - x[ja], axis=1) / thr
        w = int(np.argmin(r))
        return float(r[w]), int(ia[w]), int(ja[w])

    def path(i, j):
        anc_i = []
        u = i
        while u >= 0:
            anc_i.append(u)
            u = m.parent[u]
        si = set(anc_i)
        pj = []
        u = j
        while u not in si:
            pj.append(u)
            u = m.parent[u]
        lca = u
        pi = anc_i[:anc_i.index(lca) + 1]
        return pi + pj

    x = _build_xyz(m, bond_len, ideal_angle, tors)
    sc, wi, wj = score(x)
    for _ in range(max_iter):
        if sc >= 1.0:
            break
        cand = [c for c in path(wi, wj) if c in tors and m.role[c] != "N"]
        if not cand:
            cand = [c for c in centres if m.role[c] != "N"]
        c = cand[rng.integers(len(cand))]
        old = tors[c]
        tors[c] = rng.uniform(0.0, 2.0 * math.pi)
        x2 = _build_xyz(m, bond_len, ideal_angle, tors)
        sc2, wi2, wj2 = score(x2)
        if sc2 >= sc:
            x, sc, wi, wj = x2, sc2, wi2, wj2
        else:
            tors[c] = old
    return x


# ----------------------------------------------------------------------------
# named workloads
# ----------------------------------------------------------------------------

def c1_system(seed: int = 1) -> System:
    return bead_chain(10, seed=seed)


def c2_system(seed: int = 1806) -> System:
    return make_peptide(seed=seed, n_atoms=75)


C4_SIZES = (40, 75, 75, 120, 150, 200, 250, 300)


def c4_systems() -> List[System]:
    return [make_peptide(seed=1806 + k, n_atoms=nk) for k, nk in enumerate(C4_SIZES)]


def geometric_schedule(t0: float, t_end: float, n_steps: int) -> np.ndarray:
    """T_i = t0 (t_end / t0)^(i / n_steps), i = 0..n_steps (n_steps decrements)."""
    i = np.arange(n_steps + 1, dtype=np.float64)
    return t0 * (t_end / t0) ** (i / n_steps)
