"""FP64 CPU oracle for the PAMD hot path -- TEST INFRASTRUCTURE ONLY.

Only ``tests/``, ``__graft_entry__.smoke()`` and the ``cpu_baseline`` leg of
``bench.py`` may import this module.  It shares no code with the GPU library
(``paper_1806_06016_amd``) and never imports it.

It wraps ``oracle.c`` (liboracle.so, built with gcc) and adds the plain
numpy / pure-Python pieces that are clearer that way: the exclusion and 1-4
lists from the bond graph, the gather of resampled copies, population
observables, the adaptive temperature bisection and the annealing driver.

Paper: Christiansen, Weigel & Janke, arXiv:1806.06016.  Section references
below name the numbered PAMD scheme (steps 1-5), the resampling paragraph
after it, and the free-energy paragraph (recorded normalisers Q).
"""
from __future__ import annotations

import ctypes as C
import math
import os
import subprocess
from dataclasses import dataclass, field
from typing import Dict, List, Optional, Sequence

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")

T_BOND, T_ANGLE, T_DIHEDRAL, T_LJ, T_COUL, T_ALL = 1, 2, 4, 8, 16, 31


def build(force: bool = False) -> str:
    """Compile oracle.c into liboracle.so (gcc, -O2, OpenMP)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        subprocess.check_call(["gcc", "-O2", "-fopenmp", "-fPIC", "-shared", "-o", _LIB, _SRC, "-lm"])
    return _LIB


class _OraSys(C.Structure):
    _fields_ = [
        ("n", C.c_int32), ("mass", C.c_void_p), ("charge", C.c_void_p), ("sigma", C.c_void_p),
        ("eps", C.c_void_p),
        ("nb", C.c_int32), ("bidx", C.c_void_p), ("bk", C.c_void_p), ("br0", C.c_void_p),
        ("na", C.c_int32), ("aidx", C.c_void_p), ("ak", C.c_void_p), ("at0", C.c_void_p),
        ("nd", C.c_int32), ("didx", C.c_void_p), ("dk", C.c_void_p), ("dn", C.c_void_p),
        ("ddelta", C.c_void_p),
        ("np", C.c_int32), ("pidx", C.c_void_p), ("ps_lj", C.c_void_p), ("ps_c", C.c_void_p),
        ("coulomb_k", C.c_double), ("dielectric", C.c_int32), ("pad", C.c_int32),
    ]


class _OraRng(C.Structure):
    _fields_ = [("seed_lo", C.c_uint32), ("seed_hi", C.c_uint32), ("run", C.c_uint32),
                ("pad", C.c_uint32)]


class _OraMd(C.Structure):
    _fields_ = [("dt", C.c_double), ("kB", C.c_double), ("T", C.c_double), ("p24", C.c_uint32),
                ("step0", C.c_uint32), ("n_steps", C.c_int32), ("mask", C.c_int32),
                ("gamma", C.c_double), ("langevin", C.c_int32), ("pad", C.c_int32)]


_lib = None


def lib():
    global _lib
    if _lib is None:
        # PAMD_ORACLE_LIB: another build of oracle.c (the sanitizer test uses it)
        _lib = C.CDLL(os.environ.get("PAMD_ORACLE_LIB") or build())
        vp, i32, i64, d = C.c_void_p, C.c_int32, C.c_int64, C.c_double
        _lib.ora_philox4x32_10.argtypes = [vp, vp, vp]
        _lib.ora_energy_forces.argtypes = [vp, vp, vp, vp, i32]
        _lib.ora_energy_forces.restype = d
        _lib.ora_energy_forces_batch.argtypes = [vp, i32, vp, vp, vp, vp, i32]
        _lib.ora_init_velocities.argtypes = [vp, vp, i32, vp, d, d, vp]
        _lib.ora_md_steps.argtypes = [vp, vp, vp, i32, vp, vp, vp, vp, vp, vp]
        _lib.ora_lse.argtypes = [i64, vp, d, vp, vp, vp, vp]
        _lib.ora_lse.restype = i32
        _lib.ora_resample_uniforms.argtypes = [vp, i64, C.c_uint32, vp]
        _lib.ora_multinomial_uniforms.argtypes = [vp, i64, C.c_uint32, vp]
        _lib.ora_counts.argtypes = [i64, vp, d, d, d, i64, vp, vp, vp]
        _lib.ora_counts.restype = i64
        _lib.ora_weight_variance.argtypes = [i64, vp, d]
        _lib.ora_weight_variance.restype = d
    return _lib


def _p(a: Optional[np.ndarray]):
    return None if a is None else a.ctypes.data


# ----------------------------------------------------------------------------
# topology: exclusions and 1-4 pairs from the bond graph
# ----------------------------------------------------------------------------

def pair_list(n: int, bonds: np.ndarray, scale14_lj: float, scale14_coul: float):
    """All unordered pairs i < j except those 1 or 2 bonds apart; pairs exactly
    3 bonds apart (1-4) carry the 1-4 scale factors, all others scale 1."""
    nbr: List[set] = [set() for _ in range(n)]
    for a, b in bonds:
        nbr[int(a)].add(int(b))
        nbr[int(b)].add(int(a))
    dist = [dict() for _ in range(n)]
    for s in range(n):
        dist[s][s] = 0
        frontier = [s]
        for d in (1, 2, 3):
            nxt = []
            for u in frontier:
                for w in nbr[u]:
                    if w not in dist[s]:
                        dist[s][w] = d
                        nxt.append(w)
            frontier = nxt
    idx, slj, sc = [], [], []
    for i in range(n):
        for j in range(i + 1, n):
            d = dist[i].get(j, 99)
            if d <= 2:
                continue
            idx.append((i, j))
            if d == 3:
                slj.append(scale14_lj)
                sc.append(scale14_coul)
            else:
                slj.append(1.0)
                sc.append(1.0)
    return (np.ascontiguousarray(np.array(idx, np.int32).reshape(-1, 2)),
            np.ascontiguousarray(np.array(slj, np.float64)),
            np.ascontiguousarray(np.array(sc, np.float64)))


class OracleSystem:
    """Holds the C descriptor and keeps the numpy arrays it points to alive."""

    def __init__(self, sysd):
        self.src = sysd
        self.n = int(sysd.n_atoms)
        self.mass = np.ascontiguousarray(sysd.mass, np.float64)
        self.kB = float(sysd.kB)
        keep = {}

        def f64(a):
            a = np.ascontiguousarray(a, np.float64)
            keep[id(a)] = a
            return a

        def i32(a):
            a = np.ascontiguousarray(a, np.int32)
            keep[id(a)] = a
            return a

        self.pidx, self.ps_lj, self.ps_c = pair_list(self.n, sysd.bonds, sysd.scale14_lj,
                                                     sysd.scale14_coul)
        s = _OraSys()
        s.n = self.n
        s.mass = _p(f64(sysd.mass)); s.charge = _p(f64(sysd.charge))
        s.sigma = _p(f64(sysd.sigma)); s.eps = _p(f64(sysd.epsilon))
        s.nb = len(sysd.bonds); s.bidx = _p(i32(sysd.bonds)); s.bk = _p(f64(sysd.bond_k))
        s.br0 = _p(f64(sysd.bond_r0))
        s.na = len(sysd.angles); s.aidx = _p(i32(sysd.angles)); s.ak = _p(f64(sysd.angle_k))
        s.at0 = _p(f64(sysd.angle_theta0))
        s.nd = len(sysd.dihedrals); s.didx = _p(i32(sysd.dihedrals)); s.dk = _p(f64(sysd.dih_k))
        s.dn = _p(i32(sysd.dih_n)); s.ddelta = _p(f64(sysd.dih_delta))
        s.np = len(self.pidx); s.pidx = _p(self.pidx); s.ps_lj = _p(self.ps_lj)
        s.ps_c = _p(self.ps_c)
        s.coulomb_k = float(sysd.coulomb_k); s.dielectric = int(sysd.dielectric)
        self._keep = keep
        self.c = s

    @property
    def ref(self):
        return C.byref(self.c)


def _rng(seed: int, run: int = 0) -> _OraRng:
    g = _OraRng()
    g.seed_lo = seed & 0xFFFFFFFF
    g.seed_hi = (seed >> 32) & 0xFFFFFFFF
    g.run = run
    return g


def philox(ctr: Sequence[int], key: Sequence[int]) -> np.ndarray:
    c = np.ascontiguousarray(np.array(ctr, np.uint32))
    k = np.ascontiguousarray(np.array(key, np.uint32))
    o = np.zeros(4, np.uint32)
    lib().ora_philox4x32_10(_p(c), _p(k), _p(o))
    return o


def collision_p24(nu: float, dt: float) -> int:
    """Andersen collision probability per atom and step, p = 1 - exp(-nu dt),
    as a 24-bit integer threshold round(p 2^24)."""
    return int(round((1.0 - math.exp(-nu * dt)) * 16777216.0))


# ----------------------------------------------------------------------------
# energies / forces, MD
# ----------------------------------------------------------------------------

def energy_forces(osys: OracleSystem, x: np.ndarray, mask: int = T_ALL, want_terms: bool = False):
    """x: [R, n, 3] or [n, 3].  Returns (E [R], F [R, n, 3][, terms [R, 5]])."""
    x = np.ascontiguousarray(x, np.float64)
    single = x.ndim == 2
    xb = x.reshape(-1, osys.n, 3)
    R = xb.shape[0]
    F = np.zeros_like(xb)
    E = np.zeros(R)
    terms = np.zeros((R, 5)) if want_terms else None
    lib().ora_energy_forces_batch(osys.ref, R, _p(xb), _p(F), _p(E), _p(terms), mask)
    if single:
        out = (E[0], F[0]) + ((terms[0],) if want_terms else ())
    else:
        out = (E, F) + ((terms,) if want_terms else ())
    return out


def init_velocities(osys: OracleSystem, R: int, T: float, seed: int, run: int = 0,
                    slots: Optional[np.ndarray] = None) -> np.ndarray:
    """PAMD step 1 velocities: Maxwell-Boltzmann at T from stream 3."""
    v = np.zeros((R, osys.n, 3))
    g = _rng(seed, run)
    sl = None if slots is None else np.ascontiguousarray(slots, np.uint32)
    lib().ora_init_velocities(osys.ref, C.byref(g), R, _p(sl), osys.kB, float(T), _p(v))
    return v


def md_steps(osys: OracleSystem, x: np.ndarray, v: np.ndarray, n_steps: int, T: float, dt: float,
             nu: float, seed: int, step0: int, run: int = 0, slots: Optional[np.ndarray] = None,
             mask: int = T_ALL, p24: Optional[int] = None, want_collisions: bool = False,
             thermostat: str = "andersen"):
    """PAMD step 3 on every replica (in place on x, v [R, n, 3]).  thermostat
    "andersen" (nu = collision frequency) or "langevin" (nu = friction gamma,
    B-A-O-A-B splitting).  Returns (E_pot [R], E_kin [R][, collisions [R]])."""
    assert x.flags.c_contiguous and v.flags.c_contiguous and x.dtype == np.float64
    R = x.shape[0]
    g = _rng(seed, run)
    p = _OraMd()
    p.dt = dt; p.kB = osys.kB; p.T = float(T)
    p.p24 = collision_p24(nu, dt) if p24 is None else int(p24)
    p.step0 = int(step0); p.n_steps = int(n_steps); p.mask = mask
    p.langevin = {"andersen": 0, "langevin": 1}[thermostat]
    p.gamma = float(nu)
    if p.langevin:
        p.p24 = 0
    Ep = np.zeros(R)
    Ek = np.zeros(R)
    col = np.zeros(R, np.int64) if want_collisions else None
    sl = None if slots is None else np.ascontiguousarray(slots, np.uint32)
    lib().ora_md_steps(osys.ref, C.byref(g), C.byref(p), R, _p(sl), _p(x), _p(v), _p(Ep), _p(Ek),
                       _p(col))
    return (Ep, Ek, col) if want_collisions else (Ep, Ek)


# ----------------------------------------------------------------------------
# resampling (PAMD step 2)
# ----------------------------------------------------------------------------

def lse(E: np.ndarray, dbeta: float):
    """min m, S = sum exp(-dbeta (E - m)), S2, ln Q = -dbeta m + ln S - ln R."""
    E = np.ascontiguousarray(E, np.float64)
    m, S, S2, lq = C.c_double(), C.c_double(), C.c_double(), C.c_double()
    st = lib().ora_lse(len(E), _p(E), float(dbeta), C.byref(m), C.byref(S), C.byref(S2), C.byref(lq))
    if st != 0:
        raise FloatingPointError("non-finite energy")
    return m.value, S.value, S2.value, lq.value


def resample_uniforms(R: int, temp_index: int, seed: int, run: int = 0) -> np.ndarray:
    u = np.zeros(R)
    g = _rng(seed, run)
    lib().ora_resample_uniforms(C.byref(g), R, temp_index, _p(u))
    return u


def copy_counts(E: np.ndarray, dbeta: float, R_target: int, u: np.ndarray, m=None, S=None):
    """Nearest-integer resampling with random rounding.  Returns (c [R], tau [R])."""
    E = np.ascontiguousarray(E, np.float64)
    u = np.ascontiguousarray(u, np.float64)
    if m is None:
        m, S, _, _ = lse(E, dbeta)
    c = np.zeros(len(E), np.int32)
    tau = np.zeros(len(E))
    lib().ora_counts(len(E), _p(E), float(dbeta), float(m), float(S), int(R_target), _p(u), _p(c),
                     _p(tau))
    return c, tau


def multinomial_uniforms(n_draws: int, temp_index: int, seed: int, run: int = 0) -> np.ndarray:
    """Uniforms of the multinomial draws: Philox stream 4, counter (k, i, 0, 4)."""
    u = np.zeros(n_draws)
    g = _rng(seed, run)
    lib().ora_multinomial_uniforms(C.byref(g), n_draws, temp_index, _p(u))
    return u


def multinomial_counts(E: np.ndarray, dbeta: float, u: np.ndarray, m=None):
    """The paper's resampling rule (PAMD step 2 and the paragraph after it):
    len(u) independent draws from the categorical distribution p_j = w_j / sum w
    (the tau_j / R of the scheme), w_j = exp(-dbeta (E_j - m)).  Draw k picks the
    first j whose running sum W_j = w_0 + ... + w_j exceeds u_k W_{R-1}; should
    rounding leave no such j (u_k W_{R-1} == W_{R-1}), the first j with
    W_j == W_{R-1}.  Returns (c [R], W [R]); sum c = len(u)."""
    E = np.ascontiguousarray(E, np.float64)
    if m is None:
        m = float(E.min())
    w = np.exp(-dbeta * (E - m))
    W = np.cumsum(w)                      # left to right
    t = np.asarray(u, np.float64) * W[-1]
    j = np.searchsorted(W, t, side="right")
    tail = j >= len(E)
    j[tail] = np.searchsorted(W, t[tail], side="left")
    return np.bincount(j, minlength=len(E)).astype(np.int32), W


def resampling_counts(mode: str, E: np.ndarray, dbeta: float, R_target: int, temp_index: int,
                      seed: int, run: int = 0, m=None, S=None) -> np.ndarray:
    """Copy numbers of one resampling in the given mode: "nearest" (random
    rounding of tau_j, stream 2), "multinomial" (R_target draws, stream 4) or
    "none" (every copy kept once: annealing without resampling)."""
    if mode == "nearest":
        u = resample_uniforms(len(E), temp_index, seed, run)
        return copy_counts(E, dbeta, R_target, u, m, S)[0]
    if mode == "multinomial":
        u = multinomial_uniforms(R_target, temp_index, seed, run)
        return multinomial_counts(E, dbeta, u, m)[0]
    if mode == "none":
        return np.ones(len(E), np.int32)
    raise ValueError(mode)


def weight_variance(E: np.ndarray, dbeta: float) -> float:
    E = np.ascontiguousarray(E, np.float64)
    return lib().ora_weight_variance(len(E), _p(E), float(dbeta))


def recentre(x: np.ndarray, mass: np.ndarray) -> np.ndarray:
    """Translate every replica so its centre of mass sits at the origin."""
    com = np.einsum("rac,a->rc", x, mass) / mass.sum()
    return x - com[:, None, :]


def gather(counts: np.ndarray, arrays: Sequence[np.ndarray]) -> List[np.ndarray]:
    """Copies of source j fill consecutive new slots in increasing j."""
    src = np.repeat(np.arange(len(counts)), counts)
    return [a[src] for a in arrays]


def adaptive_dbeta(E: np.ndarray, dbeta_max: float, v_target: float = 0.1, iters: int = 64):
    """Largest dbeta in [0, dbeta_max] with normalised weight variance <= v_target
    (V grows monotonically with dbeta).  Returns dbeta_max itself when V there
    is already within target.  Bisection, lower bracket end returned."""
    if weight_variance(E, dbeta_max) <= v_target:
        return dbeta_max
    lo, hi = 0.0, dbeta_max
    for _ in range(iters):
        mid = 0.5 * (lo + hi)
        if weight_variance(E, mid) <= v_target:
            lo = mid
        else:
            hi = mid
        if hi - lo <= 1e-12 * hi:
            break
    return lo


def observables(E: np.ndarray, K: np.ndarray, ancestor: np.ndarray, n_atoms: int, kB: float, T: float):
    """PAMD step 4: population averages at T."""
    R = len(E)
    Em = E.mean()
    E2 = (E * E).mean()
    Km = K.mean()
    return dict(R=R, E_mean=Em, E2_mean=E2, K_mean=Km,
                T_measured=2.0 * Km / (3.0 * n_atoms * kB),
                Cv=(E2 - Em * Em) / (kB * T * T) / kB if R > 0 else float("nan"),
                families=int(len(np.unique(ancestor))))


# ----------------------------------------------------------------------------
# the annealing driver (PAMD steps 1-5)
# ----------------------------------------------------------------------------

@dataclass
class AnnealResult:
    T: List[float] = field(default_factory=list)
    R: List[int] = field(default_factory=list)
    lnQ: List[float] = field(default_factory=list)
    obs: List[Dict] = field(default_factory=list)
    x: Optional[np.ndarray] = None
    v: Optional[np.ndarray] = None

    @property
    def sum_lnQ(self) -> float:
        return float(np.sum(self.lnQ))


def anneal(sysd, R: int, T0: float, schedule: Optional[Sequence[float]], theta: int, theta_eq: int,
           dt: float, nu: float, seed: int, T_final: Optional[float] = None, v_target: float = 0.1,
           x0: Optional[np.ndarray] = None, v0: Optional[np.ndarray] = None, run: int = 0,
           resampling: str = "nearest", max_temps: int = 10000,
           thermostat: str = "andersen") -> AnnealResult:
    """Plain PAMD run.  schedule: list of temperatures T_0 > T_1 > ... (T_0 = T0),
    or None for the adaptive choice (normalised weight variance = v_target,
    down to T_final).  x0/v0 optionally give the initial population.
    resampling: "nearest", "multinomial" or "none" (resampling_counts); with
    "none" every copy is handed over to itself, so the population is R
    independent annealing runs (the ablation the paper calls "anneal")."""
    osys = OracleSystem(sysd)
    n = osys.n
    kB = osys.kB
    if x0 is None:
        x = np.ascontiguousarray(np.broadcast_to(sysd.x_init, (R, n, 3)).astype(np.float64))
    else:
        x = np.ascontiguousarray(x0, np.float64).copy()
    v = init_velocities(osys, R, T0, seed, run) if v0 is None else np.ascontiguousarray(v0).copy()
    anc = np.arange(R, dtype=np.int64)
    step = 0
    Ep, Ek = md_steps(osys, x, v, theta_eq, T0, dt, nu, seed, step, run, thermostat=thermostat)
    step += theta_eq
    res = AnnealResult()
    res.T.append(T0); res.R.append(R); res.lnQ.append(0.0)
    res.obs.append(observables(Ep, Ek, anc, n, kB, T0))
    T_prev = T0
    i = 0
    while True:
        if schedule is not None:
            if i + 1 >= len(schedule):
                break
            T_next = float(schedule[i + 1])
        else:
            if T_prev <= T_final * (1 + 1e-12) or i >= max_temps:
                break
            dmax = 1.0 / (kB * T_final) - 1.0 / (kB * T_prev)
            db = adaptive_dbeta(Ep, dmax, v_target)
            T_next = T_final if db == dmax else 1.0 / (kB * (db + 1.0 / (kB * T_prev)))
        i += 1
        dbeta = 1.0 / (kB * T_next) - 1.0 / (kB * T_prev)
        m, S, S2, lq = lse(Ep, dbeta)
        c = resampling_counts(resampling, Ep, dbeta, R, i, seed, run, m, S)
        x, v, Ep, anc = gather(c, [x, v, Ep, anc])
        x = np.ascontiguousarray(recentre(x, osys.mass))
        v = np.ascontiguousarray(v * math.sqrt(T_next / T_prev))
        Ep, Ek = md_steps(osys, x, v, theta, T_next, dt, nu, seed, step, run, thermostat=thermostat)
        step += theta
        res.T.append(T_next); res.R.append(len(Ep)); res.lnQ.append(lq)
        res.obs.append(observables(Ep, Ek, anc, n, kB, T_next))
        T_prev = T_next
    res.x, res.v = x, v
    return res
