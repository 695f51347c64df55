"""FP64 oracle of the learned multiple-time-step (MTS) surrogate -- TEST
INFRASTRUCTURE ONLY (tests/, smoke and the benchmark's CPU leg).

Not part of the paper: a per-atom MLP surrogate of the nonbonded force, used
as the inner force of an r-RESPA splitting whose outer impulse applies the
exact-minus-surrogate nonbonded force, so the dynamics still follows the exact
Hamiltonian (the paper's MD update of PAMD step 3 is what it accelerates).

Definitions (all FP64):
  features  G[i, t, k] = sum_{j in P(i), type(j) = t} phi_k(r_ij),
            phi_k(r) = exp(-(r - mu_k)^2 / (2 s^2)), mu_k = 0.1 + 1.1 k / 31,
            s = 1.1 / 31 (nm), t = 0..7, k = 0..31 (256 features per atom);
            P(i): partners of i in the nonbonded pair set (1-2 and 1-3 pairs
            excluded, 1-4 pairs included unscaled)
  MLP       E_i = w3 . silu(W2^T silu(W1^T G_i + b1) + b2) + b3,
            silu(x) = x / (1 + e^-x); E_NN = sum_i E_i (one MLP shared by all atoms)
  forces    F = -grad_x E_NN
  loss      L = mean over configurations, atoms, components of (F_NN - F_target)^2
  RESPA     outer step Dt = M dt: v += Dt/2 (F_nb - F_NN)/m; M velocity-Verlet
            steps of dt with F_bonded + F_NN; v += Dt/2 (F_nb - F_NN)/m; then
            Andersen collisions with p = 1 - exp(-nu Dt), drawn with the MD step
            counter at the start of the outer step (step0 + o M) as the Philox
            step word.
"""
from __future__ import annotations

import math
from typing import Callable, Dict, Optional

import numpy as np

from pamd_inputs.weights import surrogate_weights

from . import oracle as O

N_TYPES = 8
N_RBF = 32
N_FEAT = N_TYPES * N_RBF
H1 = 128
H2 = 128
MU = 0.1 + 1.1 * np.arange(N_RBF) / 31.0
SIG = 1.1 / 31.0


def nn_pairs(sysd):
    """Unordered pairs of the nonbonded set (1-4 included, unscaled)."""
    pidx, _, _ = O.pair_list(sysd.n_atoms, sysd.bonds, 1.0, 1.0)
    return pidx


def init_weights(seed: int = 0, scale: float = 1.0) -> Dict[str, np.ndarray]:
    """Seeded Glorot-style initial weights (the shared input generator)."""
    return surrogate_weights(seed, scale)


def _silu(x):
    return x / (1.0 + np.exp(-x))


def _dsilu(x):
    s = 1.0 / (1.0 + np.exp(-x))
    return s * (1.0 + x * (1.0 - s))


def features(x: np.ndarray, atype: np.ndarray, pairs: np.ndarray):
    """x [B, N, 3] -> G [B, N, 8, 32], plus per-pair r, unit vectors and phi."""
    i, j = pairs[:, 0], pairs[:, 1]
    d = x[:, i] - x[:, j]                      # [B, P, 3]
    r = np.sqrt((d * d).sum(-1))               # [B, P]
    phi = np.exp(-((r[..., None] - MU) ** 2) / (2 * SIG * SIG))   # [B, P, 32]
    B, N = x.shape[0], x.shape[1]
    G = np.zeros((B, N, N_TYPES, N_RBF))
    for p in range(len(pairs)):
        G[:, i[p], atype[j[p]]] += phi[:, p]
        G[:, j[p], atype[i[p]]] += phi[:, p]
    return G, r, d, phi


def mlp(Gf: np.ndarray, w: Dict[str, np.ndarray]):
    """Gf [rows, 256] -> per-row energies and dE/dG [rows, 256]."""
    h1 = Gf @ w["W1"] + w["b1"]
    a1 = _silu(h1)
    h2 = a1 @ w["W2"] + w["b2"]
    a2 = _silu(h2)
    e = a2 @ w["w3"] + w["b3"][0]
    g2 = w["w3"][None, :] * _dsilu(h2)
    g1 = (g2 @ w["W2"].T) * _dsilu(h1)
    gG = g1 @ w["W1"].T
    return e, gG


def energy_forces(x: np.ndarray, atype: np.ndarray, pairs: np.ndarray, w: Dict[str, np.ndarray]):
    """x [B, N, 3] -> (E_NN [B], F_NN [B, N, 3])."""
    B, N = x.shape[0], x.shape[1]
    G, r, d, phi = features(x, atype, pairs)
    e, gG = mlp(G.reshape(B * N, N_FEAT), w)
    E = e.reshape(B, N).sum(1)
    gG = gG.reshape(B, N, N_TYPES, N_RBF)
    i, j = pairs[:, 0], pairs[:, 1]
    dphi = -(r[..., None] - MU) / (SIG * SIG) * phi                  # d phi / d r
    s = (gG[:, i, atype[j]] * dphi).sum(-1) + (gG[:, j, atype[i]] * dphi).sum(-1)   # dE/dr [B, P]
    fpair = -(s / r)[..., None] * d                                   # force on i
    F = np.zeros_like(x)
    for p in range(len(pairs)):
        F[:, i[p]] += fpair[:, p]
        F[:, j[p]] -= fpair[:, p]
    return E, F


def force_loss(x, F_target, atype, pairs, w):
    E, F = energy_forces(x, atype, pairs, w)
    return float(np.mean((F - F_target) ** 2))


def loss_grad_torch(x, F_target, atype, pairs, w):
    """dL/dW of the force-matching loss by plain PyTorch CPU autograd in float64
    (the forces themselves are a gradient, so this is a second derivative)."""
    import torch
    t = {k: torch.tensor(v, dtype=torch.float64, requires_grad=True) for k, v in w.items()}
    X = torch.tensor(x, dtype=torch.float64, requires_grad=True)
    i = torch.tensor(pairs[:, 0])
    j = torch.tensor(pairs[:, 1])
    ty = torch.tensor(atype, dtype=torch.long)
    mu = torch.tensor(MU)
    d = X[:, i] - X[:, j]
    r = torch.sqrt((d * d).sum(-1))
    phi = torch.exp(-((r[..., None] - mu) ** 2) / (2 * SIG * SIG))
    B, N = x.shape[0], x.shape[1]
    G = torch.zeros(B, N, N_TYPES, N_RBF, dtype=torch.float64)
    G = G.index_put((torch.arange(B)[:, None].expand(B, len(pairs)), i[None].expand(B, -1),
                     ty[j][None].expand(B, -1)), phi, accumulate=True)
    G = G.index_put((torch.arange(B)[:, None].expand(B, len(pairs)), j[None].expand(B, -1),
                     ty[i][None].expand(B, -1)), phi, accumulate=True)
    Gf = G.reshape(B * N, N_FEAT)
    a1 = torch.nn.functional.silu(Gf @ t["W1"] + t["b1"])
    a2 = torch.nn.functional.silu(a1 @ t["W2"] + t["b2"])
    E = (a2 @ t["w3"] + t["b3"][0]).sum()
    (gx,) = torch.autograd.grad(E, X, create_graph=True)
    F = -gx
    L = ((F - torch.tensor(F_target)) ** 2).mean()
    L.backward()
    # b3 shifts every energy by a constant: no force depends on it (grad None)
    return float(L.detach()), {k: (v.grad.numpy().copy() if v.grad is not None else np.zeros(v.shape))
                      for k, v in t.items()}


def respa_steps(osys, sysd, x, v, n_outer: int, outer_ratio: int, dt_inner: float, T: float, nu: float,
                seed: int, step0: int, nn_force: Callable[[np.ndarray], np.ndarray], run: int = 0):
    """r-RESPA with Andersen collisions after each outer step (in place on x, v).
    nn_force(x [R, N, 3]) -> F_NN [R, N, 3].  Returns (E_pot [R], E_kin [R])."""
    R, N = x.shape[0], x.shape[1]
    m = osys.mass[None, :, None]
    Dt = outer_ratio * dt_inner
    bonded = O.T_BOND | O.T_ANGLE | O.T_DIHEDRAL
    nonb = O.T_LJ | O.T_COUL
    p24 = O.collision_p24(nu, Dt)
    for o in range(n_outer):
        Fnb = O.energy_forces(osys, x, nonb)[1]
        Fnn = nn_force(x)
        v += 0.5 * Dt * (Fnb - Fnn) / m
        Fin = O.energy_forces(osys, x, bonded)[1] + Fnn
        for q in range(outer_ratio):
            v += 0.5 * dt_inner * Fin / m
            x += dt_inner * v
            Fnn = nn_force(x)
            Fin = O.energy_forces(osys, x, bonded)[1] + Fnn
            v += 0.5 * dt_inner * Fin / m
        Fnb = O.energy_forces(osys, x, nonb)[1]
        v += 0.5 * Dt * (Fnb - Fnn) / m
        # Andersen collisions, one draw per atom per outer step
        _andersen(osys, x, v, T, p24, seed, step0 + o * outer_ratio, run)
    Ep = O.energy_forces(osys, x)[0]
    Ek = 0.5 * (m * v * v).sum((1, 2))
    return Ep, Ek


def _andersen(osys, x, v, T, p24, seed, step, run):
    """One round of Andersen collisions with the collision words of `step`
    (same draw layout as the MD step)."""
    if p24 == 0:
        return
    R, N = x.shape[0], x.shape[1]
    key = [seed & 0xFFFFFFFF, ((seed >> 32) + run) & 0xFFFFFFFF]
    for r in range(R):
        for a in range(N):
            w = O.philox([r, step, (a & 15) + 16 * (a >> 6), 0], key)
            if (int(w[(a >> 4) & 3]) >> 8) < p24:
                wv = O.philox([r, step, a, 1], key)
                u = [((int(q) >> 8) + 0.5) / 16777216.0 for q in wv]
                r0 = math.sqrt(-2 * math.log(u[0]))
                r1 = math.sqrt(-2 * math.log(u[2]))
                z = (r0 * math.cos(2 * math.pi * u[1]), r0 * math.sin(2 * math.pi * u[1]),
                     r1 * math.cos(2 * math.pi * u[3]))
                sd = math.sqrt(osys.kB * T / osys.mass[a])
                v[r, a] = [sd * z[0], sd * z[1], sd * z[2]]
