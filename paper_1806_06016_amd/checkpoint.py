"""Checkpoint and resume of a population-annealing run.

A checkpoint holds, for every run of a context, the population (positions,
velocities, potential energies, family ancestors) and the run's scalars
(temperature, previous temperature, running sum of ln Q, last ln Q, population
size, MD step counter, temperature index).  Every random stream of the library
is a counter-based function of (seed, run, replica slot, MD step or
temperature index), so a context created with the same parameters and given
this state continues exactly as the uninterrupted run would: the same
collisions, the same resampling draws, the same temperatures.

The file is a NumPy ``.npz`` archive of plain arrays (read back with
``allow_pickle=False``).  Device-side extras that are not part of a run's
state — a temperature schedule set with ``set_schedule``, captured graphs, an
attached surrogate — are set again by the caller after ``restore``.
"""
from __future__ import annotations

from typing import Dict, List, Sequence

import numpy as np

from .pamd import PAMD_FP32, PAMD_FP64

FORMAT = 1
_F64 = ("T", "T_prev", "sum_lnQ", "lnQ_last")
_I64 = ("R", "step", "temp_index")


def write(path: str, states: Sequence[Dict], precision: int) -> None:
    """Writes the states (dicts as returned by ``Pamd.get_state`` with
    positions and velocities) of every run."""
    arrays = {"format": np.array([FORMAT], np.int64), "precision": np.array([precision], np.int64),
              "n_runs": np.array([len(states)], np.int64)}
    for r, st in enumerate(states):
        R = int(st["R"])
        x = np.asarray(st["x"], np.float64)
        if x.ndim != 3 or x.shape[0] != R or x.shape[2] != 3:
            raise ValueError(f"run {r}: positions must be [R][n_atoms][3] with R = {R}")
        arrays[f"x{r}"] = x
        arrays[f"v{r}"] = np.asarray(st["v"], np.float64)
        arrays[f"E_pot{r}"] = np.asarray(st["E_pot"], np.float64)
        arrays[f"ancestor{r}"] = np.asarray(st["ancestor"], np.int32)
        arrays[f"f64_{r}"] = np.array([st[k] for k in _F64], np.float64)
        arrays[f"i64_{r}"] = np.array([st[k] for k in _I64], np.int64)
        if arrays[f"v{r}"].shape != x.shape or arrays[f"E_pot{r}"].shape != (R,) or \
                arrays[f"ancestor{r}"].shape != (R,):
            raise ValueError(f"run {r}: inconsistent array shapes")
    with open(path, "wb") as f:
        np.savez(f, **arrays)


def read(path: str) -> Dict:
    """Returns {"precision": p, "runs": [state dict per run]}."""
    with np.load(path, allow_pickle=False) as z:
        if int(z["format"][0]) != FORMAT:
            raise ValueError(f"unknown checkpoint format {int(z['format'][0])}")
        runs: List[Dict] = []
        for r in range(int(z["n_runs"][0])):
            st = {k: float(v) for k, v in zip(_F64, z[f"f64_{r}"])}
            st.update({k: int(v) for k, v in zip(_I64, z[f"i64_{r}"])})
            st.update(x=z[f"x{r}"], v=z[f"v{r}"], E_pot=z[f"E_pot{r}"], ancestor=z[f"ancestor{r}"])
            runs.append(st)
        return {"precision": int(z["precision"][0]), "runs": runs}


def save(p, path: str) -> None:
    """Checkpoint every run of context ``p`` (a ``Pamd``)."""
    write(path, [p.get_state(r) for r in range(len(p.n_atoms))], PAMD_FP32 if p.fp32 else PAMD_FP64)


def restore(p, path: str) -> None:
    """Load a checkpoint into context ``p``, created with the parameters of
    the checkpointed one (same molecules, precision, seed, R_target, dt, bath,
    resampling mode, T_final / V_target)."""
    ck = read(path)
    if ck["precision"] != (PAMD_FP32 if p.fp32 else PAMD_FP64):
        raise ValueError("checkpoint precision differs from the context's")
    if len(ck["runs"]) != len(p.n_atoms):
        raise ValueError(f"checkpoint holds {len(ck['runs'])} runs, the context {len(p.n_atoms)}")
    for r, st in enumerate(ck["runs"]):
        if st["x"].shape[1] != p.n_atoms[r]:
            raise ValueError(f"run {r}: {st['x'].shape[1]} atoms in the checkpoint, {p.n_atoms[r]} in the context")
        if st["R"] > p.R_cap:
            raise ValueError(f"run {r}: population {st['R']} exceeds the context's R_cap {p.R_cap}")
    for r, st in enumerate(ck["runs"]):
        p.set_state(r, st["x"], st["v"], T=st["T"], step=st["step"], temp_index=st["temp_index"],
                    E_pot=st["E_pot"], ancestor=st["ancestor"], T_prev=st["T_prev"], sum_lnQ=st["sum_lnQ"],
                    lnQ_last=st["lnQ_last"])
