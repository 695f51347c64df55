"""Launch-shape autotuner for the persistent MD kernels.

Times ``pamd_md_steps`` of a probe population on the GPU for each candidate
launch shape and keeps the fastest:

* one molecule (``autotune``): waves per workgroup of the register-tile
  kernel (which sets replicas per workgroup, LDS per workgroup and therefore
  waves per CU); the probe runs the kernel of the run's thermostat (the
  Langevin variant holds more registers);
* several independent runs in one context (``autotune_batched``): the layout
  of every run small enough for the register tile (the batched wide launch,
  one replica per wavefront, or register-tile launches of four replicas per
  wavefront) and the waves per workgroup of the wide launch, timed on the
  whole context at its real population sizes.

Results are cached per (system sizes, dielectric, precision, thermostat, GPU
architecture, library build, probe size) in a JSON file, so a run pays for the
sweep once.
"""
from __future__ import annotations

import hashlib
import json
import os
from typing import Dict, Optional, Sequence

from .pamd import LIB_PATH, Pamd, PAMD_FP32, TILE_ATOMS

CANDIDATES = (16, 12, 8, 4)
WIDE_CANDIDATES = (4, 3, 2, 1)


def _cache_path() -> str:
    base = os.environ.get("XDG_CACHE_HOME", os.path.join(os.path.expanduser("~"), ".cache"))
    return os.path.join(base, "pamd_autotune.json")


def _key(systems, precision: int, R_probe: int, thermostat: str) -> str:
    import torch
    arch = torch.cuda.get_device_properties(0).gcnArchName
    with open(LIB_PATH, "rb") as f:
        lib = hashlib.sha256(f.read()).hexdigest()[:16]
    sizes = "_".join(str(s.n_atoms) for s in systems)
    return f"N{sizes}-diel{int(systems[0].dielectric)}-p{precision}-{thermostat}-{arch}-{lib}-R{R_probe}"


def _load(path: str) -> Dict:
    if os.path.exists(path):
        try:
            return json.load(open(path))
        except (OSError, ValueError):
            pass
    return {}


def _store(path: str, cache: Dict) -> None:
    try:
        os.makedirs(os.path.dirname(path), exist_ok=True)
        with open(path, "w") as f:
            json.dump(cache, f, indent=1)
    except OSError:
        pass


def _time_md(p, theta_probe: int, reps: int = 3) -> float:
    """Best of `reps` timed pamd_md_steps(theta_probe) calls after one untimed one (ms)."""
    import torch
    p.md_steps(theta_probe)
    torch.cuda.synchronize()
    best = None
    for _ in range(reps):
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record(p.stream)
        p.md_steps(theta_probe)
        e1.record(p.stream)
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1)
        best = ms if best is None else min(best, ms)
    return best


def autotune(sysd, precision: int = PAMD_FP32, R_probe: int = 65536, theta_probe: int = 100,
             candidates: Sequence[int] = CANDIDATES, T0: float = 700.0, dt: float = 0.001,
             use_cache: bool = True, cache_path: Optional[str] = None, thermostat: str = "andersen") -> Dict:
    """Returns {"waves_per_block": w, "timings": {w: replica-steps/s}, "cached": bool}.

    The probe population should be the one the run will use (or large): the
    persistent kernel hands out 4-replica work items to every resident wave,
    and a probe with about one item per wave times the tail, not the rate."""
    import torch
    path = cache_path or _cache_path()
    key = _key([sysd], precision, R_probe, thermostat)
    cache = _load(path) if use_cache else {}
    if key in cache:
        return dict(cache[key], cached=True)
    timings = {}
    for w in candidates:
        p = Pamd([sysd], R_target=R_probe, T0=T0, dt=dt, nu=1.0, seed=1, precision=precision,
                 waves_per_block=w, thermostat=thermostat)
        timings[w] = R_probe * theta_probe / (_time_md(p, theta_probe) / 1e3)
        p.close()
    choice = max(timings, key=timings.get)
    entry = {"waves_per_block": int(choice), "timings": {str(k): v for k, v in timings.items()}}
    if use_cache:
        cache[key] = entry
        _store(path, cache)
    return dict(entry, cached=False)


TILE_SMALL_CANDIDATES = (8, 4)   # register-tile waves per workgroup tried for small populations


def autotune_batched(systems: Sequence, R_each: int, precision: int = PAMD_FP32, theta_probe: int = 100,
                     wide_candidates: Sequence[int] = WIDE_CANDIDATES, T0: float = 700.0, dt: float = 0.0005,
                     use_cache: bool = True, cache_path: Optional[str] = None,
                     thermostat: str = "andersen") -> Dict:
    """Launch shape of a context of several runs (R_each replicas each).

    Candidates: every run in the batched wide launch, or the runs that fit
    the register tile (at most 80 atoms) in register-tile launches and the
    rest in the wide launch (all of them in register-tile launches when no
    molecule needs the wide layout); the wide launch, where some run takes
    it, with 4, 3, 2 or 1 waves per workgroup (register-tile launches at 16
    waves per workgroup).
    When the register-tile split wins, its launches are then also timed at
    8 and 4 waves per workgroup: a small population (R_each / 4 work items
    against 16 waves on every CU) otherwise lands on the few CUs whose waves
    claim the items first.  Each candidate times the whole context's MD step
    at the run's population sizes.  Returns {"layout": [per run "wide" /
    "tile"], "wide_waves_per_block": w, "waves_per_block": register-tile
    waves (0: the library's default), "timings": {candidate:
    replica-steps/s}, "cached": bool}."""
    import torch
    systems = list(systems)
    path = cache_path or _cache_path()
    key = "batched-tw-" + _key(systems, precision, R_each, thermostat)
    cache = _load(path) if use_cache else {}
    if key in cache:
        return dict(cache[key], cached=True)
    small = [s.n_atoms <= TILE_ATOMS for s in systems]
    layouts = {"wide": ["wide"] * len(systems)}
    if any(small):
        # every run of at most 80 atoms in register-tile launches (all of them
        # when no molecule needs the wide layout)
        layouts["tile_small"] = ["tile" if sm else "wide" for sm in small]
    timings, shapes = {}, {}

    def probe(cand, lay, w, tw):
        p = Pamd(systems, R_target=R_each, T0=T0, dt=dt, nu=1.0, seed=1, precision=precision,
                 thermostat=thermostat, layout=lay, wide_waves=w, waves_per_block=tw)
        ms = _time_md(p, theta_probe)
        timings[cand] = R_each * len(systems) * theta_probe / (ms / 1e3)
        shapes[cand] = (lay, w, tw)
        p.close()

    for lname, lay in layouts.items():
        # the wide launch's shape only matters when some run takes it
        for w in (wide_candidates if "wide" in lay else (0,)):
            probe(f"{lname}/w{w}", lay, w, 0)
    choice = max(timings, key=timings.get)
    if "tile" in shapes[choice][0]:
        lay, w = shapes[choice][0], shapes[choice][1]
        for tw in TILE_SMALL_CANDIDATES:
            probe(f"tile_small/w{w}/t{tw}", lay, w, tw)
        choice = max(timings, key=timings.get)
    torch.cuda.synchronize()
    entry = {"layout": shapes[choice][0], "wide_waves_per_block": int(shapes[choice][1]),
             "waves_per_block": int(shapes[choice][2]), "choice": choice, "timings": timings}
    if use_cache:
        cache[key] = entry
        _store(path, cache)
    return dict(entry, cached=False)
