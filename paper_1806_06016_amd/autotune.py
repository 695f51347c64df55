"""Launch-shape autotuner for the persistent MD kernel.

Times ``pamd_md_steps`` of a probe population on the GPU for each candidate
number of waves per workgroup (which sets replicas per workgroup, LDS per
workgroup and therefore waves per CU) and keeps the fastest.  The probe runs
the kernel of the run's thermostat (the Langevin variant holds more registers).
Results are cached per (system size, dielectric, precision, thermostat, GPU
architecture, library build, probe size) in a JSON file, so a run pays for the
sweep once.
"""
from __future__ import annotations

import hashlib
import json
import os
from typing import Dict, Optional, Sequence

from .pamd import LIB_PATH, Pamd, PAMD_FP32

CANDIDATES = (16, 12, 8, 4)


def _cache_path() -> str:
    base = os.environ.get("XDG_CACHE_HOME", os.path.join(os.path.expanduser("~"), ".cache"))
    return os.path.join(base, "pamd_autotune.json")


def _key(sysd, precision: int, R_probe: int, thermostat: str) -> str:
    import torch
    arch = torch.cuda.get_device_properties(0).gcnArchName
    with open(LIB_PATH, "rb") as f:
        lib = hashlib.sha256(f.read()).hexdigest()[:16]
    return f"N{sysd.n_atoms}-diel{int(sysd.dielectric)}-p{precision}-{thermostat}-{arch}-{lib}-R{R_probe}"


def autotune(sysd, precision: int = PAMD_FP32, R_probe: int = 65536, theta_probe: int = 100,
             candidates: Sequence[int] = CANDIDATES, T0: float = 700.0, dt: float = 0.001,
             use_cache: bool = True, cache_path: Optional[str] = None, thermostat: str = "andersen") -> Dict:
    """Returns {"waves_per_block": w, "timings": {w: replica-steps/s}, "cached": bool}.

    The probe population should be the one the run will use (or large): the
    persistent kernel hands out 4-replica work items to every resident wave,
    and a probe with about one item per wave times the tail, not the rate."""
    import torch
    path = cache_path or _cache_path()
    key = _key(sysd, precision, R_probe, thermostat)
    cache = {}
    if use_cache and os.path.exists(path):
        try:
            cache = json.load(open(path))
        except (OSError, ValueError):
            cache = {}
        if key in cache:
            return dict(cache[key], cached=True)
    timings = {}
    for w in candidates:
        p = Pamd([sysd], R_target=R_probe, T0=T0, dt=dt, nu=1.0, seed=1, precision=precision,
                 waves_per_block=w, thermostat=thermostat)
        p.md_steps(theta_probe)
        torch.cuda.synchronize()
        best = None
        for _ in range(3):
            e0 = torch.cuda.Event(enable_timing=True)
            e1 = torch.cuda.Event(enable_timing=True)
            e0.record(p.stream)
            p.md_steps(theta_probe)
            e1.record(p.stream)
            torch.cuda.synchronize()
            ms = e0.elapsed_time(e1)
            best = ms if best is None else min(best, ms)
        timings[w] = R_probe * theta_probe / (best / 1e3)
        p.close()
    choice = max(timings, key=timings.get)
    entry = {"waves_per_block": int(choice), "timings": {str(k): v for k, v in timings.items()}}
    if use_cache:
        cache[key] = entry
        try:
            os.makedirs(os.path.dirname(path), exist_ok=True)
            with open(path, "w") as f:
                json.dump(cache, f, indent=1)
        except OSError:
            pass
    return dict(entry, cached=False)
