"""Population-annealing driver: one PA run (or a batch of runs) from a JSON
configuration, one JSON line per temperature.

PAMD steps in the paper's order: an equilibrated population at T_0 (step 1),
then per temperature the resampling to the next temperature (step 2, with the
normaliser Q recorded), θ MD steps (step 3) and the population observables
(step 4), until the last temperature (step 5).  Every step runs in the
library's kernels; this module only sequences the calls, times them with HIP
events on the context's stream, logs, and checkpoints.

Configuration keys (see ``configs/*.json``):

* ``systems``: list of {"kind": "bead_chain" | "peptide" | "gaussian_chain",
  "n_atoms": N, "seed": s} (several entries: one batched context);
* ``R``, ``T0``, ``theta``, ``theta_eq``, ``dt``, ``nu``, ``seed``;
* ``precision``: "fp32" | "fp64"; ``resampling``: "nearest" | "multinomial" |
  "none"; ``thermostat``: "andersen" | "langevin";
* ``schedule``: {"kind": "geometric", "T_final": T, "steps": n} or
  {"kind": "adaptive", "T_final": T, "V_target": V}.

Logged per temperature and run: temperature index, T, R, ln Q, sum ln Q,
<E_pot>, sigma_E, C_v, measured T, families, normalised weight variance of the
step, MD and resampling milliseconds, wall seconds since the start.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time
from typing import Dict, List, Optional

KINDS = ("bead_chain", "peptide", "gaussian_chain")
REQUIRED = ("systems", "R", "T0", "theta", "theta_eq", "dt", "nu", "seed", "schedule")


def load_config(path_or_dict) -> Dict:
    """Reads and checks a configuration (a path to JSON or a dict)."""
    cfg = dict(path_or_dict) if isinstance(path_or_dict, dict) else json.load(open(path_or_dict))
    missing = [k for k in REQUIRED if k not in cfg]
    if missing:
        raise ValueError(f"configuration lacks {missing}")
    if not cfg["systems"] or any(s.get("kind") not in KINDS for s in cfg["systems"]):
        raise ValueError(f"every system needs a kind in {KINDS}")
    sch = cfg["schedule"]
    if sch.get("kind") == "geometric":
        if not (0 < sch["T_final"] < cfg["T0"]) or int(sch["steps"]) < 1:
            raise ValueError("geometric schedule needs 0 < T_final < T0 and steps >= 1")
    elif sch.get("kind") == "adaptive":
        if not (0 < sch["T_final"] < cfg["T0"]) or not sch.get("V_target", 0.1) > 0:
            raise ValueError("adaptive schedule needs 0 < T_final < T0 and V_target > 0")
    else:
        raise ValueError("schedule kind must be geometric or adaptive")
    cfg.setdefault("precision", "fp32")
    cfg.setdefault("resampling", "nearest")
    cfg.setdefault("thermostat", "andersen")
    if cfg["precision"] not in ("fp32", "fp64"):
        raise ValueError("precision must be fp32 or fp64")
    for k in ("R", "theta", "theta_eq"):
        if int(cfg[k]) < (1 if k != "theta_eq" else 0):
            raise ValueError(f"{k} out of range")
    return cfg


def temperatures(cfg) -> Optional[List[float]]:
    """The geometric schedule T_0 .. T_n (None for the adaptive one)."""
    sch = cfg["schedule"]
    if sch["kind"] != "geometric":
        return None
    n = int(sch["steps"])
    return [cfg["T0"] * (sch["T_final"] / cfg["T0"]) ** (i / n) for i in range(n + 1)]


def build_systems(cfg):
    from pamd_inputs import systems as S
    out = []
    for s in cfg["systems"]:
        if s["kind"] == "bead_chain":
            out.append(S.bead_chain(int(s["n_atoms"]), seed=int(s.get("seed", 1))))
        elif s["kind"] == "peptide":
            out.append(S.make_peptide(seed=int(s.get("seed", 1806)), n_atoms=int(s["n_atoms"])))
        else:
            out.append(S.gaussian_chain(int(s["n_atoms"]), float(s.get("k", 100.0)), float(s.get("r0", 0.0))))
    return out


def _record(o: Dict, md_ms: float, rs_ms: float, t0: float, run: int) -> Dict:
    var = max(o["E2_mean"] - o["E_mean"] ** 2, 0.0)
    return {"run": run, "temp_index": int(o["temp_index"]), "T": o["T"], "R": int(o["R"]), "lnQ": o["lnQ_last"],
            "sum_lnQ": o["sum_lnQ"], "E_mean": o["E_mean"], "E_sd": math.sqrt(var), "Cv": o["Cv"],
            "T_measured": o["T_measured"], "families": int(o["families"]), "V": o["V_last"], "md_ms": md_ms,
            "resample_ms": rs_ms, "wall_s": time.perf_counter() - t0}


def run_pamd(cfg, log=None, checkpoint: Optional[str] = None, checkpoint_every: int = 0, resume: bool = False,
             max_temps: Optional[int] = None) -> List[Dict]:
    """Runs the configuration; returns the per-temperature records (also
    written to `log`, a path or a text stream, one JSON object per line).
    With `checkpoint`, the state is saved every `checkpoint_every`
    temperatures; `resume` restarts from that file instead of equilibrating."""
    import torch
    from . import checkpoint as CK
    from .pamd import Pamd, PAMD_FP32, PAMD_FP64, load_library

    cfg = load_config(cfg)
    load_library()
    systems = build_systems(cfg)
    sch = cfg["schedule"]
    temps = temperatures(cfg)
    adaptive = temps is None
    p = Pamd(systems, R_target=int(cfg["R"]), T0=float(cfg["T0"]), dt=float(cfg["dt"]), nu=float(cfg["nu"]),
             seed=int(cfg["seed"]), precision=PAMD_FP32 if cfg["precision"] == "fp32" else PAMD_FP64,
             T_final=float(sch["T_final"]) if adaptive else None, V_target=float(sch.get("V_target", 0.1)),
             resampling=cfg["resampling"], thermostat=cfg["thermostat"])
    own = None
    if isinstance(log, str):
        own = log = open(log, "a" if resume else "w")
    t0 = time.perf_counter()
    records: List[Dict] = []

    def timed(fn):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(p.stream)
        fn()
        e1.record(p.stream)
        e1.synchronize()
        return e0.elapsed_time(e1)

    def emit(md_ms, rs_ms):
        for r, o in enumerate(p.observables()):
            rec = _record(o, md_ms, rs_ms, t0, r)
            records.append(rec)
            if log is not None:
                log.write(json.dumps(rec) + "\n")
                log.flush()

    try:
        if resume:
            if not checkpoint or not os.path.exists(checkpoint):
                raise FileNotFoundError(f"no checkpoint to resume from: {checkpoint}")
            CK.restore(p, checkpoint)
        else:
            emit(timed(lambda: p.md_steps(int(cfg["theta_eq"]))), 0.0)
        done = 0
        while max_temps is None or done < max_temps:
            i = int(p.observables()[0]["temp_index"])
            if adaptive:
                if all(o["T"] <= float(sch["T_final"]) for o in p.observables()):
                    break
                rs = timed(lambda: p.resample(None))
            else:
                if i + 1 >= len(temps):
                    break
                rs = timed(lambda: p.resample([temps[i + 1]] * len(systems)))
            md = timed(lambda: p.md_steps(int(cfg["theta"])))
            emit(md, rs)
            done += 1
            if checkpoint and checkpoint_every > 0 and (i + 1) % checkpoint_every == 0:
                CK.save(p, checkpoint)
    finally:
        p.close()
        if own is not None:
            own.close()
    return records


def main(argv=None):
    ap = argparse.ArgumentParser(description="Population-annealing MD run from a JSON configuration")
    ap.add_argument("config", help="JSON configuration (paper_1806_06016_amd/configs/*.json)")
    ap.add_argument("--log", default="-", help="JSON lines output (default: stdout)")
    ap.add_argument("--checkpoint", default="", help="checkpoint file (.npz)")
    ap.add_argument("--checkpoint-every", type=int, default=0, help="save every this many temperatures")
    ap.add_argument("--resume", action="store_true", help="continue from --checkpoint")
    ap.add_argument("--max-temps", type=int, default=None, help="stop after this many temperature steps")
    a = ap.parse_args(argv)
    log = sys.stdout if a.log == "-" else a.log
    run_pamd(a.config, log=log, checkpoint=a.checkpoint or None, checkpoint_every=a.checkpoint_every,
             resume=a.resume, max_temps=a.max_temps)


if __name__ == "__main__":
    main()
