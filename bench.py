"""Benchmark of the PAMD hot path on one MI355X.

Workload: the 75-atom synthetic peptide (74 bonds, 132 angles, 178 dihedrals,
2569 nonbonded pairs), R = 1e5 replicas, theta = 1000 velocity-Verlet steps
(dt = 1 fs, Andersen nu = 1/ps) per temperature, adaptive temperature steps
(normalised weight variance 0.1) from 700 K towards 250 K.  One benchmark
"step" is one PAMD temperature step: resample (adaptive T, weights, copy
numbers, prefix sum, gather) + theta MD steps of every replica + population
observables.  Inputs are synthetic and resident in HBM before timing.

Prints one JSON line (metric replica-MD steps/s, whole job).
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

# MI355X published peaks
PEAK_FP32_VALU_TFLOPS = 157.3
PEAK_HBM_GBS = 8000.0


def algorithmic_flops_per_replica_step(sysd) -> float:
    """Algorithmic work of one MD step of one replica (FMA = 2 flops,
    transcendentals not counted): ~25 flops per nonbonded pair, 21 per bond,
    70 per angle, 110 per dihedral, 18 per atom for the integrator."""
    n = sysd.n_atoms
    pairs = n * (n - 1) // 2 - len(sysd.bonds) - len(sysd.angles)
    return 25.0 * pairs + 21.0 * len(sysd.bonds) + 70.0 * len(sysd.angles) + 110.0 * len(sysd.dihedrals) \
        + 18.0 * n, pairs


def measured_traffic(name: str = "k_md_traffic.txt"):
    """HBM bytes per MD-kernel launch from the committed rocprofv3 counter
    summary, or None when the kernel source changed since it was taken."""
    import hashlib
    path = os.path.join(ROOT, "profiles", name)
    src = os.path.join(ROOT, "paper_1806_06016_amd", "csrc", "md_kernel.hip")
    try:
        kv = {}
        for line in open(path):
            if "=" in line and not line.lstrip().startswith("#"):
                k, v = line.split("=", 1)
                kv[k.strip()] = v.strip()
        sha = hashlib.sha256(open(src, "rb").read()).hexdigest()[:16]
        if kv.get("kernel_source_sha256_prefix") != sha:
            return None
        return int(kv["fetch_bytes_per_launch"]) + int(kv["write_bytes_per_launch"])
    except (OSError, KeyError, ValueError):
        return None


def _oracle_sample(R: int, seconds_target: float):
    """R replicas of the 75-atom peptide at 700 K through the FP64 oracle for
    about seconds_target: (replica-steps/s, steps, seconds)."""
    import numpy as np
    from oracle import oracle as O
    from pamd_inputs import systems as S
    sysd = S.c2_system()
    osys = O.OracleSystem(sysd)
    x = np.ascontiguousarray(np.broadcast_to(sysd.x_init, (R, sysd.n_atoms, 3)).astype(np.float64))
    v = O.init_velocities(osys, R, 700.0, seed=1806)
    t0 = time.perf_counter()
    O.md_steps(osys, x, v, 20, 700.0, 0.001, 1.0, 1806, 0)
    dt1 = time.perf_counter() - t0
    steps = max(20, int(seconds_target / max(dt1, 1e-6) * 20))
    t0 = time.perf_counter()
    O.md_steps(osys, x, v, steps, 700.0, 0.001, 1.0, 1806, 20)
    el = time.perf_counter() - t0
    return R * steps / el, steps, el


def cpu_baseline_one_core(seconds_target: float = 8.0):
    """The same oracle sample on one core: a child process with OpenMP held
    to one thread."""
    import subprocess
    code = ("import json, sys; sys.path.insert(0, %r); import bench; "
            "r, n, el = bench._oracle_sample(16, %r); print(json.dumps([r, n, el]))") % (ROOT, seconds_target)
    env = dict(os.environ, OMP_NUM_THREADS="1")
    out = subprocess.run([sys.executable, "-c", code], env=env, capture_output=True, text=True, timeout=300)
    r, n, el = json.loads(out.stdout.strip().splitlines()[-1])
    return dict(value=r, cores=1, sample=f"16 replicas x {n} steps of the 75-atom peptide at 700 K (FP64 oracle, "
                                         f"one thread, {el:.1f} s)")


def cpu_baseline(seconds_target: float = 15.0):
    """The FP64 oracle (plain C, OpenMP over replicas) on the host cores, on a
    bounded sample of the same workload: R_s replicas x theta_s steps of the
    75-atom peptide at 700 K, and the same on one core.  Returns replica-steps/s."""
    threads = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
    R = max(64, 8 * threads)
    r, steps, el = _oracle_sample(R, seconds_target)
    return dict(value=r, unit="replica-MD steps/s", cores=threads, kind="oracle",
                sample=f"{R} replicas x {steps} steps of the 75-atom peptide at 700 K (FP64 oracle, "
                       f"{el:.1f} s)", one_core=cpu_baseline_one_core())


def cpu_baseline_batched(systems, R_each: int, seconds_target: float = 15.0):
    """The FP64 oracle on a bounded sample of the batched workload: for each
    molecule, R_s replicas x a few steps at 700 K; the mixed rate weights each
    molecule by its population (R_each replicas of every molecule)."""
    import numpy as np
    from oracle import oracle as O
    threads = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
    Rs = max(16, 2 * threads)
    per = seconds_target / len(systems)
    t_total = 0.0
    rates = {}
    for sysd in systems:
        osys = O.OracleSystem(sysd)
        x = np.ascontiguousarray(np.broadcast_to(sysd.x_init, (Rs, sysd.n_atoms, 3)).astype(np.float64))
        v = O.init_velocities(osys, Rs, 700.0, seed=1806)
        t0 = time.perf_counter()
        O.md_steps(osys, x, v, 5, 700.0, 0.001, 1.0, 1806, 0)
        d5 = time.perf_counter() - t0
        steps = max(5, int(per / max(d5, 1e-6) * 5))
        t0 = time.perf_counter()
        O.md_steps(osys, x, v, steps, 700.0, 0.001, 1.0, 1806, 5)
        el = time.perf_counter() - t0
        rates[sysd.n_atoms] = Rs * steps / el
        t_total += R_each / rates[sysd.n_atoms]
    value = R_each * len(systems) / t_total
    return dict(value=value, unit="replica-MD steps/s", cores=threads, kind="oracle",
                sample=f"{Rs} replicas of each molecule at 700 K for ~{per:.1f} s each; per-molecule rates "
                       f"{ {k: round(r) for k, r in rates.items()} } combined at equal populations")


def _attainable(result):
    """Adds the measured ceiling of FP32 VALU work without packed FP32 (every
    kernel here is built that way): a kernel of independent all-VGPR FMAs,
    timed live (close to the published FP32 vector peak on gfx950)."""
    from paper_1806_06016_amd import pamd
    rate = pamd.fp32_fma_rate()
    rf = result["roofline"]
    rf["attainable_fp32_fma"] = rate
    rf["frac_of_attainable"] = rf["achieved"] / rate


def batched(args):
    """Eight independent runs of seeded peptides with 40, 75, 75, 120, 150,
    200, 250 and 300 atoms, R = 4096 each, in one context: the runs above 80
    atoms share one persistent wide launch per MD phase, and the autotuner
    chooses for the runs of at most 80 atoms between that launch and
    register-tile launches of their own, and the wide launch's waves per
    workgroup; geometric schedule 700 K -> 250 K over 40 steps (the device
    schedule, replayed from HIP graphs); theta = 1000 steps of 0.5 fs."""
    import numpy as np
    import torch
    from pamd_inputs import systems as S
    from paper_1806_06016_amd import Pamd, PAMD_FP32
    systems = S.c4_systems()
    R = 4096 if args.replicas == 100000 else args.replicas
    sched = S.geometric_schedule(700.0, 250.0, 40)
    # dt = 0.5 fs: at 1 fs the FP64 oracle itself blows up within 200 steps at
    # 700 K for the 120-250-atom molecules (oppositely charged hydrogens fall
    # into the steep Lennard-Jones wall); at 0.5 fs 2048-replica oracle runs stay finite
    tuned = None
    layout, wide_waves, tile_waves = "auto", args.waves, 0
    if args.waves == 0 and not args.no_autotune:
        from paper_1806_06016_amd.autotune import autotune_batched
        tuned = autotune_batched(systems, R)
        layout, wide_waves = tuned["layout"], tuned["wide_waves_per_block"]
        tile_waves = tuned.get("waves_per_block", 0)
    p = Pamd(systems, R_target=R, T0=700.0, dt=0.0005, nu=1.0, seed=1806, precision=PAMD_FP32,
             layout=layout, wide_waves=wide_waves, waves_per_block=tile_waves)
    for r in range(len(systems)):
        p.set_schedule(r, sched)
    info = dict(p.launch_info(), runs=[dict(atoms=s.n_atoms, **p.run_launch(r)) for r, s in enumerate(systems)],
                autotune=tuned)
    stream = torch.cuda.current_stream()
    calibration_copy(args.copy_mb)
    p.md_steps(args.theta_eq)
    p.observables()
    p.graph_capture(0, "schedule", slot=0, parts="resample")
    p.graph_capture(args.theta, "schedule", slot=1, parts="md")
    fl = [algorithmic_flops_per_replica_step(s) for s in systems]
    ev = []
    for _ in range(args.warmup):
        p.graph_launch(0)
        p.graph_launch(1)
        p.observables()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    steps_total = flops_total = pairs_total = 0.0
    for _ in range(args.steps):
        p.graph_launch(0)
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        p.graph_launch(1)
        e1.record(stream)
        ev.append((e0, e1))
        obs = p.observables()
        for k, o in enumerate(obs):
            steps_total += o["R"] * args.theta
            flops_total += o["R"] * args.theta * fl[k][0]
            pairs_total += o["R"] * args.theta * fl[k][1]
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    md_s = sum(a.elapsed_time(b) for a, b in ev) / 1e3
    achieved = flops_total / md_s / 1e12
    result = {
        "metric": "replica-MD steps/s", "value": steps_total / el, "unit": "replica-MD steps/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": el / args.steps * 1e3,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f32 (FP64 energy sums, weights, Q)", "data": "synthetic",
        "config": {"workload": "batched PAMD: 8 synthetic peptides (40, 75, 75, 120, 150, 200, 250, 300 atoms), "
                               "R=4096 each, one persistent launch, geometric 700->250 K in 40 steps, theta=1000, "
                               "dt=0.5 fs",
                   "replicas_per_run": R, "theta": args.theta, "T": obs[0]["T"]},
        "pair_interactions_per_s": pairs_total / el,
        "md_kernel_ms_avg": md_s / args.steps * 1e3,
        "md_kernel_ms_median": float(np.median([a.elapsed_time(b) for a, b in ev])),
        "launch": info,
        "roofline": {"bound": "alu", "achieved": achieved, "peak": PEAK_FP32_VALU_TFLOPS, "unit": "TFLOP/s",
                     "frac": achieved / PEAK_FP32_VALU_TFLOPS,
                     "traffic": measured_traffic("k_md_wide_traffic.txt") if R == 4096 and args.theta == 1000
                     else None},
    }
    p.close()
    _attainable(result)
    if not args.no_cpu_baseline:
        result["cpu_baseline"] = cpu_baseline_batched(systems, R, args.cpu_seconds)
    return result


def calibration_copy(mb):
    """One device-to-device copy of `mb` MiB: the reference kernel whose HBM
    counters scale FETCH_SIZE / WRITE_SIZE to bytes (known size)."""
    if mb <= 0:
        return
    import torch
    src = torch.ones(mb << 20, dtype=torch.uint8, device="cuda")
    dst = torch.empty_like(src)
    dst.copy_(src)
    torch.cuda.synchronize()
    del src, dst


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=4, help="timed PAMD temperature steps")
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--replicas", type=int, default=100000)
    ap.add_argument("--theta", type=int, default=1000)
    ap.add_argument("--theta-eq", type=int, default=1000)
    ap.add_argument("--waves", type=int, default=0, help="waves per workgroup (0: automatic)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
    ap.add_argument("--no-graph", action="store_true", help="eager launches instead of HIP graphs")
    ap.add_argument("--no-autotune", action="store_true")
    ap.add_argument("--valu-forms", action="store_true",
                    help="only measure the issue cost of single VALU instruction forms (1, 2, 4, 8 waves per SIMD)")
    ap.add_argument("--copy-mb", type=int, default=0,
                    help="also run one device-to-device copy of this many MiB (calibrates HBM byte counters)")
    ap.add_argument("--resampling", choices=("nearest", "multinomial", "none"), default="nearest",
                    help="copy-number rule of the resampling step (none: annealing without resampling)")
    ap.add_argument("--thermostat", choices=("andersen", "langevin"), default="andersen",
                    help="heat bath of the MD steps (langevin: friction 1/ps, B-A-O-A-B)")
    ap.add_argument("--workload", choices=("peptide", "batched"), default="peptide",
                    help="peptide: one 75-atom run at R=1e5 (the headline); batched: 8 uneven peptides "
                         "(40..300 atoms, R=4096 each) in one persistent launch")
    args = ap.parse_args()
    if args.gpus != 1:
        print(json.dumps({"error": "this build runs on one GPU only; --gpus must be 1"}))
        sys.exit(2)
    if args.valu_forms:
        from paper_1806_06016_amd import pamd
        pamd.load_library()
        print(json.dumps({"valu_issue_cycles": [pamd.valu_issue_rates(w) for w in (1, 2, 4, 8)],
                          "fp32_fma_tflops": pamd.fp32_fma_rate()}))
        return
    if args.workload == "batched":
        print(json.dumps(batched(args)))
        return

    import numpy as np
    import torch
    from pamd_inputs import systems as S
    from paper_1806_06016_amd import Pamd, PAMD_FP32

    sysd = S.c2_system()
    flops_rs, pairs = algorithmic_flops_per_replica_step(sysd)
    R = args.replicas
    T0, T_final, dt, nu, seed = 700.0, 250.0, 0.001, 1.0, 1806
    tuned = None
    waves = args.waves
    if waves == 0 and not args.no_autotune:
        from paper_1806_06016_amd.autotune import autotune
        tuned = autotune(sysd, PAMD_FP32, R_probe=min(R, 131072), thermostat=args.thermostat)
        waves = tuned["waves_per_block"]
    p = Pamd([sysd], R_target=R, T0=T0, dt=dt, nu=nu, seed=seed, precision=PAMD_FP32,
             V_target=0.1, T_final=T_final, waves_per_block=waves, resampling=args.resampling,
             thermostat=args.thermostat)
    info = p.launch_info()
    stream = torch.cuda.current_stream()
    calibration_copy(args.copy_mb)
    # setup (untimed): equilibration at T0; one-time graph captures (slot 0:
    # adaptive resampling, slot 1: theta MD steps), replayed every temperature
    p.md_steps(args.theta_eq)
    p.observables()
    use_graph = not args.no_graph
    if use_graph:
        p.graph_capture(0, "adaptive", slot=0, parts="resample")
        p.graph_capture(args.theta, "adaptive", slot=1, parts="md")

    ev_md = []
    ev_rs = []
    R_steps = 0

    def temperature_step(record: bool):
        nonlocal R_steps
        if record:
            r0 = torch.cuda.Event(enable_timing=True)
            r1 = torch.cuda.Event(enable_timing=True)
            r0.record(stream)
        if use_graph:
            p.graph_launch(0)
        else:
            p.resample(None)
        if record:
            r1.record(stream)
            ev_rs.append((r0, r1))
            e0 = torch.cuda.Event(enable_timing=True)
            e1 = torch.cuda.Event(enable_timing=True)
            e0.record(stream)
        if use_graph:
            p.graph_launch(1)
        else:
            p.md_steps(args.theta)
        if record:
            e1.record(stream)
            ev_md.append((e0, e1))
        return p.observables()[0]

    for _ in range(args.warmup):
        temperature_step(False)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    obs_log = []
    for _ in range(args.steps):
        o = temperature_step(True)
        obs_log.append(o)
        R_steps += o["R"] * args.theta
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    md_ms = [a.elapsed_time(b) for a, b in ev_md]
    rs_ms = [a.elapsed_time(b) for a, b in ev_rs]
    # gather traffic of one resampling: read + write of R 6 x npad FP32 slabs
    # (npad = 80 for the 75-atom peptide), energies and ancestors
    slab_bytes = 6 * 80 * 4
    gather_bytes = R * (2 * slab_bytes + 2 * 8 + 2 * 4)
    md_s = sum(md_ms) / 1e3
    value = R_steps / el
    achieved = flops_rs * R_steps / md_s / 1e12
    result = {
        "metric": "replica-MD steps/s",
        "value": value,
        "unit": "replica-MD steps/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": el / args.steps * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32 (FP64 energy sums, weights, Q)",
        "data": "synthetic",
        "config": {"workload": "PAMD, 75-atom synthetic peptide, R=1e5, theta=1000, adaptive T (V=0.1), "
                               "dt=1 fs, " + ("Andersen nu=1/ps" if args.thermostat == "andersen"
                                              else "Langevin gamma=1/ps (B-A-O-A-B)"),
                   "resampling": args.resampling, "thermostat": args.thermostat, "replicas": R, "theta": args.theta, "atoms": sysd.n_atoms, "pairs": pairs,
                   "T_range": [obs_log[0]["T"], obs_log[-1]["T"]]},
        "pair_interactions_per_s": value * pairs,
        "md_kernel_ms_avg": float(np.mean(md_ms)),
        "md_kernel_ms_median": float(np.median(md_ms)),
        "md_replica_steps_per_s": R_steps / md_s,
        "resampling": {"mode": args.resampling, "ms_avg": float(np.mean(rs_ms)),
                       "gather_bytes": gather_bytes,
                       "GB_per_s_whole_step": gather_bytes / (float(np.mean(rs_ms)) * 1e-3) / 1e9},
        "launch": dict(info, graph=use_graph, autotune=tuned),
        "roofline": {"bound": "alu", "achieved": achieved, "peak": PEAK_FP32_VALU_TFLOPS, "unit": "TFLOP/s",
                     "frac": achieved / PEAK_FP32_VALU_TFLOPS,
                     # counters of the Andersen-bath kernel at the default workload only
                     "traffic": measured_traffic() if R == 100000 and args.theta == 1000
                     and args.thermostat == "andersen" else None,
                     "flops_per_replica_step": flops_rs},
    }
    p.close()
    _attainable(result)
    if not args.no_cpu_baseline:
        result["cpu_baseline"] = cpu_baseline(args.cpu_seconds)
    print(json.dumps(result))


if __name__ == "__main__":
    main()
