"""Training and evaluation of the learned r-RESPA surrogate, all on the GPU
through the C ABI (argument marshalling and bookkeeping only here).

    python -m paper_1806_06016_amd.mts [--quick]

1. Training data: a population of the 75-atom peptide annealed from 700 K to
   300 K over 41 geometric temperatures (resampling as in the main path),
   snapshots of every replica every theta/4 MD steps: positions and exact
   nonbonded forces (pamd_export_configs).
2. Training: force-matching loss, Adam with a cosine-decayed step size,
   random batches of 256 configurations, 10 % held out.
3. Evaluation at equal physical time, NVE from 256 replicas of the final
   300 K population over a 10 ps window: energy drift as the mean over
   replicas of |slope| of a least-squares line through E_tot(t) per atom
   (kJ/mol/ps/atom) and the RMS of E_tot(t) - E_tot(0), and throughput
   (replica time steps per second, simulated time per second, R = 1e5) for
   plain velocity Verlet at dt = 0.5, 1, 1.5, 2 and 2.5 fs, r-RESPA with the
   trained surrogate (inner 1 fs, outer 2, 3 and 4 fs) and r-RESPA with a
   zero surrogate (the whole nonbonded force in the outer impulse: the method
   without the network).
4. Equal drift: a straight line through log(drift) against log(dt) of the
   plain runs gives the plain time step with the drift of each r-RESPA case;
   plain velocity Verlet's simulated time per second there (its cost per
   step does not depend on dt) is set against the r-RESPA case's.
Prints one JSON line.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time
from typing import Dict, Optional

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

from paper_1806_06016_amd import pamd as B  # noqa: E402
from pamd_inputs import systems as S  # noqa: E402
from pamd_inputs.weights import surrogate_weights  # noqa: E402


def geometric(T0: float, T1: float, n: int):
    return [T0 * (T1 / T0) ** (i / (n - 1)) for i in range(n)]


def collect(sysd, R: int, temps, theta: int, snaps_per_T: int, seed: int, dt: float = 0.001):
    """Annealed population snapshots -> (x, F_nb) CUDA float32 [n_conf, n, 3]."""
    import torch
    p = B.Pamd([sysd], R_target=R, T0=temps[0], dt=dt, nu=1.0, seed=seed, precision=B.PAMD_FP32)
    p.md_steps(theta)
    xs, fs = [], []
    for i, T in enumerate(temps):
        if i > 0:
            p.resample([T])
        for _ in range(snaps_per_T):
            p.md_steps(theta // snaps_per_T)
            x, f = p.export_configs(0, 0, None)
            xs.append(x)
            fs.append(f)
    state = p.get_state(0)
    p.close()
    torch.cuda.synchronize()
    return torch.cat(xs), torch.cat(fs), state


def train(nn, x, f, steps: int, batch: int = 256, lr0: float = 1e-3, seed: int = 0, val_frac: float = 0.1):
    import torch
    n = x.shape[0]
    g = torch.Generator(device="cuda")
    g.manual_seed(seed)
    perm = torch.randperm(n, generator=g, device="cuda")
    nv = max(1, int(val_frac * n))
    vi, ti = perm[:nv], perm[nv:]
    loss = torch.zeros(1, dtype=torch.float32, device="cuda")
    hist = []
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for it in range(steps):
        lr = 0.5 * lr0 * (1.0 + math.cos(math.pi * it / steps))
        idx = ti[torch.randint(0, ti.numel(), (batch,), generator=g, device="cuda")]
        nn.train_step(x[idx].contiguous(), f[idx].contiguous(), max(lr, 1e-7), loss)
        if it % max(1, steps // 20) == 0 or it == steps - 1:
            hist.append((it, float(loss.item())))
    torch.cuda.synchronize()
    el = time.perf_counter() - t0

    def mean_loss(ids):
        s, m = 0.0, 0
        chunk = nn.max_conf          # the largest batch the surrogate's workspace takes
        for c0 in range(0, ids.numel(), chunk):
            c = ids[c0:c0 + chunk]
            lv, _ = nn.loss_grad(x[c].contiguous(), f[c].contiguous(), want_grad=False)
            s += float(lv.item()) * c.numel()
            m += c.numel()
        return s / m

    val = mean_loss(vi)
    f2 = float((f[vi] ** 2).mean().item())
    return dict(train_seconds=el, steps=steps, batch=batch, history=hist, val_loss=val,
                val_rel_force_rms=math.sqrt(val / f2), n_train=int(ti.numel()), n_val=int(nv))


def nve_run(sysd, x0, v0, dt: float, nn=None, M: int = 1, window_ps: float = 10.0, sample_ps: float = 0.1,
            seed: int = 7) -> Dict:
    """NVE (nu = 0) from (x0, v0): drift of E_tot and wall time of the MD."""
    import torch
    R = x0.shape[0]
    p = B.Pamd([sysd], R_target=R, T0=300.0, dt=dt, nu=0.0, seed=seed, precision=B.PAMD_FP32)
    p.set_state(0, x0, v0, T=300.0)
    if nn is not None:
        p.set_mts(nn, M)
    p.md_steps(0)
    st = p.get_state(0)
    E0 = st["E_pot"] + st["E_kin"]
    n_sample = int(round(window_ps / sample_ps))
    k = int(round(sample_ps / dt))
    if nn is not None:
        k = max(M, k // M * M)
    dev = []
    times = []
    s0, s1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    ms = 0.0
    unstable = False
    for _ in range(n_sample):
        s0.record(p.stream)
        p.md_steps(k)
        s1.record(p.stream)
        try:
            st = p.get_state(0)
        except B.PamdError as e:
            if e.code != B.PAMD_ERR_NONFINITE:
                raise
            unstable = True          # some replica's energy became non-finite
            break
        ms += s0.elapsed_time(s1)
        E = st["E_pot"] + st["E_kin"]
        dev.append(E - E0)
        times.append(len(dev) * k * dt)
    done = len(dev) * k
    out = dict(dt_fs=dt * 1000.0, outer_fs=(M * dt * 1000.0 if nn is not None else dt * 1000.0),
               replicas=R, steps=done, md_ms=ms, unstable=unstable)
    if unstable or not dev:
        out["rms_drift_kJmol"] = float("inf")
        out["drift_kJmol_ps_atom"] = float("inf")
    else:
        dv = np.array(dev)                                   # [samples, replicas]
        out["rms_drift_kJmol"] = float(np.sqrt(np.mean(dv ** 2)))
        # least-squares slope of E_tot(t) - E_tot(0) through (0, 0) and the samples, per replica
        t = np.concatenate([[0.0], times])
        y = np.vstack([np.zeros(dv.shape[1]), dv])
        tc = t - t.mean()
        slope = (tc[:, None] * (y - y.mean(0))).sum(0) / (tc * tc).sum()
        out["drift_kJmol_ps_atom"] = float(np.mean(np.abs(slope)) / sysd.n_atoms)
    if done > 0 and ms > 0:
        out["replica_steps_per_s"] = R * done / (ms / 1000.0)
        out["replica_ps_per_s"] = out["replica_steps_per_s"] * dt
    p.close()
    return out


def throughput(sysd, x0, v0, dt: float, nn=None, M: int = 1, R: int = 100000, steps: int = 400) -> Dict:
    """Replica time steps per second at population size R (inputs resident)."""
    import torch
    steps = max(M, steps // max(M, 1) * max(M, 1))   # whole outer steps
    rep = int(math.ceil(R / x0.shape[0]))
    x = np.concatenate([x0] * rep)[:R]
    v = np.concatenate([v0] * rep)[:R]
    p = B.Pamd([sysd], R_target=R, T0=300.0, dt=dt, nu=1.0, seed=3, precision=B.PAMD_FP32)
    p.set_state(0, x, v, T=300.0)
    if nn is not None:
        p.set_mts(nn, M)
    p.md_steps(steps // 4 // max(M, 1) * max(M, 1) or max(M, 1))
    torch.cuda.synchronize()
    s0, s1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    s0.record(p.stream)
    p.md_steps(steps)
    s1.record(p.stream)
    s1.synchronize()
    ms = s0.elapsed_time(s1)
    p.close()
    return dict(R=R, steps=steps, ms=ms, replica_steps_per_s=R * steps / (ms / 1000.0),
                replica_ps_per_s=R * steps * dt / (ms / 1000.0))


def anneal_curve(sysd, R: int, sched, theta: int, theta_eq: int, seed: int, nn=None, M: int = 1,
                 dt: float = 0.001) -> np.ndarray:
    """<E_pot>(T) of one PAMD run (nearest-integer resampling, Andersen
    1/ps): theta_eq plain velocity-Verlet steps at sched[0], then for every
    further temperature a resampling and theta steps of dt, by plain velocity
    Verlet or, with a surrogate, by r-RESPA with outer step M dt."""
    p = B.Pamd([sysd], R_target=R, T0=sched[0], dt=dt, nu=1.0, seed=seed, precision=B.PAMD_FP32)
    p.md_steps(theta_eq)
    E = [p.observables()[0]["E_mean"]]
    if nn is not None:
        p.set_mts(nn, M)
    for T in sched[1:]:
        p.resample([T])
        p.md_steps(theta)
        E.append(p.observables()[0]["E_mean"])
    p.close()
    return np.array(E)


def equal_drift(plain: Dict[float, Dict], case: Dict) -> Dict:
    """Plain velocity Verlet at the drift of `case`: a least-squares line
    through log(drift) against log(dt) of the plain runs (dt in fs -> result)
    gives the time step dt* with that drift; plain MD costs the same per step
    at any dt, so its simulated time per second at dt* is its measured
    replica-steps/s times dt*.  Returns dt*, that rate and the case's rate
    over it."""
    pts = [(dt, r) for dt, r in plain.items() if np.isfinite(r["drift_kJmol_ps_atom"]) and r["drift_kJmol_ps_atom"] > 0]
    d = case["drift_kJmol_ps_atom"]
    if len(pts) < 2 or not np.isfinite(d) or d <= 0:
        return dict(dt_equal_fs=None, plain_replica_ps_per_s=None, speedup=None)
    lx = np.log([p[0] for p in pts])
    ly = np.log([p[1]["drift_kJmol_ps_atom"] for p in pts])
    b, a = np.polyfit(lx, ly, 1)                 # log drift = a + b log dt
    dt_eq = float(np.exp((math.log(d) - a) / b))
    steps_per_s = float(np.mean([p[1]["throughput"]["replica_steps_per_s"] for p in pts]))
    plain_rate = steps_per_s * dt_eq * 1e-3      # replica-ps/s
    return dict(dt_equal_fs=dt_eq, drift_exponent=float(b), plain_replica_ps_per_s=plain_rate,
                speedup=case["throughput"]["replica_ps_per_s"] / plain_rate,
                extrapolated=bool(dt_eq > max(p[0] for p in pts) or dt_eq < min(p[0] for p in pts)))


def kernel_timing(R: int, reps: int = 5) -> Dict:
    """Surrogate inference on R perturbed peptide configurations and training
    steps on batches of 256 (seeded weights): the workload of the kernel
    profiles."""
    import torch
    sysd = S.c2_system()
    nn = B.PamdNN(sysd, sysd.atype, max_conf=R)
    nn.set_weights(surrogate_weights(3))
    rng = np.random.default_rng(1)
    x = torch.tensor(sysd.x_init[None] + rng.normal(0, 0.01, (R,) + sysd.x_init.shape), dtype=torch.float32,
                     device="cuda")
    for _ in range(2):
        E, F = nn.forces(x)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(reps):
        E, F = nn.forces(x)
    torch.cuda.synchronize()
    fwd = (time.perf_counter() - t0) / reps
    xb, fb = x[:256].contiguous(), (1.1 * F[:256]).contiguous()
    loss = torch.zeros(1, dtype=torch.float32, device="cuda")
    for _ in range(5):
        nn.train_step(xb, fb, 1e-4, loss)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(20):
        nn.train_step(xb, fb, 1e-4, loss)
    torch.cuda.synchronize()
    tr = (time.perf_counter() - t0) / 20
    nn.close()
    return dict(R=R, forces_ms=fwd * 1e3, ns_per_replica=fwd * 1e9 / R, train_step_ms_batch256=tr * 1e3)


def main(argv=None):
    import torch
    ap = argparse.ArgumentParser()
    ap.add_argument("--kernels", type=int, default=0, metavar="R",
                    help="only time surrogate inference on R configurations and training steps")
    ap.add_argument("--quick", action="store_true", help="small data / training / windows")
    ap.add_argument("--replicas", type=int, default=10000, help="population of the data collection")
    ap.add_argument("--train-steps", type=int, default=20000)
    ap.add_argument("--window-ps", type=float, default=10.0)
    ap.add_argument("--save", default="", help="write the trained parameters (.npy)")
    a = ap.parse_args(argv)
    if a.kernels > 0:
        B.load_library()
        print(json.dumps(kernel_timing(a.kernels)))
        return
    if a.quick:
        a.replicas, a.train_steps, a.window_ps = 1000, 300, 1.0
    B.load_library()
    sysd = S.c2_system()
    temps = geometric(700.0, 300.0, 41)
    t0 = time.perf_counter()
    x, f, st = collect(sysd, a.replicas, temps, 1000, 4, seed=11)
    t_collect = time.perf_counter() - t0
    print(f"collected {x.shape[0]} configurations in {t_collect:.1f} s", flush=True)
    nn = B.PamdNN(sysd, sysd.atype, max_conf=4096)     # validation loss in chunks of 4096 configurations
    nn.set_weights(surrogate_weights(2024, 0.5))
    tr = train(nn, x, f, a.train_steps)
    print(f"trained: val relative force RMS {tr['val_rel_force_rms']:.3f} in {tr['train_seconds']:.1f} s",
          flush=True)
    if a.save:
        np.save(a.save, B.pack_params(nn.get_weights()))
    del x, f
    torch.cuda.empty_cache()
    # NVE starts: 256 replicas of the final 300 K population
    R0 = 256
    x0, v0 = st["x"][:R0], st["v"][:R0]
    zero = B.PamdNN(sysd, sysd.atype)
    cases = [(f"vv_{dt}fs", dt * 1e-3, None, 1) for dt in (0.5, 1.0, 1.5, 2.0, 2.5)]
    cases += [(f"respa_nn_{M}fs", 0.001, nn, M) for M in (2, 3, 4)]
    cases += [(f"respa_zero_{M}fs", 0.001, zero, M) for M in (2, 3, 4)]
    res = {}
    for name, dt, net, M in cases:
        d = nve_run(sysd, x0, v0, dt, net, M, window_ps=a.window_ps)
        thr = throughput(sysd, x0, v0, dt, net, M, R=20000 if a.quick else 100000)
        d["throughput"] = thr
        res[name] = d
        print(name, json.dumps({k: v for k, v in d.items() if k != "throughput"}),
              "throughput", json.dumps(thr), flush=True)
    plain = {float(n[3:-2]): r for n, r in res.items() if n.startswith("vv_")}
    eq = {n: equal_drift(plain, r) for n, r in res.items() if n.startswith("respa_")}
    for n, e in eq.items():
        print(n, "at equal drift:", json.dumps(e), flush=True)
    line = dict(metric="replica_ps_per_s", data="synthetic", config=dict(workload="peptide75 MTS surrogate",
                collect_replicas=a.replicas, temperatures=41), training=tr, cases=res, equal_drift=eq,
                collect_seconds=t_collect)
    print(json.dumps(line))
    nn.close()
    zero.close()


if __name__ == "__main__":
    main()
