"""What resampling buys: population annealing against plain annealing of
independent copies on the 75-atom synthetic peptide, all on the GPU through
the C ABI (bookkeeping only here).

    python -m paper_1806_06016_amd.ablation [--replicas R] [--seeds K]

The synthetic analogue of the paper's comparison of measured against bath
temperature (PA with two sweep lengths theta, and PA with resampling switched
off) and of its lowest-temperature energy histograms: the paper's eight
temperatures 700 ... 200 K, the Langevin bath (friction 1/ps, dt = 0.5 fs),
a population equilibrated at 700 K for theta_eq steps, then theta steps at
each lower temperature.  Variants: PA with the paper's multinomial
resampling at theta = 1000 and 4375, PA with nearest-integer resampling at
theta = 4375, and "anneal" (resampling off) at theta = 4375.  Per variant and
temperature: measured (kinetic) temperature, <E_pot>, families, mean and
standard error over independent seeds; at 200 K the E_pot histogram.
Prints one JSON line.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

from paper_1806_06016_amd import pamd as B  # noqa: E402
from pamd_inputs import systems as S  # noqa: E402

TEMPS = [700.0, 585.0, 489.0, 409.0, 342.0, 286.0, 239.0, 200.0]
VARIANTS = [("PA multinomial", "multinomial", 1000), ("PA multinomial", "multinomial", 4375),
            ("PA nearest", "nearest", 4375), ("anneal", "none", 4375)]


def run(sysd, mode: str, theta: int, R: int, seed: int, theta_eq: int, dt: float = 0.0005,
        gamma: float = 1.0):
    """One annealing run; returns per-temperature observables and the final
    potential energies."""
    p = B.Pamd([sysd], R_target=R, T0=TEMPS[0], dt=dt, nu=gamma, seed=seed, precision=B.PAMD_FP32,
               thermostat="langevin", resampling=mode)
    p.md_steps(theta_eq)
    rows = []
    for i, T in enumerate(TEMPS):
        if i > 0:
            p.resample([T])
            p.md_steps(theta)
        o = p.observables()[0]
        rows.append(dict(T=o["T"], T_measured=o["T_measured"], E_mean=o["E_mean"], R=o["R"],
                         families=o["families"], sum_lnQ=o["sum_lnQ"]))
    E = p.get_state(0, want_xv=False)["E_pot"]
    p.close()
    return rows, E


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("--replicas", type=int, default=10000)
    ap.add_argument("--seeds", type=int, default=4)
    ap.add_argument("--theta-eq", type=int, default=20000)
    ap.add_argument("--bins", type=int, default=24)
    args = ap.parse_args(argv)
    sysd = S.c2_system()
    out = {"system": "75-atom synthetic peptide", "replicas": args.replicas, "seeds": args.seeds,
           "temperatures": TEMPS, "dt_fs": 0.5, "gamma_per_ps": 1.0, "theta_eq": args.theta_eq, "variants": []}
    finals = {}
    t0 = time.perf_counter()
    for name, mode, theta in VARIANTS:
        per_seed, E_last = [], []
        for k in range(args.seeds):
            rows, E = run(sysd, mode, theta, args.replicas, 1000 + k, args.theta_eq)
            per_seed.append(rows)
            E_last.append(E)
            print(f"{name} theta={theta} seed {k}: <E>(200 K) {rows[-1]['E_mean']:.2f}, "
                  f"T_m {rows[-1]['T_measured']:.1f}", file=sys.stderr, flush=True)
        key = f"{name}, theta={theta}"
        finals[key] = np.concatenate(E_last)

        def stat(field):
            a = np.array([[r[field] for r in rows] for rows in per_seed])
            return a.mean(0).tolist(), (a.std(0, ddof=1) / np.sqrt(len(a))).tolist() if len(a) > 1 else None

        Tm, Tm_se = stat("T_measured")
        Em, Em_se = stat("E_mean")
        fam, _ = stat("families")
        out["variants"].append(dict(variant=key, T_measured=Tm, T_measured_se=Tm_se, E_mean=Em, E_mean_se=Em_se,
                                    families=fam))
    lo = min(float(e.min()) for e in finals.values())
    hi = max(float(e.max()) for e in finals.values())
    edges = np.linspace(lo, hi, args.bins + 1)
    out["histogram_200K"] = {"edges": edges.tolist(),
                             **{k: np.histogram(e, edges)[0].tolist() for k, e in finals.items()}}
    out["seconds"] = time.perf_counter() - t0
    print(json.dumps(out))


if __name__ == "__main__":
    main()
