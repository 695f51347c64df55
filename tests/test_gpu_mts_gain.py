"""GPU: what the trained surrogate gains over r-RESPA without it.

The surrogate is trained on the GPU (the library's own forward, backward and
Adam kernels) on configurations and exact nonbonded forces that PAMD itself
generates (a 2000-replica population annealed 700 -> 300 K, snapshots every
250 steps).  With F_NN = 0 the outer impulse of r-RESPA carries the whole
nonbonded force (relative residual 1); the trained network must cut the
held-out residual |F_nb - F_NN| / |F_nb| below 0.5 and keep a 4 fs outer step
stable over 1 ps of NVE dynamics.  Plain velocity Verlet stays the reference for
the r-RESPA runs: annealed <E_pot>(T) with the trained surrogate (outer step
2 fs) agrees with plain velocity Verlet (1 fs) under the covariance-aware
rule of energy_curve_stats (8 + 8 independently seeded runs of a reduced
anneal, 700 -> 500 K in 9 geometric steps, theta = 160 fs, R = 300).
"""
import math

import numpy as np
import pytest

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

from energy_curve_stats import compare_energy_curves, report  # noqa: E402
from pamd_inputs import systems as S  # noqa: E402
from pamd_inputs.weights import surrogate_weights  # noqa: E402


@pytest.fixture(scope="module")
def B():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1806_06016_amd import pamd
    pamd.load_library()
    return pamd


def test_trained_surrogate_reduces_the_outer_impulse(B):
    from paper_1806_06016_amd import mts
    sysd = S.c2_system()
    print("collecting training data", flush=True)
    x, f, st = mts.collect(sysd, 2000, mts.geometric(700.0, 300.0, 41), 1000, 4, seed=5)
    nn = B.PamdNN(sysd, sysd.atype)
    nn.set_weights(surrogate_weights(2024, 0.5))
    print(f"training on {x.shape[0]} configurations", flush=True)
    tr = mts.train(nn, x, f, steps=3000, seed=1)
    print("held-out relative force residual", tr["val_rel_force_rms"])
    assert tr["val_rel_force_rms"] < 0.5
    del x, f
    # 1 ps of NVE with a 4 fs outer step from the final 300 K population
    x0, v0 = st["x"][:128], st["v"][:128]
    d = mts.nve_run(sysd, x0, v0, 0.001, nn, 4, window_ps=1.0, sample_ps=0.1)
    print("r-RESPA 4 fs with the trained surrogate:", d)
    assert not d["unstable"] and math.isfinite(d["rms_drift_kJmol"])
    # plain MD as the reference: annealed <E_pot>(T), r-RESPA + surrogate against velocity Verlet
    sched = S.geometric_schedule(700.0, 500.0, 9)
    print("annealing: plain velocity Verlet and r-RESPA with the trained surrogate, 8 + 8 runs", flush=True)
    vv = np.array([mts.anneal_curve(sysd, 300, sched, 160, 400, seed) for seed in range(1, 9)])
    rs = np.array([mts.anneal_curve(sysd, 300, sched, 160, 400, seed, nn=nn, M=2) for seed in range(11, 19)])
    res = compare_energy_curves(rs, vv)
    print(report(res))
    assert res["p_hotelling"] > 0.01 and res["p_count"] > 0.01 and res["p_max"] > 0.01
    nn.close()
