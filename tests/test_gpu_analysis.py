"""The library's population analysis (host FP64 entry points of the C ABI)
against the oracle, and on a PA run of the GPU path.

* family / binning errors, rho_t, family entropy: 1e-12 relative to the oracle
  (different summation order only);
* WHAM: refined ln Z within 1e-9 of the oracle's (both iterate to 1e-11), the
  reweighted <E>, <E^2> within 1e-10 relative;
* error paths: too few bins, non-finite values, empty sample sets;
* end to end: a PA run of the zero-rest-length Gaussian chain on the GPU
  (FP64), energies of every temperature collected from the device, WHAM
  started from the running sum of ln Q: ln Z(T_N) - ln Z(T_0) within 0.3 of
  the exact 13.5 ln(1/4) (one run of R = 1000: statistical error ~0.1), the
  reweighted <U> at temperatures between the grid points within 2 % of
  13.5 T, and the family error at the last temperature not below the naive one.
"""
import math

import numpy as np
import pytest

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

from oracle import analysis as A  # noqa: E402
from pamd_inputs import systems as S  # noqa: E402


@pytest.fixture(scope="module")
def B():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1806_06016_amd import pamd
    pamd.load_library()
    return pamd


@pytest.mark.parametrize("R,F", [(1, 1), (2, 1), (1000, 1000), (1000, 37), (4099, 300)])
def test_family_and_binning_errors_match_oracle(B, R, F):
    rng = np.random.default_rng(R + F)
    O = rng.normal(-300.0, 20.0, R)
    anc = rng.integers(0, F, R).astype(np.int32) * 7 + 3
    g = B.family_error(O, anc)
    o = A.family_error(O, anc)
    for k in ("mean", "naive_se", "family_se", "rho_t", "family_entropy"):
        assert abs(g[k] - o[k]) <= 1e-12 * max(1.0, abs(o[k])), k
    assert g["families"] == o["families"]
    for b in (1, 3, 8):
        if R // b >= 2:
            assert abs(B.binning_error(O, b) / A.binning_error(O, b) - 1) < 1e-12


def test_error_paths(B):
    with pytest.raises(B.PamdError) as e:
        B.binning_error(np.ones(5), 3)
    assert e.value.code == B.PAMD_ERR_ARG
    with pytest.raises(B.PamdError) as e:
        B.family_error(np.array([1.0, np.nan]), np.array([0, 1]))
    assert e.value.code == B.PAMD_ERR_NONFINITE
    with pytest.raises(B.PamdError) as e:
        B.wham([1.0, 0.5], [np.ones(3), np.ones(0)], [0.0, 0.0])
    assert e.value.code == B.PAMD_ERR_ARG


def test_wham_matches_oracle(B):
    betas = 1.0 / (2.0 * 0.25 ** (np.arange(21) / 20))
    rng = np.random.default_rng(5)
    samples = [rng.gamma(13.5, 1.0 / b, 200 + 37 * l) for l, b in enumerate(betas)]
    start = rng.normal(0, 1, 21)
    z, it = B.wham(betas, samples, start, tol=1e-11)
    zo, ito = A.wham(betas, samples, start, tol=1e-11)
    print("iterations", it, ito)
    assert np.abs(z - zo).max() < 1e-9 and abs(it - ito) <= 1
    assert z[0] == start[0]
    for bq in (betas[0], 0.7, betas[-1]):
        e1, e2 = B.wham_average(bq, betas, samples, z)
        o1, o2 = A.wham_average(bq, betas, samples, zo)
        assert abs(e1 / o1 - 1) < 1e-10 and abs(e2 / o2 - 1) < 1e-10


def test_pa_run_free_energy_refined_by_wham(B):
    sysd = S.gaussian_chain(10, 100.0, 0.0)
    sched = S.geometric_schedule(2.0, 0.5, 20)
    R = 1000
    rng = np.random.default_rng(17)
    b = rng.normal(0, math.sqrt(2.0 / 100.0), (R, 9, 3))
    x0 = np.zeros((R, 10, 3))
    x0[:, 1:] = np.cumsum(b, axis=1)
    p = B.Pamd([sysd], R_target=R, T0=2.0, dt=0.002, nu=1.0, seed=23, precision=0)
    p.set_state(0, np.ascontiguousarray(x0), p.get_state(0)["v"], T=2.0)
    p.md_steps(100)
    samples, lnq = [p.get_state(0, want_xv=False)["E_pot"]], [0.0]
    for T in sched[1:]:
        p.resample([T])
        p.md_steps(100)
        st = p.get_state(0, want_xv=False)
        samples.append(st["E_pot"])
        lnq.append(st["sum_lnQ"])
    last = p.get_state(0, want_xv=False)
    p.close()
    betas = 1.0 / sched
    exact = 13.5 * math.log(0.25)
    z, it = B.wham(betas, samples, lnq, tol=1e-10)
    print(f"sum lnQ {lnq[-1]:.4f}  WHAM {z[-1] - z[0]:.4f}  exact {exact:.4f}  ({it} iterations)")
    assert abs(lnq[-1] - exact) < 0.3 and abs(z[-1] - z[0] - exact) < 0.3
    for l in (5, 15):
        Tq = math.sqrt(sched[l] * sched[l + 1])
        Em, _ = B.wham_average(1.0 / Tq, betas, samples, z)
        assert abs(Em / (13.5 * Tq) - 1) < 0.02
    fe = B.family_error(last["E_pot"], last["ancestor"])
    print("families", fe["families"], "rho_t", fe["rho_t"], "naive", fe["naive_se"], "family", fe["family_se"])
    assert fe["families"] < R and fe["rho_t"] > 1.0
    assert fe["family_se"] >= fe["naive_se"] * 0.9
