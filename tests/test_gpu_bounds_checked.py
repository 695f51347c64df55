"""GPU: the bounds-checked build (libpamd_check.so: the resampling kernels
compiled with PAMD_BOUNDS_CHECK, which verify every destination offset of the
scan and every source slot of the gather on the device and raise
PAMD_ERR_INTERNAL instead of an out-of-range access).  Whole anneals with each
copy-number rule, a fluctuating population size, a capacity overflow and the
batched wide layout run without an index error, and give exactly the results
of the production library (the same kernels but for the checks)."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

from pamd_inputs import systems as S  # noqa: E402


@pytest.fixture(scope="module")
def B():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1806_06016_amd import pamd
    pamd.load_library()
    pamd.load_library(pamd.CHECK_LIB_PATH)
    return pamd


def _anneal(B, library, systems, mode, R):
    p = B.Pamd(systems, R_target=R, T0=700.0, dt=0.0005, nu=1.0, seed=12, precision=B.PAMD_FP32,
               resampling=mode, T_final=400.0, library=library)
    p.md_steps(20)
    out = []
    for _ in range(4):
        p.resample(None)          # adaptive steps: copy numbers fluctuate around R
        p.md_steps(20)
        obs = p.observables()
        out.append([(o["R"], o["T"], o["sum_lnQ"], o["E_mean"], o["families"]) for o in obs])
    states = [p.get_state(r) for r in range(len(systems))]
    p.close()
    return out, states


@pytest.mark.parametrize("mode", ["nearest", "multinomial", "none"])
@pytest.mark.parametrize("which", ["peptide", "batched"])
def test_checked_build_runs_clean_and_matches(B, mode, which):
    systems = [S.c2_system()] if which == "peptide" else [S.make_peptide(1806, 40), S.make_peptide(1809, 120)]
    print("bounds-checked anneal", which, mode, flush=True)
    a, sa = _anneal(B, B.CHECK_LIB_PATH, systems, mode, 700)
    b, sb = _anneal(B, B.LIB_PATH, systems, mode, 700)
    assert a == b
    for x, y in zip(sa, sb):
        assert np.array_equal(x["x"], y["x"]) and np.array_equal(x["ancestor"], y["ancestor"])


def test_checked_build_reports_capacity_not_an_index_error(B):
    """Every fractional copy number rounded up: the scan sees the overflow and
    writes nothing (PAMD_ERR_CAPACITY, not PAMD_ERR_INTERNAL)."""
    sysd = S.c1_system()
    R = 200
    p = B.Pamd([sysd], R_target=R, T0=2.0, dt=0.002, nu=1.0, seed=3, precision=B.PAMD_FP64, R_cap=220,
               library=B.CHECK_LIB_PATH)
    E = np.where(np.arange(R) < 100, 0.0, 50.0)
    st = p.get_state(0)
    p.set_state(0, st["x"][:R], st["v"][:R], T=2.0, E_pot=E)
    p.resample([1.0], uniforms=torch.zeros(p.R_cap, dtype=torch.float64, device="cuda"))
    with pytest.raises(B.PamdError) as ei:
        p.observables()
    assert ei.value.code == B.PAMD_ERR_CAPACITY
    p.close()
