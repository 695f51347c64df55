"""GPU: a run checkpointed part-way and resumed in a fresh context ends in
exactly the state of the uninterrupted run (positions, velocities, energies,
ancestors, temperatures, sum ln Q, counters), through the C ABI."""
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
    return pamd


CASES = {
    # FP32 peptide, nearest-integer rounding, Andersen bath, adaptive temperatures
    "peptide": dict(sys=lambda: [S.c2_system()], kw=dict(R_target=2000, T0=700.0, dt=0.001, nu=1.0, seed=5,
                                                      precision=1, T_final=400.0), temps=None, theta=40),
    # FP64 bead chain, multinomial draws, Langevin bath, explicit temperatures
    "chain": dict(sys=lambda: [S.c1_system()], kw=dict(R_target=500, T0=2.0, dt=0.002, nu=2.0, seed=6, precision=0,
                                                    resampling="multinomial", thermostat="langevin"),
                  temps=list(S.geometric_schedule(2.0, 0.5, 8)[1:]), theta=50),
    # FP32, two runs in one context: a 40-atom peptide in a register-tile launch
    # and a 120-atom one in the wide launch, geometric device schedule
    "batched": dict(sys=lambda: [S.make_peptide(1807, 40), S.make_peptide(1809, 120)],
                    kw=dict(R_target=300, T0=700.0, dt=0.0005, nu=1.0, seed=8, precision=1,
                            layout=["tile", "wide"]),
                    temps=list(S.geometric_schedule(700.0, 500.0, 8)[1:]), theta=30),
}


def _advance(p, case, first, last):
    for i in range(first, last):
        p.resample(None if case["temps"] is None else [case["temps"][i]] * p.n_runs)
        p.md_steps(case["theta"])


@pytest.mark.parametrize("which", sorted(CASES))
def test_resumed_run_equals_uninterrupted(B, which, tmp_path):
    from paper_1806_06016_amd import checkpoint as CK
    case = CASES[which]
    systems = case["sys"]()
    path = str(tmp_path / "ck.npz")
    a = B.Pamd(systems, **case["kw"])
    a.md_steps(case["theta"])
    _advance(a, case, 0, 3)
    CK.save(a, path)
    _advance(a, case, 3, 6)
    refs = [a.get_state(r) for r in range(len(systems))]
    a.close()
    b = B.Pamd(systems, **case["kw"])
    CK.restore(b, path)
    _advance(b, case, 3, 6)
    gots = [b.get_state(r) for r in range(len(systems))]
    obs = b.observables()
    b.close()
    for r, (ref, got) in enumerate(zip(refs, gots)):
        print(which, r, {k: ref[k] for k in ("T", "R", "temp_index", "step", "sum_lnQ")})
        for k in ("x", "v", "E_pot", "E_kin", "ancestor"):
            assert np.array_equal(ref[k], got[k]), (r, k)
        for k in ("R", "T", "T_prev", "sum_lnQ", "lnQ_last", "step", "temp_index"):
            assert ref[k] == got[k], (r, k)
        assert ref["temp_index"] == 6 and obs[r]["T"] == ref["T"]
