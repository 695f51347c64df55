"""GPU: the roofline calibrations run and return plausible figures (the FP32
FMA rate of all-VGPR FMAs, the issue cost of single VALU instruction forms)."""
import math

import pytest

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def B():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1806_06016_amd import pamd
    pamd.load_library()
    return pamd


def test_fma_rate_and_instruction_forms(B):
    tf = B.fp32_fma_rate()
    print("FP32 FMA TFLOP/s", tf, flush=True)
    assert 10.0 < tf < 200.0
    r = B.valu_issue_rates(4)
    print(r, flush=True)
    assert 0.5 < r["clock_ghz"] < 3.5
    cyc = r["cycles_per_instr"]
    assert set(cyc) == set(B.VALU_FORMS)
    assert all(math.isfinite(v) and 0.5 < v < 64.0 for v in cyc.values())
    with pytest.raises(B.PamdError):
        st = B.load_library().pamd_valu_issue_rates(None, 4, None, None, None)
        if st != B.PAMD_OK:
            raise B.PamdError(st, "rejected")
