"""CPU: the equal-drift comparison of the r-RESPA evaluation (host
arithmetic of paper_1806_06016_amd.mts, no GPU)."""
import math

import pytest

from paper_1806_06016_amd import mts


def _case(drift, steps_per_s=None, ps_per_s=None):
    thr = {}
    if steps_per_s is not None:
        thr["replica_steps_per_s"] = steps_per_s
    if ps_per_s is not None:
        thr["replica_ps_per_s"] = ps_per_s
    return {"drift_kJmol_ps_atom": drift, "throughput": thr}


def test_equal_drift_recovers_the_time_step_of_a_power_law():
    """Plain drift c dt^2 at dt = 0.5 .. 2 fs and a constant cost per step:
    a case with drift c 1.3^2 sits at dt* = 1.3 fs, where plain MD simulates
    4e8 x 1.3e-3 replica-ps per second."""
    c = 0.02
    plain = {dt: _case(c * dt ** 2, steps_per_s=4e8) for dt in (0.5, 1.0, 1.5, 2.0)}
    case = _case(c * 1.3 ** 2, ps_per_s=1e4)
    e = mts.equal_drift(plain, case)
    assert e["dt_equal_fs"] == pytest.approx(1.3, rel=1e-9)
    assert e["drift_exponent"] == pytest.approx(2.0, rel=1e-9)
    assert e["plain_replica_ps_per_s"] == pytest.approx(4e8 * 1.3e-3, rel=1e-9)
    assert e["speedup"] == pytest.approx(1e4 / (4e8 * 1.3e-3), rel=1e-9)
    assert not e["extrapolated"]
    assert mts.equal_drift(plain, _case(c * 3.0 ** 2, ps_per_s=1.0))["extrapolated"]


def test_equal_drift_without_a_finite_case_drift():
    plain = {dt: _case(0.1 * dt ** 2, steps_per_s=1e8) for dt in (1.0, 2.0)}
    e = mts.equal_drift(plain, _case(math.inf, ps_per_s=1.0))
    assert e["dt_equal_fs"] is None and e["speedup"] is None
