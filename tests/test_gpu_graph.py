"""GPU: HIP-graph replay of a PAMD temperature step, device schedules and the
autotuner, all through the C ABI."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

from oracle import oracle as O  # noqa: E402
from pamd_inputs import systems as S  # noqa: E402


@pytest.fixture(scope="module")
def B():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1806_06016_amd import pamd
    pamd.load_library()
    return pamd


def _state(p):
    st = p.get_state(0)
    return st["x"], st["v"], st["E_pot"], st["ancestor"], st["T"], st["sum_lnQ"]


@pytest.mark.parametrize("mode,thermostat,resampling", [("adaptive", "andersen", "nearest"),
                                                        ("schedule", "andersen", "nearest"),
                                                        ("adaptive", "langevin", "multinomial"),
                                                        ("schedule", "langevin", "none")])
def test_graph_replay_matches_eager(B, mode, thermostat, resampling):
    """One capture replayed for several temperatures equals the eager call
    sequence bit for bit, with eager work (observables, state reads) between
    replays; both baths and every resampling rule (the multinomial draws and
    the Langevin noise come from device-side counters inside the graph)."""
    sysd = S.c2_system()
    R, theta = 1000, 40
    sched = S.geometric_schedule(700.0, 250.0, 40)
    kw = dict(R_target=R, T0=700.0, dt=0.001, nu=1.0, seed=11, T_final=250.0, V_target=0.1,
              thermostat=thermostat, resampling=resampling)
    pe = B.Pamd([sysd], **kw)
    pg = B.Pamd([sysd], **kw)
    for p in (pe, pg):
        p.set_schedule(0, sched)
        p.md_steps(theta)
    pg.graph_capture(theta, mode)              # slot 0, resample + MD
    for it in range(4):
        pe.resample([0.0 if mode == "adaptive" else -1.0])
        pe.md_steps(theta)
        oe = pe.observables()[0]
        pg.graph_launch()
        og = pg.observables()[0]
        assert oe["T"] == og["T"] and oe["R"] == og["R"] and oe["temp_index"] == it + 1
        for a, b in zip(_state(pe), _state(pg)):
            assert np.array_equal(a, b)
        if mode == "schedule":
            assert abs(og["T"] - sched[it + 1]) < 1e-12
    pe.close()
    pg.close()


def test_schedule_mode_equals_explicit_temperatures(B):
    sysd = S.c1_system()
    sched = S.geometric_schedule(2.0, 0.5, 20)
    kw = dict(R_target=300, T0=2.0, dt=0.002, nu=1.0, seed=5, precision=0)
    pa = B.Pamd([sysd], **kw)
    pb = B.Pamd([sysd], **kw)
    pb.set_schedule(0, sched)
    for p in (pa, pb):
        p.md_steps(100)
    for i in range(1, 5):
        pa.resample([sched[i]])
        pb.resample([-1.0])
        pa.md_steps(50)
        pb.md_steps(50)
        for a, b in zip(_state(pa), _state(pb)):
            assert np.array_equal(a, b)
    pa.close()
    pb.close()


def test_autotuner_returns_a_candidate(B, tmp_path):
    from paper_1806_06016_amd.autotune import autotune
    sysd = S.c2_system()
    r = autotune(sysd, R_probe=4096, theta_probe=10, candidates=(16, 8), cache_path=str(tmp_path / "c.json"))
    assert r["waves_per_block"] in (16, 8) and not r["cached"]
    r2 = autotune(sysd, R_probe=4096, theta_probe=10, candidates=(16, 8), cache_path=str(tmp_path / "c.json"))
    assert r2["cached"] and r2["waves_per_block"] == r["waves_per_block"]
    # the Langevin kernel is another instantiation: probed and cached on its own
    r3 = autotune(sysd, R_probe=4096, theta_probe=10, candidates=(16, 8), cache_path=str(tmp_path / "c.json"),
                  thermostat="langevin")
    assert r3["waves_per_block"] in (16, 8) and not r3["cached"]
    r4 = autotune(sysd, R_probe=4096, theta_probe=10, candidates=(16, 8), cache_path=str(tmp_path / "c.json"),
                  thermostat="langevin")
    assert r4["cached"] and r4["waves_per_block"] == r3["waves_per_block"]
