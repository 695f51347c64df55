"""GPU: the annealing driver end to end on the bead-chain configuration (FP64,
R = 256, 21 temperatures): its per-temperature <E_pot> and sum ln Q equal the
oracle's anneal with the same seeds, the JSON-lines log holds every record,
and a run interrupted and resumed from the driver's checkpoint ends exactly
as the uninterrupted one."""
import json
import os

import numpy as np
import pytest

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

from oracle import oracle as O  # noqa: E402

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CFG = os.path.join(ROOT, "paper_1806_06016_amd", "configs", "bead_chain10_R256.json")


@pytest.fixture(scope="module")
def D():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1806_06016_amd import driver
    return driver


def test_bead_chain_run_matches_oracle(D, tmp_path):
    log = str(tmp_path / "run.jsonl")
    recs = D.run_pamd(CFG, log=log)
    lines = [json.loads(s) for s in open(log)]
    assert lines == json.loads(json.dumps(recs))
    assert [r["temp_index"] for r in recs] == list(range(21))
    cfg = D.load_config(CFG)
    sysd = D.build_systems(cfg)[0]
    res = O.anneal(sysd, cfg["R"], cfg["T0"], D.temperatures(cfg), theta=cfg["theta"], theta_eq=cfg["theta_eq"],
                   dt=cfg["dt"], nu=cfg["nu"], seed=cfg["seed"])
    Eo = np.array([o["E_mean"] for o in res.obs])
    E = np.array([r["E_mean"] for r in recs])
    print("max rel dE", np.max(np.abs(E - Eo) / np.abs(Eo)))
    assert np.allclose(E, Eo, rtol=1e-6, atol=1e-8)
    assert abs(recs[-1]["sum_lnQ"] - res.sum_lnQ) < 1e-7
    assert abs(recs[-1]["T"] - 0.5) < 1e-15 and all(r["md_ms"] > 0 for r in recs)


def test_driver_resume_equals_uninterrupted(D, tmp_path):
    full = D.run_pamd(CFG)
    ck = str(tmp_path / "ck.npz")
    first = D.run_pamd(CFG, checkpoint=ck, checkpoint_every=4, max_temps=9)
    assert first[-1]["temp_index"] == 9
    rest = D.run_pamd(CFG, checkpoint=ck, resume=True)
    # the checkpoint holds temperature 8; the resumed run redoes 9 .. 20
    assert [r["temp_index"] for r in rest] == list(range(9, 21))
    for a, b in zip(full[9:], rest):
        for k in ("T", "R", "lnQ", "sum_lnQ", "E_mean", "E_sd", "families", "V"):
            assert a[k] == b[k], (a["temp_index"], k)
