"""CPU checks of the annealing driver's host logic: configuration checks,
the geometric schedule, the shipped configurations."""
import glob
import os

import numpy as np
import pytest

from paper_1806_06016_amd import driver as D
from pamd_inputs import systems as S

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CONFIGS = sorted(glob.glob(os.path.join(ROOT, "paper_1806_06016_amd", "configs", "*.json")))


def _base():
    return D.load_config(os.path.join(ROOT, "paper_1806_06016_amd", "configs", "bead_chain10_R256.json"))


def test_shipped_configurations_load():
    assert len(CONFIGS) >= 4
    for f in CONFIGS:
        cfg = D.load_config(f)
        assert cfg["precision"] in ("fp32", "fp64")


def test_geometric_schedule_is_the_generators():
    cfg = _base()
    T = D.temperatures(cfg)
    ref = S.geometric_schedule(2.0, 0.5, 20)
    assert len(T) == 21 and T[0] == 2.0
    assert np.allclose(T, ref, rtol=1e-15, atol=0)
    assert abs(T[-1] - 0.5) < 1e-15


@pytest.mark.parametrize("patch", [
    {"R": 0}, {"theta": 0}, {"precision": "fp16"}, {"systems": []}, {"systems": [{"kind": "water"}]},
    {"schedule": {"kind": "geometric", "T_final": 3.0, "steps": 20}},
    {"schedule": {"kind": "geometric", "T_final": 0.5, "steps": 0}},
    {"schedule": {"kind": "adaptive", "T_final": 0.5, "V_target": 0.0}},
    {"schedule": {"kind": "linear", "T_final": 0.5}},
])
def test_bad_configurations_are_rejected(patch):
    cfg = dict(_base(), **patch)
    with pytest.raises(ValueError):
        D.load_config(cfg)


def test_missing_keys_are_named():
    cfg = _base()
    del cfg["theta"]
    with pytest.raises(ValueError, match="theta"):
        D.load_config(cfg)
