"""CPU checks of the checkpoint file format and of restore's validation (the
resumed-run equality test runs on the GPU)."""
import numpy as np
import pytest

from paper_1806_06016_amd import checkpoint as CK
from paper_1806_06016_amd.pamd import PAMD_FP32, PAMD_FP64


def _state(R, n, seed):
    rng = np.random.default_rng(seed)
    return dict(R=R, T=612.5 + seed, T_prev=630.25, sum_lnQ=-17.125 * seed, lnQ_last=-0.5, step=1234 + seed,
                temp_index=7, x=rng.normal(size=(R, n, 3)), v=rng.normal(size=(R, n, 3)),
                E_pot=rng.normal(size=R), E_kin=rng.normal(size=R), ancestor=rng.integers(0, 10 ** 6, R).astype(np.int32))


class _Ctx:
    """Stands in for a Pamd context: the attributes restore reads and a
    recording set_state."""

    def __init__(self, n_atoms, R_cap, fp32, states=None):
        self.n_atoms, self.R_cap, self.fp32 = list(n_atoms), R_cap, fp32
        self.states = states or []
        self.calls = []

    def get_state(self, run):
        return self.states[run]

    def set_state(self, run, x, v, **kw):
        self.calls.append((run, x, v, kw))


def test_round_trip_is_exact(tmp_path):
    states = [_state(37, 75, 1), _state(5, 12, 2)]
    path = str(tmp_path / "ck.npz")
    CK.save(_Ctx([75, 12], 100, True, states), path)
    ck = CK.read(path)
    assert ck["precision"] == PAMD_FP32 and len(ck["runs"]) == 2
    for a, b in zip(states, ck["runs"]):
        for k in ("x", "v", "E_pot", "ancestor"):
            assert np.array_equal(a[k], b[k]) and b[k].dtype == (np.int32 if k == "ancestor" else np.float64)
        for k in ("R", "T", "T_prev", "sum_lnQ", "lnQ_last", "step", "temp_index"):
            assert a[k] == b[k]


def test_restore_passes_every_field(tmp_path):
    st = _state(9, 20, 3)
    path = str(tmp_path / "ck.npz")
    CK.write(path, [st], PAMD_FP64)
    ctx = _Ctx([20], 16, False)
    CK.restore(ctx, path)
    (run, x, v, kw), = ctx.calls
    assert run == 0 and np.array_equal(x, st["x"]) and np.array_equal(v, st["v"])
    assert np.array_equal(kw["E_pot"], st["E_pot"]) and np.array_equal(kw["ancestor"], st["ancestor"])
    for k in ("T", "T_prev", "sum_lnQ", "lnQ_last", "step", "temp_index"):
        assert kw[k] == st[k], k


@pytest.mark.parametrize("ctx,msg", [(_Ctx([20], 16, True), "precision"), (_Ctx([20, 20], 16, False), "runs"),
                                     (_Ctx([21], 16, False), "atoms"), (_Ctx([20], 8, False), "R_cap")])
def test_restore_rejects_a_different_context(tmp_path, ctx, msg):
    path = str(tmp_path / "ck.npz")
    CK.write(path, [_state(9, 20, 4)], PAMD_FP64)
    with pytest.raises(ValueError, match=msg):
        CK.restore(ctx, path)
    assert not ctx.calls


def test_inconsistent_state_is_not_written(tmp_path):
    st = _state(9, 20, 5)
    st["E_pot"] = st["E_pot"][:8]
    with pytest.raises(ValueError):
        CK.write(str(tmp_path / "ck.npz"), [st], PAMD_FP32)
