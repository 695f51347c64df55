"""CPU check of the batched autotuner's search logic (the GPU context and its
timing replaced by a scripted stand-in): which candidates it times, that a
register-tile split is refined over the register-tile launch shape, and that
the fastest candidate is returned."""
import pytest

torch = pytest.importorskip("torch")

from paper_1806_06016_amd import autotune as A  # noqa: E402


class _Sys:
    def __init__(self, n):
        self.n_atoms = n


def _run(monkeypatch, rate):
    """rate(layout tuple, wide waves, tile waves) -> replica-steps/s of a candidate."""
    made = []

    class FakePamd:
        def __init__(self, systems, **kw):
            self.shape = (tuple(kw["layout"]), kw["wide_waves"], kw["waves_per_block"])
            made.append(self.shape)

        def close(self):
            pass

    def fake_time(p, theta):
        return 1e3 * 4 * 512 * theta / rate(*p.shape)   # ms for 4 runs x 512 replicas

    monkeypatch.setattr(A, "Pamd", FakePamd)
    monkeypatch.setattr(A, "_time_md", fake_time)
    monkeypatch.setattr(A, "_key", lambda *a, **k: "cpu-test")
    monkeypatch.setattr(torch.cuda, "synchronize", lambda *a, **k: None)
    systems = [_Sys(40), _Sys(75), _Sys(120), _Sys(300)]
    return A.autotune_batched(systems, 512, theta_probe=10, use_cache=False), made


def test_tile_split_is_refined_over_tile_waves(monkeypatch):
    def rate(lay, w, tw):
        base = 2e7 if lay[0] == "tile" else 1e7
        return base * (1.0 + 0.01 * w) * (1.5 if tw == 4 else 1.0)

    t, made = _run(monkeypatch, rate)
    first = {f"{l}/w{w}" for l in ("wide", "tile_small") for w in A.WIDE_CANDIDATES}
    assert set(t["timings"]) == first | {f"tile_small/w4/t{tw}" for tw in A.TILE_SMALL_CANDIDATES}
    assert t["choice"] == "tile_small/w4/t4"
    assert t["layout"] == ["tile", "tile", "wide", "wide"]
    assert (t["wide_waves_per_block"], t["waves_per_block"]) == (4, 4)
    assert len(made) == len(t["timings"])


def test_all_wide_wins_without_refinement(monkeypatch):
    def rate(lay, w, tw):
        return (3e7 if lay[0] == "wide" else 1e7) * (1.0 + 0.01 * (5 - w))

    t, _ = _run(monkeypatch, rate)
    assert set(t["timings"]) == {f"{l}/w{w}" for l in ("wide", "tile_small") for w in A.WIDE_CANDIDATES}
    assert t["choice"] == "wide/w1"
    assert t["layout"] == ["wide"] * 4 and t["waves_per_block"] == 0


def test_all_small_molecules_compare_all_tile_with_all_wide(monkeypatch):
    """Runs that all fit the register tile: all-wide (each wide launch shape)
    against all register-tile launches, which wins here and is refined."""
    def rate(lay, w, tw):
        return (3e7 if lay[0] == "tile" else 1e7) * (1.1 if tw == 8 else 1.0)

    made = []

    class FakePamd:
        def __init__(self, systems, **kw):
            self.shape = (tuple(kw["layout"]), kw["wide_waves"], kw["waves_per_block"])
            made.append(self.shape)

        def close(self):
            pass

    monkeypatch.setattr(A, "Pamd", FakePamd)
    monkeypatch.setattr(A, "_time_md", lambda p, theta: 1e3 * 2 * 512 * theta / rate(*p.shape))
    monkeypatch.setattr(A, "_key", lambda *a, **k: "cpu-test")
    monkeypatch.setattr(torch.cuda, "synchronize", lambda *a, **k: None)
    t = A.autotune_batched([_Sys(40), _Sys(75)], 512, theta_probe=10, use_cache=False)
    assert set(t["timings"]) == ({f"wide/w{w}" for w in A.WIDE_CANDIDATES} | {"tile_small/w0"}
                                 | {f"tile_small/w0/t{tw}" for tw in A.TILE_SMALL_CANDIDATES})
    assert t["choice"] == "tile_small/w0/t8"
    assert t["layout"] == ["tile", "tile"] and t["waves_per_block"] == 8
