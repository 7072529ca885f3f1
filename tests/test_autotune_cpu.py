"""Host logic of the schedule autotuner: the knob grid, the cache key, the
cache lookup and the coordinate descent (with the GPU timing replaced by a
cost function, so no kernel runs)."""

import json

import numpy as np
import pytest

from paper_1802_06952_amd import autotune as at


def test_knob_grid_defaults_first():
    v = at.knob_values(14, 0, 1 << 14, [6, 7])
    assert v["tile_bits"][0] == 10 and set(v["tile_bits"]) == {9, 10, 11}
    assert v["max_stages"] == [2, 1]
    assert v["copies_per_launch"] == [0, (1 << 14) // 4]
    # the model's depth (-1) first, then one level either side of each side's choice
    assert v["materialize_level"][0] == -1
    assert sorted(v["materialize_level"][1:]) == [5, 6, 7, 8]
    assert v["tail_max_qubits"] == [10, 8]
    assert v["no_exchange"] == [0, 1]


def test_knob_grid_span_not_power_of_two():
    v = at.knob_values(3, 1, 6, [0])
    assert v["copies_per_launch"] == [0]
    assert v["materialize_level"] == [-1, 1]


def test_key_depends_on_every_input():
    bits = np.arange(8, dtype=np.uint64)
    k = at.workload_key("c", 3, bits, 0, 4)
    assert k == at.workload_key("c", 3, bits.copy(), 0, 4)
    assert len({k, at.workload_key("d", 3, bits, 0, 4), at.workload_key("c", 5, bits, 0, 4),
                at.workload_key("c", 3, bits[::-1].copy(), 0, 4),
                at.workload_key("c", 3, bits, 0, 2)}) == 5


def test_cache_used_only_when_key_matches(tmp_path):
    p = tmp_path / "tuned.json"
    p.write_text(json.dumps({"workloads": {"w": {"key": "abc", "opts": {"tile_bits": 9}}}}))
    assert at.tuned_opts("w", "abc", str(p)) == {"tile_bits": 9}
    assert at.tuned_opts("w", "abd", str(p)) is None
    assert at.tuned_opts("other", "abc", str(p)) is None
    assert at.tuned_opts("w", "abc", str(tmp_path / "missing.json")) is None


def test_committed_cache_is_well_formed():
    store = at.load_tuned()
    for name, e in store.items():
        assert len(e["key"]) == 24
        assert set(e["opts"]) <= {"tile_bits", "max_stages", "copies_per_launch",
                                  "materialize_level", "tail_max_qubits", "no_exchange"}
        assert e["ms"] <= e["default_ms"] + 1e-9


class _FakePlan:
    n_cuts = 4

    def __init__(self, *a, **k):
        pass

    def dump(self, k0, k1):
        return {"sides": [{"lstar": 3}, {"lstar": 2}]}

    def close(self):
        pass


def test_coordinate_descent_finds_separable_minimum(monkeypatch):
    """With a cost that is a sum of per-knob terms, one sweep of coordinate
    descent reaches the global minimum of the grid."""
    best = {"tile_bits": 9, "max_stages": 1, "copies_per_launch": 0,
            "materialize_level": 4, "tail_max_qubits": 8, "no_exchange": 1}

    def cost(text, mask, bits, k0, k1, opts, reps, stream):
        return 1.0 + sum(0.1 * (opts[k] != v) for k, v in best.items())

    monkeypatch.setattr(at, "Plan", _FakePlan)
    monkeypatch.setattr(at, "time_opts", cost)
    r = at.autotune("c", 1, np.zeros(4, dtype=np.uint64), 0, 16)
    assert r["opts"] == best
    assert r["ms"] == pytest.approx(1000.0)
    assert r["default_ms"] == pytest.approx(1000.0 + 500.0)
    # every tried set is recorded once, the default first
    assert r["tried"][0]["opts"] == {"tile_bits": 10, "max_stages": 2, "copies_per_launch": 0,
                                     "materialize_level": -1, "tail_max_qubits": 10,
                                     "no_exchange": 0}
    assert len({json.dumps(t["opts"], sort_keys=True) for t in r["tried"]}) == len(r["tried"])


def test_rejected_knob_sets_are_skipped(monkeypatch):
    def cost(text, mask, bits, k0, k1, opts, reps, stream):
        if opts["tile_bits"] == 11:
            raise at.QSError(1, "tile too wide")
        return 2.0 - 0.5 * (opts["tile_bits"] == 9)

    monkeypatch.setattr(at, "Plan", _FakePlan)
    monkeypatch.setattr(at, "time_opts", cost)
    r = at.autotune("c", 1, np.zeros(4, dtype=np.uint64), 0, 16)
    assert r["opts"]["tile_bits"] == 9
    assert any(t["ms"] is None for t in r["tried"])
