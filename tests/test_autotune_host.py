"""Host logic of the autotuner (no GPU): shape keys, the coordinate-descent
driver and the cache file."""

import json

from paper_2303_09855_amd import autotune as at


def test_shape_key_bands():
    assert at.shape_key(960, 0, 10, 768, 1000) == "D960_s0_K10_np512_nq512"
    assert at.shape_key(960, 0, 10, 512, 1023) == at.shape_key(960, 0, 10, 1023, 600)
    assert at.shape_key(256, 1, 100, 1, 1) == "D256_s1_K100_np1_nq1"


def test_coordinate_descent_finds_the_separable_minimum_and_skips_infeasible():
    target = {"a": 3, "b": 0.25, "c": 2}
    choices = {"a": [1, 2, 3, 4], "b": [0.125, 0.25, 0.5], "c": [1, 2, 3]}

    def cost(cfg):
        if cfg["a"] == 4:
            return None                       # violates the recall constraint
        return sum(abs(cfg[k] - target[k]) for k in cfg)

    best, best_cost, n = at.coordinate_descent(cost, {"a": 1, "b": 0.5, "c": 3}, choices)
    assert best == target and best_cost == 0
    assert n <= 1 + 2 * sum(len(v) for v in choices.values())


def test_cache_round_trip(tmp_path):
    path = tmp_path / "tune.json"
    t = at.Autotuner(str(path))
    assert t.lookup("k") is None
    t.cache["k"] = {"key": "k", "delta_d": 32, "knobs": {"dense_frac": 0.125}, "ms": 1.0,
                    "recall_vs_fds": 1.0, "evaluations": 3}
    t._write()
    again = at.Autotuner(str(path))
    assert again.lookup("k")["delta_d"] == 32
    assert json.loads(path.read_text())["k"]["ms"] == 1.0
