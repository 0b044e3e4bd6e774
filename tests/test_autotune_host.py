"""The autotuner's search and cache on the CPU: coordinate search keeps a
new value only when it beats the best by 1% (in the objective's direction),
records every trial, and the cache round-trips through save / load."""
import json

import paper_1705_06965_amd.autotune as at


def test_coordinate_search_higher_is_better():
    # objective peaks at a=3, then b=2 adds 3%
    f = lambda p: 100 - 5 * (p["a"] - 3) ** 2 + 3 * (p["b"] == 2)  # noqa: E731
    best, v, trials = at.coordinate_search(f, {"a": 1, "b": 0}, [("a", [1, 2, 3, 4]),
                                                                  ("b", [0, 1, 2])], log=lambda s: None)
    assert best == {"a": 3, "b": 2}
    assert v == f(best)
    assert [t["params"] for t in trials][0] == {"a": 1, "b": 0}
    assert len(trials) == 1 + 3 + 2   # the defaults, then every value that differs from the best


def test_coordinate_search_lower_is_better_and_none():
    # None (did not keep up) never wins; a 0.5% gain is not enough
    table = {1: 100.0, 2: None, 3: 99.6, 4: 80.0}
    best, v, trials = at.coordinate_search(lambda p: table[p["k"]], {"k": 1}, [("k", [2, 3, 4])],
                                           log=lambda s: None, lower_is_better=True)
    assert best == {"k": 4} and v == 80.0
    assert [t["value"] for t in trials] == [100.0, None, 99.6, 80.0]


def test_cache_round_trip(tmp_path, monkeypatch):
    cache = tmp_path / "tuned.json"
    monkeypatch.setattr(at, "CACHE", str(cache))
    assert at.load("kv") == at.DEFAULTS_BY["kv"]
    at.save("kv", {"params": {"grid": 8}, "trials": []})
    at.save("serve", {"params": {"grid": 32}, "trials": []})
    d = json.loads(cache.read_text())
    assert len(d) == 2
    assert at.load("kv") == dict(at.DEFAULTS_BY["kv"], grid=8)
    assert at.load("serve")["grid"] == 32 and at.load("serve")["sleep_max"] == 64
