"""The autotuner's JSON cache (host logic only)."""
import json

from paper_0909_4039_amd import tune_cache


def test_round_trip_and_keys(tmp_path, monkeypatch):
    path = str(tmp_path / "tune.json")
    k1 = tune_cache.key("AMD Instinct MI355X", 64, (1024, 32768), "step")
    k2 = tune_cache.key("AMD Instinct MI355X", 32, (1024, 32768), "step")
    assert k1 != k2 and "1024x32768" in k1
    assert tune_cache.lookup(path, k1) is None
    tune_cache.store(path, k1, (96, 2))
    tune_cache.store(path, k2, (64, 2))
    assert tune_cache.lookup(path, k1) == [96, 2]
    assert tune_cache.lookup(path, k2) == [64, 2]
    assert json.load(open(path))[k1] == [96, 2]
    # no path: nothing is cached
    monkeypatch.delenv(tune_cache.ENV, raising=False)
    assert tune_cache.cache_path(None) is None
    tune_cache.store(None, k1, (1, 1))
    monkeypatch.setenv(tune_cache.ENV, path)
    assert tune_cache.cache_path(None) == path


def test_unreadable_cache_is_ignored(tmp_path):
    path = tmp_path / "tune.json"
    path.write_text("{not json")
    k = tune_cache.key("gpu", 64, (8, 8), "step")
    assert tune_cache.lookup(str(path), k) is None
    tune_cache.store(str(path), k, (4, 1))          # rewritten whole
    assert tune_cache.lookup(str(path), k) == [4, 1]
