"""Host logic of the persisted autotuner choices (no GPU)."""

import json


def test_cache_round_trip_and_keys(tmp_path, monkeypatch):
    from paper_1211_0126_amd import tuning_cache as tc
    path = str(tmp_path / "sub" / "tune.json")
    monkeypatch.setenv("TMQCD_TUNE_CACHE", path)
    assert tc.cache_path() == path
    assert tc.load() == {}
    k1 = tc.key("MI355X", (32, 32, 32, 64), 0.1632, 0.003, 2, 2, 16)
    k2 = tc.key("MI355X", (32, 32, 32, 64), 0.1632, 0.003, 2, 2, 32)
    k3 = tc.key("MI355X", (24, 24, 24, 48), 0.1632, 0.003, 2, 2, 16)
    assert len({k1, k2, k3}) == 3
    tc.save({k1: {"lane_rhs": 2, "tiles": 0}})
    tc.save(dict(tc.load(), **{k2: {"lane_rhs": 4, "tiles": 1}}))
    d = json.load(open(path))
    assert d[k1]["lane_rhs"] == 2 and d[k2]["tiles"] == 1


def test_corrupt_cache_reads_empty(tmp_path):
    from paper_1211_0126_amd import tuning_cache as tc
    p = tmp_path / "bad.json"
    p.write_text("{not json")
    assert tc.load(str(p)) == {}
    p.write_text("[1, 2]")
    assert tc.load(str(p)) == {}
