"""Autotuner bookkeeping on the CPU (cache keys and persistence)."""
import importlib
import json


def test_cache_roundtrip(tmp_path, monkeypatch):
    monkeypatch.setenv("PCR_TUNE_CACHE", str(tmp_path / "t.json"))
    from paper_2104_07526_amd import tune
    tune = importlib.reload(tune)
    k = tune._key("batch", 145_000_000, "v64")
    assert "n~2^27" in k
    tune._store(k, {"tune": {"ppt": 8}, "table": [[1.0, {"ppt": 8}]]})
    assert json.load(open(tmp_path / "t.json"))[k]["tune"] == {"ppt": 8}
    assert tune._load()[k]["table"][0][0] == 1.0
