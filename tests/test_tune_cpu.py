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


def test_candidates_cover_the_shape_ranges():
    """The batch tuner tries 1-16 points per thread and 64-1024 threads per
    workgroup (per-view passes, tiles of at most 4096 points) and groups of
    2-32 views in the grouped passes (one-wavefront workgroups)."""
    from paper_2104_07526_amd import tune
    per_view = [c for c in tune.BATCH_CANDIDATES if c["group"] == 1]
    assert {c["ppt"] for c in per_view} == {1, 2, 4, 8, 16}
    assert {c["wg"] for c in per_view} == {64, 256, 1024}
    assert all(c["ppt"] * c["wg"] <= 4096 for c in per_view)
    batched = [c for c in tune.BATCH_CANDIDATES if c["group"] != 1]
    assert {c["group"] for c in batched} == {2, 4, 8, 16, 32}
    assert all(c["wg"] == 64 for c in batched)
