"""The autotuner's cache on the host (no GPU): keys separate architectures
and workload shapes, and a stored choice survives a fresh process (the JSON
file) while an unreadable or partial record is ignored."""
import json

from paper_2506_00225_amd import autotune


def test_shape_key_separates_arch_and_shape():
    a = autotune.shape_key("gfx950", "score", 500000, 102, 16, [(480, 640), (120, 160)])
    assert a == "gfx950|score|n=500000|C=102|k=16|views=480x640,120x160"
    assert a != autotune.shape_key("gfx942", "score", 500000, 102, 16, [(480, 640), (120, 160)])
    assert a != autotune.shape_key("gfx950", "score", 500000, 102, 16, [(120, 160), (480, 640)])
    assert a != autotune.shape_key("gfx950", "mapping", 500000, 102, 16, [(480, 640), (120, 160)])


def test_store_and_load_through_the_json_file(tmp_path):
    path = str(tmp_path / "sub" / "autotune.json")
    autotune.clear_cache()
    knobs = (1, 2, 2048, 1, 32, 8)
    autotune.store("k1", knobs, ms=1.23456, path=path)
    autotune.store("k2", (2, 1, 0, 0, 44, 6), path=path)
    autotune.clear_cache()  # as a fresh process would start
    assert autotune.load_cached("k1", path=path) == knobs
    data = json.load(open(path))
    assert data["k1"]["ms"] == 1.2346 and data["k1"]["bwd_batch"] == 32 and set(data) == {"k1", "k2"}
    assert autotune.load_cached("missing", path=path) is None


def test_partial_or_broken_records_are_ignored(tmp_path):
    path = str(tmp_path / "autotune.json")
    json.dump({"old": {"sem_accumulators": 1, "tile_order": 1}}, open(path, "w"))
    autotune.clear_cache()
    assert autotune.load_cached("old", path=path) is None
    open(path, "w").write("{not json")
    assert autotune.load_cached("old", path=path) is None
    autotune.store("new", (0, 0, 0, 0, 0, 0), path=path)  # a broken file is not replaced: memory only
    assert autotune.load_cached("new", path=path) == (0, 0, 0, 0, 0, 0)


def test_empty_cache_path_means_memory_only(monkeypatch):
    monkeypatch.setenv("SGR_AUTOTUNE_CACHE", "")
    assert autotune.cache_path() is None
