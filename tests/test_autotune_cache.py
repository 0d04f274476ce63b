"""Host logic of the autotuner's persistent cache (no GPU)."""
import json

from paper_2406_05128_amd import autotune as at


def test_cache_roundtrip(tmp_path, monkeypatch):
    path = tmp_path / "sub" / "tune.json"
    monkeypatch.setenv("TVLP_AUTOTUNE_CACHE", str(path))
    k1 = at.cache_key("AMD Instinct MI355X", 22, 64, 48000)
    k2 = at.cache_key("AMD Instinct MI355X", 16, 4, 16000)
    assert at.lookup(k1) is None
    at.store(k1, {"chunk": 264, "chained": True, "ms": 0.9})
    at.store(k2, {"chunk": 128, "ms": 0.05})
    assert at.lookup(k1) == {"chunk": 264, "chained": True, "ms": 0.9}
    assert at.lookup(k2) == {"chunk": 128, "chained": False, "ms": 0.05}
    assert set(json.loads(path.read_text())) == {k1, k2}
    # the carry constraint and the library build are part of the key
    assert at.cache_key("d", 22, 64, 48000, "free") != at.cache_key("d", 22, 64, 48000)
    assert at.cache_key("d", 22, 64, 48000, lib="a") != at.cache_key("d", 22, 64, 48000, lib="b")
    assert at.cache_key("d", 22, 64, 48000, lib="a").endswith("|lib=a")


def test_build_id_names_the_library_file():
    from paper_2406_05128_amd import _lib
    bid = _lib.build_id()
    assert len(bid) == 16 and int(bid, 16) >= 0
    assert _lib.build_id() == bid


def test_corrupt_or_invalid_entries_are_ignored(tmp_path, monkeypatch):
    path = tmp_path / "tune.json"
    monkeypatch.setenv("TVLP_AUTOTUNE_CACHE", str(path))
    path.write_text("{not json")
    assert at.lookup("x") is None
    path.write_text(json.dumps({"x": {"chunk": -3}, "y": [1, 2]}))
    assert at.lookup("x") is None and at.lookup("y") is None
    at.store("z", {"chunk": 66, "ms": 1.0})  # rewrites a valid file
    assert at.lookup("z")["chunk"] == 66
