"""The tuning cache holds one entry per GPU key (architecture, HIP version, CU count):
saving adds or replaces that entry, loading returns only the matching one."""
import json

from paper_2212_05098_amd import tune


def test_cache_entries_by_key(tmp_path):
    path = str(tmp_path / "cache.json")
    a = {"key": "gfx950:sramecc+:xnack-|hip 7.0|256 CUs", "ops": {"0": [8192, 4, 0]}, "batch": [16384, 4, 2]}
    b = {"key": "gfx942|hip 6.4|304 CUs", "ops": {"0": [4096, 2, 1]}, "batch": None}
    tune.save(a, path)
    tune.save(b, path)
    assert tune.load(path, key=a["key"]) == a
    assert tune.load(path, key=b["key"]) == b
    assert tune.load(path, key="gfx000|hip 0|1 CUs") is None
    a2 = dict(a, ops={"0": [4096, 8, 2]})
    tune.save(a2, path)
    assert tune.load(path, key=a["key"]) == a2
    with open(path) as f:
        assert len(json.load(f)["entries"]) == 2


def test_old_format_is_ignored(tmp_path):
    path = str(tmp_path / "old.json")
    with open(path, "w") as f:
        json.dump({"device": "x", "ops": {"0": [8192, 4, 0]}}, f)
    assert tune.load(path, key="anything") is None
    tune.save({"key": "k", "ops": {}, "batch": None}, path)
    assert tune.load(path, key="k") == {"key": "k", "ops": {}, "batch": None}
