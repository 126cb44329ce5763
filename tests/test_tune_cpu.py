"""Autotuner bookkeeping on the host: signatures, the cache file, and the
candidate chunk lengths (all feasible, the automatic one included)."""

import json

from paper_1503_06189_amd import synth, tune, xengine


def test_signature_is_order_free_and_shape_sensitive():
    a = [(64, 1, 1024, 256), (256, 2, 4096, 256)]
    assert tune.signature(a) == tune.signature(list(reversed(a)))
    assert tune.signature(a) != tune.signature([(64, 1, 1024, 256), (256, 2, 4352, 256)])


def test_cache_roundtrip(tmp_path):
    path = str(tmp_path / "t.json")
    assert tune.load_cache(path) == {}
    tune._store("gfx950/256cu|abc", {"chunk_steps": 300, "ms": 1.0}, path)
    tune._store("gfx950/256cu|def", {"chunk_steps": 64, "ms": 2.0}, path)
    data = json.load(open(path))
    assert data["gfx950/256cu|abc"]["chunk_steps"] == 300
    assert tune.load_cache(path)["gfx950/256cu|def"]["chunk_steps"] == 64
    (tmp_path / "bad.json").write_text("{not json")
    assert tune.load_cache(str(tmp_path / "bad.json")) == {}


def test_candidates_are_feasible():
    shapes = [(s.N, 1, s.T, 256) for s in synth.batched_specs()]
    c = tune.candidates(shapes, 256)
    auto = xengine.batch_query(shapes, n_cu=256).chunk_steps
    assert auto in c and (1 << 18) in c and c == sorted(c)
    for cs in c:
        xengine.batch_query(shapes, n_cu=256, chunk_steps=cs)   # fits the workspace


def test_geometries_only_for_small_instances():
    assert tune.geometries([(64, 1, 1024, 256), (512, 1, 4096, 256)]) == ["super", "halves"]
    assert tune.geometries([(129, 1, 1024, 256), (512, 1, 4096, 256)]) == ["auto"]


def test_old_cache_entries_are_not_used(tmp_path):
    """Entries without a geometry (an older cache) do not count as hits:
    the choice returned always carries a geometry."""
    path = str(tmp_path / "t.json")
    tune._store("k", {"chunk_steps": 300, "ms": 1.0}, path)
    assert tune.load_cache(path)["k"].get("version") != tune.CACHE_VERSION
    c = tune.Choice(300, "halves")
    assert (c.chunk_steps, c.geometry) == (300, "halves")


def test_best_by_geometry_takes_each_geometrys_fastest_plan():
    from paper_1503_06189_amd import tune
    entry = {"timings_ms": {"super/256": 1.5, "super/512": 1.2, "halves/256": 1.3,
                            "halves/512": 1.4}}
    assert tune.best_by_geometry(entry) == {"super": 1.2, "halves": 1.3}
    assert tune.best_by_geometry({}) == {}
