"""Host logic of the launch-parameter autotuner (no GPU): the search finds
the fastest candidate of a synthetic cost, the cache stores it under its key
and a second call takes it from there without running anything."""
import os

from paper_2212_07597_amd import autotune


class FakeSampler:
    """Stands in for Sampler: the 'kernel time' of a run is a function of
    the tuning, smallest at chain_cap 8, an emit grid of 2x the default and
    tile maps off."""

    DEFAULT_GRID = 1024

    def __init__(self):
        self.t = dict(autotune.DEFAULT)
        self.runs = 0

    def set_tuning(self, chain_cap=16, chain_grid=0, emit_grid=0, graphs=1, tile_map_tiles=0):
        assert 1 <= chain_cap <= 64
        self.t = dict(chain_cap=chain_cap, chain_grid=chain_grid, emit_grid=emit_grid, graphs=graphs,
                      tile_map_tiles=tile_map_tiles)

    def get_tuning(self):
        t = dict(self.t)
        t["chain_grid"] = t["chain_grid"] or self.DEFAULT_GRID
        t["emit_grid"] = t["emit_grid"] or self.DEFAULT_GRID
        return t

    def last_timing(self):
        t = self.get_tuning()
        ms = 1.0 + abs(t["chain_cap"] - 8) / 100 + abs(t["emit_grid"] - 2048) / 1e4 + abs(t["chain_grid"] - 1024) / 1e5
        ms += 0.01 if t["tile_map_tiles"] != autotune.TILE_MAPS_NEVER else 0.0
        return ms, ms + 0.1


def test_search_finds_the_fastest_and_caches_it(tmp_path):
    s = FakeSampler()
    calls = []

    def workload():
        calls.append(1)

    path = os.path.join(tmp_path, "tuning.json")
    r = autotune.tune(s, workload, "t0-e13", cache_path=path, reps=2, key="gfx950/cu256/t0-e13")
    assert not r["from_cache"]
    assert r["tuning"]["chain_cap"] == 8 and r["tuning"]["emit_grid"] == 2048 and r["tuning"]["chain_grid"] == 0
    assert r["tuning"]["tile_map_tiles"] == autotune.TILE_MAPS_NEVER
    assert s.t == r["tuning"] and s.t["graphs"] == 1
    assert len(calls) == 3 * len(r["tried"])  # one untimed run and reps timed ones per candidate
    # a second process with the same key: no runs, the same choice
    s2 = FakeSampler()
    calls.clear()
    r2 = autotune.tune(s2, workload, "t0-e13", cache_path=path, reps=2, key="gfx950/cu256/t0-e13")
    assert r2["from_cache"] and r2["tuning"] == r["tuning"] and not calls and s2.t == r["tuning"]
    # another key searches again
    r3 = autotune.tune(FakeSampler(), workload, "t5-e8", cache_path=path, reps=1, key="gfx950/cu256/t5-e8")
    assert not r3["from_cache"]
    assert set(autotune.load_cache(path)) == {"gfx950/cu256/t0-e13", "gfx950/cu256/t5-e8"}


def test_size_classes():
    assert autotune.size_class(1, 1e8) == "t0-e13"
    assert autotune.size_class(1024, 1.5e8) == "t5-e9"
    assert autotune.size_class(1, 5e8) == "t0-e14"
    assert autotune.size_class(0, 0) == "t0-e0"


def test_unreadable_cache_is_empty(tmp_path):
    p = os.path.join(tmp_path, "bad.json")
    open(p, "w").write("{not json")
    assert autotune.load_cache(p) == {}
    assert autotune.load_cache(os.path.join(tmp_path, "missing.json")) == {}
