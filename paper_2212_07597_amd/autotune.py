"""Autotuner of the sampler's launch parameters (``Sampler.set_tuning``).

The parameters trade work between the passes without changing any result:
whether long traces get tile maps before the resolve pass
(``tile_map_tiles``: the library default, or never, for workloads whose tiles
never qualify and would only pay for the check), how many distinct chains
the summary pass follows through a segment before it leaves the segment to
be followed from its actual entry (``chain_cap``), and the grid sizes of the
two grid-stride passes over the records (``chain_grid``, ``emit_grid``).  For one workload (a callable that submits
a batch to the sampler and runs it), the tuner times candidates on the GPU
one parameter at a time, keeps the fastest, and caches the choice in a JSON
file keyed by (GPU architecture, compute-unit count, size class), so a later
process with the same key skips the search.

The timing is the sampler's own: the HIP events around the five sampling
passes of the last run (``Sampler.last_timing``), the median of ``reps``
runs per candidate.
"""
from __future__ import annotations

import json
import math
import os
import statistics

DEFAULT = {"chain_cap": 16, "chain_grid": 0, "emit_grid": 0, "graphs": 1, "tile_map_tiles": 0}
CHAIN_CAPS = (4, 8, 16, 32, 64)
TILE_MAPS_NEVER = 0xFFFFFFFF
GRID_FACTORS = (0.5, 1, 2)


def default_cache_path():
    base = os.environ.get("XDG_CACHE_HOME") or os.path.join(os.path.expanduser("~"), ".cache")
    return os.environ.get("SMP_TUNING_CACHE") or os.path.join(base, "scalene_sampler", "tuning.json")


def size_class(n_traces, total_events):
    """Bucket of a batch: traces and mean events per trace, each to the
    nearest power of four (single traces: t0)."""
    n_traces = max(int(n_traces), 1)
    mean = max(total_events / n_traces, 1.0)
    return f"t{round(math.log(n_traces, 4))}-e{round(math.log(mean, 4))}"


def device_key(device=0):
    import torch

    p = torch.cuda.get_device_properties(device)
    return f"{getattr(p, 'gcnArchName', p.name)}/cu{p.multi_processor_count}"


def load_cache(path):
    try:
        with open(path) as f:
            data = json.load(f)
        return data if isinstance(data, dict) else {}
    except (OSError, ValueError):
        return {}


def save_cache(path, data):
    os.makedirs(os.path.dirname(path) or ".", exist_ok=True)
    tmp = path + ".tmp"
    with open(tmp, "w") as f:
        json.dump(data, f, indent=1, sort_keys=True)
    os.replace(tmp, path)


def measure(sampler, workload, tuning, reps):
    """Median kernel milliseconds of the five sampling passes over reps runs
    of workload() under tuning (one untimed run first), launched plainly so
    that every run records its own timing events."""
    sampler.set_tuning(**{**tuning, "graphs": 0})
    workload()
    times = []
    for _ in range(reps):
        workload()
        times.append(sampler.last_timing()[0])
    return statistics.median(times)


def candidates(param, defaults):
    """Values tried for one parameter; grids are factors of the device's
    default (as many workgroups as it holds at once)."""
    if param == "chain_cap":
        return list(CHAIN_CAPS)
    if param == "tile_map_tiles":
        return [0, TILE_MAPS_NEVER]
    base = defaults[param]
    return sorted({max(1, int(round(base * f))) for f in GRID_FACTORS})


def tune(sampler, workload, size, *, cache_path=None, reps=3, key=None, log=None):
    """Tune the sampler's launch parameters for workload (a callable running
    one batch through ``sampler``), or take them from the cache.  Leaves the
    chosen tuning set on the sampler and returns
    {"key", "tuning", "ms", "tried", "from_cache"}."""
    path = cache_path or default_cache_path()
    key = key or f"{device_key()}/{size}"
    cache = load_cache(path)
    hit = cache.get(key)
    if hit and isinstance(hit.get("tuning"), dict):
        sampler.set_tuning(**{**DEFAULT, **hit["tuning"]})
        return {"key": key, "tuning": hit["tuning"], "ms": hit.get("ms"), "tried": hit.get("tried", {}),
                "from_cache": True}
    sampler.set_tuning(**DEFAULT)
    resolved = sampler.get_tuning()  # the device defaults of the grids
    best = dict(DEFAULT)
    tried = {}

    def name(t):
        return ",".join(f"{k}={t[k]}" for k in ("tile_map_tiles", "chain_cap", "chain_grid", "emit_grid"))

    best_ms = measure(sampler, workload, best, reps)
    tried[name(best)] = round(best_ms, 4)
    for param in ("tile_map_tiles", "chain_cap", "emit_grid", "chain_grid"):
        for v in candidates(param, resolved):
            cand = dict(best)
            cand[param] = v
            if param in ("chain_grid", "emit_grid") and v == resolved[param]:
                cand[param] = 0  # the default itself
            if name(cand) in tried:
                continue
            ms = measure(sampler, workload, cand, reps)
            tried[name(cand)] = round(ms, 4)
            if log:
                log(f"  tune {name(cand)}: {ms:.4f} ms")
            if ms < best_ms:
                best, best_ms = cand, ms
    sampler.set_tuning(**best)
    cache[key] = {"tuning": best, "ms": round(best_ms, 4), "tried": tried}
    save_cache(path, cache)
    return {"key": key, "tuning": best, "ms": round(best_ms, 4), "tried": tried, "from_cache": False}
