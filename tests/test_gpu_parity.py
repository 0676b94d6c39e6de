"""GPU parity: the HIP path (through the C ABI) against the CPU oracle.

Everything the method computes is integer, so every comparison is exact:
sample records, tracked objects, the twelve per-line arrays, scalars, leak
rationals and gates.
"""
import json
import os
import sys

import numpy as np
import pytest

import oracle
import paper_2212_07597_amd as smp
import tracegen as tg
from parity_util import compare

pytestmark = pytest.mark.gpu

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def sampler():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    s = smp.Sampler(workspace=48 << 30)
    yield s
    s.close()
    del s
    torch.cuda.empty_cache()


def run_batch(sampler, cases):
    """cases: list of (label, events, kwargs).  One run() for all of them."""
    ids = []
    for label, ev, kw in cases:
        p = smp.make_params(kw["threshold"], kw["num_lines"], kw.get("copy_threshold"),
                            kw.get("quantum_us", 10_000), kw.get("options", 0))
        ids.append(sampler.submit_trace(ev, p))
    say(f"  run of {len(cases)} traces")
    sampler.run(blocking=True)
    return [sampler.fetch_profile(i) for i in ids]


def check_batch(sampler, cases):
    outs = run_batch(sampler, cases)
    for (label, ev, kw), g in zip(cases, outs):
        o = oracle.run(ev, **kw)
        compare(g, o, label)


def test_golden_fixtures(sampler):
    say("golden fixtures")
    cases = []
    expects = []
    for name in sorted(os.listdir(GOLDEN)):
        if not (name.startswith("W") and name.endswith(".json")):  # the threshold sampler's fixtures
            continue
        d = json.load(open(os.path.join(GOLDEN, name)))
        for k, c in enumerate(d.get("cases", [d])):
            ev = tg.make_events([tuple(r) for r in c["events"]])
            p = c["params"]
            kw = dict(threshold=p["threshold"], num_lines=p["num_lines"], copy_threshold=p.get("copy_threshold"),
                      quantum_us=p.get("quantum_us", 10_000), options=p.get("options", 0))
            cases.append((f"{d['id']}.{k}", ev, kw))
            expects.append(c["expect"])
    outs = run_batch(sampler, cases)
    for (label, ev, kw), g, exp in zip(cases, outs, expects):
        got = [[int(x["event_idx"]), int(x["line"]), int(x["F"]), int(x["py"]), int(x["nat"])] for x in g["samples"]]
        assert got == exp["samples"], label
        for key in ("final_F", "peak_F", "peak_sampled_F"):
            if key in exp:
                assert g[key] == exp[key], (label, key)
        compare(g, oracle.run(ev, **kw), label)


def tiny_trace(rng, n, kinds=True):
    rows = []
    for i in range(n):
        kind = 0
        if kinds and rng.random() < 0.15:
            kind = 1 if rng.random() < 0.5 else 2
        if kind == 0:
            d = int(rng.integers(-40, 41))
        else:
            d = int(rng.integers(0, 30))
        rows.append((d, int(rng.integers(1, 12)), int(rng.integers(0, 5)), int(rng.integers(0, 2)), kind))
    return tg.make_events(rows)


def test_tiny_random_batch(sampler):
    say("tiny random traces, one batch")
    rng = np.random.default_rng(99)
    cases = []
    for i in range(300):
        n = int(rng.integers(0, 50))
        T = int(rng.integers(1, 60))
        opts = int(rng.integers(0, 4))
        cases.append((f"tiny{i}", tiny_trace(rng, n), dict(threshold=T, num_lines=5,
                                                           copy_threshold=int(rng.integers(1, 20)), options=opts)))
    check_batch(sampler, cases)


@pytest.mark.parametrize("n", [1, 63, 64, 65, 511, 512, 513, 1023, 1025, 4096 + 17])
def test_segment_boundaries(sampler, n):
    say(f"segment boundary n={n}")
    rng = np.random.default_rng(n)
    ev = tiny_trace(rng, n)
    cases = [(f"b{n}T{T}", ev, dict(threshold=T, num_lines=5)) for T in (1, 5, 30, 100, 1000)]
    check_batch(sampler, cases)


def random_trace(rng, n):
    """tiny_trace's distribution, drawn with numpy (for long traces)."""
    ev = np.zeros(n, dtype=tg.EVENT_DTYPE)
    kind = np.where(rng.random(n) < 0.15, rng.integers(1, 3, n), 0)
    ev["delta"] = np.where(kind == 0, rng.integers(-40, 41, n), rng.integers(0, 30, n))
    ev["ptr"] = rng.integers(1, 12, n)
    ev["line"] = rng.integers(0, 5, n)
    ev["flags"] = rng.integers(0, 2, n) | (kind << 1)
    return ev


@pytest.mark.parametrize("n", [512 * 512 - 1, 512 * 512, 512 * 512 + 1, 2 * 512 * 512 + 3])
def test_tile_boundaries(sampler, n):
    """Traces ending just before, at and just after a tile boundary (512
    segments of 512 events), with thresholds that leave the tiles dense
    (many stops) and sparse (T far above what a segment moves, with a few
    samples per tile or none)."""
    say(f"tile boundary n={n}")
    ev = random_trace(np.random.default_rng(n), n)
    cases = [(f"t{n}T{T}", ev, dict(threshold=T, num_lines=5)) for T in (30, 1000, 3000, 200_000)]
    check_batch(sampler, cases)


def test_config1_mix(sampler):
    say("config-1 mix: seeds x thresholds")
    cases = []
    for seed in (1, 2, 3):
        ev, _ = tg.config1(seed=seed)
        for T in (256 * tg.KiB, tg.MiB, 10 * tg.MiB, 3 * tg.MiB + 1):
            cases.append((f"c1 s{seed} T{T}", ev, dict(threshold=T, num_lines=64)))
    check_batch(sampler, cases)


def adversarial_cases():
    out = []
    n = 20_000
    mono = tg.make_events([(1, i + 1, i % 3, 0) for i in range(n)])
    for T in (1, 7, 1000, n - 1, n, n + 1, 10 ** 9):
        out.append((f"mono T{T}", mono, dict(threshold=T, num_lines=3)))
    zeros = tg.make_events([(0, i + 1, 0, 0) for i in range(3000)])
    out.append(("zeros", zeros, dict(threshold=1, num_lines=1)))
    alt = tg.make_events([((-1) ** i * 50, i + 1, i % 2, i % 2) for i in range(5000)])
    for T in (49, 50, 51, 100):
        out.append((f"alt T{T}", alt, dict(threshold=T, num_lines=2)))
    # forced events every 37 events in a drift of small steps
    rows = []
    for i in range(30_000):
        d = 10_000 if i % 37 == 0 else (3 if i % 2 else -2)
        if i % 74 == 0:
            d = -10_000
        rows.append((d, i + 1, i % 11, i % 2))
    forced = tg.make_events(rows)
    for T in (1000, 4000, 5001, 9000):
        out.append((f"forced T{T}", forced, dict(threshold=T, num_lines=11)))
    # slow drift with rare samples (segments that never collapse)
    rng = np.random.default_rng(5)
    steps = rng.integers(-100, 130, 50_000)
    drift = tg.make_events([(int(d), i + 1, i % 7, int(d) & 1) for i, d in enumerate(steps)])
    for T in (5_000, 40_000, 200_000):
        out.append((f"drift T{T}", drift, dict(threshold=T, num_lines=7)))
    # leak heavy: free every tracked allocation right after it is sampled
    rows = []
    pid = 1
    for i in range(10_000):
        rows.append((100, pid, i % 5, 0))
        if i % 3 == 0:
            rows.append((-100, pid, (i + 1) % 5, 0))
        pid += 1
    leak = tg.make_events(rows)
    for T in (100, 250, 1000):
        for opt in (0, smp.OPT_RESOLVE_AT_END):
            out.append((f"leak T{T} o{opt}", leak, dict(threshold=T, num_lines=5, options=opt)))
    # prime threshold option
    ev, _ = tg.config1(seed=4, n=30_000)
    out.append(("prime", ev, dict(threshold=tg.MiB, num_lines=64, options=smp.OPT_PRIME_T)))
    return out


def test_adversarial(sampler):
    say("adversarial traces")
    check_batch(sampler, adversarial_cases())


def multi_tile_cases():
    """Traces spanning several tiles of 512 segments (262,144 events each) whose
    segment maps are rarely or never total, so that chain states travel
    serially across waves and tiles, and segments whose chains do not all
    coincide have to be followed from their actual entry."""
    out = []
    n = 3 * 1024 * 512 + 777
    mono = np.zeros(n, dtype=tg.EVENT_DTYPE)
    mono["delta"] = 1
    mono["ptr"] = np.arange(1, n + 1)
    mono["line"] = np.arange(n) % 3
    for T in (10 ** 9, 700, 1023, 100_000):
        out.append((f"mono3t T{T}", mono, dict(threshold=T, num_lines=3)))
    rng = np.random.default_rng(17)
    drift = np.zeros(2 * 1024 * 512 + 5, dtype=tg.EVENT_DTYPE)
    drift["delta"] = rng.integers(-100, 101, drift.shape[0])
    drift["ptr"] = np.arange(1, drift.shape[0] + 1)
    drift["line"] = rng.integers(0, 5, drift.shape[0])
    drift["flags"] = (rng.random(drift.shape[0]) < 0.3).astype(np.uint8)
    for T in (300, 2_000, 30_000, 10 ** 7):
        out.append((f"drift2t T{T}", drift, dict(threshold=T, num_lines=5)))
    for nseg in (1024, 1025, 2048):
        for extra in (0, 1):
            m = nseg * 512 - (1 - extra) * 3
            out.append((f"edge n{m}", mono[:m], dict(threshold=5000, num_lines=3)))
    return out


def test_multi_tile_chains(sampler):
    say("multi-tile traces with unresolved chains")
    cases = multi_tile_cases()
    for i in range(0, len(cases), 4):
        check_batch(sampler, cases[i:i + 4])


def tile_map_cases():
    """Traces of several tiles (512 segments of 512 events) whose segments
    move the footprint far less than T, so that tiles get tile maps: a
    config-5 mix (a few samples per tile), the same at thresholds where only
    some segments move less than T, the same with one allocation above 2T in
    its third tile (a segment every entry samples in: that tile gets no map
    and the tiles after it are chained by the resolve pass), a drift, and a
    monotone trace whose every node is a new maximum (more chains than a map
    follows: no map)."""
    n = 5 * 512 * 512 + 1234
    ev, kw = tg.config5(seed=51, n=n)
    c5 = dict(copy_threshold=kw["copy_threshold"], num_lines=kw["num_lines"], quantum_us=kw["quantum_us"])
    out = [(f"c5mix T{T >> 20}M", ev, dict(threshold=T, **c5))
           for T in (64 * tg.MiB, 32 * tg.MiB, 16 * tg.MiB, 4 * tg.MiB)]
    big = ev.copy()
    i = 2 * 512 * 512 + 4321
    big["delta"][i] = 200 * tg.MiB
    big["flags"][i] = 0
    out.append(("c5mix forced", big, dict(threshold=64 * tg.MiB, **c5)))
    rng = np.random.default_rng(23)
    drift = np.zeros(3 * 512 * 512 + 77, dtype=tg.EVENT_DTYPE)
    drift["delta"] = rng.integers(-100, 101, drift.shape[0])
    drift["ptr"] = np.arange(1, drift.shape[0] + 1)
    drift["line"] = rng.integers(0, 5, drift.shape[0])
    for T in (3_000, 30_000):
        out.append((f"drift T{T}", drift, dict(threshold=T, num_lines=5)))
    # A walk of +-50 steps reflected inside [-1000, 1000]: every segment
    # moves above and below its start (two or more chains: SIM maps), the
    # tile's extremes stop growing early (few sources) and stay far apart
    # from 2T, so every tile's map keeps entries that never sample (U open).
    # A sawtooth (+50, -50) has one chain per segment (CONST maps): no map.
    n4 = 4 * 512 * 512 + 333
    steps = np.where(np.random.default_rng(29).random(n4) < 0.5, 50, -50)
    f, d = 0, np.empty(n4, dtype=np.int64)
    for i, st in enumerate(steps.tolist()):
        if not -1000 <= f + st <= 1000:
            st = -st
        d[i] = st
        f += st
    band = np.zeros(n4, dtype=tg.EVENT_DTYPE)
    band["delta"] = d
    band["ptr"] = np.arange(1, n4 + 1)
    band["line"] = np.arange(n4) % 3
    out.append(("band T1000000", band, dict(threshold=10 ** 6, num_lines=3)))
    saw = band.copy()
    saw["delta"] = np.where(np.arange(n4) % 2 == 0, 50, -50)
    out.append(("saw T1000000", saw, dict(threshold=10 ** 6, num_lines=3)))
    mono = np.zeros(2 * 512 * 512 + 9, dtype=tg.EVENT_DTYPE)
    mono["delta"] = 1
    mono["ptr"] = np.arange(1, mono.shape[0] + 1)
    out.append(("mono T1e6", mono, dict(threshold=10 ** 6, num_lines=1)))
    return out


def test_tile_maps(sampler):
    """Tile maps forced on for every multi-tile trace: each trace alone (with
    the map counters), then all of them in one launch."""
    say("tile maps")
    cases = tile_map_cases()
    try:
        sampler.set_tuning(tile_map_tiles=1)
        mapped = {}
        for case in cases:
            check_batch(sampler, [case])
            c = sampler.last_counters()
            mapped[case[0]] = (c[5], c[6])
            say(f"  {case[0]}: {c[5]} tiles mapped, {c[6]} chained through maps")
        ntile = -(-cases[0][1].shape[0] // (512 * 512))
        assert mapped["c5mix T64M"] == (ntile, ntile)
        assert mapped["c5mix forced"][0] == ntile - 1 and mapped["c5mix forced"][1] == 2
        nb = -(-(4 * 512 * 512 + 333) // (512 * 512))
        assert mapped["band T1000000"] == (nb, nb)
        assert mapped["saw T1000000"] == (0, 0)
        # (its two full tiles get no map; the short last one may)
        assert mapped["mono T1e6"][0] <= 1 and mapped["mono T1e6"][1] == 0
        check_batch(sampler, cases)
    finally:
        sampler.set_tuning()


def test_copy_and_timer_mix(sampler):
    say("copy + timer mix")
    ev = tg.mix(9, 300_000, num_lines=1000, zipf_s=1.05, copy_frac=0.10, timer_frac=0.01)
    cases = [("c5mix Tc=T", ev, dict(threshold=4 * tg.MiB, copy_threshold=4 * tg.MiB, num_lines=1000)),
             ("c5mix Tc odd", ev, dict(threshold=4 * tg.MiB, copy_threshold=3 * tg.MiB + 7, num_lines=1000)),
             ("c5mix T64M", ev, dict(threshold=64 * tg.MiB, num_lines=1000))]
    check_batch(sampler, cases)


def test_errors(sampler):
    say("error codes")
    ok = tg.make_events([(5, 1, 0, 0)] * 700)
    bad_line = ok.copy()
    bad_line["line"][650] = 9
    bad_kind = ok.copy()
    bad_kind["flags"][3] = 6
    bad_copy = ok.copy()
    bad_copy["flags"][100] = 2
    bad_copy["delta"][100] = -1
    big = tg.make_events([((1 << 52) - 1, i + 1, 0, 0) for i in range(1200)])
    cases = [("ok", ok, dict(threshold=10, num_lines=1)), ("bad_line", bad_line, dict(threshold=10, num_lines=1)),
             ("bad_kind", bad_kind, dict(threshold=10, num_lines=1)),
             ("bad_copy", bad_copy, dict(threshold=10, num_lines=1)),
             ("overflow", big, dict(threshold=10, num_lines=1))]
    outs = run_batch(sampler, cases)
    want = [smp.SMP_OK, smp.SMP_EINVAL, smp.SMP_EINVAL, smp.SMP_EINVAL, smp.SMP_EOVERFLOW]
    assert [o["status"] for o in outs] == want
    for (label, ev, kw), g in zip(cases, outs):
        assert oracle.run(ev, **kw)["status"] == g["status"], label


def test_pass_event_mask(sampler):
    say("pass event mask")
    ev, kw = tg.config1(seed=11, n=50_000)
    p = smp.make_params(kw["threshold"], kw["num_lines"])
    o = oracle.run(ev, threshold=kw["threshold"], num_lines=kw["num_lines"])
    try:
        sampler.set_pass_events(0x30)  # only the two events around the emit pass
        tid = sampler.submit_trace(ev, p)
        sampler.run(blocking=True)
        t = sampler.last_pass_timing()
        assert t["emit"] > 0, t
        assert all(t[k] == -1 for k in smp.PASS_NAMES if k != "emit"), t
        assert sampler.last_timing() == (-1, -1)
        g = sampler.fetch_profile(tid)
        compare(g, o, "mask 0x30")
        sampler.set_pass_events(0x7F)
        tid = sampler.submit_trace(ev, p)
        sampler.run(blocking=True)
        t = sampler.last_pass_timing()
        assert all(t[k] > 0 for k in smp.PASS_NAMES), t
        assert all(x > 0 for x in sampler.last_timing())
        compare(sampler.fetch_profile(tid), o, "mask 0x3F")
        with pytest.raises(smp.SamplerError):
            sampler.set_pass_events(0x80)
    finally:
        sampler.set_pass_events(0x7F)


def test_batch_submit_and_release(sampler):
    say("submit_traces / release_traces")
    import torch
    cases = [tg.config1(seed=31 + i, n=n) for i, n in enumerate((1, 700, 50_000, 200_000))]
    params = [smp.make_params(kw["threshold"], kw["num_lines"]) for _, kw in cases]
    # device tensors: results equal the oracle's
    devs = [torch.from_numpy(ev.view(np.uint8)).to("cuda") for ev, _ in cases]
    ids = sampler.submit_traces(devs, params)
    assert len(ids) == len(cases)
    sampler.run(blocking=True)
    for (ev, kw), tid in zip(cases, ids):
        compare(sampler.fetch_profile(tid), oracle.run(ev, threshold=kw["threshold"], num_lines=kw["num_lines"]),
                "submit_traces")
    # host arrays, released without copying out: sample counts and statuses
    ids = sampler.submit_traces([ev for ev, _ in cases], params)
    sampler.run(blocking=True)
    got = sampler.release_traces(ids)
    want = [oracle.run(ev, threshold=kw["threshold"], num_lines=kw["num_lines"]) for ev, kw in cases]
    assert got == [(o["K"], smp.SMP_OK) for o in want]
    with pytest.raises(smp.SamplerError):
        sampler.release_traces(ids)  # already released
    # the same batch with its parameters as a prebuilt ctypes array
    params_arr = (smp.Params * len(params))(*params)
    ids = sampler.submit_traces(devs, params_arr)
    sampler.run(blocking=True)
    assert sampler.release_traces(ids) == [(o["K"], smp.SMP_OK) for o in want]


def test_run_splits_over_4096_traces(sampler):
    """One run() over 5,000 pending traces: more than one launch's
    descriptor table holds (4,096), so the batch is split over two run
    slots.  Every trace must still equal the oracle."""
    say("run() over 5000 traces (split over two slots)")
    rng = np.random.default_rng(4096)
    cases = []
    for i in range(5000):
        n = int(rng.integers(0, 1500))
        T = (64 * tg.KiB, 256 * tg.KiB, tg.MiB)[i % 3]
        ev = tg.mix(10_000 + i, n, num_lines=32, zipf_s=1.1) if n else tg.make_events([])
        cases.append((f"split t{i}", ev, dict(threshold=T, num_lines=32)))
    check_batch(sampler, cases)


def test_ten_runs_reuse_busy_slots(sampler):
    """Ten non-blocking run() calls before any fetch: the sampler has eight
    run slots, so the ninth and tenth launches wait for and reuse the
    oldest busy slot.  Every trace of every launch must equal the oracle."""
    say("ten non-blocking runs before any fetch (slot reuse)")
    import torch
    runs = []
    for r in range(10):
        batch = []
        for k in range(3):
            n = 200_000 + 150_000 * k + 7 * r
            ev, kw = tg.config1(seed=700 + 10 * r + k, n=n)
            dev = torch.from_numpy(ev.view(np.uint8)).to("cuda")
            tid = sampler.submit_trace(dev, smp.make_params(kw["threshold"], kw["num_lines"]))
            batch.append((tid, ev, kw))
        sampler.run(blocking=False)
        runs.append(batch)
    for r, batch in enumerate(runs):
        for tid, ev, kw in batch:
            g = sampler.fetch_profile(tid)
            compare(g, oracle.run(ev, threshold=kw["threshold"], num_lines=kw["num_lines"]), f"run {r}")


def graph_cases():
    rng = np.random.default_rng(2024)
    cases = [(f"g tiny{i}", tiny_trace(rng, int(rng.integers(1, 60))), dict(threshold=int(rng.integers(1, 40)),
                                                                          num_lines=5)) for i in range(6)]
    for seed, n in ((61, 50_000), (62, 300_000), (63, 1_100_000)):
        ev, kw = tg.config1(seed=seed, n=n)
        cases.append((f"g c1 s{seed}", ev, dict(threshold=kw["threshold"], num_lines=kw["num_lines"])))
    # a slow drift: segments whose chains never collapse
    drift = next(ev for name, ev, _ in adversarial_cases() if name.startswith("drift"))
    cases.append(("g drift", drift, dict(threshold=40_000, num_lines=7)))
    return cases


def test_graph_replays_equal_oracle(sampler):
    """The same batch shape launched five times without timing events
    between passes: the first launch is plain, the second captures the
    launch sequence as a HIP graph, the later ones replay it.  Eager torch
    work and synchronisations run between the replays; every launch's
    profiles must equal the oracle's, and the start and end events around
    the graph must time this launch.  A launch that asks for events between
    passes is plain again, and also exact."""
    say("graph capture and replays")
    import torch
    cases = graph_cases()
    want = [oracle.run(ev, **kw) for _, ev, kw in cases]
    before = sampler.launch_stats()
    x = torch.arange(1 << 20, device="cuda", dtype=torch.int64)
    try:
        sampler.set_pass_events(0x40)  # the launch's start event only
        for rep in range(5):
            outs = run_batch(sampler, cases)
            main_ms, total_ms = sampler.last_timing()
            assert main_ms == -1 and 0 < total_ms < 50, (rep, main_ms, total_ms)
            for (label, _, _), g, o in zip(cases, outs, want):
                compare(g, o, f"{label} launch {rep}")
            # eager work on the device between replays
            y = (x * 3 + rep).sum()
            torch.cuda.synchronize()
            assert int(y) == 3 * ((1 << 20) * ((1 << 20) - 1) // 2) + rep * (1 << 20)
        mid = sampler.launch_stats()
        assert mid["captured"] - before["captured"] >= 1, (before, mid)
        assert mid["replayed"] - before["replayed"] >= 3, (before, mid)
        sampler.set_pass_events(0x7F)
        outs = run_batch(sampler, cases)
        assert sampler.launch_stats()["plain"] == mid["plain"] + 1
        assert all(v > 0 for v in sampler.last_pass_timing().values())
        for (label, _, _), g, o in zip(cases, outs, want):
            compare(g, o, f"{label} with pass events")
    finally:
        sampler.set_pass_events(0x7F)


@pytest.mark.parametrize("tuning", [dict(chain_cap=1), dict(chain_cap=8, chain_grid=1, emit_grid=1),
                                    dict(chain_cap=64, chain_grid=3, emit_grid=7, graphs=0),
                                    dict(chain_cap=48, chain_grid=4096, emit_grid=4096)])
def test_results_do_not_depend_on_tuning(sampler, tuning):
    say(f"parity under tuning {tuning}")
    cases = graph_cases() + multi_tile_cases()[:2]
    try:
        sampler.set_tuning(**tuning)
        got = sampler.get_tuning()
        for k, v in tuning.items():
            assert got[k] == v, (k, got)
        check_batch(sampler, cases)
    finally:
        sampler.set_tuning()
    with pytest.raises(smp.SamplerError):
        sampler.set_tuning(chain_cap=65)
    with pytest.raises(smp.SamplerError):
        sampler.set_tuning(chain_cap=0)


def test_budget_admission(sampler):
    say("admission by budget")
    import torch
    p = smp.make_params(10, 4)
    need = smp.workspace_bytes(10_000, p, ev_on_device=False)
    ws = torch.empty(smp.sampler_fixed_bytes() + need + 4096, dtype=torch.uint8, device="cuda")
    s = smp.Sampler(workspace=ws)
    ev = tg.make_events([(1, i + 1, 0, 0) for i in range(10_000)])
    tid = s.submit_trace(ev, p)
    assert s.try_submit(ev, p)[0] == smp.SMP_EBUDGET
    assert s.try_submit(tg.make_events([(1, 1, 0, 0)] * 100_000), p)[0] == smp.SMP_ETOOBIG
    s.run(blocking=True)
    assert s.poll(tid)
    r = s.fetch_profile(tid)
    compare(r, oracle.run(ev, threshold=10, num_lines=4))
    tid2 = s.submit_trace(ev, p)  # space is free again
    s.run(blocking=True)
    compare(s.fetch_profile(tid2), oracle.run(ev, threshold=10, num_lines=4))
    s.close()


def test_alone_equals_in_batch(sampler):
    say("determinism: alone vs in a batch")
    ev, _ = tg.config1(seed=7, n=50_000)
    kw = dict(threshold=tg.MiB, num_lines=64)
    alone = run_batch(sampler, [("alone", ev, kw)])[0]
    others = [(f"o{i}", tg.config1(seed=100 + i, n=20_000 + 997 * i)[0], kw) for i in range(20)]
    mixed = run_batch(sampler, others[:10] + [("mid", ev, kw)] + others[10:])[10]
    compare(alone, mixed, "alone vs batch")
    compare(alone, oracle.run(ev, **kw), "alone vs oracle")


def test_device_resident_events(sampler):
    say("device-resident events")
    import torch
    ev, _ = tg.config1(seed=8)
    dev = torch.from_numpy(ev.view(np.uint8)).to("cuda")
    p = smp.make_params(tg.MiB, 64)
    tid = sampler.submit_trace(dev, p)
    sampler.run(blocking=True)
    compare(sampler.fetch_profile(tid), oracle.run(ev, threshold=tg.MiB, num_lines=64))


def test_pinned_fetch(sampler):
    """A profile fetched into page-locked arrays equals the oracle (and so
    the pageable fetch), including a trace with no samples."""
    say("pinned fetch")
    ev, _ = tg.config1(seed=9)
    flat = np.zeros(1000, dtype=tg.EVENT_DTYPE)
    flat["ptr"] = np.arange(1, 1001)
    cases = [("c1 s9", ev, dict(threshold=tg.MiB, num_lines=64)), ("flat", flat, dict(threshold=tg.MiB, num_lines=4))]
    ids = [sampler.submit_trace(e, smp.make_params(kw["threshold"], kw["num_lines"])) for _, e, kw in cases]
    sampler.run(blocking=True)
    for (label, e, kw), tid in zip(cases, ids):
        g = sampler.fetch_profile(tid, pinned=True)
        compare(g, oracle.run(e, **kw), label + " pinned")


def test_config3_batch(sampler):
    say("config 3: 1024 traces in one launch")
    plan = tg.config3_plan()
    cases = []
    for t, (n, T, seed) in enumerate(plan):
        ev, kw = tg.config3_trace(n, T, seed)
        cases.append((f"c3 t{t}", ev, dict(threshold=kw["threshold"], num_lines=kw["num_lines"])))
    outs = run_batch(sampler, cases)
    say("  oracle")
    for (label, ev, kw), g in zip(cases, outs):
        compare(g, oracle.run(ev, **kw), label)


def test_config2_full(sampler):
    say("config 2: 1e8 events, generating")
    import torch
    ev, kw = tg.config2()
    dev = torch.from_numpy(ev.view(np.uint8)).to("cuda")
    p = smp.make_params(kw["threshold"], kw["num_lines"])
    say("  gpu")
    tid = sampler.submit_trace(dev, p)
    sampler.run(blocking=True)
    g = sampler.fetch_profile(tid)
    del dev
    say("  oracle")
    o = oracle.run(ev, threshold=kw["threshold"], num_lines=kw["num_lines"])
    compare(g, o, "config2")
    assert g["K"] > 1_000_000


def test_config5_mix_1e8(sampler):
    say("config-5 mix at 1e8 events, generating")
    import torch
    ev, kw = tg.config5(n=100_000_000)
    dev = torch.from_numpy(ev.view(np.uint8)).to("cuda")
    p = smp.make_params(kw["threshold"], kw["num_lines"], kw["copy_threshold"], kw["quantum_us"])
    say("  gpu")
    tid = sampler.submit_trace(dev, p)
    sampler.run(blocking=True)
    g = sampler.fetch_profile(tid)
    del dev
    say("  oracle")
    o = oracle.run(ev, threshold=kw["threshold"], num_lines=kw["num_lines"], copy_threshold=kw["copy_threshold"],
                   quantum_us=kw["quantum_us"])
    compare(g, o, "config5 1e8")


def test_config5_full(sampler):
    """The full config-5 trace (5e8 events, copy and timer events, 1e6
    lines), compared field by field with the oracle."""
    say("config 5: 5e8 events, generating")
    import torch
    ev, kw = tg.config5()
    dev = torch.from_numpy(ev.view(np.uint8)).to("cuda")
    p = smp.make_params(kw["threshold"], kw["num_lines"], kw["copy_threshold"], kw["quantum_us"])
    say("  gpu")
    tid = sampler.submit_trace(dev, p)
    sampler.run(blocking=True)
    g = sampler.fetch_profile(tid)
    del dev
    torch.cuda.empty_cache()
    say("  oracle")
    o = oracle.run(ev, threshold=kw["threshold"], num_lines=kw["num_lines"], copy_threshold=kw["copy_threshold"],
                   quantum_us=kw["quantum_us"])
    compare(g, o, "config5")
    assert g["K"] > 10_000
