"""Pins for the CPU oracle (no GPU).

The oracle is checked against things other than itself: hand-worked
fixtures (tests/golden, each citing the paper passage whose rule it applies),
brute-force enumeration of every candidate sample set on tiny traces, closed
forms, a second independent formulation (first-crossing search + chain
iteration, and the leak rule restated as one window compare per tracked
object), and invariants that hold at any size.
"""
import glob
import itertools
import json
import os

import numpy as np
import pytest

import oracle
import tracegen as tg

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


# ------------------------------------------------------------ helpers --

def events_from_rows(rows):
    return tg.make_events([tuple(r) for r in rows])


def run_case(params, rows):
    ev = events_from_rows(rows)
    p = dict(params)
    return oracle.run(ev, threshold=p["threshold"], num_lines=p["num_lines"],
                      copy_threshold=p.get("copy_threshold"), quantum_us=p.get("quantum_us", 10_000),
                      options=p.get("options", 0))


def check_expect(r, exp, num_lines):
    assert r["status"] == oracle.OK
    s = r["samples"]
    got = [[int(x["event_idx"]), int(x["line"]), int(x["F"]), int(x["py"]), int(x["nat"])] for x in s]
    assert got == exp["samples"]
    for key in ("final_F", "peak_F", "peak_sampled_F"):
        if key in exp:
            assert r[key] == exp[key], key
    if "lines" in exp:
        for name in oracle.HIST_NAMES:
            want = np.zeros(num_lines, np.int64)
            for line, v in exp["lines"].get(name, {}).items():
                want[int(line)] = v
            np.testing.assert_array_equal(r[name], want, err_msg=name)
    if "tracked" in exp:
        t = r["tracked"]
        got_t = [[int(x["event_idx"]), int(x["line"]), int(x["ptr"]), int(x["freed"])] for x in t]
        assert got_t == exp["tracked"]
    if "leak" in exp:
        for line in range(num_lines):
            if str(line) in exp["leak"]:
                e = exp["leak"][str(line)]
                assert [r["lap_num"][line], r["lap_den"][line]] == e["laplace"]
                assert [r["lit_num"][line], r["lit_den"][line]] == e["literal"]
            else:
                assert r["lap_den"][line] == 0 and r["lit_den"][line] == 0


# ---------------------------------------------------- golden fixtures --

def _golden_cases():
    out = []
    for path in sorted(glob.glob(os.path.join(GOLDEN, "W*.json"))):
        d = json.load(open(path))
        if "cases" in d:
            for k, c in enumerate(d["cases"]):
                out.append(pytest.param(c["params"], c["events"], c["expect"], id=f"{d['id']}.{k}"))
        else:
            out.append(pytest.param(d["params"], d["events"], d["expect"], id=d["id"]))
    return out


@pytest.mark.parametrize("params,rows,expect", _golden_cases())
def test_golden(params, rows, expect):
    r = run_case(params, rows)
    check_expect(r, expect, params["num_lines"])


def test_w4_peak_only_view_misses_first_object():
    """Section 6.3: a peak-only profile would show only the second object;
    the threshold sampler attributes the 4 GB to both allocation lines."""
    d = json.load(open(os.path.join(GOLDEN, "W4.json")))
    r = run_case(d["params"], d["events"])
    assert r["growth_bytes"][0] == 1 << 32 and r["growth_bytes"][2] == (1 << 32) + 8
    # neither site passes the 95 % report gate with a single observation
    assert not r["lap_gate"].any() and not r["lit_gate"].any()


def test_w9_threshold_is_prime_above_10mb():
    d = json.load(open(os.path.join(GOLDEN, "W9.json")))
    r = run_case(d["params"], d["events"])
    t = r["threshold_used"]
    assert t >= 10 * tg.MiB and all(t % k for k in range(2, int(t ** 0.5) + 1))
    assert all(any(v % k == 0 for k in range(2, int(v ** 0.5) + 1)) for v in range(10 * tg.MiB, t))


# -------------------------------------------------------- brute force --

def footprint(ev):
    kind = (ev["flags"] >> 1) & 3
    d = np.where(kind == 0, ev["delta"], 0).astype(np.int64)
    return np.concatenate([[0], np.cumsum(d)])


def satisfies_definition(F, T, nodes):
    """Every consecutive pair (from the virtual node 0) is a first crossing
    and nothing crosses after the last sample."""
    prev = 0
    for s in nodes:
        if abs(int(F[s]) - int(F[prev])) < T:
            return False
        for j in range(prev + 1, s):
            if abs(int(F[j]) - int(F[prev])) >= T:
                return False
        prev = s
    for j in range(prev + 1, len(F)):
        if abs(int(F[j]) - int(F[prev])) >= T:
            return False
    return True


def brute_force_samples(ev, T):
    F = footprint(ev)
    n = len(ev)
    hits = []
    for mask in range(1 << n):
        nodes = [i + 1 for i in range(n) if mask >> i & 1]
        if satisfies_definition(F, T, nodes):
            hits.append([x - 1 for x in nodes])
    return hits


def random_tiny_trace(rng, n, with_other_kinds):
    rows = []
    for i in range(n):
        kind = 0
        if with_other_kinds and rng.random() < 0.2:
            kind = 1 if rng.random() < 0.5 else 2
        d = int(rng.integers(-3, 4)) if kind == 0 else int(rng.integers(0, 4))
        rows.append((d, i + 1, int(rng.integers(0, 3)), int(rng.integers(0, 2)), kind))
    return events_from_rows(rows)


def test_brute_force_exhaustive_small_alphabet():
    """All traces of 4 memory events with deltas in {+-1,+-2,+-3}, T in 1..5:
    exactly one index set satisfies the definition and it is the oracle's."""
    alphabet = [-3, -2, -1, 1, 2, 3]
    for T in range(1, 6):
        for ds in itertools.product(alphabet, repeat=4):
            ev = events_from_rows([(d, i + 1, 0, 0, 0) for i, d in enumerate(ds)])
            hits = brute_force_samples(ev, T)
            assert len(hits) == 1, (ds, T, hits)
            r = oracle.run(ev, threshold=T, num_lines=1)
            assert list(r["samples"]["event_idx"]) == hits[0], (ds, T)


def test_brute_force_random_up_to_12():
    rng = np.random.default_rng(1234)
    for trial in range(150):
        n = int(rng.integers(1, 13))
        T = int(rng.integers(1, 7))
        ev = random_tiny_trace(rng, n, with_other_kinds=bool(trial % 2))
        hits = brute_force_samples(ev, T)
        assert len(hits) == 1
        r = oracle.run(ev, threshold=T, num_lines=3)
        assert list(r["samples"]["event_idx"]) == hits[0]


# ------------------------------------------------------- closed forms --

def test_threshold_one_samples_every_nonzero_memory_event():
    rng = np.random.default_rng(7)
    ev = random_tiny_trace(rng, 400, with_other_kinds=True)
    ev["delta"][::7] = np.where((ev["flags"][::7] >> 1) == 0, 0, ev["delta"][::7])
    r = oracle.run(ev, threshold=1, num_lines=3)
    kind = (ev["flags"] >> 1) & 3
    want = np.flatnonzero((kind == 0) & (ev["delta"] != 0))
    np.testing.assert_array_equal(r["samples"]["event_idx"], want)


def test_threshold_above_total_variation_never_samples():
    ev, _ = tg.config1(seed=11, n=5000)
    kind = (ev["flags"] >> 1) & 3
    tv = int(np.abs(np.where(kind == 0, ev["delta"], 0)).sum())
    r = oracle.run(ev, threshold=tv + 1, num_lines=64)
    assert r["K"] == 0 and r["H"] == 0


@pytest.mark.parametrize("T", [1, 3, 10, 64])
def test_monotone_unit_steps(T):
    n = 1000
    ev = events_from_rows([(1, i + 1, 0, 0, 0) for i in range(n)])
    r = oracle.run(ev, threshold=T, num_lines=1)
    assert r["K"] == n // T
    np.testing.assert_array_equal(r["samples"]["event_idx"], np.arange(1, n // T + 1) * T - 1)
    np.testing.assert_array_equal(r["samples"]["F"], np.arange(1, n // T + 1) * T)
    # every sample is a new maximum, so every one is tracked and none freed
    assert r["H"] == n // T and r["leak_frees"][0] == 0


def test_leak_gates_and_printed_formula():
    m = np.array([18, 19, 38, 39, 4, 0, 1, 5], np.int64)
    f = np.array([0, 0, 1, 1, 4, 0, 1, 2], np.int64)
    s = oracle.leak_scores(m, f)
    # Laplace gate: likelihood (m-f+1)/(m+2) > 0.95
    assert list(s["lap_gate"]) == [0, 1, 0, 1, 0, 0, 0, 0]
    assert (s["lap_num"][0], s["lap_den"][0]) == (19, 20)
    assert (s["lap_num"][1], s["lap_den"][1]) == (20, 21)
    # the printed formula goes negative when every tracked object was freed
    assert (s["lit_num"][4], s["lit_den"][4]) == (-3, 2)
    assert (s["lap_num"][4], s["lap_den"][4]) == (1, 6)
    assert s["lap_den"][5] == 0 and s["lit_den"][5] == 0
    # exact: num/den equals the real-valued formulas
    for i in (0, 1, 2, 3, 6, 7):
        assert abs(s["lap_num"][i] / s["lap_den"][i] - (1 - (f[i] + 1) / (m[i] + 2))) < 1e-12
        assert abs(s["lit_num"][i] / s["lit_den"][i] - (1 - (f[i] + 1) / (m[i] - f[i] + 2))) < 1e-12


# ------------------------------------------------ second formulation --

def chain_by_search(F, T):
    """Samples by iterating 'first later node whose footprint differs from the
    reference by at least T' from the virtual node 0."""
    out = []
    r = 0
    n = len(F) - 1
    while True:
        nxt = None
        start = r + 1
        step = 256
        while start <= n:
            seg = F[start:start + step]
            hit = np.flatnonzero(np.abs(seg - F[r]) >= T)
            if hit.size:
                nxt = start + int(hit[0])
                break
            start += step
            step *= 2
        if nxt is None:
            return out
        out.append(nxt)
        r = nxt


def restated_profile(ev, T, num_lines):
    """Per-line attribution and leak counts recomputed from the sample chain
    with prefix sums and one window compare per tracked object."""
    kind = (ev["flags"] >> 1) & 3
    mem = kind == 0
    d = np.where(mem, ev["delta"], 0).astype(np.int64)
    pyd = np.where(mem & ((ev["flags"] & 1) == 0), ev["delta"], 0).astype(np.int64)
    F = np.concatenate([[0], np.cumsum(d)])
    P = np.concatenate([[0], np.cumsum(pyd)])
    nodes = chain_by_search(F, T)
    lines = ev["line"]
    out = {name: np.zeros(num_lines, np.int64) for name in oracle.HIST_NAMES}
    prev = 0
    hwm = 0
    tracked = []
    samples = []
    for s in nodes:
        ln = int(lines[s - 1])
        py = int(P[s] - P[prev])
        nat = int(F[s] - F[prev]) - py
        samples.append((s - 1, ln, int(F[s]), py, nat))
        out["py_bytes"][ln] += py
        out["nat_bytes"][ln] += nat
        delta = int(F[s] - F[prev])
        if delta > 0:
            out["growth_n"][ln] += 1
            out["growth_bytes"][ln] += delta
            if F[s] > hwm:
                tracked.append((s - 1, ln, int(ev["ptr"][s - 1])))
                out["leak_mallocs"][ln] += 1
                hwm = int(F[s])
        else:
            out["shrink_n"][ln] += 1
            out["shrink_bytes"][ln] += -delta
        prev = s
    frees = np.flatnonzero(mem & (ev["delta"] < 0))
    freed = []
    for h, (idx, ln, ptr) in enumerate(tracked):
        end = tracked[h + 1][0] if h + 1 < len(tracked) else len(ev)
        lo, hi = np.searchsorted(frees, idx, "right"), np.searchsorted(frees, end, "left")
        hit = bool((ev["ptr"][frees[lo:hi]] == ptr).any())
        freed.append(hit)
        if h + 1 < len(tracked) and hit:
            out["leak_frees"][ln] += 1
    return samples, out, tracked, freed


@pytest.mark.parametrize("seed,T,gen", [(1, tg.MiB, "c1"), (2, 256 * tg.KiB, "c1"), (3, 10 * tg.MiB, "c1"),
                                        (4, 10 * tg.MiB, "c2")])
def test_second_formulation_agrees(seed, T, gen):
    if gen == "c1":
        ev = tg.mix(seed, 100_000, num_lines=64)
        L = 64
    else:
        ev = tg.lifetime(seed, 200_000, num_lines=500)
        L = 500
    r = oracle.run(ev, threshold=T, num_lines=L)
    samples, prof, tracked, freed = restated_profile(ev, T, L)
    got = [tuple(int(v) for v in row) for row in r["samples"][["event_idx", "line", "F", "py", "nat"]].tolist()]
    assert got == samples
    for name in ("py_bytes", "nat_bytes", "growth_n", "shrink_n", "growth_bytes", "shrink_bytes",
                 "leak_mallocs", "leak_frees"):
        np.testing.assert_array_equal(r[name], prof[name], err_msg=name)
    assert [tuple(int(v) for v in x) for x in r["tracked"][["event_idx", "line", "ptr"]].tolist()] == tracked
    assert [bool(x) for x in r["tracked"]["freed"]] == freed


# --------------------------------------------------------- invariants --

def check_invariants(ev, r, T, Tc, q):
    kind = (ev["flags"] >> 1) & 3
    mem = kind == 0
    d = np.where(mem, ev["delta"], 0).astype(np.int64)
    F = np.concatenate([[0], np.cumsum(d)])
    s = r["samples"]
    K = r["K"]
    # telescoping: per-line sampled bytes sum to the footprint at the last sample
    last = int(s["F"][-1]) if K else 0
    assert int(r["py_bytes"].sum() + r["nat_bytes"].sum()) == last
    np.testing.assert_array_equal(s["py"] + s["nat"], np.diff(np.concatenate([[0], s["F"]])))
    np.testing.assert_array_equal(s["F"], F[s["event_idx"].astype(np.int64) + 1])
    assert int(r["growth_n"].sum() + r["shrink_n"].sum()) == K
    # each step is at least T and at most T - 1 + |trigger delta|
    steps = np.abs(np.diff(np.concatenate([[0], s["F"]])))
    trig = np.abs(ev["delta"][s["event_idx"]])
    assert (steps >= T).all() and (steps <= T - 1 + trig).all()
    # threshold sampling never takes more samples than deterministic rate-based sampling
    tv = int(np.abs(d).sum())
    assert K <= tv // T
    # corrected lower bound on the number of samples
    assert abs(int(F[-1])) <= (K + 1) * (T - 1) + int(trig.sum())
    # leak counts
    assert int(r["leak_mallocs"].sum()) == r["H"]
    assert int(r["leak_frees"].sum()) <= max(r["H"] - 1, 0)
    assert (r["leak_frees"] <= r["leak_mallocs"]).all()
    # copy and timer totals
    C = int(np.where(kind == 1, ev["delta"], 0).sum())
    assert int(r["copy_exact"].sum()) == C
    assert int(r["copy_sampled"].sum()) == (C // Tc) * Tc
    nt = int((kind == 2).sum())
    assert int(r["py_time_us"].sum()) == q * nt
    assert int(r["nat_time_us"].sum()) == int(np.where(kind == 2, ev["delta"], 0).sum())
    assert r["final_F"] == int(F[-1]) and r["peak_F"] == max(0, int(F.max()))


@pytest.mark.parametrize("seed", [1, 2, 3])
@pytest.mark.parametrize("T", [256 * tg.KiB, tg.MiB, 10 * tg.MiB])
def test_invariants_config1_mix(seed, T):
    ev, _ = tg.config1(seed=seed)
    r = oracle.run(ev, threshold=T, num_lines=64)
    check_invariants(ev, r, T, T, 10_000)


def test_invariants_with_copy_and_timer():
    ev = tg.mix(9, 200_000, num_lines=1000, zipf_s=1.05, copy_frac=0.10, timer_frac=0.01)
    T, Tc = 4 * tg.MiB, 3 * tg.MiB + 7
    r = oracle.run(ev, threshold=T, copy_threshold=Tc, num_lines=1000, quantum_us=10_000)
    check_invariants(ev, r, T, Tc, 10_000)
    kind = (ev["flags"] >> 1) & 3
    # copy samples, per event, from the cumulative copy count
    c = np.cumsum(np.where(kind == 1, ev["delta"], 0))
    n_i = c // Tc - np.concatenate([[0], c[:-1]]) // Tc
    want = np.zeros(1000, np.int64)
    np.add.at(want, ev["line"], np.where(kind == 1, n_i * Tc, 0))
    np.testing.assert_array_equal(r["copy_sampled"], want)


# ----------------------------------------------------- error handling --

def test_errors():
    ok = [(5, 1, 0, 0, 0)]
    assert run_case({"threshold": 10, "num_lines": 1}, ok)["status"] == oracle.OK
    assert run_case({"threshold": 10, "num_lines": 1}, [(5, 1, 1, 0, 0)])["status"] == oracle.EINVAL
    assert run_case({"threshold": 10, "num_lines": 1}, [(5, 1, 0, 0, 3)])["status"] == oracle.EINVAL
    assert run_case({"threshold": 10, "num_lines": 1}, [(-5, 0, 0, 0, 1)])["status"] == oracle.EINVAL
    assert run_case({"threshold": 10, "num_lines": 1}, [(1 << 32, 0, 0, 0, 2)])["status"] == oracle.EINVAL
    assert run_case({"threshold": 10, "num_lines": 1}, [(1 << 52, 1, 0, 0, 0)])["status"] == oracle.EINVAL
    assert run_case({"threshold": 0, "num_lines": 1}, ok)["status"] == oracle.EINVAL
    big = (1 << 52) - 1
    rows = [(big, i + 1, 0, 0, 0) for i in range(600)]
    assert run_case({"threshold": 10, "num_lines": 1}, rows)["status"] == oracle.EOVERFLOW
    # invalid input wins over overflow
    assert run_case({"threshold": 10, "num_lines": 1}, rows + [(1, 1, 5, 0, 0)])["status"] == oracle.EINVAL


def test_resolve_at_end_option():
    rows = [(20, 1, 0, 0, 0), (-20, 1, 1, 0, 0)]
    r0 = run_case({"threshold": 10, "num_lines": 2}, rows)
    r1 = run_case({"threshold": 10, "num_lines": 2, "options": oracle.OPT_RESOLVE_AT_END}, rows)
    assert r0["leak_frees"][0] == 0 and r0["tracked"]["freed"][0] == 1
    assert r1["leak_frees"][0] == 1


def test_empty_trace():
    r = oracle.run(np.zeros(0, tg.EVENT_DTYPE), threshold=10, num_lines=3)
    assert r["status"] == oracle.OK and r["K"] == 0 and r["final_F"] == 0


# ------------------------------------------- rate-based sampling (3.2) --

def _rate(rows, params):
    return oracle.rate(events_from_rows(rows), params["threshold"], params["num_lines"], params.get("options", 0))


def test_rate_golden():
    """Hand-worked rate-based counts for the golden fixtures' events."""
    spec = json.load(open(os.path.join(GOLDEN, "rate.json")))
    for case in spec["cases"]:
        w = json.load(open(os.path.join(GOLDEN, case["fixture"] + ".json")))
        st, K, counts = _rate(w["events"], w["params"])
        assert st == oracle.OK
        assert K == case["K"] == sum(case["per_event"]), case["fixture"]
        want = np.zeros(w["params"]["num_lines"], np.int64)
        for line, v in case["lines"].items():
            want[int(line)] = v
        np.testing.assert_array_equal(counts, want, err_msg=case["fixture"])
        # per event: the same trace cut after each event
        for i in range(len(w["events"])):
            _, Ki, _ = _rate(w["events"][: i + 1], w["params"])
            assert Ki == sum(case["per_event"][: i + 1]), (case["fixture"], i)


@pytest.mark.parametrize("d,T,n", [(6, 10, 7), (7, 3, 1000), (1, 1, 513), (4096, 1 << 20, 5000), (10, 10, 64)])
def test_rate_closed_form(d, T, n):
    """Events of equal size d (alternating allocations and frees, lines in
    turn): K = floor(n d / T); the lines share it, and with T dividing d every
    event takes exactly d / T samples."""
    rows = [(d if i % 2 == 0 else -d, i, i % 3, 0, 0) for i in range(n)]
    st, K, counts = _rate(rows, {"threshold": T, "num_lines": 3})
    assert st == oracle.OK
    assert K == (n * d) // T
    assert int(counts.sum()) == K
    if d % T == 0:
        want = [(d // T) * len(range(l, n, 3)) for l in range(3)]
        assert counts.tolist() == want


def test_rate_volume_at_t_one():
    """With T = 1 every byte is a sample: K = sum of |delta| over memory events."""
    ev, _ = tg.config1(seed=3, n=5_000)
    mem = ((ev["flags"] >> 1) & 3) == 0
    st, K, counts = oracle.rate(ev, 1, 64)
    assert st == oracle.OK
    assert K == int(np.abs(ev["delta"][mem].astype(object)).sum())
    assert int(counts.sum()) == K


@pytest.mark.parametrize("seed", [1, 2, 3])
def test_rate_bounds_threshold_count(seed):
    """A threshold sample needs T bytes of net change since the last one, so
    at least T bytes of volume: K_threshold <= K_rate on any trace (the
    paper's comparison of the two samplers, made exact)."""
    ev, kw = tg.config1(seed=seed, n=30_000)
    for T in (1 << 12, 1 << 16, 1 << 20, 10_000_019):
        r = oracle.run(ev, threshold=T, num_lines=kw["num_lines"])
        st, K, _ = oracle.rate(ev, T, kw["num_lines"])
        assert st == oracle.OK and r["status"] == oracle.OK
        assert len(r["samples"]) <= K


def test_rate_errors():
    st, K, _ = _rate([(5, 1, 0, 0, 0), (5, 1, 0, 0, 3)], {"threshold": 10, "num_lines": 1})
    assert st == oracle.EINVAL
    st, _, _ = _rate([(5, 1, 2, 0, 0)], {"threshold": 10, "num_lines": 2})
    assert st == oracle.EINVAL
    big = (1 << 52) - 1
    rows = [(big if i % 2 == 0 else -big, 1, 0, 0, 0) for i in range(1025)]
    st, _, _ = _rate(rows, {"threshold": 1 << 40, "num_lines": 1})
    assert st == oracle.EOVERFLOW
    st, K, _ = _rate(rows[:1000], {"threshold": 1 << 40, "num_lines": 1})
    assert st == oracle.OK and K == (1000 * big) >> 40


# ------------------------------------------- report line filter (5) --

def _rl(time=None, mem=None, L=None):
    L = L or len(time if time is not None else mem)
    z = np.zeros(L, np.int64)
    t = np.asarray(time, np.int64) if time is not None else z
    m = np.asarray(mem, np.int64) if mem is not None else z
    return oracle.report_lines(t, z, m).tolist()


def test_report_lines_hand_cases():
    """Section 5: lines with at least 1 % of the time or of the memory, with
    the line before and after each."""
    assert _rl(mem=[0, 0, 10, 0, 0]) == [1, 2, 3]
    assert _rl(mem=[10, 0, 0, 0, 0]) == [0, 1]          # no line before line 0
    assert _rl(mem=[0, 0, 0, 0, 10]) == [3, 4]          # none after the last
    assert _rl(time=[1] * 100) == list(range(100))      # exactly 1 % each: "at least"
    assert _rl(time=[1] * 101) == []                    # just under 1 % each
    assert _rl(time=[0] * 7) == []                      # no time at all
    # the two criteria: line 2 by time, line 8 by memory
    t = [0] * 12
    t[2] = 5
    m = [0] * 12
    m[8] = 7
    assert _rl(time=t, mem=m) == [1, 2, 3, 7, 8, 9]
    # Python and native time add up: 0.6 % + 0.6 % of the time
    py = np.zeros(200, np.int64)
    nat = np.zeros(200, np.int64)
    py[:] = 1
    py[50], nat[50] = 3, 3     # line 50: 6 of 205
    z = np.zeros(200, np.int64)
    assert oracle.report_lines(py, nat, z).tolist() == [49, 50, 51]
    # non-positive values never qualify and do not count in the total
    assert _rl(mem=[-100, 1, 0]) == [0, 1, 2]


def test_report_lines_keeps_the_300_line_bound():
    """Section 5: a profile never holds more than 300 lines.  Lines 0-99
    each hold exactly 1 % of the time and lines 300-349 each 2 % of the
    memory: 150 lines qualify, so the 100 with the largest share stay - the
    50 memory lines and the 50 time lines of lowest id - each with its
    neighbours."""
    t = [0] * 400
    m = [0] * 400
    for l in range(100):
        t[l] = 1
    for l in range(300, 350):
        m[l] = 2
    got = _rl(time=t, mem=m)
    assert got == list(range(0, 51)) + list(range(299, 351))
    assert len(got) <= 300
    # 101 qualify: line 290 by time (99 % of it) and lines 150-249 by memory
    # (exactly 1 % each); of the tied memory lines the highest id drops out
    t = [0] * 300
    m = [0] * 300
    for l in range(101):
        t[l] = 100    # 101 lines at 100/1,010,100 each: far below 1 % of the time
    t[290] = 1_000_000
    for l in range(150, 250):
        m[l] = 1
    assert _rl(time=t, mem=m) == list(range(149, 250)) + [289, 290, 291]


@pytest.mark.parametrize("seed", range(8))
def test_report_lines_bounds(seed):
    """At most 100 lines can hold 1 % of one total, so one criterion alone
    selects at most 300 lines with neighbours, the same as with no cap; both
    criteria together also stay within 300 and within the union of the two
    selections.  Flat distributions (seeds 6, 7) make over 100 lines qualify."""
    rng = np.random.default_rng(seed)
    L = int(rng.integers(1, 5000))
    if seed < 6:
        t = (rng.pareto(1.0 + seed / 3, L) * 100).astype(np.int64)
        m = (rng.pareto(0.8 + seed / 4, L) * 1000).astype(np.int64)
    else:
        L = 5000
        t = np.where(np.arange(L) < 100, 100, 0).astype(np.int64)
        m = np.where((np.arange(L) >= 2000) & (np.arange(L) < 2100), rng.integers(90, 110, L), 0).astype(np.int64)
    z = np.zeros(L, np.int64)
    sel_t = oracle.report_lines(t, z, z)
    sel_m = oracle.report_lines(z, z, m)
    both = oracle.report_lines(t, z, m)
    assert len(sel_t) <= 300 and len(sel_m) <= 300 and len(both) <= 300
    assert set(both.tolist()) <= set(sel_t.tolist()) | set(sel_m.tolist())
    if seed >= 6:
        # over 100 lines qualify: exactly 100 remain, each with its neighbours
        assert 100 <= len(both) <= 300


# ------------------------------------------------ leak report (3.4) --

def _samples(xs, ys):
    s = np.zeros(len(xs), oracle.SAMPLE_DTYPE)
    s["event_idx"] = xs
    s["F"] = ys
    return s


def test_leak_report_slope_hand_cases():
    """Section 3.4: leaks are reported only when overall memory grows by at
    least 1 % (read as the fitted rise over the sampled span against the
    peak sampled footprint)."""
    g = np.ones(3, np.uint8)
    z = np.zeros(3, np.int64)
    ok, rep, _ = oracle.leak_report(_samples(range(10), [10 * i for i in range(10)]), g, z, z)
    assert ok and rep.tolist() == [1, 1, 1]                  # a straight rise
    ok, _, _ = oracle.leak_report(_samples(range(10), [50] * 10), g, z, z)
    assert not ok                                              # flat: slope 0
    ok, _, _ = oracle.leak_report(_samples(range(10), [90 - 10 * i for i in range(10)]), g, z, z)
    assert not ok                                              # falling
    ok, _, _ = oracle.leak_report(_samples([5], [100]), g, z, z)
    assert not ok                                              # one sample
    # two samples: slope (y1 - y0) / (x1 - x0), rise y1 - y0, peak max(y0, y1)
    ok, _, _ = oracle.leak_report(_samples([0, 7], [1000, 1010]), g, z, z)
    assert not ok                                              # rise 10 of peak 1010: 1000 < 1010
    ok, _, _ = oracle.leak_report(_samples([0, 7], [990, 1000]), g, z, z)
    assert ok                                                  # rise 10 of peak 1000: exactly 1 %
    ok, _, _ = oracle.leak_report(_samples([0, 7], [991, 1000]), g, z, z)
    assert not ok                                              # rise 9 of peak 1000: 900 < 1000
    ok, rep, _ = oracle.leak_report(_samples(range(4), [0, 1, 2, 3]), np.array([1, 0, 1], np.uint8), z, z)
    assert rep.tolist() == [1, 0, 1]                           # gate and slope
    ok, _, el = oracle.leak_report(_samples([0], [0]), g, np.array([5, 6, 7]), np.array([1, 2, 3]))
    assert el == 24


@pytest.mark.parametrize("seed", range(5))
def test_leak_report_slope_against_float_fit(seed):
    """Away from the 1 % boundary the exact decision agrees with a
    floating-point least-squares fit (numpy.polyfit), an independent
    formulation."""
    rng = np.random.default_rng(seed)
    for _ in range(40):
        K = int(rng.integers(2, 400))
        x = np.sort(rng.choice(1 << 20, K, replace=False)).astype(np.int64)
        trend = rng.normal(0, 2e-3)
        y = (1e6 + trend * 1e6 * (x - x[0]) / max(1, x[-1] - x[0]) + rng.normal(0, 1e3, K)).astype(np.int64)
        b = np.polyfit(x.astype(np.float64), y.astype(np.float64), 1)[0]
        rise = b * (x[-1] - x[0])
        ratio = 100 * rise / y.max()
        if abs(ratio - 1) < 0.01:
            continue
        ok, _, _ = oracle.leak_report(_samples(x, y), np.ones(1, np.uint8), np.zeros(1, np.int64),
                                      np.zeros(1, np.int64))
        assert ok == (ratio >= 1), (K, ratio)


# ------------------------------------- per-line timelines and RDP (5) --

def _tl(xs, ys, lines=0, L=1, max_points=100):
    s = np.zeros(len(xs), oracle.SAMPLE_DTYPE)
    s["event_idx"] = xs
    s["F"] = ys
    s["line"] = lines
    return oracle.timeline_points(s, L, max_points)


def _float_rdp(x, y, eps):
    """Textbook recursive RDP in floating point (an independent formulation)."""
    def rec(i, j, out):
        if j - i < 2:
            return
        dx, dy = x[j] - x[i], y[j] - y[i]
        d = [abs(dx * (y[k] - y[i]) - dy * (x[k] - x[i])) / np.hypot(dx, dy) for k in range(i + 1, j)]
        k = int(np.argmax(d)) + i + 1
        if d[k - i - 1] > eps:
            out.add(k)
            rec(i, k, out)
            rec(k, j, out)
    out = {0, len(x) - 1}
    rec(0, len(x) - 1, out)
    return sorted(out)


def test_timeline_hand_cases():
    """Section 5: each line's footprint log reduced by RDP to about 100
    points."""
    assert _tl(range(5), [0, 10, 20, 30, 40]).tolist() == [1, 0, 0, 0, 1]     # collinear: the chord
    assert _tl(range(5), [0, 0, 50, 0, 0]).tolist() == [1] * 5                # nothing collinear, <= 100
    y = [7 * i for i in range(1000)]
    y[400] += 1 << 40
    k = _tl(range(1000), y)
    assert np.flatnonzero(k).tolist() == [0, 399, 400, 401, 999]              # a line and one spike: its corners
    assert _tl([3], [5]).tolist() == [1] and _tl([], []).tolist() == []


def test_timeline_lines_are_independent():
    rng = np.random.default_rng(3)
    n = 900
    x = np.arange(n) * 3
    y = np.cumsum(rng.integers(-1000, 1000, n))
    lines = rng.integers(0, 4, n)
    both = _tl(x, y, lines, L=4)
    for l in range(4):
        m = lines == l
        alone = _tl(x[m], y[m])
        assert both[m].tolist() == alone.tolist()


@pytest.mark.parametrize("seed", range(4))
def test_timeline_bound_and_minimal_eps(seed):
    """At most 100 points per line, always the first and last sample; the
    chosen eps is the smallest candidate that gets there, so the next smaller
    one keeps more than 100; and the kept set equals a floating-point
    recursive RDP at that eps (random walks: no ties at the threshold)."""
    rng = np.random.default_rng(seed)
    n = int(rng.integers(150, 1200))
    x = np.cumsum(rng.integers(1, 50, n))
    y = np.cumsum(rng.normal(0, 1e5, n)).astype(np.int64)
    k = _tl(x, y)
    kept = np.flatnonzero(k).tolist()
    assert len(kept) <= 100 and kept[0] == 0 and kept[-1] == n - 1
    xi, yi = [int(v) for v in x], [int(v) for v in y]
    cands = [0] + [1 << e for e in range(63)]
    eps = next(e for e in cands if len(oracle._rdp_keep(xi, yi, e * e)) <= 100)
    prev = cands[cands.index(eps) - 1] if eps else None
    if prev is not None:
        assert len(oracle._rdp_keep(xi, yi, prev * prev)) > 100
    assert kept == _float_rdp(np.array(x, float), np.array(y, float), float(eps))


# ------------------------------------- timelines, the paper's procedure (5) --

def test_splitmix64_matches_its_published_outputs():
    """The first outputs of splitmix64 from state 0, as published with the
    generator, and the input generator's own implementation (written
    separately) for other states."""
    import tracegen as tg
    g = oracle.splitmix64(0)
    assert [next(g) for _ in range(3)] == [0xE220A8397B1DCDAF, 0x6E789E6AA1B965F4, 0x06C45D188009454F]
    for s in (1, 12345, (1 << 64) - 1, 0x9E3779B97F4A7C15):
        assert next(oracle.splitmix64(s)) == tg.lib().tg_splitmix64(s)


def test_selection_sampling_is_uniform():
    """Algorithm S takes exactly k of N candidates, in order, and every
    k-subset is equally likely: over 20,000 seeds each of the 10 subsets of
    2 out of 5 appears 2,000 times give or take ~42 (one standard
    deviation); a bias of a few per cent in any draw would show."""
    from collections import Counter
    counts = Counter()
    for seed in range(20_000):
        sel = oracle.select_uniform(list(range(5)), 2, oracle.splitmix64(seed))
        assert len(sel) == 2 and sel == sorted(sel)
        counts[tuple(sel)] += 1
    assert len(counts) == 10
    assert all(abs(c - 2000) < 250 for c in counts.values()), counts
    assert oracle.select_uniform(list(range(7)), 7, oracle.splitmix64(3)) == list(range(7))
    assert oracle.select_uniform(list(range(7)), 0, oracle.splitmix64(3)) == []


def test_timeline_points_sampled_follows_the_paper():
    """Section 5: RDP with an approximate eps, then logs still longer than
    the limit downsampled at random to exactly the limit."""
    def samples(points):
        s = np.zeros(len(points), oracle.SAMPLE_DTYPE)
        for i, (line, x, y) in enumerate(points):
            s[i] = (x, line, y, 0, 0)
        return s
    # a zigzag of 40 points 1000 apart with range 1000 and a limit of 10:
    # eps = 100; every corner lies ~1000 from its chord, so RDP keeps all 40
    # and the random step keeps exactly 10 of them, chosen by the seed
    zig = [(0, 1000 * i, 1000 if i % 2 else 0) for i in range(40)]
    k1 = oracle.timeline_points_sampled(samples(zig), 1, max_points=10, seed=1)
    k2 = oracle.timeline_points_sampled(samples(zig), 1, max_points=10, seed=2)
    assert k1.sum() == 10 and k2.sum() == 10 and not np.array_equal(k1, k2)
    # a straight ramp: RDP keeps the two ends only, the random step never
    # applies and the seed does not matter
    ramp = [(0, 1000 * i, 5000 * i) for i in range(40)]
    for seed in range(3):
        assert np.flatnonzero(oracle.timeline_points_sampled(samples(ramp), 1, 10, seed)).tolist() == [0, 39]
    # eps = range // limit: points (0,0) (1000,b) (2000,0) (3000,0) (4000,100)
    # have range 100, so eps = 10 with a limit of 10.  The chord of the whole
    # run puts (3000,0) farthest (kept); on the chord (0,0)-(3000,0) the point
    # (1000,b) lies exactly b away: kept only when b > 10 (strict), and then
    # (2000,0) lies 5.5 from its new chord and is dropped.
    for b, want in ((10, [0, 3, 4]), (11, [0, 1, 3, 4])):
        pts = [(0, 0, 0), (0, 1000, b), (0, 2000, 0), (0, 3000, 0), (0, 4000, 100)]
        assert np.flatnonzero(oracle.timeline_points_sampled(samples(pts), 1, 10, 0)).tolist() == want, b
    # lines are separate: line 0 is downsampled, line 1 keeps its RDP points
    # (a short zigzag: every point kept, 5 <= 10), line 2 is out of range
    mix = zig + [(1, 1000 * i, 1000 if i % 2 else 0) for i in range(5)] + [(2, 5, 5)]
    k = oracle.timeline_points_sampled(samples(mix), 2, max_points=10, seed=9)
    assert k[:40].sum() == 10 and k[40:45].tolist() == [1] * 5 and k[45] == 0
