"""Host-side checks of the C-ABI library (no GPU calls)."""
import ctypes
import os
import re
import subprocess

import numpy as np

import paper_2212_07597_amd as smp
from paper_2212_07597_amd import _build

HEADER = os.path.join(_build.ROOT, "include", "scalene_sampler.h")


def declared_functions():
    src = open(HEADER).read()
    return re.findall(r"SMP_API\s+[\w\s\*]+?\b(\w+)\s*\(", src)


def test_library_exports_every_declared_symbol():
    names = declared_functions()
    assert set(names) == set(smp.EXPORTED)
    out = subprocess.run(["nm", "-D", "--defined-only", _build.LIB_PATH], capture_output=True, text=True).stdout
    exported = {line.split()[-1] for line in out.splitlines() if " T " in line}
    missing = [n for n in names if n not in exported]
    assert not missing, missing
    L = smp.lib()
    for n in names:
        assert hasattr(L, n)


def test_library_is_built_for_gfx950():
    # the offload bundle of our own build names its target
    blob = open(_build.LIB_PATH, "rb").read()
    assert b"amdgcn-amd-amdhsa--gfx950" in blob


def test_error_strings():
    for code in range(0, 9):
        s = smp.error_string(code)
        assert s and s != "unknown status"
    assert smp.error_string(99) == "unknown status"


def test_workspace_bytes_host_logic():
    p = smp.make_params(1 << 20, 64)
    a = smp.workspace_bytes(1000, p, ev_on_device=True)
    b = smp.workspace_bytes(1000, p, ev_on_device=False)
    assert a > 0 and b >= a + 24 * 1000
    assert smp.workspace_bytes(2000, p) > a
    # linear growth: about 52 bytes of output capacity per event plus small terms
    big = smp.workspace_bytes(10_000_000, p)
    assert 50 * 10_000_000 < big < 60 * 10_000_000
    # invalid parameters give 0
    assert smp.workspace_bytes(10, smp.make_params(0, 64)) == 0
    assert smp.workspace_bytes(10, smp.make_params(10, 0)) == 0
    assert smp.workspace_bytes(10, smp.Params(10, 10, 4, 0, 8, 0)) == 0
    assert smp.workspace_bytes(1 << 32, p) == 0
    assert smp.sampler_fixed_bytes() > 0


def test_create_rejects_bad_workspace_without_touching_the_gpu():
    h = ctypes.c_void_p()
    L = smp.lib()
    assert L.sampler_create(0, None, 0, None, 1 << 20, ctypes.byref(h)) == smp.SMP_EINVAL
    assert L.sampler_create(0, None, 0, ctypes.c_void_p(0x1001), 1 << 20, ctypes.byref(h)) == smp.SMP_EINVAL
    assert L.sampler_create(0, None, 0, ctypes.c_void_p(0x1000), 16, ctypes.byref(h)) == smp.SMP_EINVAL


def test_record_layouts_match_header():
    assert smp.SAMPLE_DTYPE.itemsize == 24 + 8  # 32-byte sample
    assert smp.TRACKED_DTYPE.itemsize == 16
    assert ctypes.sizeof(smp.Params) == 32
    assert ctypes.sizeof(smp.Tuning) == 20  # five uint32 fields, as smp_tuning_t


def test_report_lines_matches_oracle():
    """The library's report line filter (host code) against the oracle's, on
    skewed, flat, sparse and negative per-line values, edge sizes included."""
    import oracle

    rng = np.random.default_rng(7)
    sizes = [0, 1, 2, 3, 99, 100, 101, 300, 5000, 20000]
    for i, L in enumerate(sizes * 4):
        kind = i // len(sizes)
        if kind == 0:    # skewed
            py = (rng.pareto(1.1, L) * 50).astype(np.int64)
            nat = (rng.pareto(1.5, L) * 50).astype(np.int64)
            gb = (rng.pareto(0.9, L) * 1e6).astype(np.int64)
        elif kind == 1:  # flat with a few large lines, many zeros
            py = np.where(rng.random(L) < 0.3, 1, 0).astype(np.int64)
            nat = np.zeros(L, np.int64)
            gb = np.where(rng.random(L) < 0.01, 1 << 40, 0).astype(np.int64)
        elif kind == 2:  # signed values (per-line sums wrap modulo 2^64)
            py = rng.integers(-1000, 1000, L).astype(np.int64)
            nat = rng.integers(-10, 10, L).astype(np.int64)
            gb = rng.integers(-(1 << 62), 1 << 62, L).astype(np.int64)
        else:            # over 100 lines qualify: 100 at exactly 1 % of the time, and 40 at
                         # 2 % and 20 at 1 % of the memory (ties of equal shares across criteria)
            py = np.zeros(L, np.int64)
            nat = np.zeros(L, np.int64)
            gb = np.zeros(L, np.int64)
            if L >= 100:
                py[rng.choice(L, 100, replace=False)] = 7
                ids = rng.choice(L, min(L, 60), replace=False)
                gb[ids[:40]] = 2 << 30
                gb[ids[40:]] = 1 << 30
        got = smp.report_lines(py, nat, gb)
        want = oracle.report_lines(py, nat, gb)
        assert got.tolist() == want.tolist(), (L, kind)


def test_leak_report_matches_oracle():
    """The library's growth test (exact, on 256-bit integers of four limbs)
    against the oracle's Python integers: random sample sets from tiny to
    extreme magnitudes (event indices near 2^32, footprints near +-2^60),
    and two-sample sets placed exactly on and around the 1 % boundary."""
    import oracle

    rng = np.random.default_rng(11)
    L = 5
    gate = np.array([1, 0, 1, 1, 0], np.uint8)
    py = rng.integers(-(1 << 62), 1 << 62, L).astype(np.int64)
    nat = rng.integers(-(1 << 62), 1 << 62, L).astype(np.int64)

    def both(x, y):
        s = np.zeros(len(x), smp.SAMPLE_DTYPE)
        s["event_idx"] = x
        s["F"] = y
        got = smp.leak_report(s, gate, py, nat)
        want = oracle.leak_report(s, gate, py, nat)
        assert got[0] == want[0] and got[1].tolist() == want[1].tolist() and got[2] == want[2], (x[:4], y[:4])
        return got[0]

    seen = set()
    for trial in range(300):
        K = int(rng.integers(0, 3000 if trial % 10 else 20))
        top = [1 << 10, 1 << 20, (1 << 32) - 1][trial % 3]
        x = np.sort(rng.choice(top, min(K, top), replace=False)).astype(np.uint32)
        mag_ = [1 << 20, 1 << 40, 1 << 60][(trial // 3) % 3]
        base = int(rng.integers(-mag_, mag_))
        drift = rng.normal(0, mag_ / 50)
        y = np.clip(base + drift * np.linspace(0, 1, len(x)) + rng.normal(0, mag_ / 100, len(x)),
                    -(1 << 60), 1 << 60).astype(np.int64)
        seen.add(both(x, y))
    assert seen == {True, False}
    # exactly 1 %: rise r of peak 100 r passes, peak 100 r + 1 does not
    for r in (1, 7, 1 << 20, 1 << 50):
        for peak, want in ((100 * r, True), (100 * r + 1, False)):
            assert both(np.array([3, (1 << 32) - 1], np.uint32), np.array([peak - r, peak], np.int64)) == want


def test_timeline_points_match_oracle():
    """The library's per-line RDP (iterative, binary search over eps, 256-bit
    distance test) against the oracle's on random multi-line sample sets,
    from small values to event indices near 2^32 and footprints near 2^60,
    including lines with fewer than max_points samples and out-of-range
    lines."""
    import oracle

    rng = np.random.default_rng(5)
    for trial in range(40):
        K = int(rng.integers(0, 4000))
        L = int(rng.integers(1, 9))
        x = np.sort(rng.choice((1 << 32) - 1 if trial % 2 else 1 << 16, K, replace=False)).astype(np.uint32)
        scale = [1e2, 1e9, 1e16][trial % 3]
        y = np.clip(np.cumsum(rng.normal(0, scale, K)), -(1 << 60), 1 << 60).astype(np.int64)
        s = np.zeros(K, smp.SAMPLE_DTYPE)
        s["event_idx"] = x
        s["F"] = y
        s["line"] = rng.integers(0, L + 1, K)  # line L is out of range: no timeline
        mp = [100, 2, 7][trial % 3]
        got = smp.timeline_points(s, L, mp)
        want = oracle.timeline_points(s, L, mp)
        assert got.tolist() == want.tolist(), (trial, K, L)


def test_rate_noalloc_refuses_sizes_over_its_scratch_on_the_host():
    # the size and argument checks come before any device call, so this runs
    # without a GPU: one dummy record pointer with a count above the maximum
    dummy = (ctypes.c_uint8 * 24)()
    out = (ctypes.c_int64 * 4)()
    res = (ctypes.c_uint64 * 2)()
    L = smp.lib()
    rc = L.rate_run_noalloc(ctypes.addressof(dummy), smp.RATE_NOALLOC_MAX_EVENTS + 1, 10, 4,
                            ctypes.addressof(out), ctypes.addressof(res), None)
    assert rc == smp.SMP_ETOOBIG
    # invalid arguments: threshold 0, no line counts
    assert L.rate_run_noalloc(ctypes.addressof(dummy), 1, 0, 4, ctypes.addressof(out), ctypes.addressof(res),
                              None) == smp.SMP_EINVAL
    assert L.rate_run_noalloc(ctypes.addressof(dummy), 1, 10, 4, None, ctypes.addressof(res), None) == smp.SMP_EINVAL
    # the header's maximum and the binding's agree
    src = open(HEADER).read()
    assert "#define SMP_RATE_NOALLOC_MAX_EVENTS (1ull << 29)" in src and smp.RATE_NOALLOC_MAX_EVENTS == 1 << 29


def test_timeline_points_sampled_matches_oracle():
    """The library's RDP-plus-downsampling timelines against the oracle's:
    random walks on several lines, limits small enough that the random step
    applies, several seeds, magnitudes up to event indices near 2^32 and
    footprints near 2^60."""
    import oracle

    rng = np.random.default_rng(5)
    for case in range(40):
        n = int(rng.integers(0, 600))
        L = int(rng.integers(1, 6))
        s = np.zeros(n, smp.SAMPLE_DTYPE)
        s["event_idx"] = np.sort(rng.integers(0, 1 << (32 if case % 3 == 0 else 20), n))
        scale = 1 << (60 if case % 4 == 0 else 20)
        s["F"] = np.clip(np.cumsum(rng.integers(-scale // 64, scale // 64, n)), -(1 << 60), 1 << 60)
        s["line"] = rng.integers(0, L + 1, n)  # line L is out of range
        maxp = int(rng.choice([2, 3, 10, 100]))
        seed = int(rng.integers(0, 1 << 63))
        got = smp.timeline_points_sampled(s, L, maxp, seed)
        want = oracle.timeline_points_sampled(s, L, maxp, seed)
        assert got.tolist() == want.tolist(), case
        for line in range(L):
            assert got[s["line"] == line].sum() <= maxp
