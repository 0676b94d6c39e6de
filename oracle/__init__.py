"""CPU oracle for the threshold sampler - TEST INFRASTRUCTURE ONLY.

Only ``tests/``, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may import this package.  The product path never does.

``oracle.c`` (built to ``liboracle.so`` by ``__graft_entry__.build()``) is a
single sequential loop in the paper's counter form (section 3.2 for sampling,
3.3 for sample contents, 3.4 for the leak rule and score, 3.5 for copy volume,
2.1 for the Python/native time split).  This module only marshals arguments.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "liboracle.so")

OK, EINVAL, EOVERFLOW, ENOMEM = 0, 1, 6, 7
OPT_PRIME_T, OPT_RESOLVE_AT_END = 1, 2

HIST_NAMES = (
    "py_bytes", "nat_bytes", "growth_n", "shrink_n", "growth_bytes", "shrink_bytes",
    "leak_mallocs", "leak_frees", "copy_sampled", "copy_exact", "py_time_us", "nat_time_us",
)

SAMPLE_DTYPE = np.dtype([("event_idx", "<u4"), ("line", "<u4"), ("F", "<i8"), ("py", "<i8"), ("nat", "<i8")])
TRACKED_DTYPE = np.dtype([("event_idx", "<u4"), ("line", "<u4"), ("ptr", "<u4"), ("freed", "<u4")])


class _Params(ctypes.Structure):
    _fields_ = [
        ("threshold", ctypes.c_int64),
        ("copy_threshold", ctypes.c_int64),
        ("num_lines", ctypes.c_uint32),
        ("quantum_us", ctypes.c_uint32),
        ("options", ctypes.c_uint32),
        ("reserved", ctypes.c_uint32),
    ]


class _Result(ctypes.Structure):
    _fields_ = [
        ("status", ctypes.c_int),
        ("num_lines", ctypes.c_uint32),
        ("threshold_used", ctypes.c_int64),
        ("n_samples", ctypes.c_uint64),
        ("n_tracked", ctypes.c_uint64),
        ("final_F", ctypes.c_int64),
        ("peak_F", ctypes.c_int64),
        ("peak_sampled_F", ctypes.c_int64),
        ("samples", ctypes.c_void_p),
        ("tracked", ctypes.c_void_p),
        ("hist", ctypes.c_void_p),
        ("samples_cap", ctypes.c_uint64),
        ("tracked_cap", ctypes.c_uint64),
    ]


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is not built; run __graft_entry__.build()")
        L = ctypes.CDLL(LIB_PATH)
        L.oracle_run.argtypes = [ctypes.c_void_p, ctypes.c_uint64, ctypes.POINTER(_Params),
                                 ctypes.POINTER(ctypes.POINTER(_Result))]
        L.oracle_run.restype = ctypes.c_int
        L.oracle_free.argtypes = [ctypes.POINTER(_Result)]
        L.oracle_free.restype = None
        L.oracle_prime_at_least.argtypes = [ctypes.c_int64]
        L.oracle_prime_at_least.restype = ctypes.c_int64
        p64 = ctypes.POINTER(ctypes.c_int64)
        p8 = ctypes.POINTER(ctypes.c_uint8)
        L.oracle_leak_scores.argtypes = [p64, p64, ctypes.c_uint32, p64, p64, p64, p64, p8, p8]
        L.oracle_rate.argtypes = [ctypes.c_void_p, ctypes.c_uint64, ctypes.c_int64, ctypes.c_uint32,
                                  ctypes.POINTER(ctypes.c_int64), ctypes.POINTER(ctypes.c_uint64)]
        L.oracle_rate.restype = ctypes.c_int
        L.oracle_leak_scores.restype = None
        _lib = L
    return _lib


def prime_at_least(t: int) -> int:
    return int(lib().oracle_prime_at_least(t))


def _ptr(a, ct):
    return a.ctypes.data_as(ctypes.POINTER(ct))


def leak_scores(mallocs, frees):
    """Exact reduced rationals (Laplace and as-printed) and 95 % gates per line."""
    m = np.ascontiguousarray(mallocs, dtype=np.int64)
    f = np.ascontiguousarray(frees, dtype=np.int64)
    n = m.shape[0]
    out = {k: np.empty(n, np.int64) for k in ("lap_num", "lap_den", "lit_num", "lit_den")}
    out["lap_gate"] = np.empty(n, np.uint8)
    out["lit_gate"] = np.empty(n, np.uint8)
    lib().oracle_leak_scores(_ptr(m, ctypes.c_int64), _ptr(f, ctypes.c_int64), n,
                             _ptr(out["lap_num"], ctypes.c_int64), _ptr(out["lap_den"], ctypes.c_int64),
                             _ptr(out["lit_num"], ctypes.c_int64), _ptr(out["lit_den"], ctypes.c_int64),
                             _ptr(out["lap_gate"], ctypes.c_uint8), _ptr(out["lit_gate"], ctypes.c_uint8))
    return out


def run(events, threshold, num_lines, copy_threshold=None, quantum_us=10_000, options=0):
    """Run the sequential sampler over a 24-byte-record event array.

    Returns a dict: status, samples (SAMPLE_DTYPE), tracked (TRACKED_DTYPE), the
    twelve per-line int64 arrays, final_F, peak_F, peak_sampled_F,
    threshold_used, K, H and the leak rationals/gates.
    """
    ev = np.ascontiguousarray(events)
    if ev.dtype.itemsize != 24:
        raise ValueError("events must be 24-byte records")
    p = _Params(int(threshold), int(copy_threshold if copy_threshold is not None else threshold),
                int(num_lines), int(quantum_us), int(options), 0)
    rp = ctypes.POINTER(_Result)()
    lib().oracle_run(ev.ctypes.data if ev.size else None, ev.shape[0], ctypes.byref(p), ctypes.byref(rp))
    try:
        r = rp.contents
        out = {"status": int(r.status), "threshold_used": int(r.threshold_used)}
        if r.status != OK:
            return out
        K, H, L = int(r.n_samples), int(r.n_tracked), int(r.num_lines)
        out["K"], out["H"] = K, H
        out["samples"] = (np.ctypeslib.as_array(ctypes.cast(r.samples, ctypes.POINTER(ctypes.c_uint8)),
                                                shape=(K * SAMPLE_DTYPE.itemsize,)).view(SAMPLE_DTYPE).copy()
                          if K else np.zeros(0, SAMPLE_DTYPE))
        out["tracked"] = (np.ctypeslib.as_array(ctypes.cast(r.tracked, ctypes.POINTER(ctypes.c_uint8)),
                                                shape=(H * TRACKED_DTYPE.itemsize,)).view(TRACKED_DTYPE).copy()
                          if H else np.zeros(0, TRACKED_DTYPE))
        hist = np.ctypeslib.as_array(ctypes.cast(r.hist, ctypes.POINTER(ctypes.c_int64)),
                                     shape=(len(HIST_NAMES) * L,)).copy().reshape(len(HIST_NAMES), L)
        for k, name in enumerate(HIST_NAMES):
            out[name] = hist[k]
        out["final_F"] = int(r.final_F)
        out["peak_F"] = int(r.peak_F)
        out["peak_sampled_F"] = int(r.peak_sampled_F)
        out.update(leak_scores(out["leak_mallocs"], out["leak_frees"]))
        return out
    finally:
        lib().oracle_free(rp)


def rate(events, threshold, num_lines, options=0):
    """Deterministic rate-based sampling (section 3.2): one sample per T bytes
    allocated or freed.  Returns (status, K, samples per line)."""
    ev = np.ascontiguousarray(events)
    T = prime_at_least(threshold) if options & OPT_PRIME_T else threshold
    counts = np.zeros(num_lines, np.int64)
    K = ctypes.c_uint64(0)
    st = lib().oracle_rate(ev.ctypes.data if ev.size else None, ev.shape[0], T, num_lines,
                           counts.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)), ctypes.byref(K))
    return int(st), int(K.value), counts


def report_lines(py_time, nat_time, growth_bytes, max_qualifying=100):
    """Report line filter (section 5): the lines with at least 1 % of the
    execution time or at least 1 % of the memory, each with the line before
    and the line after it, never more than 300 lines in all.  A line's time
    is py_time + nat_time, its memory its growth bytes; only positive values
    count, in the totals and as shares.  The paper's bound holds for one
    criterion (at most 100 lines can hold 1 % of one total); with both, the
    100 qualifying lines with the largest share are kept, a line's share
    being the larger of its time share and its memory share (ties: the lower
    line id).  Exact rational arithmetic; returns the ids ascending."""
    from fractions import Fraction

    L = len(py_time)
    t = [int(py_time[l]) + int(nat_time[l]) for l in range(L)]
    m = [int(growth_bytes[l]) for l in range(L)]
    tot_t = sum(x for x in t if x > 0)
    tot_m = sum(x for x in m if x > 0)
    share = {}
    for l in range(L):
        by_time = t[l] > 0 and 100 * t[l] >= tot_t
        by_mem = m[l] > 0 and 100 * m[l] >= tot_m
        if by_time or by_mem:
            st = Fraction(t[l], tot_t) if t[l] > 0 else Fraction(0)
            sm = Fraction(m[l], tot_m) if m[l] > 0 else Fraction(0)
            share[l] = max(st, sm)
    kept = sorted(share, key=lambda l: (-share[l], l))[:max_qualifying]
    out = set()
    for l in kept:
        out.update(c for c in (l - 1, l, l + 1) if 0 <= c < L)
    return np.array(sorted(out), dtype=np.uint32)


def _wrap64(v):
    v &= (1 << 64) - 1
    return v - (1 << 64) if v >> 63 else v


def leak_report(samples, gate, py_time_us, nat_time_us):
    """Leak report filter (section 3.4), in Python's exact integers.

    The slope of overall memory growth: the least-squares line of the
    sampled footprint F against the event index over the K samples; it
    passes when its rise over the sampled span is at least 1 % of the peak
    sampled footprint: 100 b (x_K - x_1) >= max F, b = (K Sxy - Sx Sy) /
    (K Sxx - Sx^2).  K < 2 or a peak <= 0 never passes.  A line's leak is
    reported when its likelihood gate is set and the slope passes.  The
    elapsed time that a leak rate divides by is the trace's total Python plus
    native time (the per-line values summed modulo 2^64, as they wrap).
    Returns (slope_ok, reported per line, elapsed_us)."""
    x = [int(v) for v in samples["event_idx"]]
    y = [int(v) for v in samples["F"]]
    K = len(x)
    ok = False
    if K >= 2 and max(y) > 0:
        Sx, Sy = sum(x), sum(y)
        Sxx = sum(v * v for v in x)
        Sxy = sum(a * b for a, b in zip(x, y))
        num = K * Sxy - Sx * Sy
        den = K * Sxx - Sx * Sx
        ok = den > 0 and 100 * num * (x[-1] - x[0]) >= max(y) * den
    reported = (np.asarray(gate, np.uint8) != 0) & ok
    elapsed = _wrap64(sum(int(a) + int(b) for a, b in zip(py_time_us, nat_time_us)))
    return ok, reported.astype(np.uint8), elapsed


def _rdp_keep(x, y, eps2):
    """Ramer-Douglas-Peucker over the points (x[i], y[i]), exact: a point is
    kept when its distance from the chord of its run exceeds eps, i.e.
    cross^2 > eps^2 (dx^2 + dy^2); the farthest point of a run (the first
    on ties) splits it.  Returns the kept indices, ascending."""
    n = len(x)
    if n <= 2:
        return list(range(n))
    keep = {0, n - 1}
    runs = [(0, n - 1)]
    while runs:
        i, j = runs.pop()
        if j - i < 2:
            continue
        dx, dy = x[j] - x[i], y[j] - y[i]
        best, bk = -1, -1
        for k in range(i + 1, j):
            c = abs(dx * (y[k] - y[i]) - dy * (x[k] - x[i]))
            if c > best:
                best, bk = c, k
        if best * best > eps2 * (dx * dx + dy * dy):
            keep.add(bk)
            runs.append((i, bk))
            runs.append((bk, j))
    return sorted(keep)


def timeline_points(samples, num_lines, max_points=100):
    """Per-line memory timelines (section 5): each line's samples in rank
    order as points (event index, footprint), reduced by RDP with the
    smallest eps in {0, 1, 2, 4, ..., 2^62} that leaves at most max_points
    points.  Returns a keep flag per sample."""
    lines = [int(v) for v in samples["line"]]
    xs = [int(v) for v in samples["event_idx"]]
    ys = [int(v) for v in samples["F"]]
    by_line = {}
    for r, l in enumerate(lines):
        if l < num_lines:
            by_line.setdefault(l, []).append(r)
    keep = np.zeros(len(lines), np.uint8)
    cands = [0] + [1 << e for e in range(63)]
    for l, idx in by_line.items():
        x = [xs[r] for r in idx]
        y = [ys[r] for r in idx]
        chosen = None
        for eps in cands:   # the kept set only shrinks as eps grows
            kept = _rdp_keep(x, y, eps * eps)
            if len(kept) <= max_points:
                chosen = kept
                break
        for k in chosen:
            keep[idx[k]] = 1
    return keep


_M64 = (1 << 64) - 1


def splitmix64(state):
    """The splitmix64 generator (Steele, Lea and Flood, 2014): yields its
    outputs from the given 64-bit state."""
    while True:
        state = (state + 0x9E3779B97F4A7C15) & _M64
        z = state
        z = ((z ^ (z >> 30)) * 0xBF58476D1CE4E5B9) & _M64
        z = ((z ^ (z >> 27)) * 0x94D049BB133111EB) & _M64
        yield z ^ (z >> 31)


def select_uniform(candidates, k, gen):
    """Selection sampling (Knuth, TAOCP vol. 2, 3.4.2, Algorithm S): a
    uniform k-subset of candidates, in order.  The t-th of N candidates is
    taken with probability (k - m) / (N - t), m the number taken so far,
    drawn as floor(x (N - t) / 2^64) < k - m for x the next output of gen."""
    n = len(candidates)
    out = []
    for t, c in enumerate(candidates):
        if len(out) == k:
            break
        x = next(gen)
        if (x * (n - t)) >> 64 < k - len(out):
            out.append(c)
    return out


def timeline_points_sampled(samples, num_lines, max_points=100, seed=0):
    """Per-line memory timelines by the paper's procedure (section 5): RDP
    with an approximate eps, the line's footprint range over max_points
    (integer division), then every log still longer than max_points
    downsampled at random to exactly max_points of its RDP points (uniform,
    by selection sampling on splitmix64 started at seed + line).  Returns a
    keep flag per sample."""
    lines = [int(v) for v in samples["line"]]
    xs = [int(v) for v in samples["event_idx"]]
    ys = [int(v) for v in samples["F"]]
    by_line = {}
    for r, l in enumerate(lines):
        if l < num_lines:
            by_line.setdefault(l, []).append(r)
    keep = np.zeros(len(lines), np.uint8)
    for l, idx in by_line.items():
        x = [xs[r] for r in idx]
        y = [ys[r] for r in idx]
        eps = (max(y) - min(y)) // max_points
        kept = _rdp_keep(x, y, eps * eps)
        if len(kept) > max_points:
            kept = select_uniform(kept, max_points, splitmix64((seed + l) & _M64))
        for k in kept:
            keep[idx[k]] = 1
    return keep
