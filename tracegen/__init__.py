"""Seeded synthetic event traces (inputs only; none of the sampler's arithmetic).

The C source ``tracegen.c`` beside this file is compiled into
``libtracegen.so`` by ``__graft_entry__.build()``.  Every array returned here
uses the 24-byte record ``EVENT_DTYPE``.

Workload recipes (the paper's pyperformance runs are not available, so these
stand in for them; the shapes follow the paper's description of Python
memory behaviour: many small object allocations, rare large native arrays):

* ``config1`` - 1e5 events, 55 % allocations with log-uniform sizes in
  [16 B, 1 MiB], 45 % frees of a uniformly chosen live pointer, 1 % of
  allocations never freed, 64 lines Zipf(1.1), 70 % Python, T = 1 MiB.
* ``config2`` - 1e8 events; allocations are 95 % Python objects of 16*k bytes
  (k-1 geometric, p = 1/4, k <= 32) and 5 % native arrays log-uniform in
  [1 MiB, 256 MiB]; exponential lifetimes with mean 1e4 events; 0.1 % leaked;
  10,000 lines Zipf(1.2); T = 10 MiB.
* ``config3`` - 1024 traces of floor(10^(3+3u)) events with the config-1 mix,
  1,000 lines Zipf(1.1), T drawn from {256 KiB, 1 MiB, 10 MiB}.
* ``config4`` - served requests: Poisson arrivals, LogNormal(ln 5e4, 1.5)
  lengths capped at 2e7, config-1 mix, T = 1 MiB.
* ``config5`` - 5e8 events: config-1 mix plus 10 % copy events and 1 % timer
  events (delay exponential, mean 50 us); 1e6 lines Zipf(1.05); 0.01 %
  leaked; T = Tc = 64 MiB, quantum 10,000 us.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

EVENT_DTYPE = np.dtype(
    [("delta", "<i8"), ("ptr", "<u4"), ("line", "<u4"), ("flags", "u1"), ("pad", "u1", (7,))],
    align=False,
)
assert EVENT_DTYPE.itemsize == 24

KIND_MEM, KIND_COPY, KIND_TIMER = 0, 1, 2
KiB, MiB = 1 << 10, 1 << 20

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libtracegen.so")


class _MixParams(ctypes.Structure):
    _fields_ = [
        ("num_lines", ctypes.c_uint32),
        ("zipf_s", ctypes.c_double),
        ("alloc_frac", ctypes.c_double),
        ("py_frac", ctypes.c_double),
        ("leak_frac", ctypes.c_double),
        ("size_lo", ctypes.c_int64),
        ("size_hi", ctypes.c_int64),
        ("copy_frac", ctypes.c_double),
        ("timer_frac", ctypes.c_double),
        ("timer_mean_us", ctypes.c_double),
    ]


class _LifeParams(ctypes.Structure):
    _fields_ = [
        ("num_lines", ctypes.c_uint32),
        ("zipf_s", ctypes.c_double),
        ("small_frac", ctypes.c_double),
        ("geo_p", ctypes.c_double),
        ("k_max", ctypes.c_uint32),
        ("big_lo", ctypes.c_int64),
        ("big_hi", ctypes.c_int64),
        ("life_mean", ctypes.c_double),
        ("leak_frac", ctypes.c_double),
    ]


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is not built; run __graft_entry__.build()")
        L = ctypes.CDLL(LIB_PATH)
        u64, u32, dbl, vp = ctypes.c_uint64, ctypes.c_uint32, ctypes.c_double, ctypes.c_void_p
        L.tg_mix.argtypes = [u64, u64, ctypes.POINTER(_MixParams), vp]
        L.tg_mix.restype = ctypes.c_int
        L.tg_lifetime.argtypes = [u64, u64, ctypes.POINTER(_LifeParams), vp]
        L.tg_lifetime.restype = ctypes.c_int
        L.tg_plan_batch.argtypes = [u64, u32, dbl, dbl, u32, vp, vp, vp]
        L.tg_plan_batch.restype = ctypes.c_int
        L.tg_plan_serve.argtypes = [u64, u32, dbl, dbl, dbl, u64, vp, vp, vp]
        L.tg_plan_serve.restype = ctypes.c_int
        L.tg_digest.argtypes = [vp, u64]
        L.tg_digest.restype = u64
        L.tg_splitmix64.argtypes = [u64]
        L.tg_splitmix64.restype = u64
        L.tg_det_log.argtypes = [dbl]
        L.tg_det_log.restype = dbl
        L.tg_det_exp.argtypes = [dbl]
        L.tg_det_exp.restype = dbl
        _lib = L
    return _lib


def mix(seed, n, *, num_lines=64, zipf_s=1.1, alloc_frac=0.55, py_frac=0.70, leak_frac=0.01,
        size_lo=16, size_hi=MiB, copy_frac=0.0, timer_frac=0.0, timer_mean_us=50.0, out=None):
    """Uniform-live mix (configs 1, 3, 4, 5)."""
    p = _MixParams(num_lines, zipf_s, alloc_frac, py_frac, leak_frac, size_lo, size_hi,
                   copy_frac, timer_frac, timer_mean_us)
    ev = np.empty(n, dtype=EVENT_DTYPE) if out is None else out
    assert ev.dtype == EVENT_DTYPE and ev.shape[0] >= n and ev.flags.c_contiguous
    rc = lib().tg_mix(seed, n, ctypes.byref(p), ev.ctypes.data)
    if rc:
        raise RuntimeError(f"tg_mix failed: {rc}")
    return ev[:n]


def lifetime(seed, n, *, num_lines=10000, zipf_s=1.2, small_frac=0.95, geo_p=0.25, k_max=32,
             big_lo=MiB, big_hi=256 * MiB, life_mean=1e4, leak_frac=0.001, out=None):
    """Lifetime mix (config 2)."""
    p = _LifeParams(num_lines, zipf_s, small_frac, geo_p, k_max, big_lo, big_hi, life_mean, leak_frac)
    ev = np.empty(n, dtype=EVENT_DTYPE) if out is None else out
    assert ev.dtype == EVENT_DTYPE and ev.shape[0] >= n and ev.flags.c_contiguous
    rc = lib().tg_lifetime(seed, n, ctypes.byref(p), ev.ctypes.data)
    if rc:
        raise RuntimeError(f"tg_lifetime failed: {rc}")
    return ev[:n]


def digest(arr) -> int:
    a = np.ascontiguousarray(arr)
    return int(lib().tg_digest(a.ctypes.data, a.nbytes))


# ------------------------------------------------------------------ configs --

def config1(seed=1, n=100_000):
    """Returns (events, params dict)."""
    ev = mix(seed, n, num_lines=64, zipf_s=1.1, leak_frac=0.01)
    return ev, dict(threshold=MiB, copy_threshold=MiB, num_lines=64, quantum_us=10_000)


def config2(seed=2, n=100_000_000, out=None):
    ev = lifetime(seed, n, out=out)
    return ev, dict(threshold=10 * MiB, copy_threshold=10 * MiB, num_lines=10_000, quantum_us=10_000)


C3_THRESHOLDS = (256 * KiB, MiB, 10 * MiB)


def config3_plan(base_seed=3, n_traces=1024):
    lens = np.empty(n_traces, np.uint64)
    tidx = np.empty(n_traces, np.uint32)
    seeds = np.empty(n_traces, np.uint64)
    rc = lib().tg_plan_batch(base_seed, n_traces, 3.0, 6.0, len(C3_THRESHOLDS),
                             lens.ctypes.data, tidx.ctypes.data, seeds.ctypes.data)
    if rc:
        raise RuntimeError("tg_plan_batch failed")
    return [(int(lens[t]), C3_THRESHOLDS[int(tidx[t])], int(seeds[t])) for t in range(n_traces)]


def config3_trace(length, threshold, seed):
    ev = mix(seed, length, num_lines=1000, zipf_s=1.1, leak_frac=0.01)
    return ev, dict(threshold=threshold, copy_threshold=threshold, num_lines=1000, quantum_us=10_000)


def config4_plan(base_seed=4, n_req=10_000, rate=1000.0, median=5e4, sigma=1.5, cap=20_000_000):
    lens = np.empty(n_req, np.uint64)
    arr = np.empty(n_req, np.uint64)
    seeds = np.empty(n_req, np.uint64)
    rc = lib().tg_plan_serve(base_seed, n_req, rate, median, sigma, cap,
                             lens.ctypes.data, arr.ctypes.data, seeds.ctypes.data)
    if rc:
        raise RuntimeError("tg_plan_serve failed")
    return [(int(lens[i]), int(arr[i]), int(seeds[i])) for i in range(n_req)]


def config4_trace(length, seed):
    ev = mix(seed, length, num_lines=64, zipf_s=1.1, leak_frac=0.01)
    return ev, dict(threshold=MiB, copy_threshold=MiB, num_lines=64, quantum_us=10_000)


def config5(seed=5, n=500_000_000, out=None):
    ev = mix(seed, n, num_lines=1_000_000, zipf_s=1.05, leak_frac=0.0001,
             copy_frac=0.10, timer_frac=0.01, timer_mean_us=50.0, out=out)
    return ev, dict(threshold=64 * MiB, copy_threshold=64 * MiB, num_lines=1_000_000, quantum_us=10_000)


def make_events(rows):
    """Build a trace from tuples (delta, ptr, line, pn[, kind]) - for hand-written cases."""
    ev = np.zeros(len(rows), dtype=EVENT_DTYPE)
    for i, r in enumerate(rows):
        delta, ptr, line, pn = r[:4]
        kind = r[4] if len(r) > 4 else KIND_MEM
        ev[i]["delta"] = delta
        ev[i]["ptr"] = ptr
        ev[i]["line"] = line
        ev[i]["flags"] = (pn & 1) | (kind << 1)
    return ev
