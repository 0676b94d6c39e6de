"""MI355X threshold sampler: Python binding of the C ABI in include/scalene_sampler.h.

This module only marshals arguments; every step of the method runs in the HIP
kernels of ``libscalene_hip.so``.  PyTorch provides device memory (the
workspace, device-resident event buffers) and streams.  If the library is not
built, importing works but every call raises.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

from ._build import LIB_PATH

SMP_OK, SMP_EINVAL, SMP_EBUDGET, SMP_ETOOBIG, SMP_EAGAIN = 0, 1, 2, 3, 4
SMP_EDEVICE, SMP_EOVERFLOW, SMP_ENOMEM, SMP_ESTATE = 5, 6, 7, 8
OPT_PRIME_T, OPT_RESOLVE_AT_END = 1, 2

HIST_NAMES = (
    "py_bytes", "nat_bytes", "growth_n", "shrink_n", "growth_bytes", "shrink_bytes",
    "leak_mallocs", "leak_frees", "copy_sampled", "copy_exact", "py_time_us", "nat_time_us",
)
LEAK_NAMES = ("lap_num", "lap_den", "lit_num", "lit_den")
GATE_NAMES = ("lap_gate", "lit_gate")

SAMPLE_DTYPE = np.dtype([("event_idx", "<u4"), ("line", "<u4"), ("F", "<i8"), ("py", "<i8"), ("nat", "<i8")])
TRACKED_DTYPE = np.dtype([("event_idx", "<u4"), ("line", "<u4"), ("ptr", "<u4"), ("freed", "<u4")])

EXPORTED = ("workspace_bytes", "sampler_create", "submit_trace", "run", "poll", "fetch_profile",
            "trace_device_results", "submit_traces", "release_traces", "sampler_last_timing",
            "sampler_set_pass_events", "sampler_last_pass_timing", "sampler_last_counters", "sampler_fixed_bytes",
            "sampler_set_tuning", "sampler_get_tuning", "sampler_launch_stats",
            "sampler_destroy", "error_string", "rate_workspace_bytes", "rate_run", "rate_run_noalloc", "report_lines",
            "leak_report", "timeline_points", "timeline_points_sampled")

PASS_NAMES = ("summarize", "resolve", "chain", "scan", "emit")


class Params(ctypes.Structure):
    _fields_ = [
        ("threshold", ctypes.c_int64),
        ("copy_threshold", ctypes.c_int64),
        ("num_lines", ctypes.c_uint32),
        ("quantum_us", ctypes.c_uint32),
        ("options", ctypes.c_uint32),
        ("reserved", ctypes.c_uint32),
    ]


class ProfileSizes(ctypes.Structure):
    _fields_ = [
        ("n_samples", ctypes.c_uint64),
        ("n_tracked", ctypes.c_uint64),
        ("num_lines", ctypes.c_uint32),
        ("status", ctypes.c_int32),
    ]


class Profile(ctypes.Structure):
    _fields_ = [
        ("samples", ctypes.c_void_p),
        ("tracked", ctypes.c_void_p),
        ("hist", ctypes.c_void_p),
        ("leak", ctypes.c_void_p),
        ("gates", ctypes.c_void_p),
        ("final_F", ctypes.c_int64),
        ("peak_F", ctypes.c_int64),
        ("peak_sampled_F", ctypes.c_int64),
        ("threshold_used", ctypes.c_int64),
        ("n_samples", ctypes.c_uint64),
        ("n_tracked", ctypes.c_uint64),
        ("status", ctypes.c_int32),
        ("reserved", ctypes.c_int32),
    ]


class Tuning(ctypes.Structure):
    _fields_ = [
        ("chain_cap", ctypes.c_uint32),
        ("chain_grid", ctypes.c_uint32),
        ("emit_grid", ctypes.c_uint32),
        ("graphs", ctypes.c_uint32),
        ("tile_map_tiles", ctypes.c_uint32),
    ]


def _host_array(shape, dtype, pinned):
    """An uninitialised host array; with ``pinned``, a view of a page-locked
    torch buffer (the array keeps the buffer alive)."""
    dtype = np.dtype(dtype)
    if not pinned:
        return np.empty(shape, dtype)
    import torch
    count = int(np.prod(shape, dtype=np.int64))
    buf = torch.empty(max(count * dtype.itemsize, 1), dtype=torch.uint8, pin_memory=True)
    return buf.numpy()[: count * dtype.itemsize].view(dtype).reshape(shape)


class SamplerError(RuntimeError):
    def __init__(self, fn, code):
        super().__init__(f"{fn} failed: {code} ({error_string(code)})")
        self.code = code


_lib = None


def lib():
    """The loaded C library; raises if it is not built (no fallback exists)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"HIP library {LIB_PATH} is not built; run __graft_entry__.build()")
        L = ctypes.CDLL(LIB_PATH)
        u64, i32, vp = ctypes.c_uint64, ctypes.c_int, ctypes.c_void_p
        L.workspace_bytes.argtypes = [u64, ctypes.POINTER(Params), i32]
        L.workspace_bytes.restype = u64
        L.sampler_create.argtypes = [i32, vp, u64, vp, u64, ctypes.POINTER(vp)]
        L.sampler_create.restype = i32
        L.submit_trace.argtypes = [vp, vp, u64, ctypes.POINTER(Params), i32, ctypes.POINTER(u64)]
        L.submit_trace.restype = i32
        L.submit_traces.argtypes = [vp, ctypes.c_uint32, ctypes.POINTER(vp), ctypes.POINTER(u64), ctypes.POINTER(Params),
                                    i32, ctypes.POINTER(u64), ctypes.POINTER(ctypes.c_uint32)]
        L.submit_traces.restype = i32
        L.release_traces.argtypes = [vp, ctypes.c_uint32, ctypes.POINTER(u64), ctypes.POINTER(u64),
                                     ctypes.POINTER(ctypes.c_int32), ctypes.POINTER(ctypes.c_uint32)]
        L.release_traces.restype = i32
        L.run.argtypes = [vp, i32]
        L.run.restype = i32
        L.poll.argtypes = [vp, u64]
        L.poll.restype = i32
        L.fetch_profile.argtypes = [vp, u64, ctypes.POINTER(ProfileSizes), ctypes.POINTER(Profile)]
        L.fetch_profile.restype = i32
        L.trace_device_results.argtypes = [vp, u64, ctypes.POINTER(vp), ctypes.POINTER(vp), ctypes.POINTER(u64)]
        L.trace_device_results.restype = i32
        L.sampler_last_timing.argtypes = [vp, ctypes.POINTER(ctypes.c_float), ctypes.POINTER(ctypes.c_float)]
        L.sampler_last_timing.restype = i32
        L.sampler_last_pass_timing.argtypes = [vp, ctypes.POINTER(ctypes.c_float)]
        L.sampler_last_pass_timing.restype = i32
        L.sampler_set_pass_events.argtypes = [vp, ctypes.c_uint32]
        L.sampler_set_pass_events.restype = i32
        L.sampler_last_counters.argtypes = [vp, ctypes.POINTER(ctypes.c_uint64)]
        L.sampler_last_counters.restype = i32
        L.sampler_set_tuning.argtypes = [vp, ctypes.POINTER(Tuning)]
        L.sampler_set_tuning.restype = i32
        L.sampler_get_tuning.argtypes = [vp, ctypes.POINTER(Tuning)]
        L.sampler_get_tuning.restype = i32
        L.sampler_launch_stats.argtypes = [vp, ctypes.POINTER(ctypes.c_uint64)]
        L.sampler_launch_stats.restype = i32
        L.sampler_fixed_bytes.argtypes = []
        L.sampler_fixed_bytes.restype = u64
        L.sampler_destroy.argtypes = [vp]
        L.sampler_destroy.restype = None
        L.error_string.argtypes = [i32]
        L.error_string.restype = ctypes.c_char_p
        L.rate_workspace_bytes.argtypes = [u64]
        L.rate_workspace_bytes.restype = u64
        L.rate_run.argtypes = [vp, u64, ctypes.c_int64, ctypes.c_uint32, vp, u64, vp, vp, vp]
        L.rate_run.restype = i32
        L.rate_run_noalloc.argtypes = [vp, u64, ctypes.c_int64, ctypes.c_uint32, vp, vp, vp]
        L.rate_run_noalloc.restype = i32
        p64 = ctypes.POINTER(ctypes.c_int64)
        L.report_lines.argtypes = [p64, p64, p64, ctypes.c_uint32, ctypes.POINTER(ctypes.c_uint32),
                                   ctypes.POINTER(ctypes.c_uint32)]
        L.report_lines.restype = i32
        L.leak_report.argtypes = [vp, u64, ctypes.POINTER(ctypes.c_uint8), p64, p64, ctypes.c_uint32,
                                  ctypes.POINTER(ctypes.c_int32), ctypes.POINTER(ctypes.c_uint8), p64]
        L.leak_report.restype = i32
        L.timeline_points.argtypes = [vp, u64, ctypes.c_uint32, ctypes.c_uint32, ctypes.POINTER(ctypes.c_uint8)]
        L.timeline_points.restype = i32
        L.timeline_points_sampled.argtypes = [vp, u64, ctypes.c_uint32, ctypes.c_uint32, u64,
                                              ctypes.POINTER(ctypes.c_uint8)]
        L.timeline_points_sampled.restype = i32
        _lib = L
    return _lib


def error_string(code: int) -> str:
    return lib().error_string(int(code)).decode()


def make_params(threshold, num_lines, copy_threshold=None, quantum_us=10_000, options=0) -> Params:
    return Params(int(threshold), int(copy_threshold if copy_threshold is not None else threshold),
                  int(num_lines), int(quantum_us), int(options), 0)


def workspace_bytes(n_events, params: Params, ev_on_device=True) -> int:
    return int(lib().workspace_bytes(int(n_events), ctypes.byref(params), 1 if ev_on_device else 0))


def sampler_fixed_bytes() -> int:
    return int(lib().sampler_fixed_bytes())


def rate_workspace_bytes(n_events) -> int:
    return int(lib().rate_workspace_bytes(int(n_events)))


def rate_run(events, threshold, num_lines, *, workspace=None, line_counts=None, result=None, stream=None,
             sync=True):
    """Rate-based sampling (section 3.2) of one trace on the GPU.

    ``events``: a CUDA uint8 tensor holding the 24-byte records.  Buffers
    not given are allocated with torch on the events' device; ``stream``
    defaults to torch's current stream.  With ``sync`` the call waits and
    returns (status, K, samples per line as numpy); otherwise it returns the
    device tensors (line_counts, result) and the results are ready when the
    stream reaches them."""
    import torch

    if not (isinstance(events, torch.Tensor) and events.is_cuda and events.dtype == torch.uint8):
        raise TypeError("events must be a CUDA uint8 tensor of 24-byte records")
    if events.numel() % 24:
        raise ValueError("events must hold whole 24-byte records")
    n = events.numel() // 24
    dev = events.device
    if workspace is None:
        workspace = torch.empty(rate_workspace_bytes(n), dtype=torch.uint8, device=dev)
    if line_counts is None:
        line_counts = torch.empty(int(num_lines), dtype=torch.int64, device=dev)
    if result is None:
        result = torch.empty(2, dtype=torch.int64, device=dev)
    if stream is None:
        stream = torch.cuda.current_stream(dev)
    code = lib().rate_run(events.data_ptr() if n else None, n, int(threshold), int(num_lines), workspace.data_ptr(),
                          workspace.numel(), line_counts.data_ptr(), result.data_ptr(), stream.cuda_stream)
    _check("rate_run", code)
    if not sync:
        return line_counts, result
    stream.synchronize()
    r = result.cpu().numpy()
    return int(r[1]), int(r[0]), line_counts.cpu().numpy()


RATE_NOALLOC_MAX_EVENTS = 1 << 29


def rate_run_noalloc(events, threshold, num_lines, line_counts, result, stream=None):
    """rate_run with the library's own scratch (the C entry point allocates
    nothing): ``line_counts`` (int64, num_lines) and ``result`` (int64, 2)
    are caller-owned CUDA tensors, written when the stream reaches them.
    Calls that overlap on one GPU race (they share its scratch)."""
    import torch

    if not (isinstance(events, torch.Tensor) and events.is_cuda and events.dtype == torch.uint8):
        raise TypeError("events must be a CUDA uint8 tensor of 24-byte records")
    if events.numel() % 24:
        raise ValueError("events must hold whole 24-byte records")
    for t, name, k in ((line_counts, "line_counts", int(num_lines)), (result, "result", 2)):
        if not (isinstance(t, torch.Tensor) and t.is_cuda and t.dtype == torch.int64 and t.numel() >= k
                and t.is_contiguous()):
            raise TypeError(f"{name} must be a contiguous CUDA int64 tensor of at least {k} values")
    n = events.numel() // 24
    if stream is None:
        stream = torch.cuda.current_stream(events.device)
    _check("rate_run_noalloc", lib().rate_run_noalloc(events.data_ptr() if n else None, n, int(threshold),
                                                      int(num_lines), line_counts.data_ptr(), result.data_ptr(),
                                                      stream.cuda_stream))


def report_lines(py_time_us, nat_time_us, growth_bytes):
    """Report line filter (section 5): ids of the lines with at least 1 % of
    the time or of the memory, with their neighbours, ascending (numpy)."""
    a = [np.ascontiguousarray(x, dtype=np.int64) for x in (py_time_us, nat_time_us, growth_bytes)]
    L = a[0].shape[0]
    if a[1].shape[0] != L or a[2].shape[0] != L:
        raise ValueError("the three arrays must have one value per line")
    out = np.zeros(max(L, 1), np.uint32)
    k = ctypes.c_uint32(0)
    p = ctypes.POINTER(ctypes.c_int64)
    _check("report_lines", lib().report_lines(a[0].ctypes.data_as(p), a[1].ctypes.data_as(p), a[2].ctypes.data_as(p),
                                              L, out.ctypes.data_as(ctypes.POINTER(ctypes.c_uint32)),
                                              ctypes.byref(k)))
    return out[: k.value].copy()


def leak_report(samples, gate, py_time_us, nat_time_us):
    """Leak report filter (section 3.4): (growth test passed, reported flag
    per line, elapsed microseconds) from a profile's samples (SAMPLE_DTYPE,
    rank order), one row of its report gates and its time arrays."""
    smp_ = np.ascontiguousarray(samples, dtype=SAMPLE_DTYPE)
    g = np.ascontiguousarray(gate, dtype=np.uint8)
    a = [np.ascontiguousarray(x, dtype=np.int64) for x in (py_time_us, nat_time_us)]
    L = g.shape[0]
    if a[0].shape[0] != L or a[1].shape[0] != L:
        raise ValueError("gate and the time arrays must have one value per line")
    rep = np.zeros(max(L, 1), np.uint8)
    ok = ctypes.c_int32(0)
    el = ctypes.c_int64(0)
    p = ctypes.POINTER(ctypes.c_int64)
    _check("leak_report", lib().leak_report(smp_.ctypes.data if smp_.size else None, smp_.shape[0],
                                            g.ctypes.data_as(ctypes.POINTER(ctypes.c_uint8)), a[0].ctypes.data_as(p),
                                            a[1].ctypes.data_as(p), L, ctypes.byref(ok),
                                            rep.ctypes.data_as(ctypes.POINTER(ctypes.c_uint8)), ctypes.byref(el)))
    return bool(ok.value), rep[:L].copy(), int(el.value)


def timeline_points(samples, num_lines, max_points=100):
    """Per-line memory timelines (section 5): a keep flag per sample, 1 for
    the points of its line's RDP-reduced footprint log (<= max_points)."""
    smp_ = np.ascontiguousarray(samples, dtype=SAMPLE_DTYPE)
    keep = np.zeros(max(smp_.shape[0], 1), np.uint8)
    _check("timeline_points", lib().timeline_points(smp_.ctypes.data if smp_.size else None, smp_.shape[0],
                                                    int(num_lines), int(max_points),
                                                    keep.ctypes.data_as(ctypes.POINTER(ctypes.c_uint8))))
    return keep[: smp_.shape[0]].copy()


def timeline_points_sampled(samples, num_lines, max_points=100, seed=0):
    """Per-line memory timelines by the paper's procedure (section 5): RDP at
    an approximate eps, then a seeded random downsampling of longer logs to
    exactly max_points points.  A keep flag per sample."""
    smp_ = np.ascontiguousarray(samples, dtype=SAMPLE_DTYPE)
    keep = np.zeros(max(smp_.shape[0], 1), np.uint8)
    _check("timeline_points_sampled",
           lib().timeline_points_sampled(smp_.ctypes.data if smp_.size else None, smp_.shape[0], int(num_lines),
                                         int(max_points), int(seed) & ((1 << 64) - 1),
                                         keep.ctypes.data_as(ctypes.POINTER(ctypes.c_uint8))))
    return keep[: smp_.shape[0]].copy()


def _check(fn, code):
    if code != SMP_OK:
        raise SamplerError(fn, code)


class Sampler:
    """One sampler on one GPU: a workspace tensor, a stream and the C handle.

    ``workspace`` bytes of device memory are allocated with torch (or pass a
    uint8 CUDA tensor).  ``stream`` defaults to torch's current stream.
    """

    def __init__(self, workspace=1 << 30, device=0, stream=None, mem_budget=0):
        import torch

        self.torch = torch
        self.device = torch.device("cuda", device)
        if isinstance(workspace, torch.Tensor):
            self.ws = workspace
        else:
            self.ws = torch.empty(int(workspace), dtype=torch.uint8, device=self.device)
        self.stream = stream if stream is not None else torch.cuda.current_stream(self.device)
        h = ctypes.c_void_p()
        _check("sampler_create", lib().sampler_create(device, ctypes.c_void_p(self.stream.cuda_stream), int(mem_budget),
                                                      ctypes.c_void_p(self.ws.data_ptr()), self.ws.numel(),
                                                      ctypes.byref(h)))
        self.h = h
        self._keep = {}

    def close(self):
        if getattr(self, "h", None):
            lib().sampler_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # -- C ABI mirrors --
    def submit_trace(self, events, params: Params):
        """events: numpy array of 24-byte records (copied before returning), a
        CUDA tensor holding them (borrowed until fetch) or a pinned CPU tensor
        (copied asynchronously, kept until fetch).  Returns the trace id."""
        tid = ctypes.c_uint64()
        if hasattr(events, "data_ptr"):
            n = events.numel() * events.element_size() // 24
            mode = 1 if events.is_cuda else 2
            if mode == 2 and not events.is_pinned():
                raise ValueError("CPU tensors must be pinned; pass a numpy array for pageable memory")
            rc = lib().submit_trace(self.h, ctypes.c_void_p(events.data_ptr()), n, ctypes.byref(params), mode,
                                    ctypes.byref(tid))
            if rc == SMP_OK:
                self._keep[tid.value] = events
        else:
            ev = np.ascontiguousarray(events)
            n = ev.nbytes // 24
            rc = lib().submit_trace(self.h, ctypes.c_void_p(ev.ctypes.data if n else 0), n, ctypes.byref(params), 0,
                                    ctypes.byref(tid))
        _check("submit_trace", rc)
        return tid.value

    def try_submit(self, events, params: Params):
        """Like submit_trace but returns (status, id) instead of raising on budget codes."""
        try:
            return SMP_OK, self.submit_trace(events, params)
        except SamplerError as e:
            if e.code in (SMP_EBUDGET, SMP_ETOOBIG):
                return e.code, None
            raise

    def run(self, blocking=False):
        _check("run", lib().run(self.h, 1 if blocking else 0))

    def poll(self, trace_id) -> bool:
        rc = lib().poll(self.h, int(trace_id))
        if rc == SMP_EAGAIN:
            return False
        _check("poll", rc)
        return True

    def fetch_profile(self, trace_id, pinned=False) -> dict:
        """The trace's whole profile as numpy arrays (and release of the trace).
        With ``pinned`` the arrays live in page-locked host memory from torch's
        pinned allocator, which the device copies into directly instead of
        through staging buffers (for large profiles fetched repeatedly)."""
        sizes = ProfileSizes()
        _check("fetch_profile", lib().fetch_profile(self.h, int(trace_id), ctypes.byref(sizes), None))
        K, H, L = int(sizes.n_samples), int(sizes.n_tracked), int(sizes.num_lines)
        samples = _host_array(K, SAMPLE_DTYPE, pinned)
        tracked = _host_array(H, TRACKED_DTYPE, pinned)
        hist = _host_array((len(HIST_NAMES), L), np.int64, pinned)
        leak = _host_array((len(LEAK_NAMES), L), np.int64, pinned)
        gates = _host_array((len(GATE_NAMES), L), np.uint8, pinned)
        out = Profile(samples.ctypes.data if K else None, tracked.ctypes.data if H else None, hist.ctypes.data,
                      leak.ctypes.data, gates.ctypes.data)
        _check("fetch_profile", lib().fetch_profile(self.h, int(trace_id), ctypes.byref(sizes), ctypes.byref(out)))
        self._keep.pop(int(trace_id), None)
        res = {"status": int(out.status), "K": K, "H": H, "samples": samples, "tracked": tracked,
               "final_F": int(out.final_F), "peak_F": int(out.peak_F), "peak_sampled_F": int(out.peak_sampled_F),
               "threshold_used": int(out.threshold_used)}
        for k, name in enumerate(HIST_NAMES):
            res[name] = hist[k]
        for k, name in enumerate(LEAK_NAMES):
            res[name] = leak[k]
        for k, name in enumerate(GATE_NAMES):
            res[name] = gates[k]
        return res

    def submit_traces(self, events_list, params_list):
        """Admit several traces with one call (all CUDA tensors, borrowed until
        fetch, or all numpy arrays, copied).  params_list is a list of Params,
        or a ctypes array of Params built once for a batch that is submitted
        again and again.  Returns their ids.  If one is refused, raises
        SamplerError whose .ids holds the admitted ones."""
        k = len(events_list)
        if len(params_list) != k:
            raise ValueError("one Params per trace")
        if k == 0:
            return []
        on_dev = all(getattr(e, "is_cuda", False) for e in events_list)
        if not on_dev and any(hasattr(e, "data_ptr") for e in events_list):
            raise ValueError("pass all CUDA tensors or all numpy arrays")
        arrs = events_list if on_dev else [np.ascontiguousarray(e) for e in events_list]
        if on_dev:
            ptrs = np.fromiter((e.data_ptr() for e in arrs), dtype=np.uint64, count=k)
        else:
            ptrs = np.fromiter((a.ctypes.data if a.nbytes else 0 for a in arrs), dtype=np.uint64, count=k)
        ns = np.fromiter((e.nbytes for e in arrs), dtype=np.uint64, count=k) // np.uint64(24)
        p_a = params_list if isinstance(params_list, ctypes.Array) else (Params * k)(*params_list)
        ids = np.zeros(k, dtype=np.uint64)
        done = ctypes.c_uint32()
        rc = lib().submit_traces(self.h, k, ptrs.ctypes.data_as(ctypes.POINTER(ctypes.c_void_p)),
                                 ns.ctypes.data_as(ctypes.POINTER(ctypes.c_uint64)), p_a, 1 if on_dev else 0,
                                 ids.ctypes.data_as(ctypes.POINTER(ctypes.c_uint64)), ctypes.byref(done))
        out = ids[:done.value].tolist()
        if on_dev:
            self._keep.update(zip(out, arrs))
        if rc != SMP_OK:
            err = SamplerError("submit_traces", rc)
            err.ids = out
            raise err
        return out

    def release_traces(self, trace_ids):
        """release() for several traces with one call; returns [(n_samples, status)]."""
        k = len(trace_ids)
        if k == 0:
            return []
        ids = np.asarray(trace_ids, dtype=np.uint64)
        ns = np.zeros(k, dtype=np.uint64)
        st = np.zeros(k, dtype=np.int32)
        done = ctypes.c_uint32()
        rc = lib().release_traces(self.h, k, ids.ctypes.data_as(ctypes.POINTER(ctypes.c_uint64)),
                                  ns.ctypes.data_as(ctypes.POINTER(ctypes.c_uint64)),
                                  st.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)), ctypes.byref(done))
        keep = self._keep
        for t in ids[:done.value].tolist():
            keep.pop(t, None)
        _check("release_traces", rc)
        return list(zip(ns.tolist(), st.tolist()))

    def release(self, trace_id):
        """Wait for a trace and free its workspace without copying results out.
        Returns (n_samples, status)."""
        sizes = ProfileSizes()
        empty = Profile()
        _check("fetch_profile", lib().fetch_profile(self.h, int(trace_id), ctypes.byref(sizes), ctypes.byref(empty)))
        self._keep.pop(int(trace_id), None)
        return int(sizes.n_samples), int(sizes.status)

    def last_timing(self):
        a, b = ctypes.c_float(), ctypes.c_float()
        _check("sampler_last_timing", lib().sampler_last_timing(self.h, ctypes.byref(a), ctypes.byref(b)))
        return float(a.value), float(b.value)

    def set_pass_events(self, mask):
        """Which timing events later runs record (bit p: before sampling pass
        p, bit 5: after the last pass, bit 6: the launch's start); default
        0x7F."""
        _check("sampler_set_pass_events", lib().sampler_set_pass_events(self.h, mask))

    def last_pass_timing(self):
        """Milliseconds of each sampling pass of the last run, by PASS_NAMES
        (-1 for a pass whose events were not recorded)."""
        buf = (ctypes.c_float * len(PASS_NAMES))()
        _check("sampler_last_pass_timing", lib().sampler_last_pass_timing(self.h, buf))
        return dict(zip(PASS_NAMES, (float(x) for x in buf)))

    def set_tuning(self, chain_cap=16, chain_grid=0, emit_grid=0, graphs=1, tile_map_tiles=0):
        """Launch parameters of later runs (no effect on results)."""
        _check("sampler_set_tuning", lib().sampler_set_tuning(self.h, ctypes.byref(
            Tuning(int(chain_cap), int(chain_grid), int(emit_grid), int(graphs), int(tile_map_tiles)))))

    def get_tuning(self):
        t = Tuning()
        _check("sampler_get_tuning", lib().sampler_get_tuning(self.h, ctypes.byref(t)))
        return {"chain_cap": t.chain_cap, "chain_grid": t.chain_grid, "emit_grid": t.emit_grid, "graphs": t.graphs,
                "tile_map_tiles": t.tile_map_tiles}

    def launch_stats(self):
        """(plain launch sequences, graphs captured, graph replays) so far."""
        buf = (ctypes.c_uint64 * 3)()
        _check("sampler_launch_stats", lib().sampler_launch_stats(self.h, buf))
        return {"plain": int(buf[0]), "captured": int(buf[1]), "replayed": int(buf[2])}

    def last_counters(self):
        buf = (ctypes.c_uint64 * 32)()
        _check("sampler_last_counters", lib().sampler_last_counters(self.h, buf))
        return list(buf)

    # -- convenience --
    def profile(self, events, threshold, num_lines, copy_threshold=None, quantum_us=10_000, options=0):
        p = make_params(threshold, num_lines, copy_threshold, quantum_us, options)
        tid = self.submit_trace(events, p)
        self.run(blocking=True)
        return self.fetch_profile(tid)
