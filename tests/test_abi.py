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


def test_report_lines_matches_oracle():
    """The library's report line filter (host code) against the oracle's, on
    skewed, flat, sparse and negative per-line values, edge sizes included."""
    import oracle

    rng = np.random.default_rng(7)
    sizes = [0, 1, 2, 3, 99, 100, 101, 300, 5000, 20000]
    for i, L in enumerate(sizes * 3):
        kind = i // len(sizes)
        if kind == 0:    # skewed
            py = (rng.pareto(1.1, L) * 50).astype(np.int64)
            nat = (rng.pareto(1.5, L) * 50).astype(np.int64)
            gb = (rng.pareto(0.9, L) * 1e6).astype(np.int64)
        elif kind == 1:  # flat with a few large lines, many zeros
            py = np.where(rng.random(L) < 0.3, 1, 0).astype(np.int64)
            nat = np.zeros(L, np.int64)
            gb = np.where(rng.random(L) < 0.01, 1 << 40, 0).astype(np.int64)
        else:            # signed values (per-line sums wrap modulo 2^64)
            py = rng.integers(-1000, 1000, L).astype(np.int64)
            nat = rng.integers(-10, 10, L).astype(np.int64)
            gb = rng.integers(-(1 << 62), 1 << 62, L).astype(np.int64)
        got = smp.report_lines(py, nat, gb)
        want = oracle.report_lines(py, nat, gb)
        assert got.tolist() == want.tolist(), (L, kind)
