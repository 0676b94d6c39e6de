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
