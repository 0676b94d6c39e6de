"""The no-allocation entry point (rate_run_noalloc) against rate_run.

rate_run_noalloc runs the rate-based sampler (section 3.2) with the
library's own device scratch instead of a caller workspace.  Both entry
points are called through the C ABI on the same device-resident traces and
their outputs (status, K, samples per line) must be identical (integer work:
bit-exact), and equal the oracle's.  Two calls in a row, the second with a
smaller input, show that the shared scratch holds nothing over between
calls.  The last case asks for more events than the scratch allows: it is
refused on the host, before anything is launched.
"""
import sys

import numpy as np
import pytest

import oracle
import paper_2212_07597_amd as smp
import tracegen as tg

pytestmark = pytest.mark.gpu


def say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def run_both(dev, T, L):
    import torch

    lc = torch.full((L,), -7, dtype=torch.int64, device="cuda")  # stale values the call must overwrite
    res = torch.full((2,), -7, dtype=torch.int64, device="cuda")
    smp.rate_run_noalloc(dev, T, L, lc, res)
    torch.cuda.synchronize()
    got = (int(res[1]), int(res[0]), lc.cpu().numpy())
    want = smp.rate_run(dev, T, L)
    return got, want


def test_noalloc_matches_rate_run_on_two_calls():
    import torch

    cases = [("config-1 mix, 400,000 events", tg.config1(seed=21, n=400_000)[0], tg.MiB, 64),
             ("config-1 mix, 70,001 events", tg.config1(seed=22, n=70_001)[0], 256 * tg.KiB, 64)]
    for label, ev, T, L in cases:
        say(f"rate_run_noalloc vs rate_run: {label}")
        dev = torch.from_numpy(ev.view(np.uint8)).to("cuda")
        (st, K, counts), (st2, K2, counts2) = run_both(dev, T, L)
        assert (st, K) == (st2, K2) == (smp.SMP_OK, K2), label
        np.testing.assert_array_equal(counts, counts2, err_msg=label)
        ost, oK, ocounts = oracle.rate(ev, T, L)
        assert (st, K) == (ost, oK), label
        np.testing.assert_array_equal(counts, ocounts, err_msg=label)


def test_noalloc_status_and_empty_trace():
    import torch

    say("rate_run_noalloc: malformed record, then an empty trace")
    ev = tg.config1(seed=23, n=5000)[0].copy()
    ev["line"][4321] = 64  # line >= num_lines: malformed
    dev = torch.from_numpy(ev.view(np.uint8)).to("cuda")
    (st, _, _), (st2, _, _) = run_both(dev, tg.MiB, 64)
    assert st == st2 == smp.SMP_EINVAL
    empty = torch.empty(0, dtype=torch.uint8, device="cuda")
    (st, K, counts), (st2, K2, counts2) = run_both(empty, 10, 3)
    assert (st, K) == (st2, K2) == (smp.SMP_OK, 0) and not counts.any()


def test_noalloc_refuses_more_than_its_scratch_holds():
    import ctypes

    import torch

    say("rate_run_noalloc: size above the maximum")
    lc = torch.zeros(4, dtype=torch.int64, device="cuda")
    res = torch.zeros(2, dtype=torch.int64, device="cuda")
    one = torch.zeros(24, dtype=torch.uint8, device="cuda")
    # the size check comes before any device access, so one record's pointer
    # with a larger count is never read
    rc = smp.lib().rate_run_noalloc(ctypes.c_void_p(one.data_ptr()), smp.RATE_NOALLOC_MAX_EVENTS + 1, 10, 4,
                                    ctypes.c_void_p(lc.data_ptr()), ctypes.c_void_p(res.data_ptr()), None)
    assert rc == smp.SMP_ETOOBIG
