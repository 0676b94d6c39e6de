"""Served traces on the GPU: continuous batching with admission by budget.

Every served profile must equal the oracle's for that trace, so each result is
the same alone and in the mix (tolerance 0: all outputs are integers).
"""
import sys

import numpy as np
import pytest

import oracle
import paper_2212_07597_amd as smp
import tracegen as tg
from paper_2212_07597_amd import serve
from parity_util import compare

pytestmark = pytest.mark.gpu


def say(m):
    print(m, flush=True)
    sys.stdout.flush()


def requests(n, rate, cap, seed=41):
    import torch
    out = []
    for i, (length, arr, s) in enumerate(tg.config4_plan(base_seed=seed, n_req=n, rate=rate, cap=cap)):
        ev, kw = tg.config4_trace(length, s)
        pinned = torch.from_numpy(ev.view(np.uint8)).pin_memory()
        out.append((serve.Request(i, arr, pinned, smp.make_params(kw["threshold"], kw["num_lines"]), length), ev))
    return out


def test_served_results_equal_oracle_under_budget_pressure():
    say("serving: 150 requests at 2000/s with a tight budget")
    pairs = requests(150, 2000.0, cap=400_000)
    reqs = [r for r, _ in pairs]
    p = reqs[0].params
    budget = max(smp.workspace_bytes(r.n_events, p, ev_on_device=False) for r in reqs) * 3
    s = smp.Sampler(workspace=smp.sampler_fixed_bytes() + budget + (1 << 20))
    try:
        out, _ = serve.serve(s, reqs, max_inflight=3, keep_profiles=True)
    finally:
        s.close()
    assert all(o.status == "ok" for o in out.values())
    say("  oracle")
    for r, ev in pairs:
        compare(out[r.rid].profile, oracle.run(ev, threshold=p.threshold, num_lines=p.num_lines), f"request {r.rid}")


def test_served_rejects_a_trace_over_budget():
    say("serving: rejection")
    pairs = requests(6, 500.0, cap=200_000, seed=7)
    reqs = [r for r, _ in pairs]
    p = reqs[0].params
    sizes = sorted(smp.workspace_bytes(r.n_events, p, ev_on_device=False) for r in reqs)
    budget = sizes[-1] - 1
    s = smp.Sampler(workspace=smp.sampler_fixed_bytes() + budget + 4096, mem_budget=budget)
    try:
        out, _ = serve.serve(s, reqs, max_inflight=2)
    finally:
        s.close()
    for r in reqs:
        want = "rejected" if smp.workspace_bytes(r.n_events, p, ev_on_device=False) > budget else "ok"
        assert out[r.rid].status == want
