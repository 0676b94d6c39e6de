"""Scheduling logic of the serving loop, on the CPU.

A test-only fake sampler stands in for the C library: it keeps the same
budget rule (workspace bytes per trace), completes batches after a short
delay and answers with the CPU oracle.  It is a test double, not a product
path; the GPU serving test runs the real library.
"""
import time

import numpy as np
import pytest

import oracle
import tracegen as tg
from paper_2212_07597_amd import serve

PER_EVENT = 100  # fake workspace bytes per event


class FakeSampler:
    def __init__(self, budget, delay_s=0.002):
        self.budget = budget
        self.used = 0
        self.peak = 0
        self.delay = delay_s
        self.next = 1
        self.traces = {}
        self.launches = []
        self.submit_order = []

    def try_submit(self, events, params):
        need = PER_EVENT * len(events)
        if need > self.budget:
            return serve.SMP_ETOOBIG, None
        if self.used + need > self.budget:
            return serve.SMP_EBUDGET, None
        tid = self.next
        self.next += 1
        self.used += need
        self.peak = max(self.peak, self.used)
        self.traces[tid] = {"ev": events, "p": params, "need": need, "done_at": None}
        self.submit_order.append(tid)
        return serve.SMP_OK, tid

    def run(self, blocking=False):
        batch = [t for t, d in self.traces.items() if d["done_at"] is None]
        self.launches.append(batch)
        for t in batch:
            self.traces[t]["done_at"] = time.perf_counter() + self.delay
        if blocking:
            time.sleep(self.delay)

    def poll(self, tid):
        return time.perf_counter() >= self.traces[tid]["done_at"]

    def fetch_profile(self, tid):
        d = self.traces.pop(tid)
        self.used -= d["need"]
        p = d["p"]
        return oracle.run(d["ev"], threshold=p["threshold"], num_lines=p["num_lines"])


def make_requests(n, rate, seed=4, max_len=5000):
    plan = tg.config4_plan(base_seed=seed, n_req=n, rate=rate, median=800, sigma=1.0, cap=max_len)
    reqs = []
    for i, (length, arr_ns, s) in enumerate(plan):
        ev, kw = tg.config4_trace(length, s)
        reqs.append(serve.Request(i, arr_ns, ev, {"threshold": 64 * 1024, "num_lines": 64}, length))
    return reqs


def test_serve_admits_in_order_and_respects_budget():
    reqs = make_requests(60, rate=20_000)
    fake = FakeSampler(budget=PER_EVENT * 6000)
    out, makespan = serve.serve(fake, reqs, max_inflight=2, keep_profiles=True)
    assert set(out) == {r.rid for r in reqs}
    assert fake.peak <= fake.budget
    assert fake.submit_order == sorted(fake.submit_order)
    for r in reqs:
        o = out[r.rid]
        assert o.status == "ok"
        want = oracle.run(r.events, threshold=64 * 1024, num_lines=64)
        np.testing.assert_array_equal(o.profile["samples"], want["samples"])
        assert o.latency_ns >= 0
    # requests arriving while batches run are grouped: fewer launches than requests
    assert len(fake.launches) < len(reqs)
    assert max(len(b) for b in fake.launches) > 1


def test_serve_rejects_a_trace_larger_than_the_budget():
    reqs = make_requests(10, rate=5_000)
    big = reqs[3]
    fake = FakeSampler(budget=PER_EVENT * (big.n_events - 1) if big.n_events > 1 else 1)
    out, _ = serve.serve(fake, reqs, max_inflight=2)
    assert out[big.rid].status == "rejected"
    for r in reqs:
        if PER_EVENT * r.n_events > fake.budget:
            assert out[r.rid].status == "rejected"
        else:
            assert out[r.rid].status == "ok"


def test_plain_path_runs_one_request_per_launch():
    reqs = make_requests(8, rate=10_000)
    fake = FakeSampler(budget=PER_EVENT * 10_000)
    out, _ = serve.serve_plain(fake, reqs)
    assert all(o.status == "ok" for o in out.values())
    assert [len(b) for b in fake.launches] == [1] * len(reqs)


def test_latency_stats():
    outs = {i: serve.Outcome(i, "ok", latency_ns=i * 1_000_000) for i in range(101)}
    st = serve.latency_stats(outs)
    assert st["p50_ms"] == pytest.approx(50.0) and st["p99_ms"] == pytest.approx(99.0)
