"""Continuous-batching request loop over the C ABI (served traces, config 4).

Requests arrive over time, each a trace of events in pinned host memory.
The loop:

* admits arrived requests in arrival order while the workspace budget has room
  (``submit_trace`` returns SMP_EBUDGET otherwise; the request waits, and it is
  rejected for good on SMP_ETOOBIG);
* launches every admitted, not yet launched request as one batch whenever
  fewer than ``max_inflight`` batches are on the GPU.  Consecutive launches
  go to the library's two launch streams, so a batch that arrives while
  another runs overlaps with it;
* fetches finished requests, which frees their workspace and admits waiting
  ones.

``serve_plain`` is the comparison path: one request per launch, in arrival
order, each launch waited for before the next.

All sampling work happens in the library's kernels; this module only
schedules.  The sampler argument may be any object with the ``Sampler``
methods, which lets the scheduling logic be tested without a GPU.
"""
from __future__ import annotations

import time
from dataclasses import dataclass, field

SMP_OK, SMP_EBUDGET, SMP_ETOOBIG = 0, 2, 3


@dataclass
class Request:
    rid: int
    arrival_ns: int
    events: object          # pinned CPU tensor, CUDA tensor or numpy array
    params: object          # Params
    n_events: int


@dataclass
class Outcome:
    rid: int
    status: str             # "ok", "rejected"
    latency_ns: int = 0
    profile: dict = field(default_factory=dict)


class _Clock:
    def __init__(self):
        self.t0 = time.perf_counter_ns()

    def now(self):
        return time.perf_counter_ns() - self.t0


def serve(sampler, requests, max_inflight=4, keep_profiles=False, clock=None, idle_sleep_s=20e-6):
    """Replay ``requests`` (sorted by arrival_ns) in real time.

    Returns (outcomes by rid, makespan_ns)."""
    clock = clock or _Clock()
    reqs = sorted(requests, key=lambda r: r.arrival_ns)
    nxt = 0                    # next request not yet arrived
    waiting = []               # arrived, not admitted (FIFO)
    admitted = []              # (rid, tid) admitted, not launched
    running = []               # list of batches: list of (rid, tid)
    outcomes = {}
    arrival = {r.rid: r.arrival_ns for r in reqs}
    last_done = 0
    while nxt < len(reqs) or waiting or admitted or running:
        did = False
        now = clock.now()
        while nxt < len(reqs) and reqs[nxt].arrival_ns <= now:
            waiting.append(reqs[nxt])
            nxt += 1
            did = True
        # admission in arrival order
        while waiting:
            r = waiting[0]
            code, tid = sampler.try_submit(r.events, r.params)
            if code == SMP_OK:
                admitted.append((r.rid, tid))
            elif code == SMP_ETOOBIG:
                outcomes[r.rid] = Outcome(r.rid, "rejected")
            else:
                break      # budget full: wait for a completion
            waiting.pop(0)
            did = True
        # launch the admitted requests as one batch
        if admitted and len(running) < max_inflight:
            sampler.run(blocking=False)
            running.append(admitted)
            admitted = []
            did = True
        # completions (a batch finishes as a whole)
        still = []
        for batch in running:
            if sampler.poll(batch[0][1]):
                t = clock.now()
                for rid, tid in batch:
                    prof = sampler.fetch_profile(tid)
                    outcomes[rid] = Outcome(rid, "ok", t - arrival[rid], prof if keep_profiles else {})
                last_done = t
                did = True
            else:
                still.append(batch)
        running = still
        if not did:
            if running:
                time.sleep(idle_sleep_s)
            elif nxt < len(reqs):
                wait_ns = reqs[nxt].arrival_ns - clock.now()
                if wait_ns > 0:
                    time.sleep(min(wait_ns / 1e9, 1e-3))
    return outcomes, last_done


def serve_plain(sampler, requests, keep_profiles=False, clock=None):
    """One request per launch, in arrival order, each waited for."""
    clock = clock or _Clock()
    reqs = sorted(requests, key=lambda r: r.arrival_ns)
    outcomes = {}
    last_done = 0
    for r in reqs:
        wait_ns = r.arrival_ns - clock.now()
        if wait_ns > 0:
            time.sleep(wait_ns / 1e9)
        code, tid = sampler.try_submit(r.events, r.params)
        if code != SMP_OK:
            outcomes[r.rid] = Outcome(r.rid, "rejected")
            continue
        sampler.run(blocking=True)
        prof = sampler.fetch_profile(tid)
        t = clock.now()
        outcomes[r.rid] = Outcome(r.rid, "ok", t - r.arrival_ns, prof if keep_profiles else {})
        last_done = t
    return outcomes, last_done


def latency_stats(outcomes):
    import numpy as np
    lat = np.array([o.latency_ns for o in outcomes.values() if o.status == "ok"], dtype=np.float64)
    if lat.size == 0:
        return {"p50_ms": None, "p99_ms": None, "served": 0}
    return {"p50_ms": float(np.percentile(lat, 50) / 1e6), "p99_ms": float(np.percentile(lat, 99) / 1e6),
            "mean_ms": float(lat.mean() / 1e6), "served": int(lat.size),
            "rejected": int(sum(o.status == "rejected" for o in outcomes.values()))}
