"""Benchmark: one pass of the whole sampler over one synthetic trace per step.

Workload (single GPU): config 2 - one trace of 1e8 events (lifetime mix: 95 %
small Python objects, 5 % native arrays of 1-256 MiB, exponential lifetimes,
10,000 lines, T = 10 MiB).  The trace is generated on the host (seeded),
copied to HBM once, and every step runs submit_trace (device-resident
events) + run + release on the sampler's stream.  Inputs are resident in HBM
when the timed region starts.

Prints one JSON line with events/s, the roofline figures of the dominant
kernel (the slowest of the three passes over the records, summarize / chain /
emit, each of which reads every 24-byte record once: algorithmic bytes =
24 B x events over that kernel's own HIP-event duration in the timed steps)
and the CPU oracle timed on the host as a baseline.  The per-pass breakdown
(pass_ms, kernel_ms) comes from untimed steps that record events around
every pass; the timed steps record only the two around the dominant pass,
because each event between two kernels idles the GPU for a few microseconds.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "trace events/s + HBM GB/s (batched/served vs plain); p50/p99 trace latency"
HBM_PEAK_GBS = 8000.0
BYTES_PER_EVENT = 24


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def measured_traffic(kernel):
    """HBM bytes per launch of `kernel` on this workload, from the committed
    rocprofv3 counter summary (FETCH_SIZE + WRITE_SIZE, calibrated against a
    plain copy), or None if that summary was taken on other kernel sources."""
    path = os.path.join(ROOT, "profiles", "config2_hbm_traffic.md")
    try:
        text = open(path).read()
    except OSError:
        return None
    kv = {}
    for line in text.splitlines():
        key, sep, val = line.partition(": ")
        if sep and key in ("kernel", "traffic_bytes_per_launch", "kernel_sources_sha256"):
            kv[key] = val.strip()
    h = hashlib.sha256()
    for f in ("sampler_kernels.hip", "sampler_device.h"):
        with open(os.path.join(ROOT, "paper_2212_07597_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    if kv.get("kernel") != kernel or kv.get("kernel_sources_sha256") != h.hexdigest():
        return None
    return int(kv["traffic_bytes_per_launch"])


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--events", type=int, default=100_000_000)
    ap.add_argument("--seed", type=int, default=2)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-seconds", type=float, default=10.0)
    ap.add_argument("--no-extras", action="store_true", help="skip every extra measurement (same as --extras '')")
    ap.add_argument("--extras", default="rate,config5,batched,served",
                    help="comma-separated extra measurements: rate, config5, batched, served")
    ap.add_argument("--served-requests", type=int, default=1000)
    args = ap.parse_args()

    if args.gpus != 1:
        print(f"bench.py measures one GPU only (got --gpus {args.gpus}); the sampler has no multi-GPU path.",
              file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    import __graft_entry__ as ge
    ge.build_if_missing()
    import paper_2212_07597_amd as smp
    import tracegen as tg

    log(f"generating config 2 ({args.events} events)")
    t0 = time.time()
    ev, kw = tg.config2(seed=args.seed, n=args.events)
    log(f"  generated in {time.time() - t0:.1f}s")
    n = ev.shape[0]
    dev = torch.from_numpy(ev.view(np.uint8)).to("cuda")
    params = smp.make_params(kw["threshold"], kw["num_lines"])
    need = smp.workspace_bytes(n, params, ev_on_device=True)
    s = smp.Sampler(workspace=smp.sampler_fixed_bytes() + need + (1 << 20))
    stream = s.stream

    def step():
        tid = s.submit_trace(dev, params)
        s.run(blocking=True)
        return tid

    last = {"K": 0}

    def release(tid):
        K, status = s.release(tid)
        if status != smp.SMP_OK:
            raise RuntimeError(f"trace status {status}")
        last["K"] = K

    log("warmup")
    for _ in range(args.warmup):
        release(step())
    torch.cuda.synchronize()

    # Per-pass breakdown (untimed): events around every pass.  It names the
    # dominant record pass; the timed loop then records only the two events
    # around that pass, since each event between kernels idles the GPU.
    pass_ms, main_list, launch_list = [], [], []
    for _ in range(max(args.warmup, 3)):
        tid = step()
        pass_ms.append(s.last_pass_timing())
        main_list.append(s.last_timing()[0])
        launch_list.append(s.last_timing()[1])
        release(tid)
    passes = {k: sum(p[k] for p in pass_ms) / len(pass_ms) for k in smp.PASS_NAMES}
    main_ms = sum(main_list) / len(main_list)
    record_passes = ("summarize", "chain", "emit")
    dominant = max(record_passes, key=lambda k: passes[k])
    di = smp.PASS_NAMES.index(dominant)
    s.set_pass_events((1 << di) | (1 << (di + 1)))

    dom_ms = []
    log(f"timing {args.steps} steps")
    torch.cuda.synchronize()
    t_start = time.perf_counter()
    for _ in range(args.steps):
        tid = step()
        dom_ms.append(s.last_pass_timing()[dominant])
        release(tid)
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t_start
    s.set_pass_events(0x7F)
    K = last["K"]

    ms_per_step = elapsed * 1e3 / args.steps
    value = n * args.steps / elapsed
    launch_ms = sum(launch_list) / len(launch_list)
    dom_timed = sum(dom_ms) / len(dom_ms)
    achieved = BYTES_PER_EVENT * n / (dom_timed * 1e-3) / 1e9

    cpu = None
    if not args.no_cpu_baseline:
        import oracle
        log("cpu baseline (oracle)")
        reps = 0
        t0 = time.perf_counter()
        while True:
            r = oracle.run(ev, threshold=kw["threshold"], num_lines=kw["num_lines"])
            reps += 1
            if time.perf_counter() - t0 >= args.cpu_seconds:
                break
        dt = time.perf_counter() - t0
        assert r["K"] == K, (r["K"], K)
        cpu = {"value": round(n * reps / dt, 1), "unit": "events/s", "cores": 1, "kind": "oracle",
               "sample": f"the full config-2 trace ({n} events), {reps} sequential pass(es), one host thread"}

    extras = {}
    want = set() if args.no_extras else {x for x in args.extras.split(",") if x}
    if "rate" in want:
        extras["rate"] = bench_rate(smp, tg, torch, np, s, dev, n, kw, K)
    s.close()
    del dev
    torch.cuda.empty_cache()
    if "config5" in want:
        extras["config5"] = bench_config5(smp, tg, torch, np)
    if "batched" in want:
        extras["batched"] = bench_batched(smp, tg, torch, np, cpu=not args.no_cpu_baseline)
    if "served" in want:
        extras["served"] = bench_served(smp, tg, torch, np, args.served_requests)

    out = {
        "metric": METRIC,
        "value": round(value, 1),
        "unit": "events/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_per_step, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "int64",
        "data": "synthetic",
        "config": {"workload": "config2: one trace, 1e8 events, lifetime mix (95% Python 16-512 B, 5% native "
                               "1-256 MiB, exp lifetimes mean 1e4), 10000 lines Zipf 1.2, T=10 MiB",
                   "events": n, "samples": K, "seed": args.seed, "path": "plain one-trace-per-launch",
                   "kernel_ms": round(main_ms, 4), "launch_sequence_ms": round(launch_ms, 4),
                   "pass_ms": {k: round(v, 4) for k, v in passes.items()},
                   "dominant_pass_ms_timed": round(dom_timed, 4)},
        "roofline": {"bound": "hbm", "kernel": "k_" + dominant, "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS,
                     "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4),
                     "traffic": measured_traffic("k_" + dominant), "traffic_unit": "HBM bytes per launch",
                     "algorithmic_bytes": BYTES_PER_EVENT * n},
        "cpu_baseline": cpu,
    }
    out.update(extras)
    print(json.dumps(out), flush=True)


def bench_rate(smp, tg, torch, np, s, dev, n, kw, K_thr, steps=10):
    """Rate-based sampling (section 3.2, one sample per T bytes allocated or
    freed) on the headline trace, timed with HIP events around `steps`
    calls; and the sample counts of the two samplers side by side (the
    paper's comparison) on config 1 and on 32 config-3 traces."""
    T, L = kw["threshold"], kw["num_lines"]
    log("rate-based sampler")
    ws = torch.empty(smp.rate_workspace_bytes(n), dtype=torch.uint8, device="cuda")
    lc = torch.empty(L, dtype=torch.int64, device="cuda")
    res = torch.empty(2, dtype=torch.int64, device="cuda")
    st = torch.cuda.current_stream()
    for _ in range(2):
        smp.rate_run(dev, T, L, workspace=ws, line_counts=lc, result=res, stream=st, sync=False)
    st.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(st)
    for _ in range(steps):
        smp.rate_run(dev, T, L, workspace=ws, line_counts=lc, result=res, stream=st, sync=False)
    e1.record(st)
    e1.synchronize()
    ms = e0.elapsed_time(e1) / steps
    r = res.cpu().numpy()
    if int(r[1]) != smp.SMP_OK:
        raise RuntimeError(f"rate status {int(r[1])}")
    K_rate = int(r[0])

    def counts(ev, kw_):
        d = torch.from_numpy(ev.view(np.uint8)).to("cuda")
        tid = s.submit_trace(d, smp.make_params(kw_["threshold"], kw_["num_lines"]))
        s.run(blocking=True)
        k_thr, status = s.release(tid)
        stt, k_rate, _ = smp.rate_run(d, kw_["threshold"], kw_["num_lines"])
        if status != smp.SMP_OK or stt != smp.SMP_OK:
            raise RuntimeError("status")
        return k_thr, k_rate

    ev1, kw1 = tg.config1(seed=1)
    k1t, k1r = counts(ev1, kw1)
    ratios = []
    for (n3, T3, seed3) in tg.config3_plan()[::32]:
        ev3, kw3 = tg.config3_trace(n3, T3, seed3)
        kt, kr = counts(ev3, kw3)
        ratios.append(kr / max(kt, 1))
    ratios.sort()
    return {"workload": "config2 (the headline trace), T = 10 MiB; the rate path reads the records twice",
            "ms": round(ms, 4), "events_per_s": round(n / (ms * 1e-3), 1),
            "hbm_gbs_algorithmic": round(2 * BYTES_PER_EVENT * n / (ms * 1e-3) / 1e9, 1),
            "K_rate": K_rate, "K_threshold": K_thr, "rate_over_threshold": round(K_rate / max(K_thr, 1), 2),
            "config1": {"K_threshold": k1t, "K_rate": k1r, "rate_over_threshold": round(k1r / max(k1t, 1), 2)},
            "config3_32_traces": {"median_rate_over_threshold": round(ratios[len(ratios) // 2], 2),
                                  "max_rate_over_threshold": round(ratios[-1], 2)}}


def bench_config5(smp, tg, torch, np, steps=3):
    """Config 5: one trace of 5e8 events (config-1 mix with 10 % copy and 1 %
    timer events, 1e6 lines Zipf 1.05, T = Tc = 64 MiB, quantum 10,000 us),
    resident in HBM; plain one-trace-per-launch steps as in the main line."""
    log("config 5: generating 5e8 events")
    ev, kw = tg.config5()
    n = len(ev)
    dev = torch.from_numpy(ev.view(np.uint8)).to("cuda")
    del ev
    p = smp.make_params(kw["threshold"], kw["num_lines"], copy_threshold=kw["copy_threshold"],
                        quantum_us=kw["quantum_us"])
    s = smp.Sampler(workspace=smp.sampler_fixed_bytes() + smp.workspace_bytes(n, p, ev_on_device=True) + (1 << 20))

    def step():
        tid = s.submit_trace(dev, p)
        s.run(blocking=True)
        out = (s.last_pass_timing(), s.last_timing()[0])
        K, status = s.release(tid)
        if status != smp.SMP_OK:
            raise RuntimeError(f"config 5 trace status {status}")
        return out + (K,)

    step()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    runs = [step() for _ in range(steps)]
    dt = (time.perf_counter() - t0) / steps
    s.close()
    del dev
    torch.cuda.empty_cache()
    passes = {k: sum(r[0][k] for r in runs) / len(runs) for k in smp.PASS_NAMES}
    dominant = max(("summarize", "chain", "emit"), key=lambda k: passes[k])
    achieved = BYTES_PER_EVENT * n / (passes[dominant] * 1e-3) / 1e9
    return {"workload": "config5: one trace, 5e8 events, config-1 mix + 10% copy + 1% timer events, 1e6 lines "
                        "Zipf 1.05, T=Tc=64 MiB, quantum 10000 us",
            "events": n, "samples": runs[-1][2], "ms_per_step": round(dt * 1e3, 3), "events_per_s": round(n / dt, 1),
            "kernel_ms": round(sum(r[1] for r in runs) / len(runs), 4),
            "pass_ms": {k: round(v, 4) for k, v in passes.items()},
            "roofline": {"bound": "hbm", "kernel": "k_" + dominant, "achieved": round(achieved, 1),
                         "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4)}}


def bench_batched(smp, tg, torch, np, steps=3, cpu=True):
    """Config 3: 1024 traces (log-uniform 1e3-1e6 events, T from {256 KiB,
    1 MiB, 10 MiB}) in one launch, against a loop of one launch per trace;
    and, beside it, the oracle over the same traces on all host cores (a
    thread pool, one trace per task; the oracle releases the interpreter
    lock while it runs)."""
    log("batched: generating config 3")
    plan = tg.config3_plan()
    traces = [tg.config3_trace(n, T, seed) for (n, T, seed) in plan]
    total = sum(len(ev) for ev, _ in traces)
    devs = [torch.from_numpy(ev.view(np.uint8)).to("cuda") for ev, _ in traces]
    params = [smp.make_params(kw["threshold"], kw["num_lines"]) for _, kw in traces]
    need = sum(smp.workspace_bytes(len(ev), p) for (ev, _), p in zip(traces, params))
    s = smp.Sampler(workspace=smp.sampler_fixed_bytes() + need + (64 << 20))

    pass_runs = []

    def batched():
        ids = s.submit_traces(devs, params)
        s.run(blocking=True)
        km, _ = s.last_timing()
        pass_runs.append(s.last_pass_timing())
        s.release_traces(ids)
        return km

    def plain():
        for d, p in zip(devs, params):
            tid = s.submit_trace(d, p)
            s.run(blocking=True)
            s.release(tid)

    batched()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    kms = [batched() for _ in range(steps)]
    tb = (time.perf_counter() - t0) / steps
    plain()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    plain()
    tp = time.perf_counter() - t0
    s.close()
    del devs
    torch.cuda.empty_cache()
    kms_avg = sum(kms) / len(kms)
    cpu_all = None
    if cpu:
        import concurrent.futures
        import oracle
        cores = min(16, os.cpu_count() or 1)  # the GPU machine's host share
        log(f"batched: oracle on {cores} host threads")

        def one(t):
            ev, kw = t
            return oracle.run(ev, threshold=kw["threshold"], num_lines=kw["num_lines"])["status"]

        t0 = time.perf_counter()
        with concurrent.futures.ThreadPoolExecutor(max_workers=cores) as ex:
            st = list(ex.map(one, sorted(traces, key=lambda t: -len(t[0]))))
        tc = time.perf_counter() - t0
        if any(v != 0 for v in st):
            raise RuntimeError("oracle status")
        cpu_all = {"value": round(total / tc, 1), "unit": "events/s", "cores": cores, "kind": "oracle",
                   "sample": "all 1024 config-3 traces once, one trace per task, longest first"}
    return {"workload": "config3: 1024 traces, lengths 10^(3+3u), config-1 mix, 1000 lines, T in {256K,1M,10M}",
            "cpu_baseline_all_cores": cpu_all,
            "events": total, "batched_events_per_s": round(total / tb, 1), "batched_ms": round(tb * 1e3, 3),
            "batched_kernel_ms": round(kms_avg, 3),
            "batched_pass_ms": {k: round(sum(r[k] for r in pass_runs[1:]) / max(len(pass_runs) - 1, 1), 4)
                                for k in smp.PASS_NAMES},
            "batched_kernel_hbm_gbs": round(BYTES_PER_EVENT * total / (kms_avg * 1e-3) / 1e9, 1),
            "plain_events_per_s": round(total / tp, 1), "plain_ms": round(tp * 1e3, 3),
            "speedup_vs_plain": round(tp / tb, 2)}


def bench_served(smp, tg, torch, np, n_req, rates=(200.0, 1000.0, 5000.0)):
    """Config 4: Poisson arrivals, LogNormal(ln 5e4, 1.5) lengths capped at
    2e7, config-1 mix, T = 1 MiB, events in pinned host memory (each request
    crosses PCIe), 32 GiB admission budget.  Served (continuous batching)
    against plain (one launch per request, in order)."""
    from paper_2212_07597_amd import serve
    log(f"served: generating {n_req} requests")
    plan = tg.config4_plan(base_seed=4, n_req=n_req, rate=1000.0)
    pool = []
    for i, (length, _, seed) in enumerate(plan):
        ev, kw = tg.config4_trace(length, seed)
        pool.append((torch.from_numpy(ev.view(np.uint8)).pin_memory(), length, kw))
    p = smp.make_params(pool[0][2]["threshold"], pool[0][2]["num_lines"])
    budget = 32 << 30
    s = smp.Sampler(workspace=smp.sampler_fixed_bytes() + budget + (1 << 20))
    out = {"workload": "config4: Poisson arrivals, LogNormal(ln 5e4, 1.5) lengths capped at 2e7, config-1 mix, "
                       "T=1 MiB, pinned host events, 32 GiB budget",
           "requests": n_req, "events": int(sum(x[1] for x in pool)), "rates": {}}
    for rate in rates:
        arr = tg.config4_plan(base_seed=40 + int(rate), n_req=n_req, rate=rate)
        reqs = [serve.Request(i, a, pool[i][0], p, pool[i][1]) for i, (_, a, _) in enumerate(arr)]
        log(f"served: rate {rate}/s")
        o_s, mk_s = serve.serve(s, reqs, max_inflight=4)
        o_p, mk_p = serve.serve_plain(s, reqs)
        st_s, st_p = serve.latency_stats(o_s), serve.latency_stats(o_p)
        out["rates"][str(int(rate))] = {
            "served": {**st_s, "events_per_s": round(out["events"] / (mk_s / 1e9), 1)},
            "plain": {**st_p, "events_per_s": round(out["events"] / (mk_p / 1e9), 1)}}
    s.close()
    return out


if __name__ == "__main__":
    main()
