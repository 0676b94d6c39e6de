"""Benchmark: one pass of the whole sampler over one synthetic trace per step.

Workload (single GPU): config 2 - one trace of 1e8 events (lifetime mix: 95 %
small Python objects, 5 % native arrays of 1-256 MiB, exponential lifetimes,
10,000 lines, T = 10 MiB).  The trace is generated on the host (seeded),
copied to HBM once, and every step runs submit_trace (device-resident
events) + run + release.  Inputs are resident in HBM when the timed region
starts.  The headline steps are issued back to back, two in flight on two
run slots: a step's launch is queued while the previous step runs, and the
previous step is released once the next has been launched (every step still
runs the whole launch sequence).  The same steps one after another, each
waited for, are reported beside it (config.serialized).

Prints one JSON line with events/s, the roofline figures of the dominant
kernel (the slowest of the five sampling passes; its algorithmic bytes are
the 24-byte record of every event, over that kernel's own HIP-event duration
in the serialized steps), the whole launch against the same bytes, and the
CPU oracle timed on one pinned host core as a baseline.  The per-pass
breakdown (pass_ms, kernel_ms) comes from untimed steps that record events
around every pass; the serialized steps record only the two around the
dominant pass, because each event between two kernels idles the GPU for a
few microseconds.  An end-to-end figure (pinned host events -> HBM, the
launch, and the full profile copied back) is reported beside it, never as
`value`.

``--only config5|batched|served`` runs one extra measurement alone and
prints its JSON (for profiling one workload at a time).
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import statistics
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "trace events/s + HBM GB/s (batched/served vs plain); p50/p99 trace latency"
HBM_PEAK_GBS = 8000.0
BYTES_PER_EVENT = 24
# the GPU machine gives one GPU's process a share of 16 host CPUs
HOST_CPU_SHARE = 16


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def measured_traffic(kernel, workload="config2"):
    """HBM bytes per launch of `kernel` on this workload, from the committed
    rocprofv3 counter summary (FETCH_SIZE + WRITE_SIZE, calibrated against a
    plain copy), or None if that summary was taken on other kernel sources."""
    path = os.path.join(ROOT, "profiles", f"{workload}_hbm_traffic.md")
    try:
        text = open(path).read()
    except OSError:
        return None
    kv = {}
    for line in text.splitlines():
        key, sep, val = line.partition(": ")
        if sep and key in ("kernel", "traffic_bytes_per_launch", "kernel_sources_sha256"):
            kv[key] = val.strip()
    if kv.get("kernel") != kernel or kv.get("kernel_sources_sha256") != kernel_sources_sha256():
        return None
    return int(kv["traffic_bytes_per_launch"])


def kernel_sources_sha256():
    h = hashlib.sha256()
    for f in ("sampler_kernels.hip", "sampler_device.h"):
        with open(os.path.join(ROOT, "paper_2212_07597_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def host_info():
    model = "unknown"
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                model = line.split(":", 1)[1].strip()
                break
    except OSError:
        pass
    ram_gib = None
    try:
        for line in open("/proc/meminfo"):
            if line.startswith("MemTotal:"):
                ram_gib = round(int(line.split()[1]) / (1 << 20), 1)
                break
    except OSError:
        pass
    return {"cpu_model": model, "nproc": os.cpu_count(), "cpus_allowed": len(os.sched_getaffinity(0)),
            "ram_gib": ram_gib}


def pinned_median_rate(fn, n_events, min_runs=5, min_seconds=10.0):
    """Run fn() (one oracle pass over n_events events) with this thread
    pinned to one CPU, at least min_runs times and min_seconds long; return
    (median events/s over the runs, runs, the CPU)."""
    allowed = sorted(os.sched_getaffinity(0))
    core = allowed[0]
    os.sched_setaffinity(0, {core})
    try:
        rates = []
        t_all = time.perf_counter()
        while len(rates) < min_runs or time.perf_counter() - t_all < min_seconds:
            t0 = time.perf_counter()
            fn()
            rates.append(n_events / (time.perf_counter() - t0))
    finally:
        os.sched_setaffinity(0, set(allowed))
    return statistics.median(rates), len(rates), core


def roofline(pass_ms, n_events, kernel_ms, workload, dom=None):
    """Dominant kernel (the slowest sampling pass unless named) and the whole
    launch, both against the algorithmic 24 bytes per event; traffic from the
    workload's committed counter summary."""
    dom = dom or max(pass_ms, key=lambda k: pass_ms[k])
    traffic = measured_traffic("k_" + dom, workload)
    algo = BYTES_PER_EVENT * n_events
    ach = algo / (pass_ms[dom] * 1e-3) / 1e9
    whole = algo / (kernel_ms * 1e-3) / 1e9
    return dom, {"bound": "hbm", "kernel": "k_" + dom, "achieved": round(ach, 1), "peak": HBM_PEAK_GBS,
                 "unit": "GB/s", "frac": round(ach / HBM_PEAK_GBS, 4), "traffic": traffic,
                 "traffic_unit": "HBM bytes per launch", "algorithmic_bytes": algo,
                 "whole_launch": {"kernel_ms": round(kernel_ms, 4), "achieved": round(whole, 1),
                                  "frac": round(whole / HBM_PEAK_GBS, 4)}}


def tuner(args):
    """f(sampler, workload, n_traces, total_events) -> the launch parameters
    used (autotuned unless --no-tune) for the report."""
    def run(sampler, workload, n_traces, total_events):
        if args.no_tune:
            sampler.set_tuning()
            return {"tuning": sampler.get_tuning(), "autotuned": False}
        from paper_2212_07597_amd import autotune
        t0 = time.perf_counter()
        r = autotune.tune(sampler, workload, autotune.size_class(n_traces, total_events),
                          cache_path=args.tuning_cache, log=log)
        return {"autotuned": True, "key": r["key"], "chosen": r["tuning"], "resolved": sampler.get_tuning(),
                "kernel_ms_tuned": r["ms"], "from_cache": r["from_cache"], "candidates_ms": r["tried"],
                "search_s": round(time.perf_counter() - t0, 2)}
    return run


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
    ap.add_argument("--extras", default="e2e,rate,config5,batched,served",
                    help="comma-separated extra measurements: e2e, rate, config5, batched, served")
    ap.add_argument("--only", choices=("config5", "batched", "served"),
                    help="run this one extra measurement alone and print its JSON")
    ap.add_argument("--no-tune", action="store_true", help="default launch parameters instead of the autotuner's")
    ap.add_argument("--tuning-cache", default=None, help="autotuner cache file (default: the user's cache directory)")
    ap.add_argument("--served-requests", type=int, default=1000)
    ap.add_argument("--served-rates", default="200,1000,5000", help="arrival rates (requests/s) of the served run")
    ap.add_argument("--served-no-plain", action="store_true", help="skip the one-launch-per-request comparison")
    ap.add_argument("--batched-no-plain", action="store_true", help="skip the one-launch-per-trace comparison")
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

    cpu = not args.no_cpu_baseline
    if args.only:
        if args.only == "config5":
            out = bench_config5(smp, tg, torch, np, cpu=cpu, tune=tuner(args))
        elif args.only == "batched":
            out = bench_batched(smp, tg, torch, np, cpu=cpu, tune=tuner(args), plain_compare=not args.batched_no_plain)
        else:
            out = bench_served(smp, tg, torch, np, args.served_requests, served_rates(args), not args.served_no_plain)
        print(json.dumps(out), flush=True)
        return

    log(f"generating config 2 ({args.events} events)")
    t0 = time.time()
    ev, kw = tg.config2(seed=args.seed, n=args.events)
    log(f"  generated in {time.time() - t0:.1f}s")
    n = ev.shape[0]
    dev = torch.from_numpy(ev.view(np.uint8)).to("cuda")
    params = smp.make_params(kw["threshold"], kw["num_lines"])
    want = set() if args.no_extras else {x for x in args.extras.split(",") if x}
    # room for two traces in flight (the back-to-back steps) and for one with
    # a device copy of its events (the end-to-end steps)
    need = max(2 * smp.workspace_bytes(n, params, ev_on_device=True),
               smp.workspace_bytes(n, params, ev_on_device="e2e" not in want))
    s = smp.Sampler(workspace=smp.sampler_fixed_bytes() + need + (1 << 20))

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

    tuned = tuner(args)(s, lambda: release(step()), 1, n)

    log("warmup")
    for _ in range(args.warmup):
        release(step())
    torch.cuda.synchronize()

    # Per-pass breakdown (untimed): events around every pass.  It names the
    # dominant pass; the timed loop then records only the two events around
    # that pass, since each event between kernels idles the GPU.
    pass_ms, main_list, launch_list = [], [], []
    for _ in range(max(args.warmup, 3)):
        tid = step()
        pass_ms.append(s.last_pass_timing())
        main_list.append(s.last_timing()[0])
        launch_list.append(s.last_timing()[1])
        release(tid)
    passes = {k: sum(p[k] for p in pass_ms) / len(pass_ms) for k in smp.PASS_NAMES}
    main_ms = sum(main_list) / len(main_list)
    dominant = max(passes, key=lambda k: passes[k])
    di = smp.PASS_NAMES.index(dominant)
    s.set_pass_events((1 << di) | (1 << (di + 1)))

    # One step after another, each waited for: the dominant pass's own time
    # and the serialized step (host launch latency and completion wake-up
    # included in every step).
    dom_ms = []
    log(f"timing {args.steps} serialized steps")
    torch.cuda.synchronize()
    t_ser = time.perf_counter()
    for _ in range(args.steps):
        tid = step()
        dom_ms.append(s.last_pass_timing()[dominant])
        release(tid)
    torch.cuda.synchronize()
    elapsed_ser = time.perf_counter() - t_ser
    # The headline: the same steps issued back to back, two in flight on two
    # run slots (a step's launch is queued while the previous step runs, and
    # the previous step is released once the next has been launched), with
    # only the start event, so each launch sequence replays as a HIP graph.
    s.set_pass_events(0x40)

    def back_to_back(steps):
        prev = None
        for _ in range(steps):
            tid = s.submit_trace(dev, params)
            s.run(blocking=False)
            if prev is not None:
                release(prev)
            prev = tid
        release(prev)

    back_to_back(6)
    torch.cuda.synchronize()
    log(f"timing {args.steps} back-to-back steps")
    t_start = time.perf_counter()
    back_to_back(args.steps)
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t_start
    s.set_pass_events(0x7F)
    K = last["K"]
    s_stats = s.launch_stats()

    ms_per_step = elapsed * 1e3 / args.steps
    value = n * args.steps / elapsed
    launch_ms = sum(launch_list) / len(launch_list)
    dom_timed = sum(dom_ms) / len(dom_ms)
    timed_passes = dict(passes)
    timed_passes[dominant] = dom_timed
    _, roof = roofline(timed_passes, n, main_ms, "config2", dom=dominant)

    extras = {}
    if "e2e" in want:
        extras["end_to_end"] = bench_e2e(smp, torch, np, s, ev, params, K)

    cpu_base = None
    if cpu:
        import oracle
        log("cpu baseline (oracle, one pinned core)")
        got = {}

        def one():
            got["r"] = oracle.run(ev, threshold=kw["threshold"], num_lines=kw["num_lines"])

        rate, runs, core = pinned_median_rate(one, n, min_runs=5, min_seconds=args.cpu_seconds)
        assert got["r"]["K"] == K, (got["r"]["K"], K)
        cpu_base = {"value": round(rate, 1), "unit": "events/s", "cores": 1, "kind": "oracle",
                    "sample": f"the full config-2 trace ({n} events); median of {runs} sequential passes "
                              f"(>= 5 and >= {args.cpu_seconds:g} s), one thread pinned to CPU {core}",
                    "host": host_info()}

    if "rate" in want:
        extras["rate"] = bench_rate(smp, tg, torch, np, s, dev, n, kw, K)
    s.close()
    del dev
    torch.cuda.empty_cache()
    if "config5" in want:
        extras["config5"] = bench_config5(smp, tg, torch, np, cpu=cpu, tune=tuner(args))
    if "batched" in want:
        extras["batched"] = bench_batched(smp, tg, torch, np, cpu=cpu, tune=tuner(args))
    if "served" in want:
        extras["served"] = bench_served(smp, tg, torch, np, args.served_requests, served_rates(args),
                                        not args.served_no_plain)

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
                   "events": n, "samples": K, "seed": args.seed,
                   "path": "one trace per launch, launches replayed as HIP graphs, two steps in flight",
                   "kernel_ms": round(main_ms, 4), "launch_sequence_ms": round(launch_ms, 4),
                   "pass_ms": {k: round(v, 4) for k, v in passes.items()},
                   "dominant_pass_ms_timed": round(dom_timed, 4), "tuning": tuned,
                   "steps_in_flight": 2,
                   "serialized": {"ms_per_step": round(elapsed_ser * 1e3 / args.steps, 4),
                                  "events_per_s": round(n * args.steps / elapsed_ser, 1)},
                   "launches": s_stats},
        "roofline": roof,
        "cpu_baseline": cpu_base,
    }
    out.update(extras)
    print(json.dumps(out), flush=True)


def bench_e2e(smp, torch, np, s, ev, params, K, reps=3):
    """End to end on the headline trace: events in pinned host memory copied
    to HBM (submit_trace), the launch, and the whole profile copied back into
    pinned host arrays (fetch_profile: samples, tracked list, per-line
    arrays).  Phases are timed one after another with a wait between them;
    median of reps."""
    log("end to end (pinned host events, full profile fetch)")
    host = torch.from_numpy(ev.view(np.uint8)).pin_memory()
    rows = []
    for _ in range(reps + 1):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        tid = s.submit_trace(host, params)
        s.stream.synchronize()
        t1 = time.perf_counter()
        s.run(blocking=True)
        t2 = time.perf_counter()
        prof = s.fetch_profile(tid, pinned=True)
        t3 = time.perf_counter()
        if prof["status"] != smp.SMP_OK or prof["K"] != K:
            raise RuntimeError("end-to-end profile differs from the device-resident one")
        rows.append((t1 - t0, t2 - t1, t3 - t2, t3 - t0))
    rows = rows[1:]  # the first pass warms the pinned pages and the copy engines
    med = [statistics.median(r[i] for r in rows) * 1e3 for i in range(4)]
    n = len(ev)
    return {"workload": "config2, events in pinned host memory; H2D + run + fetch of the whole profile into pinned host arrays",
            "h2d_ms": round(med[0], 3), "run_ms": round(med[1], 3), "fetch_ms": round(med[2], 3),
            "ms": round(med[3], 3), "events_per_s": round(n / (med[3] * 1e-3), 1),
            "h2d_gbs": round(BYTES_PER_EVENT * n / (med[0] * 1e-3) / 1e9, 1), "reps": reps}


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


def bench_config5(smp, tg, torch, np, steps=3, cpu=True, tune=None):
    """Config 5: one trace of 5e8 events (config-1 mix with 10 % copy and 1 %
    timer events, 1e6 lines Zipf 1.05, T = Tc = 64 MiB, quantum 10,000 us),
    resident in HBM; plain one-trace-per-launch steps as in the main line;
    the oracle on one pinned core (median of 3 passes over the full trace)."""
    log("config 5: generating 5e8 events")
    ev, kw = tg.config5()
    n = len(ev)
    dev = torch.from_numpy(ev.view(np.uint8)).to("cuda")
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

    tuned = tune(s, step, 1, n) if tune else None
    step()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    runs = [step() for _ in range(steps)]
    dt = (time.perf_counter() - t0) / steps
    s.close()
    del dev
    torch.cuda.empty_cache()
    passes = {k: sum(r[0][k] for r in runs) / len(runs) for k in smp.PASS_NAMES}
    kernel_ms = sum(r[1] for r in runs) / len(runs)
    _, roof = roofline(passes, n, kernel_ms, "config5")
    K = runs[-1][2]
    cpu_base = None
    if cpu:
        import oracle
        log("config 5: oracle on one pinned core")
        got = {}

        def one():
            got["r"] = oracle.run(ev, threshold=kw["threshold"], num_lines=kw["num_lines"],
                                  copy_threshold=kw["copy_threshold"], quantum_us=kw["quantum_us"])

        rate, nrun, core = pinned_median_rate(one, n, min_runs=3, min_seconds=0.0)
        if got["r"]["K"] != K:
            raise RuntimeError("config 5: oracle and GPU sample counts differ")
        cpu_base = {"value": round(rate, 1), "unit": "events/s", "cores": 1, "kind": "oracle",
                    "sample": f"the full config-5 trace ({n} events); median of {nrun} passes, one thread pinned "
                              f"to CPU {core}", "host": host_info()}
    del ev
    return {"workload": "config5: one trace, 5e8 events, config-1 mix + 10% copy + 1% timer events, 1e6 lines "
                        "Zipf 1.05, T=Tc=64 MiB, quantum 10000 us",
            "events": n, "samples": K, "ms_per_step": round(dt * 1e3, 3), "events_per_s": round(n / dt, 1),
            "kernel_ms": round(kernel_ms, 4),
            "pass_ms": {k: round(v, 4) for k, v in passes.items()},
            "roofline": roof, "tuning": tuned, "cpu_baseline": cpu_base}


def bench_batched(smp, tg, torch, np, steps=3, cpu=True, tune=None, plain_compare=True):
    """Config 3: 1024 traces (log-uniform 1e3-1e6 events, T from {256 KiB,
    1 MiB, 10 MiB}) in one launch, against a loop of one launch per trace;
    and, beside it, the oracle over the same traces on one pinned core and
    on the host's CPU share (a thread pool, one trace per task; the oracle
    releases the interpreter lock while it runs)."""
    log("batched: generating config 3")
    plan = tg.config3_plan()
    traces = [tg.config3_trace(n, T, seed) for (n, T, seed) in plan]
    total = sum(len(ev) for ev, _ in traces)
    devs = [torch.from_numpy(ev.view(np.uint8)).to("cuda") for ev, _ in traces]
    params = [smp.make_params(kw["threshold"], kw["num_lines"]) for _, kw in traces]
    params_arr = (smp.Params * len(params))(*params)  # built once: the batch is submitted every step
    need = sum(smp.workspace_bytes(len(ev), p) for (ev, _), p in zip(traces, params))
    # room for two batches in flight (the back-to-back batches)
    s = smp.Sampler(workspace=smp.sampler_fixed_bytes() + 2 * need + (64 << 20))

    phases = []

    def batched():
        t0 = time.perf_counter()
        ids = s.submit_traces(devs, params_arr)
        t1 = time.perf_counter()
        s.run(blocking=True)
        t2 = time.perf_counter()
        km, launch = s.last_timing()
        s.release_traces(ids)
        t3 = time.perf_counter()
        phases.append((t1 - t0, t2 - t1, t3 - t2, launch))
        return km

    def one_batch():
        ids = s.submit_traces(devs, params_arr)
        s.run(blocking=True)
        s.release_traces(ids)

    tuned = tune(s, one_batch, len(devs), total) if tune else None

    def plain():
        for d, p in zip(devs, params):
            tid = s.submit_trace(d, p)
            s.run(blocking=True)
            s.release(tid)

    # per-pass breakdown (untimed): events around every pass, plain launches
    pass_runs, kms = [], []
    for _ in range(3):
        kms.append(batched())
        pass_runs.append(s.last_pass_timing())
    # timed: only the launch's start event, so its launch sequence replays
    # as a HIP graph once captured
    s.set_pass_events(0x40)
    batched()
    batched()
    torch.cuda.synchronize()
    phases.clear()
    t0 = time.perf_counter()
    for _ in range(steps):
        batched()
    tb = (time.perf_counter() - t0) / steps
    # the same batches back to back, two in flight on two run slots (a
    # batch is released once the next one has been launched)

    def back_to_back(n_batches):
        prev = None
        for _ in range(n_batches):
            ids = s.submit_traces(devs, params_arr)
            s.run(blocking=False)
            if prev is not None:
                s.release_traces(prev)
            prev = ids
        s.release_traces(prev)

    back_to_back(3)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    back_to_back(steps)
    torch.cuda.synchronize()
    tb2 = (time.perf_counter() - t0) / steps
    s.set_pass_events(0x7F)
    s_stats = s.launch_stats()
    tp = None
    if plain_compare:
        plain()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        plain()
        tp = time.perf_counter() - t0
    s.close()
    del devs
    torch.cuda.empty_cache()
    kms_avg = sum(kms) / len(kms)
    passes = {k: sum(r[k] for r in pass_runs) / len(pass_runs) for k in smp.PASS_NAMES}
    _, roof = roofline(passes, total, kms_avg, "config3")
    cpu_one = cpu_all = None
    if cpu:
        import concurrent.futures
        import oracle

        def one(t):
            ev, kw = t
            return oracle.run(ev, threshold=kw["threshold"], num_lines=kw["num_lines"])["status"]

        log("batched: oracle on one pinned core")

        def all_traces():
            for t in traces:
                if one(t) != 0:
                    raise RuntimeError("oracle status")

        rate, nrun, core = pinned_median_rate(all_traces, total, min_runs=5, min_seconds=0.0)
        cpu_one = {"value": round(rate, 1), "unit": "events/s", "cores": 1, "kind": "oracle",
                   "sample": f"all 1024 config-3 traces in order; median of {nrun} passes, one thread pinned to "
                             f"CPU {core}"}
        workers = min(HOST_CPU_SHARE, len(os.sched_getaffinity(0)))
        log(f"batched: oracle on {workers} host threads")
        order = sorted(traces, key=lambda t: -len(t[0]))
        rates = []
        with concurrent.futures.ThreadPoolExecutor(max_workers=workers) as ex:
            for _ in range(3):
                t0 = time.perf_counter()
                st = list(ex.map(one, order))
                rates.append(total / (time.perf_counter() - t0))
                if any(v != 0 for v in st):
                    raise RuntimeError("oracle status")
        cpu_all = {"value": round(statistics.median(rates), 1), "unit": "events/s", "cores": workers,
                   "kind": "oracle",
                   "sample": f"all 1024 config-3 traces, one trace per task, longest first, on a pool of {workers} "
                             f"threads (the host CPU share of one GPU, capped at {HOST_CPU_SHARE}); median of 3",
                   "host": host_info()}
    return {"workload": "config3: 1024 traces, lengths 10^(3+3u), config-1 mix, 1000 lines, T in {256K,1M,10M}",
            "cpu_baseline_one_core": cpu_one, "cpu_baseline_all_cores": cpu_all,
            "events": total, "batched_events_per_s": round(total / tb, 1), "batched_ms": round(tb * 1e3, 3),
            "batched_kernel_ms": round(kms_avg, 3),
            "back_to_back": {"ms_per_batch": round(tb2 * 1e3, 3), "events_per_s": round(total / tb2, 1),
                             "batches_in_flight": 2},
            "batched_phase_ms": {k: round(statistics.median(p[i] for p in phases) * (1 if i == 3 else 1e3), 3)
                                 for i, k in enumerate(("submit_traces", "run_blocking", "release_traces",
                                                        "launch_sequence_gpu"))},
            "batched_pass_ms": {k: round(v, 4) for k, v in passes.items()},
            "roofline": roof, "tuning": tuned, "launches": s_stats,
            "plain_events_per_s": round(total / tp, 1) if tp else None, "plain_ms": round(tp * 1e3, 3) if tp else None,
            "speedup_vs_plain": round(tp / tb, 2) if tp else None}


def served_rates(args):
    return tuple(float(x) for x in args.served_rates.split(",") if x)


def bench_served(smp, tg, torch, np, n_req, rates=(200.0, 1000.0, 5000.0), plain=True):
    """Config 4: Poisson arrivals, LogNormal(ln 5e4, 1.5) lengths capped at
    2e7, config-1 mix, T = 1 MiB, events in pinned host memory (each request
    crosses PCIe), 32 GiB admission budget.  Served (continuous batching)
    against plain (one launch per request, in order).  The PCIe part of the
    latency is reported beside it: the pinned host-to-device copy rate
    measured here, and each request's copy time at that rate."""
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
    # pinned host-to-device copy rate (256 MiB, median of 5)
    src = torch.empty(256 << 20, dtype=torch.uint8).pin_memory()
    dst = torch.empty(256 << 20, dtype=torch.uint8, device="cuda")
    bw = []
    for _ in range(6):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        dst.copy_(src, non_blocking=True)
        torch.cuda.synchronize()
        bw.append((256 << 20) / (time.perf_counter() - t0))
    h2d = statistics.median(bw[1:])
    del src, dst
    copy_ms = np.array([BYTES_PER_EVENT * x[1] / h2d * 1e3 for x in pool])
    out = {"workload": "config4: Poisson arrivals, LogNormal(ln 5e4, 1.5) lengths capped at 2e7, config-1 mix, "
                       "T=1 MiB, pinned host events, 32 GiB budget",
           "requests": n_req, "events": int(sum(x[1] for x in pool)),
           "h2d": {"gbs": round(h2d / 1e9, 2), "request_copy_ms_p50": round(float(np.percentile(copy_ms, 50)), 4),
                   "request_copy_ms_p99": round(float(np.percentile(copy_ms, 99)), 4),
                   "note": "pinned host-to-device copy time of each request's events at the measured rate; "
                           "part of every served and plain latency"},
           "rates": {}}
    for rate in rates:
        arr = tg.config4_plan(base_seed=40 + int(rate), n_req=n_req, rate=rate)
        reqs = [serve.Request(i, a, pool[i][0], p, pool[i][1]) for i, (_, a, _) in enumerate(arr)]
        log(f"served: rate {rate}/s")
        o_s, mk_s = serve.serve(s, reqs, max_inflight=4)
        st_s = serve.latency_stats(o_s)
        out["rates"][str(int(rate))] = {"served": {**st_s, "events_per_s": round(out["events"] / (mk_s / 1e9), 1)}}
        if plain:
            o_p, mk_p = serve.serve_plain(s, reqs)
            st_p = serve.latency_stats(o_p)
            out["rates"][str(int(rate))]["plain"] = {**st_p, "events_per_s": round(out["events"] / (mk_p / 1e9), 1)}
    s.close()
    return out


if __name__ == "__main__":
    main()
