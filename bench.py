#!/usr/bin/env python3
"""Benchmark: instruction-graph generation throughput and per-task latency.

Headline workload: the batched workload -- 256 seeded task streams of uneven
size (1-3-D buffers of 2^10..2^24 elements, 16..1024 chunks, 50..2000 tasks,
one_to_one / neighborhood / slice / all readers), analysed in one persistent
launch with one workgroup per stream and replayed as a HIP graph.  One step
is one full analysis of all 256 recorded streams from scratch (reset +
analysis kernel, one graph launch); the recorded commands are resident in
HBM before the timed region starts.  Output: one JSON line.

Metric: instructions + edges generated per second (whole job), with the p50
/ p99 per-task scheduling latency (device clock, from the start of a task's
intake to the moment its records are complete, lookahead holding included
and also reported on its own).

The same line carries objects for the single-stream workloads (2-D stencil,
N-body, 1-D stencil), each with its own roofline, and for serving.

Roofline numerator: algorithmic bytes = 74 I + 16 Bnd + 9 E + 64 U_w + 4 U_r
+ 88 U_b + 48 (mapper boxes), with I, Bnd, E the record counts and the other
terms the oracle's counts of allocation-map writer updates, reader
insertions, buffer-map updates and range-mapper boxes (stored with the
oracle's results under tests/golden/, written by the oracle alone).
"""
import argparse
import hashlib
import json
import os
import platform
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "instructions+edges generated/sec and p99 per-task scheduling latency"
PEAK_HBM_GBS = 8000.0
KERNEL_SRC = os.path.join(ROOT, "paper_2503_10516_amd", "csrc", "ig_kernels.hip")
PROFILES = os.path.join(ROOT, "profiles")
GOLDEN = os.path.join(ROOT, "tests", "golden")
DIGEST_KEYS = ("n_instructions", "n_bindings", "n_edges", "digest_instructions", "digest_bindings", "digest_edges")


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def load_json(path):
    try:
        with open(path) as f:
            return json.load(f)
    except (OSError, ValueError):
        return None


def algorithmic_bytes(t):
    """Bytes the method must move for one analysis (per-term weights of the
    device layout: 74 B per instruction record, 16 B per binding, 9 B per
    edge, 64 B per allocation-map writer update, 4 B per reader insertion,
    88 B per buffer-map update, 48 B per mapper box)."""
    return (74 * t["n_instructions"] + 16 * t["n_bindings"] + 9 * t["n_edges"] + 64 * t["u_w"] + 4 * t["u_r"]
            + 88 * t["u_b"] + 48 * t["map_boxes"])


def kernel_sha(src=None):
    with open(src or KERNEL_SRC, "rb") as f:
        return hashlib.sha256(f.read()).hexdigest()[:16]


def measured_traffic(name, src=None):
    """HBM bytes per launch from a committed rocprofv3 counter summary, if it
    was taken on the current kernel source (src, default the analysis
    kernel's)."""
    d = load_json(os.path.join(PROFILES, name))
    if not d or d.get("kernel_sha") != kernel_sha(src):
        return None
    return d.get("hbm_bytes_per_launch")


def host_info():
    model = platform.processor() or "unknown"
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    try:
        avail = len(os.sched_getaffinity(0))
    except AttributeError:
        avail = os.cpu_count()
    return {"cpu_model": model, "nproc": avail, "os_cpu_count": os.cpu_count()}


def copy_bandwidth():
    """Achievable HBM bandwidth: a plain 1 GiB device-to-device copy (reads
    1 GiB, writes 1 GiB), median of 5, in GB/s."""
    import numpy as np
    import torch
    a = torch.empty(1 << 30, dtype=torch.uint8, device="cuda")
    b = torch.empty_like(a)
    b.copy_(a)
    torch.cuda.synchronize()
    ms = []
    for _ in range(5):
        s, e = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        s.record()
        b.copy_(a)
        e.record()
        e.synchronize()
        ms.append(s.elapsed_time(e))
    del a, b
    torch.cuda.empty_cache()
    return 2.0 * (1 << 30) / (float(np.median(ms)) / 1e3) / 1e9


def roofline(ab, kernel_s, copy_gbs, traffic):
    achieved = ab / kernel_s / 1e9
    return {"bound": "hbm", "achieved": achieved, "peak": PEAK_HBM_GBS, "unit": "GB/s",
            "frac": achieved / PEAK_HBM_GBS, "traffic": traffic, "kernel": "ig_analyse",
            "kernel_ms": kernel_s * 1e3, "algorithmic_bytes": ab,
            "copy_gbs": copy_gbs, "frac_of_copy": achieved / copy_gbs if copy_gbs else None}


def latency_summary(times_ns):
    """p50/p99 of per-task latency (intake start -> records complete), of
    the lookahead holding part (intake end -> compile start) and of the
    rest, in microseconds."""
    import numpy as np
    lat = (times_ns[:, 3] - times_ns[:, 0]) / 1e3
    hold = (times_ns[:, 2] - times_ns[:, 1]) / 1e3
    work = lat - hold
    pct = lambda x, q: float(np.percentile(x, q)) if len(x) else 0.0
    return {"p50_task_latency_us": pct(lat, 50), "p99_task_latency_us": pct(lat, 99),
            "p50_holding_us": pct(hold, 50), "p99_holding_us": pct(hold, 99),
            "p50_analysis_us": pct(work, 50), "p99_analysis_us": pct(work, 99),
            "held_tasks": int((hold > 5.0).sum())}


# ---------------------------------------------------------------------------
# CPU baseline: the oracle (test infrastructure), never tuned for this
# ---------------------------------------------------------------------------

def _oracle_one(i):
    import oracle
    from paper_2503_10516_amd import streams as S
    s = S.batched_stream(S.BATCHED_SEED, i, w_all=S.BATCHED_W_ALL, w_slice=S.BATCHED_W_SLICE)
    r = oracle.run_stream(s, fetch=False)
    return i, r["seconds"], r["stats"]["n_instructions"] + r["stats"]["n_edges"]


def cpu_baseline_batched(gold, reps):
    """The oracle over the host's cores (one process per stream at a time)
    on a bounded sample of the batched workload: every 8th stream whose
    stored single-core oracle time is at most 5 s.  Median of `reps` runs."""
    import numpy as np
    from multiprocessing import get_context
    rows = gold["streams"]
    sample = [r["index"] for r in rows if r["index"] % 8 == 0 and r["oracle_seconds"] <= 5.0]
    info = host_info()
    procs = max(1, min(16, info["nproc"], len(sample)))
    rates, walls, cpu = [], [], []
    # fresh interpreters (spawn): the workers never touch the GPU
    with get_context("spawn").Pool(procs) as pool:
        for _ in range(reps):
            t0 = time.perf_counter()
            out = pool.map(_oracle_one, sorted(sample, key=lambda i: -rows[i]["oracle_seconds"]), chunksize=1)
            wall = time.perf_counter() - t0
            recs = sum(o[2] for o in out)
            rates.append(recs / wall)
            walls.append(wall)
            cpu.append(sum(o[1] for o in out))
    k = int(np.argsort(rates)[len(rates) // 2])
    stored_sample = sum(rows[i]["oracle_seconds"] for i in sample)
    speed = stored_sample / cpu[k]  # this host's core speed relative to the stored run
    all_recs = sum(r["n_instructions"] + r["n_edges"] for r in rows)
    all_cpu = sum(r["oracle_seconds"] for r in rows) / speed
    return {"value": rates[k], "unit": "records/s", "cores": procs, "kind": "oracle",
            "sample": f"{len(sample)} of the 256 batched streams (every 8th index whose single-core oracle time "
                      f"is <= 5 s; {recs} records), one stream per process on {procs} processes, median of "
                      f"{reps} runs; wall {walls[k]:.2f} s, {cpu[k]:.1f} s of oracle CPU time",
            "cpu_model": info["cpu_model"], "nproc": info["nproc"],
            "full_batch_estimate": {
                "records": all_recs, "single_core_s": all_cpu,
                "records_per_s_on_all_cores": all_recs / (all_cpu / procs),
                "note": "the stored single-core oracle times of all 256 streams (tests/golden), scaled by this "
                        "host's measured speed on the sample; heavy streams run slower per record than the "
                        "sample, so this is the representative CPU figure"}}


def oracle_median(stream, reps):
    import numpy as np
    import oracle
    secs, recs = [], 0
    for _ in range(reps):
        r = oracle.run_stream(stream, fetch=False)
        secs.append(r["seconds"])
        recs = r["stats"]["n_instructions"] + r["stats"]["n_edges"]
    med = float(np.median(secs))
    return {"value": recs / med, "unit": "records/s", "cores": 1, "kind": "oracle", "median_of": reps,
            "seconds": med}


# ---------------------------------------------------------------------------
# Config 4: the batched workload (headline)
# ---------------------------------------------------------------------------

def run_batched(args, copy_gbs):
    import numpy as np
    import torch
    from paper_2503_10516_amd import autotune, batch, streams

    t = time.perf_counter()
    ss = streams.batched()
    log(f"batched: generated {len(ss)} streams, {sum(s.n_tasks for s in ss)} tasks ({time.perf_counter() - t:.1f} s)")
    gold = load_json(os.path.join(GOLDEN, "batched_digests.json"))
    if args.batch_threads == 0:
        tuned = autotune.tune(ss, log=log)
    else:
        tuned = {"threads": args.batch_threads}
    threads = tuned["threads"]
    bt = batch.Batch(ss, threads=threads)
    t = time.perf_counter()
    grown = bt.size(window=args.batch_window,
                    log=lambda k, n, p: log(f"batched sizing: launch {k}, {n} streams active, "
                                            f"{int((p[:, 2] != 0).sum())} out of capacity"))
    log(f"batched: first analysis and sizing {time.perf_counter() - t:.1f} s, re-sized {grown}")
    cnt = bt.counts()
    records = int(cnt[:, 0].sum() + cnt[:, 2].sum())
    rows = {r["index"]: r for r in gold["streams"]} if gold else {}

    def digests_equal():
        return sum(all(ctx.stats()[k] == rows[i][k] for k in DIGEST_KEYS)
                   for i, ctx in enumerate(bt.contexts) if i in rows)

    matched_before = digests_equal()
    log(f"batched: {matched_before}/{len(rows)} streams equal their oracle digests")
    bt.capture()
    stream = torch.cuda.current_stream()
    for k in range(args.warmup):
        bt.launch()
        torch.cuda.synchronize()
        log(f"batched: warmup launch {k}")
    starts = [torch.cuda.Event(enable_timing=True) for _ in range(args.steps)]
    ends = [torch.cuda.Event(enable_timing=True) for _ in range(args.steps)]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for k in range(args.steps):
        starts[k].record(stream)
        bt.launch()  # reset + ig_analyse over the 256 streams, one graph launch
        ends[k].record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    kernel_ms = [a.elapsed_time(b) for a, b in zip(starts, ends)]
    prog = bt.progress()
    assert (prog[:, 2] == 0).all() and (bt.counts() == cnt).all()
    matched_after = digests_equal()
    log(f"batched: {args.steps} timed launches, {wall / args.steps:.3f} s each; "
        f"{matched_after}/{len(rows)} streams equal their oracle digests after them")
    times = [c.task_times_ns() for c in bt.contexts]
    lat = latency_summary(np.concatenate(times))
    terms = {k: sum(r[k] for r in gold["streams"]) for k in
             ("n_instructions", "n_bindings", "n_edges", "u_w", "u_r", "u_b", "map_boxes")} if gold else None
    ab = algorithmic_bytes(terms) if terms else None
    kern_s = float(np.mean(kernel_ms)) / 1e3
    heavy = bt.order[0]
    # the plain single-stream path on a sample: every 32nd stream by weight
    sample = bt.order[::32]
    t_single, rec_single = 0.0, 0
    for i in sample:
        c = bt.contexts[i]
        c.rewind()
        torch.cuda.synchronize()
        t = time.perf_counter()
        c.flush()
        torch.cuda.synchronize()
        t_single += time.perf_counter() - t
        rec_single += int(cnt[i, 0] + cnt[i, 2])
    out = {
        "records": records, "instructions": int(cnt[:, 0].sum()), "edges": int(cnt[:, 2].sum()),
        "bindings": int(cnt[:, 1].sum()), "tasks": int(cnt[:, 3].sum()), "wall_s": wall,
        "kernel_ms": kernel_ms, "roofline": roofline(ab, kern_s, copy_gbs, measured_traffic(
            "ig_analyse_batched_counters.json")) if ab else None,
        "byte_terms": terms, "threads_per_stream": threads, "autotune": tuned, "resized": grown,
        "oracle_digests_matched": f"{matched_after}/{len(rows)} after the timed launches "
                                  f"({matched_before}/{len(rows)} before)",
        "single_stream_sample": {"streams": len(sample), "records": rec_single, "seconds": t_single,
                                 "records_per_s": rec_single / t_single},
        "vs_single_stream": (records * args.steps / wall) / (rec_single / t_single),
        "heaviest_stream": {"name": ss[heavy].name, "records": int(cnt[heavy, 0] + cnt[heavy, 2]),
                            "tasks": int(cnt[heavy, 3]),
                            "analysis_ms": float(times[heavy][:, 3].max() / 1e6)},
    }
    out.update(lat)
    if "ooo" in set(args.workloads.split(",")):
        out["ooo"] = ooo_run(bt.contexts, max(x.nodes * x.devices for x in ss), max(args.steps, 3), copy_gbs,
                             "ig_ooo_batched_counters.json")
        out["ooo"]["workload"] = ("engine over the 256 batched graphs, one workgroup each, one launch: 2 lanes "
                                  "per device, 2 host lanes, window 1024, eager assignment")
        log(f"ooo batched: {out['ooo']['instructions_per_s']:.3g} instructions/s, "
            f"{np.median(out['ooo']['run_ms']):.1f} ms")
    bt.close()
    return records, out, gold


# ---------------------------------------------------------------------------
# Single streams (configs 1-3)
# ---------------------------------------------------------------------------

def run_single(name, stream, golden_name, steps, threads, copy_gbs, oracle_reps):
    import numpy as np
    import torch
    from paper_2503_10516_amd import binding
    gold = load_json(os.path.join(GOLDEN, golden_name))
    ctx = binding.make_context(stream, threads=threads)
    ctx.record(stream)
    ctx.flush()
    if ctx.sync() != 0:
        raise SystemExit(f"{name}: analysis failed")
    st = ctx.stats()
    equal = gold is not None and all(st[k] == gold[k] for k in DIGEST_KEYS)
    n_instr, n_bind, n_edge, n_tasks = ctx.counts()
    records = n_instr + n_edge
    s0 = torch.cuda.current_stream()
    starts = [torch.cuda.Event(enable_timing=True) for _ in range(steps)]
    ends = [torch.cuda.Event(enable_timing=True) for _ in range(steps)]
    ctx.rewind()
    ctx.flush()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for k in range(steps):
        ctx.rewind()
        starts[k].record(s0)
        ctx.flush()  # one launch of ig_analyse
        ends[k].record(s0)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    assert ctx.sync() == 0 and ctx.counts()[0] == n_instr and ctx.counts()[2] == n_edge
    kern_s = float(np.mean([a.elapsed_time(b) for a, b in zip(starts, ends)])) / 1e3
    lat = latency_summary(ctx.task_times_ns())
    ctx.close()
    out = {"workload": name, "records_per_s": records * steps / wall, "ms_per_analysis": wall / steps * 1e3,
           "instructions": n_instr, "edges": n_edge, "bindings": n_bind, "tasks": n_tasks, "steps": steps,
           "oracle_digests_equal": equal,
           "roofline": roofline(algorithmic_bytes(gold), kern_s, copy_gbs, None) if gold else None}
    out.update(lat)
    if oracle_reps:
        out["cpu_oracle"] = oracle_median(stream, oracle_reps)
    elif gold:
        out["cpu_oracle"] = {"value": records / gold["oracle_seconds"], "unit": "records/s", "cores": 1,
                             "kind": "oracle", "stored": True,
                             "note": "not timed here: the stored single-core time of the run that wrote "
                                     "tests/golden (this build's container CPU)", "seconds": gold["oracle_seconds"]}
    return out


def run_task_graph_horizons(threads):
    """Horizons from the task graph (horizon mode 1) on a few streams: the
    2-D stencil (a chain: the same graph as the fixed step) and three
    batched streams (fewer horizons where tasks run side by side), each
    analysed on the GPU and compared with the oracle run here."""
    import torch
    import oracle
    from paper_2503_10516_amd import binding, streams
    cases = [("stencil2d", streams.stencil_2d())] + \
        [(f"batched_{i}", streams.batched_stream(streams.BATCHED_SEED, i, w_all=streams.BATCHED_W_ALL,
                                                 w_slice=streams.BATCHED_W_SLICE)) for i in (0, 5, 12)]
    out = []
    for name, s in cases:
        row = {"stream": name}
        for mode in (0, 1):
            s.horizon_mode = mode
            ctx = binding.make_context(s, threads=threads)
            ctx.record(s)
            torch.cuda.synchronize()
            t = time.perf_counter()
            ctx.flush()
            assert ctx.sync() == 0
            torch.cuda.synchronize()
            dt = time.perf_counter() - t
            st = ctx.stats()
            ctx.close()
            # the oracle beside it: its time is this object's CPU baseline,
            # and its digests are compared with the device's
            t = time.perf_counter()
            ref = oracle.run_stream(s, fetch=False)["stats"]
            oracle_s = time.perf_counter() - t
            rec = st["n_instructions"] + st["n_edges"]
            row[f"mode{mode}"] = {"gpu_ms": dt * 1e3, "horizons": st["per_kind"][5], "records": rec,
                                  "oracle_equal": all(st[k] == ref[k] for k in DIGEST_KEYS),
                                  "cpu_baseline": {"value": rec / oracle_s, "unit": "records/s", "cores": 1,
                                                   "kind": "oracle", "sample": "the whole stream, one run"}}
        s.horizon_mode = 0
        out.append(row)
        log(f"task-graph horizons {name}: {row['mode0']['horizons']} -> {row['mode1']['horizons']} horizons, "
            f"oracle equal {row['mode1']['oracle_equal']}")
    return out


# ---------------------------------------------------------------------------
# Host-staged device-to-device copies (Sec. 3.3, last paragraph)
# ---------------------------------------------------------------------------

def run_staged(steps, threads):
    """The 2-D stencil with staging on (devices that cannot copy to each
    other): analysis throughput and the digests against the oracle run
    here."""
    import dataclasses
    import numpy as np
    import torch
    import oracle
    from paper_2503_10516_amd import binding, streams
    s = dataclasses.replace(streams.stencil_2d(), staging=1, name="stencil2d_staged")
    ctx = binding.make_context(s, threads=threads)
    ctx.record(s)
    times = []
    for k in range(steps + 1):
        if k:
            ctx.rewind()
        torch.cuda.synchronize()
        t = time.perf_counter()
        ctx.flush()
        assert ctx.sync() == 0
        torch.cuda.synchronize()
        times.append(time.perf_counter() - t)
    st = ctx.stats()
    ctx.close()
    t = time.perf_counter()
    ref = oracle.run_stream(s, fetch=False)["stats"]
    oracle_s = time.perf_counter() - t
    rec = st["n_instructions"] + st["n_edges"]
    sec = float(np.median(times[1:]))
    return {"workload": "2-D 5-point stencil (4096x4096, 1000 tasks, 16 nodes x 8 devices, 128 chunks) with "
                        "device-to-device copies within a node staged through pinned host memory",
            "records": rec, "copies": st["per_kind"][2], "ms_per_analysis": sec * 1e3, "records_per_s": rec / sec,
            "oracle_equal": all(st[k] == ref[k] for k in DIGEST_KEYS),
            "cpu_baseline": {"value": rec / oracle_s, "unit": "records/s", "cores": 1, "kind": "oracle",
                             "sample": "the whole stream, one run"}}


# ---------------------------------------------------------------------------
# Out-of-order engine simulation (Sec. 4.1) over finished graphs
# ---------------------------------------------------------------------------

def ooo_algorithmic_bytes(n_instr, n_edges):
    """Bytes the engine must move at least: per instruction its result slot
    (32 written), its in-flight record (24 written), its lane class,
    duration and the two offset pairs (28 read); per edge the successor entry
    (4) and the successor's dependency-state record (24: half read, half
    written)."""
    return 84 * n_instr + 28 * n_edges


OOO_SRC = os.path.join(ROOT, "paper_2503_10516_amd", "csrc", "ig_ooo.hip")


def ooo_run(contexts, devices, steps, copy_gbs, counters=None):
    """Time `steps` runs of the engine over the contexts' graphs (one launch
    of the preparation kernels and the engine, HIP events on the stream)."""
    import numpy as np
    import torch
    from paper_2503_10516_amd import binding
    p = binding.ooo_params(devices)
    sim = binding.OooSimulation(contexts, p)
    stream = torch.cuda.current_stream()
    sim.run(stream)
    torch.cuda.synchronize()
    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(steps)]
    for a, b in ev:
        a.record(stream)
        sim.run(stream)
        b.record(stream)
    torch.cuda.synchronize()
    ms = [a.elapsed_time(b) for a, b in ev]
    summ = [sim.summary(i) for i in range(len(contexts))]
    sim.close()
    n = sum(int(c.counts()[0]) for c in contexts)
    ne = sum(int(c.counts()[2]) for c in contexts)
    sec = float(np.median(ms)) / 1e3
    ab = ooo_algorithmic_bytes(n, ne)
    return {"graphs": len(contexts), "instructions": n, "edges": ne, "run_ms": ms,
            "instructions_per_s": n / sec, "summaries": summ if len(summ) == 1 else None,
            "makespan_ns_max": max(s["makespan"] for s in summ),
            "eager_fraction": sum(s["eager"] for s in summ) / max(1, n),
            "roofline": {"bound": "hbm", "achieved": ab / sec / 1e9, "peak": PEAK_HBM_GBS, "unit": "GB/s",
                         "frac": ab / sec / 1e9 / PEAK_HBM_GBS,
                         "traffic": measured_traffic(counters, OOO_SRC) if counters else None,
                         "kernel": "ig_ooo_prep_* + ig_ooo_engine", "algorithmic_bytes": ab,
                         "frac_of_copy": ab / sec / 1e9 / copy_gbs if copy_gbs else None}}


def run_ooo_stencil2d(steps, threads, copy_gbs):
    """The engine over the 2-D stencil's graph (one workgroup), compared
    with the oracle's engine stored in tests/golden."""
    import numpy as np
    from paper_2503_10516_amd import binding, streams
    s = streams.stencil_2d()
    ctx = binding.make_context(s, threads=threads)
    ctx.record(s)
    ctx.flush()
    assert ctx.sync() == 0
    out = ooo_run([ctx], s.nodes * s.devices, steps, copy_gbs, "ig_ooo_stencil2d_counters.json")
    gold = load_json(os.path.join(GOLDEN, "stencil2d_full_ooo.json"))
    if gold:
        sim = binding.OooSimulation([ctx], binding.ooo_params(s.nodes * s.devices))
        sim.run()
        slots, summ = sim.fetch(0)
        sim.close()
        import hashlib
        out["oracle_equal"] = summ == gold["summary"] and \
            hashlib.sha256(slots.tobytes()).hexdigest() == gold["slots_sha256"]
        secs = gold["runs"][0]["oracle_seconds"]
        out["cpu_baseline"] = {"value": out["instructions"] / secs, "unit": "instructions/s", "cores": 1,
                               "kind": "oracle", "sample": f"the oracle's engine over the same graph, {secs} s on one "
                                                           "core of the host that wrote tests/golden (stored)"}
    ctx.close()
    out["workload"] = ("engine over the 2-D stencil's graph (16 nodes x 8 devices, 1000 tasks): 2 lanes per "
                       "device, 2 host lanes, window 1024, eager assignment, cost model of binding.ooo_params")
    return out


def run_serving(args):
    from paper_2503_10516_amd import serve, streams
    sessions = streams.serving_sessions(n_sessions=args.serving_sessions)
    gold = load_json(os.path.join(GOLDEN, "serving_digests.json")) or {}
    server = serve.Server(slots=64, threads=args.threads)
    out = {"workload": f"{len(sessions)} sessions (seed 0x{streams.SERVING_SEED:x}) drawn from the 1-D stencil, "
                       f"the 2-D stencil (1000 tasks), N-body (50 steps) and the growing pattern "
                       f"(queue cap 1..64); 64 slots", "sweep": []}
    for rate in [float(r) for r in args.serving_rates.split(",") if r]:
        r = server.run(sessions, rate, log=log)
        matched = checked = 0
        for s, st in zip(sessions, r.pop("session_stats")):
            kind = s.name.split("_", 1)[1]
            if kind in gold:
                checked += 1
                matched += all(st[k] == gold[kind][k] for k in DIGEST_KEYS)
        r["oracle_digests_matched"] = f"{matched}/{checked}"
        log(f"serving rate {rate:.0e}: p50 {r['p50_latency_us']:.0f} us, p99 {r['p99_latency_us']:.0f} us, "
            f"{r['tasks_per_s']:.0f} tasks/s, {matched}/{checked} sessions equal their oracle digests")
        out["sweep"].append(r)
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--threads", type=int, default=256, help="workgroup size of the single-stream objects")
    ap.add_argument("--workloads", default="stencil2d,nbody,stencil1d,tdag,serving,ooo,staged",
                    help="comma list of objects beside the batched headline: stencil2d, nbody, stencil1d, tdag "
                         "(horizons from the task graph), serving, ooo (the out-of-order engine simulated over "
                         "the 2-D stencil's and the batched graphs), staged (host-staged device copies)")
    ap.add_argument("--batch-threads", type=int, default=0, help="0: autotune")
    ap.add_argument("--batch-window", type=int, default=400, help="commands per launch while sizing")
    ap.add_argument("--serving-rates", default="1e3,1e5")
    ap.add_argument("--serving-sessions", type=int, default=32)
    ap.add_argument("--oracle-reps", type=int, default=5, help="oracle runs (median) of the small single streams")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="run only a plain 1 GiB device-to-device copy (scale for the HBM counters)")
    args = ap.parse_args()
    if args.copy_calibration:
        import torch
        a = torch.ones(1 << 28, dtype=torch.float32, device="cuda")
        b = torch.empty_like(a)
        for _ in range(3):
            b.copy_(a)
        torch.cuda.synchronize()
        print(json.dumps({"copy_bytes_read": a.numel() * 4, "copy_bytes_written": b.numel() * 4, "launches": 3}))
        return
    if args.gpus != 1:
        print(json.dumps({"error": "this benchmark runs on exactly one GPU: the analysed cluster is simulated, "
                                   "so --gpus must be 1"}))
        sys.exit(2)

    import torch
    from paper_2503_10516_amd import streams

    torch.cuda.set_device(0)
    copy_gbs = copy_bandwidth()
    log(f"device copy bandwidth {copy_gbs:.0f} GB/s")
    records, batched, gold = run_batched(args, copy_gbs)
    wall = batched.pop("wall_s")
    line = {
        "metric": METRIC,
        "value": records * args.steps / wall,
        "unit": "records/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": wall / args.steps * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "int64",
        "data": "synthetic",
        "config": {"workload": f"batched: 256 seeded task streams (seed "
                               f"0x{streams.BATCHED_SEED:x}) of uneven size in one graph launch, one workgroup "
                               f"per stream: 1-3-D buffers of 2^10..2^24 elements, 16..1024 chunks over 8-128 "
                               f"simulated devices, 50..2000 tasks; all/slice read weights "
                               f"{streams.BATCHED_W_ALL}/{streams.BATCHED_W_SLICE}",
                   "streams": 256, "tasks": batched["tasks"], "instructions": batched["instructions"],
                   "edges": batched["edges"], "threads_per_stream": batched["threads_per_stream"]},
        "p50_task_latency_us": batched["p50_task_latency_us"],
        "p99_task_latency_us": batched["p99_task_latency_us"],
        "roofline": batched.pop("roofline"),
    }
    if not args.no_cpu_baseline and gold:
        line["cpu_baseline"] = cpu_baseline_batched(gold, reps=3)
        log(f"cpu baseline: {line['cpu_baseline']['value']:.3g} records/s on {line['cpu_baseline']['cores']} cores")
    else:
        line["cpu_baseline"] = None
    line["batched"] = batched
    torch.cuda.empty_cache()
    work = set(w for w in args.workloads.split(",") if w)
    if "stencil2d" in work:
        line["stencil2d"] = run_single("2-D 5-point stencil: 2 buffers of 4096x4096, 1000 tasks, neighborhood(1,1) "
                                       "read + one_to_one write, 16 nodes x 8 devices, 128 chunks",
                                       streams.stencil_2d(), "stencil2d_full.json", max(args.steps, 5),
                                       args.threads, copy_gbs, args.oracle_reps)
        log(f"stencil2d: {line['stencil2d']['records_per_s']:.3g} records/s")
    if "nbody" in work:
        line["nbody"] = run_single("N-body: 2 buffers of 2^20 x 16 B, 500 steps (1000 tasks), all read + "
                                   "read_write, 16 nodes x 8 devices, 128 chunks", streams.nbody(),
                                   "nbody_full.json", 1, args.threads, copy_gbs, 0)
        log(f"nbody: {line['nbody']['records_per_s']:.3g} records/s")
        torch.cuda.empty_cache()
    if "stencil1d" in work:
        line["stencil1d"] = run_single("1-D 3-point stencil: 2 buffers of 4096, 64 tasks, 2 devices",
                                       streams.stencil_1d(), "stencil1d_full.json", max(args.steps, 10),
                                       args.threads, copy_gbs, 10)
    if "tdag" in work:
        line["task_graph_horizons"] = run_task_graph_horizons(args.threads)
    if "serving" in work:
        line["serving"] = run_serving(args)
    if "staged" in work:
        line["staged"] = run_staged(max(args.steps, 3), args.threads)
        log(f"staged stencil2d: {line['staged']['records_per_s']:.3g} records/s, oracle equal "
            f"{line['staged']['oracle_equal']}")
    if "ooo" in work:
        line["ooo"] = {"stencil2d": run_ooo_stencil2d(max(args.steps, 3), args.threads, copy_gbs),
                       "batched": line["batched"].pop("ooo", None)}
        log(f"ooo stencil2d: {line['ooo']['stencil2d']['instructions_per_s']:.3g} instructions/s")
    print(json.dumps(line))


if __name__ == "__main__":
    main()
