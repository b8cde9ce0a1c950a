#!/usr/bin/env python3
"""Benchmark: instruction-graph generation throughput and per-task latency.

Workload: the 2-D 5-point stencil (WaveSim access pattern) -- two 4096 x 4096
buffers, 1000 tasks, neighborhood(1,1) read + one_to_one write, 16 simulated
nodes x 8 devices, 128 row-block chunks, lookahead on.  One step analyses the
whole recorded stream from scratch on one MI355X (rewind + one launch of the
analysis kernel); the recorded commands are resident in HBM before the timed
region starts.  Output: one JSON line.

Metric: instructions + edges generated per second (whole job), with the p50 /
p99 per-task scheduling latency (device clock, from the start of a task's
intake to the moment its records are complete, lookahead holding included).
"""
import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "instructions+edges generated/sec and p99 per-task scheduling latency"
PEAK_HBM_GBS = 8000.0
KERNEL_SRC = os.path.join(ROOT, "paper_2503_10516_amd", "csrc", "ig_kernels.hip")
COUNTERS = os.path.join(ROOT, "profiles", "ig_analyse_stencil2d_counters.json")


def algorithmic_bytes(n_instr, n_bind, n_edge, stream):
    """Bytes the method must move per analysis: the output records in their
    device layout (74 B per instruction, 12 B per binding, 9 B per edge) and
    the task descriptors it reads (64 B + 80 B per accessor)."""
    inp = 0
    for c in stream.cmds:
        inp += 64 + 80 * len(c[1].accesses) if c[0] == "task" else 16
    return 74 * n_instr + 12 * n_bind + 9 * n_edge + inp


def kernel_sha():
    with open(KERNEL_SRC, "rb") as f:
        return hashlib.sha256(f.read()).hexdigest()[:16]


def measured_traffic():
    """HBM bytes per launch from the committed rocprofv3 counter summary, if
    it was taken on the current kernel source."""
    try:
        with open(COUNTERS) as f:
            d = json.load(f)
    except (OSError, ValueError):
        return None
    if d.get("kernel_sha") != kernel_sha():
        return None
    return d.get("hbm_bytes_per_launch")


def cpu_baseline(stream):
    import oracle  # test infrastructure, timed here as the CPU reference
    t0 = time.perf_counter()
    out = oracle.run_stream(stream, fetch=False)
    dt = time.perf_counter() - t0
    st = out["stats"]
    n = st["n_instructions"] + st["n_edges"]
    return {"value": n / dt, "unit": "records/s", "cores": 1, "kind": "oracle",
            "sample": f"the whole workload ({stream.n_tasks} tasks, {n} records), single-threaded C++17 oracle, "
                      f"{dt:.2f} s"}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--threads", type=int, default=256)
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

    import numpy as np
    import torch
    from paper_2503_10516_amd import binding, streams

    torch.cuda.set_device(0)
    s = streams.stencil_2d()
    ctx = binding.make_context(s, threads=args.threads)
    ctx.record(s)
    ctx.flush()  # uploads the recorded commands, first analysis
    if ctx.sync() != 0:
        raise SystemExit("analysis failed")
    n_instr, n_bind, n_edge, n_tasks = ctx.counts()
    records = n_instr + n_edge
    stream = torch.cuda.current_stream()
    for _ in range(args.warmup):
        ctx.rewind()
        ctx.flush()
    torch.cuda.synchronize()

    starts = [torch.cuda.Event(enable_timing=True) for _ in range(args.steps)]
    ends = [torch.cuda.Event(enable_timing=True) for _ in range(args.steps)]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for k in range(args.steps):
        ctx.rewind()
        starts[k].record(stream)
        ctx.flush()  # one launch of ig_analyse
        ends[k].record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    if ctx.sync() != 0:
        raise SystemExit("analysis failed")
    assert ctx.counts()[0] == n_instr and ctx.counts()[2] == n_edge
    kernel_ms = [a.elapsed_time(b) for a, b in zip(starts, ends)]
    avg_kernel_s = sum(kernel_ms) / len(kernel_ms) / 1e3
    times = ctx.task_times_ns()
    lat_us = (times[:, 1] - times[:, 0]) / 1e3
    ab = algorithmic_bytes(n_instr, n_bind, n_edge, s)
    achieved = ab / avg_kernel_s / 1e9
    traffic = measured_traffic()
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
        "config": {"workload": "2-D 5-point stencil: 2 buffers of 4096x4096, 1000 tasks, neighborhood(1,1) read + "
                               "one_to_one write, 16 nodes x 8 devices, 128 chunks, lookahead on",
                   "instructions": n_instr, "edges": n_edge, "bindings": n_bind, "tasks": n_tasks,
                   "threads_per_stream": args.threads},
        "p50_task_latency_us": float(np.percentile(lat_us, 50)),
        "p99_task_latency_us": float(np.percentile(lat_us, 99)),
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": PEAK_HBM_GBS, "unit": "GB/s",
                     "frac": achieved / PEAK_HBM_GBS, "traffic": traffic,
                     "kernel": "ig_analyse", "kernel_ms": avg_kernel_s * 1e3, "algorithmic_bytes": ab},
    }
    if not args.no_cpu_baseline:
        line["cpu_baseline"] = cpu_baseline(s)
    else:
        line["cpu_baseline"] = None
    ctx.close()
    print(json.dumps(line))


if __name__ == "__main__":
    main()
