"""Per-phase device time of the analysis of single streams.

Needs the profiling build of the library (the same sources compiled with
IG_PHASE_PROFILE, which stamps the device clock between the phases of every
command on thread 0; the product build has no stamps):

    python -c "import __graft_entry__ as g; g.build_hip('paper_2503_10516_amd/libig_phases.so', ['-DIG_PHASE_PROFILE'])"
    python -m paper_2503_10516_amd.phase_profile paper_2503_10516_amd/libig_phases.so b248,b13,growing_q8 [threads]

Stream names: bN = stream N of the batched workload, stencil2d, nbody,
growing (unbounded queue), growing_qW (queue cap W), growing_nola.
"""
from __future__ import annotations

import sys
import time

from . import batch as BT
from . import binding as B
from . import streams as S

PHASES = ["INTAKE_REGIONS", "INTAKE_CHECKS", "LOOKAHEAD", "COMPILE_REGIONS", "ALLOC", "COH_COUNT", "SCANS",
          "COH_EMIT", "INBOX", "KERNELS", "EDGES_OUT", "SYNC", "OTHER"]


def make(name):
    if name.startswith("b"):
        return S.batched_stream(S.BATCHED_SEED, int(name[1:]), w_all=S.BATCHED_W_ALL, w_slice=S.BATCHED_W_SLICE)
    if name == "stencil2d":
        return S.stencil_2d()
    if name == "nbody":
        return S.nbody()
    if name == "growing_nola":
        return S.growing(lookahead=0)
    if name.startswith("growing_q"):
        return S.growing(queue_cap=int(name[len("growing_q"):]))
    if name == "growing":
        return S.growing()
    raise ValueError(name)


def profile(lib_path, name, threads=256):
    """Analyse one stream (growing capacities on overflow); returns
    (seconds, stats) with stats["phase_us"] per phase."""
    import torch
    s = make(name)
    caps = B.estimate_caps(s)
    caps.update(BT.fixed_caps(s))
    for _ in range(4):
        ctx = B.make_context(s, lib_path=lib_path, threads=threads, **caps)
        ctx.record(s)
        torch.cuda.synchronize()
        t = time.perf_counter()
        ctx.flush()
        st = ctx.sync()
        torch.cuda.synchronize()
        dt = time.perf_counter() - t
        if st == B.IG_E_CAPACITY:
            ctx.close()
            for k in ("cap_instructions", "cap_edges", "cap_state_words", "cap_unit", "cap_scratch"):
                caps[k] = int(caps[k] * 3)
            continue
        if st != 0:
            raise B.IgError("analysis", st)
        stats = ctx.stats()
        ctx.close()
        return s, dt, stats
    raise B.IgError("capacity", B.IG_E_CAPACITY)


def main(argv):
    import torch
    lib_path, names = argv[0], argv[1].split(",")
    threads = int(argv[2]) if len(argv) > 2 else 256
    torch.cuda.set_device(0)
    for name in names:
        s, dt, st = profile(lib_path, name, threads)
        print(f"{name}: {s.n_tasks} tasks, {s.chunks} chunks, {s.nodes}x{s.devices} devices, {threads} threads: "
              f"{dt:.3f} s, {st['n_instructions']} instructions, {st['n_edges']} edges", flush=True)
        total = sum(st["phase_us"]) or 1.0
        for k, p in enumerate(PHASES):
            if st["phase_count"][k]:
                print(f"    {p:16s} {st['phase_us'][k] / 1e3:10.1f} ms  {100 * st['phase_us'][k] / total:5.1f}%  "
                      f"n={st['phase_count'][k]}", flush=True)


if __name__ == "__main__":
    main(sys.argv[1:])
