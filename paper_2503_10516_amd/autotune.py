"""Autotuning of the batched launch.

The knob that changes only speed, never the output, is the workgroup size
per stream (`threads`): 64 keeps a stream inside one wavefront, so its
barriers are cheap, while larger groups give each simulated device a team of
threads for its large scans.  A batched launch lasts as long as its heaviest
stream, so the tuner times each candidate on the heaviest streams of the
batch (by projected records), each cut to a prefix that contains its first
task with an all-like read (the tasks that dominate them), next to evenly
spaced lighter streams, and keeps the candidate with the lowest median over
`reps` runs.

The command window per launch only bounds the sizing launches (a stream
re-created with larger capacities is re-run before anything is timed); the
timed graph launch analyses every stream in one launch, so the window is not
tuned.
"""
from __future__ import annotations

import time
from typing import Dict, List, Optional, Sequence

import numpy as np

from . import batch as BT
from . import streams as S


def _allish(task) -> bool:
    return any(a.mode == S.READ and (a.mapper in (S.ALL, S.FIXED) or (a.mapper == S.SLICE and a.slice_dim == 0))
               for a in task.accesses)


def _cut(s, commands: int, name: str):
    cut = s.cmds[:commands]
    if cut[-1][0] != "shutdown":
        cut = cut + [("shutdown",)]
    return S.Stream(s.nodes, s.devices, s.chunks, s.horizon_step, s.lookahead, s.flush_horizons, s.queue_cap,
                    cmds=cut, name=name)


def sample_streams(streams: Sequence, n_heavy: int = 8, n_spread: int = 8, commands: int = 60,
                   heavy_commands: int = 200) -> List:
    """The n_heavy heaviest streams, each cut after its first all-like read
    task (at least heavy_commands commands), and n_spread lighter ones cut to
    `commands` commands."""
    order = sorted(range(len(streams)), key=lambda i: -BT.projected_records(streams[i]))
    out = []
    for i in order[:n_heavy]:
        s = streams[i]
        first = next((q for q, c in enumerate(s.cmds) if c[0] == "task" and _allish(c[1])), None)
        n = heavy_commands if first is None else max(heavy_commands, first + 16)
        out.append(_cut(s, n, s.name + f"_first{n}"))
    rest = order[n_heavy:]
    if rest and n_spread:
        step = max(1, len(rest) // n_spread)
        for i in rest[::step][:n_spread]:
            out.append(_cut(streams[i], commands, streams[i].name + f"_first{commands}"))
    return out


def _sync():
    try:
        import torch
        if torch.cuda.is_available():
            torch.cuda.synchronize()
    except ImportError:
        pass


def tune(streams: Sequence, thread_candidates=(64, 128, 256), reps: int = 3,
         lib_path: Optional[str] = None, log=None) -> Dict[str, object]:
    """Returns {"threads": t, "seconds": {t: median s}, "runs": {t: [s, ...]}}."""
    sample = sample_streams(streams)
    runs: Dict[int, List[float]] = {}
    for t in thread_candidates:
        bt = BT.Batch(sample, threads=t, lib_path=lib_path)
        bt.size()
        runs[t] = []
        for _ in range(reps):
            _sync()
            t0 = time.perf_counter()
            bt.analyse(bt.order)
            _sync()
            runs[t].append(time.perf_counter() - t0)
        bt.close()
        if log is not None:
            log(f"autotune threads={t}: median {np.median(runs[t]) * 1e3:.1f} ms of {reps}")
    med = {t: float(np.median(v)) for t, v in runs.items()}
    best = min(med, key=med.get)
    return {"threads": best, "seconds": {str(t): v for t, v in med.items()},
            "runs": {str(t): v for t, v in runs.items()}, "sample_streams": len(sample)}
