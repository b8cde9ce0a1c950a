"""Autotuning of the batched launch.

Two knobs change only speed, never the output: the workgroup size per
stream (`threads`: 64 keeps a stream inside one wavefront, so its barriers
are cheap, while larger groups give streams with many simulated devices a
worker per device) and the command window per launch.  The tuner times each
candidate on a sample of the batch -- the heaviest streams by projected
records plus evenly spaced lighter ones, each cut to its first commands --
and keeps the fastest.
"""
from __future__ import annotations

import time
from typing import Dict, List, Optional, Sequence

from . import batch as BT
from . import streams as S


def sample_streams(streams: Sequence, n_heavy: int = 2, n_spread: int = 4, commands: int = 60) -> List:
    order = sorted(range(len(streams)), key=lambda i: -BT.projected_records(streams[i]))
    pick = order[:n_heavy]
    rest = order[n_heavy:]
    if rest and n_spread:
        step = max(1, len(rest) // n_spread)
        pick += rest[::step][:n_spread]
    out = []
    for i in pick:
        s = streams[i]
        cut = s.cmds[:commands]
        if cut[-1][0] != "shutdown":
            cut = cut + [("shutdown",)]
        out.append(S.Stream(s.nodes, s.devices, s.chunks, s.horizon_step, s.lookahead, s.flush_horizons,
                            s.queue_cap, cmds=cut, name=s.name + f"_first{commands}"))
    return out


def _sync():
    try:
        import torch
        if torch.cuda.is_available():
            torch.cuda.synchronize()
    except ImportError:
        pass


def tune(streams: Sequence, thread_candidates=(64, 256), window_candidates=(0,), reps: int = 1,
         lib_path: Optional[str] = None, log=None) -> Dict[str, object]:
    """Returns {"threads": t, "window": w, "seconds": {(t, w): s}}."""
    sample = sample_streams(streams)
    timings = {}
    for t in thread_candidates:
        bt = BT.Batch(sample, threads=t, lib_path=lib_path)
        bt.size()
        for w in window_candidates:
            best = float("inf")
            for _ in range(reps):
                _sync()
                t0 = time.perf_counter()
                bt.analyse(bt.order, window=w)
                _sync()
                best = min(best, time.perf_counter() - t0)
            timings[(t, w)] = best
            if log is not None:
                log(f"autotune threads={t} window={w}: {best * 1e3:.1f} ms")
        bt.close()
    (t, w) = min(timings, key=timings.get)
    return {"threads": t, "window": w, "seconds": {f"{k[0]}/{k[1]}": v for k, v in timings.items()}}
