"""Serving: a request loop with continuous batching of command streams.

Sessions (independent user programs, each its own context) are admitted
into a fixed number of slots as slots and arena memory free up.  Tasks
arrive over time; the host records each arrived task into its session's
context while the device analyses the previous window, and every launch
analyses the new commands of all sessions that have any, in one batched
launch (one workgroup per session).  Region maps stay resident on the device
between launches.  A task's latency runs from its arrival until the launch
after which its records are complete (lookahead holding included).

Arrivals: one Poisson process over all tasks; the k-th arrival goes to the
admitted sessions round-robin (sessions submit their tasks in order).  A
task that arrives while no admitted session has tasks left waits for the
next admission, and that wait counts in its latency.
"""
from __future__ import annotations

import time
from collections import deque
from typing import Callable, Dict, List, Optional, Sequence

import numpy as np

from . import binding as B
from . import streams as S


class _HostEvent:
    """Launches of the host test build complete synchronously."""

    def query(self) -> bool:
        return True


class _Session:
    def __init__(self, index: int, stream, lib_path=None, threads: int = 256):
        self.index = index
        self.stream = stream
        self.caps = B.estimate_caps(stream)
        self.bytes = session_bytes(stream, self.caps, lib_path, threads)
        # commands before the first task, then each task with the non-task
        # commands that follow it
        self.prefix: List[tuple] = []
        self.units: List[List[tuple]] = []
        for c in stream.cmds:
            if c[0] == "task":
                self.units.append([c])
            elif self.units:
                self.units[-1].append(c)
            else:
                self.prefix.append(c)
        self.n_tasks = len(self.units)
        # descriptors are built before serving starts (client-side work)
        self.descs = [B.task_desc(u[0][1]) for u in self.units]
        self.arrival = np.full(self.n_tasks, np.nan)
        self.done_at = np.full(self.n_tasks, np.nan)
        self.submitted = 0
        self.done = 0
        self.ctx: Optional[B.Context] = None
        self.pending = False  # recorded commands not yet analysed
        self.recorded = 0     # commands recorded into the context
        self.stats: Optional[Dict[str, object]] = None


def session_bytes(stream, caps, lib_path=None, threads: int = 256) -> int:
    import ctypes
    kw = stream.desc()
    kw.update(caps)
    d = B.ContextDesc()
    d.nodes, d.devices_per_node, d.chunks = kw["nodes"], kw["devices"], kw["chunks"]
    d.horizon_step, d.lookahead = kw["horizon_step"], kw["lookahead"]
    d.flush_horizons, d.queue_cap = kw["flush_horizons"], kw["queue_cap"]
    d.cap_commands, d.cap_instructions, d.cap_edges = kw["cap_commands"], kw["cap_instructions"], kw["cap_edges"]
    d.threads = threads
    n = ctypes.c_uint64()
    st = B.lib(lib_path).ig_arena_bytes(ctypes.byref(d), ctypes.byref(n))
    if st != 0:
        raise B.IgError("ig_arena_bytes", st)
    return int(n.value)


class Server:
    """Continuous-batching analysis server over `slots` concurrent sessions
    and an arena memory budget."""

    def __init__(self, slots: int = 64, threads: int = 256, mem_budget: int = 96 << 30,
                 lib_path: Optional[str] = None, window: int = 16):
        # window: commands per session per launch (0: all pending); short
        # launches report completions often and keep one long session from
        # holding back the others
        self.window = window
        self.slots = slots
        self.threads = threads
        self.mem_budget = mem_budget
        self.lib_path = lib_path

    def run(self, streams: Sequence, rate: float, seed: int = S.SERVING_SEED,
            log: Optional[Callable[[str], None]] = None, keep_stats: bool = True) -> Dict[str, object]:
        sessions = [_Session(i, s, self.lib_path, self.threads) for i, s in enumerate(streams)]
        host = self.lib_path is not None
        total = sum(s.n_tasks for s in sessions)
        arrivals = S.poisson_arrivals(total, rate, seed)
        waiting = deque(sessions)  # not yet admitted
        active: List[_Session] = []
        rr: deque = deque()  # admitted sessions with tasks left to submit
        mem_used = 0
        next_arr = 0
        finished = 0
        launches = 0
        launch_sizes = []
        inflight: Optional[tuple] = None
        t0 = time.perf_counter()
        last_log = t0

        def admit(now):
            nonlocal mem_used
            while waiting and len(active) < self.slots:
                s = waiting[0]
                if active and mem_used + s.bytes > self.mem_budget:
                    return
                waiting.popleft()
                s.ctx = B.make_context(s.stream, lib_path=self.lib_path, threads=self.threads, **s.caps)
                for c in s.prefix:
                    s.ctx.record_command(c)
                s.recorded = len(s.prefix)
                s.pending = True
                mem_used += s.bytes
                active.append(s)
                rr.append(s)

        while finished < len(sessions):
            now = time.perf_counter() - t0
            admit(now)
            # arrivals up to now, round-robin over sessions with tasks left
            while next_arr < total and arrivals[next_arr] <= now and rr:
                s = rr.popleft()
                s.arrival[s.submitted] = arrivals[next_arr]
                unit = s.units[s.submitted]
                s.ctx.submit_desc(s.descs[s.submitted])
                for c in unit[1:]:
                    s.ctx.record_command(c)
                s.recorded += len(unit)
                s.submitted += 1
                s.pending = True
                next_arr += 1
                if s.submitted < s.n_tasks:
                    rr.append(s)
            # the device: collect the finished launch, start the next one
            if inflight is not None and not inflight[0].query():
                continue
            if inflight is not None:
                t_done = time.perf_counter() - t0
                _, launched = inflight
                inflight = None
                prog = B.batch_progress([s.ctx for s in launched])
                for s, p in zip(launched, prog):
                    if p[2] != 0:
                        raise B.IgError(f"analysis of {s.stream.name}", int(p[2]))
                    d = int(p[0])
                    if d > s.done:
                        s.done_at[s.done:d] = t_done
                        s.done = d
                    if p[5] < s.recorded:
                        s.pending = True
                    if p[3] == 1 and s.done == s.n_tasks:
                        if keep_stats:
                            s.stats = s.ctx.stats()
                        s.ctx.close()
                        s.ctx = None
                        active.remove(s)
                        mem_used -= s.bytes
                        finished += 1
                admit(t_done)
            ready = [s for s in active if s.pending]
            if ready:
                B.batch_flush([s.ctx for s in ready], window=self.window)
                if host:
                    ev = _HostEvent()
                else:
                    import torch
                    ev = torch.cuda.Event()
                    ev.record(torch.cuda.current_stream())
                for s in ready:
                    s.pending = False
                inflight = (ev, ready)
                launches += 1
                launch_sizes.append(len(ready))
            if log is not None and time.perf_counter() - last_log > 5.0:
                last_log = time.perf_counter()
                log(f"serving rate {rate:.0e}: {finished}/{len(sessions)} sessions done, "
                    f"{next_arr}/{total} tasks arrived, {launches} launches")
        wall = time.perf_counter() - t0
        lat = np.concatenate([s.done_at - s.arrival for s in sessions])
        recs = sum(s.stats["n_instructions"] + s.stats["n_edges"] for s in sessions) if keep_stats else 0
        return {
            "rate": rate, "sessions": len(sessions), "tasks": total, "wall_s": wall,
            "tasks_per_s": total / wall, "records_per_s": recs / wall,
            "p50_latency_us": float(np.percentile(lat, 50) * 1e6),
            "p99_latency_us": float(np.percentile(lat, 99) * 1e6),
            "launches": launches, "mean_sessions_per_launch": float(np.mean(launch_sizes)) if launch_sizes else 0.0,
            "session_stats": [s.stats for s in sessions] if keep_stats else None,
        }
