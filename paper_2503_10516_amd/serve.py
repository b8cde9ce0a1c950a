"""Serving: a request loop with continuous batching of command streams.

Sessions (independent user programs, each its own context) are admitted
into the slots of an ig_server (C ABI) as slots and arena memory free up
(ig_server_admit answers IG_E_BUSY otherwise).  Tasks arrive over time; the
host records each arrived task into its session while earlier launches run,
and every poll queues a batched launch over the sessions with new commands
(one workgroup each), up to two launches in flight on the stream.  Region
maps stay resident on the device between launches.  A task's latency runs
from its arrival until the poll that finds its records complete
(fetchable), lookahead holding included; the holding part is reported
separately from the device's per-task stamps.

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


class _Session:
    def __init__(self, index: int, stream):
        self.index = index
        self.stream = stream
        self.caps = B.estimate_caps(stream)
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
        self.slot: Optional[int] = None
        self.ctx: Optional[B.Context] = None   # recording view while admitted, then the detached context
        self.stats: Optional[Dict[str, object]] = None
        self.times: Optional[np.ndarray] = None


class Server:
    """The request loop of the serving workload over an ig_server with
    `slots` sessions and an arena budget."""

    def __init__(self, slots: int = 64, threads: int = 256, mem_budget: int = 96 << 30,
                 lib_path: Optional[str] = None, window: int = 16, max_inflight: int = 2):
        # window: commands per session per launch (0: all recorded); short
        # launches report completions often and keep one long session from
        # holding back the others
        self.window = window
        self.slots = slots
        self.threads = threads
        self.mem_budget = mem_budget
        self.lib_path = lib_path
        self.max_inflight = max_inflight

    def run(self, streams: Sequence, rate: float, seed: int = S.SERVING_SEED,
            log: Optional[Callable[[str], None]] = None, keep_stats: bool = True) -> Dict[str, object]:
        sessions = [_Session(i, s) for i, s in enumerate(streams)]
        srv = B.Server(self.slots, threads=self.threads, window=self.window, max_inflight=self.max_inflight,
                       arena_budget=self.mem_budget, lib_path=self.lib_path)
        total = sum(s.n_tasks for s in sessions)
        arrivals = S.poisson_arrivals(total, rate, seed)
        waiting = deque(sessions)  # not yet admitted
        by_slot: Dict[int, _Session] = {}
        rr: deque = deque()  # admitted sessions with tasks left to submit
        next_arr = 0
        finished = 0
        polls = launches_seen = 0
        busy_admits = 0
        t0 = time.perf_counter()
        last_log = t0
        while finished < len(sessions):
            # admission: as many waiting sessions as slots and memory allow
            while waiting:
                s = waiting[0]
                slot = srv.admit(s.stream, threads=self.threads, **s.caps)
                if slot is None:
                    busy_admits += 1
                    break
                waiting.popleft()
                s.slot = slot
                s.ctx = srv.context(slot)
                for c in s.prefix:
                    s.ctx.record_command(c)
                by_slot[slot] = s
                if s.n_tasks:
                    rr.append(s)
            # arrivals up to now, round-robin over sessions with tasks left
            now = time.perf_counter() - t0
            while next_arr < total and arrivals[next_arr] <= now and rr:
                s = rr.popleft()
                s.arrival[s.submitted] = arrivals[next_arr]
                unit = s.units[s.submitted]
                srv.submit(s.slot, s.descs[s.submitted])
                for c in unit[1:]:
                    s.ctx.record_command(c)
                s.submitted += 1
                next_arr += 1
                if s.submitted < s.n_tasks:
                    rr.append(s)
            # the device: collect finished launches, queue the next ones
            prog = srv.poll(wait=False)
            polls += 1
            t_now = time.perf_counter() - t0
            for p in prog:
                s = by_slot[p.slot]
                if p.error != 0:
                    raise B.IgError(f"analysis of {s.stream.name}", int(p.error))
                d = int(p.tasks_done)
                if d > s.done:
                    s.done_at[s.done:d] = t_now
                    s.done = d
                if p.finished and s.done == s.n_tasks and not p.in_flight:
                    ctx = srv.detach(p.slot)
                    if ctx is not None:
                        del by_slot[p.slot]
                        s.ctx = ctx
                        finished += 1
            if log is not None and time.perf_counter() - last_log > 5.0:
                last_log = time.perf_counter()
                log(f"serving rate {rate:.0e}: {finished}/{len(sessions)} sessions done, "
                    f"{next_arr}/{total} tasks arrived")
        wall = time.perf_counter() - t0
        srv.close()
        lat = np.concatenate([s.done_at - s.arrival for s in sessions])
        recs = 0
        holds = []
        for s in sessions:
            if keep_stats:
                s.stats = s.ctx.stats()
                recs += s.stats["n_instructions"] + s.stats["n_edges"]
            t = s.ctx.task_times_ns()
            holds.append((t[:, 2] - t[:, 1]) / 1e3)
            launches_seen = max(launches_seen, int(s.stats["launches"]) if keep_stats else 0)
            s.ctx.close()
            s.ctx = None
        hold = np.concatenate(holds) if holds else np.zeros(0)
        return {
            "rate": rate, "sessions": len(sessions), "tasks": total, "wall_s": wall,
            "tasks_per_s": total / wall, "records_per_s": recs / wall,
            "p50_latency_us": float(np.percentile(lat, 50) * 1e6), "p99_latency_us": float(np.percentile(lat, 99) * 1e6),
            "p50_holding_us": float(np.percentile(hold, 50)) if len(hold) else 0.0,
            "p99_holding_us": float(np.percentile(hold, 99)) if len(hold) else 0.0,
            "polls": polls, "busy_admissions": busy_admits, "launches": launches_seen,
            "window": self.window, "max_inflight": self.max_inflight,
            "session_stats": [s.stats for s in sessions] if keep_stats else [],
        }
