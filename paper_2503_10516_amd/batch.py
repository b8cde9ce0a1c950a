"""Batched analysis: many independent command streams in one launch.

Each stream keeps its own context (state, records, ids), so its graph is the
same alone and in a batch.  The analysis kernel runs one workgroup per
stream; the launch is captured as a HIP graph (reset of every context, then
the analysis) and replayed.

Workgroups are dispatched to the eight XCDs of the chip round-robin by
block index, and each XCD has its own L2.  Streams are therefore ordered by
projected work, heaviest first, so that the heaviest eight land on eight
different XCDs, the next eight likewise, and so on.

Capacities come from a projection of each stream's record counts; a stream
that still overflows is re-created with larger capacities and re-run before
anything is timed (capacities never change the output).
"""
from __future__ import annotations

from typing import Callable, Dict, List, Optional, Sequence

import numpy as np

from . import binding as B


def state_words(stream) -> int:
    """Device state heap (32-bit words) for a stream: coordinate-compressed
    cell grids per buffer plus per-allocation cell records, with room for
    power-of-two block rounding.  A sizing heuristic only."""
    C = stream.chunks
    nbh = any(a.mapper == 1 for c in stream.cmds if c[0] == "task" for a in c[1].accesses)
    words = 1 << 16
    for c in stream.cmds:
        if c[0] != "buffer":
            continue
        ext = c[2]
        cells = min(ext[0] + 1, 4 * C + 8)
        for d in (1, 2):
            cells *= min(ext[d] + 1, 10 if nbh else 3)
        words += 64 * cells
    return int(min(max(4 * words, 1 << 20), 1 << 27))


CAP_NAMES = {1: "instructions", 2: "edges", 3: "bindings", 4: "state", 5: "readers", 6: "unit", 7: "scratch",
             8: "live", 9: "commands", 10: "buffers", 11: "allocs"}
GROWABLE = {"instructions": "records", "edges": "records", "bindings": "records", "state": "state",
            "readers": "state", "unit": "unit", "scratch": "scratch"}


def _release_cached() -> None:
    try:
        import torch
        if torch.cuda.is_available():
            torch.cuda.synchronize()
            torch.cuda.empty_cache()
    except ImportError:
        pass


def fixed_caps(stream) -> Dict[str, int]:
    """Per-stream sizes of the state heap, the compile unit and the worker
    scratch, from the stream's shape (heuristics; a stream that overflows is
    re-sized)."""
    C = stream.chunks
    T = stream.nodes * stream.devices
    K = max(1, C // T)
    allish = any(a.mode & 1 and (a.mapper in (2, 4) or (a.mapper == 3 and a.slice_dim == 0))
                 for c in stream.cmds if c[0] == "task" for a in c[1].accesses)
    unit = 1 << 18
    if allish:
        unit = max(unit, 2 * (T * (C - K) + T + C))
    return {"cap_state_words": state_words(stream) * (2 if C >= 512 else 1),
            "cap_unit": unit, "cap_scratch": max(8192, 16 * C + 4096)}


def projected_records(stream) -> int:
    i, e = B.project_counts(stream)
    return i + e


class Batch:
    """Contexts for a list of streams, analysed together."""

    def __init__(self, streams: Sequence, threads: int = 256, margin: float = 2.0, floor: int = 4096,
                 lib_path: Optional[str] = None):
        self.streams = list(streams)
        self.floor = floor
        self.threads = threads
        self.lib_path = lib_path
        weight = [projected_records(s) for s in self.streams]
        # heaviest first: block b runs on XCD b % 8
        self.order = sorted(range(len(self.streams)), key=lambda i: -weight[i])
        self.margin = margin
        self.grow = [dict(records=1.0, state=1.0, unit=1.0, scratch=1.0) for _ in self.streams]
        self.contexts: List[Optional[B.Context]] = [None] * len(self.streams)
        for i in range(len(self.streams)):
            self._create(i)
        self.graph: Optional[B.BatchGraph] = None

    def _create(self, i: int) -> None:
        s = self.streams[i]
        g = self.grow[i]
        caps = B.estimate_caps(s, self.margin * g["records"], self.floor)
        base = fixed_caps(s)
        caps["cap_state_words"] = min(int(base["cap_state_words"] * g["state"]), 1 << 29)
        caps["cap_unit"] = min(int(base["cap_unit"] * g["unit"]), 1 << 26)
        caps["cap_scratch"] = min(int(base["cap_scratch"] * g["scratch"]), 1 << 22)
        ctx = B.make_context(s, lib_path=self.lib_path, threads=self.threads, **caps)
        ctx.record(s)
        self.contexts[i] = ctx

    def launch_order(self) -> List[B.Context]:
        return [self.contexts[i] for i in self.order]

    def n_commands(self, i: int) -> int:
        return len(self.streams[i].cmds)

    def analyse(self, idx: Sequence[int], window: int = 0, log: Optional[Callable] = None) -> np.ndarray:
        """Re-analyse the streams idx from the start, in launches of at most
        `window` commands per stream (0: one launch).  Streams that finish or
        fail drop out of later launches.  Returns their progress rows."""
        idx = list(idx)
        ctxs = [self.contexts[i] for i in idx]
        B.batch_rewind(ctxs)
        rows = {}
        active = list(range(len(idx)))
        launches = 0
        while active:
            part = [ctxs[a] for a in active]
            B.batch_flush(part, window=window)
            launches += 1
            prog = B.batch_progress(part)
            still = []
            for a, p in zip(active, prog):
                rows[a] = p
                if p[2] == 0 and p[5] < self.n_commands(idx[a]):
                    still.append(a)
            if log is not None:
                log(launches, len(active), prog)
            if window == 0:
                break
            active = still
        return np.array([rows[a] for a in range(len(idx))], dtype=np.int64)

    def size(self, window: int = 0, max_rounds: int = 4, log: Optional[Callable] = None) -> Dict[str, int]:
        """Analyse once; re-create and re-run the streams that ran out of a
        capacity, growing that capacity.  Returns the overflow counts by kind."""
        grown: Dict[str, int] = {}
        todo = list(self.order)
        for _ in range(max_rounds + 1):
            prog = self.analyse(todo, window, log)
            bad = []
            for i, p in zip(todo, prog):
                if p[2] == 0:
                    continue
                what = CAP_NAMES.get(int(p[4]), "?")
                if p[2] != B.IG_E_CAPACITY or what not in GROWABLE:
                    raise B.IgError(f"analysis of {self.streams[i].name} ({what})", int(p[2]))
                grown[what] = grown.get(what, 0) + 1
                self.grow[i][GROWABLE[what]] *= 3
                bad.append(i)
            if not bad:
                return grown
            for i in bad:
                self.contexts[i].close()
                self.contexts[i] = None
            _release_cached()
            for i in bad:
                self._create(i)
            todo = bad
        raise B.IgError("capacity sizing", B.IG_E_CAPACITY)

    def capture(self) -> None:
        self.graph = B.BatchGraph(self.launch_order())

    def launch(self) -> None:
        """Re-analyse every stream from the start in one graph launch."""
        if self.graph is None:
            self.capture()
        self.graph.launch()

    def progress(self) -> np.ndarray:
        return B.batch_progress(self.launch_order())

    def counts(self) -> np.ndarray:
        """(n, 4): instructions, bindings, edges, tasks per stream (input order)."""
        return np.array([c.counts() for c in self.contexts], dtype=np.int64)

    def close(self) -> None:
        if self.graph is not None:
            self.graph.close()
            self.graph = None
        for c in self.contexts:
            if c is not None:
                c.close()
        self.contexts = []
