"""ctypes binding of libig (include/ig.h): argument marshalling only.

Every step of instruction-graph generation runs in the HIP kernels of
libig.so; this module builds descriptors, hands over device memory and the
stream (from PyTorch, when a GPU is present) and copies records out.  If the
library is missing the import of `lib()` fails loudly; there is no fallback.
"""
from __future__ import annotations

import ctypes
import os
import time
from typing import Dict, List, Optional, Sequence, Tuple

import numpy as np

PKG_DIR = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(PKG_DIR, "libig.so")

INSTR_DTYPE = np.dtype([
    ("id", "<u8"), ("kind", "u1"), ("flags", "u1"), ("mem", "<u2"), ("src_mem", "<u2"),
    ("pad0", "<u2"), ("task", "<u4"), ("chunk", "<u4"), ("buffer", "<u4"), ("pad1", "<u4"),
    ("alloc", "<u8"), ("src_alloc", "<u8"), ("min", "<i8", (3,)), ("max", "<i8", (3,)),
])
BIND_DTYPE = np.dtype([("instr", "<u8"), ("access", "<u4"), ("pad", "<u4"), ("alloc", "<u8")])
EDGE_DTYPE = np.dtype([("from", "<u8"), ("to", "<u8"), ("kinds", "<u4"), ("pad", "<u4")])

IG_OK, IG_W_UNINIT_READ, IG_E_INVALID, IG_E_OVERLAPPING_WRITE, IG_E_CAPACITY, IG_E_DEVICE, IG_E_BUSY = \
    0, 1, -1, -2, -3, -4, -5
IG_E_INTERNAL = -6
IG_ALLOC, IG_COPY, IG_FREE, IG_KERNEL, IG_HORIZON, IG_EPOCH = 1, 2, 3, 4, 5, 6
IG_F_RESIZE, IG_F_INTER_NODE = 1, 2
IG_OOO_ENGINE, IG_OOO_DIRECT, IG_OOO_EAGER = 0, 1, 2


class IgError(RuntimeError):
    def __init__(self, where: str, status: int):
        detail = ""
        if status == IG_E_DEVICE:
            try:
                detail = " (" + lib().ig_last_error().decode(errors="replace") + ")"
            except Exception:
                pass
        super().__init__(f"{where} failed: {status}{detail}")
        self.status = status


class Box(ctypes.Structure):
    _fields_ = [("min", ctypes.c_int64 * 3), ("max", ctypes.c_int64 * 3)]


class Access(ctypes.Structure):
    _fields_ = [("buffer", ctypes.c_uint32), ("mode", ctypes.c_uint8), ("mapper", ctypes.c_uint8),
                ("slice_dim", ctypes.c_uint8), ("pad", ctypes.c_uint8),
                ("radius", ctypes.c_int64 * 3), ("fixed", Box)]


class TaskDesc(ctypes.Structure):
    _fields_ = [("dims", ctypes.c_uint32), ("n_access", ctypes.c_uint32), ("box", Box),
                ("access", Access * 8)]


class ContextDesc(ctypes.Structure):
    _fields_ = [("nodes", ctypes.c_uint32), ("devices_per_node", ctypes.c_uint32),
                ("chunks", ctypes.c_uint32), ("horizon_step", ctypes.c_uint32),
                ("lookahead", ctypes.c_uint32), ("flush_horizons", ctypes.c_uint32),
                ("queue_cap", ctypes.c_uint32), ("threads", ctypes.c_uint32),
                ("horizon_mode", ctypes.c_uint32), ("horizon_max_tasks", ctypes.c_uint32),
                ("staging", ctypes.c_uint32), ("pad2", ctypes.c_uint32),
                ("cap_commands", ctypes.c_uint64), ("cap_instructions", ctypes.c_uint64),
                ("cap_edges", ctypes.c_uint64), ("cap_state_words", ctypes.c_uint64),
                ("cap_unit", ctypes.c_uint64), ("cap_scratch", ctypes.c_uint64),
                ("arena", ctypes.c_void_p), ("arena_bytes", ctypes.c_uint64),
                ("stream", ctypes.c_void_p)]


class Stats(ctypes.Structure):
    _fields_ = [("n_instructions", ctypes.c_uint64), ("n_bindings", ctypes.c_uint64),
                ("n_edges", ctypes.c_uint64), ("per_kind", ctypes.c_uint64 * 8),
                ("per_dep", ctypes.c_uint64 * 5), ("resizes", ctypes.c_uint64),
                ("warnings", ctypes.c_uint64), ("tasks_submitted", ctypes.c_uint64),
                ("tasks_rejected", ctypes.c_uint64), ("digest_instructions", ctypes.c_uint64),
                ("digest_bindings", ctypes.c_uint64), ("digest_edges", ctypes.c_uint64),
                ("commands_analysed", ctypes.c_uint64), ("launches", ctypes.c_uint64),
                ("state_words_used", ctypes.c_uint64), ("reader_blocks_used", ctypes.c_uint64),
                ("capacity_exceeded", ctypes.c_uint64),
                ("phase_us", ctypes.c_double * 16), ("phase_count", ctypes.c_uint64 * 16)]


class OooParams(ctypes.Structure):
    _fields_ = [("devices", ctypes.c_uint32), ("lanes_per_device", ctypes.c_uint32),
                ("host_lanes", ctypes.c_uint32), ("window", ctypes.c_uint32), ("eager", ctypes.c_uint32),
                ("pad", ctypes.c_uint32), ("kernel_ns", ctypes.c_uint64), ("kernel_ns_per_kelem", ctypes.c_uint64),
                ("copy_ns", ctypes.c_uint64), ("copy_ns_per_kelem", ctypes.c_uint64),
                ("inter_node_ns", ctypes.c_uint64), ("alloc_ns", ctypes.c_uint64), ("free_ns", ctypes.c_uint64)]


class OooSummary(ctypes.Structure):
    _fields_ = [("makespan", ctypes.c_uint64), ("direct", ctypes.c_uint64), ("eager", ctypes.c_uint64),
                ("steps", ctypes.c_uint64), ("rounds", ctypes.c_uint64)]


OOO_SLOT_DTYPE = np.dtype([("lane", "<u4"), ("how", "<u4"), ("issue", "<u8"), ("start", "<u8"), ("end", "<u8")])


EXPORTS = [
    "ig_arena_bytes", "ig_context_create", "ig_context_destroy", "ig_buffer_create",
    "ig_buffer_destroy", "ig_submit_task", "ig_submit_tasks", "ig_epoch", "ig_shutdown",
    "ig_flush_window", "ig_batch_flush", "ig_sync", "ig_rewind", "ig_counts",
    "ig_fetch_instructions", "ig_fetch_bindings", "ig_fetch_edges", "ig_fetch_task_status",
    "ig_fetch_task_times", "ig_stats_get", "ig_status_str", "ig_batch_rewind", "ig_batch_progress",
    "ig_batch_graph_create", "ig_graph_launch", "ig_graph_destroy", "ig_batch_flush_window",
    "ig_batch_progress_noalloc", "ig_server_create", "ig_server_destroy", "ig_server_admit", "ig_server_session",
    "ig_server_submit", "ig_server_poll", "ig_server_detach", "ig_last_error",
    "ig_ooo_create", "ig_ooo_run", "ig_ooo_slots", "ig_ooo_fetch", "ig_ooo_destroy",
]

_libs: Dict[str, ctypes.CDLL] = {}


def lib(path: Optional[str] = None) -> ctypes.CDLL:
    """Load libig (the HIP build) -- or, for CPU tests only, another build of
    the same ABI named explicitly by `path`."""
    path = path or LIB_PATH
    if path in _libs:
        return _libs[path]
    if not os.path.exists(path):
        raise ImportError(f"libig not built: {path} is missing (run __graft_entry__.build())")
    L = ctypes.CDLL(path)
    P = ctypes.POINTER
    vp = ctypes.c_void_p
    L.ig_arena_bytes.argtypes = [P(ContextDesc), P(ctypes.c_uint64)]
    L.ig_context_create.argtypes = [P(ContextDesc), P(vp)]
    L.ig_context_destroy.argtypes = [vp]
    L.ig_buffer_create.argtypes = [vp, ctypes.c_uint32, P(ctypes.c_int64), ctypes.c_uint32, ctypes.c_uint32,
                                   P(ctypes.c_uint32)]
    L.ig_buffer_destroy.argtypes = [vp, ctypes.c_uint32]
    L.ig_submit_task.argtypes = [vp, P(TaskDesc), P(ctypes.c_uint64)]
    L.ig_submit_tasks.argtypes = [vp, P(TaskDesc), ctypes.c_size_t, P(ctypes.c_uint64)]
    for n in ("ig_epoch", "ig_shutdown", "ig_flush_window", "ig_sync", "ig_rewind"):
        getattr(L, n).argtypes = [vp]
    L.ig_batch_flush.argtypes = [P(vp), ctypes.c_size_t, vp]
    L.ig_batch_flush_window.argtypes = [P(vp), ctypes.c_size_t, vp, ctypes.c_uint32]
    L.ig_batch_rewind.argtypes = [P(vp), ctypes.c_size_t, vp]
    L.ig_batch_progress.argtypes = [P(vp), ctypes.c_size_t, vp, vp]
    L.ig_batch_progress_noalloc.argtypes = [P(vp), ctypes.c_size_t, vp, vp]
    L.ig_server_create.argtypes = [vp, P(vp)]
    L.ig_server_destroy.argtypes = [vp]
    L.ig_server_admit.argtypes = [vp, P(ContextDesc), P(ctypes.c_uint32)]
    L.ig_server_session.argtypes = [vp, ctypes.c_uint32, P(vp)]
    L.ig_server_submit.argtypes = [vp, ctypes.c_uint32, P(TaskDesc), P(ctypes.c_uint64)]
    L.ig_server_poll.argtypes = [vp, ctypes.c_uint32, vp, ctypes.c_size_t, P(ctypes.c_size_t)]
    L.ig_server_detach.argtypes = [vp, ctypes.c_uint32, P(vp)]
    L.ig_batch_graph_create.argtypes = [P(vp), ctypes.c_size_t, vp, P(vp)]
    L.ig_graph_launch.argtypes = [vp, vp]
    L.ig_graph_destroy.argtypes = [vp]
    L.ig_ooo_create.argtypes = [P(vp), ctypes.c_size_t, P(OooParams), P(vp)]
    L.ig_ooo_run.argtypes = [vp, vp]
    L.ig_ooo_slots.argtypes = [vp, ctypes.c_size_t, P(vp), P(ctypes.c_uint64)]
    L.ig_ooo_fetch.argtypes = [vp, ctypes.c_size_t, vp, ctypes.c_size_t, P(ctypes.c_size_t), P(OooSummary)]
    L.ig_ooo_destroy.argtypes = [vp]
    L.ig_counts.argtypes = [vp] + [P(ctypes.c_uint64)] * 4
    for n in ("ig_fetch_instructions", "ig_fetch_bindings", "ig_fetch_edges", "ig_fetch_task_status"):
        getattr(L, n).argtypes = [vp, vp, ctypes.c_size_t, P(ctypes.c_size_t)]
    L.ig_fetch_task_times.argtypes = [vp, P(ctypes.c_double), ctypes.c_size_t, P(ctypes.c_size_t)]
    L.ig_stats_get.argtypes = [vp, P(Stats)]
    L.ig_status_str.argtypes = [ctypes.c_int32]
    L.ig_last_error.argtypes = []
    L.ig_last_error.restype = ctypes.c_char_p
    L.ig_status_str.restype = ctypes.c_char_p
    for n in EXPORTS:
        if n != "ig_status_str":
            getattr(L, n).restype = ctypes.c_int32
    _libs[path] = L
    return L


def _box(lo, hi) -> Box:
    b = Box()
    for d in range(3):
        b.min[d] = int(lo[d])
        b.max[d] = int(hi[d])
    return b


def task_desc(task) -> TaskDesc:
    td = TaskDesc()
    td.dims = task.dims
    td.n_access = len(task.accesses)
    td.box = _box(task.lo, task.hi)
    for j, a in enumerate(task.accesses):
        ad = td.access[j]
        ad.buffer = a.buffer
        ad.mode = a.mode
        ad.mapper = a.mapper
        ad.slice_dim = a.slice_dim
        for d in range(3):
            ad.radius[d] = a.radius[d]
        ad.fixed = _box(a.fixed_lo, a.fixed_hi)
    return td


def project_counts(stream) -> Tuple[int, int]:
    """A rough projection of a stream's instruction and edge counts, used only
    to size device capacities (never for results).  It follows each buffer's
    coherence state coarsely: an all-like read (all, fixed, slice along the
    split dimension) of a buffer written since its last all-like read copies
    every producer chunk's part into every other device; a neighborhood read
    copies a few halo boxes per device; kernels depend on what they read and
    writers on earlier readers.  Resizes are counted per task without
    lookahead and for fixed (possibly growing) regions."""
    C = stream.chunks
    T = stream.nodes * stream.devices
    K = max(1, C // T)
    instr, edges = 1, 0
    bufs = []
    since_h = 0
    for c in stream.cmds:
        if c[0] == "buffer":
            bufs.append(dict(dirty_all=True, dirty_halo=True, host=c[4] == 1, on_dev=False, rd_all=False))
            continue
        if c[0] != "task":
            instr += 2 * T * max(1, len(bufs))
            edges += 4 * T * max(1, len(bufs)) + C
            continue
        t = c[1]
        instr += C
        edges += C * (len(t.accesses) + 1)
        for a in t.accesses:
            b = bufs[a.buffer]
            if not b["on_dev"]:
                instr += 2 * T
                edges += 4 * T
                b["on_dev"] = True
            if a.mode & 1:
                allish = a.mapper in (2, 4) or (a.mapper == 3 and a.slice_dim == 0)
                if allish:
                    cp = T * (C - K) + T if b["dirty_all"] else 0
                    edges += 3 * cp + (C * (C - K) if cp else C * T)
                    b["dirty_all"] = b["dirty_halo"] = False
                    b["rd_all"] = True
                elif a.mapper == 1:
                    cp = 3 * T if b["dirty_halo"] else 0
                    edges += 3 * cp + 3 * C
                    b["dirty_halo"] = False
                else:
                    cp = T if b["host"] else 0
                    edges += 3 * cp + C
                b["host"] = False
                instr += cp
            if a.mode & 2:
                if b["rd_all"]:
                    edges += 2 * C * T
                b["dirty_all"] = b["dirty_halo"] = True
                b["rd_all"] = b["host"] = False
            if not stream.lookahead or a.mapper == 4:
                instr += 4 * T
                edges += 8 * T + 2 * C * stream.horizon_step
        since_h += 1
        if since_h == stream.horizon_step:
            since_h = 0
            instr += 1
            edges += C + T
    return instr, edges


def estimate_caps(stream, margin: float = 2.0, floor: int = 4096) -> Dict[str, int]:
    """Output capacities for a stream: `margin` times the projected counts
    plus a floor.  A stream that still overflows reports IG_E_CAPACITY and
    can be re-run with larger capacities (run_stream does so)."""
    i, e = project_counts(stream)
    instr = min(int(margin * i) + floor, 0xFFFF0000)
    return dict(cap_commands=len(stream.cmds) + 8, cap_instructions=instr,
                cap_edges=int(margin * e) + 4 * floor)


def context_desc(L, device, stream=None, **kw):
    """A context descriptor; on "cuda" with its arena as a torch tensor and
    torch's (or the given) stream.  Returns (desc, arena, stream)."""
    d = ContextDesc()
    d.nodes, d.devices_per_node, d.chunks = kw["nodes"], kw["devices"], kw.get("chunks", 0)
    d.horizon_step, d.lookahead = kw.get("horizon_step", 0), kw.get("lookahead", 1)
    d.flush_horizons, d.queue_cap = kw.get("flush_horizons", 0), kw.get("queue_cap", 0)
    d.threads = kw.get("threads", 0)
    d.horizon_mode, d.horizon_max_tasks = kw.get("horizon_mode", 0), kw.get("horizon_max_tasks", 0)
    d.staging = kw.get("staging", 0)
    d.cap_commands, d.cap_instructions = kw.get("cap_commands", 0), kw.get("cap_instructions", 0)
    d.cap_edges, d.cap_state_words = kw.get("cap_edges", 0), kw.get("cap_state_words", 0)
    d.cap_unit, d.cap_scratch = kw.get("cap_unit", 0), kw.get("cap_scratch", 0)
    arena, s = None, None
    if device == "cuda":
        import torch
        nbytes = ctypes.c_uint64()
        st = L.ig_arena_bytes(ctypes.byref(d), ctypes.byref(nbytes))
        if st != 0:
            raise IgError("ig_arena_bytes", st)
        arena = torch.empty(int(nbytes.value), dtype=torch.uint8, device="cuda")
        d.arena = arena.data_ptr()
        d.arena_bytes = nbytes.value
        s = stream if stream is not None else torch.cuda.current_stream()
        d.stream = s.cuda_stream
    return d, arena, s


class Context:
    """One stream analysed by libig.

    device: "cuda" (default when torch sees a GPU) allocates the arena as a
    torch tensor and uses torch's current stream; "host" lets the library
    allocate (only meaningful for the CPU test build)."""

    def __init__(self, nodes, devices, chunks=0, horizon_step=0, lookahead=1, flush_horizons=0,
                 queue_cap=0, threads=0, lib_path=None, device=None, cap_commands=0,
                 cap_instructions=0, cap_edges=0, cap_state_words=0, cap_unit=0, cap_scratch=0, stream=None,
                 horizon_mode=0, horizon_max_tasks=0, staging=0):
        self.L = lib(lib_path)
        if device is None:
            device = "cuda" if lib_path is None else "host"
        self.device = device
        d, self.arena, self.torch_stream = context_desc(
            self.L, device, stream, nodes=nodes, devices=devices, chunks=chunks, horizon_step=horizon_step,
            lookahead=lookahead, flush_horizons=flush_horizons, queue_cap=queue_cap, threads=threads,
            horizon_mode=horizon_mode, horizon_max_tasks=horizon_max_tasks, staging=staging,
            cap_commands=cap_commands, cap_instructions=cap_instructions, cap_edges=cap_edges,
            cap_state_words=cap_state_words, cap_unit=cap_unit, cap_scratch=cap_scratch)
        self.desc = d
        self.h = ctypes.c_void_p()
        st = self.L.ig_context_create(ctypes.byref(d), ctypes.byref(self.h))
        if st != 0:
            raise IgError("ig_context_create", st)

    @classmethod
    def wrap(cls, L, handle, desc, arena, device) -> "Context":
        """A Context object owning an existing context handle (a session
        detached from a server)."""
        c = cls.__new__(cls)
        c.L, c.h, c.desc, c.arena, c.device, c.torch_stream = L, handle, desc, arena, device, None
        return c

    # --- recording ---------------------------------------------------------
    def buffer_create(self, dims, extent, elem_size, init) -> int:
        ext = (ctypes.c_int64 * 3)(*extent)
        out = ctypes.c_uint32()
        st = self.L.ig_buffer_create(self.h, dims, ext, elem_size, init, ctypes.byref(out))
        if st != 0:
            raise IgError("ig_buffer_create", st)
        return out.value

    def submit_desc(self, td: "TaskDesc") -> None:
        """Record a task from a descriptor built beforehand (task_desc)."""
        st = self.L.ig_submit_task(self.h, ctypes.byref(td), None)
        if st != 0:
            raise IgError("ig_submit_task", st)

    def record_command(self, c, td: Optional["TaskDesc"] = None) -> None:
        """Record one stream command (td: a prebuilt descriptor of a task)."""
        if c[0] == "task":
            if td is not None:
                self.submit_desc(td)
            else:
                self.submit(c[1])
        elif c[0] == "buffer":
            self.buffer_create(c[1], c[2], c[3], c[4])
        elif c[0] == "epoch":
            self.epoch()
        elif c[0] == "destroy":
            self.buffer_destroy(c[1])
        elif c[0] == "shutdown":
            self.shutdown()
        else:
            raise ValueError(c[0])

    def submit(self, task) -> int:
        td = task_desc(task)
        out = ctypes.c_uint64()
        st = self.L.ig_submit_task(self.h, ctypes.byref(td), ctypes.byref(out))
        if st != 0:
            raise IgError("ig_submit_task", st)
        return out.value

    def buffer_destroy(self, b):
        st = self.L.ig_buffer_destroy(self.h, b)
        if st != 0:
            raise IgError("ig_buffer_destroy", st)

    def epoch(self):
        st = self.L.ig_epoch(self.h)
        if st != 0:
            raise IgError("ig_epoch", st)

    def shutdown(self):
        st = self.L.ig_shutdown(self.h)
        if st != 0:
            raise IgError("ig_shutdown", st)

    def record(self, stream) -> None:
        for c in stream.cmds:
            if c[0] == "buffer":
                self.buffer_create(c[1], c[2], c[3], c[4])
            elif c[0] == "task":
                self.submit(c[1])
            elif c[0] == "epoch":
                self.epoch()
            elif c[0] == "destroy":
                self.buffer_destroy(c[1])
            elif c[0] == "shutdown":
                self.shutdown()
            else:
                raise ValueError(c[0])

    # --- analysis ----------------------------------------------------------
    def flush(self):
        st = self.L.ig_flush_window(self.h)
        if st != 0:
            raise IgError("ig_flush_window", st)

    def sync(self) -> int:
        return int(self.L.ig_sync(self.h))

    def rewind(self):
        st = self.L.ig_rewind(self.h)
        if st != 0:
            raise IgError("ig_rewind", st)

    def counts(self):
        v = [ctypes.c_uint64() for _ in range(4)]
        st = self.L.ig_counts(self.h, *[ctypes.byref(x) for x in v])
        if st != 0:
            raise IgError("ig_counts", st)
        return tuple(x.value for x in v)

    def _fetch(self, fn, dtype, n):
        arr = np.zeros(n, dtype=dtype)
        got = ctypes.c_size_t()
        st = fn(self.h, arr.ctypes.data_as(ctypes.c_void_p), n, ctypes.byref(got))
        if st != 0:
            raise IgError("fetch", st)
        return arr[: got.value]

    def fetch_all(self) -> Dict[str, np.ndarray]:
        ni, nb, ne, nt = self.counts()
        return dict(
            instructions=self._fetch(self.L.ig_fetch_instructions, INSTR_DTYPE, ni),
            bindings=self._fetch(self.L.ig_fetch_bindings, BIND_DTYPE, nb),
            edges=self._fetch(self.L.ig_fetch_edges, EDGE_DTYPE, ne),
            status=self._fetch(self.L.ig_fetch_task_status, np.dtype("<i4"), nt),
        )

    def task_times_ns(self) -> np.ndarray:
        """(n_tasks, 4) ns per task: intake start, intake end (compiled at
        once or queued), compilation start, records complete."""
        nt = self.counts()[3]
        arr = np.zeros((nt, 4), dtype=np.float64)
        got = ctypes.c_size_t()
        st = self.L.ig_fetch_task_times(self.h, arr.ctypes.data_as(ctypes.POINTER(ctypes.c_double)), nt,
                                        ctypes.byref(got))
        if st != 0:
            raise IgError("ig_fetch_task_times", st)
        return arr[: got.value]

    def stats(self) -> Dict[str, object]:
        s = Stats()
        st = self.L.ig_stats_get(self.h, ctypes.byref(s))
        if st != 0:
            raise IgError("ig_stats_get", st)
        out = {k: getattr(s, k) for k, _ in Stats._fields_}
        out["per_kind"] = list(s.per_kind)
        out["per_dep"] = list(s.per_dep)
        out["phase_us"] = list(s.phase_us)
        out["phase_count"] = list(s.phase_count)
        return out

    def close(self):
        if self.h:
            self.L.ig_context_destroy(self.h)
            self.h = ctypes.c_void_p()
        self.arena = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def make_context(stream, lib_path=None, device=None, threads=0, **caps) -> Context:
    kw = stream.desc()
    need = ("cap_commands", "cap_instructions", "cap_edges")
    est = {} if all(k in caps for k in need) else estimate_caps(stream)
    est.update(caps)
    return Context(lib_path=lib_path, device=device, threads=threads, **kw, **est)


def run_stream(stream, lib_path=None, device=None, threads=0, fetch=True, **caps) -> Dict[str, object]:
    """Record, analyse and (optionally) fetch one stream.  With estimated
    capacities, a capacity overflow is retried with larger ones (the output
    does not depend on them); explicit capacities are used as given."""
    margin = 2.0
    for attempt in range(4):
        kw = dict(caps) if caps else estimate_caps(stream, margin)
        ctx = make_context(stream, lib_path=lib_path, device=device, threads=threads, **kw)
        ctx.record(stream)
        t0 = time.perf_counter()
        ctx.flush()
        st = ctx.sync()
        elapsed = time.perf_counter() - t0
        if st == IG_E_CAPACITY and not caps and attempt < 3:
            ctx.close()
            margin *= 3
            continue
        if st != 0:
            ctx.close()
            raise IgError("analysis", st)
        out: Dict[str, object] = {"seconds": elapsed, "stats": ctx.stats()}
        if fetch:
            out.update(ctx.fetch_all())
        ctx.close()
        return out
    raise AssertionError("unreachable")


class Progress(ctypes.Structure):
    _fields_ = [("tasks_done", ctypes.c_uint64), ("tasks_seen", ctypes.c_uint64),
                ("error", ctypes.c_int32), ("finished", ctypes.c_uint32),
                ("capacity_exceeded", ctypes.c_uint32), ("commands_done", ctypes.c_uint32)]


def _ctx_array(contexts):
    return (ctypes.c_void_p * len(contexts))(*[c.h for c in contexts])


def _stream_ptr(stream):
    return None if stream is None else stream.cuda_stream


def batch_rewind(contexts: Sequence[Context], stream=None) -> None:
    st = contexts[0].L.ig_batch_rewind(_ctx_array(contexts), len(contexts), _stream_ptr(stream))
    if st != 0:
        raise IgError("ig_batch_rewind", st)


def batch_progress(contexts: Sequence[Context], stream=None, noalloc: bool = False) -> np.ndarray:
    """(n, 6) int64: tasks_done, tasks_seen, error, finished,
    capacity_exceeded, commands_done per context.  noalloc: use
    ig_batch_progress_noalloc (fixed device scratch, at most 4096 contexts)."""
    out = (Progress * len(contexts))()
    name = "ig_batch_progress_noalloc" if noalloc else "ig_batch_progress"
    st = getattr(contexts[0].L, name)(_ctx_array(contexts), len(contexts), _stream_ptr(stream),
                                      ctypes.cast(out, ctypes.c_void_p))
    if st != 0:
        raise IgError(name, st)
    return np.array([[p.tasks_done, p.tasks_seen, p.error, p.finished, p.capacity_exceeded, p.commands_done]
                     for p in out], dtype=np.int64)


class BatchGraph:
    """A captured re-analysis of many contexts (reset + one batched launch)."""

    def __init__(self, contexts: Sequence[Context], stream=None):
        self.L = contexts[0].L
        self.contexts = list(contexts)
        self.h = ctypes.c_void_p()
        st = self.L.ig_batch_graph_create(_ctx_array(contexts), len(contexts), _stream_ptr(stream),
                                          ctypes.byref(self.h))
        if st != 0:
            raise IgError("ig_batch_graph_create", st)

    def launch(self, stream=None) -> None:
        st = self.L.ig_graph_launch(self.h, _stream_ptr(stream))
        if st != 0:
            raise IgError("ig_graph_launch", st)

    def close(self) -> None:
        if self.h:
            self.L.ig_graph_destroy(self.h)
            self.h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def batch_flush(contexts: Sequence[Context], stream=None, window: int = 0) -> None:
    """One launch over many contexts; window > 0 analyses at most that many
    further commands per context."""
    st = contexts[0].L.ig_batch_flush_window(_ctx_array(contexts), len(contexts), _stream_ptr(stream), window)
    if st != 0:
        raise IgError("ig_batch_flush_window", st)


class ServerDesc(ctypes.Structure):
    _fields_ = [("slots", ctypes.c_uint32), ("threads", ctypes.c_uint32), ("window", ctypes.c_uint32),
                ("max_inflight", ctypes.c_uint32), ("arena_budget", ctypes.c_uint64),
                ("stage_bytes", ctypes.c_uint64), ("stream", ctypes.c_void_p)]


class SessionProgress(ctypes.Structure):
    _fields_ = [("slot", ctypes.c_uint32), ("in_flight", ctypes.c_uint32), ("tasks_done", ctypes.c_uint64),
                ("tasks_seen", ctypes.c_uint64), ("error", ctypes.c_int32), ("finished", ctypes.c_uint32),
                ("commands_done", ctypes.c_uint32), ("commands_recorded", ctypes.c_uint32)]


assert ctypes.sizeof(SessionProgress) == 40


class Server:
    """ig_server_*: sessions admitted into slots, analysed in batched
    launches queued asynchronously (continuous batching)."""

    def __init__(self, slots: int, threads: int = 256, window: int = 0, max_inflight: int = 2,
                 arena_budget: int = 0, stage_bytes: int = 0, lib_path: Optional[str] = None, stream=None):
        self.L = lib(lib_path)
        self.device = "cuda" if lib_path is None else "host"
        d = ServerDesc(slots, threads, window, max_inflight, arena_budget, stage_bytes, None)
        self.stream = None
        if self.device == "cuda":
            import torch
            self.stream = stream if stream is not None else torch.cuda.current_stream()
            d.stream = self.stream.cuda_stream
        self.slots = slots
        self.h = ctypes.c_void_p()
        st = self.L.ig_server_create(ctypes.byref(d), ctypes.byref(self.h))
        if st != 0:
            raise IgError("ig_server_create", st)
        self.sessions: Dict[int, tuple] = {}  # slot -> (desc, arena)
        self._out = (SessionProgress * slots)()

    def admit(self, stream_obj, threads: int = 0, **caps) -> Optional[int]:
        """Admit a session for a Stream (its cluster shape and lookahead
        settings; no command is recorded).  None when the server is busy."""
        kw = stream_obj.desc()
        kw.update(caps)
        kw["threads"] = threads
        d, arena, _ = context_desc(self.L, self.device, self.stream, **kw)
        slot = ctypes.c_uint32()
        st = self.L.ig_server_admit(self.h, ctypes.byref(d), ctypes.byref(slot))
        if st == IG_E_BUSY:
            return None
        if st != 0:
            raise IgError("ig_server_admit", st)
        self.sessions[slot.value] = (d, arena)
        return slot.value

    def context(self, slot: int) -> "Context":
        """A non-owning view of the session's context, for recording."""
        h = ctypes.c_void_p()
        st = self.L.ig_server_session(self.h, slot, ctypes.byref(h))
        if st != 0:
            raise IgError("ig_server_session", st)
        d, arena = self.sessions[slot]
        c = Context.wrap(self.L, h, d, arena, self.device)
        c.close = lambda: None  # the server owns it
        return c

    def submit(self, slot: int, td: "TaskDesc") -> None:
        st = self.L.ig_server_submit(self.h, slot, ctypes.byref(td), None)
        if st != 0:
            raise IgError("ig_server_submit", st)

    def poll(self, wait: bool = False) -> List[SessionProgress]:
        n = ctypes.c_size_t()
        st = self.L.ig_server_poll(self.h, 1 if wait else 0, ctypes.cast(self._out, ctypes.c_void_p), self.slots,
                                   ctypes.byref(n))
        if st != 0:
            raise IgError("ig_server_poll", st)
        return [self._out[i] for i in range(n.value)]

    def detach(self, slot: int) -> Optional["Context"]:
        """The session's context, owned by the caller from now on (None
        while a queued launch covers it)."""
        h = ctypes.c_void_p()
        st = self.L.ig_server_detach(self.h, slot, ctypes.byref(h))
        if st == IG_E_BUSY:
            return None
        if st != 0:
            raise IgError("ig_server_detach", st)
        d, arena = self.sessions.pop(slot)
        return Context.wrap(self.L, h, d, arena, self.device)

    def close(self) -> None:
        if self.h:
            self.L.ig_server_destroy(self.h)
            self.h = ctypes.c_void_p()
        self.sessions = {}

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def ooo_params(devices, lanes_per_device=2, host_lanes=2, window=1024, eager=1, kernel_ns=4000,
               kernel_ns_per_kelem=64, copy_ns=2000, copy_ns_per_kelem=32, inter_node_ns=8000, alloc_ns=20000,
               free_ns=5000) -> OooParams:
    """Engine parameters (ig_ooo_params); the defaults are the cost model
    the benchmark uses: 4 us per kernel plus 64 ns per 1024 index points,
    2 us per copy plus 32 ns per 1024 elements (+8 us between nodes), 20 us
    per allocation, 5 us per free."""
    return OooParams(devices, lanes_per_device, host_lanes, window, eager, 0, kernel_ns, kernel_ns_per_kelem,
                     copy_ns, copy_ns_per_kelem, inter_node_ns, alloc_ns, free_ns)


class OooSimulation:
    """The out-of-order engine simulated over the graphs of several contexts
    (ig_ooo_*): one workgroup per graph, one launch for all."""

    def __init__(self, contexts: Sequence[Context], params: OooParams):
        self.L = contexts[0].L
        self.n = len(contexts)
        self.h = ctypes.c_void_p()
        st = self.L.ig_ooo_create(_ctx_array(contexts), len(contexts), ctypes.byref(params), ctypes.byref(self.h))
        if st != 0:
            raise IgError("ig_ooo_create", st)

    def run(self, stream=None) -> None:
        st = self.L.ig_ooo_run(self.h, _stream_ptr(stream))
        if st != 0:
            raise IgError("ig_ooo_run", st)

    def device_slots(self, i: int):
        """(device address, count) of graph i's results."""
        ptr, n = ctypes.c_void_p(), ctypes.c_uint64()
        st = self.L.ig_ooo_slots(self.h, i, ctypes.byref(ptr), ctypes.byref(n))
        if st != 0:
            raise IgError("ig_ooo_slots", st)
        return ptr.value, n.value

    def summary(self, i: int) -> Dict[str, int]:
        """Graph i's summary alone (waits for the last run)."""
        summ = OooSummary()
        got = ctypes.c_size_t()
        st = self.L.ig_ooo_fetch(self.h, i, None, 0, ctypes.byref(got), ctypes.byref(summ))
        if st != 0:
            raise IgError(f"ig_ooo_fetch (graph {i})", st)
        return {k: getattr(summ, k) for k, _ in OooSummary._fields_}

    def fetch(self, i: int):
        """(slots as OOO_SLOT_DTYPE, summary dict) of graph i."""
        _, n = self.device_slots(i)
        out = np.zeros(n, dtype=OOO_SLOT_DTYPE)
        got = ctypes.c_size_t()
        summ = OooSummary()
        st = self.L.ig_ooo_fetch(self.h, i, out.ctypes.data if n else None, n, ctypes.byref(got), ctypes.byref(summ))
        if st != 0:
            raise IgError(f"ig_ooo_fetch (graph {i})", st)
        return out, {k: getattr(summ, k) for k, _ in OooSummary._fields_}

    def close(self) -> None:
        if self.h:
            self.L.ig_ooo_destroy(self.h)
            self.h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
