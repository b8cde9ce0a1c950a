"""CPU oracle for instruction-graph generation -- TEST INFRASTRUCTURE ONLY.

A plain sequential C++17 implementation (ig_oracle.cpp) of the method of the
paper (Sec. 3 and Sec. 4.3/4.4), loaded through ctypes.  Only the test suite,
the smoke check and the CPU-baseline leg of the benchmark may import this
package; the product library never does.  It shares no code with the HIP
implementation: the record layouts are defined again here.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
import time
from typing import Dict, List

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "ig_oracle.cpp")
LIB_PATH = os.path.join(_HERE, "libig_oracle.so")

INSTR_DTYPE = np.dtype([
    ("id", "<u8"), ("kind", "u1"), ("flags", "u1"), ("mem", "<u2"), ("src_mem", "<u2"),
    ("pad0", "<u2"), ("task", "<u4"), ("chunk", "<u4"), ("buffer", "<u4"), ("pad1", "<u4"),
    ("alloc", "<u8"), ("src_alloc", "<u8"), ("min", "<i8", (3,)), ("max", "<i8", (3,)),
])
BIND_DTYPE = np.dtype([("instr", "<u8"), ("access", "<u4"), ("pad", "<u4"), ("alloc", "<u8")])
EDGE_DTYPE = np.dtype([("from", "<u8"), ("to", "<u8"), ("kinds", "<u4"), ("pad", "<u4")])
assert INSTR_DTYPE.itemsize == 96 and BIND_DTYPE.itemsize == 24 and EDGE_DTYPE.itemsize == 24

OK, W_UNINIT_READ, E_INVALID, E_OVERLAPPING_WRITE, E_CAPACITY = 0, 1, -1, -2, -3
ALLOC, COPY, FREE, KERNEL, HORIZON, EPOCH = 1, 2, 3, 4, 5, 6
F_RESIZE, F_INTER_NODE = 1, 2
DEP_TRUE, DEP_ANTI, DEP_OUTPUT, DEP_LIFETIME, DEP_SYNC = 1, 2, 4, 8, 16
NONE32, NONE16 = 0xFFFFFFFF, 0xFFFF


class Box(ctypes.Structure):
    _fields_ = [("min", ctypes.c_int64 * 3), ("max", ctypes.c_int64 * 3)]


class AccessDesc(ctypes.Structure):
    _fields_ = [("buffer", ctypes.c_uint32), ("mode", ctypes.c_uint8), ("mapper", ctypes.c_uint8),
                ("slice_dim", ctypes.c_uint8), ("pad", ctypes.c_uint8),
                ("radius", ctypes.c_int64 * 3), ("fixed", Box)]


class TaskDesc(ctypes.Structure):
    _fields_ = [("dims", ctypes.c_uint32), ("n_access", ctypes.c_uint32), ("box", Box),
                ("access", AccessDesc * 8)]


class ContextDesc(ctypes.Structure):
    _fields_ = [("nodes", ctypes.c_uint32), ("devices_per_node", ctypes.c_uint32),
                ("chunks", ctypes.c_uint32), ("horizon_step", ctypes.c_uint32),
                ("lookahead", ctypes.c_uint32), ("flush_horizons", ctypes.c_uint32),
                ("queue_cap", ctypes.c_uint32), ("horizon_mode", ctypes.c_uint32),
                ("horizon_max_tasks", ctypes.c_uint32), ("staging", ctypes.c_uint32)]


class Stats(ctypes.Structure):
    _fields_ = [("n_instructions", ctypes.c_uint64), ("n_bindings", ctypes.c_uint64),
                ("n_edges", ctypes.c_uint64), ("per_kind", ctypes.c_uint64 * 8),
                ("per_dep", ctypes.c_uint64 * 5), ("resizes", ctypes.c_uint64),
                ("warnings", ctypes.c_uint64), ("tasks_submitted", ctypes.c_uint64),
                ("tasks_rejected", ctypes.c_uint64), ("digest_instructions", ctypes.c_uint64),
                ("digest_bindings", ctypes.c_uint64), ("digest_edges", ctypes.c_uint64),
                ("u_w", ctypes.c_uint64), ("u_r", ctypes.c_uint64), ("u_b", ctypes.c_uint64),
                ("map_boxes", ctypes.c_uint64)]


# command trace (igo_event): every call reaching the command stream, in order
EV_BUFFER, EV_TASK, EV_REJECTED, EV_HORIZON, EV_EPOCH, EV_DESTROY, EV_SHUTDOWN = 1, 2, 3, 4, 5, 6, 7
EVENT_DTYPE = np.dtype([("kind", "<u4"), ("arg", "<u4"), ("allocating", "<u4"), ("compiled_at", "<u4"),
                        ("n_instr", "<u8")])
assert EVENT_DTYPE.itemsize == 24


def build(force: bool = False) -> str:
    """Compile the oracle with g++ (plain -O2, no tuning)."""
    if force or not os.path.exists(LIB_PATH) or os.path.getmtime(LIB_PATH) < os.path.getmtime(_SRC):
        tmp = LIB_PATH + ".tmp%d" % os.getpid()
        subprocess.check_call(["g++", "-O2", "-std=c++17", "-shared", "-fPIC", "-o", tmp, _SRC])
        os.replace(tmp, LIB_PATH)
    return LIB_PATH


_lib = None


def lib() -> ctypes.CDLL:
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            build()
        L = ctypes.CDLL(LIB_PATH)
        P = ctypes.POINTER
        c_ctx = ctypes.c_void_p
        L.igo_context_create.argtypes = [P(ContextDesc), P(c_ctx)]
        L.igo_context_destroy.argtypes = [c_ctx]
        L.igo_buffer_create.argtypes = [c_ctx, ctypes.c_uint32, P(ctypes.c_int64), ctypes.c_uint32,
                                        ctypes.c_uint32, P(ctypes.c_uint32)]
        L.igo_buffer_destroy.argtypes = [c_ctx, ctypes.c_uint32]
        L.igo_submit_task.argtypes = [c_ctx, P(TaskDesc), P(ctypes.c_uint64)]
        L.igo_epoch.argtypes = [c_ctx]
        L.igo_shutdown.argtypes = [c_ctx]
        L.igo_flush_window.argtypes = [c_ctx]
        L.igo_counts.argtypes = [c_ctx] + [P(ctypes.c_uint64)] * 4
        for name in ("igo_fetch_instructions", "igo_fetch_bindings", "igo_fetch_edges",
                     "igo_fetch_task_status"):
            getattr(L, name).argtypes = [c_ctx, ctypes.c_void_p, ctypes.c_size_t, P(ctypes.c_size_t)]
        L.igo_stats_get.argtypes = [c_ctx, P(Stats)]
        L.igo_fetch_events.argtypes = [c_ctx, ctypes.c_void_p, ctypes.c_size_t, P(ctypes.c_size_t)]
        L.igo_fetch_events.restype = ctypes.c_int32
        L.igo_event_count.argtypes = [c_ctx]
        L.igo_event_count.restype = ctypes.c_size_t
        L.igo_box_subtract.argtypes = [P(Box), P(Box), P(Box)]
        L.igo_box_subtract.restype = ctypes.c_size_t
        L.igo_box_merges.argtypes = [P(Box), P(Box)]
        L.igo_canonical.argtypes = [P(Box), ctypes.c_size_t, P(Box), ctypes.c_size_t]
        L.igo_canonical.restype = ctypes.c_size_t
        L.igo_merge_fixpoint.argtypes = [P(Box), ctypes.c_size_t, P(Box), ctypes.c_size_t]
        L.igo_merge_fixpoint.restype = ctypes.c_size_t
        L.igo_split.argtypes = [ctypes.c_uint32, ctypes.c_uint32, ctypes.c_uint32, P(Box), P(Box)]
        L.igo_map.argtypes = [P(AccessDesc), ctypes.c_uint32, P(Box), ctypes.c_uint32,
                              P(ctypes.c_int64), P(Box)]
        L.igo_digest.argtypes = [P(ctypes.c_uint64), ctypes.c_size_t, ctypes.c_size_t]
        L.igo_digest.restype = ctypes.c_uint64
        for name in ("igo_context_create", "igo_context_destroy", "igo_buffer_create",
                     "igo_buffer_destroy", "igo_submit_task", "igo_epoch", "igo_shutdown",
                     "igo_flush_window", "igo_counts", "igo_fetch_instructions",
                     "igo_fetch_bindings", "igo_fetch_edges", "igo_fetch_task_status",
                     "igo_stats_get", "igo_box_merges", "igo_split", "igo_map"):
            getattr(L, name).restype = ctypes.c_int32
        _lib = L
    return _lib


# ---------------------------------------------------------------------------
# helpers shared by the tests
# ---------------------------------------------------------------------------

def make_box(lo, hi) -> Box:
    b = Box()
    for d in range(3):
        b.min[d] = int(lo[d])
        b.max[d] = int(hi[d])
    return b


def box_tuple(b: Box):
    return (tuple(b.min), tuple(b.max))


def fill_task(td: TaskDesc, task) -> None:
    td.dims = task.dims
    td.n_access = len(task.accesses)
    td.box = make_box(task.lo, task.hi)
    for j, a in enumerate(task.accesses):
        ad = td.access[j]
        ad.buffer = a.buffer
        ad.mode = a.mode
        ad.mapper = a.mapper
        ad.slice_dim = a.slice_dim
        for d in range(3):
            ad.radius[d] = a.radius[d]
        ad.fixed = make_box(a.fixed_lo, a.fixed_hi)


class OracleContext:
    """One stream analysed by the oracle."""

    def __init__(self, nodes, devices, chunks=0, horizon_step=0, lookahead=1,
                 flush_horizons=0, queue_cap=0, horizon_mode=0, horizon_max_tasks=0, staging=0):
        self.L = lib()
        d = ContextDesc(nodes, devices, chunks, horizon_step, lookahead, flush_horizons, queue_cap, horizon_mode,
                        horizon_max_tasks, staging)
        self.h = ctypes.c_void_p()
        st = self.L.igo_context_create(ctypes.byref(d), ctypes.byref(self.h))
        if st != 0:
            raise ValueError(f"igo_context_create failed: {st}")

    def close(self):
        if self.h:
            self.L.igo_context_destroy(self.h)
            self.h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def buffer_create(self, dims, extent, elem_size, init):
        ext = (ctypes.c_int64 * 3)(*extent)
        out = ctypes.c_uint32()
        st = self.L.igo_buffer_create(self.h, dims, ext, elem_size, init, ctypes.byref(out))
        return st, out.value

    def submit(self, task):
        td = TaskDesc()
        fill_task(td, task)
        out = ctypes.c_uint64()
        st = self.L.igo_submit_task(self.h, ctypes.byref(td), ctypes.byref(out))
        return st

    def buffer_destroy(self, b):
        return self.L.igo_buffer_destroy(self.h, b)

    def epoch(self):
        return self.L.igo_epoch(self.h)

    def shutdown(self):
        return self.L.igo_shutdown(self.h)

    def counts(self):
        v = [ctypes.c_uint64() for _ in range(4)]
        self.L.igo_counts(self.h, *[ctypes.byref(x) for x in v])
        return tuple(x.value for x in v)

    def _fetch(self, fn, dtype, n):
        arr = np.zeros(n, dtype=dtype)
        got = ctypes.c_size_t()
        fn(self.h, arr.ctypes.data_as(ctypes.c_void_p), n, ctypes.byref(got))
        return arr[: got.value]

    def fetch_all(self) -> Dict[str, np.ndarray]:
        ni, nb, ne, nt = self.counts()
        return dict(
            instructions=self._fetch(self.L.igo_fetch_instructions, INSTR_DTYPE, ni),
            bindings=self._fetch(self.L.igo_fetch_bindings, BIND_DTYPE, nb),
            edges=self._fetch(self.L.igo_fetch_edges, EDGE_DTYPE, ne),
            status=self._fetch(self.L.igo_fetch_task_status, np.dtype("<i4"), nt),
        )

    def events(self) -> np.ndarray:
        return self._fetch(self.L.igo_fetch_events, EVENT_DTYPE, self.L.igo_event_count(self.h))

    def stats(self) -> Dict[str, object]:
        s = Stats()
        self.L.igo_stats_get(self.h, ctypes.byref(s))
        out = {k: getattr(s, k) for k, _ in Stats._fields_}
        out["per_kind"] = list(s.per_kind)
        out["per_dep"] = list(s.per_dep)
        return out


def run_stream(stream, fetch: bool = True) -> Dict[str, object]:
    """Replay one stream through the oracle; returns records, statuses,
    per-command return codes, statistics and the analysis time (s)."""
    ctx = OracleContext(**stream.desc())
    rcs: List[int] = []
    t0 = time.perf_counter()
    for c in stream.cmds:
        kind = c[0]
        if kind == "buffer":
            st, _ = ctx.buffer_create(c[1], c[2], c[3], c[4])
        elif kind == "task":
            st = ctx.submit(c[1])
        elif kind == "epoch":
            st = ctx.epoch()
        elif kind == "destroy":
            st = ctx.buffer_destroy(c[1])
        elif kind == "shutdown":
            st = ctx.shutdown()
        else:
            raise ValueError(kind)
        rcs.append(st)
    elapsed = time.perf_counter() - t0
    out: Dict[str, object] = {"rcs": rcs, "seconds": elapsed, "stats": ctx.stats()}
    if fetch:
        out.update(ctx.fetch_all())
        out["events"] = ctx.events()
    ctx.close()
    return out


# --- box-set primitives (exported for pinning) ------------------------------

def box_subtract(a, b):
    out = (Box * 6)()
    n = lib().igo_box_subtract(ctypes.byref(make_box(*a)), ctypes.byref(make_box(*b)), out)
    return [box_tuple(out[i]) for i in range(n)]


def box_merges(a, b) -> bool:
    return bool(lib().igo_box_merges(ctypes.byref(make_box(*a)), ctypes.byref(make_box(*b))))


def canonical(boxes):
    arr = (Box * max(1, len(boxes)))(*[make_box(*b) for b in boxes])
    cap = 4096
    out = (Box * cap)()
    n = lib().igo_canonical(arr, len(boxes), out, cap)
    assert n <= cap
    return [box_tuple(out[i]) for i in range(n)]


def merge_fixpoint(boxes):
    arr = (Box * max(1, len(boxes)))(*[make_box(*b) for b in boxes])
    cap = 4096
    out = (Box * cap)()
    n = lib().igo_merge_fixpoint(arr, len(boxes), out, cap)
    return [box_tuple(out[i]) for i in range(n)]


def split(nodes, devices, chunks, lo, hi):
    out = (Box * chunks)()
    st = lib().igo_split(nodes, devices, chunks, ctypes.byref(make_box(lo, hi)), out)
    assert st == 0
    return [box_tuple(out[i]) for i in range(chunks)]


def map_range(access, task_dims, chunk, buf_dims, extent):
    ad = AccessDesc()
    ad.buffer = access.buffer
    ad.mode = access.mode
    ad.mapper = access.mapper
    ad.slice_dim = access.slice_dim
    for d in range(3):
        ad.radius[d] = access.radius[d]
    ad.fixed = make_box(access.fixed_lo, access.fixed_hi)
    out = Box()
    ext = (ctypes.c_int64 * 3)(*extent)
    lib().igo_map(ctypes.byref(ad), task_dims, ctypes.byref(make_box(*chunk)), buf_dims, ext,
                  ctypes.byref(out))
    return box_tuple(out)


def digest_words(words: np.ndarray) -> int:
    """Digest of records given as an (n, w) uint64 array."""
    w = np.ascontiguousarray(words, dtype=np.uint64)
    n, k = (w.shape[0], w.shape[1]) if w.ndim == 2 else (0, 1)
    return int(lib().igo_digest(w.ctypes.data_as(ctypes.POINTER(ctypes.c_uint64)), n, k))


# --- the out-of-order engine of Sec. 4.1, simulated over a finished graph ---

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
OOO_ENGINE, OOO_DIRECT, OOO_EAGER = 0, 1, 2


def ooo_params(devices, lanes_per_device=2, host_lanes=2, window=1024, eager=1, kernel_ns=4000,
               kernel_ns_per_kelem=64, copy_ns=2000, copy_ns_per_kelem=32, inter_node_ns=8000, alloc_ns=20000,
               free_ns=5000) -> OooParams:
    return OooParams(devices, lanes_per_device, host_lanes, window, eager, 0, kernel_ns, kernel_ns_per_kelem,
                     copy_ns, copy_ns_per_kelem, inter_node_ns, alloc_ns, free_ns)


def ooo_simulate(instructions: np.ndarray, edges: np.ndarray, params: OooParams):
    """(slots, summary) of the engine over records in the layouts above."""
    L = lib()
    fn = L.igo_ooo_simulate
    fn.argtypes = [ctypes.c_void_p, ctypes.c_size_t, ctypes.c_void_p, ctypes.c_size_t, ctypes.POINTER(OooParams),
                   ctypes.c_void_p, ctypes.POINTER(OooSummary)]
    fn.restype = ctypes.c_int32
    ins = np.ascontiguousarray(instructions, dtype=INSTR_DTYPE)
    ed = np.ascontiguousarray(edges, dtype=EDGE_DTYPE)
    out = np.zeros(len(ins), dtype=OOO_SLOT_DTYPE)
    summ = OooSummary()
    st = fn(ins.ctypes.data, len(ins), ed.ctypes.data, len(ed), ctypes.byref(params), out.ctypes.data,
            ctypes.byref(summ))
    if st != 0:
        raise ValueError(f"igo_ooo_simulate failed: {st}")
    return out, {k: getattr(summ, k) for k, _ in OooSummary._fields_}
