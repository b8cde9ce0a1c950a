"""Brute-force, per-element checks of an emitted instruction graph.

These checks pin the oracle against what the paper fixes, without restating
its rules: they execute the emitted graph symbolically, element by element,
and test what any correct instruction graph must satisfy.

  * Sequential semantics (Sec. 2.3): every kernel reads, for every element of
    every read region, exactly the version the sequential task order
    prescribes (the last earlier task writing that element, or the host
    data).
  * Schedule independence (Sec. 3, the IDAG "models concurrency"): every
    pair of conflicting accesses to one element of one allocation (write
    after write, read after write, write after read, use after alloc, free
    after use) is ordered by a path in the graph; so every topological order
    computes the same values.
  * Coherence (Sec. 3.3): a coherence copy never moves data that is already
    up to date at its destination, never moves uninitialised data, reads it
    from the memory of its original producer, and within one copy every
    element has one original producer (producer split).
  * Allocation (Sec. 3.2): allocations on one memory and buffer never overlap,
    every accessor lies in the one allocation bound to it, allocations never
    shrink, every device allocation is freed exactly once, user memory M0 is
    never freed.
  * Horizons/epochs (Sec. 3.5): they depend on exactly the execution front;
    instruction ids are a topological order (Sec. 4.1).
  * Debug checks (Sec. 4.4): overlapping writes of different chunks are
    rejected; reads outside the initialised region warn.
  * Resizes (Sec. 3.2): the resize copies out of an old allocation move
    exactly its elements that are up to date on its memory, each once.

Two checks restate a rule element by element, as a second formulation next
to the oracle's box maps, because the paper fixes them only as principles:

  * Exact edges (the dependency legend of the IDAG figure, Sec. 3.6): every
    edge and every kind bit on it is justified by some element of some
    allocation (last writer, readers since the last write, allocation
    lifetime), and no justified edge is missing.
  * The command queue (Sec. 4.3), replayed from the oracle's command trace:
    the allocating predicate of every task and the moment every command is
    compiled.

The chunk split and the range mappers are evaluated here too (per element),
straight from their definitions.
"""
from __future__ import annotations

import itertools
import random
from typing import Dict, List, Tuple

import numpy as np

ALLOC, COPY, FREE, KERNEL, HORIZON, EPOCH = 1, 2, 3, 4, 5, 6
F_RESIZE, F_INTER_NODE = 1, 2
DEP_TRUE, DEP_ANTI, DEP_OUTPUT, DEP_LIFETIME, DEP_SYNC = 1, 2, 4, 8, 16
READ, WRITE = 1, 2
ONE_TO_ONE, NEIGHBORHOOD, ALL, SLICE, FIXED = 0, 1, 2, 3, 4
NONE32, NONE16 = 0xFFFFFFFF, 0xFFFF
V_HOST, V_UNINIT, V_GARBAGE = -1, -2, -3


def split_py(nodes, devices, chunks, lo, hi):
    """Nested floor split of dimension 0 (nodes, devices, sub-chunks)."""
    per = chunks // (nodes * devices)
    out = []
    n = hi[0] - lo[0]
    for i in range(nodes):
        a, b = lo[0] + (i * n) // nodes, lo[0] + ((i + 1) * n) // nodes
        for j in range(devices):
            s, e = a + (j * (b - a)) // devices, a + ((j + 1) * (b - a)) // devices
            for u in range(per):
                c0, c1 = s + (u * (e - s)) // per, s + ((u + 1) * (e - s)) // per
                out.append(((c0, lo[1], lo[2]), (c1, hi[1], hi[2])))
    return out


def map_py(acc, chunk, bdims, ext):
    lo, hi = [0, 0, 0], [1, 1, 1]
    for d in range(bdims):
        if acc.mapper == ONE_TO_ONE:
            lo[d], hi[d] = chunk[0][d], chunk[1][d]
        elif acc.mapper == NEIGHBORHOOD:
            lo[d], hi[d] = chunk[0][d] - acc.radius[d], chunk[1][d] + acc.radius[d]
        elif acc.mapper == ALL:
            lo[d], hi[d] = 0, ext[d]
        elif acc.mapper == SLICE:
            lo[d], hi[d] = (0, ext[d]) if d == acc.slice_dim else (chunk[0][d], chunk[1][d])
        else:
            lo[d], hi[d] = acc.fixed_lo[d], acc.fixed_hi[d]
        lo[d], hi[d] = max(lo[d], 0), min(hi[d], ext[d])
    return tuple(lo), tuple(hi)


def box_empty(b):
    return any(b[0][d] >= b[1][d] for d in range(3))


def box_points(b):
    if box_empty(b):
        return []
    return list(itertools.product(*[range(b[0][d], b[1][d]) for d in range(3)]))


def box_contains(outer, inner):
    if box_empty(inner):
        return True
    return all(outer[0][d] <= inner[0][d] and inner[1][d] <= outer[1][d] for d in range(3))


def box_intersects(a, b):
    return all(max(a[0][d], b[0][d]) < min(a[1][d], b[1][d]) for d in range(3))


def rec_box(r):
    return (tuple(int(x) for x in r["min"]), tuple(int(x) for x in r["max"]))


def points_merge(a, b) -> bool:
    """Brute force of the merge relation: overlap, or two points of the boxes
    are axis neighbours (so the boxes share part of a face)."""
    pa = set(box_points(a))
    pb = set(box_points(b))
    if pa & pb:
        return True
    for p in pa:
        for d in range(3):
            for s in (-1, 1):
                q = list(p)
                q[d] += s
                if tuple(q) in pb:
                    return True
    return False


def canonical_bruteforce(points: set, shape) -> List[tuple]:
    """Dim-0-major maximal slab decomposition of a point set on a dense grid,
    straight from the definition."""
    g = np.zeros(shape, dtype=bool)
    for p in points:
        g[p] = True
    out = []
    n0, n1, n2 = shape
    i = 0
    while i < n0:
        if not g[i].any():
            i += 1
            continue
        i2 = i + 1
        while i2 < n0 and np.array_equal(g[i2], g[i]):
            i2 += 1
        j = 0
        while j < n1:
            if not g[i, j].any():
                j += 1
                continue
            j2 = j + 1
            while j2 < n1 and np.array_equal(g[i, j2], g[i, j]):
                j2 += 1
            k = 0
            while k < n2:
                if not g[i, j, k]:
                    k += 1
                    continue
                k2 = k + 1
                while k2 < n2 and g[i, j, k2]:
                    k2 += 1
                out.append(((i, j, k), (i2, j2, k2)))
                k = k2
            j = j2
        i = i2
    return out


class Failure(AssertionError):
    pass


def _require(cond, msg):
    if not cond:
        raise Failure(msg)


def check_stream(stream, out, n_random_orders: int = 2, seed: int = 0) -> Dict[str, int]:
    """Run every brute-force check on one (small) stream and its output."""
    ins = out["instructions"]
    binds = out["bindings"]
    edges = out["edges"]
    status = list(int(x) for x in out["status"])
    n = len(ins)
    _require(n > 0 and int(ins[0]["kind"]) == EPOCH, "I0 must be the initial epoch")
    _require(all(int(ins[i]["id"]) == i for i in range(n)), "instruction ids are consecutive")
    # ---------------- edges: order, uniqueness, topological ----------------
    pairs = [(int(e["to"]), int(e["from"])) for e in edges]
    _require(pairs == sorted(pairs), "edges sorted by (to, from)")
    _require(len(set(pairs)) == len(pairs), "edges unique per (from, to)")
    _require(all(f < t for t, f in pairs), "every edge goes from a lower to a higher id")
    preds: List[List[Tuple[int, int]]] = [[] for _ in range(n)]
    succ_count = [0] * n
    for e in edges:
        preds[int(e["to"])].append((int(e["from"]), int(e["kinds"])))
        succ_count[int(e["from"])] += 1
    for x in range(1, n):
        _require(len(preds[x]) > 0, f"I{x} has no incoming edge")
    # reachability (ancestors as bitsets)
    anc = [0] * n
    for x in range(n):
        a = 0
        for f, _ in preds[x]:
            a |= anc[f] | (1 << f)
        anc[x] = a

    def ordered(a, b):
        return a == b or bool((anc[b] >> a) & 1)

    # ---------------- horizons and epochs depend on the front --------------
    for x in range(1, n):
        if int(ins[x]["kind"]) in (HORIZON, EPOCH):
            has_succ_before = set()
            for t, f in pairs:
                if t < x:
                    has_succ_before.add(f)
            front = {y for y in range(x) if y not in has_succ_before}
            got = {f for f, _ in preds[x]}
            _require(got == front, f"I{x}: sync edges {sorted(got)} != front {sorted(front)}")
            _require(all(k == DEP_SYNC for _, k in preds[x]), f"I{x}: front edges are SYNC")

    # ---------------- sequential reference (task level, per element) -------
    bufs = []          # per buffer: dims, ext, init
    versions = []      # per buffer: ndarray of versions
    last_mem = []      # per buffer: memory of the last writer (0: host)
    initialised = []   # per buffer: bool ndarray
    tasks = []         # task id -> (Task, status, expected versions per buffer before it)
    for c in stream.cmds:
        if c[0] == "buffer":
            dims, ext, _, init = c[1], c[2], c[3], c[4]
            bufs.append((dims, ext, init))
            versions.append(np.full(ext, V_HOST if init else V_UNINIT, dtype=np.int64))
            last_mem.append(np.full(ext, 0 if init else -1, dtype=np.int64))
            initialised.append(np.full(ext, bool(init)))
        elif c[0] == "task":
            tk = c[1]
            tid = len(tasks)
            st = status[tid]
            chunks = split_py(stream.nodes, stream.devices, stream.chunks, tk.lo, tk.hi)
            regions = []
            for k, ch in enumerate(chunks):
                rg = []
                for a in tk.accesses:
                    dims, ext, _ = bufs[a.buffer]
                    r = map_py(a, ch, dims, ext) if not box_empty(ch) else ((0, 0, 0), (0, 0, 0))
                    rg.append(r)
                regions.append(rg)
            # overlapping writes of different chunks (per element)
            owner: Dict[tuple, int] = {}
            overlap = False
            for k, ch in enumerate(chunks):
                if box_empty(ch):
                    continue
                for a, r in zip(tk.accesses, regions[k]):
                    if a.mode & WRITE:
                        for p in box_points(r):
                            key = (a.buffer,) + p
                            if key in owner and owner[key] != k:
                                overlap = True
                            owner[key] = k
            if overlap:
                _require(st == -2, f"task {tid}: overlapping writes must be rejected (got {st})")
                tasks.append((tk, st, None, chunks, regions))
                continue
            uninit = False
            for k, ch in enumerate(chunks):
                if box_empty(ch):
                    continue
                for a, r in zip(tk.accesses, regions[k]):
                    if a.mode & READ:
                        for p in box_points(r):
                            if not initialised[a.buffer][p]:
                                uninit = True
            _require(st == (1 if uninit else 0), f"task {tid}: status {st}, expected {1 if uninit else 0}")
            snap = [v.copy() for v in versions]
            tasks.append((tk, st, snap, chunks, regions))
            per_dev = stream.chunks // (stream.nodes * stream.devices)
            for k, ch in enumerate(chunks):
                if box_empty(ch):
                    continue
                for a, r in zip(tk.accesses, regions[k]):
                    if a.mode & WRITE:
                        for p in box_points(r):
                            versions[a.buffer][p] = tid
                            last_mem[a.buffer][p] = 2 + k // per_dev
                            initialised[a.buffer][p] = True

    # ---------------- symbolic execution in emission order -----------------
    kernels = {}  # (task, chunk) -> instruction id
    bind_of: Dict[int, Dict[int, int]] = {}
    for b in binds:
        bind_of.setdefault(int(b["instr"]), {})[int(b["access"])] = int(b["alloc"])
    counts = {"copies": 0, "kernels": 0, "checked_reads": 0}

    def run(order: List[int], full_checks: bool):
        allocs: Dict[int, dict] = {}
        # user allocations appear only as copy sources on M0
        for r in ins:
            if int(r["kind"]) == COPY and int(r["src_mem"]) == 0:
                a = int(r["src_alloc"])
                b = int(r["buffer"])
                if a not in allocs:
                    dims, ext, init = bufs[b]
                    _require(init == 1, "copy from M0 needs host data")
                    allocs[a] = dict(mem=0, buffer=b, box=((0, 0, 0), tuple(ext)),
                                     data=np.full(ext, V_HOST, dtype=np.int64), alive=True)
        freed = set()
        resizing = set()
        resize_copied: Dict[int, set] = {}  # old allocation -> elements its resize copies moved
        utd = [None] * len(bufs)
        for b, (dims, ext, init) in enumerate(bufs):
            u = np.zeros(tuple(ext) + (256,), dtype=bool)
            if init:
                u[..., 0] = True
            utd[b] = u
        applied_sync = 0
        pending = None
        for x in order:
            r = ins[x]
            kind = int(r["kind"])
            if kind == ALLOC:
                a = int(r["alloc"])
                _require(a not in allocs, f"alloc {a} created twice")
                box = rec_box(r)
                b, m = int(r["buffer"]), int(r["mem"])
                _require(m >= 2, "allocations live on device memories")
                if full_checks:
                    _require(not resizing, f"I{x}: a resize chain left allocations {resizing} unfreed")
                    for o, od in allocs.items():
                        if od["alive"] and od["buffer"] == b and od["mem"] == m and box_intersects(od["box"], box):
                            # only a resize may overlap: the new allocation covers
                            # the old one, which is freed right after its copies
                            _require(box_contains(box, od["box"]), f"I{x}: alloc {a} overlaps live alloc {o}")
                            resizing.add(o)
                shape = tuple(box[1][d] - box[0][d] for d in range(3))
                allocs[a] = dict(mem=m, buffer=b, box=box, data=np.full(shape, V_GARBAGE, dtype=np.int64),
                                 alive=True)
            elif kind == FREE:
                a = int(r["alloc"])
                _require(a in allocs and allocs[a]["alive"], f"I{x}: free of dead alloc {a}")
                _require(allocs[a]["mem"] >= 2, "user memory is never freed")
                if full_checks and a in resizing:
                    # Sec. 3.2: a resize moves exactly the data of the old
                    # allocation that is up to date on its memory
                    od = allocs[a]
                    want = {p for p in box_points(od["box"]) if utd[od["buffer"]][p + (od["mem"],)]}
                    got = resize_copied.get(a, set())
                    _require(got == want, f"I{x}: resize copies out of alloc {a} move {len(got)} elements, "
                                          f"{len(want)} are up to date there (missing {sorted(want - got)[:4]}, "
                                          f"extra {sorted(got - want)[:4]})")
                allocs[a]["alive"] = False
                freed.add(a)
                resizing.discard(a)
            elif kind == COPY:
                s, d = int(r["src_alloc"]), int(r["alloc"])
                box = rec_box(r)
                _require(s in allocs and allocs[s]["alive"], f"I{x}: copy from dead alloc {s}")
                _require(d in allocs and allocs[d]["alive"], f"I{x}: copy to dead alloc {d}")
                sa, da = allocs[s], allocs[d]
                _require(box_contains(sa["box"], box) and box_contains(da["box"], box),
                         f"I{x}: copy box outside its allocations")
                _require(int(r["mem"]) == da["mem"] and int(r["src_mem"]) == sa["mem"], f"I{x}: memories")
                b = int(r["buffer"])
                resize = bool(int(r["flags"]) & F_RESIZE)
                if full_checks:
                    counts["copies"] += 1
                    if resize:
                        _require(sa["mem"] == da["mem"], "resize copies stay on one memory")
                        _require(box_contains(da["box"], sa["box"]), "allocations never shrink")
                        _require(s in resizing, f"I{x}: resize copy out of alloc {s}, which no new allocation covers")
                        moved = resize_copied.setdefault(s, set())
                        for p in box_points(box):
                            _require(p not in moved, f"I{x}: element {p} of alloc {s} moved twice by its resize")
                            moved.add(p)
                    else:
                        dm = da["mem"]
                        inter = (sa["mem"] >= 2 and (sa["mem"] - 2) // stream.devices != (dm - 2) // stream.devices)
                        _require(bool(int(r["flags"]) & F_INTER_NODE) == inter, f"I{x}: inter-node flag")
                        effs = set()
                        for p in box_points(box):
                            _require(utd[b][p].any(), f"I{x}: copies uninitialised data at {p}")
                            _require(not utd[b][p + (dm,)], f"I{x}: redundant copy at {p} (already on M{dm})")
                            _require(last_mem_live[b][p] == sa["mem"], f"I{x}: source is not the producer's memory")
                            eff = max(producer_live[b][p], applied_sync)
                            effs.add(eff)
                        _require(len(effs) == 1, f"I{x}: one copy mixes original producers {effs}")
                for p in box_points(box):
                    ps = tuple(p[dd] - sa["box"][0][dd] for dd in range(3))
                    pd = tuple(p[dd] - da["box"][0][dd] for dd in range(3))
                    da["data"][pd] = sa["data"][ps]
                    if full_checks and not resize:
                        utd[b][p + (da["mem"],)] = True
            elif kind == KERNEL:
                _require(not (full_checks and resizing), f"I{x}: resize chain left {resizing} unfreed")
                t, k = int(r["task"]), int(r["chunk"])
                tk, st, snap, chunks, regions = tasks[t]
                _require(snap is not None, f"I{x}: kernel of a rejected task")
                _require(rec_box(r) == tuple(tuple(v) for v in chunks[k]), f"I{x}: kernel box is the chunk")
                per_dev = stream.chunks // (stream.nodes * stream.devices)
                m = 2 + k // per_dev
                _require(int(r["mem"]) == m, f"I{x}: kernel memory")
                kernels[(t, k)] = x
                bd = bind_of.get(x, {})
                _require(sorted(bd) == list(range(len(tk.accesses))), f"I{x}: one binding per access")
                writes = []
                for j, a in enumerate(tk.accesses):
                    reg = regions[k][j]
                    al = bd[j]
                    if box_empty(reg):
                        _require(al == 0, f"I{x}: empty access bound to an allocation")
                        continue
                    _require(al in allocs and allocs[al]["alive"], f"I{x}: access {j} bound to dead alloc {al}")
                    ad = allocs[al]
                    _require(ad["mem"] == m and ad["buffer"] == a.buffer, f"I{x}: binding memory/buffer")
                    _require(box_contains(ad["box"], reg), f"I{x}: access {j} not inside its allocation")
                    if a.mode & READ:
                        for p in box_points(reg):
                            want = snap[a.buffer][p]
                            if want == V_UNINIT:
                                continue
                            pl = tuple(p[dd] - ad["box"][0][dd] for dd in range(3))
                            got = ad["data"][pl]
                            _require(got == want, f"I{x} (task {t} chunk {k}): element {p} of buffer "
                                                  f"{a.buffer} holds version {got}, expected {want}")
                            counts["checked_reads"] += 1
                    if a.mode & WRITE:
                        writes.append((ad, reg, a.buffer))
                for ad, reg, b in writes:
                    for p in box_points(reg):
                        pl = tuple(p[dd] - ad["box"][0][dd] for dd in range(3))
                        ad["data"][pl] = t
                        if full_checks:
                            utd[b][p] = False
                            utd[b][p + (ad["mem"],)] = True
                            last_mem_live[b][p] = ad["mem"]
                            producer_live[b][p] = x
                if full_checks:
                    counts["kernels"] += 1
            elif kind == HORIZON:
                if pending is not None:
                    applied_sync = pending
                pending = x
            elif kind == EPOCH:
                if x > 0:
                    applied_sync = x
                    pending = None
        return allocs

    # producer tracking for the producer-split check (live during the run)
    last_mem_live = [np.where(v == V_HOST, 0, -1).astype(np.int64) for v in versions]
    producer_live = [np.zeros(b[1], dtype=np.int64) for b in bufs]
    for b, (dims, ext, init) in enumerate(bufs):
        last_mem_live[b] = np.full(ext, 0 if init else -1, dtype=np.int64)
    allocs = run(list(range(n)), True)
    # every device allocation freed exactly once by shutdown
    if stream.cmds and stream.cmds[-1][0] == "shutdown":
        for a, ad in allocs.items():
            if ad["mem"] >= 2:
                _require(not ad["alive"], f"alloc {a} never freed")
    # conflicting accesses are ordered (race freedom => schedule independence)
    accesses: Dict[Tuple[int, tuple], List[Tuple[int, bool]]] = {}

    def note(a, box_, x, w):
        for p in box_points(box_):
            accesses.setdefault((a,) + (p,), []).append((x, w))

    alloc_box = {}
    for r in ins:
        if int(r["kind"]) == ALLOC:
            alloc_box[int(r["alloc"])] = rec_box(r)
    for x in range(n):
        r = ins[x]
        kind = int(r["kind"])
        if kind == ALLOC:
            note(int(r["alloc"]), rec_box(r), x, True)
        elif kind == FREE:
            note(int(r["alloc"]), rec_box(r), x, True)
        elif kind == COPY:
            note(int(r["src_alloc"]), rec_box(r), x, False)
            note(int(r["alloc"]), rec_box(r), x, True)
        elif kind == KERNEL:
            t, k = int(r["task"]), int(r["chunk"])
            tk, st, snap, chunks, regions = tasks[t]
            bd = bind_of.get(x, {})
            for j, a in enumerate(tk.accesses):
                if bd.get(j, 0) == 0:
                    continue
                if a.mode & READ:
                    note(bd[j], regions[k][j], x, False)
                if a.mode & WRITE:
                    note(bd[j], regions[k][j], x, True)
    races = 0
    for key, lst in accesses.items():
        last_w = None
        reads_since: List[int] = []
        for x, w in lst:
            if w:
                if last_w is not None:
                    _require(ordered(last_w, x), f"race: I{last_w} and I{x} both write {key}")
                for y in reads_since:
                    _require(ordered(y, x), f"race: I{y} reads and I{x} writes {key}")
                last_w, reads_since = x, []
            else:
                if last_w is not None:
                    _require(ordered(last_w, x), f"race: I{last_w} writes and I{x} reads {key}")
                reads_since.append(x)
    # a few random topological orders must compute the same versions
    rng = random.Random(seed)
    succ: List[List[int]] = [[] for _ in range(n)]
    indeg = [0] * n
    for t, f in pairs:
        succ[f].append(t)
        indeg[t] += 1
    for _ in range(n_random_orders):
        deg = list(indeg)
        ready = [x for x in range(n) if deg[x] == 0]
        order = []
        while ready:
            x = ready.pop(rng.randrange(len(ready)))
            order.append(x)
            for y in succ[x]:
                deg[y] -= 1
                if deg[y] == 0:
                    ready.append(y)
        _require(len(order) == n, "graph is acyclic")
        run(order, False)
    counts["races_checked"] = len(accesses)
    counts["edges_exact"] = check_edges_exact(stream, out, tasks, bind_of)
    if stream.cmds and stream.cmds[-1][0] == "shutdown":
        counts["queue_commands"] = check_queue(stream, out, tasks)
    return counts


# ---------------------------------------------------------------------------
# Exact edge sets: every edge is justified, element by element
# ---------------------------------------------------------------------------
EV_BUFFER, EV_TASK, EV_REJECTED, EV_HORIZON, EV_EPOCH, EV_DESTROY, EV_SHUTDOWN = 1, 2, 3, 4, 5, 6, 7


class _AllocMap:
    """Per-element allocation map: last writer and, per reader, the elements
    it has read since the last write (boolean masks over the allocation)."""

    def __init__(self, box, writer):
        self.lo = box[0]
        self.shape = tuple(box[1][d] - box[0][d] for d in range(3))
        self.writer = np.full(self.shape, writer, dtype=np.int64)
        self.readers: Dict[int, np.ndarray] = {}

    def mask(self, box):
        m = np.zeros(self.shape, dtype=bool)
        sl = tuple(slice(box[0][d] - self.lo[d], box[1][d] - self.lo[d]) for d in range(3))
        m[sl] = True
        return m


def check_edges_exact(stream, out, tasks, bind_of) -> int:
    """Every instruction's incoming edges, with their kind bits, are exactly
    those its accesses justify on some element of some allocation (the
    dependency legend of the IDAG figure, Sec. 3.6, with Sec. 3.2/3.3):

      * a read of an element: from its last writer -- TRUE, or LIFETIME when
        that writer is the allocation's ALLOC;
      * a write of an element: from every instruction that read it since its
        last write (ANTI); with no such reader, from the last writer (OUTPUT,
        or LIFETIME for the ALLOC);
      * a FREE: from every writer and reader of the allocation (LIFETIME);
      * no justified edge at all: one SYNC edge from the latest epoch or
        applied horizon.
    Everything is evaluated against the state before the instruction; ids
    older than the applied horizon read as that horizon, and an epoch replaces
    every writer and forgets every reader (Sec. 3.5).  Horizons and epochs are
    checked against the execution front elsewhere."""
    ins = out["instructions"]
    n = len(ins)
    events = out.get("events")
    _require(events is not None, "the exact edge check needs the command trace")
    kind_of = [int(k) for k in ins["kind"]]
    preds: List[Dict[int, int]] = [dict() for _ in range(n)]
    for e in out["edges"]:
        preds[int(e["to"])][int(e["from"])] = int(e["kinds"])
    # user allocations on M0: the copies that read them name them
    user_alloc = {}
    for r in ins:
        if int(r["kind"]) == COPY and int(r["src_mem"]) == 0:
            user_alloc[int(r["buffer"])] = int(r["src_alloc"])
    buf_ext = [c[2] for c in stream.cmds if c[0] == "buffer"]
    created_at = {}  # instruction count -> buffers created before that instruction
    for ev in events:
        if int(ev["kind"]) == EV_BUFFER:
            created_at.setdefault(int(ev["n_instr"]), []).append(int(ev["arg"]))
    maps: Dict[int, _AllocMap] = {}
    S, pending = 0, None

    def dep(w, data_kind):
        return DEP_LIFETIME if kind_of[w] == ALLOC else data_kind

    checked = 0
    for x in range(n):
        for b in created_at.get(x, []):
            if b in user_alloc:
                maps[user_alloc[b]] = _AllocMap(((0, 0, 0), tuple(buf_ext[b])), S)
        r = ins[x]
        kind = kind_of[x]
        if kind == HORIZON:
            if pending is not None:
                P = pending
                for am in maps.values():
                    am.writer[am.writer < P] = P
                    old = [q for q in am.readers if q < P]
                    if old:
                        merged = am.readers.get(P, np.zeros(am.shape, dtype=bool)).copy()
                        for q in old:
                            merged |= am.readers.pop(q)
                        am.readers[P] = merged
                S = P
            pending = x
            continue
        if kind == EPOCH:
            if x > 0:
                for am in maps.values():
                    am.writer[...] = x
                    am.readers.clear()
                S, pending = x, None
            continue
        want: Dict[int, int] = {}
        if kind == ALLOC:
            maps[int(r["alloc"])] = _AllocMap(rec_box(r), x)
        elif kind == FREE:
            am = maps.pop(int(r["alloc"]))
            for w in np.unique(am.writer):
                want[int(w)] = want.get(int(w), 0) | DEP_LIFETIME
            for q, msk in am.readers.items():
                if msk.any():
                    want[q] = want.get(q, 0) | DEP_LIFETIME
        else:
            if kind == COPY:
                box = rec_box(r)
                accs = [(int(r["src_alloc"]), box, READ), (int(r["alloc"]), box, WRITE)]
            else:  # KERNEL
                t, k = int(r["task"]), int(r["chunk"])
                tk, _, _, _, regions = tasks[t]
                accs = [(bind_of[x][j], regions[k][j], a.mode) for j, a in enumerate(tk.accesses)
                        if bind_of.get(x, {}).get(j, 0) != 0]
            staged = []
            for a, box, mode in accs:
                am = maps[a]
                m = am.mask(box)
                if mode & READ:
                    for w in np.unique(am.writer[m]):
                        want[int(w)] = want.get(int(w), 0) | dep(int(w), DEP_TRUE)
                if mode & WRITE:
                    read_any = np.zeros(am.shape, dtype=bool)
                    for q, msk in am.readers.items():
                        hit = msk & m
                        if hit.any():
                            want[q] = want.get(q, 0) | DEP_ANTI
                            read_any |= hit
                    for w in np.unique(am.writer[m & ~read_any]):
                        if int(w) != x:
                            want[int(w)] = want.get(int(w), 0) | dep(int(w), DEP_OUTPUT)
                staged.append((am, m, mode))
            for am, m, mode in staged:  # reads are recorded before writes
                if mode & READ:
                    am.readers[x] = am.readers.get(x, np.zeros(am.shape, dtype=bool)) | m
            for am, m, mode in staged:
                if mode & WRITE:
                    am.writer[m] = x
                    for q in list(am.readers):
                        am.readers[q] = am.readers[q] & ~m
                        if not am.readers[q].any():
                            del am.readers[q]
        if not want:
            want = {S: DEP_SYNC}
        _require(preds[x] == want, f"I{x} ({['', 'ALLOC', 'COPY', 'FREE', 'KERNEL'][kind]}): edges "
                                   f"{sorted(preds[x].items())}, justified {sorted(want.items())}")
        checked += 1
    return checked


# ---------------------------------------------------------------------------
# The command queue of Sec. 4.3, simulated from the command trace
# ---------------------------------------------------------------------------
def _merge_components(boxes):
    """Replace boxes that merge (brute-force relation: shared points or axis
    neighbours) by their bounding box until none merge."""
    v = [b for b in boxes if not box_empty(b)]
    changed = True
    while changed:
        changed = False
        for i in range(len(v)):
            for j in range(i + 1, len(v)):
                a, b = v[i], v[j]
                far = any(max(a[0][d], b[0][d]) > min(a[1][d], b[1][d]) for d in range(3))
                if not far and points_merge(a, b):
                    v[i] = (tuple(min(a[0][d], b[0][d]) for d in range(3)),
                            tuple(max(a[1][d], b[1][d]) for d in range(3)))
                    del v[j]
                    changed = True
                    break
            if changed:
                break
    return v


def tdag_horizons(stream, status) -> List[bool]:
    """Horizon placement of the task-graph mode (Sec. 3.5), from an explicit
    task graph built element by element: for each accepted task in order,
    whether a horizon follows it.

    Nodes are numbered in creation order (the initial epoch is 0; tasks,
    horizons and epochs follow).  Per buffer element: the last writer node
    and the reader nodes since.  A read depends on the writer; a write on
    the readers, else the writer; a task without dependencies on the
    synchronisation node.  The critical-path length of a node is one more
    than its dependencies' longest.  A horizon follows a task once the
    longest path has grown by horizon_step since the last horizon or epoch,
    or horizon_max_tasks tasks came since; it depends on everything, so its
    length is the longest plus one, and it makes the horizon before it the
    synchronisation node: every older writer or reader is replaced by that
    one.  An epoch replaces every writer and clears the readers."""
    step = stream.horizon_step
    cap = stream.horizon_max_tasks or 16 * step
    cp = [0]
    sync, pending = 0, None
    cp_max = cp_last = since = 0
    bufs = []
    out = []
    ti = 0

    def apply(node):
        for b in bufs:
            for p in b["w"]:
                if b["w"][p] < node:
                    b["w"][p] = node
                b["r"][p] = {node if r < node else r for r in b["r"][p]}

    for c in stream.cmds:
        if c[0] == "buffer":
            pts = box_points(((0, 0, 0), c[2]))
            bufs.append({"dims": c[1], "ext": c[2], "w": {p: 0 for p in pts}, "r": {p: set() for p in pts}})
        elif c[0] == "task":
            t = c[1]
            ok = int(status[ti]) >= 0
            ti += 1
            if not ok:
                continue
            regions = []
            for ch in split_py(stream.nodes, stream.devices, stream.chunks, t.lo, t.hi):
                if box_empty(ch):
                    continue
                for a in t.accesses:
                    b = bufs[a.buffer]
                    regions.append((a, box_points(map_py(a, ch, b["dims"], b["ext"]))))
            deps = {sync}
            for a, pts in regions:
                b = bufs[a.buffer]
                for p in pts:
                    if a.mode & READ:
                        deps.add(b["w"][p])
                    if a.mode & WRITE:
                        deps |= b["r"][p] if b["r"][p] else {b["w"][p]}
            node = len(cp)
            cp.append(1 + max(cp[d] for d in deps))
            for want in (READ, WRITE):
                for a, pts in regions:
                    if not (a.mode & want):
                        continue
                    b = bufs[a.buffer]
                    for p in pts:
                        if want == READ:
                            b["r"][p].add(node)
                        else:
                            b["w"][p] = node
                            b["r"][p] = set()
            cp_max = max(cp_max, cp[node])
            since += 1
            due = cp_max - cp_last >= step or since >= cap
            out.append(due)
            if due:
                h = len(cp)
                cp.append(cp_max + 1)
                if pending is not None:
                    apply(pending)
                    sync = pending
                pending, cp_last, since = h, cp_max, 0
        elif c[0] in ("epoch", "shutdown"):
            e = len(cp)
            cp.append(cp_max + 1)
            for b in bufs:
                for p in b["w"]:
                    b["w"][p] = e
                    b["r"][p] = set()
            sync, pending = e, None
            cp_max = cp_last = cp[e]
            since = 0
    return out


def check_queue(stream, out, tasks) -> int:
    """The lookahead queue (Sec. 4.3) replayed from the command trace.

    A command is allocating when one of its requirements (the bounding box of
    a (chunk, accessor) region on the chunk's memory) lies in no single box
    of V(m, b): the allocations live at that moment, or -- while allocating
    commands touching (m, b) are queued -- the merge components of those
    allocations and the queued requirements.  A command compiles at once when
    the queue is empty and it is not allocating; otherwise it is queued, and
    the queue flushes once flush_horizons horizons were queued after the last
    allocating command, when it holds queue_cap commands, or at an epoch, a
    buffer destruction or shutdown.  Live allocations come from the emitted
    ALLOC/FREE records before the command; the trace says which event
    compiled each command, and this must match the replay."""
    ev = out["events"]
    ins = out["instructions"]
    nb = sum(1 for c in stream.cmds if c[0] == "buffer")
    # the trace follows the stream: horizons every horizon_step accepted tasks
    seq = []
    since = 0
    for c in stream.cmds:
        if c[0] == "buffer":
            seq.append(EV_BUFFER)
        elif c[0] == "task":
            seq.append(None)  # accepted or rejected
        elif c[0] == "epoch":
            seq.append(EV_EPOCH)
        elif c[0] == "destroy":
            seq.append(EV_DESTROY)
        elif c[0] == "shutdown":
            seq.append(EV_SHUTDOWN)
    kinds = [int(e["kind"]) for e in ev]
    tdag = iter(tdag_horizons(stream, out["status"])) if getattr(stream, "horizon_mode", 0) == 1 else None
    i = 0
    for want in seq:
        _require(i < len(kinds), "command trace ends early")
        if want is None:
            _require(kinds[i] in (EV_TASK, EV_REJECTED), f"event {i}: expected a task, got {kinds[i]}")
            if kinds[i] == EV_TASK:
                since += 1
                due = next(tdag) if tdag is not None else since == stream.horizon_step
                if due:
                    since = 0
                    i += 1
                    _require(i < len(kinds) and kinds[i] == EV_HORIZON, f"event {i}: a horizon is due")
                else:
                    _require(i + 1 >= len(kinds) or kinds[i + 1] != EV_HORIZON, f"event {i + 1}: no horizon is due")
        else:
            _require(kinds[i] == want, f"event {i}: expected {want}, got {kinds[i]}")
            if want in (EV_EPOCH, EV_SHUTDOWN):
                since = 0
        i += 1
    _require(i == len(kinds), "command trace has extra events")
    del nb
    # allocation records, for the live set at any moment
    alloc_rec = {}
    free_at = {}
    for r in ins:
        if int(r["kind"]) == ALLOC:
            alloc_rec[int(r["alloc"])] = (int(r["id"]), int(r["buffer"]), int(r["mem"]), rec_box(r))
        elif int(r["kind"]) == FREE:
            free_at[int(r["alloc"])] = int(r["id"])

    def live_at(n_instr):
        live: Dict[Tuple[int, int], list] = {}
        for a, (aid, b, m, box) in alloc_rec.items():
            if aid < n_instr and free_at.get(a, 1 << 62) >= n_instr:
                live.setdefault((b, m), []).append(box)
        return live

    per_dev = stream.chunks // (stream.nodes * stream.devices)

    def requirements(t):
        tk, _, _, chunks, regions = tasks[t]
        reqs = []
        for k, ch in enumerate(chunks):
            if box_empty(ch):
                continue
            for a, rg in zip(tk.accesses, regions[k]):
                if not box_empty(rg):
                    reqs.append((a.buffer, 2 + k // per_dev, rg))
        return reqs

    expect_alloc = {}
    expect_compiled = {}
    queue = []          # event indices
    queued_reqs = []    # requirements of queued allocating commands
    h = 0

    def flush(at):
        nonlocal queue, queued_reqs, h
        for q in queue:
            expect_compiled[q] = at
        queue, queued_reqs, h = [], [], 0

    for i, e in enumerate(ev):
        k = kinds[i]
        if k in (EV_TASK, EV_HORIZON):
            if not stream.lookahead:
                expect_alloc[i] = 0
                expect_compiled[i] = i
                continue
            alloc = False
            reqs = []
            if k == EV_TASK:
                reqs = requirements(int(e["arg"]))
                live = live_at(int(e["n_instr"]))
                for b, m, box in reqs:
                    planned = [q[2] for q in queued_reqs if q[0] == b and q[1] == m]
                    V = live.get((b, m), [])
                    if queue and planned:
                        V = _merge_components(V + planned)
                    if not any(box_contains(v, box) for v in V):
                        alloc = True
                expect_alloc[i] = int(alloc)
            if not queue and not alloc:
                expect_compiled[i] = i
                continue
            queue.append(i)
            if alloc:
                h = 0
                queued_reqs += reqs
            elif k == EV_HORIZON:
                h += 1
            if h >= stream.flush_horizons or (stream.queue_cap and len(queue) >= stream.queue_cap):
                flush(i)
        elif k in (EV_EPOCH, EV_DESTROY, EV_SHUTDOWN):
            flush(i)
    _require(not queue, "commands left in the queue after shutdown")
    for i, e in enumerate(ev):
        if kinds[i] == EV_TASK and stream.lookahead:
            _require(int(e["allocating"]) == expect_alloc[i],
                     f"event {i} (task {int(e['arg'])}): allocating {int(e['allocating'])}, "
                     f"brute force {expect_alloc[i]}")
        if kinds[i] in (EV_TASK, EV_HORIZON):
            _require(int(e["compiled_at"]) == expect_compiled[i],
                     f"event {i}: compiled during event {int(e['compiled_at'])}, brute force {expect_compiled[i]}")
    return len(expect_compiled)
