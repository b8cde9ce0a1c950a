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
    return counts
