"""Seeded synthetic command streams: the inputs of instruction-graph generation.

This module only *describes* workloads: cluster shapes, buffers and the
ordered list of commands a user program would submit (buffer creation, tasks
with range-mapped accessors, epochs, buffer destruction, shutdown).  It holds
none of the analysis itself: no chunk split, no range-mapper evaluation, no
region maps.  Both the CPU oracle (through its own binding) and the HIP path
(through the product binding) consume the same `Stream` objects.

Workloads stand in for the access patterns of the paper's applications
(Sec. 5: N-body with an all-gather pattern, Listing 1; WaveSim, a 5-point
stencil; RSim, a buffer that grows by one row per time step) and for the
resize example of Listing 2.  No dataset is involved.
"""
from __future__ import annotations

from dataclasses import dataclass, field
from typing import List, Sequence, Tuple

import numpy as np

# access modes (bit set: READ_WRITE = READ | WRITE)
READ, WRITE, READ_WRITE = 1, 2, 3
# range mappers
ONE_TO_ONE, NEIGHBORHOOD, ALL, SLICE, FIXED = 0, 1, 2, 3, 4
# buffer initialisation
INIT_NONE, INIT_HOST = 0, 1

Vec3 = Tuple[int, int, int]


@dataclass(frozen=True)
class Access:
    buffer: int
    mode: int
    mapper: int
    radius: Vec3 = (0, 0, 0)
    slice_dim: int = 0
    fixed_lo: Vec3 = (0, 0, 0)
    fixed_hi: Vec3 = (0, 0, 0)


@dataclass(frozen=True)
class Task:
    dims: int
    lo: Vec3
    hi: Vec3
    accesses: Tuple[Access, ...]


@dataclass
class Stream:
    """One user program on one simulated cluster.

    cmds holds tuples:
      ("buffer", dims, extent3, elem_size, init)   -> buffer ids 0, 1, ... in order
      ("task", Task)
      ("epoch",)
      ("destroy", buffer_id)
      ("shutdown",)
    """
    nodes: int
    devices: int
    chunks: int
    horizon_step: int = 4
    lookahead: int = 1
    flush_horizons: int = 2
    queue_cap: int = 0
    horizon_mode: int = 0        # 0: a horizon every horizon_step tasks; 1: from the task graph (Sec. 3.5)
    horizon_max_tasks: int = 0   # mode 1: tasks between horizons at most (0: 16 x horizon_step)
    staging: int = 0             # 1: device-to-device copies within a node staged through pinned host memory
    cmds: List[tuple] = field(default_factory=list)
    name: str = ""

    # --- builders -----------------------------------------------------------
    def buffer(self, dims: int, extent: Sequence[int], elem_size: int = 4,
               init: int = INIT_HOST) -> int:
        ext = tuple(int(e) for e in extent) + (1,) * (3 - len(extent))
        bid = sum(1 for c in self.cmds if c[0] == "buffer")
        self.cmds.append(("buffer", dims, ext, elem_size, init))
        return bid

    def task(self, dims: int, lo: Sequence[int], hi: Sequence[int],
             accesses: Sequence[Access]) -> None:
        lo3 = tuple(int(v) for v in lo) + (0,) * (3 - len(lo))
        hi3 = tuple(int(v) for v in hi) + (1,) * (3 - len(hi))
        self.cmds.append(("task", Task(dims, lo3, hi3, tuple(accesses))))

    def epoch(self) -> None:
        self.cmds.append(("epoch",))

    def destroy(self, b: int) -> None:
        self.cmds.append(("destroy", b))

    def shutdown(self) -> None:
        self.cmds.append(("shutdown",))

    @property
    def n_tasks(self) -> int:
        return sum(1 for c in self.cmds if c[0] == "task")

    def desc(self) -> dict:
        return dict(nodes=self.nodes, devices=self.devices, chunks=self.chunks,
                    horizon_step=self.horizon_step, lookahead=self.lookahead,
                    flush_horizons=self.flush_horizons, queue_cap=self.queue_cap,
                    horizon_mode=self.horizon_mode, horizon_max_tasks=self.horizon_max_tasks, staging=self.staging)


def splitmix64(x: int) -> int:
    """Seed derivation for per-stream generators (published splitmix64)."""
    x = (x + 0x9E3779B97F4A7C15) & 0xFFFFFFFFFFFFFFFF
    z = x
    z = ((z ^ (z >> 30)) * 0xBF58476D1CE4E5B9) & 0xFFFFFFFFFFFFFFFF
    z = ((z ^ (z >> 27)) * 0x94D049BB133111EB) & 0xFFFFFFFFFFFFFFFF
    return z ^ (z >> 31)


def _full(dims: int, ext: Vec3):
    return (0, 0, 0), tuple(ext[d] if d < dims else 1 for d in range(3))


# ---------------------------------------------------------------------------
# The five workloads
# ---------------------------------------------------------------------------

def stencil_1d(n: int = 4096, tasks: int = 64, nodes: int = 1, devices: int = 2,
               chunks: int = 2, lookahead: int = 1, elem_size: int = 8,
               queue_cap: int = 0) -> Stream:
    """1-D 3-point stencil, double-buffered: task t reads neighborhood(1) of
    X_t and writes one_to_one Y_t, X/Y swapping every task."""
    s = Stream(nodes, devices, chunks, lookahead=lookahead, queue_cap=queue_cap,
               name=f"stencil1d_n{n}_t{tasks}")
    a = s.buffer(1, (n,), elem_size, INIT_HOST)
    b = s.buffer(1, (n,), elem_size, INIT_HOST)
    for t in range(tasks):
        x, y = (a, b) if t % 2 == 0 else (b, a)
        s.task(1, (0,), (n,), [Access(x, READ, NEIGHBORHOOD, (1, 0, 0)),
                               Access(y, WRITE, ONE_TO_ONE)])
    s.shutdown()
    return s


def stencil_2d(side: int = 4096, tasks: int = 1000, nodes: int = 16, devices: int = 8,
               chunks: int = 128, lookahead: int = 1, elem_size: int = 4) -> Stream:
    """2-D 5-point stencil (WaveSim access pattern): neighborhood(1,1) read of
    one buffer and one_to_one write of the other, alternating."""
    s = Stream(nodes, devices, chunks, lookahead=lookahead,
               name=f"stencil2d_{side}_t{tasks}_c{chunks}")
    a = s.buffer(2, (side, side), elem_size, INIT_HOST)
    b = s.buffer(2, (side, side), elem_size, INIT_HOST)
    for t in range(tasks):
        x, y = (a, b) if t % 2 == 0 else (b, a)
        s.task(2, (0, 0), (side, side), [Access(x, READ, NEIGHBORHOOD, (1, 1, 0)),
                                         Access(y, WRITE, ONE_TO_ONE)])
    s.shutdown()
    return s


def nbody(n: int = 1 << 20, steps: int = 500, nodes: int = 16, devices: int = 8,
          chunks: int = 128, lookahead: int = 1, init: int = INIT_HOST,
          elem_size: int = 16) -> Stream:
    """N-body (Listing 1): per step a 'timestep' task (all-read of P,
    one_to_one read_write of V) and an 'update' task (one_to_one read of V,
    one_to_one read_write of P)."""
    s = Stream(nodes, devices, chunks, lookahead=lookahead,
               name=f"nbody_n{n}_s{steps}_c{chunks}")
    p = s.buffer(1, (n,), elem_size, init)
    v = s.buffer(1, (n,), elem_size, init)
    for _ in range(steps):
        s.task(1, (0,), (n,), [Access(p, READ, ALL), Access(v, READ_WRITE, ONE_TO_ONE)])
        s.task(1, (0,), (n,), [Access(v, READ, ONE_TO_ONE), Access(p, READ_WRITE, ONE_TO_ONE)])
    s.shutdown()
    return s


def nbody_example() -> Stream:
    """The paper's worked IDAG example (Sec. 3.6): Listing 1 on one node with
    two devices, buffers uninitialised, two time steps."""
    return nbody(n=4096, steps=2, nodes=1, devices=2, chunks=2, lookahead=1,
                 init=INIT_NONE, elem_size=24)


def resize_example(lookahead: int, rows: int = 64, cols: int = 64) -> Stream:
    """Listing 2: one_to_one write followed by a neighborhood({1,1}) read of
    the same 2-D buffer, split over two devices."""
    s = Stream(1, 2, 2, lookahead=lookahead, name=f"resize_la{lookahead}")
    b = s.buffer(2, (rows, cols), 4, INIT_NONE)
    s.task(2, (0, 0), (rows, cols), [Access(b, WRITE, ONE_TO_ONE)])
    s.task(2, (0, 0), (rows, cols), [Access(b, READ, NEIGHBORHOOD, (1, 1, 0))])
    s.shutdown()
    return s


def growing(width: int = 84000, steps: int = 256, devices: int = 8, queue_cap: int = 0,
            lookahead: int = 1, init: int = INIT_HOST) -> Stream:
    """RSim's growing pattern: buffer [width x steps]; task t has index box
    [0,width) x [t,t+1), writes it one_to_one and reads the fixed region
    [0,width) x [0,t) of all earlier rows."""
    s = Stream(1, devices, devices, lookahead=lookahead, queue_cap=queue_cap,
               name=f"growing_w{width}_t{steps}_q{queue_cap}")
    b = s.buffer(2, (width, steps), 4, init)
    for t in range(steps):
        acc = [Access(b, WRITE, ONE_TO_ONE)]
        if t > 0:
            acc.append(Access(b, READ, FIXED, fixed_lo=(0, 0, 0), fixed_hi=(width, t, 1)))
        s.task(2, (0, t), (width, t + 1), acc)
    s.shutdown()
    return s


def batched_stream(master_seed: int, index: int, max_tasks: int = 2000,
                   max_log_chunks: int = 10, max_log_extent: int = 24,
                   w_all: float = 0.1, w_slice: float = 0.1) -> Stream:
    """One stream of the batched workload: random shape, 2-4 buffers, random
    range mappers, lookahead with a queue cap of 64."""
    rng = np.random.default_rng(splitmix64((master_seed + index) & 0xFFFFFFFFFFFFFFFF))
    dims = int(rng.integers(1, 4))
    e = int(rng.integers(10, max_log_extent + 1))
    # spread the exponent bits over the dims, dim 0 largest
    bits = [e // dims] * dims
    for i in range(e - sum(bits)):
        bits[i] += 1
    ext = tuple(1 << bits[d] if d < dims else 1 for d in range(3))
    c = int(rng.integers(4, max_log_chunks + 1))
    chunks = 1 << c
    node_choices = [n for n in (1, 2, 4, 8, 16) if 8 * n <= chunks]
    nodes = int(rng.choice(node_choices))
    s = Stream(nodes, 8, chunks, horizon_step=4, lookahead=1, queue_cap=64,
               name=f"batched_{index}")
    nb = int(rng.integers(2, 5))
    bufs = [s.buffer(dims, ext, 4, INIT_HOST) for _ in range(nb)]
    n_tasks = int(rng.integers(50, max_tasks + 1))
    w_o2o, w_nbh = 0.4, 0.4
    wsum = w_o2o + w_nbh + w_slice + w_all
    probs = np.array([w_o2o, w_nbh, w_slice, w_all]) / wsum
    lo, hi = _full(dims, ext)
    for t in range(n_tasks):
        wb = bufs[t % nb]
        wmode = WRITE if rng.random() < 0.5 else READ_WRITE
        acc = [Access(wb, wmode, ONE_TO_ONE)]
        others = [b for b in bufs if b != wb]
        nr = min(len(others), int(rng.integers(1, 3)))
        picks = rng.choice(len(others), size=nr, replace=False)
        for pi in sorted(int(p) for p in picks):
            kind = int(rng.choice(4, p=probs))
            rb = others[pi]
            if kind == 0:
                acc.append(Access(rb, READ, ONE_TO_ONE))
            elif kind == 1:
                r = int(rng.integers(1, 5))
                acc.append(Access(rb, READ, NEIGHBORHOOD, tuple(r if d < dims else 0 for d in range(3))))
            elif kind == 2:
                acc.append(Access(rb, READ, SLICE, slice_dim=int(rng.integers(0, dims))))
            else:
                acc.append(Access(rb, READ, ALL))
        s.task(dims, lo, hi, acc)
    s.shutdown()
    return s


BATCHED_SEED = 0x2503105160000004
SERVING_SEED = 0x2503105160000005
# Weights of the all and slice read mappers in the batched workload.  The
# workload is defined with 0.1 each; at that mix the 256 streams project to
# about 1.5e10 records (an all-read over 1024 chunks on 128 devices alone
# emits ~1.3e5 copies and ~1e6 edges), so both are lowered once, to 0.005,
# which projects to ~1.6e9 records.
BATCHED_W_ALL = 0.005
BATCHED_W_SLICE = 0.005


def batched(n_streams: int = 256, **kw) -> List[Stream]:
    kw.setdefault("w_all", BATCHED_W_ALL)
    kw.setdefault("w_slice", BATCHED_W_SLICE)
    return [batched_stream(BATCHED_SEED, i, **kw) for i in range(n_streams)]


def random_small(seed: int, n_tasks: int = 12, race_free: bool = True,
                 max_dims: int = 3, allow_epochs: bool = True,
                 allow_destroy: bool = True) -> Stream:
    """Tiny random streams for property and brute-force tests (all extents
    at most 16 per dimension).  With race_free, no task reads a region of a
    buffer that another chunk of the same task writes (the paper leaves such
    programs undefined)."""
    rng = np.random.default_rng(seed)
    nodes = int(rng.integers(1, 3))
    devices = int(rng.integers(1, 4))
    k = int(rng.integers(1, 3))
    s = Stream(nodes, devices, nodes * devices * k,
               horizon_step=int(rng.integers(1, 6)),
               lookahead=int(rng.integers(0, 2)),
               flush_horizons=int(rng.integers(1, 4)),
               queue_cap=int(rng.choice([0, 0, 2, 5])),
               name=f"random_{seed}")
    dims = int(rng.integers(1, max_dims + 1))
    ext = tuple(int(rng.integers(2, 17)) if d < dims else 1 for d in range(3))
    nb = int(rng.integers(1, 4))
    bufs = [s.buffer(dims, ext, 4, int(rng.integers(0, 2))) for _ in range(nb)]
    alive = list(bufs)
    for t in range(n_tasks):
        if not alive:
            break
        roll = rng.random()
        if allow_epochs and roll < 0.06:
            s.epoch()
            continue
        if allow_destroy and roll < 0.09 and len(alive) > 1:
            b = alive.pop(int(rng.integers(0, len(alive))))
            s.destroy(b)
            continue
        lo = [0, 0, 0]
        hi = [1, 1, 1]
        for d in range(dims):
            a = int(rng.integers(0, ext[d]))
            bnd = int(rng.integers(a + 1, ext[d] + 1))
            if rng.random() < 0.5:
                a, bnd = 0, ext[d]
            lo[d], hi[d] = a, bnd
        acc = []
        nacc = int(rng.integers(1, 4))
        written = set()
        for _ in range(nacc):
            b = alive[int(rng.integers(0, len(alive)))]
            mode = int(rng.choice([READ, READ, WRITE, READ_WRITE]))
            if mode & WRITE:
                if b in written:
                    mode = READ
                else:
                    written.add(b)
            if mode & WRITE:
                mapper = ONE_TO_ONE if rng.random() < 0.8 else SLICE
                sd = int(rng.integers(1, dims)) if (mapper == SLICE and dims > 1) else 0
                if mapper == SLICE and dims == 1:
                    mapper = ONE_TO_ONE
                acc.append(Access(b, mode, mapper, slice_dim=sd))
            else:
                mapper = int(rng.choice([ONE_TO_ONE, NEIGHBORHOOD, ALL, SLICE, FIXED]))
                if mapper == NEIGHBORHOOD:
                    r = tuple(int(rng.integers(0, 3)) if d < dims else 0 for d in range(3))
                    acc.append(Access(b, mode, mapper, radius=r))
                elif mapper == SLICE:
                    acc.append(Access(b, mode, mapper, slice_dim=int(rng.integers(0, dims))))
                elif mapper == FIXED:
                    flo = [0, 0, 0]
                    fhi = [1, 1, 1]
                    for d in range(dims):
                        a = int(rng.integers(0, ext[d]))
                        flo[d], fhi[d] = a, int(rng.integers(a, ext[d] + 1))
                    acc.append(Access(b, mode, mapper, fixed_lo=tuple(flo), fixed_hi=tuple(fhi)))
                else:
                    acc.append(Access(b, mode, mapper))
        if race_free:
            # a read of a written buffer in the same task must use the same
            # one_to_one footprint, otherwise chunks race with each other
            wb = {a.buffer for a in acc if a.mode & WRITE}
            fixed_acc = []
            for a in acc:
                if a.buffer in wb and not (a.mode & WRITE):
                    a = Access(a.buffer, READ, ONE_TO_ONE)
                fixed_acc.append(a)
            # a slice write of dim d>0 is still a chunk-disjoint write; reads of
            # that buffer must then match it
            wsl = {a.buffer: a for a in fixed_acc if a.mode & WRITE}
            acc = [Access(a.buffer, READ, wsl[a.buffer].mapper, slice_dim=wsl[a.buffer].slice_dim)
                   if (a.buffer in wsl and not (a.mode & WRITE)) else a for a in fixed_acc]
        s.task(dims, tuple(lo), tuple(hi), acc)
    s.shutdown()
    return s


def serving_sessions(seed: int = SERVING_SEED, n_sessions: int = 16,
                     nbody_steps: int = 50, stencil2d_tasks: int = 1000) -> List[Stream]:
    """Sessions of the serving workload: drawn from the 1-D stencil, the 2-D
    stencil, a shortened N-body and the growing pattern with a random queue
    cap (the lookahead window)."""
    rng = np.random.default_rng(seed)
    out = []
    for i in range(n_sessions):
        kind = int(rng.integers(0, 4))
        if kind == 0:
            s = stencil_1d()
        elif kind == 1:
            s = stencil_2d(tasks=stencil2d_tasks)
        elif kind == 2:
            s = nbody(steps=nbody_steps)
        else:
            cap = int(rng.choice([1, 2, 4, 8, 16, 32, 64]))
            s = growing(queue_cap=cap)
        s.name = f"session{i}_{s.name}"
        out.append(s)
    return out


def poisson_arrivals(n: int, rate_per_s: float, seed: int = SERVING_SEED) -> np.ndarray:
    """Arrival times (seconds) of n requests of a Poisson process."""
    rng = np.random.default_rng(seed ^ int(rate_per_s))
    return np.cumsum(rng.exponential(1.0 / rate_per_s, size=n))
