"""Helpers comparing HIP-path output with the oracle, record by record."""
import numpy as np


def first_difference(a: np.ndarray, b: np.ndarray):
    n = min(len(a), len(b))
    if n:
        ra = a[:n].view(np.uint8).reshape(n, -1)
        rb = b[:n].view(np.uint8).reshape(n, -1)
        bad = np.nonzero((ra != rb).any(axis=1))[0]
        if len(bad):
            return int(bad[0])
    if len(a) != len(b):
        return n
    return None


def assert_same(want, got, name=""):
    """Bit-exact equality of instructions, bindings, edges and task statuses
    (integer output: no tolerance)."""
    for key in ("instructions", "bindings", "edges", "status"):
        a, b = want[key], got[key]
        i = first_difference(a, b)
        assert i is None, (f"{name}: {key} differ at record {i} (len {len(a)} vs {len(b)}):\n"
                           f"  oracle {a[i] if i < len(a) else None}\n  hip    {b[i] if i < len(b) else None}")


def record_words(out):
    """The digest words of each record list (see the digest definition)."""
    ins = out["instructions"]
    w = np.zeros((len(ins), 12), dtype=np.uint64)
    w[:, 0] = ins["id"]
    w[:, 1] = (ins["kind"].astype(np.uint64) | (ins["flags"].astype(np.uint64) << np.uint64(8))
               | (ins["mem"].astype(np.uint64) << np.uint64(16)) | (ins["src_mem"].astype(np.uint64) << np.uint64(32)))
    w[:, 2] = ins["task"].astype(np.uint64) | (ins["chunk"].astype(np.uint64) << np.uint64(32))
    w[:, 3] = ins["buffer"]
    w[:, 4] = ins["alloc"]
    w[:, 5] = ins["src_alloc"]
    w[:, 6:9] = ins["min"].astype(np.uint64)
    w[:, 9:12] = ins["max"].astype(np.uint64)
    b = out["bindings"]
    wb = np.stack([b["instr"], b["access"].astype(np.uint64), b["alloc"]], axis=1).astype(np.uint64)
    e = out["edges"]
    we = np.stack([e["from"], e["to"], e["kinds"].astype(np.uint64)], axis=1).astype(np.uint64)
    return w, wb, we


def reader_run_stream(variant):
    """All-reads over several chunks per device (shared read scans, runs of
    readers), neighborhood reads that refine the grid, epochs, lookahead on
    and off and a queue cap; variant 2 leaves one buffer uninitialised."""
    from paper_2503_10516_amd import streams as S
    s = S.Stream(2, 2, 16, lookahead=variant % 2, queue_cap=3 if variant == 3 else 0, name=f"reader_runs{variant}")
    p = s.buffer(1, (512,), 8, S.INIT_HOST)
    q = s.buffer(1, (512,), 8, S.INIT_HOST if variant != 2 else S.INIT_NONE)
    for t in range(14):
        s.task(1, (0,), (512,), [S.Access(p, S.READ, S.ALL), S.Access(q, S.WRITE, S.ONE_TO_ONE)])
        if t % 3 == 0:
            s.task(1, (0,), (512,), [S.Access(q, S.READ, S.NEIGHBORHOOD, (t + 1, 0, 0)),
                                      S.Access(p, S.WRITE, S.ONE_TO_ONE)])
        if t % 5 == 4:
            s.epoch()
        if t % 4 == 1:
            s.task(1, (0,), (512,), [S.Access(q, S.READ, S.SLICE, slice_dim=0), S.Access(p, S.READ, S.ALL),
                                      S.Access(q, S.READ, S.NEIGHBORHOOD, (2, 0, 0))])
            s.task(1, (0,), (512,), [S.Access(p, S.READ_WRITE, S.ONE_TO_ONE), S.Access(q, S.READ, S.ALL)])
    s.shutdown()
    return s


def big_read_stream(variant):
    """Reads whose regions span hundreds of grid cells on every device (all,
    slice along dim 0, large fixed boxes), next to neighborhood reads of the
    same buffer in the same task, before and after them, so that some reads
    are contained in an earlier large one and some only overlap it; several
    chunks per device, up to 32 devices.  The large regions are the ones a
    team of threads scans together."""
    from paper_2503_10516_amd import streams as S
    nodes, devices, chunks, dims, ext = [(1, 8, 256, 1, (1 << 13,)), (2, 8, 256, 1, (1 << 12,)),
                                         (2, 8, 128, 2, (256, 16)), (4, 8, 256, 1, (1 << 12,))][variant]
    s = S.Stream(nodes, devices, chunks, lookahead=1, queue_cap=8 if variant == 1 else 0,
                 name=f"big_reads{variant}")
    bufs = [s.buffer(dims, ext, 4, S.INIT_HOST) for _ in range(3)]
    lo, hi = (0,) * dims, ext
    rad = lambda r: tuple(r if d < dims else 0 for d in range(3))
    half = tuple(e // 2 if d == 0 else e for d, e in enumerate(ext)) + (1,) * (3 - dims)
    for t in range(18):
        a, b, c = bufs[t % 3], bufs[(t + 1) % 3], bufs[(t + 2) % 3]
        acc = [S.Access(a, S.WRITE if t % 2 else S.READ_WRITE, S.ONE_TO_ONE)]
        k = t % 6
        if k == 0:
            acc += [S.Access(b, S.READ, S.NEIGHBORHOOD, rad(1 + t % 3)), S.Access(c, S.READ, S.ALL)]
        elif k == 1:
            acc += [S.Access(b, S.READ, S.NEIGHBORHOOD, rad(2)), S.Access(b, S.READ, S.ALL)]
        elif k == 2:
            acc += [S.Access(b, S.READ, S.ALL), S.Access(b, S.READ, S.NEIGHBORHOOD, rad(3))]
        elif k == 3:
            acc += [S.Access(c, S.READ, S.SLICE, slice_dim=0), S.Access(b, S.READ, S.NEIGHBORHOOD, rad(1))]
        elif k == 4:
            acc += [S.Access(b, S.READ, S.FIXED, fixed_lo=(0, 0, 0), fixed_hi=half),
                    S.Access(b, S.READ, S.NEIGHBORHOOD, rad(4)), S.Access(c, S.READ, S.ONE_TO_ONE)]
        else:
            acc += [S.Access(b, S.READ, S.NEIGHBORHOOD, rad(2)), S.Access(c, S.READ, S.FIXED,
                    fixed_lo=(ext[0] // 4, 0, 0), fixed_hi=tuple(3 * ext[0] // 4 if d == 0 else
                                                               (ext[d] if d < dims else 1) for d in range(3))),
                    S.Access(c, S.READ, S.ALL)]
        s.task(dims, lo, hi, acc)
        if t == 11:
            s.epoch()
    s.shutdown()
    return s


# --- the out-of-order engine simulation (Sec. 4.1) ---

OOO_PARAMS = [
    dict(lanes_per_device=1, host_lanes=1, window=1),
    dict(lanes_per_device=2, host_lanes=2, window=16),
    dict(lanes_per_device=3, host_lanes=1, window=1024, eager=0),
    dict(lanes_per_device=2, host_lanes=3, window=7),
    dict(lanes_per_device=4, host_lanes=2, window=4096, kernel_ns=1, copy_ns=1, alloc_ns=1, free_ns=1,
         kernel_ns_per_kelem=0, copy_ns_per_kelem=0, inter_node_ns=0),
]


def ooo_against_oracle(streams, contexts, kw, oracle_outs=None):
    """Simulate the engine over the contexts' graphs (one launch) and over
    the oracle's graphs of the same streams; every slot and summary must be
    equal (integer output: no tolerance)."""
    import oracle
    from paper_2503_10516_amd import binding as B
    devs = max(s.nodes * s.devices for s in streams)
    sim = B.OooSimulation(contexts, B.ooo_params(devs, **kw))
    sim.run()
    try:
        for i, s in enumerate(streams):
            o = oracle_outs[i] if oracle_outs is not None else oracle.run_stream(s)
            want, wsum = oracle.ooo_simulate(o["instructions"], o["edges"], oracle.ooo_params(devs, **kw))
            got, gsum = sim.fetch(i)
            assert len(got) == len(want), (s.name, len(got), len(want))
            j = first_difference(want, got)
            assert j is None, f"{s.name} {kw}: slot {j} differs: oracle {want[j]} hip {got[j]}"
            assert gsum == wsum, (s.name, kw, gsum, wsum)
    finally:
        sim.close()
