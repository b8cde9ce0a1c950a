"""The out-of-order engine of Sec. 4.1, simulated by the oracle: a
hand-worked graph, a closed form and invariants that hold for any graph.

The engine assigns each instruction of a finished instruction graph to an
in-order lane directly (all dependencies complete) or eagerly (every
incomplete dependency already issued to one lane of its class); the rules
are written out in oracle/ig_oracle.h."""
import numpy as np
import pytest

import oracle
from oracle import ALLOC, COPY, EPOCH, FREE, HORIZON, KERNEL
from paper_2503_10516_amd import streams as S

NONE32 = 0xFFFFFFFF


def make_graph(rows, deps):
    ins = np.zeros(len(rows), dtype=oracle.INSTR_DTYPE)
    for i, (kind, mem, vol) in enumerate(rows):
        ins[i]["id"] = i
        ins[i]["kind"] = kind
        ins[i]["mem"] = mem
        ins[i]["min"] = (0, 0, 0)
        ins[i]["max"] = (vol, 1, 1)
    ed = [(f, t) for t, fs in deps.items() for f in fs]
    edges = np.zeros(len(ed), dtype=oracle.EDGE_DTYPE)
    for i, (f, t) in enumerate(sorted(ed, key=lambda e: (e[1], e[0]))):
        edges[i]["from"], edges[i]["to"], edges[i]["kinds"] = f, t, 1
    return ins, edges


def test_hand_worked_graph():
    """Two devices with one lane each, one host lane; kernels 100 ns,
    copies 50, allocations 10.  Worked by hand: the second kernel on device
    0 is queued eagerly behind the first (issued at 10, starts at 110); the
    copy into device 0 waits until the kernel on device 1 (lane 1) has
    finished at 120, then goes eagerly behind the second kernel on lane 0
    (start 210, end 260); the horizon completes with it at 260."""
    rows = [(EPOCH, 0xFFFF, 0), (ALLOC, 2, 8), (ALLOC, 3, 8), (KERNEL, 2, 8), (KERNEL, 3, 8), (KERNEL, 2, 8),
            (COPY, 2, 8), (HORIZON, 0xFFFF, 0)]
    deps = {1: [0], 2: [0], 3: [1], 4: [2], 5: [3], 6: [4, 5], 7: [6]}
    ins, edges = make_graph(rows, deps)
    p = oracle.ooo_params(2, lanes_per_device=1, host_lanes=1, window=100, eager=1, kernel_ns=100,
                          kernel_ns_per_kelem=0, copy_ns=50, copy_ns_per_kelem=0, inter_node_ns=0, alloc_ns=10,
                          free_ns=5)
    out, summ = oracle.ooo_simulate(ins, edges, p)
    want = [(NONE32, 0, 0, 0, 0), (2, 1, 0, 0, 10), (2, 1, 0, 10, 20), (0, 1, 10, 10, 110), (1, 1, 20, 20, 120),
            (0, 2, 10, 110, 210), (0, 2, 120, 210, 260), (NONE32, 0, 260, 260, 260)]
    got = [(int(r["lane"]), int(r["how"]), int(r["issue"]), int(r["start"]), int(r["end"])) for r in out]
    assert got == want
    assert summ["makespan"] == 260 and summ["direct"] == 4 and summ["eager"] == 2


def _run(rows, deps, devices, q, host, window, eager):
    ins, edges = make_graph(rows, deps)
    p = oracle.ooo_params(devices, lanes_per_device=q, host_lanes=host, window=window, eager=eager, kernel_ns=100,
                          kernel_ns_per_kelem=0, copy_ns=50, copy_ns_per_kelem=0, inter_node_ns=0, alloc_ns=10,
                          free_ns=5)
    out, summ = oracle.ooo_simulate(ins, edges, p)
    return [(int(r["lane"]), int(r["how"]), int(r["issue"]), int(r["start"]), int(r["end"])) for r in out], summ


def test_hand_worked_lane_choice():
    """One device with two lanes: three independent kernels after an
    allocation go to lanes 0, 1 and then 0 again (the lane that frees
    first, the lower one on a tie); the kernel after the first two cannot
    queue eagerly (they sit on different lanes) and starts directly at 110
    on lane 1, which is free before lane 0."""
    rows = [(EPOCH, 0xFFFF, 0), (ALLOC, 2, 8), (KERNEL, 2, 8), (KERNEL, 2, 8), (KERNEL, 2, 8), (KERNEL, 2, 8),
            (HORIZON, 0xFFFF, 0)]
    deps = {1: [0], 2: [1], 3: [1], 4: [1], 5: [2, 3], 6: [4, 5]}
    got, summ = _run(rows, deps, 1, 2, 1, 8, 1)
    assert got == [(NONE32, 0, 0, 0, 0), (2, 1, 0, 0, 10), (0, 1, 10, 10, 110), (1, 1, 10, 10, 110),
                   (0, 1, 10, 110, 210), (1, 1, 110, 110, 210), (NONE32, 0, 210, 210, 210)]
    assert summ["makespan"] == 210 and summ["direct"] == 5 and summ["eager"] == 0


def test_hand_worked_window():
    """The window bounds how far past the oldest unassigned instruction the
    engine looks: with a window of one, the kernel on the second device
    (which only needs the epoch) waits behind the allocation chain of the
    first and the makespan grows from 120 to 210."""
    rows = [(EPOCH, 0xFFFF, 0), (ALLOC, 2, 8), (KERNEL, 2, 8), (ALLOC, 2, 8), (KERNEL, 3, 8), (HORIZON, 0xFFFF, 0)]
    deps = {1: [0], 2: [1], 3: [2], 4: [0], 5: [3, 4]}
    wide, summ = _run(rows, deps, 2, 1, 1, 8, 1)
    assert wide == [(NONE32, 0, 0, 0, 0), (2, 1, 0, 0, 10), (0, 1, 10, 10, 110), (2, 1, 110, 110, 120),
                    (1, 1, 0, 0, 100), (NONE32, 0, 120, 120, 120)]
    assert summ["makespan"] == 120
    narrow, summ = _run(rows, deps, 2, 1, 1, 1, 1)
    assert narrow == [(NONE32, 0, 0, 0, 0), (2, 1, 0, 0, 10), (0, 1, 10, 10, 110), (2, 1, 110, 110, 120),
                      (1, 1, 110, 110, 210), (NONE32, 0, 210, 210, 210)]
    assert summ["makespan"] == 210


def _graphs():
    yield oracle.run_stream(S.nbody_example()), 2
    yield oracle.run_stream(S.stencil_1d(n=256, tasks=12)), 2
    yield oracle.run_stream(S.nbody(n=64, steps=3, nodes=2, devices=2, chunks=8)), 4
    for seed in range(6):
        s = S.random_small(seed)
        yield oracle.run_stream(s), s.nodes * s.devices


def _durations(out, p):
    ins = out["instructions"]
    vol = np.prod(np.maximum(ins["max"] - ins["min"], 0), axis=1).astype(np.uint64)
    d = np.zeros(len(ins), dtype=np.uint64)
    k = ins["kind"]
    d[k == KERNEL] = p.kernel_ns + vol[k == KERNEL] * p.kernel_ns_per_kelem // 1024
    cp = k == COPY
    d[cp] = p.copy_ns + vol[cp] * p.copy_ns_per_kelem // 1024 + \
        np.where((ins["flags"][cp] & oracle.F_INTER_NODE) != 0, p.inter_node_ns, 0).astype(np.uint64)
    d[k == ALLOC] = p.alloc_ns
    d[k == FREE] = p.free_ns
    return d


def test_unbounded_lanes_give_the_critical_path():
    """With as many lanes as instructions, an unbounded window and direct
    assignment only, nothing ever waits for a lane: every instruction starts
    when its last dependency ends, and the makespan is the longest path of
    the graph weighted by the durations (computed here by a pass in id
    order, which is a topological order)."""
    for out, devs in _graphs():
        n = len(out["instructions"])
        p = oracle.ooo_params(devs, lanes_per_device=n, host_lanes=n, window=n, eager=0)
        slots, summ = oracle.ooo_simulate(out["instructions"], out["edges"], p)
        dur = _durations(out, p)
        finish = np.zeros(n, dtype=np.uint64)
        ready = np.zeros(n, dtype=np.uint64)
        by_to = {}
        for e in out["edges"]:
            by_to.setdefault(int(e["to"]), []).append(int(e["from"]))
        for x in range(n):
            ready[x] = max([finish[f] for f in by_to.get(x, [])], default=0)
            finish[x] = ready[x] + dur[x]
        assert (slots["start"] == ready).all() and (slots["end"] == finish).all()
        assert summ["makespan"] == int(finish.max()) and summ["eager"] == 0


@pytest.mark.parametrize("lanes,host,window,eager", [(1, 1, 1, 1), (1, 1, 64, 1), (2, 2, 16, 1), (3, 1, 1024, 0),
                                                      (2, 3, 7, 1)])
def test_engine_invariants(lanes, host, window, eager):
    """For any parameters: every instruction starts after each of its
    dependencies ends; a lane runs one instruction at a time, in the order
    they were issued to it; a direct instruction was issued when all its
    dependencies were complete, an eager one when each incomplete one was
    on its lane; the engine's own instructions finish as they are issued;
    kernels and copies into a device run on that device's lanes; with a
    window of one the instructions are issued in id order."""
    for out, devs in _graphs():
        ins, edges = out["instructions"], out["edges"]
        p = oracle.ooo_params(devs, lanes_per_device=lanes, host_lanes=host, window=window, eager=eager)
        slots, summ = oracle.ooo_simulate(ins, edges, p)
        dur = _durations(out, p)
        assert (slots["end"] - slots["start"] == dur).all()
        assert (slots["start"] >= slots["issue"]).all()
        for e in edges:
            f, t = int(e["from"]), int(e["to"])
            assert slots["start"][t] >= slots["end"][f]
            if slots["how"][t] == oracle.OOO_DIRECT or slots["how"][t] == oracle.OOO_ENGINE:
                assert slots["end"][f] <= slots["issue"][t]
            elif slots["end"][f] > slots["issue"][t]:  # incomplete when the eager issue happened
                assert slots["lane"][f] == slots["lane"][t] and slots["issue"][f] <= slots["issue"][t]
        for lane in set(int(x) for x in slots["lane"]) - {NONE32}:
            # several rounds can issue at one instant, so the issue time
            # orders a lane's queue only up to ties: sort by start
            idx = np.nonzero(slots["lane"] == lane)[0]
            order = idx[np.lexsort((slots["end"][idx], slots["start"][idx]))]
            s, e = slots["start"][order], slots["end"][order]
            assert (s[1:] >= e[:-1]).all()
            assert (np.diff(slots["issue"][order].astype(np.int64)) >= 0).all()
        kinds = ins["kind"]
        dev = (kinds == KERNEL) | ((kinds == COPY) & (ins["mem"] >= 2))
        assert (slots["lane"][dev] // lanes == ins["mem"][dev] - 2).all()
        eng = (kinds == HORIZON) | (kinds == EPOCH)
        assert (slots["lane"][eng] == NONE32).all() and (slots["start"][eng] == slots["issue"][eng]).all()
        if window == 1:
            assert (np.diff(slots["issue"].astype(np.int64)) >= 0).all()
        assert summ["makespan"] == int(slots["end"].max())
        if not eager:
            assert summ["eager"] == 0
