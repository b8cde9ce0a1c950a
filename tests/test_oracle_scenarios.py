"""The oracle against the paper's worked examples and closed-form counts.

* P-NB: the N-body instruction graph of Sec. 3.6 (Listing 1 on one node with
  two devices).
* P-RS: the resize of Listing 2 (Sec. 4.3) with and without lookahead.
* P-RSIM: RSim's growing pattern (Sec. 4.3, Sec. 5.3): without lookahead a
  resize every step; with lookahead one allocation per device covering the
  whole program.
* Closed-form instruction counts of the 1-D stencil, the 2-D stencil and
  N-body, derived by hand from the rules (see the design document).
"""
import pytest

import oracle
from oracle import ALLOC, COPY, DEP_SYNC, DEP_TRUE, EPOCH, F_RESIZE, FREE, HORIZON, KERNEL
from paper_2503_10516_amd import streams as S


def kinds(out):
    return [int(k) for k in out["instructions"]["kind"]]


def preds(out, x):
    return {int(e["from"]): int(e["kinds"]) for e in out["edges"] if int(e["to"]) == x}


def test_nbody_worked_example():
    out = oracle.run_stream(S.nbody_example())
    ins = out["instructions"]
    k = kinds(out)
    # I0 epoch; I1-I4 allocations: P whole on M2 and M3 (all mapper), V split
    assert k[:9] == [EPOCH, ALLOC, ALLOC, ALLOC, ALLOC, KERNEL, KERNEL, KERNEL, KERNEL]
    boxes = [(int(ins[i]["buffer"]), int(ins[i]["mem"]), int(ins[i]["min"][0]), int(ins[i]["max"][0]))
             for i in range(1, 5)]
    assert boxes == [(0, 2, 0, 4096), (0, 3, 0, 4096), (1, 2, 0, 2048), (1, 3, 2048, 4096)]
    # I5/I6 timestep kernels, I7/I8 update kernels, with no copies in between
    assert [(int(ins[i]["task"]), int(ins[i]["chunk"])) for i in range(5, 9)] == [(0, 0), (0, 1), (1, 0), (1, 1)]
    # second timestep: exactly one device-to-device copy per producer
    assert k[9:11] == [COPY, COPY]
    assert (int(ins[9]["src_mem"]), int(ins[9]["mem"])) == (3, 2)
    assert (int(ins[10]["src_mem"]), int(ins[10]["mem"])) == (2, 3)
    assert preds(out, 9)[8] & DEP_TRUE and preds(out, 10)[7] & DEP_TRUE
    # then the kernels of the second iteration and the horizon on the front
    assert k[11:16] == [KERNEL, KERNEL, KERNEL, KERNEL, HORIZON]
    assert preds(out, 15) == {13: DEP_SYNC, 14: DEP_SYNC}
    # uninitialised buffers: both first-step tasks warn
    assert list(out["status"]) == [1, 1, 0, 0]


@pytest.mark.parametrize("lookahead,resizes", [(0, 2), (1, 0)])
def test_listing2_resize(lookahead, resizes):
    out = oracle.run_stream(S.resize_example(lookahead))
    st = out["stats"]
    assert st["resizes"] == resizes
    n_resize_copies = int(((out["instructions"]["kind"] == COPY) & (out["instructions"]["flags"] & F_RESIZE > 0)).sum())
    assert n_resize_copies == resizes
    assert st["per_kind"][ALLOC] == 2 + resizes and st["per_kind"][FREE] == 2 + resizes


def test_rsim_growing_pattern():
    steps, devices, width = 32, 8, 840
    on = oracle.run_stream(S.growing(width, steps, devices, lookahead=1), fetch=True)
    # lookahead: nothing is compiled before the final epoch flushes the queue,
    # then one allocation per device covers the entire program
    allocs = on["instructions"][on["instructions"]["kind"] == ALLOC]
    assert len(allocs) == devices and on["stats"]["resizes"] == 0
    for a in allocs:
        assert tuple(a["min"][:2]) == (0, 0) and tuple(a["max"][:2]) == (width, steps)
    first_alloc = int(allocs[0]["id"])
    assert kinds(on)[1:first_alloc] == [] or all(k == HORIZON for k in kinds(on)[1:first_alloc])
    off = oracle.run_stream(S.growing(width, steps, devices, lookahead=0), fetch=False)
    # no lookahead: every step after the first resizes on every device
    assert off["stats"]["resizes"] == devices * (steps - 1)
    # a queue cap W flushes every W commands: far fewer resizes
    capped = oracle.run_stream(S.growing(width, steps, devices, lookahead=1, queue_cap=8), fetch=False)
    assert 0 < capped["stats"]["resizes"] < off["stats"]["resizes"] // 2


def closed_form_1d(tasks, lookahead):
    # epoch, 4 allocs, 2 copies from M0, 2 halo copies per later task,
    # 2 kernels per task, a horizon every 4 tasks, 4 frees, final epoch;
    # without lookahead the second task resizes both neighbourhood reads
    n = 1 + 4 + 2 + 2 * (tasks - 1) + 2 * tasks + tasks // 4 + 4 + 1
    return n if lookahead else n + 6


def closed_form_2d(tasks, chunks):
    return 1 + 2 * chunks + chunks + (tasks - 1) * (2 * chunks - 2) + chunks * tasks + tasks // 4 + 2 * chunks + 1


def closed_form_nbody(steps, chunks):
    return (1 + 2 * chunks + 2 * chunks + (steps - 1) * chunks * (chunks - 1) + 2 * steps * chunks
            + (2 * steps) // 4 + 2 * chunks + 1)


@pytest.mark.parametrize("lookahead", [0, 1])
def test_closed_form_stencil_1d(lookahead):
    out = oracle.run_stream(S.stencil_1d(lookahead=lookahead), fetch=False)
    assert out["stats"]["n_instructions"] == closed_form_1d(64, lookahead)
    assert closed_form_1d(64, 1) == 282 and closed_form_1d(64, 0) == 288


def test_closed_form_stencil_2d_reduced():
    out = oracle.run_stream(S.stencil_2d(side=512, tasks=40, nodes=4, devices=4, chunks=16), fetch=False)
    assert out["stats"]["n_instructions"] == closed_form_2d(40, 16)
    st = out["stats"]
    assert st["per_kind"][COPY] == 16 + 39 * 30 and st["resizes"] == 0


@pytest.mark.slow
def test_closed_form_stencil_2d_full():
    out = oracle.run_stream(S.stencil_2d(), fetch=False)
    assert out["stats"]["n_instructions"] == closed_form_2d(1000, 128) == 382638


def test_closed_form_nbody_reduced():
    out = oracle.run_stream(S.nbody(steps=6), fetch=False)
    assert out["stats"]["n_instructions"] == closed_form_nbody(6, 128)
    assert closed_form_nbody(500, 128) == 8240764


def group_order_stream():
    """Three devices on one node, one host-initialised buffer of 12 elements.
    Tasks 0 and 1 give the devices whole-buffer allocations in the order M3,
    M4, then M2 (allocation ids 2, 3, 4: the order of memories and the order
    of allocation ids disagree).  Task A (box [6,12)) and then task B (box
    [0,6)) write the buffer one_to_one, so every device holds one element
    range of A and one of B.  Task C reads everything on every device."""
    s = S.Stream(1, 3, 3, horizon_step=16, lookahead=0, name="group_order")
    b = s.buffer(1, (12,), 4, S.INIT_HOST)
    s.task(1, (0,), (2,), [S.Access(b, S.READ, S.FIXED, fixed_lo=(0, 0, 0), fixed_hi=(12, 1, 1))])
    s.task(1, (0,), (12,), [S.Access(b, S.READ, S.ALL)])
    s.task(1, (6,), (12,), [S.Access(b, S.WRITE, S.ONE_TO_ONE)])
    s.task(1, (0,), (6,), [S.Access(b, S.WRITE, S.ONE_TO_ONE)])
    s.task(1, (0,), (12,), [S.Access(b, S.READ, S.ALL)])
    s.shutdown()
    return s


def check_group_order(out):
    """Sec. 3.3 splits the stale part of a read by original producer and by
    source allocation; the order of the resulting copies is the reading
    "ascending (producer memory, producer, source allocation)".  Worked by
    hand for group_order_stream: after A ([6,8) on M2, [8,10) on M3, [10,12)
    on M4) and B ([0,2) on M2, [2,4) on M3, [4,6) on M4) -- A's kernels have
    the smaller ids -- task C's chunk on M2 copies from M3 first (A's range,
    then B's), then from M4; the chunk on M3 copies from M2 (allocation 4)
    before M4 (allocation 3), so memory order, not allocation order, leads."""
    ins = out["instructions"]
    c_copies = [r for r in ins if int(r["kind"]) == COPY and int(r["task"]) == 4]
    got = [(int(r["mem"]), int(r["src_mem"]), int(r["src_alloc"]), int(r["min"][0]), int(r["max"][0]))
           for r in c_copies]
    want = [(2, 3, 2, 8, 10), (2, 3, 2, 2, 4), (2, 4, 3, 10, 12), (2, 4, 3, 4, 6),
            (3, 2, 4, 6, 8), (3, 2, 4, 0, 2), (3, 4, 3, 10, 12), (3, 4, 3, 4, 6),
            (4, 2, 4, 6, 8), (4, 2, 4, 0, 2), (4, 3, 2, 8, 10), (4, 3, 2, 2, 4)]
    assert got == want, got
    kern = {(int(r["task"]), int(r["chunk"])): int(r["id"]) for r in ins if int(r["kind"]) == KERNEL}
    producer = {(3, 8): kern[(2, 1)], (3, 2): kern[(3, 1)], (4, 10): kern[(2, 2)], (4, 4): kern[(3, 2)],
                (2, 6): kern[(2, 0)], (2, 0): kern[(3, 0)]}
    assert kern[(2, 0)] < kern[(2, 1)] < kern[(2, 2)] < kern[(3, 0)]
    for r in c_copies:
        p = producer[(int(r["src_mem"]), int(r["min"][0]))]
        assert preds(out, int(r["id"])).get(p, 0) & DEP_TRUE


def test_copy_group_order_hand_worked():
    check_group_order(oracle.run_stream(group_order_stream()))


# ---------------------------------------------------------------------------
# Horizons from the task graph (Sec. 3.5, horizon_mode 1)
# ---------------------------------------------------------------------------
CHAINS = [
    ("stencil1d", lambda: S.stencil_1d()),
    ("stencil2d", lambda: S.stencil_2d(side=256, tasks=40, nodes=2, devices=4, chunks=16)),
    ("nbody", lambda: S.nbody(n=4096, steps=10, nodes=2, devices=4, chunks=16)),
    ("growing", lambda: S.growing(width=840, steps=40)),
    ("growing_nola", lambda: S.growing(width=840, steps=24, lookahead=0)),
    ("nbody_example", S.nbody_example),
]


@pytest.mark.parametrize("name,make", CHAINS, ids=[c[0] for c in CHAINS])
def test_tdag_horizons_equal_fixed_step_on_chains(name, make):
    """In these workloads every task depends on the one before it, so the
    critical path grows by one per task and the task graph asks for a
    horizon exactly every horizon_step tasks: the same graph, record by
    record, as the fixed step (282 instructions for the 1-D stencil)."""
    a, b = make(), make()
    b.horizon_mode = 1
    ra, rb = oracle.run_stream(a), oracle.run_stream(b)
    for k in ("instructions", "bindings", "edges"):
        assert ra[k].tobytes() == rb[k].tobytes(), (name, k)
    if name == "stencil1d":
        assert len(rb["instructions"]) == 282


def test_tdag_independent_tasks_horizon_by_width():
    """Tasks on four disjoint buffers, task t on buffer t mod 4: task t
    depends only on task t - 4, so the critical path grows by one every four
    tasks.  Worked by hand: with a step of 4 the path alone asks for a
    horizon after task 13 (path length 4) and task 29 (length 8, four more
    than at the first horizon); a cap of 6 tasks between horizons comes
    first, after tasks 6, 12, 18, 24 and 30."""
    def make(cap):
        s = S.Stream(1, 2, 2, lookahead=0, horizon_mode=1, horizon_max_tasks=cap)
        bufs = [s.buffer(1, (16,), 4, S.INIT_HOST) for _ in range(4)]
        for t in range(32):
            s.task(1, (0,), (16,), [S.Access(bufs[t % 4], S.READ_WRITE, S.ONE_TO_ONE)])
        s.shutdown()
        return s
    for cap, want in ((100, [13, 29]), (6, [6, 12, 18, 24, 30])):
        ev = oracle.run_stream(make(cap))["events"]
        kinds = [int(e["kind"]) for e in ev]
        tasks_before = []
        n = 0
        for k in kinds:
            if k == oracle.EV_TASK:
                n += 1
            elif k == oracle.EV_HORIZON:
                tasks_before.append(n)
        assert tasks_before == want, (cap, tasks_before)
