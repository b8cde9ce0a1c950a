"""Parity of the HIP path (libig, gfx950) with the CPU oracle.

Integer output: instructions, bindings, edges and per-task statuses must be
identical record by record, in canonical order.  Every call goes through the
C ABI of include/ig.h via the ctypes binding.
"""
import numpy as np
import pytest

import oracle
from parity import assert_same, big_read_stream, reader_run_stream, record_words
from paper_2503_10516_amd import binding as B
from paper_2503_10516_amd import streams as S

pytestmark = pytest.mark.gpu

SCENARIOS = [
    ("nbody_example", S.nbody_example),
    ("stencil1d", lambda: S.stencil_1d()),
    ("stencil1d_nola", lambda: S.stencil_1d(lookahead=0)),
    ("resize0", lambda: S.resize_example(0)),
    ("resize1", lambda: S.resize_example(1)),
    ("growing", lambda: S.growing(width=840, steps=32)),
    ("growing_nola", lambda: S.growing(width=840, steps=32, lookahead=0)),
    ("growing_cap4", lambda: S.growing(width=840, steps=32, queue_cap=4)),
    ("stencil2d_small", lambda: S.stencil_2d(side=256, tasks=24, nodes=2, devices=4, chunks=16)),
    ("nbody_small", lambda: S.nbody(n=4096, steps=6, nodes=4, devices=4, chunks=32)),
]


def run_both(s, **kw):
    print(f"[gpu] {s.name} tasks={s.n_tasks} chunks={s.chunks} {kw}", flush=True)
    return oracle.run_stream(s), B.run_stream(s, **kw)


@pytest.fixture(scope="module", autouse=True)
def _device():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    torch.cuda.set_device(0)


@pytest.mark.parametrize("name,make", SCENARIOS, ids=[s[0] for s in SCENARIOS])
def test_scenarios(name, make):
    want, got = run_both(make())
    assert_same(want, got, name)


@pytest.mark.parametrize("seed", range(40))
def test_random_streams(seed):
    s = S.random_small(seed)
    want, got = run_both(s)
    assert_same(want, got, s.name)


@pytest.mark.parametrize("threads", [64, 128, 1024])
def test_workgroup_size_does_not_change_output(threads):
    s = S.stencil_2d(side=512, tasks=20, nodes=4, devices=8, chunks=64)
    want, got = run_both(s, threads=threads)
    assert_same(want, got, f"{s.name}@{threads}")


def test_device_digest_matches_records():
    s = S.nbody(n=1 << 12, steps=4, nodes=2, devices=4, chunks=16)
    want, got = run_both(s)
    assert_same(want, got, s.name)
    w, wb, we = record_words(got)
    st = got["stats"]
    assert st["digest_instructions"] == oracle.digest_words(w) == want["stats"]["digest_instructions"]
    assert st["digest_bindings"] == oracle.digest_words(wb) == want["stats"]["digest_bindings"]
    assert st["digest_edges"] == oracle.digest_words(we) == want["stats"]["digest_edges"]
    assert st["per_kind"] == want["stats"]["per_kind"] and st["per_dep"] == want["stats"]["per_dep"]


def test_stencil2d_full_size():
    """The 2-D stencil at its full size: 4096^2, 1000 tasks, 16x8 devices, 128
    chunks -- every record compared."""
    want, got = run_both(S.stencil_2d())
    assert len(got["instructions"]) == 382638
    assert_same(want, got, "stencil2d")


def test_nbody_full_chunks_reduced_steps():
    want, got = run_both(S.nbody(steps=20))
    assert_same(want, got, "nbody20")


def test_rewind_reanalyses_identically():
    s = S.stencil_1d(n=1024, tasks=32)
    ctx = B.make_context(s)
    ctx.record(s)
    ctx.flush()
    assert ctx.sync() == 0
    first = ctx.fetch_all()
    ctx.rewind()
    ctx.flush()
    assert ctx.sync() == 0
    second = ctx.fetch_all()
    ctx.close()
    for k in first:
        assert first[k].tobytes() == second[k].tobytes()


def test_incremental_windows_match_one_window():
    """Flushing after every command gives the same graph as one flush."""
    s = S.growing(width=840, steps=24, queue_cap=5)
    want = oracle.run_stream(s)
    ctx = B.make_context(s)
    for c in s.cmds:
        ctx.record(S.Stream(s.nodes, s.devices, s.chunks, cmds=[c]))
        ctx.flush()
    assert ctx.sync() == 0
    got = ctx.fetch_all()
    ctx.close()
    assert_same(want, got, "incremental")


def test_overlapping_write_status():
    s = S.Stream(1, 2, 2, lookahead=0)
    b = s.buffer(1, (64,), 4, S.INIT_HOST)
    s.task(1, (0,), (64,), [S.Access(b, S.WRITE, S.ONE_TO_ONE)])
    s.task(1, (0,), (64,), [S.Access(b, S.WRITE, S.ALL)])
    s.task(1, (0,), (64,), [S.Access(b, S.READ, S.ALL)])
    s.shutdown()
    want, got = run_both(s)
    assert list(got["status"]) == [0, -2, 0]
    assert_same(want, got, "overlap")


def test_batched_launch_matches_single_streams():
    """One launch over many streams (one workgroup each) gives every stream
    exactly its oracle graph."""
    streams = [S.random_small(1000 + i) for i in range(24)] + [S.stencil_1d(n=512, tasks=20), S.nbody_example()]
    ctxs = []
    for s in streams:
        ctx = B.make_context(s, threads=256)
        ctx.record(s)
        ctxs.append(ctx)
    print(f"[gpu] batched launch over {len(ctxs)} streams", flush=True)
    B.batch_flush(ctxs)
    for s, ctx in zip(streams, ctxs):
        assert ctx.sync() == 0
        got = ctx.fetch_all()
        assert_same(oracle.run_stream(s), got, "batched:" + s.name)
        ctx.close()


def test_batched_generator_streams_sample():
    """Small streams of the batched workload generator, batched, against the
    oracle (the generator's large streams are checked against single-stream
    runs by the benchmark)."""
    gen = [S.batched_stream(S.BATCHED_SEED, i, max_tasks=120, max_log_chunks=6, max_log_extent=14)
           for i in range(12)]
    ctxs = []
    for s in gen:
        ctx = B.make_context(s, threads=256)
        ctx.record(s)
        ctxs.append(ctx)
    B.batch_flush(ctxs)
    for s, ctx in zip(gen, ctxs):
        assert ctx.sync() == 0
        assert_same(oracle.run_stream(s), ctx.fetch_all(), "batchgen:" + s.name)
        ctx.close()


def test_batch_graph_replays_match_oracle():
    """The captured graph (reset + batched analysis) replayed several times,
    with eager work and synchronisations between replays: every replay gives
    every stream its oracle graph."""
    import torch
    streams = [S.random_small(2000 + i) for i in range(6)] + [S.stencil_2d(side=256, tasks=24, nodes=2, devices=4,
                                                                               chunks=16), S.nbody_example()]
    ctxs = []
    for s in streams:
        ctx = B.make_context(s, threads=256)
        ctx.record(s)
        ctxs.append(ctx)
    want = [oracle.run_stream(s) for s in streams]
    g = B.BatchGraph(ctxs)
    x = torch.arange(1 << 20, device="cuda", dtype=torch.float32)
    for replay in range(3):
        print(f"[gpu] graph replay {replay}", flush=True)
        g.launch()
        for s, ctx, w in zip(streams, ctxs, want):
            assert ctx.sync() == 0
            assert_same(w, ctx.fetch_all(), f"graph{replay}:{s.name}")
        x = (x * 2 + 1).sum().expand(1 << 20).contiguous()  # eager work between replays
        torch.cuda.synchronize()
    prog = B.batch_progress(ctxs)
    assert (prog[:, 2] == 0).all() and (prog[:, 3] == 1).all()
    assert list(prog[:, 0]) == [s.n_tasks for s in streams]
    g.close()
    for c in ctxs:
        c.close()


def test_batch_class_resizes_and_matches_oracle():
    from paper_2503_10516_amd import batch as BT
    streams = [S.nbody(n=4096, steps=8, nodes=4, devices=4, chunks=32), S.stencil_1d(n=512, tasks=30),
               S.random_small(21), S.growing(width=840, steps=24, queue_cap=5)]
    bt = BT.Batch(streams, threads=256, margin=0.05, floor=16)
    assert sum(bt.size().values()) >= 1
    bt.launch()
    for s, ctx in zip(streams, bt.contexts):
        assert ctx.sync() == 0
        assert_same(oracle.run_stream(s), ctx.fetch_all(), "batch:" + s.name)
    bt.close()


DIGESTS = ("n_instructions", "n_bindings", "n_edges", "digest_instructions", "digest_bindings", "digest_edges")


def test_serving_mix_equals_each_session_alone():
    """Continuous batching on the device: sessions admitted into 3 slots as
    they free up, Poisson arrivals; each session's graph equals its oracle
    graph and its graph when analysed alone."""
    from paper_2503_10516_amd import serve
    sessions = [S.stencil_2d(side=512, tasks=40, nodes=2, devices=4, chunks=16), S.nbody(n=4096, steps=6, nodes=4,
                                                                                            devices=4, chunks=32),
                S.growing(width=840, steps=24, queue_cap=2), S.stencil_1d(n=512, tasks=30), S.random_small(31),
                S.growing(width=840, steps=16, lookahead=0)]
    print(f"[gpu] serving {len(sessions)} sessions", flush=True)
    out = serve.Server(slots=3, threads=256).run(sessions, rate=2e4)
    assert out["launches"] >= 2
    for s, st in zip(sessions, out["session_stats"]):
        want = oracle.run_stream(s, fetch=False)["stats"]
        alone = B.run_stream(s, fetch=False)["stats"]
        for k in DIGESTS:
            assert st[k] == want[k] == alone[k], (s.name, k)


@pytest.mark.parametrize("variant", range(4))
def test_reader_runs(variant):
    s = reader_run_stream(variant)
    want, got = run_both(s)
    assert_same(want, got, s.name)


@pytest.mark.parametrize("threads", [64, 1024])
def test_many_chunks_per_device(threads):
    """Eight chunks per device: shared read scans, runs of readers, copies of
    one device emitted by many threads."""
    s = S.nbody(n=1 << 14, steps=6, nodes=2, devices=4, chunks=64)
    want, got = run_both(s, threads=threads)
    assert_same(want, got, f"{s.name}@{threads}")


def test_copies_with_many_sources_on_all_threads():
    s = S.nbody(n=4096, steps=3, nodes=1, devices=2, chunks=64)
    want, got = run_both(s, threads=256)
    assert_same(want, got, s.name)


def test_windowed_batch_matches_oracle():
    """Launches bounded to a few commands per stream, then a graph replay."""
    from paper_2503_10516_amd import batch as BT
    streams = [S.stencil_2d(side=256, tasks=20, nodes=2, devices=4, chunks=32), S.random_small(41),
               S.growing(width=840, steps=20, queue_cap=3)]
    bt = BT.Batch(streams, threads=256)
    prog = bt.analyse(range(len(streams)), window=5)
    assert (prog[:, 2] == 0).all() and list(prog[:, 5]) == [len(s.cmds) for s in streams]
    for s, ctx in zip(streams, bt.contexts):
        assert ctx.sync() == 0
        assert_same(oracle.run_stream(s), ctx.fetch_all(), "window:" + s.name)
    bt.launch()
    for s, ctx in zip(streams, bt.contexts):
        assert ctx.sync() == 0
        assert_same(oracle.run_stream(s), ctx.fetch_all(), "replay:" + s.name)
    bt.close()


@pytest.mark.parametrize("variant", range(4))
@pytest.mark.parametrize("threads", [64, 256, 1024])
def test_big_reads_team_scans(variant, threads):
    """Read regions of hundreds of cells scanned by thread teams (coherence),
    shared source lists of all/slice/fixed reads across the kernels of a
    device, and buffer destruction by teams: record by record."""
    s = big_read_stream(variant)
    want, got = run_both(s, threads=threads)
    assert_same(want, got, f"{s.name}_t{threads}")


@pytest.mark.parametrize("seed", range(24))
def test_task_graph_horizons(seed):
    """Horizons from the task graph (horizon mode 1, Sec. 3.5): random
    streams, with low caps on the tasks between horizons for some."""
    from test_oracle_semantics import tdag_stream
    s = tdag_stream(seed)
    want, got = run_both(s)
    assert_same(want, got, s.name)


TDAG_LARGE = [
    ("stencil2d", lambda: S.stencil_2d(side=512, tasks=40, nodes=2, devices=4, chunks=16)),
    ("nbody", lambda: S.nbody(n=4096, steps=8, nodes=4, devices=4, chunks=32)),
    ("growing_q4", lambda: S.growing(width=840, steps=32, queue_cap=4)),
    ("batched_0", lambda: S.batched_stream(S.BATCHED_SEED, 0, max_tasks=300, w_all=0.05, w_slice=0.05)),
    ("batched_5", lambda: S.batched_stream(S.BATCHED_SEED, 5, max_tasks=300, w_all=0.05, w_slice=0.05)),
]


@pytest.mark.parametrize("name,make", TDAG_LARGE, ids=[t[0] for t in TDAG_LARGE])
def test_task_graph_horizons_larger_streams(name, make):
    s = make()
    s.horizon_mode = 1
    s.name += "_tdag"
    want, got = run_both(s)
    assert_same(want, got, s.name)


@pytest.mark.parametrize("seed", range(40))
def test_racy_random_streams(seed):
    """Reads of regions that other chunks of the same task write (a user
    race): reads see the state before the task, only overlapping writes are
    errors.  Such tasks take the ordered kernel path."""
    s = S.random_small(seed, race_free=False)
    want, got = run_both(s)
    assert_same(want, got, s.name + "_racy")


# full-size streams of the batched workload with 512-1024 chunks and all or
# slice reads over up to 128 devices (the workload's heaviest kind of task)
BATCHED_FULL = [88, 91, 165, 138, 248, 13]


def test_batched_full_size_streams_with_all_reads():
    import json
    import os
    from paper_2503_10516_amd import batch as BT
    gold = json.load(open(os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden",
                                       "batched_digests.json")))
    rows = {r["index"]: r for r in gold["streams"]}
    streams = [S.batched_stream(S.BATCHED_SEED, i, w_all=gold["w_all"], w_slice=gold["w_slice"])
               for i in BATCHED_FULL]
    for s in streams:
        print(f"[gpu] batched full {s.name}: {s.n_tasks} tasks, {s.chunks} chunks, {s.nodes} nodes", flush=True)
    bt = BT.Batch(streams, threads=256)
    bt.size(window=400)
    for i, ctx in zip(BATCHED_FULL, bt.contexts):
        assert ctx.sync() == 0
        st = ctx.stats()
        for k in DIGESTS + ("per_kind", "per_dep"):
            assert st[k] == rows[i][k], (i, k)
    bt.close()


# ---------------------------------------------------------------------------
# device-to-device copies staged through pinned host memory (Sec. 3.3, last
# paragraph), against the oracle run here
# ---------------------------------------------------------------------------

def _staged(s):
    import dataclasses
    return dataclasses.replace(s, staging=1, name=s.name + "_staged")


@pytest.mark.parametrize("index", range(30))
def test_staged_copies_equal_oracle(index):
    from test_oracle_staging import cases
    s = _staged(cases()[index])
    print(f"[gpu] staged {s.name}", flush=True)
    assert_same(oracle.run_stream(s), B.run_stream(s), s.name)


@pytest.mark.parametrize("index,threads", [(191, 256), (90, 256), (147, 1024), (138, 64)])
def test_staged_full_size_batched_streams(index, threads):
    """Full-size streams of the batched workload (512-1024 chunks over 2-8
    nodes of 8 devices) with staging, record by record."""
    s = _staged(S.batched_stream(S.BATCHED_SEED, index, w_all=S.BATCHED_W_ALL, w_slice=S.BATCHED_W_SLICE))
    print(f"[gpu] staged batched_{index}, {threads} threads", flush=True)
    assert_same(oracle.run_stream(s), B.run_stream(s, threads=threads), s.name)


def test_staged_full_size_stencil2d():
    s = _staged(S.stencil_2d())
    print("[gpu] staged stencil2d full", flush=True)
    assert_same(oracle.run_stream(s), B.run_stream(s), s.name)
