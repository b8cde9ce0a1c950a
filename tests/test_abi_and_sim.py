"""CPU checks of the product library.

* libig.so (the gfx950 build) loads and exports every function declared in
  include/ig.h -- nothing is called, so no GPU is needed.
* The kernel logic of ig_kernels.hip, compiled for the host with one
  workgroup emulated by threads and barriers (a test-only build, never used
  by the product), reproduces the oracle bit for bit on small streams.
"""
import ctypes
import os
import re
import subprocess

import pytest

import oracle
from parity import OOO_PARAMS, assert_same, big_read_stream, ooo_against_oracle, reader_run_stream
from paper_2503_10516_amd import binding as B
from paper_2503_10516_amd import streams as S

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_2503_10516_amd", "csrc")
SIM_DIR = os.path.join(ROOT, "tests", "_sim")
SIM_LIB = os.path.join(SIM_DIR, "libig_sim.so")


def declared_functions():
    text = open(os.path.join(ROOT, "include", "ig.h")).read()
    return sorted(set(re.findall(r"^\s*(?:ig_status|const char\*)\s+(ig_\w+)\s*\(", text, re.M)))


def test_header_declares_the_boundary():
    names = declared_functions()
    for n in ("ig_context_create", "ig_submit_task", "ig_flush_window", "ig_fetch_instructions",
              "ig_fetch_edges", "ig_fetch_bindings", "ig_batch_flush", "ig_stats_get"):
        assert n in names
    assert set(names) == set(B.EXPORTS)


def test_hip_library_exports_every_declared_symbol():
    path = B.LIB_PATH
    if not os.path.exists(path):
        pytest.skip("libig.so not built")
    import ctypes
    lib = ctypes.CDLL(path)
    for n in declared_functions():
        assert hasattr(lib, n), n


def _sources():
    return [os.path.join(CSRC, f) for f in ("ig_sim.cpp", "ig_api.cpp", "ig_kernels.hip", "ig_ooo.hip", "ig_dev.h")] + \
        [os.path.join(ROOT, "include", "ig.h")]


@pytest.fixture(scope="session")
def sim_lib():
    os.makedirs(SIM_DIR, exist_ok=True)
    newest = max(os.path.getmtime(p) for p in _sources())
    if not os.path.exists(SIM_LIB) or os.path.getmtime(SIM_LIB) < newest:
        tmp = SIM_LIB + ".tmp%d" % os.getpid()
        subprocess.check_call(["g++", "-std=c++17", "-O1", "-g", "-DIG_HOST_SIM", "-I" + CSRC,
                               "-I" + os.path.join(ROOT, "include"), "-x", "c++", "-fPIC", "-shared", "-o", tmp,
                               os.path.join(CSRC, "ig_sim.cpp"), os.path.join(CSRC, "ig_api.cpp"), "-lpthread"])
        os.replace(tmp, SIM_LIB)
    return SIM_LIB


SIM_SCENARIOS = [
    ("nbody_example", S.nbody_example),
    ("stencil1d", lambda: S.stencil_1d(n=256, tasks=24)),
    ("stencil1d_nola", lambda: S.stencil_1d(n=256, tasks=24, lookahead=0)),
    ("resize0", lambda: S.resize_example(0, 8, 8)),
    ("resize1", lambda: S.resize_example(1, 8, 8)),
    ("growing", lambda: S.growing(width=12, steps=8, devices=4)),
    ("growing_nola", lambda: S.growing(width=12, steps=8, devices=4, lookahead=0)),
    ("growing_cap3", lambda: S.growing(width=12, steps=8, devices=4, queue_cap=3)),
    ("stencil2d", lambda: S.stencil_2d(side=64, tasks=12, nodes=2, devices=4, chunks=8)),
    ("nbody_small", lambda: S.nbody(n=256, steps=4, nodes=2, devices=2, chunks=8)),
]


@pytest.mark.parametrize("name,make", SIM_SCENARIOS, ids=[s[0] for s in SIM_SCENARIOS])
def test_sim_scenarios(name, make, sim_lib):
    s = make()
    assert_same(oracle.run_stream(s), B.run_stream(s, lib_path=sim_lib, threads=64), name)


@pytest.mark.parametrize("seed", range(0, 60, 3))
def test_sim_random_streams(seed, sim_lib):
    s = S.random_small(seed)
    assert_same(oracle.run_stream(s), B.run_stream(s, lib_path=sim_lib, threads=64), s.name)


@pytest.mark.parametrize("seed", range(1, 60, 3))
def test_sim_racy_random_streams(seed, sim_lib):
    """Reads of regions other chunks of the same task write: reads see the
    state before the task (the ordered kernel path)."""
    s = S.random_small(seed, race_free=False)
    assert_same(oracle.run_stream(s), B.run_stream(s, lib_path=sim_lib, threads=64), s.name + "_racy")


def test_sim_invalid_arguments(sim_lib):
    ctx = B.Context(1, 2, lib_path=sim_lib, threads=64)
    b = ctx.buffer_create(2, (8, 8, 1), 4, 1)
    with pytest.raises(B.IgError) as e:
        ctx.submit(S.Task(1, (0, 0, 0), (8, 1, 1), (S.Access(b, S.READ, S.ONE_TO_ONE),)))
    assert e.value.status == B.IG_E_INVALID
    with pytest.raises(B.IgError):
        ctx.submit(S.Task(2, (0, 0, 0), (8, 8, 1), (S.Access(5, S.READ, S.ALL),)))
    with pytest.raises(B.IgError):
        B.Context(1, 2, chunks=3, lib_path=sim_lib, threads=64)
    ctx.close()


def test_sim_capacity_error_is_reported(sim_lib):
    s = S.stencil_1d(n=256, tasks=16)
    with pytest.raises(B.IgError) as e:
        B.run_stream(s, lib_path=sim_lib, threads=64, cap_instructions=40)
    assert e.value.status == B.IG_E_CAPACITY


def test_sim_batch_graph_replays_identically(sim_lib):
    streams = [S.stencil_1d(n=128, tasks=10), S.nbody_example(), S.random_small(7)]
    ctxs = []
    for s in streams:
        ctx = B.make_context(s, lib_path=sim_lib, threads=64)
        ctx.record(s)
        ctxs.append(ctx)
    g = B.BatchGraph(ctxs)
    for replay in range(2):
        g.launch()
        for s, ctx in zip(streams, ctxs):
            assert ctx.sync() == 0
            assert_same(oracle.run_stream(s), ctx.fetch_all(), f"graph{replay}:{s.name}")
    g.close()
    B.batch_rewind(ctxs)
    B.batch_flush(ctxs)
    for s, ctx in zip(streams, ctxs):
        assert ctx.sync() == 0
        assert_same(oracle.run_stream(s), ctx.fetch_all(), "rewound:" + s.name)
        ctx.close()


def test_sim_progress_is_the_compiled_prefix(sim_lib):
    """tasks_done counts the leading tasks whose records exist: every kernel
    of a done task is emitted, no kernel of a later task is."""
    s = S.stencil_1d(n=256, tasks=21)
    ctx = B.make_context(s, lib_path=sim_lib, threads=64)
    kernels_of = set()
    prev = 0
    for cut in (3, 9, 16, len(s.cmds) - 1, len(s.cmds)):
        ctx.record(S.Stream(s.nodes, s.devices, s.chunks, cmds=s.cmds[prev:cut]))
        prev = cut
        ctx.flush()
        assert ctx.sync() == 0
        done, seen, err, fin, _, _ = (int(v) for v in B.batch_progress([ctx])[0])
        assert err == 0 and done <= seen
        assert seen == sum(1 for c in s.cmds[:cut] if c[0] == "task")
        ins = ctx.fetch_all()["instructions"]  # records since the previous fetch
        kernels_of |= set(int(t) for t in ins[ins["kind"] == 4]["task"])
        assert kernels_of == set(range(done))
        assert fin == (1 if cut == len(s.cmds) else 0)
    assert done == seen == s.n_tasks
    ctx.close()


def test_sim_batch_resizes_and_matches_oracle(sim_lib):
    """Deliberately small capacities: the batch re-creates the streams that
    overflow, and every stream's graph is still its oracle graph."""
    from paper_2503_10516_amd import batch as BT
    streams = [S.nbody(n=256, steps=6, nodes=2, devices=4, chunks=8), S.stencil_1d(n=128, tasks=8),
               S.random_small(11), S.growing(width=12, steps=10, devices=4, queue_cap=3)]
    bt = BT.Batch(streams, threads=64, margin=0.05, floor=16, lib_path=sim_lib)
    info = bt.size(window=5)
    assert sum(info.values()) >= 1
    bt.launch()
    prog = bt.progress()
    assert (prog[:, 2] == 0).all() and (prog[:, 3] == 1).all()
    for s, ctx in zip(streams, bt.contexts):
        assert ctx.sync() == 0
        assert_same(oracle.run_stream(s), ctx.fetch_all(), "batch:" + s.name)
    bt.close()


def test_sim_windowed_batch_matches_oracle(sim_lib):
    """Launches bounded to a few commands per stream give the same graphs."""
    from paper_2503_10516_amd import batch as BT
    streams = [S.stencil_1d(n=128, tasks=9), S.random_small(5), S.nbody_example()]
    bt = BT.Batch(streams, threads=64, lib_path=sim_lib)
    seen = []
    prog = bt.analyse(range(len(streams)), window=4, log=lambda k, n, p: seen.append(n))
    assert len(seen) > 3 and (prog[:, 2] == 0).all()
    assert list(prog[:, 5]) == [len(s.cmds) for s in streams]
    for s, ctx in zip(streams, bt.contexts):
        assert ctx.sync() == 0
        assert_same(oracle.run_stream(s), ctx.fetch_all(), "window:" + s.name)
    bt.close()


DIGESTS = ("n_instructions", "n_bindings", "n_edges", "digest_instructions", "digest_bindings", "digest_edges")


def test_sim_serving_mix_equals_each_session_alone(sim_lib):
    """Continuous batching: sessions admitted into 2 slots as they free up,
    tasks arriving over time; every session's graph equals its oracle graph
    (which is also what it gives alone)."""
    from paper_2503_10516_amd import serve
    sessions = [S.stencil_1d(n=128, tasks=10), S.nbody_example(), S.growing(width=12, steps=8, devices=4, queue_cap=2),
                S.random_small(3), S.stencil_1d(n=64, tasks=6, lookahead=0)]
    out = serve.Server(slots=2, threads=64, lib_path=sim_lib).run(sessions, rate=2e3)
    assert out["tasks"] == sum(s.n_tasks for s in sessions)
    assert out["launches"] >= 2
    for s, st in zip(sessions, out["session_stats"]):
        want = oracle.run_stream(s, fetch=False)["stats"]
        alone = B.run_stream(s, lib_path=sim_lib, threads=64, fetch=False)["stats"]
        for k in DIGESTS:
            assert st[k] == want[k] == alone[k], (s.name, k)
    assert out["p99_latency_us"] >= out["p50_latency_us"] > 0


def test_sim_server_admission_busy_and_detach(sim_lib):
    """ig_server_*: a full server answers IG_E_BUSY, as does one whose arena
    budget a session would exceed; a session covered by a queued launch
    cannot be detached; detached sessions equal the oracle."""
    srv = B.Server(1, threads=64, lib_path=sim_lib)
    a, b = S.stencil_1d(n=128, tasks=6), S.nbody_example()
    sa = srv.admit(a, threads=64)
    assert sa == 0 and srv.admit(b, threads=64) is None
    ca = srv.context(sa)
    for c in a.cmds:
        ca.record_command(c)
    prog = srv.poll()
    assert len(prog) == 1 and prog[0].slot == 0 and prog[0].in_flight == 1
    assert srv.detach(sa) is None  # the queued launch still covers it
    prog = srv.poll()
    assert prog[0].in_flight == 0 and prog[0].finished == 1 and prog[0].tasks_done == a.n_tasks
    assert prog[0].commands_done == prog[0].commands_recorded == len(a.cmds)
    da = srv.detach(sa)
    assert da is not None and srv.poll() == []
    assert_same(oracle.run_stream(a), da.fetch_all(), "server:" + a.name)
    da.close()
    sb = srv.admit(b, threads=64)  # the slot is free again
    assert sb == 0
    srv.close()
    # budget: one arena fits, a second does not
    one = B.Server(4, threads=64, lib_path=sim_lib)
    import ctypes as ct
    d, _, _ = B.context_desc(one.L, "host", None, threads=64, **a.desc(), **B.estimate_caps(a))
    need = ct.c_uint64()
    assert one.L.ig_arena_bytes(ct.byref(d), ct.byref(need)) == 0
    one.close()
    srv = B.Server(4, threads=64, arena_budget=int(need.value * 1.5), lib_path=sim_lib)
    assert srv.admit(a, threads=64, **B.estimate_caps(a)) is not None
    assert srv.admit(a, threads=64, **B.estimate_caps(a)) is None
    srv.close()


@pytest.mark.parametrize("variant", range(4))
def test_sim_reader_runs(variant, sim_lib):
    s = reader_run_stream(variant)
    assert_same(oracle.run_stream(s), B.run_stream(s, lib_path=sim_lib, threads=64), s.name)


@pytest.mark.parametrize("variant,threads", [(0, 64), (1, 64), (2, 64), (3, 64), (0, 256), (1, 256)])
def test_sim_big_reads(variant, threads, sim_lib):
    """Large read regions scanned by thread teams equal the oracle's
    sequential consumer split."""
    s = big_read_stream(variant)
    assert_same(oracle.run_stream(s), B.run_stream(s, lib_path=sim_lib, threads=threads), s.name)


@pytest.mark.parametrize("seed", range(12))
def test_sim_task_graph_horizons(seed, sim_lib):
    """Horizons from the task graph (horizon mode 1, Sec. 3.5) in the kernel
    equal the oracle's, record by record."""
    from test_oracle_semantics import tdag_stream
    s = tdag_stream(seed)
    assert_same(oracle.run_stream(s), B.run_stream(s, lib_path=sim_lib, threads=64), s.name)


@pytest.mark.parametrize("index", [0, 3, 7])
def test_sim_batched_generator_streams(index, sim_lib):
    s = S.batched_stream(S.BATCHED_SEED, index, max_tasks=60, max_log_chunks=6, max_log_extent=12)
    assert_same(oracle.run_stream(s), B.run_stream(s, lib_path=sim_lib, threads=64), s.name)


def test_sim_copies_with_many_sources_on_all_threads(sim_lib):
    """Copies of one task are emitted by every thread of the workgroup, not
    only by the memory workers; copies whose destination cells carry runs of
    readers have more sources than the register set holds and stage them
    through per-thread scratch (sized for every thread)."""
    s = S.nbody(n=4096, steps=3, nodes=1, devices=2, chunks=64)
    assert_same(oracle.run_stream(s), B.run_stream(s, lib_path=sim_lib, threads=64), s.name)


@pytest.mark.parametrize("cap,lookahead", [(0, 1), (1, 1), (3, 1), (8, 1), (0, 0)])
def test_sim_growing_reader_lists(cap, lookahead, sim_lib):
    """Rows read by every later task: reader lists grow and are compacted
    (readers before the last epoch dropped, those before the sync point kept
    as one entry) while grid refinement copies them."""
    s = S.growing(width=24, steps=48, devices=4, queue_cap=cap, lookahead=lookahead)
    assert_same(oracle.run_stream(s), B.run_stream(s, lib_path=sim_lib, threads=64), s.name)


def test_bench_refuses_more_than_one_gpu():
    r = subprocess.run(["python3", os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True, text=True,
                       timeout=120)
    assert r.returncode == 2 and "exactly one GPU" in r.stdout


def test_sim_progress_noalloc_equals_progress(sim_lib):
    """ig_batch_progress_noalloc (fixed scratch) reports what
    ig_batch_progress reports, on two calls in a row, the second over fewer
    contexts; more than its maximum is refused."""
    streams = [S.stencil_1d(n=256, tasks=17), S.nbody_example(), S.random_small(3), S.growing(width=12, steps=6,
                                                                                             devices=4)]
    ctxs = []
    for s in streams:
        ctx = B.make_context(s, lib_path=sim_lib, threads=64)
        ctx.record(S.Stream(s.nodes, s.devices, s.chunks, cmds=s.cmds[: len(s.cmds) // 2]))
        ctxs.append(ctx)
    B.batch_flush(ctxs)
    for sub in (ctxs, ctxs[1:3]):
        want = B.batch_progress(sub)
        got = B.batch_progress(sub, noalloc=True)
        assert want.shape == got.shape == (len(sub), 6)
        assert (want == got).all(), (want, got)
    too_many = (ctypes.c_void_p * 4097)(*([ctxs[0].h] * 4097))
    out = (B.Progress * 4097)()
    assert ctxs[0].L.ig_batch_progress_noalloc(too_many, 4097, None, ctypes.cast(out, ctypes.c_void_p)) == \
        B.IG_E_CAPACITY
    for c in ctxs:
        c.close()


def _ooo_streams():
    from test_oracle_semantics import tdag_stream
    return [S.nbody_example(), S.stencil_1d(n=256, tasks=24), S.nbody(n=64, steps=3, nodes=2, devices=2, chunks=8),
            S.random_small(3), tdag_stream(5), S.growing(width=24, steps=16, devices=4)]


def test_sim_ooo_engine_equals_oracle(sim_lib):
    """The engine kernel (one emulated workgroup per graph, all graphs in one
    launch) assigns every instruction to the lane, at the moments, the
    oracle's engine does, under each parameter set."""
    streams = _ooo_streams()
    ctxs = []
    for s in streams:
        ctx = B.make_context(s, lib_path=sim_lib, threads=64)
        ctx.record(s)
        ctx.flush()
        assert ctx.sync() == 0
        ctxs.append(ctx)
    try:
        outs = [oracle.run_stream(s) for s in streams]
        for kw in OOO_PARAMS:
            ooo_against_oracle(streams, ctxs, kw, outs)
    finally:
        for c in ctxs:
            c.close()


def test_sim_ooo_rejects_bad_parameters_and_lanes(sim_lib):
    s = S.nbody_example()
    ctx = B.make_context(s, lib_path=sim_lib, threads=64)
    ctx.record(s)
    ctx.flush()
    assert ctx.sync() == 0
    try:
        for kw in (dict(window=0), dict(window=4097), dict(lanes_per_device=0), dict(host_lanes=0), dict(eager=2),
                   dict(kernel_ns=0), dict(lanes_per_device=600)):
            with pytest.raises(B.IgError):
                B.OooSimulation([ctx], B.ooo_params(2, **kw))
        # too few device lanes for the graph's memories: the graph's status
        sim = B.OooSimulation([ctx], B.ooo_params(1))
        sim.run()
        with pytest.raises(B.IgError) as e:
            sim.fetch(0)
        assert e.value.status == B.IG_E_INVALID
        sim.close()
    finally:
        ctx.close()


@pytest.mark.parametrize("index", range(8))
def test_sim_staged_copies_equal_oracle(index, sim_lib):
    """Device-to-device copies staged through pinned host memory (Sec. 3.3,
    last paragraph): the kernel's pairs, ids and edges equal the oracle's."""
    import dataclasses
    from test_oracle_staging import cases
    picks = [0, 2, 3, 4, 5, 7, 22, 26]
    s = cases()[picks[index]]
    s = dataclasses.replace(s, staging=1, name=s.name + "_staged")
    assert_same(oracle.run_stream(s), B.run_stream(s, lib_path=sim_lib, threads=64 if index % 2 else 256), s.name)


def test_sim_staged_big_reads(sim_lib):
    """Staging with large reads scanned by thread teams (the deferred path)."""
    import dataclasses
    s = dataclasses.replace(big_read_stream(1), staging=1)
    assert_same(oracle.run_stream(s), B.run_stream(s, lib_path=sim_lib, threads=256), s.name)
