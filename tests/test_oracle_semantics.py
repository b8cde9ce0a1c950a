"""The oracle against per-element brute force, and mutation tests of the pins.

Every stream here is tiny; `bruteforce.check_stream` executes the emitted
graph element by element (sequential semantics, race freedom, coherence,
allocation, resize and front invariants, exact edge sets, the command
queue).  The mutation tests plant plausible mistakes in a copy of the
oracle's source (on the CPU) and require a hand-worked pin or a brute-force
check to reject each one.
"""
import ctypes
import os
import subprocess
import tempfile

import pytest

import oracle
from bruteforce import Failure, check_stream
from paper_2503_10516_amd import streams as S

SCENARIOS = [
    ("stencil1d", lambda: S.stencil_1d(n=64, tasks=12)),
    ("stencil1d_nola", lambda: S.stencil_1d(n=64, tasks=12, lookahead=0)),
    ("stencil2d", lambda: S.stencil_2d(side=12, tasks=9, nodes=2, devices=2, chunks=4)),
    ("nbody_example", S.nbody_example),
    ("nbody_small", lambda: S.nbody(n=24, steps=4, nodes=2, devices=2, chunks=8)),
    ("resize0", lambda: S.resize_example(0, 8, 8)),
    ("resize1", lambda: S.resize_example(1, 8, 8)),
    ("growing", lambda: S.growing(width=12, steps=8, devices=4)),
    ("growing_nola", lambda: S.growing(width=12, steps=8, devices=4, lookahead=0)),
    ("growing_cap3", lambda: S.growing(width=12, steps=8, devices=4, queue_cap=3)),
]


@pytest.mark.parametrize("name,make", SCENARIOS, ids=[s[0] for s in SCENARIOS])
def test_scenarios_bruteforce(name, make):
    s = make()
    counts = check_stream(s, oracle.run_stream(s))
    assert counts["kernels"] > 0


@pytest.mark.parametrize("seed", range(80))
def test_random_streams_bruteforce(seed):
    s = S.random_small(seed)
    check_stream(s, oracle.run_stream(s), seed=seed)


def tdag_stream(seed):
    """A random stream with horizons from the task graph (Sec. 3.5); every
    third one caps the tasks between horizons low."""
    s = S.random_small(seed, n_tasks=16)
    s.horizon_mode = 1
    s.horizon_max_tasks = 3 if seed % 3 == 0 else 0
    s.horizon_step = 2 + seed % 3
    s.name += "_tdag"
    return s


@pytest.mark.parametrize("seed", range(40))
def test_random_streams_tdag_horizons_bruteforce(seed):
    """Horizon placement from an explicit element-level task graph, plus
    every other brute-force check, with horizons from the task graph."""
    s = tdag_stream(seed)
    check_stream(s, oracle.run_stream(s), seed=seed)


def test_overlapping_write_rejected_atomically():
    s = S.Stream(1, 2, 2, lookahead=0)
    b = s.buffer(1, (8,), 4, S.INIT_HOST)
    s.task(1, (0,), (8,), [S.Access(b, S.WRITE, S.ONE_TO_ONE)])
    s.task(1, (0,), (8,), [S.Access(b, S.WRITE, S.ALL)])          # both chunks write everything
    s.task(1, (0,), (8,), [S.Access(b, S.READ, S.ALL)])
    s.shutdown()
    out = oracle.run_stream(s)
    assert list(out["status"]) == [0, -2, 0]
    assert out["rcs"][2] == -2
    check_stream(s, out)
    # the rejected task leaves no trace: same graph as without it
    s2 = S.Stream(1, 2, 2, lookahead=0)
    b = s2.buffer(1, (8,), 4, S.INIT_HOST)
    s2.task(1, (0,), (8,), [S.Access(b, S.WRITE, S.ONE_TO_ONE)])
    s2.task(1, (0,), (8,), [S.Access(b, S.READ, S.ALL)])
    s2.shutdown()
    out2 = oracle.run_stream(s2)
    assert out["stats"]["digest_instructions"] != 0
    k1 = [(int(r["kind"]), int(r["mem"]), int(r["src_mem"])) for r in out["instructions"]]
    k2 = [(int(r["kind"]), int(r["mem"]), int(r["src_mem"])) for r in out2["instructions"]]
    assert k1 == k2


def test_invalid_arguments():
    ctx = oracle.OracleContext(1, 2)
    st, b = ctx.buffer_create(2, (4, 4, 1), 4, 1)
    assert st == 0
    bad_dims = S.Task(1, (0, 0, 0), (4, 1, 1), (S.Access(b, S.READ, S.ONE_TO_ONE),))
    assert ctx.submit(bad_dims) == -1
    unknown = S.Task(2, (0, 0, 0), (4, 4, 1), (S.Access(7, S.READ, S.ALL),))
    assert ctx.submit(unknown) == -1
    assert oracle.OracleContext.__init__  # context creation validates the cluster
    with pytest.raises(ValueError):
        oracle.OracleContext(1, 2, chunks=3)
    ctx.close()


# ---------------------------------------------------------------------------
# mutation tests: each mutant must fail a brute-force check
# ---------------------------------------------------------------------------
MUTANTS = {
    "no_anti_edges": ("for (uint32_t r : e.readers) s.add(r, IGO_DEP_ANTI);", ";"),
    "no_true_edges": ("s.add(e.writer, is_alloc(e.writer) ? IGO_DEP_LIFETIME : IGO_DEP_TRUE);", ";"),
    "copy_even_if_up_to_date": ("e.mask.none() || e.mask.test(m)", "e.mask.none()"),
    "no_consumer_split_update": ("mask_add(b, cb, m);", ";"),
    "kernel_write_not_recorded": ("buffer_assign(rg.buffer, rg.box, ki, m);", ";"),
    "no_resize_copy": ("if (e.mask.test(m)) {\n                            Box in", "if (false) {\n                            Box in"),
    "free_ignores_readers": ("for (uint32_t r : e.readers) s.add(r, IGO_DEP_LIFETIME);", ";"),
    "horizon_misses_front": ("for (uint32_t f : front) s.add(f, IGO_DEP_SYNC);\n        finish(hi, s);",
                              "if (!front.empty()) s.add(*front.begin(), IGO_DEP_SYNC);\n        finish(hi, s);"),
    "no_sync_fallback": ("if (s.from.empty()) s.add(sync_point, IGO_DEP_SYNC);", ";"),
    # task-graph horizons (horizon_mode 1)
    "tdag_write_ignores_readers": ("if (rg.mode & IGO_WRITE) d = std::max(d, e.rcp > cp_epoch ? eff(e.rcp) : eff(e.wcp));",
                                   "if (rg.mode & IGO_WRITE) d = std::max(d, eff(e.wcp));"),
    "tdag_reads_not_recorded": ("in.rcp = std::max(in.rcp > cp_epoch ? in.rcp : 0u, cp);", ";"),
    "tdag_horizon_late": ("c->cp_last = c->cp_max;", "c->cp_last = c->cp_max + 1;"),
    "tdag_pending_not_applied": ("if (c->cp_pending) c->cp_sync = c->cp_pending;", ";"),
    "tdag_cap_off_by_one": ("++c->tasks_since_sync >= c->horizon_max_tasks", "++c->tasks_since_sync > c->horizon_max_tasks"),
    "no_overlap_check": ("if (v[i].second != v[j].second && intersects(v[i].first, v[j].first)) {",
                         "if (false) {"),
    "producer_split_off": ("groups[std::make_tuple(e.pm, e.producer, a)]", "groups[std::make_tuple(e.pm, 0u, a)]"),
    "split_off_by_one": ("c.hi[0] = s + floor_part(e - s, u + 1, per_dev);",
                         "c.hi[0] = s + floor_part(e - s, u + 1, per_dev) + (u + 1 < per_dev ? 1 : 0);"),
    "neighborhood_one_sided": ("r.hi[d] = chunk.hi[d] + a.radius[d];", "r.hi[d] = chunk.hi[d];"),
    "horizon_substitutes_readers_too_far": ("if (r < p) r = p;", "r = p;"),
    "uninit_not_tracked": ("for (const Box& p : subtract_all({rg.box}, bf.initialised)) bf.initialised.push_back(p);",
                           ";"),
    # edges from map entries outside the accessed region
    "edges_ignore_region": ("if (!intersects(e.box, a.box)) continue;", ";"),
    # an OUTPUT edge from the writer even when readers take ANTI edges
    "output_with_anti": ("} else {\n                        s.add(e.writer, is_alloc(e.writer) ? IGO_DEP_LIFETIME : "
                         "IGO_DEP_OUTPUT);\n                    }",
                         "}\n                    s.add(e.writer, is_alloc(e.writer) ? IGO_DEP_LIFETIME : "
                         "IGO_DEP_OUTPUT);"),
    # the allocating predicate ignores the plan of queued commands
    "allocating_vs_live_only": ("std::vector<Box> v = (!queue.empty() && it != plan.end()) ? it->second : "
                                "live_boxes(r.buffer, r.mem);",
                                "std::vector<Box> v = live_boxes(r.buffer, r.mem);\n            (void)it;"),
    # a resize copies the whole old allocation, up to date or not
    "resize_copies_whole_box": ("if (e.mask.test(m)) {\n                            Box in",
                                "if (true) {\n                            Box in"),
    # copy groups in descending (producer memory, producer, source) order
    "group_order_reversed": ("std::map<std::tuple<uint16_t, uint32_t, uint32_t>, std::vector<Box>> groups;",
                             "std::map<std::tuple<uint16_t, uint32_t, uint32_t>, std::vector<Box>,\n"
                             "                         std::greater<std::tuple<uint16_t, uint32_t, uint32_t>>> groups;"),
}


def _group_order_pin():
    from test_oracle_scenarios import check_group_order, group_order_stream
    check_group_order(oracle.run_stream(group_order_stream()))


# hand-worked pins that are run against every mutant before the streams
PIN_CASES = [_group_order_pin]

def _overlap_stream():
    s = S.Stream(1, 2, 2, lookahead=0)
    b = s.buffer(1, (8,), 4, S.INIT_HOST)
    s.task(1, (0,), (8,), [S.Access(b, S.WRITE, S.ALL)])
    s.task(1, (0,), (8,), [S.Access(b, S.READ, S.ALL)])
    s.shutdown()
    return s


MUTANT_STREAMS = [_overlap_stream()] + [S.random_small(seed) for seed in range(40)] + \
    [tdag_stream(seed) for seed in range(24)] + [
    S.nbody(n=24, steps=4, nodes=2, devices=2, chunks=8),
    S.stencil_2d(side=12, tasks=9, nodes=2, devices=2, chunks=4),
    S.growing(width=12, steps=8, devices=4, lookahead=0),
    S.nbody_example(),
]


def _build_mutant(name, tmpdir):
    src = open(os.path.join(os.path.dirname(oracle.__file__), "ig_oracle.cpp")).read()
    old, new = MUTANTS[name]
    assert old in src, f"mutation site of {name} not found"
    mutated = src.replace(old, new, 1)
    path = os.path.join(tmpdir, f"{name}.cpp")
    with open(path, "w") as f:
        f.write(mutated)
    inc = os.path.dirname(oracle.__file__)
    so = os.path.join(tmpdir, f"lib{name}.so")
    subprocess.check_call(["g++", "-O1", "-std=c++17", "-shared", "-fPIC", "-I", inc, "-o", so, path])
    return so


@pytest.fixture(scope="module")
def mutant_dir():
    with tempfile.TemporaryDirectory() as d:
        yield d


@pytest.mark.parametrize("name", sorted(MUTANTS))
def test_mutant_is_caught(name, mutant_dir):
    so = _build_mutant(name, mutant_dir)
    saved_lib, saved_path = oracle._lib, oracle.LIB_PATH
    try:
        oracle._lib = None
        oracle.LIB_PATH = so
        caught = False
        for pin in PIN_CASES:
            try:
                pin()
            except AssertionError:
                caught = True
                break
        for s in [] if caught else MUTANT_STREAMS:
            try:
                check_stream(s, oracle.run_stream(s), n_random_orders=0)
            except (Failure, IndexError, KeyError):
                caught = True
                break
        assert caught, f"mutant {name} passed every brute-force check"
    finally:
        oracle._lib, oracle.LIB_PATH = saved_lib, saved_path


@pytest.mark.parametrize("seed", range(0, 80, 4))
def test_algorithmic_byte_terms(seed):
    """The R17 counters equal what the records show: one writer update per
    ALLOC, COPY and kernel write; one reader insertion per COPY and kernel
    read; one buffer-map update per coherence COPY and kernel write; one
    mapper box per non-empty chunk and accessor."""
    from bruteforce import map_py, split_py, box_empty
    s = S.random_small(seed) if seed % 8 else S.nbody(n=24, steps=4, nodes=2, devices=2, chunks=8)
    out = oracle.run_stream(s)
    ins, binds = out["instructions"], out["bindings"]
    kind = ins["kind"]
    n_alloc = int((kind == oracle.ALLOC).sum())
    n_copy = int((kind == oracle.COPY).sum())
    n_resize = int(((kind == oracle.COPY) & ((ins["flags"] & oracle.F_RESIZE) != 0)).sum())
    tasks = [c[1] for c in s.cmds if c[0] == "task"]
    kw = kr = 0
    for b in binds:
        if int(b["alloc"]) == 0:
            continue
        mode = tasks[int(ins[int(b["instr"])]["task"])].accesses[int(b["access"])].mode
        kw += bool(mode & S.WRITE)
        kr += bool(mode & S.READ)
    boxes = 0
    for t in tasks:
        for ch in split_py(s.nodes, s.devices, s.chunks, t.lo, t.hi):
            if not box_empty(ch):
                boxes += len(t.accesses)
    st = out["stats"]
    assert st["u_w"] == n_alloc + n_copy + kw
    assert st["u_r"] == n_copy + kr
    assert st["u_b"] == n_copy - n_resize + kw
    assert st["map_boxes"] == boxes
