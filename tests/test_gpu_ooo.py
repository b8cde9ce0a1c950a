"""The out-of-order engine simulation (Sec. 4.1) on the GPU against the
oracle's engine: every slot (lane, kind of assignment, issue, start, end)
and the summary, bit for bit, over graphs the HIP path generated (which
equal the oracle's, checked elsewhere).  At full size, where the oracle's
engine would take hours, the properties that hold for any correct run are
checked instead."""
import hashlib
import json
import os

import numpy as np
import pytest

import oracle
from parity import OOO_PARAMS, ooo_against_oracle
from paper_2503_10516_amd import binding as B
from paper_2503_10516_amd import streams as S

pytestmark = pytest.mark.gpu
NONE32 = 0xFFFFFFFF


@pytest.fixture(scope="module", autouse=True)
def _device():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    torch.cuda.set_device(0)


def _contexts(streams):
    ctxs = []
    for s in streams:
        ctx = B.make_context(s)
        ctx.record(s)
        ctx.flush()
        assert ctx.sync() == 0, s.name
        ctxs.append(ctx)
    return ctxs


def _streams():
    from test_oracle_semantics import tdag_stream
    out = [S.nbody_example(), S.stencil_1d(n=256, tasks=24), S.nbody(n=64, steps=3, nodes=2, devices=2, chunks=8),
           S.growing(width=24, steps=16, devices=4), S.stencil_1d(), S.nbody(n=4096, steps=3, nodes=1, devices=2,
                                                                              chunks=64)]
    out += [S.random_small(seed) for seed in range(12)]
    out += [tdag_stream(seed) for seed in range(4)]
    out += [S.batched_stream(S.BATCHED_SEED, i, max_tasks=60, max_log_chunks=6, max_log_extent=12) for i in range(6)]
    return out


@pytest.mark.parametrize("kw", OOO_PARAMS, ids=[f"p{i}" for i in range(len(OOO_PARAMS))])
def test_ooo_engine_equals_oracle(kw):
    streams = _streams()
    print(f"[gpu] ooo parity {kw} over {len(streams)} graphs", flush=True)
    ctxs = _contexts(streams)
    try:
        ooo_against_oracle(streams, ctxs, kw)
    finally:
        for c in ctxs:
            c.close()


def test_ooo_two_runs_and_rebuilt_handle():
    """A handle runs twice with equal results; a handle created after the
    contexts are re-analysed sees the same graphs."""
    streams = _streams()[:6]
    ctxs = _contexts(streams)
    try:
        sim = B.OooSimulation(ctxs, B.ooo_params(4))
        sim.run()
        first = [sim.fetch(i) for i in range(len(ctxs))]
        sim.run()
        for i in range(len(ctxs)):
            got, summ = sim.fetch(i)
            assert got.tobytes() == first[i][0].tobytes() and summ == first[i][1]
        sim.close()
        for c in ctxs:
            c.rewind()
            c.flush()
            assert c.sync() == 0
        sim = B.OooSimulation(ctxs, B.ooo_params(4))
        sim.run()
        for i in range(len(ctxs)):
            got, summ = sim.fetch(i)
            assert got.tobytes() == first[i][0].tobytes() and summ == first[i][1]
        sim.close()
    finally:
        for c in ctxs:
            c.close()


def check_engine_properties(ins, edges, slots, summ, p, devices_lanes):
    """What holds for any run of the engine (see the oracle's pins)."""
    n = len(ins)
    kinds = ins["kind"]
    vol = np.prod(np.maximum(ins["max"].astype(np.int64) - ins["min"].astype(np.int64), 0), axis=1).astype(np.uint64)
    dur = np.zeros(n, dtype=np.uint64)
    k = kinds == B.IG_KERNEL
    dur[k] = np.uint64(p.kernel_ns) + vol[k] * np.uint64(p.kernel_ns_per_kelem) // np.uint64(1024)
    c = kinds == B.IG_COPY
    dur[c] = np.uint64(p.copy_ns) + vol[c] * np.uint64(p.copy_ns_per_kelem) // np.uint64(1024) + \
        np.where((ins["flags"][c] & B.IG_F_INTER_NODE) != 0, p.inter_node_ns, 0).astype(np.uint64)
    dur[kinds == B.IG_ALLOC] = p.alloc_ns
    dur[kinds == B.IG_FREE] = p.free_ns
    assert (slots["end"] - slots["start"] == dur).all()
    assert (slots["start"] >= slots["issue"]).all()
    f = edges["from"].astype(np.int64)
    t = edges["to"].astype(np.int64)
    assert (slots["start"][t] >= slots["end"][f]).all()
    how = slots["how"][t]
    direct = how != B.IG_OOO_EAGER
    assert (slots["end"][f][direct] <= slots["issue"][t][direct]).all()
    open_ = (~direct) & (slots["end"][f] > slots["issue"][t])
    assert (slots["lane"][f][open_] == slots["lane"][t][open_]).all()
    lanes = slots["lane"]
    on = lanes != NONE32
    order = np.lexsort((slots["end"][on], slots["start"][on], lanes[on]))
    l, s, e = lanes[on][order], slots["start"][on][order], slots["end"][on][order]
    same = l[1:] == l[:-1]
    assert (s[1:][same] >= e[:-1][same]).all()
    dev = (kinds == B.IG_KERNEL) | ((kinds == B.IG_COPY) & (ins["mem"] >= 2))
    assert (lanes[dev] // p.lanes_per_device == ins["mem"][dev] - 2).all()
    eng = (kinds == B.IG_HORIZON) | (kinds == B.IG_EPOCH)
    assert (lanes[eng] == NONE32).all() and (slots["start"][eng] == slots["issue"][eng]).all()
    assert (lanes[on] < devices_lanes + p.host_lanes).all()
    assert summ["makespan"] == int(slots["end"].max())
    assert summ["direct"] == int((slots["how"] == B.IG_OOO_DIRECT).sum())
    assert summ["eager"] == int((slots["how"] == B.IG_OOO_EAGER).sum())


def test_ooo_full_size_stencil2d_properties():
    s = S.stencil_2d()
    print(f"[gpu] ooo stencil2d full: {s.n_tasks} tasks", flush=True)
    ctx = _contexts([s])[0]
    try:
        out = ctx.fetch_all()
        for kw in (dict(), dict(window=64, eager=0), dict(lanes_per_device=1, host_lanes=1, window=4096)):
            p = B.ooo_params(s.nodes * s.devices, **kw)
            sim = B.OooSimulation([ctx], p)
            sim.run()
            slots, summ = sim.fetch(0)
            sim.close()
            check_engine_properties(out["instructions"], out["edges"], slots, summ, p, s.nodes * s.devices *
                                    p.lanes_per_device)
    finally:
        ctx.close()


def test_ooo_full_size_stencil2d_against_oracle_golden():
    """Every slot of the engine over the full 2-D stencil's graph equals the
    oracle's (stored by tests/golden/make_golden.py: SHA-256 of all slots,
    the first and last 1000 verbatim, the summary), for two parameter sets."""
    here = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")
    gold = json.load(open(os.path.join(here, "stencil2d_full_ooo.json")))
    keep = np.load(os.path.join(here, "stencil2d_full_ooo_slots.npz"))
    s = S.stencil_2d()
    print("[gpu] ooo stencil2d full against the oracle golden", flush=True)
    ctx = _contexts([s])[0]
    try:
        for j, run in enumerate(gold["runs"]):
            sim = B.OooSimulation([ctx], B.ooo_params(gold["devices"], **run["params"]))
            sim.run()
            slots, summ = sim.fetch(0)
            sim.close()
            assert summ == run["summary"], (run["params"], summ)
            want = keep[f"slots{j}"]
            got = np.concatenate([slots[:1000], slots[-1000:]])
            assert got.tobytes() == want.tobytes(), run["params"]
            assert hashlib.sha256(slots.tobytes()).hexdigest() == run["slots_sha256"], run["params"]
    finally:
        ctx.close()


def _analysed(s):
    """A context holding s's graph (capacities grown on overflow)."""
    from paper_2503_10516_amd import batch as BT
    caps = B.estimate_caps(s)
    caps.update(BT.fixed_caps(s))
    for _ in range(4):
        ctx = B.make_context(s, **caps)
        ctx.record(s)
        ctx.flush()
        st = ctx.sync()
        if st == B.IG_E_CAPACITY:
            ctx.close()
            for k in ("cap_instructions", "cap_edges", "cap_state_words", "cap_unit", "cap_scratch"):
                caps[k] = int(caps[k] * 3)
            continue
        assert st == 0, (s.name, st)
        return ctx
    raise AssertionError(f"{s.name}: capacities")


@pytest.mark.parametrize("index", [191, 90, 147])
def test_ooo_full_size_batched_graphs_properties(index):
    """The engine over full-size graphs of the batched workload (512-1024
    chunks, 3-4e5 instructions, millions of edges), three at once in one
    launch as in the benchmark: every property of a correct run holds."""
    s = S.batched_stream(S.BATCHED_SEED, index, w_all=S.BATCHED_W_ALL, w_slice=S.BATCHED_W_SLICE)
    print(f"[gpu] ooo batched_{index} full size", flush=True)
    ctx = _analysed(s)
    other = _analysed(S.nbody_example())
    try:
        out = ctx.fetch_all()
        devs = s.nodes * s.devices
        p = B.ooo_params(devs)
        sim = B.OooSimulation([other, ctx], p)
        sim.run()
        slots, summ = sim.fetch(1)
        sim.close()
        check_engine_properties(out["instructions"], out["edges"], slots, summ, p, devs * p.lanes_per_device)
    finally:
        ctx.close()
        other.close()
