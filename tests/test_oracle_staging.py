"""Host-staged device-to-device copies (the closing paragraph of Sec. 3.3)
in the oracle, pinned to the direct-copy graph, which the other pins fix.

With staging, a coherence copy between two devices of one node becomes a
copy from the source device into pinned host memory M1 followed by a copy
from M1 into the destination device.  Pins:
  * contracting every such pair back into one copy gives exactly the graph
    of the same stream without staging (records, bindings, statuses; edges
    with their kinds, the pair's own edge dropped and parallel edges merged);
  * each pair is the two consecutive instructions the definition says, the
    second depending on the first by a true dependency, and each half's other
    dependencies touch only its own side: the first half's only instructions
    on the source memory (or horizons and epochs), the second half's only
    instructions on or reading from the destination memory.
"""
import dataclasses

import numpy as np
import pytest

import oracle
from paper_2503_10516_amd import streams as S

NONE16 = 0xFFFF


def staged(s):
    return dataclasses.replace(s, staging=1, name=s.name + "_staged")


def pairs(ins):
    """Indices i of the first halves (copies into M1) of staging pairs."""
    first = np.nonzero((ins["kind"] == oracle.COPY) & (ins["mem"] == 1))[0]
    return first


def contract(out):
    """The staged graph with each pair merged into one copy, ids renumbered."""
    ins, ed = out["instructions"], out["edges"]
    n = len(ins)
    is_second = np.zeros(n, dtype=bool)
    first = pairs(ins)
    is_second[first + 1] = True
    new_id = np.cumsum(~is_second) - 1  # a second half maps to its first half's id
    keep = ~is_second
    merged = ins[keep].copy()
    merged["id"] = np.arange(keep.sum(), dtype=np.uint64)
    for i in first:
        j = new_id[i]
        a, b = ins[i], ins[i + 1]
        merged[j]["mem"] = b["mem"]
        merged[j]["alloc"] = b["alloc"]
        merged[j]["src_mem"] = a["src_mem"]
        merged[j]["src_alloc"] = a["src_alloc"]
    # edges: remap, drop the pairs' own edges, merge parallel ones
    e = {}
    for f, t, k in zip(ed["from"], ed["to"], ed["kinds"]):
        nf, nt_ = int(new_id[f]), int(new_id[t])
        if nf == nt_:
            continue
        e[(nt_, nf)] = e.get((nt_, nf), 0) | int(k)
    edges = np.zeros(len(e), dtype=ed.dtype)
    for q, ((t, f), k) in enumerate(sorted(e.items())):
        edges[q]["from"], edges[q]["to"], edges[q]["kinds"] = f, t, k
    b = out["bindings"].copy()
    b["instr"] = new_id[b["instr"].astype(np.int64)]
    return merged, b, edges


def cases():
    out = [S.nbody_example(), S.stencil_1d(n=256, tasks=24), S.nbody(n=64, steps=3, nodes=2, devices=2, chunks=8),
           S.nbody(n=4096, steps=3, nodes=1, devices=4, chunks=16), S.growing(width=24, steps=16, devices=4),
           S.stencil_2d(side=64, tasks=12, nodes=2, devices=2, chunks=8)]
    out += [S.random_small(seed) for seed in range(16)]
    out += [S.random_small(seed, race_free=False) for seed in range(4)]
    out += [S.batched_stream(S.BATCHED_SEED, i, max_tasks=60, max_log_chunks=6, max_log_extent=12) for i in range(4)]
    return out


@pytest.mark.parametrize("s", cases(), ids=lambda s: s.name)
def test_staged_graph_contracts_to_the_direct_graph(s):
    direct = oracle.run_stream(s)
    st = oracle.run_stream(staged(s))
    ins, b, ed = contract(st)
    assert ins.tobytes() == direct["instructions"].tobytes()
    assert b.tobytes() == direct["bindings"].tobytes()
    assert ed.tobytes() == direct["edges"].tobytes()
    assert list(st["status"]) == list(direct["status"])


@pytest.mark.parametrize("s", cases(), ids=lambda s: s.name)
def test_staging_pairs_and_their_sides(s):
    out = oracle.run_stream(staged(s))
    ins, ed = out["instructions"], out["edges"]
    deps = {}
    for f, t, k in zip(ed["from"], ed["to"], ed["kinds"]):
        deps.setdefault(int(t), {})[int(f)] = int(k)
    n_pairs = 0
    for i in pairs(ins):
        a, b = ins[i], ins[i + 1]
        n_pairs += 1
        # the pair: device -> M1, then M1 -> device of the same node, same box
        assert a["src_mem"] >= 2 and a["alloc"] == 0 and a["flags"] == 0
        assert b["kind"] == oracle.COPY and b["src_mem"] == 1 and b["mem"] >= 2 and b["src_alloc"] == 0
        nodes_of = lambda m: (int(m) - 2) // s.devices
        assert nodes_of(a["src_mem"]) == nodes_of(b["mem"]) and a["src_mem"] != b["mem"]
        assert (a["min"] == b["min"]).all() and (a["max"] == b["max"]).all()
        assert (a["task"], a["chunk"], a["buffer"]) == (b["task"], b["chunk"], b["buffer"])
        assert deps[int(i) + 1].get(int(i)) == oracle.DEP_TRUE
        src, dst = int(a["src_mem"]), int(b["mem"])
        for f in deps.get(int(i), {}):
            r = ins[f]
            assert r["mem"] == src or r["kind"] in (oracle.HORIZON, oracle.EPOCH), (s.name, i, f)
        for f in deps[int(i) + 1]:
            if f == i:
                continue
            r = ins[f]
            assert r["mem"] == dst or r["src_mem"] == dst or r["kind"] in (oracle.HORIZON, oracle.EPOCH), \
                (s.name, i + 1, f)
    # no copy into M1 other than staging pairs, and no staging across nodes
    assert not ((ins["kind"] == oracle.COPY) & (ins["src_mem"] == 1) & (ins["mem"] >= 2) &
                (ins["src_alloc"] == 0)).sum() > n_pairs
    inter = (ins["flags"] & oracle.F_INTER_NODE) != 0
    assert (ins["mem"][inter] >= 2).all() and (ins["src_mem"][inter] >= 2).all()


def test_staging_changes_only_device_to_device_copies_within_a_node():
    """Two devices on one node exchange halves of a buffer: every one of
    their copies is staged; with two nodes of one device each, none is."""
    for nodes, devices, want_staged in ((1, 2, True), (2, 1, False)):
        s = S.nbody(n=64, steps=2, nodes=nodes, devices=devices, chunks=2)
        d = oracle.run_stream(s)["instructions"]
        st = oracle.run_stream(staged(s))["instructions"]
        dev_copies = ((d["kind"] == oracle.COPY) & (d["src_mem"] >= 2)).sum()
        assert dev_copies > 0
        if want_staged:
            assert len(pairs(st)) == dev_copies and len(st) == len(d) + dev_copies
        else:
            assert len(pairs(st)) == 0 and st.tobytes() == d.tobytes()


# Plausible mistakes in the staged path, planted in copies of the oracle:
# each must fail one of the pins above.
STAGING_MUTANTS = {
    "first_half_without_source_edges": ("                            access_edges(a1, s1);\n", "\n"),
    "second_half_without_pair_edge": ("                            s2.add(c1, IGO_DEP_TRUE);\n", "\n"),
    "staged_across_nodes": ("staging && src_mem >= 2 && !(flags & IGO_F_INTER_NODE)", "staging && src_mem >= 2"),
    "destination_edges_on_first_half": ("                            access_edges(a2, s2);\n",
                                        "                            access_edges(a2, s1);\n"),
    "source_read_not_recorded": ("                            access_apply(c1, a1);\n", "\n"),
}


@pytest.mark.parametrize("name", sorted(STAGING_MUTANTS))
def test_staging_mutant_is_caught(name, tmp_path):
    import os
    import subprocess
    src = open(os.path.join(os.path.dirname(oracle.__file__), "ig_oracle.cpp")).read()
    old, new = STAGING_MUTANTS[name]
    assert old in src, name
    path = tmp_path / f"{name}.cpp"
    path.write_text(src.replace(old, new, 1))
    so = str(tmp_path / f"lib{name}.so")
    subprocess.check_call(["g++", "-O1", "-std=c++17", "-shared", "-fPIC", "-I", os.path.dirname(oracle.__file__),
                           "-o", so, str(path)])
    saved_lib, saved_path = oracle._lib, oracle.LIB_PATH
    caught = False
    try:
        oracle._lib = None
        oracle.LIB_PATH = so
        for s in cases():
            try:
                test_staged_graph_contracts_to_the_direct_graph(s)
                test_staging_pairs_and_their_sides(s)
            except AssertionError:
                caught = True
                break
    finally:
        oracle._lib, oracle.LIB_PATH = saved_lib, saved_path
    assert caught, f"mutant {name} passes every staging pin"
