"""Write the stored expected values of the large parity cases.

Calls only the oracle (oracle/) on the seeded workloads; the GPU tests and
the benchmark compare the HIP path's counts, per-kind statistics and record
digests with these files, and its first and last records with the stored
ones.  Each document also keeps the oracle's counts of the algorithmic-bytes
terms (writer updates, reader insertions, buffer-map updates, mapper boxes),
which the benchmark's roofline numerator uses.

    python tests/golden/make_golden.py nbody_full growing_q8 ...
    python tests/golden/make_golden.py batched 6      # the 256 batched streams, 6 processes
    python tests/golden/make_golden.py serving 3      # each kind of serving session
    python tests/golden/make_golden.py ooo            # the engine simulation over the 2-D stencil's graph
"""
import json
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

import oracle  # noqa: E402
from paper_2503_10516_amd import streams as S  # noqa: E402

CASES = {
    "stencil1d_full": lambda: S.stencil_1d(),               # 1-D stencil, 4096, 64 tasks, 2 devices
    "nbody_full": lambda: S.nbody(),                       # N-body, 2^20 x 16 B, 500 steps, 16 x 8 devices
    "stencil2d_full": lambda: S.stencil_2d(),               # 2-D stencil, 4096^2, 1000 tasks
    "growing_full": lambda: S.growing(),                    # RSim pattern [84000 x 256], lookahead, unbounded queue
    "growing_nola": lambda: S.growing(lookahead=0),         # no lookahead: a resize per device per step
    "growing_q8": lambda: S.growing(queue_cap=8),           # lookahead window of 8 commands
}

KEEP = 10000  # first and last records of each list stored verbatim (<case>_records.npz)
BATCHED_FILE = "batched_digests.json"
STAT_KEYS = ("n_instructions", "n_bindings", "n_edges", "per_kind", "per_dep", "resizes", "warnings",
             "digest_instructions", "digest_bindings", "digest_edges", "u_w", "u_r", "u_b", "map_boxes")


def head_tail(arr, n):
    return np.concatenate([arr[:n], arr[-n:]]) if len(arr) > 2 * n else arr.copy()


def main(names):
    for name in names:
        s = CASES[name]()
        out = oracle.run_stream(s, fetch=True)
        st = out["stats"]
        doc = {"case": name, "stream": s.name, "oracle_seconds": round(out["seconds"], 2), "keep": KEEP}
        doc.update({k: st[k] for k in STAT_KEYS})
        doc["status"] = [int(x) for x in out["status"]]
        with open(os.path.join(HERE, f"{name}.json"), "w") as f:
            json.dump(doc, f)
        np.savez_compressed(os.path.join(HERE, f"{name}_records.npz"),
                            instructions=head_tail(out["instructions"], KEEP),
                            bindings=head_tail(out["bindings"], KEEP),
                            edges=head_tail(out["edges"], KEEP))
        print(name, st["n_instructions"], st["n_edges"], f"{doc['oracle_seconds']} s", flush=True)


def _batched_one(i):
    s = S.batched_stream(S.BATCHED_SEED, i, w_all=S.BATCHED_W_ALL, w_slice=S.BATCHED_W_SLICE)
    r = oracle.run_stream(s, fetch=False)
    o = r["stats"]
    row = {"index": i, "stream": s.name, "tasks": s.n_tasks, "oracle_seconds": round(r["seconds"], 2)}
    row.update({k: o[k] for k in STAT_KEYS})
    return row


def batched(workers):
    """Oracle statistics and digests of every stream of the batched workload
    (256 streams), computed in parallel worker processes, heaviest first (by
    the stored timing of a previous run, if any) so the pool stays busy."""
    from multiprocessing import Pool
    order = list(range(256))
    try:
        prev = json.load(open(os.path.join(HERE, BATCHED_FILE)))
        secs = {r["index"]: r.get("oracle_seconds", 0) for r in prev["streams"]}
        order.sort(key=lambda i: -secs.get(i, 0))
    except (OSError, ValueError, KeyError):
        pass
    with Pool(workers) as pool:
        rows = []
        for r in pool.imap_unordered(_batched_one, order):
            rows.append(r)
            print(r["index"], r["n_instructions"], r["n_edges"], r["oracle_seconds"], flush=True)
    rows.sort(key=lambda r: r["index"])
    with open(os.path.join(HERE, BATCHED_FILE), "w") as f:
        json.dump({"seed": S.BATCHED_SEED, "w_all": S.BATCHED_W_ALL, "w_slice": S.BATCHED_W_SLICE,
                   "streams": rows}, f, indent=0)


SERVING_FILE = "serving_digests.json"


def serving_kinds():
    """Every distinct session stream the serving workload draws."""
    out = [S.stencil_1d(), S.stencil_2d(), S.nbody(steps=50)]
    out += [S.growing(queue_cap=cap) for cap in (1, 2, 4, 8, 16, 32, 64)]
    return out


def _serving_one(i):
    s = serving_kinds()[i]
    st = oracle.run_stream(s, fetch=False)["stats"]
    return s.name, {k: st[k] for k in STAT_KEYS}


def serving(workers):
    """Oracle statistics and digests of each kind of serving session, keyed by
    stream name (sessions carry the kind's name after their session prefix)."""
    from multiprocessing import Pool
    with Pool(workers) as pool:
        rows = dict(pool.map(_serving_one, range(len(serving_kinds()))))
    with open(os.path.join(HERE, SERVING_FILE), "w") as f:
        json.dump(rows, f, indent=1)
    print(sorted(rows))


OOO_FILE = "stencil2d_full_ooo.json"
OOO_CASES = [{}, {"window": 64, "eager": 0}]  # changes to the defaults of oracle.ooo_params


def ooo():
    """The oracle's out-of-order engine (Sec. 4.1) over the 2-D stencil's
    graph: per parameter set the summary, a SHA-256 of every result slot and
    the first and last slots."""
    import hashlib
    s = S.stencil_2d()
    out = oracle.run_stream(s, fetch=True)
    doc = {"case": "stencil2d_full", "devices": s.nodes * s.devices, "runs": []}
    keep = {}
    for j, kw in enumerate(OOO_CASES):
        p = oracle.ooo_params(s.nodes * s.devices, **kw)
        t = time.time()
        slots, summ = oracle.ooo_simulate(out["instructions"], out["edges"], p)
        doc["runs"].append({"params": kw, "summary": summ, "slots_sha256": hashlib.sha256(slots.tobytes()).hexdigest(),
                            "oracle_seconds": round(time.time() - t, 1)})
        keep[f"slots{j}"] = head_tail(slots, 1000)
        print("ooo", kw, summ, flush=True)
    # the default parameters also at the top level (read by the benchmark)
    doc["summary"] = doc["runs"][0]["summary"]
    doc["slots_sha256"] = doc["runs"][0]["slots_sha256"]
    with open(os.path.join(HERE, OOO_FILE), "w") as f:
        json.dump(doc, f, indent=1)
    np.savez_compressed(os.path.join(HERE, "stencil2d_full_ooo_slots.npz"), **keep)


if __name__ == "__main__":
    if sys.argv[1:2] == ["serving"]:
        serving(int(sys.argv[2]) if len(sys.argv) > 2 else 3)
    elif sys.argv[1:2] == ["ooo"]:
        ooo()
    elif sys.argv[1:2] == ["batched"]:
        batched(int(sys.argv[2]) if len(sys.argv) > 2 else 4)
    else:
        main(sys.argv[1:] or list(CASES))
