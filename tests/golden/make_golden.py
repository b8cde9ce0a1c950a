"""Write the stored expected values of the large parity cases.

Calls only the oracle (oracle/) on the seeded workloads; the GPU tests
compare the HIP path's counts, per-kind statistics and record digests with
these files, and its first/last records with the stored ones.

    python tests/golden/make_golden.py nbody_full growing_q1 ...
    python tests/golden/make_golden.py batched 4      # the 256 batched streams, 4 processes
    python tests/golden/make_golden.py serving 3      # each kind of serving session
"""
import json
import os
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

import oracle  # noqa: E402
from paper_2503_10516_amd import streams as S  # noqa: E402

CASES = {
    "nbody_full": lambda: S.nbody(),                       # N-body, 2^20 x 16 B, 500 steps, 16 x 8 devices
    "stencil2d_full": lambda: S.stencil_2d(),               # 2-D stencil, 4096^2, 1000 tasks
    "growing_full": lambda: S.growing(),                    # RSim pattern [84000 x 256], lookahead, unbounded queue
    "growing_nola": lambda: S.growing(lookahead=0),         # no lookahead: a resize per device per step
    "growing_q8": lambda: S.growing(queue_cap=8),           # lookahead window of 8 commands
}

EDGE_KEEP = 2000  # first and last records stored verbatim
BATCHED_FILE = "batched_digests.json"


def rec_list(arr, n):
    out = []
    for r in list(arr[:n]) + list(arr[-n:]):
        out.append([int(x) if not hasattr(x, "__len__") else [int(v) for v in x] for x in r])
    return out


def main(names):
    for name in names:
        s = CASES[name]()
        t0 = time.time()
        out = oracle.run_stream(s, fetch=True)
        st = out["stats"]
        doc = {
            "case": name,
            "stream": s.name,
            "oracle_seconds": round(time.time() - t0, 2),
            "n_instructions": st["n_instructions"],
            "n_bindings": st["n_bindings"],
            "n_edges": st["n_edges"],
            "per_kind": st["per_kind"],
            "per_dep": st["per_dep"],
            "resizes": st["resizes"],
            "warnings": st["warnings"],
            "digest_instructions": st["digest_instructions"],
            "digest_bindings": st["digest_bindings"],
            "digest_edges": st["digest_edges"],
            "status": [int(x) for x in out["status"]],
            "head_tail_instructions": rec_list(out["instructions"], EDGE_KEEP // 4),
            "head_tail_edges": rec_list(out["edges"], EDGE_KEEP // 2),
        }
        with open(os.path.join(HERE, f"{name}.json"), "w") as f:
            json.dump(doc, f)
        print(name, st["n_instructions"], st["n_edges"], f"{doc['oracle_seconds']} s", flush=True)


def _batched_one(i):
    s = S.batched_stream(S.BATCHED_SEED, i, w_all=S.BATCHED_W_ALL, w_slice=S.BATCHED_W_SLICE)
    t0 = time.time()
    st = oracle.run_stream(s, fetch=False)
    o = st["stats"]
    return {"index": i, "stream": s.name, "tasks": s.n_tasks, "oracle_seconds": round(time.time() - t0, 2),
            "n_instructions": o["n_instructions"], "n_bindings": o["n_bindings"], "n_edges": o["n_edges"],
            "per_kind": o["per_kind"], "per_dep": o["per_dep"], "warnings": o["warnings"],
            "digest_instructions": o["digest_instructions"], "digest_bindings": o["digest_bindings"],
            "digest_edges": o["digest_edges"]}


def batched(workers):
    """Oracle statistics and digests of every stream of the batched workload
    (256 streams), computed in parallel worker processes."""
    from multiprocessing import Pool
    with Pool(workers) as pool:
        rows = []
        for r in pool.imap_unordered(_batched_one, range(256)):
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
    keep = ("n_instructions", "n_bindings", "n_edges", "per_kind", "per_dep", "warnings",
            "digest_instructions", "digest_bindings", "digest_edges")
    return s.name, {k: st[k] for k in keep}


def serving(workers):
    """Oracle statistics and digests of each kind of serving session, keyed by
    stream name (sessions carry the kind's name after their session prefix)."""
    from multiprocessing import Pool
    with Pool(workers) as pool:
        rows = dict(pool.map(_serving_one, range(len(serving_kinds()))))
    with open(os.path.join(HERE, SERVING_FILE), "w") as f:
        json.dump(rows, f, indent=1)
    print(sorted(rows))


if __name__ == "__main__":
    if sys.argv[1:2] == ["serving"]:
        serving(int(sys.argv[2]) if len(sys.argv) > 2 else 3)
    elif sys.argv[1:2] == ["batched"]:
        batched(int(sys.argv[2]) if len(sys.argv) > 2 else 4)
    else:
        main(sys.argv[1:] or list(CASES))
