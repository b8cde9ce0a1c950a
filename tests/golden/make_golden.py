"""Write the stored expected values of the large parity cases.

Calls only the oracle (oracle/) on the seeded workloads; the GPU tests
compare the HIP path's counts, per-kind statistics and record digests with
these files, and its first/last records with the stored ones.

    python tests/golden/make_golden.py nbody_full growing_q1 ...
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


if __name__ == "__main__":
    main(sys.argv[1:] or list(CASES))
