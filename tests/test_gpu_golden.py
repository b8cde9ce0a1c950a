"""The HIP path at full size against stored oracle results.

tests/golden/*.json were written by tests/golden/make_golden.py, which calls
only the oracle.  The device computes the three record digests; they must
equal the oracle's, together with counts, per-kind statistics, task statuses
and the stored first and last records.
"""
import json
import os

import numpy as np
import pytest

from paper_2503_10516_amd import binding as B
from paper_2503_10516_amd import streams as S

pytestmark = pytest.mark.gpu

HERE = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")
CASES = {
    "stencil1d_full": lambda: S.stencil_1d(),
    "nbody_full": lambda: S.nbody(),
    "stencil2d_full": lambda: S.stencil_2d(),
    "growing_full": lambda: S.growing(),
    "growing_nola": lambda: S.growing(lookahead=0),
    "growing_q8": lambda: S.growing(queue_cap=8),
}


@pytest.fixture(scope="module", autouse=True)
def _device():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    torch.cuda.set_device(0)


def head_tail(arr, n):
    return np.concatenate([arr[:n], arr[-n:]]) if len(arr) > 2 * n else arr


@pytest.mark.parametrize("name", sorted(CASES))
def test_full_size_against_oracle_golden(name):
    g = json.load(open(os.path.join(HERE, name + ".json")))
    rec = np.load(os.path.join(HERE, name + "_records.npz"))
    s = CASES[name]()
    print(f"[gpu] golden {name}: {s.n_tasks} tasks", flush=True)
    ctx = B.make_context(s)
    ctx.record(s)
    ctx.flush()
    assert ctx.sync() == 0
    st = ctx.stats()
    for k in ("n_instructions", "n_bindings", "n_edges", "resizes", "warnings", "digest_instructions",
              "digest_bindings", "digest_edges"):
        assert st[k] == g[k], (k, st[k], g[k])
    assert st["per_kind"] == g["per_kind"] and st["per_dep"] == g["per_dep"]
    out = ctx.fetch_all()
    ctx.close()
    assert [int(x) for x in out["status"]] == g["status"]
    # the first and last records (up to 10k of each list) bit for bit
    for key in ("instructions", "bindings", "edges"):
        want = rec[key]
        got = head_tail(out[key], g["keep"])
        assert got.dtype.itemsize == want.dtype.itemsize and len(got) == len(want), key
        assert got.tobytes() == want.tobytes(), key
    # structural properties at full size: ids are a topological order,
    # edges are sorted by (to, from) and unique
    ed = out["edges"]
    assert np.all(ed["from"] < ed["to"])
    key = ed["to"].astype(np.uint64) * np.uint64(1 << 32) + ed["from"].astype(np.uint64)
    assert np.all(key[1:] > key[:-1])
