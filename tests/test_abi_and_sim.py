"""CPU checks of the product library.

* libig.so (the gfx950 build) loads and exports every function declared in
  include/ig.h -- nothing is called, so no GPU is needed.
* The kernel logic of ig_kernels.hip, compiled for the host with one
  workgroup emulated by threads and barriers (a test-only build, never used
  by the product), reproduces the oracle bit for bit on small streams.
"""
import os
import re
import subprocess

import pytest

import oracle
from parity import assert_same
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
    return [os.path.join(CSRC, f) for f in ("ig_sim.cpp", "ig_api.cpp", "ig_kernels.hip", "ig_dev.h")] + \
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
