"""Pins of the oracle's box-set primitives against brute-force point sets.

Box algebra (Sec. 3.2 and 3.3 speak of rectangular regions and subregions):
difference, the merge relation of allocation planning, the merge fixpoint,
the canonical decomposition, the chunk split (Sec. 3.1) and the range
mappers (Sec. 2.1, Listing 2).
"""
import itertools
import random

import numpy as np
import pytest

import oracle
from bruteforce import (box_points, canonical_bruteforce, points_merge, split_py)
from paper_2503_10516_amd.streams import (ALL, FIXED, NEIGHBORHOOD, ONE_TO_ONE, READ, SLICE,
                                          Access)


def rand_box(rng, n=6, dims=3, allow_empty=False):
    lo, hi = [0, 0, 0], [1, 1, 1]
    for d in range(dims):
        a = rng.randrange(0, n)
        b = rng.randrange(a if allow_empty else a + 1, n + 1)
        lo[d], hi[d] = a, b
    return (tuple(lo), tuple(hi))


def pts(boxes):
    s = set()
    for b in boxes:
        s |= set(box_points(b))
    return s


@pytest.mark.parametrize("dims", [1, 2, 3])
def test_subtract_matches_point_sets(dims):
    rng = random.Random(dims)
    for _ in range(400):
        a, b = rand_box(rng, dims=dims), rand_box(rng, dims=dims)
        pieces = oracle.box_subtract(a, b)
        got = [set(box_points(p)) for p in pieces]
        assert all(g for g in got), "no empty pieces"
        for x, y in itertools.combinations(got, 2):
            assert not (x & y), "pieces are disjoint"
        union = set().union(*got) if got else set()
        assert union == set(box_points(a)) - set(box_points(b))
        assert len(pieces) <= 2 * dims


def test_merge_relation_matches_brute_force():
    rng = random.Random(7)
    hits = {True: 0, False: 0}
    for _ in range(1500):
        dims = rng.randrange(1, 4)
        a, b = rand_box(rng, 5, dims), rand_box(rng, 5, dims)
        got = oracle.box_merges(a, b)
        assert got == points_merge(a, b), (a, b)
        hits[got] += 1
    assert hits[True] > 100 and hits[False] > 100
    # hand cases: face, edge and corner contact in 2-D
    assert oracle.box_merges(((0, 0, 0), (2, 2, 1)), ((2, 0, 0), (4, 1, 1)))       # shared face
    assert not oracle.box_merges(((0, 0, 0), (2, 2, 1)), ((2, 2, 0), (4, 4, 1)))   # corner only
    assert not oracle.box_merges(((0, 0, 0), (2, 2, 2)), ((2, 2, 0), (4, 4, 2)))   # edge only (3-D)


def fixpoint_bruteforce(boxes):
    """Union-find over the brute-force merge relation, bounding boxes, repeat."""
    cur = [b for b in boxes if all(b[0][d] < b[1][d] for d in range(3))]
    while True:
        n = len(cur)
        parent = list(range(n))

        def find(x):
            while parent[x] != x:
                x = parent[x]
            return x
        for i in range(n):
            for j in range(i + 1, n):
                if points_merge(cur[i], cur[j]):
                    parent[find(i)] = find(j)
        groups = {}
        for i in range(n):
            groups.setdefault(find(i), []).append(cur[i])
        nxt = []
        for g in groups.values():
            lo = tuple(min(b[0][d] for b in g) for d in range(3))
            hi = tuple(max(b[1][d] for b in g) for d in range(3))
            nxt.append((lo, hi))
        if len(nxt) == len(cur):
            return sorted(nxt)
        cur = nxt


def test_merge_fixpoint_matches_bruteforce_and_is_order_free():
    rng = random.Random(11)
    for _ in range(200):
        dims = rng.randrange(1, 4)
        boxes = [rand_box(rng, 8, dims) for _ in range(rng.randrange(1, 7))]
        want = fixpoint_bruteforce(boxes)
        got = oracle.merge_fixpoint(boxes)
        assert sorted(got) == want
        shuffled = list(boxes)
        rng.shuffle(shuffled)
        assert oracle.merge_fixpoint(shuffled) == got
        # result boxes pairwise do not merge, and cover every input
        for x, y in itertools.combinations(got, 2):
            assert not points_merge(x, y)
        for b in boxes:
            assert any(all(g[0][d] <= b[0][d] and b[1][d] <= g[1][d] for d in range(3)) for g in got)


@pytest.mark.parametrize("dims", [1, 2, 3])
def test_canonical_matches_definition(dims):
    rng = random.Random(100 + dims)
    n = 6
    shape = tuple(n if d < dims else 1 for d in range(3))
    for _ in range(150):
        boxes = [rand_box(rng, n, dims) for _ in range(rng.randrange(1, 6))]
        p = pts(boxes)
        got = oracle.canonical(boxes)
        assert got == canonical_bruteforce(p, shape)
        # disjoint, exact union, ordered by min
        sets = [set(box_points(b)) for b in got]
        for x, y in itertools.combinations(sets, 2):
            assert not (x & y)
        assert set().union(*sets) == p
        assert got == sorted(got)


def test_canonical_unique_for_random_decompositions():
    rng = random.Random(5)
    for _ in range(60):
        g = np.zeros((5, 5, 3), dtype=bool)
        for b in [rand_box(rng, 5, 3) for _ in range(3)]:
            g[b[0][0]:b[1][0], b[0][1]:b[1][1], b[0][2]:b[1][2]] = True
        points = {tuple(int(v) for v in x) for x in np.argwhere(g)}
        # decompose into unit boxes, shuffled, and into random larger pieces
        units = [((x, y, z), (x + 1, y + 1, z + 1)) for (x, y, z) in points]
        rng.shuffle(units)
        want = oracle.canonical(units)
        assert want == canonical_bruteforce(points, g.shape)
        for _ in range(3):
            pieces = list(units)
            rng.shuffle(pieces)
            merged = oracle.canonical(pieces[: len(pieces) // 2]) + pieces[len(pieces) // 2:]
            assert oracle.canonical(merged) == want


def test_canonical_overlapping_inputs_and_empty():
    assert oracle.canonical([]) == []
    assert oracle.canonical([((0, 0, 0), (0, 1, 1))]) == []
    a = ((0, 0, 0), (4, 1, 1))
    assert oracle.canonical([a, a, ((1, 0, 0), (3, 1, 1))]) == [a]
    # L-shape in 2-D: cut at x=2 where the cross-section changes
    got = oracle.canonical([((0, 0, 0), (4, 2, 1)), ((0, 2, 0), (2, 4, 1))])
    assert got == [((0, 0, 0), (2, 4, 1)), ((2, 0, 0), (4, 2, 1))]


@pytest.mark.parametrize("nodes,devices,chunks,lo,hi", [
    (1, 2, 2, 0, 4096), (16, 8, 128, 0, 4096), (2, 3, 12, 5, 40), (3, 2, 6, 0, 4), (2, 2, 8, 7, 7),
    (4, 4, 64, 0, 100), (16, 8, 1024, 0, 1 << 20), (1, 1, 1, 3, 9),
])
def test_split_properties(nodes, devices, chunks, lo, hi):
    task_lo, task_hi = (lo, 0, 0), (hi, 5, 1)
    got = oracle.split(nodes, devices, chunks, task_lo, task_hi)
    assert len(got) == chunks
    # chunks tile the task range along dim 0, in order, keeping dims 1-2
    pos = lo
    for c in got:
        assert c[0][0] == pos and c[1][0] >= c[0][0]
        assert c[0][1:] == task_lo[1:] and c[1][1:] == task_hi[1:]
        pos = c[1][0]
    assert pos == hi
    n = hi - lo
    per = chunks // (nodes * devices)
    # node-level ranges: floor split, sizes differ by at most one
    node_sizes = [sum(c[1][0] - c[0][0] for c in got[i * devices * per:(i + 1) * devices * per])
                  for i in range(nodes)]
    assert max(node_sizes) - min(node_sizes) <= 1 and sum(node_sizes) == n
    assert node_sizes == [((i + 1) * n) // nodes - (i * n) // nodes for i in range(nodes)]
    # when the range divides evenly the nested split equals the flat split
    if n % chunks == 0:
        assert all(c[1][0] - c[0][0] == n // chunks for c in got)
    assert got == split_py(nodes, devices, chunks, task_lo, task_hi)


def test_split_small_range_leaves_empty_chunks():
    got = oracle.split(1, 4, 4, (0, 0, 0), (2, 1, 1))
    sizes = [c[1][0] - c[0][0] for c in got]
    assert sorted(sizes) == [0, 0, 1, 1] and sum(sizes) == 2


def test_range_mappers_hand_cases():
    ext = (10, 8, 1)
    chunk = ((0, 0, 0), (5, 8, 1))
    assert oracle.map_range(Access(0, READ, ONE_TO_ONE), 2, chunk, 2, ext) == ((0, 0, 0), (5, 8, 1))
    # neighborhood is clamped at the buffer border
    assert oracle.map_range(Access(0, READ, NEIGHBORHOOD, (1, 2, 0)), 2, chunk, 2, ext) == ((0, 0, 0), (6, 8, 1))
    assert oracle.map_range(Access(0, READ, NEIGHBORHOOD, (1, 1, 0)), 2, ((5, 2, 0), (10, 4, 1)), 2, ext) == \
        ((4, 1, 0), (10, 5, 1))
    assert oracle.map_range(Access(0, READ, ALL), 2, chunk, 2, ext) == ((0, 0, 0), (10, 8, 1))
    assert oracle.map_range(Access(0, READ, SLICE, slice_dim=0), 2, ((2, 3, 0), (4, 5, 1)), 2, ext) == \
        ((0, 3, 0), (10, 5, 1))
    assert oracle.map_range(Access(0, READ, FIXED, fixed_lo=(3, 6, 0), fixed_hi=(12, 9, 1)), 2, chunk, 2, ext) == \
        ((3, 6, 0), (10, 8, 1))
    # all on a 1-D buffer from a 2-D task
    assert oracle.map_range(Access(0, READ, ALL), 2, chunk, 1, (7, 1, 1)) == ((0, 0, 0), (7, 1, 1))


def test_digest_definition():
    # FNV-1a-64 of the bytes of one zero word, then splitmix64 mixing
    def splitmix(x):
        x = (x + 0x9E3779B97F4A7C15) & (2**64 - 1)
        x = ((x ^ (x >> 30)) * 0xBF58476D1CE4E5B9) & (2**64 - 1)
        x = ((x ^ (x >> 27)) * 0x94D049BB133111EB) & (2**64 - 1)
        return x ^ (x >> 31)

    def fnv(words):
        h = 0xcbf29ce484222325
        for w in words:
            for byte in range(8):
                h ^= (w >> (8 * byte)) & 0xFF
                h = (h * 0x100000001b3) & (2**64 - 1)
        return h
    words = np.array([[1, 2, 3], [4, 5, 6], [7, 8, 2**63]], dtype=np.uint64)
    want = sum(splitmix(fnv([int(v) for v in row]) ^ splitmix(i)) for i, row in enumerate(words)) % 2**64
    assert oracle.digest_words(words) == want
    # published splitmix64 reference value (seed 0 -> first output)
    assert splitmix(0) == 0xE220A8397B1DCDAF
