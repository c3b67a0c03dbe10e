"""Pins of the CPU oracle against things other than itself (no GPU needed).

* brute force (tests/bruteforce.py) on hypothesis-generated op sequences over a tiny key universe
  that forces duplicates, reserved-looking bit patterns and capacity exhaustion;
* Python's dict as the textbook map on larger random batches;
* the paper's printed spatial-hash constants (tests/golden), the XOR decomposition of that hash,
  and the independence of its bucket (mod 2^21) from the sign extension of the 21-bit fields;
* closed forms of the pool order, capacity exhaustion and empty-table cases;
* the invariants the chained layout must keep after every batch;
* layout independence: results are identical under every bucket count and hash.
"""
import os

import numpy as np
import pytest
from hypothesis import HealthCheck, given, settings
from hypothesis import strategies as st

import oracle
from oracle import HASH_MIX64, HASH_VOXEL21, OraclePool, OracleTable
from paper_1908_05936_amd.workloads import pack_int3
from tests.bruteforce import BrutePool, BruteTable

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")
U64MAX = (1 << 64) - 1
UNIVERSE = list(range(16)) + [0, U64MAX, U64MAX - 1, 1 << 63]


def _check(t, pool=None, from_pool=False):
    bad, what = t.check(pool, from_pool)
    assert bad == 0, f"invariant bits {what:#x}"


# ------------------------------------------------------------------------------------------
# brute force
# ------------------------------------------------------------------------------------------
keys_st = st.lists(st.sampled_from(UNIVERSE), min_size=0, max_size=24)
map_op = st.tuples(st.sampled_from(["insert", "find", "erase", "clear"]), keys_st,
                   st.lists(st.integers(0, U64MAX), min_size=24, max_size=24))


@settings(max_examples=300, deadline=None, suppress_health_check=[HealthCheck.too_slow])
@given(cap=st.integers(0, 12), bits=st.sampled_from([32, 64]), nb=st.sampled_from([1, 3, 8, 64]),
       hk=st.sampled_from([HASH_MIX64, HASH_VOXEL21]), ops=st.lists(map_op, max_size=12))
def test_map_ops_match_bruteforce(cap, bits, nb, hk, ops):
    t = OracleTable(cap, bits, hk, nb)
    b = BruteTable(cap, bits)
    mask = (1 << bits) - 1
    for kind, keys, vals in ops:
        vals = [v & mask for v in vals[:len(keys)]]
        k = np.array(keys, dtype=np.uint64)
        if kind == "insert":
            got = t.insert(k, np.array(vals, dtype=np.uint64))
            assert got.tolist() == b.insert(keys, vals)
        elif kind == "find":
            out, fd = t.find(k)
            eo, ef = b.find(keys)
            assert [int(x) for x in out] == eo and fd.tolist() == ef
        elif kind == "erase":
            assert t.erase(k).tolist() == b.erase(keys)
        else:
            t.clear()
            b.pairs = []
        assert t.size() == len(b.pairs)
        ks, vs = t.dump()
        assert list(zip(ks.tolist(), [int(v) for v in vs])) == b.dump()
        _check(t)


alloc_op = st.tuples(st.sampled_from(["insert_alloc", "erase_release", "find"]), keys_st)


@settings(max_examples=300, deadline=None, suppress_health_check=[HealthCheck.too_slow])
@given(cap=st.integers(0, 12), pcap=st.integers(0, 12), nb=st.sampled_from([1, 5, 32]),
       ops=st.lists(alloc_op, max_size=12))
def test_pool_ops_match_bruteforce(cap, pcap, nb, ops):
    t = OracleTable(cap, 32, HASH_MIX64, nb)
    p = OraclePool(pcap)
    b = BruteTable(cap, 32)
    bp = BrutePool(pcap)
    for kind, keys in ops:
        k = np.array(keys, dtype=np.uint64)
        if kind == "insert_alloc":
            out, stt = t.insert_alloc(p, k)
            eo, es = b.insert_alloc(bp, keys)
            assert out.tolist() == eo and stt.tolist() == es
        elif kind == "erase_release":
            assert t.erase_release(p, k).tolist() == b.erase_release(bp, keys)
        else:
            out, fd = t.find(k)
            eo, ef = b.find(keys)
            assert [int(x) for x in out] == eo and fd.tolist() == ef
        assert p.dump().tolist() == bp.stack
        _check(t, p, from_pool=True)


@settings(max_examples=200, deadline=None)
@given(pcap=st.integers(0, 10),
       ops=st.lists(st.tuples(st.sampled_from(["pop", "push"]), st.integers(0, 8),
                              st.lists(st.integers(-5, 20), min_size=8, max_size=8)), max_size=10))
def test_pool_stack_matches_bruteforce(pcap, ops):
    p = OraclePool(pcap)
    bp = BrutePool(pcap)
    for kind, n, vals in ops:
        if kind == "pop":
            out, stt = p.pop(n)
            eo, es = bp.pop(n)
            assert out.tolist() == eo and stt.tolist() == es
        else:
            assert p.push(np.array(vals[:n], dtype=np.int32)).tolist() == bp.push(vals[:n])
        assert p.dump().tolist() == bp.stack


@settings(max_examples=200, deadline=None)
@given(pcap=st.integers(0, 10),
       ops=st.lists(st.tuples(st.sampled_from(["pop", "push", "pop_front", "push_front"]),
                              st.integers(0, 8),
                              st.lists(st.integers(-5, 20), min_size=8, max_size=8)), max_size=12))
def test_pool_deque_matches_collections_deque(pcap, ops):
    """The pool's four deque operations (Section 4.3) against Python's collections.deque, the
    textbook double-ended queue, with the pool's fixed capacity: a pop on an empty deque gives
    -1 (status 2), a push on a full one is refused (status 2).  The dump lists front to back."""
    from collections import deque
    p = OraclePool(pcap)
    d = deque(range(pcap - 1, -1, -1))     # a fresh pool pops_back 0, 1, 2, ...
    for kind, n, vals in ops:
        if kind in ("pop", "pop_front"):
            out, stt = p.pop(n) if kind == "pop" else p.pop_front(n)
            eo, es = [], []
            for _ in range(n):
                if d:
                    eo.append(d.pop() if kind == "pop" else d.popleft())
                    es.append(1)
                else:
                    eo.append(-1)
                    es.append(2)
            assert out.tolist() == eo and stt.tolist() == es
        else:
            v = vals[:n]
            stt = p.push(np.array(v, dtype=np.int32)) if kind == "push" else \
                p.push_front(np.array(v, dtype=np.int32))
            es = []
            for x in v:
                if len(d) == pcap:
                    es.append(2)
                else:
                    (d.append if kind == "push" else d.appendleft)(x)
                    es.append(1)
            assert stt.tolist() == es
        assert p.dump().tolist() == list(d)


@settings(max_examples=150, deadline=None, suppress_health_check=[HealthCheck.too_slow])
@given(ops=st.lists(st.tuples(st.sampled_from(["insert", "erase"]),
                              st.lists(st.sampled_from(UNIVERSE), min_size=0, max_size=12)),
                    max_size=6),
       lo=st.sampled_from(UNIVERSE), hi=st.sampled_from(UNIVERSE + [U64MAX]))
def test_key_range_selection_matches_bruteforce(ops, lo, hi):
    """Range selection (Section 3.6) by key interval: the brute-force table's pairs filtered by
    lo <= key < hi and sorted, after generated insert/erase batches."""
    t = OracleTable(8, 64, HASH_MIX64, 3)
    b = BruteTable(8, 64)
    for kind, keys in ops:
        ks = np.array(keys, dtype=np.uint64)
        if kind == "insert":
            t.insert(ks, ks + np.uint64(1))
            b.insert([int(k) for k in keys], [int(k) + 1 & U64MAX for k in keys])
        else:
            t.erase(ks)
            b.erase([int(k) for k in keys])
    got_k, got_v = t.select_key_range(lo, hi)
    want = sorted((k, v) for k, v in b.pairs if lo <= k < hi)
    assert list(zip(got_k.tolist(), got_v.tolist())) == want


def test_voxel_box_selection_closed_form():
    """Selection by block box on packed coordinates: the blocks of a 9 x 9 x 9 grid around the
    origin (negative coordinates included) and four far blocks; a box selects exactly the grid
    points inside it, counted from the coordinates themselves, and keys with bit 63 set (which
    pack no block) never match."""
    g = np.arange(-4, 5)
    X, Y, Z = np.meshgrid(g, g, g, indexing="ij")
    far = np.array([[1048575, 0, 0], [-1048576, 3, 3], [0, 0, 2000], [5, -5, -700]])
    cx = np.concatenate([X.ravel(), far[:, 0]])
    cy = np.concatenate([Y.ravel(), far[:, 1]])
    cz = np.concatenate([Z.ravel(), far[:, 2]])
    keys = pack_int3(cx, cy, cz)
    t = OracleTable(2000, 64, HASH_VOXEL21, 1 << 21)
    t.insert(keys, np.arange(keys.size, dtype=np.uint64))
    t.insert(np.array([U64MAX, 1 << 63], dtype=np.uint64), np.array([7, 8], dtype=np.uint64))
    for lo3, hi3 in [((-1, -2, 0), (2, 1, 4)), ((-4, -4, -4), (4, 4, 4)), ((3, 3, 3), (2, 9, 9)),
                     ((0, 0, 0), (0, 0, 0)), ((-1048576, -1048576, -1048576), (1048575, 1048575, 1048575))]:
        inside = ((cx >= lo3[0]) & (cx <= hi3[0]) & (cy >= lo3[1]) & (cy <= hi3[1]) &
                  (cz >= lo3[2]) & (cz <= hi3[2]))
        k, v = t.select_voxel_box(lo3, hi3)
        assert k.tolist() == sorted(keys[inside].tolist())
        assert v.tolist() == [int(np.flatnonzero(keys == x)[0]) for x in k]


def test_voxel_neighbour_keys_closed_form():
    """Neighbours of packed blocks: the origin's 6 face neighbours are the unit offsets along each
    axis; 26 neighbours are every offset in {-1, 0, 1}^3 but zero, each once; a block at the edge
    of the 21-bit range wraps to the other end (packing takes each coordinate modulo 2^21)."""
    six = oracle.voxel_neighbour_keys(pack_int3([0], [0], [0]), 6)
    want = pack_int3([-1, 1, 0, 0, 0, 0], [0, 0, -1, 1, 0, 0], [0, 0, 0, 0, -1, 1])
    assert sorted(six.tolist()) == sorted(want.tolist())
    blk = pack_int3([5], [-7], [1048575])
    all26 = oracle.voxel_neighbour_keys(blk, 26)
    offs = [(dx, dy, dz) for dx in (-1, 0, 1) for dy in (-1, 0, 1) for dz in (-1, 0, 1)
            if (dx, dy, dz) != (0, 0, 0)]
    exp = pack_int3([5 + o[0] for o in offs], [-7 + o[1] for o in offs],
                    [1048575 + o[2] for o in offs])
    assert sorted(all26.tolist()) == sorted(exp.tolist()) and len(set(all26.tolist())) == 26
    # +1 on z = 2^20 - 1 wraps to -2^20
    assert int(pack_int3([5], [-7], [-1048576])[0]) in all26.tolist()
    two = oracle.voxel_neighbour_keys(pack_int3([0, 10], [0, 10], [0, 10]), 6)
    assert two.size == 12 and two[6:].tolist() == oracle.voxel_neighbour_keys(
        pack_int3([10], [10], [10]), 6).tolist()
    with pytest.raises(ValueError):
        oracle.voxel_neighbour_keys(blk, 7)


def test_fifo_free_list_closed_form():
    """pop_front of a fresh pool of capacity c returns c-1, c-2, ...; used as a first-in
    first-out free list (pop_front, push_back) released values come back after every older one."""
    p = OraclePool(6)
    out, stt = p.pop_front(3)
    assert out.tolist() == [5, 4, 3] and stt.tolist() == [1, 1, 1]
    assert p.push(np.array([4, 5], dtype=np.int32)).tolist() == [1, 1]
    out, _ = p.pop_front(5)
    assert out.tolist() == [2, 1, 0, 4, 5]
    assert p.push_front(np.array([7, 8, 9], dtype=np.int32)).tolist() == [1, 1, 1]
    assert p.dump().tolist() == [9, 8, 7]


# ------------------------------------------------------------------------------------------
# Python dict as the textbook map, at a size brute force cannot reach
# ------------------------------------------------------------------------------------------
@pytest.mark.parametrize("seed", [0, 1])
def test_dict_replay(seed):
    rng = np.random.default_rng(seed)
    universe = rng.integers(0, 1 << 64, size=3000, dtype=np.uint64)
    cap = 2000
    t = OracleTable(cap, 64, HASH_MIX64, 997)
    d = {}
    for step in range(12):
        kind = ["insert", "find", "erase"][step % 3]
        k = universe[rng.integers(0, universe.size, size=4000)]
        if kind == "insert":
            v = rng.integers(0, 1 << 64, size=k.size, dtype=np.uint64)
            got = t.insert(k, v)
            exp = []
            for kk, vv in zip(k.tolist(), v.tolist()):
                if kk in d:
                    exp.append(0)
                elif len(d) == cap:
                    exp.append(2)
                else:
                    d[kk] = vv
                    exp.append(1)
            assert got.tolist() == exp
        elif kind == "find":
            out, fd = t.find(k)
            assert fd.tolist() == [int(kk in d) for kk in k.tolist()]
            assert out.tolist() == [d.get(kk, U64MAX) for kk in k.tolist()]
        else:
            got = t.erase(k)
            exp = []
            for kk in k.tolist():
                exp.append(int(d.pop(kk, None) is not None))
            assert got.tolist() == exp
        assert t.size() == len(d)
        _check(t)


# ------------------------------------------------------------------------------------------
# spatial hash of Section 4.1
# ------------------------------------------------------------------------------------------
def _golden_constants():
    out = {}
    with open(os.path.join(GOLDEN, "voxel21_constants.txt")) as f:
        for line in f:
            if line.strip() and not line.startswith("#"):
                axis, m = line.split()
                out[axis] = int(m)
    return out


def test_voxel_hash_unit_vectors_are_the_printed_constants():
    c = _golden_constants()
    assert oracle.voxel21_hash(int(pack_int3(1, 0, 0))) == c["x"]
    assert oracle.voxel21_hash(int(pack_int3(0, 1, 0))) == c["y"]
    assert oracle.voxel21_hash(int(pack_int3(0, 0, 1))) == c["z"]
    assert oracle.voxel21_hash(0) == 0
    # a negative int converts to size_t by adding 2^64
    assert oracle.voxel21_hash(int(pack_int3(-1, 0, 0))) == (1 << 64) - c["x"]
    assert oracle.voxel21_hash(int(pack_int3(0, 0, -1))) == (1 << 64) - c["z"]
    # 2 * the x constant still fits in an int; 30 * it wraps past 2^31
    assert oracle.voxel21_hash(int(pack_int3(2, 0, 0))) == 2 * c["x"]
    wrapped = (30 * c["x"]) % (1 << 32)
    assert wrapped >= 1 << 31
    assert oracle.voxel21_hash(int(pack_int3(30, 0, 0))) == (1 << 64) - ((1 << 32) - wrapped)


def test_voxel_hash_xor_decomposition_and_21bit_buckets():
    c = _golden_constants()
    rng = np.random.default_rng(7)
    xyz = rng.integers(-(1 << 20), 1 << 20, size=(2000, 3))
    M = (1 << 21) - 1
    for x, y, z in xyz.tolist():
        h = oracle.voxel21_hash(int(pack_int3(x, y, z)))
        hx = oracle.voxel21_hash(int(pack_int3(x, 0, 0)))
        hy = oracle.voxel21_hash(int(pack_int3(0, y, 0)))
        hz = oracle.voxel21_hash(int(pack_int3(0, 0, z)))
        assert h == hx ^ hy ^ hz
        # bucket mod 2^21 depends only on the unsigned 21-bit fields, exact integer arithmetic
        ux, uy, uz = x & M, y & M, z & M
        assert h & M == ((ux * c["x"]) ^ (uy * c["y"]) ^ (uz * c["z"])) & M


def test_voxel_bucket_reduction():
    c = _golden_constants()
    t21 = OracleTable(8, 32, HASH_VOXEL21, 1 << 21)
    t1000 = OracleTable(8, 32, HASH_VOXEL21, 1000)
    k = int(pack_int3(-1, 0, 0))
    assert t21.bucket_of(k) == ((1 << 64) - c["x"]) % (1 << 21)
    assert t1000.bucket_of(k) == ((1 << 64) - c["x"]) % 1000
    assert t21.bucket_of(int(pack_int3(0, 1, 0))) == c["y"] % (1 << 21)


# ------------------------------------------------------------------------------------------
# closed forms and special cases
# ------------------------------------------------------------------------------------------
def test_fresh_pool_order_and_lifo_reuse():
    p = OraclePool(10)
    out, stt = p.pop(4)
    assert out.tolist() == [0, 1, 2, 3] and stt.tolist() == [1] * 4
    t = OracleTable(100, 32, HASH_MIX64, 17)
    p2 = OraclePool(50)
    keys = np.array([5, 9, 5, 7, 11, 9], dtype=np.uint64)
    out, stt = t.insert_alloc(p2, keys)
    # first occurrences take 0, 1, 2, 3 in order; repeats report the existing value
    assert out.tolist() == [0, 1, 0, 2, 3, 1]
    assert stt.tolist() == [1, 1, 0, 1, 1, 0]
    er = t.erase_release(p2, np.array([9, 11, 9, 5], dtype=np.uint64))
    assert er.tolist() == [1, 1, 0, 1]
    out, stt = t.insert_alloc(p2, np.array([100, 101, 102, 103], dtype=np.uint64))
    # pushed 1, 3, 0 (in batch order) -> popped in reverse, then the fresh index 4
    assert out.tolist() == [0, 3, 1, 4]


def test_capacity_exhaustion():
    C = 37
    t = OracleTable(C, 64, HASH_MIX64, 8)
    keys = np.arange(1000, 1000 + C + 5, dtype=np.uint64)
    st_ = t.insert(keys, keys)
    assert st_.tolist() == [1] * C + [2] * 5
    assert t.size() == C and t.error() & 1
    # present keys still report PRESENT at capacity; repeats of a FULL key stay FULL
    st2 = t.insert(np.array([1000, 5000, 5000], dtype=np.uint64), np.zeros(3, np.uint64))
    assert st2.tolist() == [0, 2, 2]
    t0 = OracleTable(0, 64, HASH_MIX64, 1)
    assert t0.insert(np.array([1], dtype=np.uint64), np.array([1], np.uint64)).tolist() == [2]


def test_empty_table_and_reserved_patterns():
    t = OracleTable(16, 64, HASH_MIX64, 4)
    ks = np.array([0, U64MAX, U64MAX - 1, 1 << 63], dtype=np.uint64)
    out, fd = t.find(ks)
    assert fd.tolist() == [0] * 4 and out.tolist() == [U64MAX] * 4
    assert t.erase(ks).tolist() == [0] * 4
    assert t.insert(ks, ks).tolist() == [1] * 4
    out, fd = t.find(ks)
    assert fd.tolist() == [1] * 4 and out.tolist() == ks.tolist()
    t32 = OracleTable(4, 32, HASH_MIX64, 4)
    out, fd = t32.find(ks[:1])
    assert out.dtype == np.uint32 and int(out[0]) == (1 << 32) - 1


def test_results_do_not_depend_on_layout():
    rng = np.random.default_rng(3)
    base = rng.integers(0, 1 << 64, size=300, dtype=np.uint64)
    batches = [base[rng.integers(0, 300, size=500)] for _ in range(6)]
    ref = None
    for hk, nb in [(HASH_MIX64, 1), (HASH_MIX64, 7), (HASH_MIX64, 4096), (HASH_VOXEL21, 1 << 21),
                   (HASH_VOXEL21, 13)]:
        t = OracleTable(250, 64, hk, nb)
        res = []
        for j, b in enumerate(batches):
            if j % 3 == 0:
                res.append(t.insert(b, b ^ np.uint64(0xABCDEF)).tolist())
            elif j % 3 == 1:
                res.append([x.tolist() for x in t.find(b)])
            else:
                res.append(t.erase(b).tolist())
            _check(t)
        if ref is None:
            ref = res
        assert res == ref


def test_partitioned_baseline_equals_sequential_replay():
    """The multi-core timing baseline gives the sequential oracle's results (keys never interact,
    so splitting them by hash keeps every per-key history) while no partition fills up."""
    rng = np.random.default_rng(11)
    keys = rng.integers(0, 1 << 20, size=60000, dtype=np.uint64)   # many repeated keys
    vals = rng.integers(0, 1 << 62, size=keys.size, dtype=np.uint64)
    o = oracle.OracleTable(80000, 64)
    for parts in (1, 3, 8):
        p = oracle.PartitionedOracle(80000, parts)
        o.clear()
        np.testing.assert_array_equal(p.insert(keys, vals), o.insert(keys, vals))
        q = np.concatenate([keys[:3000], rng.integers(0, 1 << 20, size=3000, dtype=np.uint64)])
        (pv, pf), (ov, of) = p.find(q), o.find(q)
        np.testing.assert_array_equal(pf, of)
        np.testing.assert_array_equal(pv, ov)
        e = keys[rng.integers(0, keys.size, size=9000)]
        np.testing.assert_array_equal(p.erase(e), o.erase(e))
        assert p.size() == o.size()


# --------------------------------------------------------------------------------------------
# the invariant checker itself: each broken invariant must be reported by its own bit
# --------------------------------------------------------------------------------------------
# (kind of corruption, bits or_check must report): see or_corrupt / or_check in oracle.c
CORRUPTIONS = [
    (1, 1),        # size counter off by one
    (2, 2),        # a second copy of a live key on the same list
    (3, 4 | 8),    # an entry filed under another bucket: wrong list, and lookup misses it
    (4, 8),        # a cyclic list
    (5, 8),        # a link past the entry array
    (6, 16),       # a free entry dropped from the free list (leaked)
    (7, 16),       # an entry both live and free
]


def _populated(hash_kind, nb, cap=64, n=40, seed=0):
    rng = np.random.default_rng(seed)
    t = OracleTable(cap, 64, hash_kind, nb)
    if hash_kind == HASH_VOXEL21:
        keys = pack_int3(rng.integers(-9, 9, n), rng.integers(-9, 9, n), rng.integers(-9, 9, n))
    else:
        keys = rng.integers(0, 1 << 64, size=n, dtype=np.uint64)
    t.insert(keys, np.arange(n, dtype=np.uint64))
    return t


@pytest.mark.parametrize("hash_kind,nb", [(HASH_MIX64, 7), (HASH_MIX64, 64), (HASH_VOXEL21, 13)])
@pytest.mark.parametrize("kind,bits", CORRUPTIONS)
def test_checker_reports_each_broken_invariant(hash_kind, nb, kind, bits):
    t = _populated(hash_kind, nb)
    assert t.check() == (0, 0)
    assert t.corrupt(kind)
    bad, what = t.check()
    assert bad > 0 and what == bits, (kind, bad, what)


def _pool_valued(cap=32, pcap=48, n=20):
    t, p = OracleTable(cap, 32), OraclePool(pcap)
    rng = np.random.default_rng(3)
    t.insert_alloc(p, rng.integers(0, 1 << 64, size=n, dtype=np.uint64))
    return t, p


@pytest.mark.parametrize("kind", [8, 9])
def test_checker_reports_broken_pool_conservation(kind):
    """A duplicated pool index, or one dropped from the pool: the pool stack and the live values
    no longer partition the pool's indices (bit 32)."""
    t, p = _pool_valued()
    assert t.check(p, values_from_pool=True) == (0, 0)
    assert t.corrupt(kind, p)
    bad, what = t.check(p, values_from_pool=True)
    assert bad > 0 and what == 32, (kind, bad, what)


def test_checker_reports_a_value_not_taken_from_the_pool():
    """A live value overwritten with an index the pool still holds: that index is both free and
    in use (bit 32), while the map's own invariants hold."""
    t, p = _pool_valued()
    keys, vals = t.dump()
    t.erase(keys[:1])
    top = p.dump()[-1]          # an index still in the pool
    t.insert(keys[:1], np.array([top], dtype=np.uint64))
    bad, what = t.check(p, values_from_pool=True)
    assert what == 32 and bad > 0
    assert t.check()[1] == 0


def test_corruption_needs_room():
    """An empty table has no live entry to break: the hook says so instead of doing nothing."""
    t = OracleTable(8, 64, HASH_MIX64, 4)
    assert not t.corrupt(2) and not t.corrupt(3) and not t.corrupt(4)
    assert t.check() == (0, 0)
