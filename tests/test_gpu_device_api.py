"""GPU tests of the device-side per-thread operations (Section 4.1: container functions called
inside kernels, one element per thread; Section 4: operations running concurrently).

The kernels run every element at once and in no fixed order, so results are checked as sets plus
the invariants that any order gives: a key repeated across threads is stored once and INSERTED
by exactly one of them (whose value it keeps), a present key is erased by exactly one thread, the
final contents equal the oracle's after the same set of changes, and the live count and layout
invariants hold.  Reads are deterministic and compared element by element.
"""
import numpy as np
import pytest
import torch

import oracle
from paper_1908_05936_amd import ct
from paper_1908_05936_amd.workloads import distinct_u64, pack_int3, rng_for

pytestmark = pytest.mark.gpu

U64MAX = (1 << 64) - 1
RESERVED = np.array([0, U64MAX, U64MAX - 1, 1 << 63], dtype=np.uint64)


@pytest.fixture(scope="module")
def dev():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    ct.lib()
    return torch.device("cuda", 0)


def g64(a, dev):
    return torch.from_numpy(np.ascontiguousarray(np.asarray(a, dtype=np.uint64)).view(np.int64)).to(dev)


def dump_sorted(t, bits):
    k, v = t.dump()
    k = k.cpu().numpy().view(np.uint64)
    v = v.cpu().numpy().view(np.uint64)
    if bits == 32:
        v = v.astype(np.uint32)
    o = np.argsort(k, kind="stable")
    return k[o], v[o]


def same(t, o, bits):
    assert t.size() == o.size()
    k, v = dump_sorted(t, bits)
    ek, ev = o.dump()
    np.testing.assert_array_equal(k, ek)
    if bits:
        np.testing.assert_array_equal(v, ev)
    assert t.check() == 0


@pytest.mark.parametrize("bits", [64, 32, 0])
def test_concurrent_inserts_of_repeated_keys(dev, bits):
    """200,000 threads insert keys drawn from 6,000 (some already present, reserved-looking ones
    included): every new key is stored once and INSERTED by exactly one thread, whose value it
    keeps; every other thread sees PRESENT."""
    rng = rng_for(101, bits)
    vk = {0: ct.VAL_NONE, 32: ct.VAL_U32, 64: ct.VAL_U64}[bits]
    t = ct.Table(60_000, vk, device=dev)
    o = oracle.OracleTable(60_000, bits, oracle.HASH_MIX64, 60_000)
    base = distinct_u64(rng, 20_000)
    bv = rng.integers(0, 1 << 31, size=base.size, dtype=np.uint64)
    if bits:
        t.insert(g64(base, dev), torch.from_numpy(bv.astype(np.int64)).to(dev).to(t.value_dtype))
    else:
        t.insert(g64(base, dev))
    o.insert(base, bv if bits else None)
    universe = np.concatenate([base[:2000], distinct_u64(rng, 4000, exclude=base), RESERVED])
    keys = universe[rng.integers(0, universe.size, size=200_000)]
    vals = rng.integers(0, 1 << 31, size=keys.size, dtype=np.uint64)
    gv = None
    if bits:
        gv = torch.from_numpy(vals.astype(np.int64)).to(dev).to(t.value_dtype)
    st, _ = t.dev_apply(ct.OP_INSERT, g64(keys, dev), gv)
    st = st.cpu().numpy()
    assert not (st == 2).any()
    present_before = np.isin(keys, base)
    assert (st[present_before] == 0).all()
    new = ~present_before
    ins = np.flatnonzero(st == 1)
    # exactly one INSERTED per distinct new key
    assert np.unique(keys[ins]).size == ins.size
    assert set(keys[ins].tolist()) == set(keys[new].tolist())
    o.insert(keys[ins], vals[ins] if bits else None)
    same(t, o, bits)


def test_concurrent_erases_and_reads(dev):
    """Each present key is removed by exactly one of the threads that erase it; finds are
    element-by-element equal to the oracle's (reads only, so no ordering is involved)."""
    rng = rng_for(103)
    t = ct.Table(80_000, ct.VAL_U64, device=dev)
    o = oracle.OracleTable(80_000, 64, oracle.HASH_MIX64, 80_000)
    base = np.concatenate([distinct_u64(rng, 50_000), RESERVED[1:3]])
    bv = rng.integers(0, 1 << 62, size=base.size, dtype=np.uint64)
    t.insert(g64(base, dev), g64(bv, dev))
    o.insert(base, bv)
    q = np.concatenate([base[rng.integers(0, base.size, size=30_000)], distinct_u64(rng, 10_000)])
    st, v = t.dev_apply(ct.OP_FIND, g64(q, dev))
    ev, ef = o.find(q)
    np.testing.assert_array_equal(st.cpu().numpy(), ef)
    np.testing.assert_array_equal(v.cpu().numpy().view(np.uint64), ev)
    er = base[rng.integers(0, base.size, size=120_000)]
    st, _ = t.dev_apply(ct.OP_ERASE, g64(er, dev))
    st = st.cpu().numpy()
    hit = np.flatnonzero(st == 1)
    assert np.unique(er[hit]).size == hit.size
    assert set(er[hit].tolist()) == set(er.tolist())
    o.erase(np.unique(er))
    same(t, o, 64)
    # the batch path keeps working on a table the device functions changed
    again = distinct_u64(rng, 5000, exclude=base)
    t.insert(g64(again, dev), g64(again, dev))
    o.insert(again, again)
    same(t, o, 64)


def test_concurrent_inserts_at_capacity(dev):
    """A table 10 keys short of its capacity: of 5,000 new keys inserted at once exactly 10 get
    in (INSERTED), the rest report FULL, and the live count ends at the capacity."""
    rng = rng_for(107)
    cap = 4096
    t = ct.Table(cap, ct.VAL_U64, device=dev)
    base = distinct_u64(rng, cap - 10)
    t.insert(g64(base, dev), g64(base, dev))
    keys = distinct_u64(rng, 5000, exclude=base)
    st, _ = t.dev_apply(ct.OP_INSERT, g64(keys, dev), g64(keys, dev))
    st = st.cpu().numpy()
    assert (st == 1).sum() == 10 and (st == 2).sum() == keys.size - 10
    assert t.size() == cap and t.check() == 0
    k, v = dump_sorted(t, 64)
    assert set(k.tolist()) == set(base.tolist()) | set(keys[st == 1].tolist())
    np.testing.assert_array_equal(k, v)


@pytest.mark.parametrize("ndirs", [6, 26])
def test_voxel_neighbour_update(dev, ndirs):
    """The neighbour update of a block map: blocks of a dense cluster ask for their neighbours at
    once (most neighbours are asked for by several blocks).  The final key set is the residents
    plus the oracle's neighbour keys, residents keep their values, and each new block's value
    names a block whose neighbour it is."""
    rng = rng_for(109, ndirs)
    c = rng.integers(-40, 40, size=(30_000, 3))
    blocks = np.unique(pack_int3(c[:, 0], c[:, 1], c[:, 2]))
    rng.shuffle(blocks)
    t = ct.Table(1 << 20, ct.VAL_U32, ct.HASH_VOXEL21, bucket_count=1 << 17, device=dev)
    resid = blocks[: blocks.size // 2]
    t.insert(g64(resid, dev), torch.arange(resid.size, dtype=torch.int32, device=dev))
    t.insert_neighbours(g64(blocks, dev), ndirs)
    nbrs = oracle.voxel_neighbour_keys(blocks, ndirs)
    want = set(resid.tolist()) | set(nbrs.tolist())
    k, v = dump_sorted(t, 32)
    assert set(k.tolist()) == want and t.size() == len(want) and t.check() == 0
    pos = {x: i for i, x in enumerate(resid.tolist())}
    per_block = nbrs.reshape(blocks.size, ndirs)
    for key, val in zip(k.tolist(), v.tolist()):
        if key in pos:
            assert val == pos[key]
        else:
            assert 0 <= val < blocks.size and key in per_block[val].tolist()
    # the sequential definition gives the same key set
    o = oracle.OracleTable(1 << 20, 32, oracle.HASH_VOXEL21, 1 << 17)
    o.insert(resid, np.arange(resid.size, dtype=np.uint64))
    o.insert(nbrs, np.repeat(np.arange(blocks.size, dtype=np.uint64), ndirs))
    np.testing.assert_array_equal(k, o.dump()[0])


def test_device_pool_push_and_pop(dev):
    """push_back and pop_back from threads (Sections 4.2-4.3) on a pool whose head has moved: the
    pops together take the pool's last entries (compared as a multiset with the oracle's pops),
    pushes store every value while there is room (compared as multisets), a push beyond the
    capacity stores exactly the room and sets the pool error."""
    rng = rng_for(113)
    cap = 100_000
    gp = ct.Pool(cap, device=dev)
    op = oracle.OraclePool(cap)
    out, _ = gp.pop_front(12_345)
    op.pop_front(12_345)
    got, st = gp.dev_pop_back(30_000)
    eo, es = op.pop(30_000)
    assert (st.cpu().numpy() == 1).all()
    np.testing.assert_array_equal(np.sort(got.cpu().numpy()), np.sort(eo))
    assert gp.size() == op.size()
    np.testing.assert_array_equal(gp.dump().cpu().numpy(), op.dump())
    vals = rng.permutation(np.arange(1_000_000, 1_040_000, dtype=np.int32))
    st = gp.dev_push_back(torch.from_numpy(vals).to(dev))
    assert (st.cpu().numpy() == 1).all()
    op.push(vals)
    assert gp.size() == op.size()
    np.testing.assert_array_equal(np.sort(gp.dump().cpu().numpy()), np.sort(op.dump()))
    room = cap - gp.size()
    more = np.arange(5_000_000, 5_000_000 + room + 777, dtype=np.int32)
    st = gp.dev_push_back(torch.from_numpy(more).to(dev)).cpu().numpy()
    assert (st == 1).sum() == room and (st == 2).sum() == 777
    assert gp.size() == cap and gp.error() & ct.ERR_POOL
    stored = set(gp.dump().cpu().numpy().tolist()) & set(more.tolist())
    assert stored == set(more[st == 1].tolist())
    got, st = gp.dev_pop_back(cap + 50)
    st = st.cpu().numpy()
    assert (st == 1).sum() == cap and gp.size() == 0


def test_voxel_neighbour_update_with_pool(dev):
    """The neighbour update allocating from the index pool: new blocks take pool indices, so the
    residents' values, the new blocks' values and the pool's remaining entries partition
    0 .. capacity - 1 exactly, and the key set is the residents plus the oracle's neighbours."""
    rng = rng_for(127)
    c = rng.integers(-30, 30, size=(20_000, 3))
    blocks = np.unique(pack_int3(c[:, 0], c[:, 1], c[:, 2]))
    rng.shuffle(blocks)
    cap = 1 << 19
    t = ct.Table(cap, ct.VAL_U32, ct.HASH_VOXEL21, bucket_count=1 << 16, device=dev)
    pool = ct.Pool(cap, device=dev)
    resid = blocks[: blocks.size // 2]
    t.insert_alloc(pool, g64(resid, dev))
    t.insert_neighbours_alloc(pool, g64(blocks, dev), 26)
    want = set(resid.tolist()) | set(oracle.voxel_neighbour_keys(blocks, 26).tolist())
    k, v = dump_sorted(t, 32)
    assert set(k.tolist()) == want and t.size() == len(want) and t.check() == 0
    left = pool.dump().cpu().numpy()
    allv = np.concatenate([v.astype(np.int64), left.astype(np.int64)])
    np.testing.assert_array_equal(np.sort(allv), np.arange(cap))
    assert pool.size() == cap - len(want)


@pytest.mark.parametrize("bits", [64, 32, 0])
def test_mixed_operations_in_one_kernel(dev, bits):
    """Inserts, erases and finds in one kernel, the same key under several operations included
    (Section 4: concurrency across all operations).  Per key, the INSERTED results and the
    successful erases must alternate from the key's state before the kernel; that fixes which
    keys are live afterwards, and the oracle, given the same changes in an order the statuses
    allow, must then hold the same contents.  Keys touched by one operation kind only are checked
    element by element."""
    rng = rng_for(107, bits)
    vk = {0: ct.VAL_NONE, 32: ct.VAL_U32, 64: ct.VAL_U64}[bits]
    cap = 200_000
    t = ct.Table(cap, vk, device=dev)
    o = oracle.OracleTable(cap, bits, oracle.HASH_MIX64, cap)
    base = np.concatenate([distinct_u64(rng, 60_000), np.array([U64MAX - 1], np.uint64)])
    bv = rng.integers(0, 1 << 31, size=base.size, dtype=np.uint64)
    if bits:
        t.insert(g64(base, dev), torch.from_numpy(bv.astype(np.int64)).to(dev).to(t.value_dtype))
    else:
        t.insert(g64(base, dev))
    o.insert(base, bv if bits else None)
    orig = dict(zip(base.tolist(), bv.tolist()))
    fresh = np.concatenate([distinct_u64(rng, 40_000, exclude=base), np.array([U64MAX], np.uint64)])
    rng.shuffle(base[:-1])
    P = {"A": base[:8000], "A2": base[8000:12000], "C": base[12000:20000], "E": base[20000:24000],
         "H": np.concatenate([base[24000:26000], base[-1:]])}
    Q = {"B": fresh[:8000], "D": fresh[8000:12000], "H": np.concatenate([fresh[12000:14000], fresh[-1:]]),
         "F": fresh[14000:20000]}
    I, F, E = ct.OP_INSERT, ct.OP_FIND, ct.OP_ERASE
    plan = [(P["A"], [E]), (P["A2"], [E, E, E]), (P["C"], [F, F]), (P["E"], [E, I]),
            (P["H"], [I] * 4 + [E] * 4 + [F] * 2), (Q["B"], [I, I, I]), (Q["D"], [I, E]),
            (Q["H"], [I] * 4 + [E] * 4 + [F] * 2), (Q["F"], [F, E])]
    keys = np.concatenate([np.repeat(k, len(ops)) for k, ops in plan])
    ops = np.concatenate([np.tile(np.array(ops, np.uint8), k.size) for k, ops in plan])
    vals = rng.integers(0, 1 << 31, size=keys.size, dtype=np.uint64)
    perm = rng.permutation(keys.size)
    keys, ops, vals = keys[perm], ops[perm], vals[perm]
    gv = torch.from_numpy(vals.astype(np.int64)).to(dev).to(t.value_dtype) if bits else None
    st, out = t.dev_apply_mixed(torch.from_numpy(ops).to(dev), g64(keys, dev), gv)
    st = st.cpu().numpy()
    if bits:
        out = out.cpu().numpy().view(np.uint64 if bits == 64 else np.uint32).astype(np.uint64)
        sentinel = U64MAX if bits == 64 else 0xFFFFFFFF
        assert (out[ops != F] == sentinel).all()
    assert not (st[ops == I] == 2).any()
    assert set(np.unique(st).tolist()) <= {0, 1}
    group = {}
    for name, ks in list(P.items()) + list(Q.items()):
        for k in ks.tolist():
            group[k] = name
    by_key = {}
    for j, k in enumerate(keys.tolist()):
        by_key.setdefault(k, []).append(j)
    live_after, new_val = {}, {}
    for k, js in by_key.items():
        g = group[k]
        was = k in orig
        ins = [j for j in js if ops[j] == I and st[j] == 1]
        hits = [j for j in js if ops[j] == E and st[j] == 1]
        finds = [j for j in js if ops[j] == F]
        if g in ("A", "A2"):
            assert len(hits) == 1, (g, k)
        elif g == "C":
            assert all(st[j] == 1 for j in finds)
            if bits:
                assert all(out[j] == orig[k] for j in finds)
        elif g == "F":
            assert not st[js].any()
            if bits:
                assert all(out[j] == sentinel for j in finds)
        elif g == "B":
            assert len(ins) == 1
        elif g == "D":
            assert len(ins) == 1
        elif g == "E":
            assert len(hits) == 1
        # alternation from the state before the kernel
        d = len(ins) - len(hits)
        assert d in ((-1, 0) if was else (0, 1)), (g, k, len(ins), len(hits))
        live_after[k] = (was and d == 0) or (not was and d == 1)
        if live_after[k] and ins:
            new_val[k] = [vals[j] for j in ins]
    # the oracle gets the same changes: every touched key erased, then the live ones inserted
    touched = np.array(sorted(by_key), dtype=np.uint64)
    o.erase(touched)
    live = [k for k in by_key if live_after[k]]
    lv = [(new_val[k][0] if k in new_val else orig[k]) for k in live]
    o.insert(np.array(live, np.uint64), np.array(lv, np.uint64) if bits else None)
    assert t.size() == o.size()
    k, v = dump_sorted(t, bits)
    ek, ev = o.dump()
    np.testing.assert_array_equal(k, ek)
    if bits:
        # a key inserted several times keeps the value of one of its INSERTED elements
        ambiguous = np.array([kk in new_val and len(new_val[kk]) > 1 for kk in k.tolist()], bool)
        np.testing.assert_array_equal(v[~ambiguous], ev[~ambiguous])
        mask = (1 << bits) - 1
        for kk, vv in zip(k[ambiguous].tolist(), v[ambiguous].tolist()):
            assert vv in [x & mask for x in new_val[kk]]
    assert t.check() == 0
    # the batch path reuses the tombstones the kernel left
    again = distinct_u64(rng, 20_000, exclude=np.concatenate([base, fresh]))
    av = again & np.uint64(0x7FFFFFFF)
    if bits:
        t.insert(g64(again, dev), torch.from_numpy(av.astype(np.int64)).to(dev).to(t.value_dtype))
    else:
        t.insert(g64(again, dev))
    o.insert(again, av if bits else None)
    same_keys = dump_sorted(t, bits)[0]
    np.testing.assert_array_equal(same_keys, o.dump()[0])
    assert t.size() == o.size() and t.check() == 0


def test_mixed_operations_at_capacity(dev):
    """Erases and inserts of distinct keys in one kernel on a table at capacity: every erase hits,
    the live count never passes the capacity, exactly the INSERTED keys join the table and FULL
    ones stay out; at least the room left before the kernel is granted."""
    rng = rng_for(109)
    cap = 4096
    t = ct.Table(cap, ct.VAL_U64, device=dev)
    base = distinct_u64(rng, 4000)
    t.insert(g64(base, dev), g64(base, dev))
    er = base[:1000]
    new = distinct_u64(rng, 3000, exclude=base)
    keys = np.concatenate([er, new])
    ops = np.concatenate([np.full(er.size, ct.OP_ERASE, np.uint8), np.full(new.size, ct.OP_INSERT, np.uint8)])
    perm = rng.permutation(keys.size)
    keys, ops = keys[perm], ops[perm]
    st, _ = t.dev_apply_mixed(torch.from_numpy(ops).to(dev), g64(keys, dev), g64(keys, dev))
    st = st.cpu().numpy()
    assert (st[ops == ct.OP_ERASE] == 1).all()
    si = st[ops == ct.OP_INSERT]
    assert set(np.unique(si).tolist()) <= {1, 2}
    inserted = keys[ops == ct.OP_INSERT][si == 1]
    assert cap - base.size <= inserted.size <= cap - base.size + er.size
    expect = np.sort(np.concatenate([base[1000:], inserted]))
    k, v = dump_sorted(t, 64)
    np.testing.assert_array_equal(k, expect)
    np.testing.assert_array_equal(v, expect)
    assert t.size() == expect.size <= cap
    assert t.check() == 0


@pytest.mark.parametrize("copies,spread", [(3, True), (64, False)])
def test_mixed_mode_repeated_inserts(dev, copies, spread):
    """Inserts only, in the mixed mode: an inserter that loses its slot to another key and then
    meets its own key further on reports PRESENT (not FULL); each key is INSERTED exactly once.
    Copies spread over the launch, or side by side in one wavefront."""
    rng = rng_for(113, copies)
    t = ct.Table(200_000, ct.VAL_U64, device=dev)
    base = distinct_u64(rng, 60_000)
    t.insert(g64(base, dev), g64(base, dev))
    fresh = distinct_u64(rng, 8000, exclude=base)
    keys = np.repeat(fresh, copies)
    if spread:
        rng.shuffle(keys)
    ops = torch.full((keys.size,), ct.OP_INSERT, dtype=torch.uint8, device=dev)
    st, _ = t.dev_apply_mixed(ops, g64(keys, dev), g64(keys, dev))
    st = st.cpu().numpy()
    assert set(np.unique(st).tolist()) <= {0, 1}
    ins = keys[st == 1]
    assert ins.size == fresh.size and np.unique(ins).size == fresh.size
    k, v = dump_sorted(t, 64)
    expect = np.sort(np.concatenate([base, fresh]))
    np.testing.assert_array_equal(k, expect)
    np.testing.assert_array_equal(v, expect)
    assert t.check() == 0


def test_mixed_mode_unknown_op_codes(dev):
    """An element whose operation code is none of insert / find / erase reports 255 and leaves the
    table alone; the other elements of the same launch run as usual."""
    rng = rng_for(127)
    t = ct.Table(10_000, ct.VAL_U64, device=dev)
    base = distinct_u64(rng, 3000)
    t.insert(g64(base, dev), g64(base, dev))
    keys = np.concatenate([base[:1000], distinct_u64(rng, 1000, exclude=base)])
    ops = np.full(keys.size, 7, np.uint8)
    ops[::2] = ct.OP_FIND
    st, out = t.dev_apply_mixed(torch.from_numpy(ops).to(dev), g64(keys, dev), g64(keys, dev))
    st = st.cpu().numpy()
    out = out.cpu().numpy().view(np.uint64)
    assert (st[ops == 7] == 255).all()
    found = np.isin(keys, base)
    np.testing.assert_array_equal(st[ops == ct.OP_FIND], found[ops == ct.OP_FIND].astype(np.uint8))
    hit = (ops == ct.OP_FIND) & found
    np.testing.assert_array_equal(out[hit], keys[hit])
    assert (out[~hit] == U64MAX).all()
    assert t.size() == base.size and t.check() == 0
    np.testing.assert_array_equal(dump_sorted(t, 64)[0], np.sort(base))


@pytest.mark.parametrize("n", [1 << 17, (1 << 17) + 37])
def test_device_finds_at_full_load(dev, n):
    """Finds through the device functions on a table filled to capacity (load 0.8, so many probes
    run past their home bucket), element by element against the oracle.  Whole wavefronts probe
    together; a ragged tail probes lane by lane."""
    rng = rng_for(131, n)
    cap = 100_000
    t = ct.Table(cap, ct.VAL_U64, device=dev)
    o = oracle.OracleTable(cap, 64, oracle.HASH_MIX64, cap)
    base = distinct_u64(rng, cap)
    bv = rng.integers(0, 1 << 63, size=cap, dtype=np.uint64)
    t.insert(g64(base, dev), g64(bv, dev))
    o.insert(base, bv)
    assert t.size() == cap
    q = np.concatenate([base[rng.integers(0, cap, size=n - n // 4)],
                        distinct_u64(rng, n // 4, exclude=base)])
    rng.shuffle(q)
    st, v = t.dev_apply(ct.OP_FIND, g64(q, dev))
    ev, ef = o.find(q)
    np.testing.assert_array_equal(st.cpu().numpy(), ef)
    np.testing.assert_array_equal(v.cpu().numpy().view(np.uint64), ev)
    # erases of half the keys through the device functions, then the finds again
    er = base[: cap // 2]
    est, _ = t.dev_apply(ct.OP_ERASE, g64(er, dev))
    assert (est.cpu().numpy() == 1).all()
    o.erase(er)
    st, v = t.dev_apply(ct.OP_FIND, g64(q, dev))
    ev, ef = o.find(q)
    np.testing.assert_array_equal(st.cpu().numpy(), ef)
    np.testing.assert_array_equal(v.cpu().numpy().view(np.uint64), ev)
    same(t, o, 64)


@pytest.mark.parametrize("set_bits", [0, 64])
def test_two_container_update_set(dev, set_bits):
    """The two-container step of Section 4.1's reconstruction example in one kernel: each thread
    asks the block map whether its key is there and inserts it into the update set.  Threads
    repeat keys; some keys are in the set already; out-of-band bit patterns included.  The set
    must end as its old keys plus the queried keys the map holds, each new key INSERTED by
    exactly one of its elements, elements of keys the map lacks reporting 255."""
    rng = rng_for(77)
    resident = np.concatenate([RESERVED[:3], distinct_u64(rng, 20000)])
    absent = distinct_u64(rng, 5000, exclude=resident)
    q = np.concatenate([resident[rng.integers(0, resident.size, 150000)],
                        absent[rng.integers(0, absent.size, 50000)], RESERVED])
    q = q[rng.permutation(q.size)]
    pre = np.concatenate([resident[:3000:3], absent[:100]])     # already in the set
    vk = ct.VAL_NONE if set_bits == 0 else ct.VAL_U64
    a = ct.Table(1 << 15, ct.VAL_U32, ct.HASH_MIX64, device=dev)
    a.insert(g64(resident, dev), torch.arange(resident.size, dtype=torch.int32, device=dev))
    b = ct.Table(1 << 15, vk, ct.HASH_MIX64, device=dev)
    b.insert(g64(pre, dev), None if vk == ct.VAL_NONE else g64(np.zeros(pre.size, np.uint64), dev))
    st = a.dev_update_set(b, g64(q, dev)).cpu().numpy()
    oa = oracle.OracleTable(1 << 15, 32)
    oa.insert(resident, np.arange(resident.size, dtype=np.uint32))
    _, in_map = oa.find(q)
    np.testing.assert_array_equal(st == 255, in_map == 0)
    ob = oracle.OracleTable(1 << 15, set_bits)
    ob.insert(pre, None if set_bits == 0 else np.zeros(pre.size, np.uint64))
    new_keys = np.setdiff1d(np.unique(q[in_map == 1]), pre)
    for key in np.unique(q[in_map == 1]):
        s = st[q == key]
        if key in new_keys:
            assert (s == ct.INSERTED).sum() == 1 and (s == ct.PRESENT).sum() == s.size - 1, key
        else:
            assert (s == ct.PRESENT).all(), key
    ob.insert(np.unique(q[in_map == 1]), None if set_bits == 0 else
              np.zeros(np.unique(q[in_map == 1]).size, np.uint64))
    same(b, ob, set_bits)
    assert a.check() == 0
