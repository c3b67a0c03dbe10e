"""GPU parity: every output of the HIP library equals the CPU oracle's, element by element.

All cases call through the C ABI (the ctypes binding in paper_1908_05936_amd.ct).  Integer
results, so the bar is bit-exact.  Sizes span many 128-byte buckets, several dedup chunks and
rank tiles, and ragged tails.
"""
import numpy as np
import pytest
import torch

import oracle
from paper_1908_05936_amd import ct
from paper_1908_05936_amd.workloads import distinct_u64, pack_int3, plain_table, rng_for

pytestmark = pytest.mark.gpu

U64MAX = (1 << 64) - 1
RESERVED = np.array([0, U64MAX, U64MAX - 1, 1 << 63, U64MAX - 2], dtype=np.uint64)


@pytest.fixture(scope="module")
def dev():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    ct.lib()
    return torch.device("cuda", 0)


def g64(a, dev):
    return torch.from_numpy(np.ascontiguousarray(np.asarray(a, dtype=np.uint64)).view(np.int64)).to(dev)


def g32(a, dev):
    return torch.from_numpy(np.ascontiguousarray(np.asarray(a).astype(np.uint32)).view(np.int32)).to(dev)


def npu(t, bits=64):
    a = t.cpu().numpy()
    return a.view(np.uint64) if bits == 64 else a.view(np.uint32)


class Pair:
    """A GPU table and an oracle table driven with the same batches; every output is compared."""

    def __init__(self, dev, capacity, bits=64, hash_kind=ct.HASH_MIX64, bucket_count=0, chunk=0,
                 pool=None, path=ct.INSERT_AUTO):
        vk = {0: ct.VAL_NONE, 32: ct.VAL_U32, 64: ct.VAL_U64}[bits]
        self.dev, self.bits = dev, bits
        self.g = ct.Table(capacity, vk, hash_kind, bucket_count, chunk, device=dev)
        self.g.set_insert_path(path)
        self.o = oracle.OracleTable(capacity, bits, hash_kind, bucket_count or max(1, capacity))
        self.gp = ct.Pool(pool, device=dev) if pool is not None else None
        self.op = oracle.OraclePool(pool) if pool is not None else None

    def insert(self, keys, vals=None):
        keys = np.asarray(keys, dtype=np.uint64)
        if self.bits == 0:
            st = self.g.insert(g64(keys, self.dev))
        elif self.bits == 32:
            st = self.g.insert(g64(keys, self.dev), g32(vals, self.dev))
        else:
            st = self.g.insert(g64(keys, self.dev), g64(vals, self.dev))
        exp = self.o.insert(keys, vals)
        np.testing.assert_array_equal(st.cpu().numpy(), exp)
        return exp

    def find(self, keys):
        keys = np.asarray(keys, dtype=np.uint64)
        v, f = self.g.find(g64(keys, self.dev))
        ev, ef = self.o.find(keys)
        np.testing.assert_array_equal(f.cpu().numpy(), ef)
        if self.bits:
            np.testing.assert_array_equal(npu(v, self.bits), ev)
        return ev, ef

    def erase(self, keys):
        keys = np.asarray(keys, dtype=np.uint64)
        er = self.g.erase(g64(keys, self.dev))
        exp = self.o.erase(keys)
        np.testing.assert_array_equal(er.cpu().numpy(), exp)
        return exp

    def insert_alloc(self, keys):
        keys = np.asarray(keys, dtype=np.uint64)
        v, st = self.g.insert_alloc(self.gp, g64(keys, self.dev))
        ev, es = self.o.insert_alloc(self.op, keys)
        np.testing.assert_array_equal(st.cpu().numpy(), es)
        np.testing.assert_array_equal(v.cpu().numpy(), ev)

    def erase_release(self, keys):
        keys = np.asarray(keys, dtype=np.uint64)
        er = self.g.erase_release(self.gp, g64(keys, self.dev))
        np.testing.assert_array_equal(er.cpu().numpy(), self.o.erase_release(self.op, keys))

    def same_state(self):
        assert self.g.size() == self.o.size()
        k, v = self.g.dump()
        k = npu(k)
        v = npu(v)
        order = np.argsort(k, kind="stable")
        ek, ev = self.o.dump()
        np.testing.assert_array_equal(k[order], ek)
        if self.bits:
            np.testing.assert_array_equal(v[order], ev.astype(np.uint64))
        assert self.g.check() == 0
        if self.gp is not None:
            np.testing.assert_array_equal(self.gp.dump().cpu().numpy(), self.op.dump())


def test_plain_table_workload(dev):
    """u64 keys / u32 values: 2^16 inserts at capacity 2^17, 50/50 find, 25 % erase, final find."""
    w = plain_table(seed=1)
    p = Pair(dev, w["capacity"], 32)
    assert (p.insert(w["insert_keys"], w["insert_vals"]) == 1).all()
    p.same_state()
    p.find(w["find1"])
    p.erase(w["erase"])
    _, f = p.find(w["find2"])
    assert int(f.sum()) == 49152
    p.same_state()


PATHS = [ct.INSERT_SPECULATIVE, ct.INSERT_RESOLVE_FIRST]


@pytest.mark.parametrize("path", PATHS)
@pytest.mark.parametrize("bits", [0, 32, 64])
@pytest.mark.parametrize("chunk", [0, 1024])
def test_duplicates_and_reserved_keys(dev, bits, chunk, path):
    rng = rng_for(11, bits + chunk)
    universe = np.concatenate([distinct_u64(rng, 3000), RESERVED])
    p = Pair(dev, 8000, bits, chunk=chunk, path=path)
    for step in range(9):
        n = [1, 7, 1023, 1025, 4099, 20000, 3, 12345, 2048][step]
        keys = universe[rng.integers(0, universe.size, size=n)]
        vals = rng.integers(0, 1 << 63, size=n, dtype=np.uint64)
        kind = step % 3
        if kind == 0:
            p.insert(keys, vals & np.uint64(0xFFFFFFFF) if bits == 32 else vals)
        elif kind == 1:
            p.find(keys)
        else:
            p.erase(keys[: n // 2])
        p.same_state()


@pytest.mark.parametrize("chunk", [0, 1024])
def test_capacity_exhaustion(dev, chunk):
    rng = rng_for(12, chunk)
    C = 3000
    p = Pair(dev, C, 64, chunk=chunk)
    keys = distinct_u64(rng, 5000)
    batch = np.concatenate([keys[:2000], keys[:500], keys[2000:5000], RESERVED])
    batch = batch[rng.permutation(batch.size)]
    st = p.insert(batch, rng.integers(0, 1 << 63, size=batch.size, dtype=np.uint64))
    assert (st == 2).any()
    p.same_state()
    assert p.g.error() & ct.ERR_FULL
    p.erase(keys[:1000])
    p.insert(keys[3000:4500], np.arange(1500, dtype=np.uint64))
    p.same_state()


def test_empty_and_degenerate(dev):
    p = Pair(dev, 100, 64)
    empty = np.zeros(0, dtype=np.uint64)
    p.insert(empty, empty)
    p.find(empty)
    p.erase(empty)
    p.find(RESERVED)       # empty table: sentinels
    p.erase(RESERVED)
    p.same_state()
    same = np.full(5000, 12345, dtype=np.uint64)   # one key, maximum contention
    p.insert(same, np.arange(5000, dtype=np.uint64))
    p.find(same[:10])
    p.erase(same)
    p.same_state()
    z = Pair(dev, 0, 32)  # capacity 0: every insert is FULL
    z.insert(np.array([1, 2, 1], dtype=np.uint64), np.array([1, 2, 3]))
    z.same_state()


def test_clear_then_reuse(dev):
    """clear empties the table (out-of-band keys included) and ends a skew hint; the cleared
    table then behaves as a new one, compared with a cleared oracle table.  The sticky error word
    survives clear until it is read."""
    rng = rng_for(29)
    chunk = 1 << 16
    # repeated keys resolved first (through the bins): the skew hint comes from that path
    p = Pair(dev, 1 << 18, 64, chunk=chunk, path=ct.INSERT_RESOLVE_FIRST)
    hot = np.full(chunk, 4242, dtype=np.uint64)      # overflows its bins: sets the skew hint
    hot[::7] = distinct_u64(rng, hot[::7].size)
    p.insert(np.concatenate([hot, RESERVED]), np.arange(chunk + RESERVED.size, dtype=np.uint64))
    assert p.g.dedup_skewed()
    p.g.clear()
    p.o.clear()
    assert p.g.size() == 0 and not p.g.dedup_skewed()
    p.find(np.concatenate([hot[:100], RESERVED]))
    p.same_state()
    keys = distinct_u64(rng, 3 * chunk + 11)
    p.insert(keys, np.arange(keys.size, dtype=np.uint64))
    p.erase(keys[::5])
    p.find(keys[:5000])
    p.same_state()
    small = Pair(dev, 4, 64)
    small.insert(distinct_u64(rng, 6), np.arange(6, dtype=np.uint64))   # two are FULL
    small.g.clear()
    small.o.clear()
    assert small.g.error() & ct.ERR_FULL     # kept through clear, cleared by reading it
    assert small.g.error() == 0
    small.insert(distinct_u64(rng, 4), np.arange(4, dtype=np.uint64))
    small.same_state()


@pytest.mark.parametrize("bits,hash_kind", [(64, ct.HASH_MIX64), (32, ct.HASH_VOXEL21),
                                             (0, ct.HASH_MIX64)])
def test_rehash_resize_snapshot_restore(dev, bits, hash_kind):
    """Host-side resizing: every live pair of a table goes into another one (a larger new table,
    or one that already holds some of the keys, which keep their value there).  The oracle side is
    the definition: its own dump inserted into its destination.  The source stays unchanged, both
    tables keep working afterwards, a destination without room is refused before anything runs,
    and a snapshot restores a table's exact contents."""
    rng = rng_for(37, bits)
    vb = 32 if bits == 32 else 64

    def vals(n):
        return rng.integers(0, 1 << vb, size=n, dtype=np.uint64) if bits else None

    src = Pair(dev, 50_000, bits, hash_kind=hash_kind, chunk=1 << 12)
    keys = distinct_u64(rng, 40_000)
    keys[:4] = RESERVED[:4]
    src.insert(keys, vals(keys.size))
    src.erase(keys[::3])
    src.insert(keys[::6], vals(keys[::6].size))
    src.same_state()
    dst = Pair(dev, 120_000, bits, hash_kind=hash_kind)
    other = np.concatenate([keys[1::5], distinct_u64(rng, 20_000), RESERVED[1:3]])
    dst.insert(other, vals(other.size))
    src.g.rehash_into(dst.g)
    ok, ov = src.o.dump()
    dst.o.insert(ok, ov if bits else None)
    dst.same_state()
    src.same_state()
    fresh = distinct_u64(rng, 30_000, exclude=np.concatenate([keys, other]))
    dst.insert(fresh, vals(fresh.size))
    dst.erase(np.concatenate([keys[::7], fresh[::2]]))
    dst.find(np.concatenate([keys, fresh[:1000]]))
    dst.same_state()
    src.erase(keys[::2])
    src.same_state()
    big = Pair(dev, 1 << 17, bits, hash_kind=hash_kind)
    big.g = src.g.resized(1 << 17)                      # a new, larger table with src's pairs
    k2, v2 = src.o.dump()
    big.o.insert(k2, v2 if bits else None)
    big.same_state()
    with pytest.raises(ct.CtError, match="capacity exhausted"):   # no room: refused
        dst.g.rehash_into(Pair(dev, 100, bits, hash_kind=hash_kind).g)
    if bits:
        with pytest.raises(ct.CtError):                 # value kinds differ
            src.g.rehash_into(ct.Table(1 << 17, ct.VAL_NONE, device=dev))
    snap_k, snap_v = src.g.snapshot()
    ek, ev = src.o.dump()
    src.insert(fresh[:5000], vals(5000))
    src.g.restore(snap_k, snap_v if bits else None)
    src.o.clear()
    src.o.insert(ek, ev if bits else None)
    src.same_state()
    src.find(np.concatenate([keys[:3000], fresh[:3000]]))


@pytest.mark.parametrize("nb", [1, 37, 1 << 10])
def test_full_physical_table_and_wraparound(dev, nb):
    """Capacity equal to every physical slot: probes wrap around the bucket array."""
    rng = rng_for(13, nb)
    C = 8 * nb
    p = Pair(dev, C, 64, bucket_count=nb)
    keys = distinct_u64(rng, C + 10)
    p.insert(keys, np.arange(keys.size, dtype=np.uint64))
    p.find(keys)
    p.erase(keys[::3])
    p.insert(keys[::3][::-1], np.arange(keys[::3].size, dtype=np.uint64))
    p.same_state()


@pytest.mark.parametrize("nb", [1 << 12, 1000])
def test_voxel_hash_table(dev, nb):
    rng = rng_for(14, nb)
    xyz = rng.integers(-50, 50, size=(20000, 3))
    from paper_1908_05936_amd.workloads import pack_int3

    keys = pack_int3(xyz[:, 0], xyz[:, 1], xyz[:, 2])
    p = Pair(dev, 8 * nb, 32, hash_kind=ct.HASH_VOXEL21, bucket_count=nb)
    p.insert(keys, np.arange(keys.size) % 1000)
    p.find(keys[::-1])
    p.erase(keys[:5000])
    p.same_state()


@pytest.mark.parametrize("pool_cap", [50000, 2000])
def test_alloc_and_release(dev, pool_cap):
    rng = rng_for(15, pool_cap)
    universe = np.concatenate([distinct_u64(rng, 8000), RESERVED])
    p = Pair(dev, 6000, 32, pool=pool_cap)
    for step in range(10):
        keys = universe[rng.integers(0, universe.size, size=int(rng.integers(1, 6000)))]
        if step % 2 == 0:
            p.insert_alloc(keys)
        else:
            p.erase_release(keys[: keys.size // 2])
        p.find(keys[:100])
        p.same_state()


def test_pool_stack(dev):
    gp = ct.Pool(1000, device=dev)
    op = oracle.OraclePool(1000)
    out, st = gp.pop(300)
    eo, es = op.pop(300)
    np.testing.assert_array_equal(out.cpu().numpy(), eo)
    np.testing.assert_array_equal(st.cpu().numpy(), es)
    vals = np.arange(5000, 5500, dtype=np.int32)
    st = gp.push(torch.from_numpy(vals).to(dev))
    np.testing.assert_array_equal(st.cpu().numpy(), op.push(vals))
    out, st = gp.pop(1500)
    eo, es = op.pop(1500)
    np.testing.assert_array_equal(out.cpu().numpy(), eo)
    np.testing.assert_array_equal(st.cpu().numpy(), es)
    assert gp.size() == op.size() == 0
    assert gp.error() & ct.ERR_POOL


def _sorted_pairs(k, v, bits):
    k = npu(k)
    v = npu(v) if bits == 64 else npu(v).astype(np.uint32)
    o = np.argsort(k, kind="stable")
    return k[o], v[o]


def test_range_selection(dev):
    """Range selection (Section 3.6): live pairs by key interval on a mix64 map and by block box
    on a voxel21 map, in unspecified order, compared as sorted sets with the oracle's selection;
    the out-of-band keys take part, and a short output buffer gets the full count and a subset."""
    rng = rng_for(47)
    p = Pair(dev, 200_000, 64)
    keys = distinct_u64(rng, 150_000)
    keys[:5] = RESERVED
    p.insert(keys, rng.integers(0, 1 << 62, size=keys.size, dtype=np.uint64))
    p.erase(keys[::4])
    q = np.sort(keys)
    for lo, hi in [(0, U64MAX), (int(q[1000]), int(q[90_000])), (int(q[5]), int(q[5]) + 1),
                   (U64MAX - 2, U64MAX), (0, 1), (1 << 63, U64MAX), (7, 7)]:
        gk, gv = p.g.select_key_range(lo, hi)
        ek, ev = p.o.select_key_range(lo, hi)
        k, v = _sorted_pairs(gk, gv, 64)
        np.testing.assert_array_equal(k, ek)
        np.testing.assert_array_equal(v, ev)
    L = ct.lib()
    kout = torch.empty(100, dtype=torch.int64, device=dev)
    cnt = ct.C.c_int64(0)
    ct._check(L.ct_select_key_range(p.g._h, 0, U64MAX, ct._ptr(kout), None, 100, ct.C.byref(cnt),
                                    ct._stream(dev)), "select")
    assert cnt.value == p.o.size() - (1 if p.o.find(np.array([U64MAX], np.uint64))[1][0] else 0)
    assert set(npu(kout).tolist()) <= set(keys.tolist())
    vox = Pair(dev, 300_000, 32, hash_kind=ct.HASH_VOXEL21, bucket_count=1 << 16)
    c = rng.integers(-300, 300, size=(250_000, 3))
    vk = np.unique(pack_int3(c[:, 0], c[:, 1], c[:, 2]))
    vox.insert(vk, np.arange(vk.size, dtype=np.uint32))
    vox.insert(np.array([U64MAX, 1 << 63], dtype=np.uint64), np.array([1, 2], dtype=np.uint32))
    for lo3, hi3 in [((-50, -60, -70), (40, 30, 20)), ((-300, -300, -300), (300, 300, 300)),
                     ((0, 0, 0), (0, 0, 0)), ((10, 10, 10), (5, 50, 50)), ((-1, -1, -1), (-1, -1, -1))]:
        gk, gv = vox.g.select_voxel_box(lo3, hi3)
        ek, ev = vox.o.select_voxel_box(lo3, hi3)
        k, v = _sorted_pairs(gk, gv, 32)
        np.testing.assert_array_equal(k, ek)
        np.testing.assert_array_equal(v, ev)


@pytest.mark.parametrize("pcap", [1, 1000, 70_001])
def test_pool_deque_front_and_back(dev, pcap):
    """The pool's four deque operations (Section 4.3) in random batches, each compared with the
    oracle pool (values, statuses, size, front-to-back contents, the sticky error).  Front
    operations move the ring's head, so later back operations and the table's pool-valued insert
    and release wrap around the end of the buffer; used as a FIFO free list (pop_front, then
    push_back of released values) the pool keeps matching."""
    rng = rng_for(43, pcap)
    gp = ct.Pool(pcap, device=dev)
    op = oracle.OraclePool(pcap)

    def same():
        assert gp.size() == op.size()
        np.testing.assert_array_equal(gp.dump().cpu().numpy(), op.dump())

    failed = False   # the sticky pool error follows the oracle's refused elements
    for step in range(24):
        kind = rng.choice(["pop", "push", "pop_front", "push_front"])
        n = int(rng.integers(0, max(2, pcap // 3)))
        if kind in ("pop", "pop_front"):
            out, st = gp.pop(n) if kind == "pop" else gp.pop_front(n)
            eo, es = op.pop(n) if kind == "pop" else op.pop_front(n)
            np.testing.assert_array_equal(out.cpu().numpy(), eo)
        else:
            vals = rng.integers(0, 1 << 31, size=n, dtype=np.int64).astype(np.int32)
            g = torch.from_numpy(vals).to(dev)
            st = gp.push(g) if kind == "push" else gp.push_front(g)
            es = op.push(vals) if kind == "push" else op.push_front(vals)
        np.testing.assert_array_equal(st.cpu().numpy(), es)
        failed |= bool((es == 2).any())
        same()
    assert bool(gp.error() & ct.ERR_POOL) == failed
    # the pool under a table, after its head has moved: insert_alloc pops the back, erase_release
    # pushes it, both through the ring
    if pcap >= 1000:
        p = Pair(dev, pcap, 32, pool=pcap)
        out, st = p.gp.pop_front(pcap // 3)
        eo, es = p.op.pop_front(pcap // 3)
        np.testing.assert_array_equal(out.cpu().numpy(), eo)
        keys = distinct_u64(rng, pcap // 2)
        p.insert_alloc(keys)
        p.erase_release(keys[::2])
        st = p.gp.push(out[: pcap // 6].contiguous())     # FIFO reuse: released at the back
        np.testing.assert_array_equal(st.cpu().numpy(), p.op.push(eo[: pcap // 6]))
        p.insert_alloc(distinct_u64(rng, pcap // 2, exclude=keys))
        p.same_state()
        assert p.gp.size() == p.op.size()
        np.testing.assert_array_equal(p.gp.dump().cpu().numpy(), p.op.dump())


@pytest.mark.parametrize("path", PATHS)
@pytest.mark.parametrize("chunk", [1 << 16, 1 << 18])
def test_skewed_batches_fold_repeats_per_tile(dev, chunk, path):
    """Zipf(1.1) batches repeat their hottest keys thousands of times per chunk and overflow the
    dedup bins; the table then folds each tile's repeated keys before binning (a diagnostic shows
    the hint), every 16th chunk retries without folding, and a batch of distinct keys ends the
    hint.  Inserts, finds, erases and pool-valued inserts are compared with the oracle after every
    batch; the reserved-looking keys ride along."""
    rng = rng_for(83)
    universe = 1 << 16
    p = Pair(dev, 1 << 20, 64, chunk=chunk, path=path)
    # speculative inserts resolve repeated keys without the bins: only the other path sets the hint
    first = path == ct.INSERT_RESOLVE_FIRST

    def zipf(n):
        k = (rng.zipf(1.1, size=n) % universe).astype(np.uint64) * np.uint64(0x9E3779B97F4A7C15)
        k[rng.integers(0, n, size=16)] = RESERVED[rng.integers(0, RESERVED.size, size=16)]
        return k

    p.insert(zipf(chunk), rng.integers(0, 1 << 62, size=chunk, dtype=np.uint64))
    assert p.g.dedup_skewed() or not first
    for rep in range(20):   # more than 16 chunks: the periodic retry without folding runs too
        n = chunk + 333 * rep
        keys = zipf(n)
        if rep % 3 == 2:
            p.erase(keys)
        else:
            p.insert(keys, rng.integers(0, 1 << 62, size=n, dtype=np.uint64))
        if rep % 5 == 0:
            p.find(np.concatenate([keys[:4000], zipf(4000)]))
    p.same_state()
    assert p.g.dedup_skewed() or not first
    distinct = rng.permutation(np.arange(1, chunk + 1, dtype=np.uint64)) * np.uint64(0xD1B54A32D192ED03)
    for _ in range(9):   # 18 chunks: one tries without folding, fits, and ends the hint
        p.insert(distinct, rng.integers(0, 1 << 62, size=chunk, dtype=np.uint64))
        p.erase(distinct)
    p.find(distinct[: 1 << 12])
    p.same_state()
    assert not p.g.dedup_skewed() or not first
    q = Pair(dev, 1 << 19, 32, chunk=chunk, pool=1 << 19, path=path)
    keys = zipf(chunk * 2 + 5)
    q.insert_alloc(keys)
    q.erase_release(keys[: chunk // 2])
    q.insert_alloc(zipf(chunk * 3))
    q.same_state()


@pytest.mark.parametrize("path", PATHS)
@pytest.mark.parametrize("chunk,universe", [(1 << 16, 1 << 15), (1 << 17, 1 << 12), (1 << 16, 3)])
def test_binned_dedup_repeated_keys(dev, chunk, universe, path):
    """Chunks of at least 2^16 elements resolve repeated keys through bins: keys drawn from a
    small universe (about 2, 32 and 20,000 copies of each key per chunk; the last overflows its bin
    and takes the dd path), reserved-looking keys mixed in, ragged batches spanning chunks;
    inserts, erases and pool-valued inserts all compared with the oracle."""
    rng = rng_for(71)
    p = Pair(dev, 1 << 19, 64, chunk=chunk, path=path)
    for rep in range(3):
        n = int(chunk * 2.5) + 77 * rep
        keys = rng.integers(0, universe, size=n, dtype=np.uint64) * np.uint64(0x9E3779B97F4A7C15)
        keys[rng.integers(0, n, size=64)] = RESERVED[rng.integers(0, RESERVED.size, size=64)]
        p.insert(keys, rng.integers(0, 1 << 62, size=n, dtype=np.uint64))
        p.find(np.concatenate([keys[:5000], rng.integers(0, 1 << 62, size=5000, dtype=np.uint64)]))
        p.erase(keys[rng.integers(0, n, size=n // 3)])
        p.same_state()
    q = Pair(dev, 1 << 18, 32, chunk=chunk, pool=1 << 18)
    keys = rng.integers(0, universe, size=chunk * 2 + 5, dtype=np.uint64) + np.uint64(7)
    q.insert_alloc(keys)
    q.erase_release(keys[: chunk // 2])
    q.insert_alloc(keys[::-1].copy())
    q.same_state()


@pytest.mark.parametrize("path", PATHS)
@pytest.mark.parametrize("every", [1, 2, 7])
def test_claim_retry_path_with_injected_losses(dev, every, path):
    """Section 4 resolves rare failed internal attempts by further attempts.  A claim here fails
    only when another key took the slot first, which natural races rarely show; the test hook
    makes the first claim of every `every`-th chunk element fail deterministically, so those
    elements all take the retry path (scan on and claim again).  Results must not change: every
    insert status, find and the final contents equal the oracle's, at several chunk sizes, with
    repeated keys, and through a rehash into a table with the same hook set."""
    rng = rng_for(97, every)
    universe = np.concatenate([distinct_u64(rng, 60000), RESERVED])
    for chunk in (1024, 1 << 16):
        p = Pair(dev, 1 << 16, 64, chunk=chunk, path=path)
        p.g.debug_inject_claim_losses(every)
        for n in (5000, 70001, 3):
            keys = universe[rng.integers(0, universe.size, size=n)]
            p.insert(keys, rng.integers(0, 1 << 63, size=n, dtype=np.uint64))
            p.find(universe[rng.integers(0, universe.size, size=4000)])
            p.same_state()
        p.erase(universe[:20000])
        p.insert(universe[:25000], np.arange(25000, dtype=np.uint64))
        p.same_state()
        dst = ct.Table(1 << 17, ct.VAL_U64, ct.HASH_MIX64, device=dev)
        dst.debug_inject_claim_losses(every)
        p.g.rehash_into(dst)
        assert dst.size() == p.o.size() and dst.check() == 0
        k, v = dst.dump()
        order = np.argsort(npu(k), kind="stable")
        ek, ev = p.o.dump()
        np.testing.assert_array_equal(npu(k)[order], ek)
        np.testing.assert_array_equal(npu(v)[order], ev)
        p.g.debug_inject_claim_losses(0)
        p.insert(universe[:30000], np.zeros(30000, dtype=np.uint64))
        p.same_state()


def test_churn_health_and_purge(dev):
    """Near full load, erase and re-insert a tenth of the keys round after round: buckets lose
    their last empty slot and tombstones pile up (health counts both).  The purge reopens the
    buckets no live key passes; afterwards every result still equals the oracle's, the layout
    invariants hold, and fewer buckets are closed.  The oracle is compared after every batch."""
    rng = rng_for(211)
    nb = 4099
    cap = int(0.8 * 8 * nb)
    p = Pair(dev, cap, 64, bucket_count=nb)
    live = distinct_u64(rng, cap)
    p.insert(live, np.arange(cap, dtype=np.uint64))
    fresh = distinct_u64(rng, 80 * cap // 10, exclude=live)
    used = 0
    closed0, tombs0 = p.g.health()
    assert tombs0 == 0
    for r in range(40):
        k = cap // 10
        out = live[rng.choice(live.size, size=k, replace=False)]
        p.erase(out)
        live = np.setdiff1d(live, out)
        new = fresh[used:used + k]
        used += k
        p.insert(new, np.full(k, r, dtype=np.uint64))
        live = np.concatenate([live, new])
        if r % 10 == 9:
            p.find(np.concatenate([live[rng.integers(0, live.size, 3000)], fresh[-3000:]]))
            p.same_state()
    closed1, tombs1 = p.g.health()
    assert closed1 > closed0 and tombs1 > 0
    p.g.purge()
    closed2, tombs2 = p.g.health()
    assert closed2 < closed1 and tombs2 < tombs1
    p.same_state()
    p.find(np.concatenate([live, fresh[-5000:]]))
    # and the table keeps working after the purge
    p.erase(live[:2000])
    p.insert(fresh[used:used + 2000], np.zeros(2000, dtype=np.uint64))
    p.same_state()


@pytest.mark.parametrize("bits", [0, 32, 64])
@pytest.mark.parametrize("chunk", [1024, 1 << 16])
def test_speculative_insert_ambiguous_copies(dev, bits, chunk):
    """A chunk that cannot reach capacity is inserted speculatively: every element claims for
    itself, and the elements that met their key (in a bucket, or by losing a claim to a copy of it)
    are resolved afterwards by lowest index.  The batches here are built to make that resolution
    do all of its work: keys present before the chunk and repeated in it, absent keys repeated
    many times, erased keys whose tombstones lie on the probe paths, one key repeated by a whole
    batch, the reserved-looking keys, and a batch inserted without a status array (the stored
    value must still be the lowest copy's).  Every output and the final contents equal the
    oracle's."""
    rng = rng_for(307, bits + chunk)
    p = Pair(dev, 1 << 18, bits, chunk=chunk, path=ct.INSERT_SPECULATIVE)
    base = distinct_u64(rng, 60000)

    def v(n):
        x = rng.integers(0, 1 << 62, size=n, dtype=np.uint64)
        return x & np.uint64(0xFFFFFFFF) if bits == 32 else x

    p.insert(base[:30000], v(30000))
    p.erase(base[:15000:2])  # tombstones and empty slots on the probe paths of later keys
    p.same_state()
    for rep in range(4):
        n = [5000, 1 << 16, 70001, 1025][rep]
        pools = [base[15000:30000], base[30000:60000], base[:15000:2], RESERVED]
        pick = [pools[j][rng.integers(0, pools[j].size, size=n)] for j in range(4)]
        which = rng.integers(0, 4, size=n)
        keys = np.empty(n, dtype=np.uint64)
        for j in range(4):
            keys[which == j] = pick[j][which == j]
        p.insert(keys, v(n))
        p.find(keys[:4000])
        p.same_state()
    one = np.full(70000, base[59999], dtype=np.uint64)  # a whole batch of one absent key
    p.erase(base[59999:60000])
    p.insert(one, v(one.size))
    p.same_state()
    # no status array: the stored values must still come from the lowest copy of each key
    keys = base[30000:60000][rng.integers(0, 30000, size=50000)]
    vals = v(keys.size)
    p.erase(keys[:10000])
    if bits == 0:
        p.g.insert(g64(keys, dev), status=False)
    elif bits == 32:
        p.g.insert(g64(keys, dev), g32(vals, dev), status=False)
    else:
        p.g.insert(g64(keys, dev), g64(vals, dev), status=False)
    p.o.insert(keys, vals)
    p.same_state()


def test_auto_path_follows_the_last_chunk(dev):
    """The default path inserts a chunk speculatively while the table's last insert chunk stored
    at least half of its keys, and resolves repeated keys first otherwise (the table reports each
    chunk through a pinned host word).  The path shows in the launches of the repeated-key kernels:
    one per speculative chunk, five per binned resolve-first chunk.  Results equal the oracle's on
    every chunk, whichever path ran."""
    rng = rng_for(331)
    chunk = 1 << 16
    p = Pair(dev, 1 << 20, 64, chunk=chunk)
    keys = distinct_u64(rng, 3 * chunk)
    a, b, c = keys[:chunk], keys[chunk:2 * chunk], keys[2 * chunk:]
    p.g.profiling(True)

    def dedup_launches(batch):
        p.g.profile_reset()
        p.insert(batch, rng.integers(0, 1 << 62, size=batch.size, dtype=np.uint64))
        return p.g.profile()["dedup"][1]

    assert dedup_launches(a) == 1      # nothing reported yet: speculative
    assert dedup_launches(a) == 1      # the last chunk stored every key: speculative (stores none)
    assert dedup_launches(a) == 5      # the last chunk stored none: repeated keys first
    assert dedup_launches(b) == 5      # still after a chunk that stored none (this one stores all)
    assert dedup_launches(c) == 1      # speculative again (stores all)
    assert dedup_launches(c) == 1      # after a chunk that stored all (this one stores none)
    assert dedup_launches(c) == 5      # the last chunk stored none
    p.g.clear()                        # an empty table starts a fresh history
    p.o.clear()
    assert dedup_launches(c) == 1
    p.g.profiling(False)
    p.same_state()


@pytest.mark.parametrize("chunk", [1024, 1 << 16])
def test_speculative_erase_repeated_and_absent(dev, chunk):
    """A speculative erase removes a found key with one compare-and-swap, so exactly one copy
    removes it; copies that lose that CAS or find nothing are listed, and the lowest listed copy
    takes the removal over from a higher remover.  Batches mix keys present once, present keys
    repeated many times, absent keys (repeated too) and the reserved-looking keys, on a table with
    tombstones; the erase flags and the contents equal the oracle's after every batch, also
    without a flag array."""
    rng = rng_for(347, chunk)
    p = Pair(dev, 1 << 18, 64, chunk=chunk, path=ct.INSERT_SPECULATIVE)
    base = distinct_u64(rng, 80000)
    p.insert(np.concatenate([base[:50000], RESERVED[:3]]), rng.integers(0, 1 << 62, size=50003, dtype=np.uint64))
    for rep in range(4):
        n = [3000, 1 << 16, 70001, 17][rep]
        pools = [base[:50000], base[:200], base[50000:], RESERVED]
        which = rng.integers(0, 4, size=n)
        keys = np.empty(n, dtype=np.uint64)
        for j in range(4):
            pick = pools[j][rng.integers(0, pools[j].size, size=n)]
            keys[which == j] = pick[which == j]
        p.erase(keys)
        p.same_state()
        p.insert(keys[: n // 2], rng.integers(0, 1 << 62, size=n // 2, dtype=np.uint64))
        p.same_state()
    keys = base[rng.integers(0, 80000, size=40000)]
    p.g.erase(g64(keys, dev), status=False)
    p.o.erase(keys)
    p.same_state()


@pytest.mark.parametrize("chunk", [1024, 1 << 16])
def test_masked_insert_alloc(dev, chunk):
    """ct_insert_alloc_batch_masked inserts only the elements whose skip byte is 0, with the same
    results as ct_insert_alloc_batch of those keys gathered in index order; skipped elements keep
    their outputs.  Masks: a find's flags (insert the misses), random masks, all-skipped and
    none-skipped; keys repeat and include the reserved-looking ones; the pool runs out in the last
    batch."""
    rng = rng_for(359, chunk)
    pcap = 60000
    p = Pair(dev, 1 << 17, 32, chunk=chunk, pool=pcap)
    universe = np.concatenate([distinct_u64(rng, 90000), RESERVED])
    for rep in range(5):
        n = [20000, 70001, 5000, 3, 90000][rep]
        keys = universe[rng.integers(0, universe.size, size=n)]
        kd = g64(keys, dev)
        if rep == 0 or rep == 4:
            _, f = p.g.find(kd)
            skip = f
        elif rep == 1:
            skip = torch.from_numpy((rng.random(n) < 0.7).astype(np.uint8)).to(dev)
        elif rep == 2:
            skip = torch.ones(n, dtype=torch.uint8, device=dev)
        else:
            skip = torch.zeros(n, dtype=torch.uint8, device=dev)
        m = skip.cpu().numpy() == 0
        v, st = p.g.insert_alloc_masked(p.gp, kd, skip)
        ev, es = p.o.insert_alloc(p.op, keys[m])
        v, st = v.cpu().numpy(), st.cpu().numpy()
        np.testing.assert_array_equal(st[m], es)
        np.testing.assert_array_equal(v[m], ev)
        assert (st[~m] == 0xFF).all() and (v[~m] == -1).all()
        p.same_state()
    assert (es == 2).any()   # the pool ran out in the last batch
