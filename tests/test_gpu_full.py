"""GPU parity at the workloads' full sizes, in the launch configuration the benchmark times.

* large table: 2^26 u64 -> u64 keys at load factor 0.8, 2^27 Zipf finds (20 % absent), erase 2^24,
  re-insert 2^24 -- statuses of every insert/erase, every find value and flag, and the final
  contents compared with the oracle in full.
* voxel blocks: 2^20 residents with pool-allocated values in a 2^21-bucket spatial-hash table, then
  100 frames of find 2^18 + insert_alloc of the misses -- every output of every frame compared.
* the largest chunk (2^24) with a ragged batch full of duplicates.
"""
import numpy as np
import pytest
import torch

import oracle
from paper_1908_05936_amd import ct
from paper_1908_05936_amd.workloads import large_table, rng_for, voxel_blocks

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def dev():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    ct.lib()
    return torch.device("cuda", 0)


def g64(a, dev):
    return torch.from_numpy(np.ascontiguousarray(np.asarray(a, dtype=np.uint64)).view(np.int64)).to(dev)


def u64(t):
    return t.cpu().numpy().view(np.uint64)


def test_large_table_full_size(dev):
    print("large table: generating", flush=True)
    w = large_table(seed=3)
    cap = w["capacity"]
    t = ct.Table(cap, ct.VAL_U64, ct.HASH_MIX64, device=dev)   # the benchmark's configuration
    o = oracle.OracleTable(cap, 64, oracle.HASH_MIX64, 1 << 24)
    print("large table: fill", flush=True)
    st = t.insert(g64(w["insert_keys"], dev), g64(w["insert_vals"], dev))
    np.testing.assert_array_equal(st.cpu().numpy(), o.insert(w["insert_keys"], w["insert_vals"]))
    print("large table: find", flush=True)
    v, f = t.find(g64(w["find"], dev))
    ev, ef = o.find(w["find"])          # every one of the 2^27 queries
    np.testing.assert_array_equal(f.cpu().numpy(), ef)
    np.testing.assert_array_equal(u64(v), ev)
    del ev, ef
    # the hit count is fixed by the workload: 80 % of the queries are live keys
    assert int(f.sum()) == w["find"].size - round(w["find"].size * 0.2)
    print("large table: erase + re-insert", flush=True)
    er = t.erase(g64(w["erase"], dev))
    np.testing.assert_array_equal(er.cpu().numpy(), o.erase(w["erase"]))
    st = t.insert(g64(w["reinsert_keys"], dev), g64(w["reinsert_vals"], dev))
    np.testing.assert_array_equal(st.cpu().numpy(), o.insert(w["reinsert_keys"], w["reinsert_vals"]))
    assert t.size() == o.size() == 1 << 26
    k, val = t.dump()
    k, val = u64(k), u64(val)
    order = np.argsort(k)
    ek, evv = o.dump()
    np.testing.assert_array_equal(k[order], ek)
    np.testing.assert_array_equal(val[order], evv)
    assert t.check() == 0


@pytest.mark.parametrize("misses", ["compacted", "masked", "graph"])
def test_voxel_frames_full_size(dev, misses):
    """100 frames of find + insert_alloc of the misses on the full voxel workload, bit-exact
    against the oracle.  The misses reach the table either compacted on the host (the find's flags
    select them) or through ct_insert_alloc_batch_masked with the find's flags as the mask, called
    directly or captured once into a HIP graph that every frame replays on a fixed input buffer."""
    print(f"voxel ({misses}): generating", flush=True)
    w = voxel_blocks(seed=2)
    nb = w["bucket_count"]
    pool_cap = w["pool_capacity"]
    t = ct.Table(pool_cap, ct.VAL_U32, ct.HASH_VOXEL21, bucket_count=nb, device=dev)
    gp = ct.Pool(pool_cap, device=dev)
    o = oracle.OracleTable(pool_cap, 32, oracle.HASH_VOXEL21, nb)
    op = oracle.OraclePool(pool_cap)
    v, st = t.insert_alloc(gp, g64(w["residents"], dev))
    ev, es = o.insert_alloc(op, w["residents"])
    np.testing.assert_array_equal(st.cpu().numpy(), es)
    np.testing.assert_array_equal(v.cpu().numpy(), ev)
    if misses == "graph":   # one capture over fixed buffers, replayed for every frame
        n = w["frames"][0].size
        assert all(q.size == n for q in w["frames"])
        qbuf = torch.empty(n, dtype=torch.int64, device=dev)
        fv = torch.empty(n, dtype=torch.int32, device=dev)
        ff = torch.empty(n, dtype=torch.uint8, device=dev)
        gv = torch.empty(n, dtype=torch.int32, device=dev)
        gs = torch.empty(n, dtype=torch.uint8, device=dev)
        graph = torch.cuda.CUDAGraph()
        with torch.cuda.graph(graph, stream=torch.cuda.Stream(dev)):
            t.find(qbuf, out=fv, found_out=ff)
            t.insert_alloc_masked(gp, qbuf, ff, gv, gs)
        torch.cuda.synchronize()
    for f, q in enumerate(w["frames"]):
        qd = g64(q, dev)
        if misses == "graph":
            qbuf.copy_(qd)              # eager work and a synchronization between replays
            torch.cuda.synchronize()
            graph.replay()
            torch.cuda.synchronize()
            v, fd = fv, ff
        else:
            v, fd = t.find(qd)
        ev, ef = o.find(q)
        np.testing.assert_array_equal(fd.cpu().numpy(), ef)
        np.testing.assert_array_equal(v.cpu().numpy().view(np.uint32), ev)
        miss = q[ef == 0]
        ev, es = o.insert_alloc(op, miss)
        if misses == "graph":
            v, st = gv.cpu().numpy(), gs.cpu().numpy()
            np.testing.assert_array_equal(st[ef == 0], es)
            np.testing.assert_array_equal(v[ef == 0], ev)
        elif misses == "compacted":
            v, st = t.insert_alloc(gp, g64(miss, dev))
            np.testing.assert_array_equal(st.cpu().numpy(), es)
            np.testing.assert_array_equal(v.cpu().numpy(), ev)
        else:
            v, st = t.insert_alloc_masked(gp, qd, fd)
            v, st = v.cpu().numpy(), st.cpu().numpy()
            np.testing.assert_array_equal(st[ef == 0], es)
            np.testing.assert_array_equal(v[ef == 0], ev)
            assert (st[ef == 1] == 0xFF).all() and (v[ef == 1] == -1).all()
        if f % 25 == 0:
            print(f"voxel: frame {f} ok", flush=True)
    assert t.size() == o.size() == 3669976
    np.testing.assert_array_equal(gp.dump().cpu().numpy(), op.dump())
    assert t.check() == 0
    assert t.check(gp) == 0   # the pool and the block map hold every index exactly once


def test_largest_chunk_with_duplicates(dev):
    rng = rng_for(41)
    n = (1 << 24) + 12345
    universe = rng.integers(0, 1 << 64, size=1 << 23, dtype=np.uint64)
    keys = universe[rng.integers(0, universe.size, size=n)]
    vals = rng.integers(0, 1 << 63, size=n, dtype=np.uint64)
    t = ct.Table(1 << 23, ct.VAL_U64, ct.HASH_MIX64, chunk=1 << 24, device=dev)
    o = oracle.OracleTable(1 << 23, 64, oracle.HASH_MIX64, 1 << 22)
    st = t.insert(g64(keys, dev), g64(vals, dev))
    np.testing.assert_array_equal(st.cpu().numpy(), o.insert(keys, vals))
    er = t.erase(g64(keys[: n // 3], dev))
    np.testing.assert_array_equal(er.cpu().numpy(), o.erase(keys[: n // 3]))
    assert t.size() == o.size()
    assert t.check() == 0
