"""Metamorphic GPU checks of the batch semantics (results equal n single-element calls in index
order), independent of the oracle: the same batch gives the same outputs whatever the chunk size
(including the binned dedup path), as n single-element batches, under any reordering that keeps
the order of equal keys, and on every repeated run."""
import numpy as np
import pytest
import torch

from paper_1908_05936_amd import ct
from paper_1908_05936_amd.workloads import rng_for

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def dev():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    ct.lib()
    return torch.device("cuda", 0)


def g64(a, dev):
    return torch.from_numpy(np.ascontiguousarray(np.asarray(a, dtype=np.uint64)).view(np.int64)).to(dev)


def batch(rng, n, universe):
    keys = rng.integers(0, universe, size=n, dtype=np.uint64) * np.uint64(0xD6E8FEB86659FD93)
    keys[rng.integers(0, n, size=8)] = np.uint64((1 << 64) - 1)   # an out-of-band key, repeated
    vals = rng.integers(0, 1 << 63, size=n, dtype=np.uint64)
    return keys, vals


def run(dev, cap, chunk, keys, vals, erase, probe):
    t = ct.Table(cap, ct.VAL_U64, ct.HASH_MIX64, chunk=chunk, device=dev)
    st = t.insert(g64(keys, dev), g64(vals, dev)).cpu().numpy()
    er = t.erase(g64(erase, dev)).cpu().numpy()
    st2 = t.insert(g64(keys[::-1].copy(), dev), g64(vals, dev)).cpu().numpy()
    v, f = t.find(g64(probe, dev))
    k, dv = t.dump()
    order = np.argsort(k.cpu().numpy().view(np.uint64), kind="stable")
    return dict(st=st, er=er, st2=st2, v=v.cpu().numpy(), f=f.cpu().numpy(),
                dump=(k.cpu().numpy()[order], dv.cpu().numpy()[order]), size=t.size())


def same(a, b):
    for k in a:
        if k == "dump":
            np.testing.assert_array_equal(a[k][0], b[k][0])
            np.testing.assert_array_equal(a[k][1], b[k][1])
        else:
            np.testing.assert_array_equal(a[k], b[k], err_msg=k)


def test_chunk_size_invariance(dev):
    rng = rng_for(81)
    n = 200_000
    keys, vals = batch(rng, n, 60_000)          # about 3 copies per key, some capacity misses
    erase = keys[rng.integers(0, n, size=n // 4)]
    probe = np.concatenate([keys[:20_000], rng.integers(0, 1 << 62, size=20_000, dtype=np.uint64)])
    ref = run(dev, 50_000, 1024, keys, vals, erase, probe)
    assert (ref["st"] == 2).any()               # the capacity was reached
    for chunk in (4096, 1 << 16, 1 << 17, 0):
        same(ref, run(dev, 50_000, chunk, keys, vals, erase, probe))


def test_batch_equals_singleton_batches(dev):
    rng = rng_for(82)
    keys, vals = batch(rng, 400, 150)
    t1 = ct.Table(120, ct.VAL_U64, ct.HASH_MIX64, device=dev)
    t2 = ct.Table(120, ct.VAL_U64, ct.HASH_MIX64, device=dev)
    st = t1.insert(g64(keys, dev), g64(vals, dev)).cpu().numpy()
    single = np.array([int(t2.insert(g64(keys[i:i + 1], dev), g64(vals[i:i + 1], dev)).cpu()[0])
                       for i in range(keys.size)], dtype=np.uint8)
    np.testing.assert_array_equal(st, single)
    er = t1.erase(g64(keys[::3].copy(), dev)).cpu().numpy()
    single = np.array([int(t2.erase(g64(keys[i:i + 1], dev)).cpu()[0]) for i in range(0, keys.size, 3)],
                      dtype=np.uint8)
    np.testing.assert_array_equal(er, single)
    v1, f1 = t1.find(g64(keys, dev))
    v2, f2 = t2.find(g64(keys, dev))
    np.testing.assert_array_equal(f1.cpu().numpy(), f2.cpu().numpy())
    np.testing.assert_array_equal(v1.cpu().numpy(), v2.cpu().numpy())


@pytest.mark.parametrize("chunk", [1024, 1 << 16])
def test_key_order_preserving_permutation(dev, chunk):
    """Reordering a batch so that the copies of each key keep their relative order permutes the
    outputs the same way (keys never interact)."""
    rng = rng_for(83)
    n = 150_000
    keys, vals = batch(rng, n, 40_000)
    # a random interleaving of the per-key subsequences: shuffle the batch, then give each key's
    # positions in the shuffled batch back to that key's elements in their original order
    perm = rng.permutation(n)
    order = np.empty(n, dtype=np.int64)
    ks = keys[perm]
    by_key = {}
    for pos, i in enumerate(perm):
        by_key.setdefault(int(keys[i]), []).append(pos)
    orig = {}
    for i in range(n):
        orig.setdefault(int(keys[i]), []).append(i)
    for k, slots in by_key.items():
        for slot, i in zip(slots, orig[k]):
            order[slot] = i
    np.testing.assert_array_equal(keys[order], ks)
    t1 = ct.Table(60_000, ct.VAL_U64, ct.HASH_MIX64, chunk=chunk, device=dev)
    t2 = ct.Table(60_000, ct.VAL_U64, ct.HASH_MIX64, chunk=chunk, device=dev)
    a = t1.insert(g64(keys, dev), g64(vals, dev)).cpu().numpy()
    b = t2.insert(g64(keys[order], dev), g64(vals[order], dev)).cpu().numpy()
    np.testing.assert_array_equal(a[order], b)
    assert t1.size() == t2.size()


def test_repeated_runs_are_identical(dev):
    rng = rng_for(84)
    keys, vals = batch(rng, 300_000, 100_000)
    erase = keys[::5].copy()
    probe = keys[::7].copy()
    ref = run(dev, 80_000, 1 << 16, keys, vals, erase, probe)
    for _ in range(3):
        same(ref, run(dev, 80_000, 1 << 16, keys, vals, erase, probe))
