"""The allocation-free insert (ct_insert_batch_noalloc) against ct_insert_batch.

Both entry points are called through the C ABI on twin tables with the same batches; statuses,
sizes and the final contents must be identical (integer results: bit-exact).  Two calls in a row,
the second smaller than the first, so the second runs on the static scratch the first left behind.
The batches hold repeated keys and cross the array's 2^15-element chunk, and the last one nears
capacity, so both insert paths (speculative, and repeated keys first with the rank pass) run out
of the static array.
"""
import numpy as np
import pytest
import torch

from paper_1908_05936_amd import ct
from paper_1908_05936_amd.workloads import distinct_u64, rng_for

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def dev():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    ct.lib()
    return torch.device("cuda", 0)


def g64(a, dev):
    return torch.from_numpy(np.ascontiguousarray(np.asarray(a, dtype=np.uint64)).view(np.int64)).to(dev)


def call(entry, table, keys, vals, bits, dev):
    """One insert through `entry` (a C-ABI function); returns the status array."""
    n = keys.size
    k = g64(keys, dev)
    if bits == 64:
        v = g64(vals, dev)
    elif bits == 32:
        v = torch.from_numpy(vals.astype(np.uint32).view(np.int32)).to(dev)
    else:
        v = None
    st = torch.empty(n, dtype=torch.uint8, device=dev)
    ct._check(entry(table._h, ct._ptr(k), ct._ptr(v), n, ct._ptr(st), ct._stream(dev)), "insert")
    return st.cpu().numpy()


def contents(table, bits):
    k, v = table.dump()
    k = k.cpu().numpy().view(np.uint64)
    order = np.argsort(k, kind="stable")
    vv = v.cpu().numpy().view(np.uint64)[order] if bits else None
    return k[order], vv


@pytest.mark.parametrize("kind,bits", [(ct.VAL_U64, 64), (ct.VAL_U32, 32), (ct.VAL_NONE, 0)])
def test_noalloc_insert_equals_insert_batch(dev, kind, bits):
    L = ct.lib()
    rng = rng_for(401, bits)
    cap = 75_000
    # the table's own chunk is 2^16 (binned repeated-key resolution); the allocation-free call
    # runs 2^15-element chunks out of its static array: results must not depend on that
    a = ct.Table(cap, kind, ct.HASH_MIX64, chunk=1 << 16, device=dev)   # ct_insert_batch
    b = ct.Table(cap, kind, ct.HASH_MIX64, chunk=1 << 16, device=dev)   # ct_insert_batch_noalloc
    universe = distinct_u64(rng, 200_000)
    sa = None
    for n in (100_003, 40_000, 70_000):   # the second call is smaller than the first
        keys = universe[rng.integers(0, n, size=n)]
        vals = rng.integers(0, 1 << 62, size=n, dtype=np.uint64) if bits else None
        if bits == 32:
            vals &= np.uint64(0xFFFFFFFF)
        sa = call(L.ct_insert_batch, a, keys, vals, bits, dev)
        sb = call(L.ct_insert_batch_noalloc, b, keys, vals, bits, dev)
        np.testing.assert_array_equal(sb, sa)
        assert b.size() == a.size()
        ka, va = contents(a, bits)
        kb, vb = contents(b, bits)
        np.testing.assert_array_equal(kb, ka)
        if bits:
            np.testing.assert_array_equal(vb, va)
        assert a.check() == 0 and b.check() == 0
    assert (sa == 2).any()   # the last batch met capacity on both paths
