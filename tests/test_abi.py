"""The C-ABI library loads, exports every symbol its headers declare, and rejects bad arguments on
the host before touching the GPU (no compute calls: this runs without a GPU)."""
import ctypes as C
import os
import re

import pytest

from paper_1908_05936_amd import ct

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    names = []
    for h in sorted(os.listdir(os.path.join(ROOT, "include"))):
        if not h.endswith(".h"):
            continue
        src = open(os.path.join(ROOT, "include", h)).read()
        src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
        names += re.findall(r"^\s*(?:const\s+)?\w+\s*\*?\s*(ct\w+|ctr\w+)\s*\(", src, flags=re.M)
    return sorted(set(names))


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(ct.LIB_PATH):
        import __graft_entry__

        __graft_entry__.build()
    return ct.lib()


def test_every_declared_symbol_is_exported(lib):
    names = _declared()
    assert len(names) >= 25, names
    for n in names:
        assert hasattr(lib, n), n
    # and the binding covers every one of them
    assert set(names) <= set(ct.SIGNATURES), set(names) - set(ct.SIGNATURES)


def test_table_bytes_and_argument_checks(lib):
    d = ct.TableDesc(1 << 17, ct.VAL_U32, ct.HASH_MIX64, 0, 0)
    nb = C.c_int64(0)
    assert lib.ct_table_bytes(C.byref(d), C.byref(nb)) == ct.CT_OK
    # 2^14 buckets of 128 B plus header and scratch
    assert nb.value >= (1 << 14) * 128
    bad = [
        ct.TableDesc(-1, ct.VAL_U32, ct.HASH_MIX64, 0, 0),      # negative capacity
        ct.TableDesc(100, 7, ct.HASH_MIX64, 0, 0),              # unknown value kind
        ct.TableDesc(100, ct.VAL_U32, 9, 0, 0),                 # unknown hash
        ct.TableDesc(100, ct.VAL_U32, ct.HASH_MIX64, 12, 0),    # 8 * 12 < 100
        ct.TableDesc(100, ct.VAL_U32, ct.HASH_MIX64, 0, 1000),  # chunk not a power of two
        ct.TableDesc(100, ct.VAL_U32, ct.HASH_MIX64, 0, 512),   # chunk below 1024
    ]
    for b in bad:
        assert lib.ct_table_bytes(C.byref(b), C.byref(nb)) == ct.CT_E_INVALID
    # null handles and negative counts are rejected before any HIP call
    assert lib.ct_insert_batch(None, None, None, 0, None, None) == ct.CT_E_INVALID
    assert lib.ct_find_batch(None, None, 5, None, None, None) == ct.CT_E_INVALID
    assert lib.ct_erase_batch(None, None, -1, None, None) == ct.CT_E_INVALID
    assert lib.ct_size(None, None, None) == ct.CT_E_INVALID
    assert lib.ct_pool_pop_batch(None, 1, None, None, None) == ct.CT_E_INVALID
    out = C.c_void_p()
    assert lib.ct_table_init(None, 0, C.byref(d), None, C.byref(out)) == ct.CT_E_INVALID
    assert lib.ct_pool_bytes(-5, C.byref(nb)) == ct.CT_E_INVALID
    assert lib.ct_pool_bytes(1000, C.byref(nb)) == ct.CT_OK and nb.value >= 4000
    assert lib.ctr_copy(None, None, 16, None) == ct.CT_E_INVALID
    assert lib.ct_status_str(ct.CT_E_FULL) == b"capacity exhausted"
    # the resize, selection, deque-front and device-side entry points check their arguments too
    cnt = C.c_int64(0)
    assert lib.ct_table_rehash(None, None, None) == ct.CT_E_INVALID
    assert lib.ct_select_key_range(None, 0, 1, None, None, 0, C.byref(cnt), None) == ct.CT_E_INVALID
    lo3 = (C.c_int32 * 3)(0, 0, 0)
    assert lib.ct_select_voxel_box(None, lo3, lo3, None, None, 0, C.byref(cnt), None) == ct.CT_E_INVALID
    assert lib.ct_pool_pop_front_batch(None, 1, None, None, None) == ct.CT_E_INVALID
    assert lib.ct_pool_push_front_batch(None, None, 1, None, None) == ct.CT_E_INVALID
    buf = (C.c_uint8 * 4096)()
    assert lib.ct_table_device_view(None, 0, buf, 4096) == ct.CT_E_INVALID
    assert lib.ct_pool_device_view(None, buf, 4096) == ct.CT_E_INVALID
    assert lib.ct_dev_apply(None, ct.OP_INSERT, None, None, 1, None, None, None) == ct.CT_E_INVALID
    assert lib.ct_dev_apply_mixed(None, None, None, None, 1, None, None, None) == ct.CT_E_INVALID
    assert lib.ct_dev_pool_apply(None, 0, None, 1, None, None, None) == ct.CT_E_INVALID
    assert lib.ct_voxel_insert_neighbours(None, None, 1, 6, None) == ct.CT_E_INVALID
    assert lib.ct_voxel_insert_neighbours_alloc(None, None, None, 1, 6, None) == ct.CT_E_INVALID
    assert lib.ct_table_dedup_skewed(None, None, None) == ct.CT_E_INVALID
    assert lib.ct_check_invariants(None, None, C.byref(cnt), None) == ct.CT_E_INVALID
    assert lib.ct_dev_update_set(None, None, None, 1, None, None) == ct.CT_E_INVALID
    assert lib.ct_table_debug_inject_claim_losses(None, 1, None) == ct.CT_E_INVALID
    assert lib.ct_table_health(None, C.byref(cnt), None, None) == ct.CT_E_INVALID
    assert lib.ct_table_purge(None, None) == ct.CT_E_INVALID
    # grouped-plan options: merge runs and the block sizes 128 .. 1024 are known, others refused
    plan = C.c_void_p()
    assert lib.ct_plan_create(C.byref(plan)) == ct.CT_OK
    nb = C.c_int64(0)
    for opt in (0, ct.GROUP_MERGE_RUNS, ct.GROUP_BLOCK[128], ct.GROUP_BLOCK[1024] | 1):
        assert lib.ct_plan_group_bytes(plan, opt, C.byref(nb)) == ct.CT_OK, opt
    for opt in (4, 5 << 8, 11 << 8, 1 << 12):
        assert lib.ct_plan_group_bytes(plan, opt, C.byref(nb)) == ct.CT_E_INVALID, opt
    assert lib.ct_plan_destroy(plan) == ct.CT_OK


def test_product_path_does_not_reach_the_oracle():
    # the package never imports the CPU oracle: it is test infrastructure only
    pkg = os.path.join(ROOT, "paper_1908_05936_amd")
    for dirpath, _, files in os.walk(pkg):
        for f in files:
            if f.endswith((".py", ".hip", ".h", ".cpp")):
                src = open(os.path.join(dirpath, f)).read()
                assert "import oracle" not in src and "from oracle" not in src, f
                assert "liboracle" not in src, f
