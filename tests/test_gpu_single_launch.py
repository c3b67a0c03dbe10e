"""The grouped multi-table schedule as ONE kernel launch (ct_plan_launch_single, a cooperative
launch with grid-wide barriers between stages): every result equals the oracle's, as for the
per-stage launches."""
import numpy as np
import pytest
import torch

import oracle
from paper_1908_05936_amd import ct
from paper_1908_05936_amd.workloads import multi_table
from test_gpu_multi import PATHS, Run, expected, g32, g64, listing_schedule, mixed_kinds_schedule, small

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def dev():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    ct.lib()
    return torch.device("cuda", 0)


@pytest.mark.parametrize("chunk,merge,max_blocks", [(0, False, 0), (1024, False, 0), (0, True, 0),
                                                    (1024, True, 0), (1024, False, 7)])
def test_single_launch_matches_oracle(dev, chunk, merge, max_blocks):
    """The grouped schedule as one cooperative launch: stage by stage, the grid's workgroups take
    the stage's blocks in turn and meet at a grid-wide barrier.  A grid of 7 workgroups makes each
    one run many blocks of every stage.  A second launch (the plan starts with clears) gives the
    same results."""
    w = small()
    exp, tabs = expected(w)
    r = Run(w, dev, chunk=chunk)
    p = r.plan(dev)
    p.group(merge_runs=merge)
    p.launch_single(max_blocks)
    r.check(exp)
    for t, o in zip(r.tables, tabs):
        assert t.size() == o.size()
        assert t.check() == 0
    r.scramble()
    p.launch_single(max_blocks)
    r.check(exp)


@pytest.mark.parametrize("path", PATHS)
@pytest.mark.parametrize("max_blocks", [0, 5])
def test_single_launch_insert_paths(dev, path, max_blocks):
    """Speculative steps and their resolution stages inside the one launch: repeated, present and
    out-of-band keys, each table on the given insert path; two launches in a row."""
    w = listing_schedule()
    exp, tabs = expected(w)
    r = Run(w, dev, chunk=2048, path=path)
    p = r.plan(dev)
    p.group(merge_runs=True)
    for rep in range(2):
        r.scramble()
        p.launch_single(max_blocks)
        r.check(exp)
        for t, o in zip(r.tables, tabs):
            assert t.size() == o.size()
            assert t.check() == 0


def test_single_launch_needs_256_thread_stages(dev):
    w = small()
    r = Run(w, dev)
    p = r.plan(dev)
    p.group(block=512)
    with pytest.raises(ct.CtError):
        p.launch_single()


def test_single_launch_full_size(dev):
    """The full 256-table schedule (2^10..2^20 entries) in one launch, every result bit-exact."""
    w = multi_table(seed=4)
    exp, tabs = expected(w)
    r = Run(w, dev)
    p = r.plan(dev)
    p.group(merge_runs=True)
    p.launch_single()
    r.check(exp)
    for t, o in zip(r.tables, tabs):
        assert t.size() == o.size()


def test_single_launch_mixed_value_kinds_and_capacity(dev):
    """Sets, u32 and u64 maps in one schedule, repeated keys, inserts that reach capacity (the
    rank stages run inside the launch too), chunk 1024 (several levels per operation)."""
    tables, sched = mixed_kinds_schedule()
    bits = {ct.VAL_NONE: 0, ct.VAL_U32: 32, ct.VAL_U64: 64}
    otabs = [oracle.OracleTable(t["capacity"], bits[t["kind"]]) for t in tables]
    gtabs = [ct.Table(t["capacity"], t["kind"], ct.HASH_MIX64, chunk=1024, device=dev) for t in tables]
    p = ct.Plan(device=dev)
    for g in gtabs:
        p.add(g, ct.OP_CLEAR)
    outs, exp = [], []
    for ti, kind, keys, vals in sched:
        g, o, vk = gtabs[ti], otabs[ti], tables[ti]["kind"]
        k = g64(keys, dev)
        flags = torch.full((keys.size,), 7, dtype=torch.uint8, device=dev)
        vout = None
        if kind == "insert":
            v = g32(vals, dev) if vk == ct.VAL_U32 else (g64(vals, dev) if vk == ct.VAL_U64 else None)
            p.add(g, ct.OP_INSERT, keys=k, vals=v, flags_out=flags)
            exp.append((o.insert(keys, vals), None))
        elif kind == "find":
            if vk != ct.VAL_NONE:
                vout = torch.empty(keys.size, dtype=torch.int32 if vk == ct.VAL_U32 else torch.int64,
                                   device=dev)
            p.add(g, ct.OP_FIND, keys=k, vals_out=vout, flags_out=flags)
            v, f = o.find(keys)
            exp.append((f, v if vk != ct.VAL_NONE else None))
        else:
            p.add(g, ct.OP_ERASE, keys=k, flags_out=flags)
            exp.append((o.erase(keys), None))
        outs.append((flags, vout, vk))
    p.group(merge_runs=True)
    p.launch_single()
    torch.cuda.synchronize()
    for (flags, vout, vk), (ef, ev) in zip(outs, exp):
        np.testing.assert_array_equal(flags.cpu().numpy(), ef)
        if ev is not None:
            got = vout.cpu().numpy().view(np.uint32 if vk == ct.VAL_U32 else np.uint64)
            np.testing.assert_array_equal(got, ev)
    for g, o in zip(gtabs, otabs):
        assert g.size() == o.size()
        assert g.check() == 0
