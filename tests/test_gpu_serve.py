"""GPU serving loop: every request served in the mix gets exactly the result the oracle gives when
the table's requests are replayed in arrival order, the same as when that table is served alone;
admission never exceeds its byte budget or slot cap."""
import numpy as np
import pytest
import torch

import oracle
from paper_1908_05936_amd import ct
from paper_1908_05936_amd.serve import Request, Server, build_tables, poisson_arrivals
from paper_1908_05936_amd.workloads import Serving

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def dev():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    ct.lib()
    return torch.device("cuda", 0)


def small_workload():
    return Serving(seed=5, n_tables=6, entries_log2=(10, 14), req_log2=(4, 12), rank_pool=1 << 16)


def oracle_tables(sv):
    tabs = []
    for t, (e, u) in enumerate(zip(sv.entries, sv.universe)):
        o = oracle.OracleTable(u, 64, oracle.HASH_MIX64, max(1, u // 4))
        o.insert(sv.resident(t, 0, e), np.arange(e, dtype=np.uint64))
        tabs.append(o)
    return tabs


def expected(tabs, reqs):
    out = {}
    for r in sorted(reqs, key=lambda r: r.rid):   # arrival order = request id order
        o = tabs[r.table]
        if r.kind == "insert":
            out[r.rid] = {"status": o.insert(r.keys, r.vals)}
        elif r.kind == "find":
            v, f = o.find(r.keys)
            out[r.rid] = {"vals": v, "found": f}
        else:
            out[r.rid] = {"erased": o.erase(r.keys)}
    return out


def same(r, exp):
    for k, v in exp.items():
        got = r.result[k]
        if k == "vals":
            got = got.view(np.uint64)
        np.testing.assert_array_equal(got, v, err_msg=f"request {r.rid} {r.kind} {k}")


def draw(sv, n):
    return [Request(*x) for x in sv.requests(n)]


@pytest.mark.parametrize("chunk", [0, 1024])
def test_served_results_match_sequential_replay(dev, chunk):
    sv = small_workload()
    tables = build_tables(sv, dev, chunk=chunk)
    reqs = draw(sv, 400)
    budget = 1 << 18
    srv = Server(tables, dev, streams=4, budget_bytes=budget, max_inflight=8)
    srv.run(reqs, poisson_arrivals(np.random.default_rng(1), len(reqs), 20000.0))
    exp = expected(oracle_tables(sv), reqs)
    for r in reqs:
        same(r, exp[r.rid])
    assert srv.peak_slots <= 8
    biggest = max(r.staging_bytes() for r in reqs)
    assert srv.peak_bytes <= max(budget, biggest)
    assert srv.batches < len(reqs)   # some requests were coalesced
    for t, o in zip(tables, oracle_tables_after(sv, reqs)):
        assert t.size() == o.size()


def oracle_tables_after(sv, reqs):
    tabs = oracle_tables(sv)
    expected(tabs, reqs)
    return tabs


def test_result_alone_equals_result_in_mix(dev):
    sv = small_workload()
    tables = build_tables(sv, dev)
    reqs = draw(sv, 300)
    Server(tables, dev, streams=4).run(reqs, np.zeros(len(reqs)))   # all at once: the mix
    t0 = reqs[0].table
    alone = [Request(r.rid, r.table, r.kind, r.keys, r.vals) for r in reqs if r.table == t0]
    sv2 = small_workload()
    tables2 = build_tables(sv2, dev)
    Server(tables2, dev, streams=1).run(alone, np.zeros(len(alone)))
    mix = {r.rid: r for r in reqs}
    for a in alone:
        for k, v in a.result.items():
            np.testing.assert_array_equal(v, mix[a.rid].result[k])


def test_sweep_runs_and_reports(dev):
    from paper_1908_05936_amd.serve import sweep
    sv = small_workload()
    tables = build_tables(sv, dev)
    res = sweep(sv, tables, dev, fractions=(0.5, 1.0), warmup=20, measured=100, pool_size=50,
                log=lambda m: None)
    assert res["requests"]["distinct"] == 50
    assert len(res["points"]) == 2
    for p in res["points"]:
        assert p["requests"] == 100
        assert 0 < p["p50_ms"] <= p["p99_ms"]
        assert p["peak_inflight_batches"] <= res["max_inflight"]
