"""Serving sweep on the 64-table workload: tables of 2^16..2^26 entries (u64 keys and values)
provisioned to a common physical footprint, Poisson arrivals of insert/find/erase requests
(20/70/10, 2^8..2^20 keys, Zipf(1.1)) offered at fractions of the saturated throughput, p50/p99
latency and achieved keys/s per point, as one JSON line.

    python -m paper_1908_05936_amd.bench_serve [--footprint-gb 40] [--warmup 2000]
        [--measured 20000] [--distinct 4000] [--budget-mb 1024] [--insert-path auto]
        [--out FILE]
"""
from __future__ import annotations

import argparse
import json
import sys
import time

import torch

from . import ct, serve
from .workloads import Serving


def run(footprint_gb=40.0, warmup=2000, measured=20000, distinct=4000, budget_mb=1024,
        max_inflight=64, streams=8, n_tables=64, entries_log2=(16, 26), seed=5,
        fractions=(0.1, 0.25, 0.5, 0.75, 0.9, 1.0, 1.2), insert_path="auto", log=print):
    dev = torch.device("cuda", 0)
    sv = Serving(seed=seed, n_tables=n_tables, entries_log2=entries_log2)
    head = serve.headroom_for(sv, footprint_gb * 1e9)
    mb = 1 << 21
    t0 = time.perf_counter()
    tables = serve.build_tables(sv, dev, headroom=head, chunk=serve.serving_chunk(mb))
    for t in tables:
        t.set_insert_path({"auto": ct.INSERT_AUTO, "resolve-first": ct.INSERT_RESOLVE_FIRST,
                           "speculative": ct.INSERT_SPECULATIVE}[insert_path])
    nbytes = sum(t.nbytes for t in tables)
    log(f"[serve] {n_tables} tables, {sum(sv.entries) / 1e6:.1f} M resident entries, "
        f"{nbytes / 1e9:.2f} GB, headroom {head:.3f}, built in {time.perf_counter() - t0:.1f} s")
    res = serve.sweep(sv, tables, dev, fractions=fractions, warmup=warmup, measured=measured,
                      pool_size=distinct, streams=streams, budget_bytes=budget_mb << 20,
                      max_inflight=max_inflight, max_batch_keys=mb, log=log)
    res.update(workload="serving-64-tables", tables=n_tables, table_bytes=nbytes,
               resident_entries=sum(sv.entries), headroom=head, seed=seed, insert_path=insert_path)
    return res


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("--footprint-gb", type=float, default=40.0)
    ap.add_argument("--warmup", type=int, default=2000)
    ap.add_argument("--measured", type=int, default=20000)
    ap.add_argument("--distinct", type=int, default=4000)
    ap.add_argument("--budget-mb", type=int, default=1024)
    ap.add_argument("--max-inflight", type=int, default=64)
    ap.add_argument("--streams", type=int, default=8)
    ap.add_argument("--insert-path", choices=["auto", "resolve-first", "speculative"], default="auto")
    ap.add_argument("--out", default=None)
    ap.add_argument("--wait-stdin", action="store_true",
                    help="start only after a line arrives on stdin (exit at end of input)")
    a = ap.parse_args(argv)
    if a.wait_stdin and not sys.stdin.readline():
        return
    res = run(a.footprint_gb, a.warmup, a.measured, a.distinct, a.budget_mb, a.max_inflight,
              a.streams, insert_path=a.insert_path,
              log=lambda m: print(m, file=sys.stderr, flush=True))
    line = json.dumps(res)
    print(line, flush=True)
    if a.out:
        with open(a.out, "w") as f:
            f.write(line + "\n")


if __name__ == "__main__":
    main()
