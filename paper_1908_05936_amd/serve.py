"""Continuous-batching serving of requests against device-resident tables.

The server itself is native (include/ct_server.h): a worker thread keeps one FIFO per table,
admits the oldest waiting table head -- merged with the same-kind requests queued right behind it
-- while its staging space fits in the device staging buffer (the HBM admission budget) and a batch
slot is free, runs each batch on its table's stream (copies in, the table's batch call, copies
out, completion event) and stamps every request with its submission and completion times.  This
module marshals requests into pinned host memory, submits them at their arrival times, and turns
the times into latency statistics.
"""
from __future__ import annotations

import time
from dataclasses import dataclass, field

import numpy as np
import torch

from . import ct

OPS = {"insert": ct.OP_INSERT, "find": ct.OP_FIND, "erase": ct.OP_ERASE}


@dataclass
class Request:
    rid: int
    table: int
    kind: str          # "insert" | "find" | "erase"
    keys: np.ndarray   # uint64
    vals: np.ndarray | None = None
    arrival: float = 0.0   # submission time, seconds on the server's clock
    done: float = 0.0      # completion time seen by the server, same clock
    status: int = 0
    result: dict = field(default_factory=dict)
    hkeys: torch.Tensor | None = None   # pinned host arrays (see pin)
    hvals: torch.Tensor | None = None
    hflags: torch.Tensor | None = None
    hvout: torch.Tensor | None = None

    def pin(self):
        """Place inputs and result arrays in pinned host memory, where a server receives and
        answers requests."""
        if self.hkeys is None:
            self.hkeys = torch.from_numpy(np.ascontiguousarray(self.keys).view(np.int64)).pin_memory()
            if self.vals is not None:
                self.hvals = torch.from_numpy(
                    np.ascontiguousarray(self.vals).view(np.int64)).pin_memory()
        if self.hflags is None:
            n = self.keys.size
            self.hflags = torch.empty(n, dtype=torch.uint8, pin_memory=True)
            if self.kind == "find":
                self.hvout = torch.empty(n, dtype=torch.int64, pin_memory=True)
        return self

    def fresh(self, rid: int) -> "Request":
        """A not-yet-served copy with id `rid` sharing this request's pinned inputs and result
        arrays (for load generation, where results are not read)."""
        return Request(rid, self.table, self.kind, self.keys, self.vals, hkeys=self.hkeys,
                       hvals=self.hvals, hflags=self.hflags, hvout=self.hvout)

    def staging_bytes(self, value_bytes: int = 8) -> int:
        n = self.keys.size
        vb = value_bytes if self.kind in ("insert", "find") else 0
        return n * (8 + vb + 1)

    def _collect(self):
        f = self.hflags.numpy().copy()
        if self.kind == "insert":
            self.result = {"status": f}
        elif self.kind == "find":
            self.result = {"vals": self.hvout.numpy().copy(), "found": f}
        else:
            self.result = {"erased": f}


class Server:
    """Serve requests against `tables` (ct.Table, VAL_U64) through the native server."""

    def __init__(self, tables, device, streams: int = 8, budget_bytes: int = 1 << 30,
                 max_inflight: int = 64, max_batch_keys: int = 1 << 21):
        self.native = ct.NativeServer(tables, budget_bytes, streams=streams,
                                      max_inflight=max_inflight, max_batch_keys=max_batch_keys,
                                      device=device)
        self.budget = int(budget_bytes)
        self.max_inflight = int(max_inflight)

    def close(self):
        self.native.close()

    def run(self, requests, arrivals, collect: bool = True):
        """Submit `requests` at host times `arrivals` (seconds from now, ascending), wait for
        all of them, and fill in their times, status and (if `collect`) results."""
        by_ticket = {}
        for r in requests:
            r.pin()
        t0 = time.perf_counter()
        for at, r in zip(arrivals, requests):
            wait = at - (time.perf_counter() - t0)
            if wait > 3e-4:
                time.sleep(wait - 2e-4)
            while time.perf_counter() - t0 < at:
                pass
            tk = self.native.submit(r.table, OPS[r.kind], r.hkeys, r.hvals, r.hvout, r.hflags)
            by_ticket[tk] = r
        self.native.wait_idle()
        tk, sub, done, st = self.native.poll(len(by_ticket) + 1)
        for k, a, d, s in zip(tk.tolist(), sub.tolist(), done.tolist(), st.tolist()):
            r = by_ticket.pop(k)
            r.arrival, r.done, r.status = a * 1e-9, d * 1e-9, s
            if collect:
                r._collect()
        if by_ticket:
            raise RuntimeError(f"{len(by_ticket)} requests were not reported complete")
        return self.native.stats()

    @property
    def stats(self):
        return self.native.stats()


def serving_chunk(max_batch_keys: int = 1 << 21) -> int:
    """Insert/erase chunk for serving tables: half the largest coalesced batch (scratch is about
    34-109 bytes per chunk element and table, so the chunk is sized to requests, not to capacity)."""
    return max(1024, max_batch_keys // 2)


def build_tables(sv, device, headroom: float = 1.0, chunk: int = 0, threads: int = 8,
                 block: int = 1 << 23):
    """Tables of `sv` (a workloads.Serving) with capacity = universe * headroom (every key of the
    universe fits) and the resident half inserted, values = key index.  Resident keys are drawn on
    `threads` host threads, `block` keys at a time."""
    from concurrent.futures import ThreadPoolExecutor
    tables = []
    jobs = []
    for t, (e, u) in enumerate(zip(sv.entries, sv.universe)):
        tables.append(ct.Table(int(u * headroom), ct.VAL_U64, ct.HASH_MIX64, chunk=chunk,
                               device=device))
        jobs += [(t, lo, min(e, lo + block)) for lo in range(0, e, block)]
    with ThreadPoolExecutor(max(1, threads)) as ex:
        for w in range(0, len(jobs), threads):     # bounded window of host key blocks
            win = jobs[w:w + threads]
            for (t, lo, hi), keys in zip(win, ex.map(lambda j: sv.resident(*j), win)):
                k = torch.from_numpy(keys.view(np.int64)).to(device)
                v = torch.arange(lo, hi, dtype=torch.int64, device=device)
                tables[t].insert(k, v, status=False)
    torch.cuda.synchronize()
    return tables


def headroom_for(sv, target_bytes: float) -> float:
    """Common capacity factor over the universes that makes the tables' slots total
    `target_bytes` at 16 bytes per slot (at least 1: every key of the universe fits)."""
    return max(1.0, target_bytes / 16.0 / float(sum(sv.universe)))


def poisson_arrivals(rng, n: int, rate_per_s: float) -> np.ndarray:
    return np.cumsum(rng.exponential(1.0 / rate_per_s, size=n))


def latency_stats(reqs, before=()) -> dict:
    """p50/p99/mean latency (ms) of `reqs`, and their keys per second over the window from the
    later of their first arrival and the last completion among `before` (the warm-up requests
    served ahead of them) to their last completion."""
    lat = np.array([r.done - r.arrival for r in reqs]) * 1e3
    keys = sum(r.keys.size for r in reqs)
    start = min(r.arrival for r in reqs)
    if before:
        start = max(start, max(r.done for r in before))
    span = max(r.done for r in reqs) - start
    return dict(requests=len(reqs), p50_ms=float(np.percentile(lat, 50)),
                p99_ms=float(np.percentile(lat, 99)), mean_ms=float(lat.mean()),
                achieved_Mkeys_s=keys / span / 1e6)


def sweep(sv, tables, device, fractions=(0.1, 0.25, 0.5, 0.75, 0.9, 1.0, 1.2), warmup=200,
          measured=2000, pool_size=None, streams=8, budget_bytes=1 << 30, max_inflight=64,
          max_batch_keys=1 << 21, threads=8, log=print):
    """Saturated throughput (every request queued at once), then Poisson arrivals offered at
    `fractions` of it; p50/p99 latency over the `measured` requests after `warmup` at each point.

    A pool of `pool_size` distinct requests (default warmup + measured) is drawn and pinned once;
    every point serves fresh copies of it in order, cycling when the point needs more.  The
    tables keep their state from point to point, as a long-running server's would."""
    rng = np.random.default_rng(sv.seed + 99)
    total = warmup + measured
    pool = [Request(*x).pin() for x in sv.requests(min(pool_size or total, total), threads)]
    mean_keys = float(np.mean([r.keys.size for r in pool]))
    next_id = [0]

    def serve(arrivals):
        reqs = []
        for i in range(total):
            reqs.append(pool[i % len(pool)].fresh(next_id[0]))
            next_id[0] += 1
        srv = Server(tables, device, streams=streams, budget_bytes=budget_bytes,
                     max_inflight=max_inflight, max_batch_keys=max_batch_keys)
        st = srv.run(reqs, arrivals, collect=False)
        srv.close()
        if st["error"] or any(r.status for r in reqs):
            raise RuntimeError(f"serving failed: {st}")
        return st, reqs

    srv, reqs = serve(np.zeros(total))
    sat = latency_stats(reqs[warmup:], reqs[:warmup])
    sat_span = max(r.done for r in reqs) - min(r.arrival for r in reqs)
    sat_worker = dict(dispatch_share=srv["dispatch_ns"] * 1e-9 / sat_span,
                      retire_share=srv["retire_ns"] * 1e-9 / sat_span,
                      batches=srv["batches"])
    sat_keys = sat["achieved_Mkeys_s"] * 1e6
    log(f"[serve] saturated {sat['achieved_Mkeys_s']:.1f} Mkeys/s, {srv['batches']} batches, "
        f"p50 {sat['p50_ms']:.2f} ms p99 {sat['p99_ms']:.2f} ms")
    points = []
    for f in fractions:
        rate = f * sat_keys / mean_keys
        srv, reqs = serve(poisson_arrivals(rng, total, rate))
        st = latency_stats(reqs[warmup:], reqs[:warmup])
        st.update(offered_fraction=f, offered_Mkeys_s=f * sat_keys / 1e6, batches=srv["batches"],
                  peak_staging_bytes=srv["peak_staging_bytes"],
                  peak_inflight_batches=srv["peak_inflight"])
        log(f"[serve] {f:.2f} x: p50 {st['p50_ms']:.2f} ms p99 {st['p99_ms']:.2f} ms "
            f"achieved {st['achieved_Mkeys_s']:.1f} Mkeys/s")
        points.append(st)
    return dict(saturated_Mkeys_s=sat["achieved_Mkeys_s"], saturated_worker=sat_worker,
                saturated_p50_ms=sat["p50_ms"],
                saturated_p99_ms=sat["p99_ms"], mean_request_keys=mean_keys, points=points,
                requests=dict(warmup=warmup, measured=measured, distinct=len(pool)),
                budget_bytes=budget_bytes, max_inflight=max_inflight, streams=streams,
                max_batch_keys=max_batch_keys)
