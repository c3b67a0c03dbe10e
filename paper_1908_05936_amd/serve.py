"""Continuous-batching serving loop over device-resident tables.

Requests (insert / find / erase batches for one table) arrive over time.  The server keeps one
FIFO per table and a global arrival order, and on every turn of its loop it:

1. moves requests whose arrival time has passed into their table's FIFO (arrival stamped);
2. retires finished batches: a batch is done when the HIP event recorded after its last copy has
   completed; each request of the batch gets its slice of the results and its latency
   (completion seen on the host minus arrival);
3. admits work in arrival order: the head request of each table, together with the requests of
   the same kind queued right behind it on that table (coalesced into one batch), is admitted if
   the in-flight staging bytes stay within the HBM budget and a batch slot is free; otherwise
   admission stops (back-pressure, nothing is dropped).

An admitted batch is copied from pinned host memory, run by the library on the table's stream,
and its results copied back to pinned host memory, all enqueued asynchronously.  Tables are spread
over several streams, so batches of different tables overlap on the device, while a table's
batches stay in arrival order on its stream.  Merging consecutive same-kind requests of one table
keeps the sequential result of each request (a batch is the composition of its parts in order).

All container work runs in the HIP library through ``paper_1908_05936_amd.ct``; this module
only moves bytes and keeps the books.
"""
from __future__ import annotations

import collections
import time
from dataclasses import dataclass, field

import numpy as np
import torch

from . import ct

VALUE_BYTES = 8


@dataclass
class Request:
    rid: int
    table: int
    kind: str          # "insert" | "find" | "erase"
    keys: np.ndarray   # uint64
    vals: np.ndarray | None = None
    arrival: float = 0.0
    done: float = 0.0
    result: dict = field(default_factory=dict)
    hkeys: torch.Tensor | None = None   # pinned host copies (see pin)
    hvals: torch.Tensor | None = None

    def pin(self):
        """Place keys (and values) in pinned host memory, where a server receives them."""
        if self.hkeys is None:
            self.hkeys = torch.from_numpy(np.ascontiguousarray(self.keys).view(np.int64)).pin_memory()
            if self.vals is not None:
                self.hvals = torch.from_numpy(
                    np.ascontiguousarray(self.vals).view(np.int64)).pin_memory()
        return self

    def fresh(self, rid: int) -> "Request":
        """A not-yet-served copy with id `rid` sharing this request's (pinned) keys and values."""
        return Request(rid, self.table, self.kind, self.keys, self.vals, hkeys=self.hkeys,
                       hvals=self.hvals)

    def staging_bytes(self) -> int:
        n = self.keys.size
        if self.kind == "insert":
            return n * (8 + VALUE_BYTES + 1)
        if self.kind == "find":
            return n * (8 + VALUE_BYTES + 1)
        return n * (8 + 1)


def _to_pinned(t: torch.Tensor) -> torch.Tensor:
    """Asynchronous device-to-host copy into freshly allocated pinned memory."""
    h = torch.empty(t.shape, dtype=t.dtype, pin_memory=True)
    h.copy_(t, non_blocking=True)
    return h


class _Batch:
    def __init__(self, reqs, event, outs, nbytes):
        self.reqs = reqs
        self.event = event
        self.outs = outs
        self.nbytes = nbytes


class Server:
    """Serve requests against `tables` (ct.Table with VAL_U64 values)."""

    def __init__(self, tables, device, streams: int = 8, budget_bytes: int = 1 << 30,
                 max_inflight: int = 64, max_batch_keys: int = 1 << 21):
        self.tables = tables
        self.dev = device
        self.streams = [torch.cuda.Stream(device) for _ in range(streams)]
        self.budget = int(budget_bytes)
        self.max_inflight = int(max_inflight)
        self.max_batch = int(max_batch_keys)
        self.queues = [collections.deque() for _ in tables]
        self.inflight: list[_Batch] = []
        self.inflight_bytes = 0
        self.peak_bytes = 0
        self.peak_slots = 0
        self.batches = 0
        self.order = collections.deque()  # tables in arrival order of their queued heads

    # -- admission and dispatch -----------------------------------------------------------
    def _dispatch(self, t: int, reqs):
        kind = reqs[0].kind
        n = sum(r.keys.size for r in reqs)
        s = self.streams[t % len(self.streams)]
        tab = self.tables[t]
        with torch.cuda.stream(s):
            dk = torch.empty(n, dtype=torch.int64, device=self.dev)
            dv = torch.empty(n, dtype=torch.int64, device=self.dev) if kind == "insert" else None
            off = 0
            for r in reqs:      # coalesce on the device: one async copy per request
                r.pin()
                m = r.keys.size
                dk[off:off + m].copy_(r.hkeys, non_blocking=True)
                if dv is not None:
                    dv[off:off + m].copy_(r.hvals, non_blocking=True)
                off += m
            outs = {}
            if kind == "insert":
                st = tab.insert(dk, dv)
                outs["status"] = _to_pinned(st)
                keep = (dk, dv, st)
            elif kind == "find":
                v, f = tab.find(dk)
                outs["vals"] = _to_pinned(v)
                outs["found"] = _to_pinned(f)
                keep = (dk, v, f)
            else:
                er = tab.erase(dk)
                outs["erased"] = _to_pinned(er)
                keep = (dk, er)
            ev = torch.cuda.Event()
            ev.record(s)
        nbytes = sum(r.staging_bytes() for r in reqs)
        b = _Batch(reqs, ev, outs, nbytes)
        b.keep = keep
        self.inflight.append(b)
        self.inflight_bytes += nbytes
        self.peak_bytes = max(self.peak_bytes, self.inflight_bytes)
        self.peak_slots = max(self.peak_slots, len(self.inflight))
        self.batches += 1

    def _admit(self):
        while self.order:
            t = self.order[0]
            q = self.queues[t]
            if not q:
                self.order.popleft()
                continue
            head = q[0]
            if len(self.inflight) >= self.max_inflight:
                return
            if self.inflight_bytes + head.staging_bytes() > self.budget and self.inflight:
                return  # back-pressure in arrival order
            reqs = [q.popleft()]
            nbytes = head.staging_bytes()
            nkeys = head.keys.size
            while q and q[0].kind == head.kind and nkeys + q[0].keys.size <= self.max_batch and \
                    self.inflight_bytes + nbytes + q[0].staging_bytes() <= self.budget:
                r = q.popleft()
                reqs.append(r)
                nbytes += r.staging_bytes()
                nkeys += r.keys.size
            self.order.popleft()
            if q:
                self.order.append(t)   # its next head waits behind the other tables' heads
            self._dispatch(t, reqs)

    def _retire(self):
        still = []
        now = None
        for b in self.inflight:
            if b.event.query():
                now = now or time.perf_counter()
                off = 0
                for r in b.reqs:
                    n = r.keys.size
                    r.result = {k: v[off:off + n].numpy() for k, v in b.outs.items()}
                    r.done = now
                    off += n
                self.inflight_bytes -= b.nbytes
            else:
                still.append(b)
        self.inflight = still

    # -- driving -------------------------------------------------------------------------
    def run(self, requests, arrivals):
        """Serve `requests` arriving at host times `arrivals` (seconds from the start)."""
        pending = collections.deque(zip(arrivals, requests))
        t0 = time.perf_counter()
        while pending or any(self.queues) or self.inflight:
            now = time.perf_counter() - t0
            while pending and pending[0][0] <= now:
                at, r = pending.popleft()
                r.arrival = t0 + at
                q = self.queues[r.table]
                if not q:
                    self.order.append(r.table)
                q.append(r)
            self._retire()
            self._admit()
            if not self.inflight and not any(self.queues) and pending:
                wait = pending[0][0] - (time.perf_counter() - t0)
                if wait > 0:
                    time.sleep(min(wait, 1e-3))
        return time.perf_counter() - t0


def serving_chunk(max_batch_keys: int = 1 << 21) -> int:
    """Insert/erase chunk for serving tables: half the largest coalesced batch (scratch is about
    34 bytes per chunk element and table, so the chunk is sized to requests, not to capacity)."""
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


def latency_stats(reqs) -> dict:
    lat = np.array([r.done - r.arrival for r in reqs]) * 1e3
    keys = sum(r.keys.size for r in reqs)
    span = max(r.done for r in reqs) - min(r.arrival for r in reqs)
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
        srv.run(reqs, arrivals)
        return srv, reqs

    srv, reqs = serve(np.zeros(total))
    sat = latency_stats(reqs[warmup:])
    sat_keys = sat["achieved_Mkeys_s"] * 1e6
    log(f"[serve] saturated {sat['achieved_Mkeys_s']:.1f} Mkeys/s, {srv.batches} batches, "
        f"p50 {sat['p50_ms']:.2f} ms p99 {sat['p99_ms']:.2f} ms")
    points = []
    for f in fractions:
        rate = f * sat_keys / mean_keys
        srv, reqs = serve(poisson_arrivals(rng, total, rate))
        st = latency_stats(reqs[warmup:])
        st.update(offered_fraction=f, offered_Mkeys_s=f * sat_keys / 1e6, batches=srv.batches,
                  peak_inflight_bytes=srv.peak_bytes, peak_inflight_batches=srv.peak_slots)
        log(f"[serve] {f:.2f} x: p50 {st['p50_ms']:.2f} ms p99 {st['p99_ms']:.2f} ms "
            f"achieved {st['achieved_Mkeys_s']:.1f} Mkeys/s")
        points.append(st)
    return dict(saturated_Mkeys_s=sat["achieved_Mkeys_s"], saturated_p50_ms=sat["p50_ms"],
                saturated_p99_ms=sat["p99_ms"], mean_request_keys=mean_keys, points=points,
                requests=dict(warmup=warmup, measured=measured, distinct=len(pool)),
                budget_bytes=budget_bytes, max_inflight=max_inflight, streams=streams,
                max_batch_keys=max_batch_keys)
