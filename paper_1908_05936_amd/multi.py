"""Multi-table execution helpers: build a plan from a schedule, time it, and tune its launch.

Every operation still runs in the HIP library (ct_plan_* in include/ct.h); this module only
creates tables and device arrays, records the schedule into a plan, and measures launches.

Autotuner.  The knobs of a plan run are
  * lanes       -- 0: the grouped form (one launch per pipeline stage per level, covering every
                   table); -1: the grouped form as one cooperative launch (ct_plan_launch_single:
                   the stages separated by grid-wide barriers inside the kernel; 256-thread stages);
                   1..8: side streams the tables are spread over, each operation running its own
                   pipeline (operations on different tables overlap on the device; a table's
                   operations keep their order),
  * merge       -- grouped form only: merge each table's runs of same-kind operations into one
                   operation over gathered copies (fewer levels and launches, more memory),
  * chunk       -- per-table insert/erase chunk (a larger chunk means fewer chained sub-operations
                   for big batches on small tables, at 34-109 bytes of scratch per chunk element),
  * provision   -- physical slots per requested capacity (1.0 = the requested load factor; more
                   slots lower the physical load and shorten probes, at the cost of memory),
  * block       -- grouped form only: threads per block of the find / insert / erase stages
                   (128, 256, 512, 1024: more blocks in flight against fewer waves per block).
The lane-group width that probes one key is fixed at 8 lanes x 16 bytes = one 128-byte bucket
line: the layout's bucket is one such line, and a 4-lane probe of 64-byte half lines would need a
table of 64-byte buckets (4 slots), which the measured gather ceilings rule out (35.3 G 128-byte
lines/s x 8 slots against 40.5 G 64-byte lines/s x 4 slots per second of probing).  The tuner does coordinate descent from the
defaults on one seed's schedule and reports the choice, which a caller then evaluates on a
schedule drawn with another seed.  Results are cached in a JSON file keyed by device name and
workload signature.
"""
from __future__ import annotations

import json
import os
import time

import numpy as np
import torch

from . import ct

OPS = {"insert": ct.OP_INSERT, "find": ct.OP_FIND, "erase": ct.OP_ERASE}
DEFAULT = dict(lanes=0, merge=False, chunk=0, provision=1.0, block=256)


def _g64(a, dev):
    return torch.from_numpy(np.ascontiguousarray(np.asarray(a, dtype=np.uint64)).view(np.int64)).to(dev)


def _g32(a, dev):
    return torch.from_numpy(np.ascontiguousarray(np.asarray(a, dtype=np.uint32)).view(np.int32)).to(dev)


class Workload:
    """Device-resident tables, inputs and outputs for one schedule."""

    def __init__(self, w: dict, dev, chunk: int = 0, provision: float = 1.0):
        self.w = w
        self.dev = dev
        self.tables = []
        max_batch = {}
        for ti, _, keys, _ in w["schedule"]:
            max_batch[ti] = max(max_batch.get(ti, 0), keys.size)
        for i, t in enumerate(w["tables"]):
            nb = int(np.ceil(t["capacity"] * provision / 8)) if provision != 1.0 else 0
            ch = chunk
            if chunk < 0:  # chunk = the table's largest batch
                ch = max(1024, 1 << int(np.ceil(np.log2(max(max_batch.get(i, 1), 1)))))
            self.tables.append(ct.Table(t["capacity"], ct.VAL_U32, ct.HASH_MIX64, bucket_count=nb,
                                        chunk=ch, device=dev))
        self.ops = []
        for ti, kind, keys, vals in w["schedule"]:
            k = _g64(keys, dev)
            v = _g32(vals, dev) if vals is not None else None
            flags = torch.empty(keys.size, dtype=torch.uint8, device=dev)
            vout = torch.empty(keys.size, dtype=torch.int32, device=dev) if kind == "find" else None
            self.ops.append((ti, kind, k, v, flags, vout))
        self.n_keys = int(sum(k.numel() for _, _, k, _, _, _ in self.ops))
        self.table_bytes = int(sum(t.nbytes for t in self.tables))

    def plan(self) -> ct.Plan:
        p = ct.Plan(device=self.dev)
        for t in self.tables:
            p.add(t, ct.OP_CLEAR)
        for ti, kind, k, v, flags, vout in self.ops:
            p.add(self.tables[ti], OPS[kind], keys=k, vals=v, vals_out=vout, flags_out=flags)
        return p

    def per_batch(self):
        """The same schedule as single-table calls, one library call per operation."""
        for t in self.tables:
            t.clear()
        for ti, kind, k, v, flags, vout in self.ops:
            t = self.tables[ti]
            if kind == "insert":
                ct._check(ct.lib().ct_insert_batch(t._h, ct._ptr(k), ct._ptr(v), k.numel(),
                                                   ct._ptr(flags), ct._stream(self.dev)), "insert")
            elif kind == "find":
                ct._check(ct.lib().ct_find_batch(t._h, ct._ptr(k), k.numel(), ct._ptr(vout),
                                                 ct._ptr(flags), ct._stream(self.dev)), "find")
            else:
                ct._check(ct.lib().ct_erase_batch(t._h, ct._ptr(k), k.numel(), ct._ptr(flags),
                                                  ct._stream(self.dev)), "erase")


def time_fn(fn, reps=3, warmup=1):
    """Median device time (s) of `fn` over `reps` runs, events on the current stream."""
    for _ in range(warmup):
        fn()
    torch.cuda.synchronize()
    ts = []
    for _ in range(reps):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        fn()
        e1.record()
        torch.cuda.synchronize()
        ts.append(e0.elapsed_time(e1) * 1e-3)
    return float(np.median(ts))


def runner(p: ct.Plan, lanes: int, merge: bool = False, block: int = 256):
    """Callable running plan `p` once: grouped (lanes 0, built on first use), grouped as one
    cooperative launch (lanes -1, 256-thread stages) or on side streams."""
    if lanes <= 0:
        if getattr(p, "_gbuf", None) is None:
            p.group(merge_runs=merge, block=block if lanes == 0 else 256)
        return p.launch_grouped if lanes == 0 else p.launch_single
    return lambda: p.launch(lanes)


def signature(w: dict) -> str:
    sizes = [t["capacity"] for t in w["tables"]]
    return (f"tables={len(sizes)},cap_sum={sum(sizes)},ops={len(w['schedule'])},"
            f"keys={sum(x[2].size for x in w['schedule'])}")


def tune(w: dict, dev, cache: str | None = None, reps: int = 3, log=print) -> dict:
    """Coordinate descent over lanes, chunk, provision and run merging on schedule `w` (up to two
    sweeps over the knobs)."""
    key = f"{torch.cuda.get_device_name(dev)}|{signature(w)}"
    if cache and os.path.exists(cache):
        try:
            got = json.load(open(cache)).get(key)
            if got:
                return got
        except (OSError, ValueError):
            pass
    best = dict(DEFAULT)
    trials = []
    built = {}

    def run(cfg):
        wk = (cfg["chunk"], cfg["provision"])
        if wk not in built:
            built.clear()
            torch.cuda.empty_cache()
            built[wk] = Workload(w, dev, chunk=cfg["chunk"], provision=cfg["provision"])
        wl = built[wk]
        p = wl.plan()
        try:
            t = time_fn(runner(p, cfg["lanes"], cfg.get("merge", False), cfg.get("block", 256)),
                        reps=reps)
        except ct.CtError as e:
            if cfg["lanes"] >= 0:
                raise
            t = float("inf")   # the device refused the cooperative launch: not a candidate
            log(f"[tune] {cfg}: {e}")
        trials.append(dict(cfg, seconds=t))
        log(f"[tune] {cfg} -> {t * 1e3:.2f} ms")
        return t

    best_t = run(best)
    space = [("lanes", [0, -1, 1, 2, 4, 8]), ("chunk", [0, -1]), ("provision", [1.0, 1.25, 1.5]),
             ("merge", [False, True]), ("block", [128, 256, 512, 1024])]
    seen = {repr(sorted(best.items()))}
    for sweep in range(2):  # a second sweep revisits each knob at the others' new values
        improved = False
        for name, values in space:
            if name == "merge" and best["lanes"] > 0:
                continue   # a knob of the grouped forms only
            if name == "block" and best["lanes"] != 0:
                continue   # the single launch runs 256-thread stages
            for v in values:
                cfg = dict(best, **{name: v})
                if repr(sorted(cfg.items())) in seen:
                    continue
                seen.add(repr(sorted(cfg.items())))
                t = run(cfg)
                if t < best_t:
                    best, best_t, improved = cfg, t, True
        if not improved:
            break
    result = dict(best, seconds=best_t, trials=len(trials))
    if cache:
        try:
            data = json.load(open(cache)) if os.path.exists(cache) else {}
        except (OSError, ValueError):
            data = {}
        data[key] = result
        os.makedirs(os.path.dirname(os.path.abspath(cache)), exist_ok=True)
        json.dump(data, open(cache, "w"), indent=1)
    return result


def measure(w: dict, dev, cfg: dict, reps: int = 5, graph_replays: int = 10) -> dict:
    """Plan run, its HIP-graph replay and one-stream per-batch calls on schedule `w` with `cfg`."""
    wl = Workload(w, dev, chunk=cfg["chunk"], provision=cfg["provision"])
    p = wl.plan()
    t_plan = time_fn(runner(p, cfg["lanes"], cfg.get("merge", False), cfg.get("block", 256)),
                     reps=reps)
    s = torch.cuda.Stream(dev)
    if cfg["lanes"] <= 0:
        p.capture_grouped(stream=s)   # (the single launch is one submission already)
    else:
        p.capture(cfg["lanes"], stream=s)

    def replays():
        with torch.cuda.stream(s):
            for _ in range(graph_replays):
                p.replay(s)

    torch.cuda.synchronize()
    w0 = time.perf_counter()
    replays()
    s.synchronize()
    t_graph = (time.perf_counter() - w0) / graph_replays
    t_batch = time_fn(wl.per_batch, reps=max(1, reps // 2))
    n = wl.n_keys
    extra = {}
    if cfg["lanes"] <= 0:
        extra = dict(zip(("grouped_launches", "grouped_steps"), p.group_info()))
    # the grouped form as one cooperative launch, whatever form was chosen
    p1 = wl.plan()
    p1.group(merge_runs=cfg.get("merge", False), block=256)
    try:
        t_single = time_fn(p1.launch_single, reps=reps)
        extra.update(single_launch_ms=t_single * 1e3,
                     single_launch_Mkeys_s=wl.n_keys / t_single / 1e6)
    except ct.CtError as e:
        extra.update(single_launch_ms=None, single_launch_error=str(e))
    del p1
    t_streams = time_fn(lambda: p.launch(4), reps=reps)
    return dict(extra, keys=n, ops=len(w["schedule"]), tables=len(w["tables"]),
                streams4_ms=t_streams * 1e3,
                table_bytes=wl.table_bytes, plan_ms=t_plan * 1e3, graph_replay_ms=t_graph * 1e3,
                per_batch_ms=t_batch * 1e3, plan_Mkeys_s=n / t_plan / 1e6,
                graph_Mkeys_s=n / t_graph / 1e6, per_batch_Mkeys_s=n / t_batch / 1e6,
                speedup_vs_per_batch=t_batch / t_plan, config=cfg)
