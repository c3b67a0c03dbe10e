"""Benchmark of the batch hash-container hot path on one MI355X.

One step is one pass of the whole path over the large-table workload, on a table already resident
in HBM: clear, fill 2^26 distinct u64 keys with u64 values (load factor 0 -> 0.8 of 83,886,080
slots, 1.342 GB), find 2^27 queries (Zipf(1.1) popularity over the live keys, 20 % absent), erase
2^24 live keys, re-insert 2^24 fresh keys (load 0.6 -> 0.8).  Inputs are generated once and kept
on the GPU; only the container calls are timed.

The printed JSON line carries:
  value        whole-step throughput, container operations per second (Mops/s)
  breakdown    per-operation Mops/s from HIP events on the library's stream
  insert_marginal_Mops_s  2^20 fresh keys inserted into the table at load 0.8
  roofline     the dominant kernel's algorithmic bytes per launch / its mean duration vs 8 TB/s
  random_access the same kernels against ceilings measured in this run on this chip
  rehash       the table rehashed into one of twice the capacity (host-side resize)
  mixed_device_ops  finds, inserts and erases in one device-side kernel on the step's table, the
               same work as three batch calls, and its finds alone in a read-only launch
  pool         the index pool at 2^24 keys: insert_alloc, erase_release, bare pop and push
  voxel        the voxel-block frames: per-frame p50/p99, find and insert_alloc Mkeys/s
  multi_table  the 256-table schedule, tuned in this run: plan, graph replay and per-batch
               keys/s, and the fraction of the R1/R2 ceiling of its own mix at its footprint
  served       the serving sweep on 64 device-resident tables: p50/p99 latency and achieved
               keys/s at fractions of the saturated rate
  cpu_baseline the CPU oracle timed on a bounded sample of the same workload
"""
from __future__ import annotations

import argparse
import json
import os
import platform
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
# algorithmic bytes per operation (what the method itself must move)
FIND_BYTES = 8 + 8 + 1 + 128        # key in, value out, found flag; one 128-byte bucket line read
INSERT_BYTES = 8 + 8 + 1 + 2 * 128  # key, value in, status out; bucket line read and written back
ERASE_BYTES = 8 + 1 + 2 * 128       # key in, flag out; bucket line read and written back
METRIC = "find & insert Mops/s at load 0.8 (1 GPU); served p50/p99 batch latency"
PMC_SUMMARY = os.path.join(ROOT, "profiles", "pmc_large_table.md")
INSERT_PATHS = {"auto": 0, "resolve-first": 1, "speculative": 2}   # ct_table_set_insert_path
KERNEL_SOURCES = ["include/ct.h", "paper_1908_05936_amd/csrc/ct_device.h",
                  "paper_1908_05936_amd/csrc/ct_dev_api.h",
                  "paper_1908_05936_amd/csrc/ct_table.hip"]


def kernel_source_hash() -> str:
    """SHA-256 of the kernel sources with comments and blank space removed, so that recorded
    counter figures stay attached to the code they measured and not to its comments."""
    import hashlib
    import re

    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        with open(os.path.join(ROOT, f), encoding="utf-8") as fh:
            src = fh.read()
        src = re.sub(r"/\*.*?\*/", " ", src, flags=re.S)   # block comments
        src = re.sub(r"//[^\n]*", " ", src)                  # line comments
        h.update(" ".join(src.split()).encode())
    return h.hexdigest()


def recorded_traffic():
    """Per-launch HBM bytes of each kernel from the committed counter summary, if it was taken
    from the kernels as they are now (same source hash); else None."""
    try:
        text = open(PMC_SUMMARY).read()
    except OSError:
        return None
    start = text.find("```json")
    if start < 0:
        return None
    end = text.find("```", start + 7)
    try:
        data = json.loads(text[start + 7:end])
    except ValueError:
        return None
    if data.get("source_sha256") != kernel_source_hash():
        return None
    return data


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--log2-keys", type=int, default=26)
    ap.add_argument("--log2-queries", type=int, default=27)
    ap.add_argument("--log2-churn", type=int, default=24)
    ap.add_argument("--chunk", type=int, default=0, help="table chunk (0 = library default)")
    ap.add_argument("--no-serve", action="store_true", help="skip the serving sweep")
    ap.add_argument("--no-voxel", action="store_true", help="skip the voxel-block frames")
    ap.add_argument("--no-pool", action="store_true", help="skip the index-pool operations")
    ap.add_argument("--no-multi", action="store_true",
                    help="skip the tuned 256-table schedule")
    ap.add_argument("--no-rehash", action="store_true", help="skip the resize (rehash) figure")
    ap.add_argument("--no-mixed", action="store_true",
                    help="skip the mixed device-side operations figure")
    ap.add_argument("--insert-path", choices=["auto", "resolve-first", "speculative"], default="auto",
                    help="how insert chunks resolve repeated keys (ct_table_set_insert_path)")
    ap.add_argument("--no-find-uniform", action="store_true",
                    help="skip the uniform-popularity find (counter runs keep to the step's kernels)")
    ap.add_argument("--serve-footprint-gb", type=float, default=40.0)
    ap.add_argument("--serve-warmup", type=int, default=200)
    ap.add_argument("--serve-measured", type=int, default=2000)
    ap.add_argument("--serve-distinct", type=int, default=1000)
    ap.add_argument("--serve-timeout", type=float, default=300.0,
                    help="seconds the serving sweep may take before it is stopped")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-ceilings", action="store_true")
    ap.add_argument("--cpu-sample-shift", type=int, default=2,
                    help="oracle sample = the workload with every size divided by 2^shift")
    return ap.parse_args()


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def to_dev(a, dev):
    import torch

    return torch.from_numpy(np.ascontiguousarray(a).view(np.int64)).to(dev)


def measure_ceilings(ct, torch, dev, nlines, find_keys, uniform_keys, fill_keys=None):
    """Random 128-byte line gathers (R1), gather + CAS (R2), bare CAS (R3), stream copy (R4) at
    the table's footprint (nlines = the table's bucket count, so a key's line is its home
    bucket); R5 replays the find's own key stream through the R1 kernel and the fill's key stream
    through the R2 kernel."""
    buf = torch.zeros(nlines * 128, dtype=torch.uint8, device=dev)
    out = torch.empty(uniform_keys.numel(), dtype=torch.int64, device=dev)
    res = {}

    def timed(fn, reps=5):
        fn()
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(reps):
            fn()
        e1.record()
        torch.cuda.synchronize()
        return e0.elapsed_time(e1) / reps * 1e-3

    n = uniform_keys.numel()
    t = timed(lambda: ct.gather(buf, nlines, 128, uniform_keys, out))
    res["R1_gather128_Mlines_s"] = n / t / 1e6
    t = timed(lambda: ct.gather(buf, nlines * 2, 64, uniform_keys, out))
    res["R1_gather64_Mlines_s"] = n / t / 1e6
    t = timed(lambda: ct.gather(buf, nlines, 128, uniform_keys, out, cas=True))
    res["R2_gather128_cas_Mops_s"] = n / t / 1e6
    t = timed(lambda: ct.gather(buf, nlines, 128, uniform_keys, out, cas=True, store=True))
    res["R6_gather128_cas_store_Mops_s"] = n / t / 1e6
    t = timed(lambda: ct.cas_words(buf, nlines * 16, uniform_keys))
    res["R3_cas_Mops_s"] = n / t / 1e6
    nb = min(buf.numel(), 1 << 30)
    dst = torch.empty(nb, dtype=torch.uint8, device=dev)
    t = timed(lambda: ct.copy(buf, dst, nb))
    res["R4_copy_GB_s"] = 2 * nb / t / 1e9
    del dst
    out2 = torch.empty(find_keys.numel(), dtype=torch.int64, device=dev)
    t = timed(lambda: ct.gather(buf, nlines, 128, find_keys, out2))
    res["R5_find_stream_Mlines_s"] = find_keys.numel() / t / 1e6
    if fill_keys is not None:
        del out2
        out2 = torch.empty(fill_keys.numel(), dtype=torch.int64, device=dev)
        t = timed(lambda: ct.gather(buf, nlines, 128, fill_keys, out2, cas=True))
        res["R5_insert_stream_Mops_s"] = fill_keys.numel() / t / 1e6
    del buf, out, out2
    torch.cuda.empty_cache()
    # the same gathers (and gather + CAS) over the footprints of the other workloads: L2 (4 MiB
    # per XCD), the 256 MiB last-level cache, HBM at the large table's and the serving tables' size
    sweep = {}
    keys = uniform_keys[: 1 << 24]
    for name, nbytes in (("2MiB", 2 << 20), ("32MiB", 32 << 20), ("256MiB", 256 << 20),
                         ("1.34GB", nlines * 128), ("40GB", 40 << 30)):
        lines = nbytes // 128
        b = torch.zeros(lines * 128, dtype=torch.uint8, device=dev)
        o = torch.empty(keys.numel(), dtype=torch.int64, device=dev)
        t1 = timed(lambda: ct.gather(b, lines, 128, keys, o))
        t2 = timed(lambda: ct.gather(b, lines, 128, keys, o, cas=True))
        sweep[name] = {"R1_Mlines_s": keys.numel() / t1 / 1e6, "R2_Mops_s": keys.numel() / t2 / 1e6}
        del b, o
        torch.cuda.empty_cache()
    res["by_footprint"] = sweep
    return res


def host_cpu_model() -> str:
    """The host CPU's model name as the kernel reports it (first processor), else the machine."""
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return platform.processor() or platform.machine()


def cpu_baseline(shift, seed=3, runs=5):
    """The oracle as it stands, single-threaded, on the workload scaled down by 2^shift: the
    median of `runs` runs, each on a fresh oracle table (generation excluded)."""
    import oracle
    from paper_1908_05936_amd.workloads import large_table

    w = large_table(seed=seed, log2_keys=26 - shift, log2_queries=27 - shift, log2_churn=24 - shift)
    ops = w["insert_keys"].size + w["find"].size + w["erase"].size + w["reinsert_keys"].size

    def one(table):
        t0 = time.perf_counter()
        table.insert(w["insert_keys"], w["insert_vals"])
        table.find(w["find"])
        table.erase(w["erase"])
        table.insert(w["reinsert_keys"], w["reinsert_vals"])
        return time.perf_counter() - t0

    seq = []
    for _ in range(runs):
        o = oracle.OracleTable(w["capacity"], 64)
        seq.append(one(o))
        del o
    dt = float(np.median(seq))
    # the same sample on all host cores available to this process (up to 16): partitioned by key
    # hash, one oracle table and thread per partition, index order kept within each partition
    parts = max(1, min(16, len(os.sched_getaffinity(0)) if hasattr(os, "sched_getaffinity")
                      else os.cpu_count() or 1))
    par = []
    for _ in range(runs):
        po = oracle.PartitionedOracle(w["capacity"], parts)
        par.append(one(po))
        del po
    dtp = float(np.median(par))
    return {
        "value": ops / dt / 1e6,
        "unit": "Mops/s",
        "cores": 1,
        "kind": "oracle",
        "sample": (f"large_table scaled by 1/{1 << shift}: fill 2^{26 - shift}, "
                   f"2^{27 - shift} Zipf(1.1) finds (20% absent), erase 2^{24 - shift}, "
                   f"re-insert 2^{24 - shift}; {ops} ops, median {dt:.2f} s of {runs} runs "
                   f"(min {min(seq):.2f}, max {max(seq):.2f}), single thread"),
        "runs": runs,
        "host_cpu": host_cpu_model(),
        "host_threads_available": os.cpu_count(),
        "partitioned": {"value": ops / dtp / 1e6, "unit": "Mops/s", "cores": parts,
                        "kind": "oracle tables partitioned by key hash, one thread each",
                        "seconds": dtp, "runs": runs},
    }


def find_uniform(op_clear, op_fill, dev, K_fill, n_fill, n_find, n_hit, L, h, s, vals_out, found):
    """The find with uniform popularity (n_hit live keys drawn uniformly, the rest absent) right
    after a fill: no hot buckets, so it is compared with the uniform gather ceiling R1.  Mops/s,
    median of 3 runs timed with HIP events."""
    import torch
    from paper_1908_05936_amd import ct

    op_clear()
    op_fill()
    g = torch.Generator(device=dev)
    g.manual_seed(7)
    idx = torch.randint(0, n_fill, (n_hit,), device=dev, generator=g)
    absent = torch.randint(-(1 << 62), 1 << 62, (n_find - n_hit,), device=dev, generator=g)
    q = torch.cat([K_fill[idx], absent])[torch.randperm(n_find, device=dev, generator=g)]
    del idx, absent
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    ts = []
    for _ in range(3):
        e0.record()
        ct._check(L.ct_find_batch(h, ct._ptr(q), n_find, ct._ptr(vals_out), ct._ptr(found), s),
                  "find uniform")
        e1.record()
        torch.cuda.synchronize()
        ts.append(e0.elapsed_time(e1) * 1e-3)
    return n_find / float(np.median(ts)) / 1e6


def marginal_insert(dev, L, h, s, n=1 << 20, reps=3):
    """Insert n fresh keys into the table as the step leaves it (load 0.8), then erase them again
    (untimed) so the next run starts from the same state: Mops/s of the insert, median of `reps`
    runs timed with HIP events.  Fresh uniform u64 keys collide with a live key with probability
    about n * 2^26 / 2^64, so every status must read INSERTED."""
    import torch
    from paper_1908_05936_amd import ct

    g = torch.Generator(device=dev)
    g.manual_seed(11)
    keys = torch.randint(-(1 << 62), 1 << 62, (n,), device=dev, generator=g)
    vals = torch.arange(n, dtype=torch.int64, device=dev)
    st = torch.empty(n, dtype=torch.uint8, device=dev)
    er = torch.empty(n, dtype=torch.uint8, device=dev)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    ts = []
    for _ in range(reps):
        e0.record()
        ct._check(L.ct_insert_batch(h, ct._ptr(keys), ct._ptr(vals), n, ct._ptr(st), s), "marginal")
        e1.record()
        torch.cuda.synchronize()
        ts.append(e0.elapsed_time(e1) * 1e-3)
        assert int((st == 1).sum()) == n
        ct._check(L.ct_erase_batch(h, ct._ptr(keys), n, ct._ptr(er), s), "marginal erase")
    torch.cuda.synchronize()
    return n / float(np.median(ts)) / 1e6


def rehash_leg(table, K_re, V_re):
    """Host-side resize: the table as the step leaves it (2^26 live pairs at load 0.8) rehashed
    into a new table of twice the capacity.  Time of the whole call (its two size reads included)
    from HIP events on the stream, then a check of the size and of the re-inserted keys' values."""
    import torch
    from paper_1908_05936_amd import ct

    n = table.size()
    dst = ct.Table(2 * table.capacity, ct.VAL_U64, ct.HASH_MIX64, device=table.device)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    table.rehash_into(dst)
    e1.record()
    torch.cuda.synchronize()
    sec = e0.elapsed_time(e1) * 1e-3
    assert dst.size() == n
    v, f = dst.find(K_re)
    assert bool(f.all()) and bool((v == V_re).all())
    out = {"pairs": n, "ms": sec * 1e3, "Mpairs_s": n / sec / 1e6,
           "dst_capacity": dst.capacity, "dst_bytes": dst.nbytes}
    log(f"[rehash] {n} pairs into capacity {dst.capacity}: {out['ms']:.2f} ms, "
        f"{out['Mpairs_s']:.0f} Mpairs/s")
    del dst
    torch.cuda.empty_cache()
    return out


def mixed_device_leg(table, K_re, V_re, n=1 << 24):
    """Device-side operations of mixed kinds in one kernel (ct_dev_apply_mixed) on the table as the
    step leaves it (2^26 live pairs at load 0.8): n elements, 70% finds of resident keys, 20%
    inserts of fresh keys, 10% erases of other resident keys, in random order.  Every status is
    fixed by the workload and checked.  The same three operations are then timed as three batches
    of the batch path, on the same table state (the mixed call undone first), and the finds alone
    through a read-only device-side launch."""
    import torch
    from paper_1908_05936_amd import ct

    dev = table.device
    n_er, n_ins = n // 10, n // 5
    n_find = n - n_er - n_ins
    g = torch.Generator(device=dev)
    g.manual_seed(13)
    er = K_re[:n_er]
    er_v = V_re[:n_er]
    fidx = torch.randint(0, K_re.numel() - n_er, (n_find,), device=dev, generator=g)
    fq, fv = K_re[n_er:][fidx], V_re[n_er:][fidx]
    fresh = torch.randint(-(1 << 62), 1 << 62, (n_ins,), device=dev, generator=g)
    keys = torch.cat([fq, fresh, er])
    ops = torch.cat([torch.full((n_find,), ct.OP_FIND, dtype=torch.uint8, device=dev),
                     torch.full((n_ins,), ct.OP_INSERT, dtype=torch.uint8, device=dev),
                     torch.full((n_er,), ct.OP_ERASE, dtype=torch.uint8, device=dev)])
    perm = torch.randperm(n, device=dev, generator=g)
    keys, ops = keys[perm].contiguous(), ops[perm].contiguous()
    vals = keys.clone()
    n0 = table.size()
    wk = fq[:64].clone()
    table.dev_apply_mixed(torch.full((64,), ct.OP_FIND, dtype=torch.uint8, device=dev), wk, wk)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    st, _ = table.dev_apply_mixed(ops, keys, vals)
    e1.record()
    torch.cuda.synchronize()
    sec = e0.elapsed_time(e1) * 1e-3
    assert bool((st == 1).all()), "every find hits, every fresh key is INSERTED, every erase hits"
    assert table.size() == n0 + n_ins - n_er
    # undo, then the batch path on the same state
    table.erase(fresh)
    table.insert(er, er_v)
    assert table.size() == n0
    torch.cuda.synchronize()
    # the finds alone through a read-only device-side launch
    e0.record()
    rst, rv = table.dev_apply(ct.OP_FIND, fq)
    e1.record()
    torch.cuda.synchronize()
    rsec = e0.elapsed_time(e1) * 1e-3
    assert bool((rst == 1).all()) and bool((rv == fv).all())
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(4)]
    ev[0].record()
    v, f = table.find(fq)
    ev[1].record()
    table.insert(fresh, fresh)
    ev[2].record()
    table.erase(er)
    ev[3].record()
    torch.cuda.synchronize()
    bsec = ev[0].elapsed_time(ev[3]) * 1e-3
    assert bool(f.all()) and bool((v == fv).all()) and table.size() == n0 + n_ins - n_er
    fsec = ev[0].elapsed_time(ev[1]) * 1e-3
    out = {"n": n, "mix": "70% find / 20% insert / 10% erase", "ms": sec * 1e3,
           "Mops_s": n / sec / 1e6, "batch_path_ms": bsec * 1e3, "batch_path_Mops_s": n / bsec / 1e6,
           "finds": n_find, "read_only_find_ms": rsec * 1e3, "batch_find_ms": fsec * 1e3}
    log(f"[mixed device ops] {n} in one kernel: {out['ms']:.2f} ms, {out['Mops_s']:.0f} Mops/s; "
        f"as three batches {out['batch_path_ms']:.2f} ms; the {n_find} finds alone: read-only "
        f"device launch {out['read_only_find_ms']:.2f} ms, batch {out['batch_find_ms']:.2f} ms")
    return out


def pool_ops(dev, keys, reps=3):
    """The index pool (vector/deque back operations) at scale: n = keys.numel() distinct keys into
    a table of capacity n / 0.8 whose values are popped from a pool of capacity n, then released
    back (erase_release); also bare pops and pushes of n indices.  Mops/s, medians of `reps` runs
    timed with HIP events after one warm-up; the table is cleared before each insert."""
    import torch
    from paper_1908_05936_amd import ct

    L = ct.lib()
    s = ct._stream(dev)
    P = ct._ptr
    n = keys.numel()
    t = ct.Table(int(n / 0.8), ct.VAL_U32, ct.HASH_MIX64, device=dev)
    pool = ct.Pool(n, device=dev)
    idx = torch.empty(n, dtype=torch.int32, device=dev)
    st = torch.empty(n, dtype=torch.uint8, device=dev)
    er = torch.empty(n, dtype=torch.uint8, device=dev)
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(6)]
    times = {k: [] for k in ("insert_alloc", "erase_release", "pop", "push")}
    for r in range(reps + 1):
        ct._check(L.ct_clear(t._h, s), "clear")
        ev[0].record()
        ct._check(L.ct_insert_alloc_batch(t._h, pool._h, P(keys), n, P(idx), P(st), s), "insert_alloc")
        ev[1].record()
        ct._check(L.ct_erase_release_batch(t._h, pool._h, P(keys), n, P(er), s), "erase_release")
        ev[2].record()
        ct._check(L.ct_pool_pop_batch(pool._h, n, P(idx), P(st), s), "pop")
        ev[3].record()
        ct._check(L.ct_pool_push_batch(pool._h, P(idx), n, P(st), s), "push")
        ev[4].record()
        torch.cuda.synchronize()
        if r == 0:   # the warm-up also checks the results the workload fixes
            assert int(er.sum()) == n and pool.size() == n and t.size() == 0
            continue
        for j, k in enumerate(times):
            times[k].append(ev[j].elapsed_time(ev[j + 1]) * 1e-3)
    out = {k + "_Mops_s": n / float(np.median(v)) / 1e6 for k, v in times.items()}
    out["workload"] = (f"{n} distinct u64 keys, table capacity {int(n / 0.8)} (u32 values from a "
                       f"pool of {n} indices)")
    log(f"[pool] insert_alloc {out['insert_alloc_Mops_s']:.0f} erase_release "
        f"{out['erase_release_Mops_s']:.0f} pop {out['pop_Mops_s']:.0f} push "
        f"{out['push_Mops_s']:.0f} Mops/s")
    return out


def side_leg(name: str, fn) -> dict:
    """Run one of the line's side measurements; a Python-level failure (a refused launch, say)
    becomes an error entry instead of losing the whole line."""
    try:
        return fn()
    except Exception as e:  # noqa: BLE001  (any failure of a side leg is reported, not raised)
        log(f"[{name}] failed: {e!r}")
        return {"error": repr(e)}


def multi_table_leg(dev) -> dict:
    """The 256-table schedule (tables of 2^10..2^20 entries at load factors 0.5-0.9, a fill then a
    20/70/10 insert/find/erase mix of batches of 2^6..2^18 keys): the autotuner picks the execution
    form, merged runs, chunk, provisioning and block size on the seed-4 schedule in this run, and
    the choice is measured on the seed-6 schedule: plan run, HIP-graph replay and one library call
    per operation.  The ceiling is the schedule's own mix at its footprint: every insert or erase
    key costs one random line gather + CAS (R2), every find key one random line gather (R1), both
    measured here over a buffer of the tables' total size."""
    import torch
    from paper_1908_05936_amd import ct
    from paper_1908_05936_amd.multi import measure, tune
    from paper_1908_05936_amd.workloads import multi_table

    t0 = time.perf_counter()
    cfg = tune(multi_table(seed=4), dev, log=lambda m: None)
    torch.cuda.empty_cache()
    tune_s = time.perf_counter() - t0
    we = multi_table(seed=6)
    knobs = dict(lanes=cfg["lanes"], merge=cfg.get("merge", False), chunk=cfg["chunk"],
                 provision=cfg["provision"], block=cfg.get("block", 256))
    res = measure(we, dev, knobs)
    count = {"insert": 0, "find": 0, "erase": 0}
    for _, kind, keys, _ in we["schedule"]:
        count[kind] += keys.size
    del we
    torch.cuda.empty_cache()
    lines = max(1, res["table_bytes"] // 128)
    buf = torch.zeros(lines * 128, dtype=torch.uint8, device=dev)
    g = torch.Generator(device=dev)
    g.manual_seed(5)
    keys = torch.randint(0, 1 << 62, (1 << 24,), device=dev, generator=g)
    out = torch.empty(keys.numel(), dtype=torch.int64, device=dev)

    def timed(fn, reps=5):
        fn()
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(reps):
            fn()
        e1.record()
        torch.cuda.synchronize()
        return e0.elapsed_time(e1) / reps * 1e-3

    r1 = keys.numel() / timed(lambda: ct.gather(buf, lines, 128, keys, out))
    r2 = keys.numel() / timed(lambda: ct.gather(buf, lines, 128, keys, out, cas=True))
    del buf, keys, out
    torch.cuda.empty_cache()
    ceiling_s = (count["insert"] + count["erase"]) / r2 + count["find"] / r1
    best_ms = min(res["graph_replay_ms"], res["plan_ms"])
    out = {
        "workload": (f"{res['tables']} tables (2^10..2^20 entries, load 0.5-0.9, u64 keys, u32 "
                     f"values), {res['ops']} operations, {res['keys']} keys: fill, then 20/70/10 "
                     "insert/find/erase batches of 2^6..2^18 keys; tuned on seed 4, measured on "
                     "seed 6"),
        "tuned": knobs, "tuning_trials": cfg.get("trials"), "tuning_s": tune_s,
        "keys": res["keys"], "insert_keys": count["insert"], "find_keys": count["find"],
        "erase_keys": count["erase"], "table_bytes": res["table_bytes"],
        "plan_ms": res["plan_ms"], "graph_replay_ms": res["graph_replay_ms"],
        "per_batch_ms": res["per_batch_ms"], "streams4_ms": res["streams4_ms"],
        "plan_Mkeys_s": res["plan_Mkeys_s"], "graph_Mkeys_s": res["graph_Mkeys_s"],
        "per_batch_Mkeys_s": res["per_batch_Mkeys_s"],
        "speedup_vs_per_batch": res["per_batch_ms"] / best_ms,
        "grouped_launches": res.get("grouped_launches"), "grouped_steps": res.get("grouped_steps"),
        "single_launch_ms": res.get("single_launch_ms"),
        "single_launch_Mkeys_s": res.get("single_launch_Mkeys_s"),
        "R1_Mlines_s_at_footprint": r1 / 1e6, "R2_Mops_s_at_footprint": r2 / 1e6,
        "ceiling_ms": ceiling_s * 1e3,
        "frac_of_random_access_ceiling": ceiling_s / (best_ms * 1e-3),
    }
    log(f"[multi] tuned {knobs} in {tune_s:.0f} s; graph {res['graph_replay_ms']:.2f} ms "
        f"({res['graph_Mkeys_s']:.0f} Mkeys/s), per-batch {res['per_batch_ms']:.2f} ms; "
        f"{out['frac_of_random_access_ceiling']:.2f} of the R1/R2 ceiling at "
        f"{res['table_bytes'] / 1e9:.2f} GB")
    return out


def served_leg(child, timeout: float) -> dict:
    """Release the waiting serving child (bench_serve, same code path as in-process) and read its
    JSON line; its log goes to this process's stderr.  An error entry if it fails or does not
    finish within `timeout` seconds (then it is killed)."""
    import subprocess
    try:
        out, _ = child.communicate("go\n", timeout=timeout)
    except subprocess.TimeoutExpired:
        child.kill()
        child.communicate()
        log(f"the serving sweep did not finish within {timeout:.0f} s; it was stopped")
        return {"error": f"the serving sweep did not finish within {timeout:.0f} s"}
    if child.returncode != 0 or not out.strip():
        return {"error": f"the serving sweep exited with status {child.returncode}"}
    return json.loads(out.strip().splitlines()[-1])


def main():
    a = parse()
    if a.gpus != 1:
        print(f"bench.py runs on one GPU only; --gpus {a.gpus} is not supported "
              "(the container path runs on a single GPU; tables would shard by key hash across "
              "GPUs, which this library does not do)",
              file=sys.stderr)
        sys.exit(2)
    # the serving sweep runs in a child process, started here before this process touches the
    # GPU and held until the rest of the line is measured: if the sweep does not finish within
    # --serve-timeout seconds, the line is printed without it
    serve_child = None
    if not a.no_serve:
        import subprocess
        serve_child = subprocess.Popen(
            [sys.executable, "-u", "-m", "paper_1908_05936_amd.bench_serve", "--wait-stdin",
             "--footprint-gb", str(a.serve_footprint_gb), "--warmup", str(a.serve_warmup),
             "--measured", str(a.serve_measured), "--distinct", str(a.serve_distinct)],
            cwd=ROOT, stdin=subprocess.PIPE, stdout=subprocess.PIPE, text=True)
    import torch

    from paper_1908_05936_amd import ct
    from paper_1908_05936_amd.workloads import large_table

    dev = torch.device("cuda", 0)
    ct.lib()
    t0 = time.perf_counter()
    w = large_table(seed=3, log2_keys=a.log2_keys, log2_queries=a.log2_queries, log2_churn=a.log2_churn)
    log(f"generated workload in {time.perf_counter() - t0:.1f} s")
    n_fill = w["insert_keys"].size
    n_find = w["find"].size
    n_er = w["erase"].size
    n_re = w["reinsert_keys"].size
    cap = w["capacity"]
    K_fill, V_fill = to_dev(w["insert_keys"], dev), to_dev(w["insert_vals"], dev)
    Q = to_dev(w["find"], dev)
    E = to_dev(w["erase"], dev)
    K_re, V_re = to_dev(w["reinsert_keys"], dev), to_dev(w["reinsert_vals"], dev)
    n_present_expected = int(round(n_find * 0.8))
    del w

    table = ct.Table(cap, ct.VAL_U64, ct.HASH_MIX64, chunk=a.chunk, device=dev)
    table.set_insert_path(INSERT_PATHS[a.insert_path])
    st_fill = torch.empty(n_fill, dtype=torch.uint8, device=dev)
    vals_out = torch.empty(n_find, dtype=torch.int64, device=dev)
    found = torch.empty(n_find, dtype=torch.uint8, device=dev)
    erased = torch.empty(n_er, dtype=torch.uint8, device=dev)
    st_re = torch.empty(n_re, dtype=torch.uint8, device=dev)
    L = ct.lib()
    h = table._h
    s = ct._stream(dev)
    P = ct._ptr

    def op_clear():
        ct._check(L.ct_clear(h, s), "clear")

    def op_fill():
        ct._check(L.ct_insert_batch(h, P(K_fill), P(V_fill), n_fill, P(st_fill), s), "fill")

    def op_find():
        ct._check(L.ct_find_batch(h, P(Q), n_find, P(vals_out), P(found), s), "find")

    def op_erase():
        ct._check(L.ct_erase_batch(h, P(E), n_er, P(erased), s), "erase")

    def op_reins():
        ct._check(L.ct_insert_batch(h, P(K_re), P(V_re), n_re, P(st_re), s), "reinsert")

    ops = [("clear", op_clear), ("insert_fill", op_fill), ("find", op_find), ("erase", op_erase),
           ("insert_churn", op_reins)]
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(len(ops) + 1)]

    def step(timing):
        if timing:
            ev[0].record()
        for j, (_, fn) in enumerate(ops):
            fn()
            if timing:
                ev[j + 1].record()

    for _ in range(a.warmup):
        step(False)
    torch.cuda.synchronize()
    # sanity of the last warm-up step: sizes and hit counts the workload fixes
    if a.warmup:
        assert int((st_fill == 1).sum()) == n_fill
        assert int(found.sum()) == n_present_expected, int(found.sum())
        assert int(erased.sum()) == n_er and int((st_re == 1).sum()) == n_re
        assert table.size() == n_fill
    per = {name: 0.0 for name, _ in ops}
    torch.cuda.synchronize()
    w0 = time.perf_counter()
    for _ in range(a.steps):
        step(True)
        torch.cuda.synchronize()
        for j, (name, _) in enumerate(ops):
            per[name] += ev[j].elapsed_time(ev[j + 1]) * 1e-3
    torch.cuda.synchronize()
    wall = time.perf_counter() - w0
    # per-kernel times: the same number of steps again, with the library's event profiler on (it
    # records two events around every launch, so it stays out of the timed steps above)
    table.profiling(True)
    table.profile_reset()
    for _ in range(a.steps):
        step(False)
    torch.cuda.synchronize()
    total_ops = n_fill + n_find + n_er + n_re
    dev_time = sum(per.values())
    ms_step = wall / a.steps * 1e3
    counts = {"clear": 0, "insert_fill": n_fill, "find": n_find, "erase": n_er, "insert_churn": n_re}
    breakdown = {name: {"ms": per[name] / a.steps * 1e3,
                        "Mops_s": (counts[name] * a.steps / per[name] / 1e6) if counts[name] else None}
                 for name, _ in ops}
    # clear rewrites every 16-byte slot: the table's bytes over its time against HBM bandwidth
    breakdown["clear"]["GB_s"] = table.bucket_count * 128 * a.steps / per["clear"] / 1e9
    breakdown["clear"]["frac_of_hbm_peak"] = breakdown["clear"]["GB_s"] / HBM_PEAK_GBS
    prof = table.profile()
    table.profiling(False)
    n_ins = (n_fill + n_re) * a.steps
    kern = {
        "k_find": (prof["find"], FIND_BYTES * n_find * a.steps),
        "k_insert": (prof["insert"], INSERT_BYTES * n_ins),
        "k_erase": (prof["erase"], ERASE_BYTES * n_er * a.steps),
        "k_dedup": (prof["dedup"], None),
    }
    kernels = {}
    for name, ((ms, launches), alg) in kern.items():
        kernels[name] = {"ms_per_step": ms / a.steps, "launches_per_step": launches / a.steps,
                         "share_of_step": ms / (dev_time * 1e3) if dev_time else None}
        if alg is not None and ms:
            kernels[name]["achieved_GB_s"] = alg / (ms * 1e-3) / 1e9
            kernels[name]["algorithmic_bytes_per_launch"] = alg / launches
    dominant = max(("k_find", "k_insert", "k_erase"), key=lambda k: kernels[k]["ms_per_step"])
    traffic = recorded_traffic()
    tr, rname = None, None
    if traffic and dominant in traffic.get("kernels", {}):
        tk = traffic["kernels"][dominant]
        tr = tk["fetch_bytes_per_launch"] + tk["write_bytes_per_launch"]
        rname = tk.get("rocprof_name")
    dk = kernels[dominant]
    roof = {
        "kernel": dominant,          # the library profiler's kernel kind
        "rocprof_name": rname,       # the kernel of that kind in the committed profiles
        "bound": "hbm",
        "achieved": dk["achieved_GB_s"],
        "peak": HBM_PEAK_GBS,
        "unit": "GB/s",
        "frac": dk["achieved_GB_s"] / HBM_PEAK_GBS,
        "traffic": tr,
        "algorithmic_bytes_per_launch": dk["algorithmic_bytes_per_launch"],
        "mean_launch_ms": dk["ms_per_step"] / dk["launches_per_step"],
    }
    line = {
        "metric": METRIC,
        "value": total_ops * a.steps / dev_time / 1e6,
        "unit": "Mops/s",
        "n_gpus": 1,
        "steps": a.steps,
        "warmup": a.warmup,
        "ms_per_step": ms_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "u64",
        "data": "synthetic",
        "config": {
            "workload": (f"large_table: 2^{a.log2_keys} distinct u64 keys -> u64 values at load factor 0.8 "
                         f"({cap} slots, {cap * 16 / 1e9:.3f} GB), 2^{a.log2_queries} finds Zipf(1.1) "
                         f"with 20% absent, erase 2^{a.log2_churn}, re-insert 2^{a.log2_churn} fresh"),
            "capacity": cap,
            "bucket_count": table.bucket_count,
            "chunk": table.chunk,
            "insert_path": a.insert_path,
            "ops_per_step": total_ops,
            "wall_Mops_s": total_ops * a.steps / wall / 1e6,
        },
        "breakdown": breakdown,
        "kernels": kernels,
        "roofline": roof,
    }
    line["insert_marginal_Mops_s"] = marginal_insert(dev, L, h, s)
    log(f"marginal insert of 2^20 fresh keys at load 0.8: {line['insert_marginal_Mops_s']:.0f} Mops/s")
    if not a.no_rehash:
        line["rehash"] = side_leg("rehash", lambda: rehash_leg(table, K_re, V_re))
    if not a.no_mixed:
        line["mixed_device_ops"] = side_leg("mixed", lambda: mixed_device_leg(table, K_re, V_re))
    if not a.no_find_uniform:
        line["find_uniform_Mops_s"] = find_uniform(op_clear, op_fill, dev, K_fill, n_fill, n_find,
                                                   n_present_expected, L, h, s, vals_out, found)
    if not a.no_ceilings:
        rng = np.random.default_rng(99)
        uni = torch.from_numpy(rng.integers(0, 1 << 63, size=n_find, dtype=np.int64)).to(dev)
        del vals_out, found
        torch.cuda.empty_cache()
        ceil = measure_ceilings(ct, torch, dev, table.bucket_count, Q, uni, K_fill)
        f_mops = breakdown["find"]["Mops_s"]
        i_mops = breakdown["insert_fill"]["Mops_s"]
        ceil["find_frac_of_R1"] = f_mops / ceil["R1_gather128_Mlines_s"]
        ceil["find_frac_of_R5"] = f_mops / ceil["R5_find_stream_Mlines_s"]
        ceil["insert_frac_of_R2"] = i_mops / ceil["R2_gather128_cas_Mops_s"]
        ceil["insert_frac_of_R5"] = i_mops / ceil["R5_insert_stream_Mops_s"]
        ceil["insert_frac_of_R6"] = i_mops / ceil["R6_gather128_cas_store_Mops_s"]
        if "find_uniform_Mops_s" in line:
            ceil["find_uniform_frac_of_R1"] = (line["find_uniform_Mops_s"]
                                               / ceil["R1_gather128_Mlines_s"])
        line["random_access"] = ceil
    if not a.no_pool:
        line["pool"] = side_leg("pool", lambda: pool_ops(dev, K_fill[: min(n_fill, 1 << 24)]))
    if not a.no_voxel:
        from paper_1908_05936_amd import bench_voxel
        line["voxel"] = side_leg("voxel", lambda: bench_voxel.run(log=log))
    if "find_Mkeys_s" in line.get("voxel", {}) and "random_access" in line:
        # the voxel table is 2^21 buckets of 128 bytes: its find is compared with the gather
        # ceiling at that footprint (256 MiB, the last-level cache's size)
        r1 = line["random_access"]["by_footprint"]["256MiB"]["R1_Mlines_s"]
        line["voxel"]["find_R1_256MiB_Mlines_s"] = r1
        line["voxel"]["find_frac_of_R1_256MiB"] = line["voxel"]["find_Mkeys_s"] / r1
    if not a.no_multi:
        line["multi_table"] = side_leg("multi", lambda: multi_table_leg(dev))
    if serve_child is not None:
        del table, K_fill, V_fill, Q, E, K_re, V_re
        torch.cuda.empty_cache()
        res = served_leg(serve_child, a.serve_timeout)
        line["served"] = res if "error" in res else {
            "workload": (f"{res['tables']} tables, {res['resident_entries']} resident u64->u64 "
                         f"entries, {res['table_bytes'] / 1e9:.1f} GB; requests 20/70/10 "
                         "insert/find/erase, 2^8..2^20 keys, Zipf(1.1); Poisson arrivals"),
            "saturated_Mkeys_s": res["saturated_Mkeys_s"],
            "points": [{k: p[k] for k in ("offered_fraction", "p50_ms", "p99_ms", "achieved_Mkeys_s",
                                          "batches")} for p in res["points"]],
            "requests_per_point": res["requests"],
            "budget_bytes": res["budget_bytes"], "max_inflight": res["max_inflight"],
            "streams": res["streams"],
        }
    if not a.no_cpu_baseline:
        log("timing the CPU oracle sample")
        line["cpu_baseline"] = cpu_baseline(a.cpu_sample_shift)
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
