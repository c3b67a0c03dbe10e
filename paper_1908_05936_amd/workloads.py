"""Seeded synthetic workloads for the batch container operations.

This module only draws inputs: keys, values, query mixes and their order.  It holds none of the
containers' arithmetic (no hashing, no probing, no batch semantics), so the CPU reference and the
GPU library can both be fed from it without sharing any of the method.

Every generator takes an explicit seed and uses numpy's PCG64 generator, so a run is reproducible
on any machine with the same numpy.  Keys are returned as ``numpy.uint64`` arrays; all 2^64 key
values are legal inputs (the containers mark slot occupancy without reserving key values,
Section 5.1), so the draws are over the full 64-bit range.

Workloads (sizes are parameters so tests can run scaled-down copies):

* ``plain_table``   -- uniform distinct keys, values = batch index, a 50/50 present/absent find,
                      an erase of a quarter of the keys and a final find of all keys.
* ``large_table``   -- distinct uniform keys at load factor 0.8, Zipf(1.1) find popularity with a
                      share of absent keys, then erase + re-insert of fresh keys.
* ``voxel_blocks``  -- packed signed 21-bit int3 block coordinates sampled on spheres and planes in
                      a 4096^3 grid, visited by a moving frustum (the reconstruction use case of
                      Section 4.1).
"""
from __future__ import annotations

import math

import numpy as np

U64 = np.uint64
M21 = (1 << 21) - 1


def rng_for(seed: int, stream: int = 0) -> np.random.Generator:
    """Independent PCG64 stream ``stream`` of seed ``seed``."""
    return np.random.Generator(np.random.PCG64(np.random.SeedSequence([int(seed), int(stream)])))


def uniform_u64(rng: np.random.Generator, n: int) -> np.ndarray:
    return rng.integers(0, 1 << 64, size=int(n), dtype=np.uint64, endpoint=False)


def distinct_u64(rng: np.random.Generator, n: int, exclude: np.ndarray | None = None) -> np.ndarray:
    """``n`` distinct uniform u64 keys in draw order; repeats (and members of ``exclude``) are redrawn."""
    n = int(n)
    out = np.empty(0, dtype=np.uint64)
    excl = np.empty(0, dtype=np.uint64) if exclude is None else np.unique(np.asarray(exclude, np.uint64))
    while out.size < n:
        need = n - out.size
        cand = np.concatenate([out, uniform_u64(rng, need + need // 64 + 16)])
        _, first = np.unique(cand, return_index=True)
        keep = np.zeros(cand.size, dtype=bool)
        keep[first] = True
        if excl.size:
            keep &= ~np.isin(cand, excl)
        out = cand[keep][:n] if keep.sum() >= n else cand[keep]
    return out


def splitmix64(seed: int, start: int, n: int) -> np.ndarray:
    """Outputs ``start .. start+n-1`` of the splitmix64 generator seeded with ``seed``
    (Steele, Lea & Flood 2014).  Its output function is a bijection of the 64-bit state and the
    states of distinct counters differ, so outputs of distinct counters are distinct keys: disjoint
    counter ranges give disjoint key sets without any de-duplication pass.
    """
    gamma = np.uint64(0x9E3779B97F4A7C15)
    i = np.arange(int(start) + 1, int(start) + int(n) + 1, dtype=np.uint64)
    z = np.uint64(int(seed) & ((1 << 64) - 1)) + i * gamma
    z = (z ^ (z >> np.uint64(30))) * np.uint64(0xBF58476D1CE4E5B9)
    z = (z ^ (z >> np.uint64(27))) * np.uint64(0x94D049BB133111EB)
    return z ^ (z >> np.uint64(31))


def zipf_ranks(rng: np.random.Generator, n: int, num_elements: int, exponent: float) -> np.ndarray:
    """``n`` ranks in [1, num_elements] with P(k) proportional to k^-exponent.

    Rejection-inversion (Hoermann & Derflinger 1996, "Rejection-inversion to generate variates
    from monotone discrete distributions"): the continuous hat g(x) = x^-s dominates the
    probabilities in the sense that the mass g gives to [k - 1/2, k + 1/2] is at least k^-s (g is
    convex).  With G an antiderivative of g, a point u drawn uniformly from [G(1/2), G(N + 1/2)]
    is inverted to x = G^-1(u) and rounded to the nearest rank k; the point is kept when it falls
    into the last k^-s of the slice [G(k - 1/2), G(k + 1/2)] that maps to k, so each rank is kept
    with probability proportional to k^-s, and the rest are drawn again.
    """
    s = float(exponent)
    if s <= 0.0:
        raise ValueError("the exponent must be positive")
    N = float(num_elements)
    a = 1.0 - s

    def g(x):
        return np.power(x, -s)

    if a == 0.0:   # s == 1: G = log
        G, Ginv = np.log, np.exp
    else:          # G(x) = (x^a - 1) / a, written with expm1 / log1p to keep small a exact
        def G(x):
            return np.expm1(a * np.log(x)) / a

        def Ginv(u):
            return np.exp(np.log1p(a * u) / a)

    lo, hi = G(np.float64(0.5)), G(np.float64(N + 0.5))
    out = np.empty(int(n), dtype=np.int64)
    todo = np.arange(int(n))
    while todo.size:
        u = lo + rng.random(todo.size) * (hi - lo)
        k = np.clip(np.floor(Ginv(u) + 0.5), 1.0, N)
        keep = u >= G(k + 0.5) - g(k)
        out[todo[keep]] = k[keep].astype(np.int64)
        todo = todo[~keep]
    return out


# --------------------------------------------------------------------------------------------
# plain single table: u64 keys, u32 values = batch index
# --------------------------------------------------------------------------------------------
def plain_table(seed: int = 1, log2_keys: int = 16, log2_capacity: int = 17) -> dict:
    rng = rng_for(seed)
    n = 1 << log2_keys
    keys = distinct_u64(rng, n)
    vals = np.arange(n, dtype=np.uint32)
    half = n // 2
    present = keys[rng.integers(0, n, size=half)]
    absent = distinct_u64(rng, n - half, exclude=keys)
    q1 = np.concatenate([present, absent])
    q1 = q1[rng.permutation(q1.size)]
    erase = keys[rng.choice(n, size=n // 4, replace=False)]
    q2 = keys[rng.permutation(n)]
    return dict(capacity=1 << log2_capacity, insert_keys=keys, insert_vals=vals, find1=q1,
                erase=erase, find2=q2)


# --------------------------------------------------------------------------------------------
# large table at load factor 0.8: u64 keys, u64 values = insertion ordinal
# --------------------------------------------------------------------------------------------
def large_table(seed: int = 3, log2_keys: int = 26, log2_queries: int = 27, log2_churn: int = 24,
                absent_frac: float = 0.2, zipf_s: float = 1.1, load_factor: float = 0.8,
                uniform: bool = False) -> dict:
    """Fill to ``load_factor``, Zipf finds with ``absent_frac`` absent keys, erase + fresh re-insert.

    ``capacity`` = live keys / load factor, the number of 16-byte slots (2^26 keys -> 83,886,080
    slots, 1.342 GB).  The churn (erase 2^24 then insert 2^24 fresh keys) returns to the same load.
    """
    rng = rng_for(seed)
    n = 1 << log2_keys
    nq = 1 << log2_queries
    nc = 1 << log2_churn
    capacity = int(round(n / load_factor))
    keys = splitmix64(seed, 0, n)
    vals = np.arange(n, dtype=np.uint64)
    n_abs = int(round(nq * absent_frac))
    n_pre = nq - n_abs
    if uniform:
        pre = keys[rng.integers(0, n, size=n_pre)]
    else:
        perm = rng.permutation(n)                     # rank r (1-based) -> keys[perm[r-1]]
        ranks = zipf_ranks(rng, n_pre, n, zipf_s)
        pre = keys[perm[ranks - 1]]
    fresh = splitmix64(seed, n, n_abs + nc)          # disjoint from the live keys
    absent = fresh[:n_abs]
    q = np.concatenate([pre, absent])
    q = q[rng.permutation(nq)]
    erase = keys[rng.choice(n, size=nc, replace=False)]
    reins = fresh[n_abs:]
    reins_vals = np.arange(n, n + nc, dtype=np.uint64)
    return dict(capacity=capacity, insert_keys=keys, insert_vals=vals, find=q, erase=erase,
                reinsert_keys=reins, reinsert_vals=reins_vals)


# --------------------------------------------------------------------------------------------
# voxel-block coordinates
# --------------------------------------------------------------------------------------------
def pack_int3(x, y, z) -> np.ndarray:
    """Pack signed 21-bit block coordinates into one u64: x in bits 0-20, y in 21-41, z in 42-62.

    This is the key encoding of the voxel workload (an input format, not part of the method):
    each component is taken modulo 2^21 (two's complement), bit 63 is zero.
    """
    x = np.asarray(x, dtype=np.int64).astype(np.uint64) & U64(M21)
    y = np.asarray(y, dtype=np.int64).astype(np.uint64) & U64(M21)
    z = np.asarray(z, dtype=np.int64).astype(np.uint64) & U64(M21)
    return x | (y << U64(21)) | (z << U64(42))


def _surface_points(rng, n_spheres, n_planes, grid_half, r_lo, r_hi, npts):
    """Area-weighted uniform points on spheres and clipped planes inside [-grid_half, grid_half)^3."""
    radii = rng.uniform(r_lo, r_hi, size=n_spheres)
    centres = np.stack([rng.uniform(-grid_half + r, grid_half - r, size=3) for r in radii])
    normals = rng.normal(size=(n_planes, 3))
    normals /= np.linalg.norm(normals, axis=1, keepdims=True)
    anchors = rng.uniform(-grid_half / 2, grid_half / 2, size=(n_planes, 3))
    # plane area inside the cube: approximate by the square of side 2*grid_half spanned in the plane
    sphere_area = 4.0 * math.pi * radii ** 2
    plane_area = np.full(n_planes, (2.0 * grid_half) ** 2)
    w = np.concatenate([sphere_area, plane_area])
    w = w / w.sum()
    which = rng.choice(w.size, size=npts, p=w)
    pts = np.empty((npts, 3))
    sph = which < n_spheres
    ns = int(sph.sum())
    d = rng.normal(size=(ns, 3))
    d /= np.linalg.norm(d, axis=1, keepdims=True)
    idx = which[sph]
    pts[sph] = centres[idx] + d * radii[idx, None]
    pl = ~sph
    pidx = which[pl] - n_spheres
    nrm = normals[pidx]
    # orthonormal basis (u, v) of each plane
    a = np.where(np.abs(nrm[:, :1]) < 0.9, np.array([[1.0, 0, 0]]), np.array([[0, 1.0, 0]]))
    u = np.cross(nrm, a)
    u /= np.linalg.norm(u, axis=1, keepdims=True)
    v = np.cross(nrm, u)
    st = rng.uniform(-2.0 * grid_half, 2.0 * grid_half, size=(pl.sum(), 2))
    pts[pl] = anchors[pidx] + u * st[:, :1] + v * st[:, 1:]
    inside = np.all((pts >= -grid_half) & (pts < grid_half), axis=1)
    return pts[inside]


def voxel_blocks(seed: int = 2, n_distinct: int = 1 << 22, n_resident: int = 1 << 20,
                 frames: int = 100, frame_queries: int = 1 << 18, hit_frac: float = 0.9,
                 n_spheres: int = 64, n_planes: int = 8, grid: int = 4096,
                 r_lo: float = 50.0, r_hi: float = 400.0) -> dict:
    """Reconstruction-style block keys visited by a frustum that moves along a seeded direction.

    The distinct surface blocks are sorted by their projection on a random unit direction; the
    first ``n_resident`` are the initial residents.  Frame f queries ``frame_queries`` keys: the
    next ``misses`` unseen blocks along the path plus ``hits`` blocks drawn without replacement from
    the trailing resident window, shuffled.  The caller inserts the misses after each find.
    """
    rng = rng_for(seed)
    half = grid // 2
    blocks = np.empty((0, 3), dtype=np.int64)
    keys = np.empty(0, dtype=np.uint64)
    while blocks.shape[0] < n_distinct:
        need = n_distinct - blocks.shape[0]
        pts = _surface_points(rng, n_spheres, n_planes, half, r_lo, r_hi, max(need * 2, 4096))
        b = np.floor(pts).astype(np.int64)
        b = np.concatenate([blocks, b])
        k = np.concatenate([keys, pack_int3(b[blocks.shape[0]:, 0], b[blocks.shape[0]:, 1],
                                            b[blocks.shape[0]:, 2])])
        _, first = np.unique(k, return_index=True)   # the packing is injective on the grid
        first.sort()
        first = first[:n_distinct]
        blocks, keys = b[first], k[first]
    d = rng.normal(size=3)
    d /= np.linalg.norm(d)
    proj = blocks.astype(np.float64) @ d
    order = np.lexsort((keys, proj))
    path = keys[order]
    misses = int(round(frame_queries * (1.0 - hit_frac)))
    hits = frame_queries - misses
    window = n_resident // 2
    frame_list = []
    for f in range(frames):
        end = n_resident + misses * f
        new = path[end:end + misses]
        lo = max(0, end - window)
        hit = path[lo + rng.choice(end - lo, size=hits, replace=False)]
        q = np.concatenate([hit, new])
        frame_list.append(q[rng.permutation(q.size)])
    return dict(path=path, residents=path[:n_resident], frames=frame_list,
                pool_capacity=1 << 22, bucket_count=1 << 21)


# --------------------------------------------------------------------------------------------
# many tables, one schedule
# --------------------------------------------------------------------------------------------
def _log_uniform_int(rng, lo_log2, hi_log2, size=None):
    return np.rint(np.exp2(rng.uniform(lo_log2, hi_log2, size=size))).astype(np.int64)


def multi_table(seed: int = 4, n_tables: int = 256, entries_log2=(10, 20), lf=(0.5, 0.9),
                batch_log2=(6, 18), mix_ops_per_table: int = 4, mix=(0.2, 0.7, 0.1)) -> dict:
    """Independent tables of log-uniform size and load factor, then one interleaved schedule.

    Phase 1 fills table t to entries_t fresh keys with insert batches of log-uniform size (the last
    one truncated); phase 2 runs `mix_ops_per_table` operations per table drawn insert / find /
    erase with probabilities `mix`.  Finds ask half live and half never-inserted keys; erases take
    live keys; phase-2 inserts take half fresh and half live keys.  Per-table order is sequential;
    the tables are interleaved by a seeded draw weighted by the operations each has left.
    Values are u32.  Returns tables [{capacity, entries, load_factor}] and schedule
    [(table, op, keys, vals)] with op in {"insert", "find", "erase"}.
    """
    rng = rng_for(seed)
    tables, per_table = [], []
    counter = 0
    for t in range(n_tables):
        entries = int(_log_uniform_int(rng, *entries_log2))
        load = float(rng.uniform(*lf))
        cap = int(math.ceil(entries / load))
        tables.append(dict(capacity=cap, entries=entries, load_factor=load))
        keys = splitmix64(seed * 1000003 + t, 0, entries)
        fresh_next = entries
        ops = []
        pos = 0
        while pos < entries:
            b = int(_log_uniform_int(rng, *batch_log2))
            k = keys[pos:pos + b]
            ops.append(("insert", k, rng.integers(0, 1 << 32, size=k.size, dtype=np.uint64).astype(np.uint32)))
            pos += k.size
        for _ in range(mix_ops_per_table):
            kind = rng.choice(["insert", "find", "erase"], p=list(mix))
            b = int(_log_uniform_int(rng, *batch_log2))
            if kind == "find":
                half = b // 2
                k = np.concatenate([keys[rng.integers(0, entries, size=half)],
                                    splitmix64(seed * 1000003 + t, fresh_next, b - half)])
                fresh_next += b - half
                k = k[rng.permutation(k.size)]
                ops.append(("find", k, None))
            elif kind == "erase":
                ops.append(("erase", keys[rng.integers(0, entries, size=b)], None))
            else:
                half = b // 2
                k = np.concatenate([splitmix64(seed * 1000003 + t, fresh_next, half),
                                    keys[rng.integers(0, entries, size=b - half)]])
                fresh_next += half
                k = k[rng.permutation(k.size)]
                ops.append(("insert", k, rng.integers(0, 1 << 32, size=k.size, dtype=np.uint64).astype(np.uint32)))
        per_table.append(ops)
    left = np.array([len(o) for o in per_table], dtype=np.float64)
    nxt = [0] * n_tables
    schedule = []
    while left.sum() > 0:
        t = int(rng.choice(n_tables, p=left / left.sum()))
        kind, k, v = per_table[t][nxt[t]]
        schedule.append((t, kind, k, v))
        nxt[t] += 1
        left[t] -= 1
    return dict(tables=tables, schedule=schedule)


# --------------------------------------------------------------------------------------------
# serving: many resident tables, Poisson arrivals of uneven requests
# --------------------------------------------------------------------------------------------
def splitmix64_at(seed: int, idx) -> np.ndarray:
    """splitmix64 outputs at arbitrary counter positions `idx` (same values as ``splitmix64``)."""
    gamma = np.uint64(0x9E3779B97F4A7C15)
    i = np.asarray(idx, dtype=np.uint64) + np.uint64(1)
    z = np.uint64(int(seed) & ((1 << 64) - 1)) + i * gamma
    z = (z ^ (z >> np.uint64(30))) * np.uint64(0xBF58476D1CE4E5B9)
    z = (z ^ (z >> np.uint64(27))) * np.uint64(0x94D049BB133111EB)
    return z ^ (z >> np.uint64(31))


class Serving:
    """Tables of log-uniform size with a key universe of twice their entries (the first half
    resident at start) and a stream of requests: table uniform, kind by `mix` (insert, find,
    erase), size log-uniform, keys Zipf(`zipf_s`) over a seeded permutation of the table's
    universe, values request_id * 2^32 + position.  Requests are drawn on demand, so the key
    universe is never materialised: key(t, j) = splitmix64 output j of the table's seed, and the
    permutation is j = (a * (rank - 1) + b) mod U with a coprime to U.
    """

    def __init__(self, seed: int = 5, n_tables: int = 64, entries_log2=(16, 26),
                 req_log2=(8, 20), mix=(0.2, 0.7, 0.1), zipf_s: float = 1.1,
                 rank_pool: int = 1 << 22):
        self.seed = seed
        self.rng = rng_for(seed, 1)
        r0 = rng_for(seed, 0)
        self.entries = [int(x) for x in _log_uniform_int(r0, *entries_log2, size=n_tables)]
        self.universe = [2 * e for e in self.entries]
        self.seeds = [seed * 7919 + t for t in range(n_tables)]
        self.perm = []
        for u in self.universe:
            while True:
                a = int(r0.integers(1, u))
                if math.gcd(a, u) == 1:
                    break
            self.perm.append((a, int(r0.integers(0, u))))
        self.req_log2 = req_log2
        self.mix = mix
        umax = max(self.universe)
        self.ranks = zipf_ranks(r0, rank_pool, umax, zipf_s)  # shared pool, filtered per table
        self._ranks2 = np.concatenate([self.ranks, self.ranks])  # windows wrap around the pool
        self.next_id = 0

    def resident(self, t: int, lo: int, hi: int) -> np.ndarray:
        """Keys j in [lo, hi) of table t's resident half."""
        return splitmix64_at(self.seeds[t], np.arange(lo, hi, dtype=np.uint64))

    def _header(self):
        """Draw the next request's id, table, kind and Zipf ranks (the sequential part)."""
        rng = self.rng
        t = int(rng.integers(0, len(self.entries)))
        kind = ["insert", "find", "erase"][int(rng.choice(3, p=list(self.mix)))]
        n = int(_log_uniform_int(rng, *self.req_log2))
        u = self.universe[t]
        parts, have = [], 0
        pool = self.ranks.size
        while have < n:
            off = int(rng.integers(0, pool))
            m = min(2 * n + 64, pool)
            r = self._ranks2[off:off + m]
            r = r[r <= u]
            parts.append(r)
            have += r.size
        ranks = np.concatenate(parts)[:n] if len(parts) > 1 else parts[0][:n]
        rid = self.next_id
        self.next_id += 1
        return rid, t, kind, ranks

    def _materialise(self, head):
        rid, t, kind, ranks = head
        a, b = self.perm[t]
        u = self.universe[t]
        j = (a * (ranks - 1) + b) % u        # a, rank < 2^28: the product fits in int64
        keys = splitmix64_at(self.seeds[t], j.astype(np.uint64))
        vals = None
        if kind == "insert":
            vals = (np.uint64(rid) << np.uint64(32)) + np.arange(ranks.size, dtype=np.uint64)
        return rid, t, kind, keys, vals

    def request(self):
        """(id, table, kind, keys, vals) of the next request."""
        return self._materialise(self._header())

    def requests(self, k: int, threads: int = 8):
        """The next `k` requests, equal to `k` calls of ``request``; keys computed on `threads`
        host threads."""
        heads = [self._header() for _ in range(k)]
        if threads <= 1:
            return [self._materialise(h) for h in heads]
        from concurrent.futures import ThreadPoolExecutor
        with ThreadPoolExecutor(threads) as ex:
            return list(ex.map(self._materialise, heads))
