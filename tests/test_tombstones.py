"""Tombstone churn, on a host model of the table layout (no GPU).

The model follows the layout the kernels use: buckets of 8 slots, a probe sequence home,
home + s, home + 2s, ... (mod a prime bucket count) per key; a lookup stops at the first bucket
holding the key or an empty slot; an insert takes the first free (empty or tombstone) slot at or
before the first bucket holding an empty slot; an erase leaves an empty slot where its bucket
already holds one and a tombstone otherwise.  Its results are checked against a dict.

Under churn near full load a bucket that loses its last empty slot never regains one, so the
walks of absent keys grow without bound.  The purge (ct_table_purge) reopens every bucket that no
live key's walk passes, turning its tombstones into empty slots; with it the walks stay short and
the results do not change.
"""
import random

EMPTY, TOMB = -1, -2


class Model:
    def __init__(self, nb, seed=0):
        self.nb = nb
        self.slots = [[EMPTY] * 8 for _ in range(nb)]
        self.rng = random.Random(seed)

    def seq(self, key):
        h = hash((key, 0x9E37)) & ((1 << 62) - 1)
        home = h % self.nb
        step = 1 + (h // self.nb) % (self.nb - 1)
        b = home
        for _ in range(self.nb):
            yield b
            b = (b + step) % self.nb

    def find(self, key):
        """(found, buckets visited)."""
        n = 0
        for b in self.seq(key):
            n += 1
            row = self.slots[b]
            if key in row:
                return True, n
            if EMPTY in row:
                return False, n
        return False, n

    def insert(self, key):
        free = None
        for b in self.seq(key):
            row = self.slots[b]
            if key in row:
                return False
            if free is None:
                for c in range(8):
                    if row[c] in (EMPTY, TOMB):
                        free = (b, c)
                        break
            if EMPTY in row:
                break
        assert free is not None, "table physically full"
        self.slots[free[0]][free[1]] = key
        return True

    def erase(self, key):
        for b in self.seq(key):
            row = self.slots[b]
            if key in row:
                c = row.index(key)
                row[c] = EMPTY if EMPTY in row else TOMB
                return True
            if EMPTY in row:
                return False
        return False

    def purge(self):
        passed = [False] * self.nb
        for at in range(self.nb):
            for key in self.slots[at]:
                if key in (EMPTY, TOMB):
                    continue
                for b in self.seq(key):
                    if b == at:
                        break
                    passed[b] = True
        for b in range(self.nb):
            if not passed[b]:
                self.slots[b] = [EMPTY if k == TOMB else k for k in self.slots[b]]

    def closed(self):
        return sum(EMPTY not in row for row in self.slots)


def churn(purge_every, rounds=120, nb=251, load=0.8, frac=0.1, seed=1):
    """Fill to `load`, then `rounds` of erasing and re-inserting `frac` of the keys; returns the
    mean walk of absent-key lookups per round and the closed-bucket counts."""
    rng = random.Random(seed)
    m, ref = Model(nb, seed), {}
    n = int(load * nb * 8)
    nxt = 0
    for _ in range(n):
        nxt += 1
        assert m.insert(nxt) == (nxt not in ref)
        ref[nxt] = 1
    walks, closed = [], []
    for r in range(rounds):
        live = list(ref)
        for key in rng.sample(live, int(frac * n)):
            assert m.erase(key)
            del ref[key]
        for _ in range(int(frac * n)):
            nxt += 1
            assert m.insert(nxt)
            ref[nxt] = 1
        if purge_every and (r + 1) % purge_every == 0:
            m.purge()
        probes = [m.find(-(k + 10)) for k in range(400)]
        assert not any(f for f, _ in probes)
        walks.append(sum(w for _, w in probes) / len(probes))
        closed.append(m.closed())
        for key in rng.sample(list(ref), 50):
            assert m.find(key)[0]
    return walks, closed, m, ref


def test_churn_without_purge_closes_buckets_and_lengthens_walks():
    walks, closed, _, _ = churn(purge_every=0)
    assert closed[-1] > 2 * closed[0]
    assert walks[-1] > 2 * walks[0]


def test_purge_keeps_walks_short_and_results_unchanged():
    walks, closed, m, ref = churn(purge_every=1)
    free_walks, free_closed, _, _ = churn(purge_every=0)
    # without the purge every bucket closes and an absent key walks all of them; with it the
    # walks settle at a few buckets
    assert free_walks[-1] == 251
    assert max(walks) < 8.0
    assert closed[-1] < free_closed[-1]
    assert walks[-1] < free_walks[-1] / 20
    # every live key is still found, and nothing else is
    for key in ref:
        assert m.find(key)[0]
    assert sum(k not in (EMPTY, TOMB) for row in m.slots for k in row) == len(ref)
