"""Host model of the speculative insert protocol (repeated keys resolved after the table update).

Elements of one insert chunk run as interleaved threads over a small bucketed table with the
layout rules of the GPU tables: 8 slots per bucket, a per-key probe sequence, occupancy in the key
word (EMPTY / TOMB), lookups stopping at the first bucket that holds the key or an EMPTY slot.
Every read of one slot and every compare-and-swap is a separate step, and a random scheduler picks
which thread takes the next step, so a bucket "read" by a thread may mix slot states from before
and after other threads' claims.  Each thread probes, claims the first free slot it saw, and on a
lost claim either stops (the winner holds its own key) or scans on while watching for its key.

After all threads end, a claimer whose key has a listed (ambiguous) copy of lower index hands the
insert to the lowest such copy; the model finds that copy both ways the kernels can (listed keys
into a table that claimers look up, or claimers into a table that listed copies lower) and
checks that they agree.  The test checks, over many
random schedules, tables with tombstones, and batches full of repeated and present keys, that

* no key is ever stored twice (the uniqueness of Section 4.1);
* statuses and the final contents equal the sequential replay (the batch semantics: the lowest
  index of a key acts first, later copies see the state it left).

The model is the protocol, not the kernel: the kernel's own results are compared with the oracle
on the GPU.
"""
import random

EMPTY = -1
TOMB = -2
SLOTS = 8
PRESENT, INSERTED = 0, 1


class Table:
    def __init__(self, nb, seed):
        self.nb = nb
        self.keys = [EMPTY] * (nb * SLOTS)
        self.vals = [0] * (nb * SLOTS)
        r = random.Random(seed)
        self.salt = r.randrange(1 << 30)

    def home_step(self, key):
        h = (key * 2654435761 + self.salt) & 0xFFFFFFFF
        home = h % self.nb
        step = 1 + (h >> 8) % (self.nb - 1) if self.nb > 1 else 0
        return home, step

    def seq(self, key):
        b, st = self.home_step(key)
        for _ in range(self.nb):
            yield b
            b = (b + st) % self.nb

    # sequential operations (used to build the state before the chunk)
    def find(self, key):
        for b in self.seq(key):
            row = self.keys[b * SLOTS:(b + 1) * SLOTS]
            if key in row:
                return b * SLOTS + row.index(key)
            if EMPTY in row:
                return None
        return None

    def insert_seq(self, key, val):
        if self.find(key) is not None:
            return PRESENT
        for b in self.seq(key):
            row = self.keys[b * SLOTS:(b + 1) * SLOTS]
            for c in range(SLOTS):
                if row[c] in (EMPTY, TOMB):
                    self.keys[b * SLOTS + c] = key
                    self.vals[b * SLOTS + c] = val
                    return INSERTED
        raise AssertionError("table physically full")

    def erase_seq(self, key):
        p = self.find(key)
        if p is None:
            return 0
        b = p // SLOTS
        row = self.keys[b * SLOTS:(b + 1) * SLOTS]
        self.keys[p] = EMPTY if EMPTY in row else TOMB
        return 1


def element(t, key, watch=True):
    """One element of a speculative chunk; yields ('r', slot) and ('cas', slot, expected, key)."""
    fb = fc = fexp = None
    for b in t.seq(key):
        row = []
        for c in range(SLOTS):
            v = yield ("r", b * SLOTS + c)
            row.append(v)
        if key in row:
            return ("amb", None)
        if fb is None:
            free = [c for c in range(SLOTS) if row[c] in (EMPTY, TOMB)]
            if free:
                fb, fc, fexp = b, free[0], row[free[0]]
        if EMPTY in row:
            break
    if fb is None:
        return ("full", None)
    ok, seen = yield ("cas", fb * SLOTS + fc, fexp, key)
    if ok:
        return ("claimed", fb * SLOTS + fc)
    if seen == key and watch:
        return ("amb", None)
    # the retry scans on from the bucket of the lost slot, watching for the key
    b, st = fb, t.home_step(key)[1]
    for _ in range(t.nb):
        row = []
        for c in range(SLOTS):
            v = yield ("r", b * SLOTS + c)
            row.append(v)
        if key in row and watch:
            return ("amb", None)
        for c in range(SLOTS):
            if row[c] in (EMPTY, TOMB):
                ok, seen = yield ("cas", b * SLOTS + c, row[c], key)
                if ok:
                    return ("claimed", b * SLOTS + c)
                if seen == key and watch:
                    return ("amb", None)
        b = (b + st) % t.nb
    return ("full", None)


def run_chunk(t, keys, vals, rng, watch=True):
    threads = {i: element(t, k, watch) for i, k in enumerate(keys)}
    pending = {}
    for i, g in threads.items():
        pending[i] = next(g)
    outcome = {}
    while pending:
        i = rng.choice(list(pending))
        op = pending[i]
        g = threads[i]
        if op[0] == "r":
            reply = t.keys[op[1]]
        else:
            _, slot, expected, desired = op
            cur = t.keys[slot]
            if cur == expected:
                t.keys[slot] = desired
                reply = (True, cur)
            else:
                reply = (False, cur)
        try:
            pending[i] = g.send(reply)
        except StopIteration as stop:
            outcome[i] = stop.value
            del pending[i]
            if stop.value[0] == "claimed":
                t.vals[stop.value[1]] = vals[i]
    for kind, _ in outcome.values():
        if kind == "full":
            raise AssertionError("FULL in a chunk that fits")
    a = resolve_by_listed(outcome, keys)
    b = resolve_by_claimers(outcome, keys)
    assert a == b, "the two resolution directions disagree"
    status = [PRESENT] * len(keys)
    for c, (kind, _) in outcome.items():
        if kind == "claimed":
            status[c] = INSERTED
    for c, m in a.items():
        t.vals[outcome[c][1]] = vals[m]
        status[m], status[c] = INSERTED, PRESENT
    return status


def resolve_by_listed(outcome, keys):
    """Listed keys enter the table with their lowest listed index; each claimer looks itself up.
    Returns {claimer: listed copy that takes the insert over}."""
    low = {}
    for i, (kind, _) in outcome.items():
        if kind == "amb":
            low[keys[i]] = min(low.get(keys[i], i), i)
    return {c: low[keys[c]] for c, (kind, _) in outcome.items()
            if kind == "claimed" and keys[c] in low and low[keys[c]] < c}


def resolve_by_claimers(outcome, keys):
    """Claimers enter the table; each listed copy below its key's claimer lowers the claimer's
    word, which the claimer checks afterwards."""
    entry = {keys[c]: c for c, (kind, _) in outcome.items() if kind == "claimed"}
    word = {}
    for i, (kind, _) in outcome.items():
        if kind == "amb" and keys[i] in entry and i < entry[keys[i]]:
            c = entry[keys[i]]
            word[c] = min(word.get(c, i), i)
    return word


def contents(t):
    return {k: v for k, v in zip(t.keys, t.vals) if k >= 0}


def one_case(seed, watch=True):
    rng = random.Random(seed)
    nb = rng.choice([1, 2, 3, 5, 7])
    universe = rng.randrange(4, 8 * nb + 8)
    t = Table(nb, seed)
    ref = Table(nb, seed)
    # a history of inserts and erases leaves tombstones on the probe paths
    for _ in range(rng.randrange(0, 6 * nb)):
        k = rng.randrange(universe)
        if rng.random() < 0.6 and sum(1 for x in t.keys if x >= 0) < 8 * nb - 1:
            for tab in (t, ref):
                tab.insert_seq(k, 1000 + k)
        else:
            for tab in (t, ref):
                tab.erase_seq(k)
    live = sum(1 for x in t.keys if x >= 0)
    room = 8 * nb - live  # capacity = every slot: the chunk cannot meet FULL when n <= room
    n = rng.randrange(1, max(2, min(room, 24)) + 1) if room else 0
    n = min(n, room)
    keys = [rng.randrange(universe) for _ in range(n)]
    vals = [5000 + 7 * i for i in range(n)]
    got = run_chunk(t, keys, vals, rng, watch)
    want = [ref.insert_seq(k, v) for k, v in zip(keys, vals)]
    assert got == want, (seed, keys, got, want)
    stored = [x for x in t.keys if x >= 0]
    assert len(stored) == len(set(stored)), (seed, "a key is stored twice")
    assert contents(t) == contents(ref), seed
    for k in stored:  # every live key is reachable by the lookup rule
        assert t.find(k) is not None, (seed, k)


def test_speculative_insert_matches_sequential_replay():
    for seed in range(3000):
        one_case(seed)


def test_without_the_watch_a_key_can_be_stored_twice():
    """The rescan after a lost claim must watch for the key.  A rescan that looks for free slots
    only (a plausible mistake, planted here in the model) stores some key twice, or breaks the
    replay, under some of the same random schedules."""
    failures = 0
    for seed in range(3000):
        try:
            one_case(seed, watch=False)
        except AssertionError:
            failures += 1
    assert failures > 0
