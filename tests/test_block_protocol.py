"""Host model of the block protocol of the bin scatter kernels (no GPU).

A scatter block stages its elements in LDS and writes them out in a loop over the staged count,
which a block-wide scan produces: lane 63 of every wave stores its wave's sum in one LDS word and
every thread adds the words up.  A wave that leaves the kernel before the scan never stores its
word, and that word then holds whatever an earlier workgroup left in LDS.

The kernels decide whether to leave from the chunk's overflow flag, which other blocks of the same
launch may raise while a block starts.  When each wave read the flag on its own, the waves of one
block could disagree: the staying waves then added stale words into the staged count.  The LDS
words our kernels initialise are mostly all-ones (empty keys, "no index" markers), and an
all-ones word in place of wave 0's sum makes the staged count 2^32 - 1.  The staging loop counts
with a 32-bit position that steps by the block size, so it wraps around before it reaches that
count and never ends: the kernel runs forever, its stream never completes, and a server waiting
for that stream's batches stalls with the GPU busy.

The kernels now read the flag once per block (one thread, then a barrier), so all waves leave or
none does, and the staging loop is bounded by the tile size whatever the scan returns.  This model
replays both protocols at wave granularity.
"""
import itertools

import pytest

MASK = (1 << 32) - 1
BLOCK = 256          # threads per block
WAVES = BLOCK // 64
TILE = 2048          # elements a block stages at most
TRIP_CAP = (1 << 24) + 2   # more trips than any 32-bit count can need without wrapping


def scan_total(alive, counts, stale):
    """Staged count as the block scan computes it: live waves store their sums, the words of
    waves that left keep the stale LDS values; every thread adds the WAVES words (mod 2^32)."""
    words = list(stale)
    for w in range(WAVES):
        if alive[w]:
            words[w] = sum(counts[w * 64:(w + 1) * 64]) & MASK
    return sum(words) & MASK


def staging_trips(tid, total, bounded):
    """Trips of thread `tid` through the staging loop (p += BLOCK on a 32-bit p), stopped at
    TRIP_CAP.  bounded: the loop runs to min(total, TILE), as the kernels now do."""
    end = min(total, TILE) if bounded else total
    p, trips = tid, 0
    while p < end:
        p = (p + BLOCK) & MASK
        trips += 1
        if trips >= TRIP_CAP:
            break
    return trips


def per_wave_decisions(flag_seen_by_wave):
    """Old protocol: each wave leaves when its own read of the flag saw it raised."""
    return [not seen for seen in flag_seen_by_wave]


def per_block_decision(flag_seen_by_wave):
    """Current protocol: thread 0 (wave 0) reads the flag, a barrier shares it with every wave."""
    stay = not flag_seen_by_wave[0]
    return [stay] * WAVES


def tile_counts(n_elements):
    """Per-thread contributions of a tile of n elements spread over 16 bins (threads 0..15)."""
    counts = [0] * BLOCK
    for j in range(n_elements):
        counts[j % 16] += 1
    return counts


def test_per_wave_reads_can_wrap_the_staging_loop():
    """The failure: wave 0 saw the raised flag and left, waves 1-3 did not; wave 0's scan word
    holds an all-ones LDS value.  The staged count is 2^32 - 1 and thread 0 never leaves the
    loop (its position wraps past 2^32 first)."""
    alive = per_wave_decisions([True, False, False, False])
    assert alive == [False, True, True, True]
    total = scan_total(alive, tile_counts(2048), stale=[MASK, 0, 0, 0])
    assert total == MASK
    assert staging_trips(0, total, bounded=False) == TRIP_CAP   # never ended by itself
    assert staging_trips(255, total, bounded=False) < TRIP_CAP   # the last lane gets out


def test_per_block_decision_is_uniform_and_the_loop_bounded():
    """Every interleaving of the four waves' reads gives one decision for the whole block, and
    with any stale LDS words the staging loop takes at most TILE / BLOCK trips."""
    stale_words = [0, 1, 7, MASK, MASK - 255, 1 << 31, 0xDEADBEEF]
    for seen in itertools.product([False, True], repeat=WAVES):
        alive = per_block_decision(list(seen))
        assert len(set(alive)) == 1
        if not alive[0]:
            continue
        for stale in itertools.product(stale_words, repeat=2):
            total = scan_total(alive, tile_counts(2048), stale=[stale[0], stale[1], 0, 0])
            assert total == 2048          # no stale word reaches the count
            for tid in (0, 17, 255):
                assert staging_trips(tid, total, bounded=True) <= TILE // BLOCK


@pytest.mark.parametrize("stale", [MASK, MASK - 3, 1 << 31, 0xDEADBEEF])
def test_bound_alone_stops_any_stale_count(stale):
    """Even a count polluted by stale words (the failure's state) ends the bounded loop within
    TILE / BLOCK trips: the bound is the second line of defence."""
    alive = [False, True, True, True]
    total = scan_total(alive, tile_counts(100), stale=[stale, 0, 0, 0])
    for tid in range(0, BLOCK, 37):
        assert staging_trips(tid, total, bounded=True) <= TILE // BLOCK
