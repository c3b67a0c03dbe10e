// Device-side per-thread operations on a table, for use inside user HIP kernels.
//
// Section 4.1 has the containers' functions called from inside kernels, one element per thread,
// and Section 4 states that the operations may run concurrently.  A kernel takes a DevView by
// value (ct_table_device_view fills one on the host) and calls dev_insert / dev_erase / dev_find
// / dev_contains from any lane, under any control flow.  The view's mode is the contract:
//
//   kDevRead    find and contains only.
//   kDevInsert  insert, find and contains, the same key from several threads included: a key is
//               stored once, and exactly one of its inserters sees INSERTED.  Inserts claim only
//               empty slots, never tombstones, and a slot never becomes empty again while the
//               kernel runs, so every inserter of a key walks the same probe sequence to the same
//               first empty slot.  A find of a key that another thread is inserting at that moment
//               may see the key before its value: the value is defined once the kernel has ended.
//   kDevErase   erase, find and contains: each present key is removed once (exactly one of its
//               erasers sees true).  An erase leaves an empty slot only where its bucket already
//               had one, so no probe sequence that passed the bucket is cut short.
//   kDevMixed   insert, erase, find and contains in one kernel, the same key from several threads
//               and by several operations included.  A slot only ever goes empty -> key ->
//               tombstone: inserts claim only empty slots and erases always leave tombstones, so
//               the argument of kDevInsert still holds and a key is live in at most one slot.
//               Each insert and erase takes effect at one compare-and-swap, so per key the
//               INSERTED results and the successful erases alternate.  Tombstones accumulate:
//               once no probe sequence of a key reaches an empty slot, its insert reports FULL.
//
// The thread that stores a new key takes one unit of capacity (one atomic add per wave) after its
// claim; with none left it takes the key out again (a tombstone) and reports FULL, so FULL means
// the table held its capacity.  Near capacity, a concurrent thread may see such a key for that
// moment.  The live count is exact once the kernel ends.  In kDevMixed an erase may remove a key
// between its claim and its unit and return a unit that was not taken yet; the inserter then
// makes up for it, and a third insert may have used that unit in between, so at capacity the
// count can pass the capacity by the number of such races.  Key words are read with agent-scope
// atomic loads, which see other compute units' claims.
#pragma once

#include "ct_device.h"

namespace ct {

enum : int32_t { kDevRead = 0, kDevInsert = 1, kDevErase = 2, kDevMixed = 3 };

// Live-count striping: a launch that cannot meet the capacity (the host or a set-up kernel has
// shown that the live count plus every insert it may make fits) counts its changes into
// kStripes words of the table's partial-count array, 128 bytes apart and picked by workgroup,
// instead of all into the header's one word, whose atomics would serialise; a fold kernel adds
// them to the live count after the launch.  Views handed to user kernels never stripe.
constexpr int kStripes = 64;
constexpr int kStripeStride = 16;                        // int64 words: 128 bytes
constexpr int kStripeFlag = kStripes * kStripeStride;    // word set by the set-up kernel

struct DevView {
  TableView t;
  int32_t mode;
  int32_t striped;  // 1: count into the stripes, no capacity checks
};

__device__ __forceinline__ uint64_t dev_key(const TableView& t, uint64_t pos) {
  return __hip_atomic_load(&t.bk[pos >> 3].s[pos & 7].key, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// This lane's probe of `key` from slot `from` of its sequence (from = home * 8 at the start):
// the key's slot, or kNoPos once a bucket with an empty slot ends the sequence (or every bucket
// was seen); *empty gets the first empty slot at or after `from` in sequence order, else kNoPos.
__device__ __forceinline__ uint64_t dev_probe(const TableView& t, uint64_t key, const Seq& sq,
                                              uint64_t b, int c0, uint64_t* empty) {
  *empty = kNoPos;
  for (uint64_t r = 0; r < t.nb; ++r) {
    // the bucket's eight key words in flight together, then the scan: the order of the reads
    // within a bucket does not matter, since a slot never returns to a state it has left
    uint64_t kk[kSlots];
#pragma unroll
    for (int c = 0; c < kSlots; ++c) kk[c] = dev_key(t, b * kSlots + (uint64_t)c);
    bool end = false;
#pragma unroll
    for (int c = 0; c < kSlots; ++c) {
      if (c < c0) continue;
      if (kk[c] == key) return b * kSlots + (uint64_t)c;
      if (kk[c] == kEmpty && !end) {
        end = true;
        if (*empty == kNoPos) *empty = b * kSlots + (uint64_t)c;
      }
    }
    if (end) return kNoPos;
    c0 = 0;
    b = next_bucket(t, b, sq.step);
  }
  return kNoPos;
}

// The same probe from the home bucket for a wave whose 64 lanes all call it together.  In step
// r (0..7) lane v reads slot v & 7 of the bucket that owner lane 8r + (v >> 3) probes next, so
// eight lanes read one 128-byte line together and a step of the wave makes 64 line requests
// instead of 512.  Ballots hand each owner the eight comparisons of its bucket.  Owners whose
// probe has ended read nothing useful (their lanes still read for the others), and the loop ends
// when every owner has ended, after at most nb buckets each.
__device__ __forceinline__ uint64_t dev_probe_wave(const TableView& t, uint64_t key, const Seq& sq,
                                                   uint64_t* empty) {
  const int lane = (int)wave_lane();
  const int me_round = lane >> 3;        // the step in which this lane's bucket is read
  const int me_shift = 8 * (lane & 7);   // and the ballot bits that hold its slots
  uint64_t b = sq.home;
  uint64_t res = kNoPos;
  uint64_t seen = 0;
  bool pending = true;
  *empty = kNoPos;
  for (;;) {
    const uint64_t pm = __ballot(pending);
    if (!pm) break;
    uint64_t kk[kSlots];
#pragma unroll
    for (int r = 0; r < kSlots; ++r) {
      const int o = 8 * r + (lane >> 3);
      const uint64_t bo = __shfl(b, o, 64);
      const bool po = (pm >> o) & 1ull;
      // an ended owner's lanes read slot v & 7 of bucket 0: a load every lane makes, in bounds
      kk[r] = dev_key(t, (po ? bo : 0ull) * kSlots + (uint64_t)(lane & 7));
    }
    uint32_t my_eq = 0, my_em = 0;
#pragma unroll
    for (int r = 0; r < kSlots; ++r) {
      const int o = 8 * r + (lane >> 3);
      const uint64_t ko = __shfl(key, o, 64);
      const uint64_t eq = __ballot(kk[r] == ko);
      const uint64_t em = __ballot(kk[r] == kEmpty);
      if (r == me_round) {
        my_eq = (uint32_t)(eq >> me_shift) & 0xFFu;
        my_em = (uint32_t)(em >> me_shift) & 0xFFu;
      }
    }
    if (pending) {
      if (my_eq) {
        res = b * kSlots + (uint64_t)__builtin_ctz(my_eq);
        if (my_em && (uint32_t)__builtin_ctz(my_em) < (uint32_t)__builtin_ctz(my_eq))
          *empty = b * kSlots + (uint64_t)__builtin_ctz(my_em);
        pending = false;
      } else if (my_em) {
        *empty = b * kSlots + (uint64_t)__builtin_ctz(my_em);
        pending = false;
      } else if (++seen >= t.nb) {
        pending = false;
      } else {
        b = next_bucket(t, b, sq.step);
      }
    }
  }
  return res;
}

// The probe from the home bucket: the whole wave together where it can, else lane by lane.
__device__ __forceinline__ uint64_t dev_probe_home(const TableView& t, uint64_t key, const Seq& sq,
                                                   uint64_t* empty) {
  if (__ballot(1) == ~0ull) return dev_probe_wave(t, key, sq, empty);
  return dev_probe(t, key, sq, sq.home, 0, empty);
}

// The wave's lanes that reach this call add `sign` each to the live count (or to their stripe).
__device__ __forceinline__ void dev_count_add(const DevView& v, int64_t sign) {
  const uint64_t m = __ballot(1);
  if (wave_lane() == __builtin_ctzll(m)) {
    const int64_t d = sign * (int64_t)__builtin_popcountll(m);
    if (v.striped)
      __hip_atomic_fetch_add(&v.t.bcnt[(blockIdx.x % kStripes) * kStripeStride], d,
                             __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    else
      __hip_atomic_fetch_add(&v.t.hdr->size, (uint64_t)d, __ATOMIC_RELAXED,
                             __HIP_MEMORY_SCOPE_AGENT);
  }
}

// Every lane that reaches this call adds one to the live count, whatever the capacity.
__device__ __forceinline__ void dev_count(const DevView& v) { dev_count_add(v, 1); }

// Every lane that reaches this call takes one from the live count: one atomic per wave.
__device__ __forceinline__ void dev_uncount(const DevView& v) { dev_count_add(v, -1); }

// Capacity for the lanes of the wave that arrive together: one fetch-and-add of their number on
// the live count (a compare-and-swap loop on that one address made the waves retry each other
// for seconds), then the leader gives back what lies beyond the capacity.  The adds order all
// reservations, and lane r of a wave holds position old + r: exactly the positions below the
// capacity are granted, however the adds and give-backs interleave.
__device__ __forceinline__ bool dev_reserve(const DevView& v) {
  if (v.striped) {  // the launch cannot meet the capacity
    dev_count(v);
    return true;
  }
  const TableView& t = v.t;
  const uint64_t m = __ballot(1);
  const int leader = __builtin_ctzll(m);
  const uint32_t rank = (uint32_t)__builtin_popcountll(m & ((1ull << wave_lane()) - 1ull));
  uint64_t old = 0;
  if (wave_lane() == leader) {
    const uint64_t want = (uint64_t)__builtin_popcountll(m);
    old = __hip_atomic_fetch_add(&t.hdr->size, want, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    const uint64_t room = old < t.cap ? t.cap - old : 0;
    if (want > room)
      __hip_atomic_fetch_sub(&t.hdr->size, want - room, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  }
  old = __shfl(old, leader, 64);
  return old + rank < t.cap;
}

// The insert of kDevMixed: claim, then capacity, as in kDevInsert.  An erase may remove the key
// between the two and return a unit the insert has not taken yet; the insert sees that when it
// takes its unit or tries to take the key back, and then leaves the count as the erase expects
// (one unit for a key that lived and was erased, so INSERTED).  The value of an out-of-band key
// that is inserted, erased and inserted again within one kernel is that of one of its inserts.
template <class Take>
__device__ inline uint8_t dev_insert_mixed(const DevView& v, uint64_t key, Take take) {
  const TableView& t = v.t;
  if (key >= kTomb) {
    const int s = (int)(key - kTomb);
    uint32_t* live = &t.hdr->spec_live[s];
    uint32_t expected = 0;
    if (!__hip_atomic_compare_exchange_strong(live, &expected, 1u, __ATOMIC_RELAXED,
                                              __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT))
      return kPresent;
    uint64_t val = 0;
    const bool unit = dev_reserve(v);
    if (!unit || !take(&val)) {
      expected = 1;
      if (__hip_atomic_compare_exchange_strong(live, &expected, 0u, __ATOMIC_RELAXED,
                                               __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) {
        if (unit) dev_uncount(v);
        return kFull;
      }
      if (!unit) dev_count(v);  // erased after the claim: that erase returned this unit
      return kInserted;
    }
    t.hdr->spec_val[s] = val;
    return kInserted;
  }
  const Seq sq = probe_seq(t, key);
  uint64_t empty;
  if (dev_probe_home(t, key, sq, &empty) != kNoPos) return kPresent;
  for (;;) {
    if (empty == kNoPos) return kFull;  // no empty slot left on the key's sequence
    uint64_t* kw = &t.bk[empty >> 3].s[empty & 7].key;
    uint64_t expected = kEmpty;
    if (cas64(kw, expected, key)) {
      uint64_t val = 0;
      const bool unit = dev_reserve(v);
      if (!unit || !take(&val)) {
        expected = key;
        if (cas64(kw, expected, kTomb)) {
          if (unit) dev_uncount(v);
          return kFull;
        }
        if (!unit) dev_count(v);  // erased after the claim: that erase returned this unit
        return kInserted;
      }
      t.bk[empty >> 3].s[empty & 7].val = val;
      return kInserted;
    }
    if (expected == key) return kPresent;
    uint64_t b = empty >> 3;
    int c = (int)(empty & 7) + 1;
    if (c == kSlots) {
      c = 0;
      b = next_bucket(t, b, sq.step);
    }
    if (dev_probe(t, key, sq, b, c, &empty) != kNoPos) return kPresent;
  }
}

// The insert, with the stored value produced after the claim: `take(&value)` runs once the thread
// holds the slot and a unit of capacity, and may refuse (then the claim is undone as for FULL).
// kPresent, kInserted or kFull.  The slot is claimed first, so only the one thread that stores
// the key asks for capacity; without it the key is taken out again (the slot becomes a
// tombstone) and the insert reports FULL.
template <class Take>
__device__ inline uint8_t dev_insert_with(const DevView& v, uint64_t key, Take take) {
  const TableView& t = v.t;
  if (v.mode == kDevMixed) return dev_insert_mixed(v, key, take);
  if (key >= kTomb) {  // out-of-band keys live in the header
    const int s = (int)(key - kTomb);
    uint32_t expected = 0;
    if (!__hip_atomic_compare_exchange_strong(&t.hdr->spec_live[s], &expected, 1u, __ATOMIC_RELAXED,
                                              __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT))
      return kPresent;
    uint64_t val = 0;
    if (!dev_reserve(v)) {
      __hip_atomic_store(&t.hdr->spec_live[s], 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      return kFull;
    }
    if (!take(&val)) {
      dev_uncount(v);
      __hip_atomic_store(&t.hdr->spec_live[s], 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      return kFull;
    }
    t.hdr->spec_val[s] = val;
    return kInserted;
  }
  const Seq sq = probe_seq(t, key);
  uint64_t empty;
  if (dev_probe_home(t, key, sq, &empty) != kNoPos) return kPresent;
  for (;;) {
    if (empty == kNoPos) return kFull;  // every bucket holds keys or tombstones
    uint64_t* kw = &t.bk[empty >> 3].s[empty & 7].key;
    uint64_t expected = kEmpty;
    if (cas64(kw, expected, key)) {
      uint64_t val = 0;
      if (!dev_reserve(v)) {
        __hip_atomic_store(kw, kTomb, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        return kFull;
      }
      if (!take(&val)) {
        dev_uncount(v);
        __hip_atomic_store(kw, kTomb, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        return kFull;
      }
      t.bk[empty >> 3].s[empty & 7].val = val;
      return kInserted;
    }
    if (expected == key) return kPresent;  // another thread stored it in the same first empty slot
    // another key took the slot: go on from the next slot of the sequence
    uint64_t b = empty >> 3;
    int c = (int)(empty & 7) + 1;
    if (c == kSlots) {
      c = 0;
      b = next_bucket(t, b, sq.step);
    }
    if (dev_probe(t, key, sq, b, c, &empty) != kNoPos) return kPresent;
  }
}

__device__ inline uint8_t dev_insert(const DevView& v, uint64_t key, uint64_t val) {
  return dev_insert_with(v, key, [val](uint64_t* out) {
    *out = val;
    return true;
  });
}

// Whether the key was present (and is now removed).
__device__ inline bool dev_erase(const DevView& v, uint64_t key) {
  const TableView& t = v.t;
  if (key >= kTomb) {
    const int s = (int)(key - kTomb);
    uint32_t expected = 1;
    if (!__hip_atomic_compare_exchange_strong(&t.hdr->spec_live[s], &expected, 0u, __ATOMIC_RELAXED,
                                              __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT))
      return false;
    dev_uncount(v);
    return true;
  }
  const Seq sq = probe_seq(t, key);
  uint64_t empty;
  const uint64_t pos = dev_probe_home(t, key, sq, &empty);
  if (pos == kNoPos) return false;
  // an empty slot only where the bucket already holds one, and never while inserts run
  bool has_empty = false;
  if (v.mode != kDevMixed)
    for (int c = 0; c < kSlots; ++c) has_empty |= dev_key(t, (pos & ~7ull) + (uint64_t)c) == kEmpty;
  uint64_t expected = key;
  if (!cas64(&t.bk[pos >> 3].s[pos & 7].key, expected, has_empty ? kEmpty : kTomb)) return false;
  dev_uncount(v);
  return true;
}

// Whether the key is present; *val (nullable) gets its value.
__device__ inline bool dev_find(const DevView& v, uint64_t key, uint64_t* val) {
  const TableView& t = v.t;
  if (key >= kTomb) {
    const int s = (int)(key - kTomb);
    if (!__hip_atomic_load(&t.hdr->spec_live[s], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) return false;
    if (val) *val = t.hdr->spec_val[s];
    return true;
  }
  const Seq sq = probe_seq(t, key);
  uint64_t empty;
  const uint64_t pos = dev_probe_home(t, key, sq, &empty);
  if (pos == kNoPos) return false;
  if (val) *val = t.bk[pos >> 3].s[pos & 7].val;
  return true;
}

__device__ inline bool dev_contains(const DevView& v, uint64_t key) {
  return dev_find(v, key, nullptr);
}

// ---------------------------------------------------------------------------------------------
// Device-side vector / deque back operations on an index pool (Sections 4.2-4.3: push_back and
// pop_back called from threads).  A kernel either pushes or pops; each is one atomic per wave on
// the pool's size.  The adds (or subtractions) order the lanes: lane r of a wave takes position
// old + r (old - 1 - r for pops), and exactly the positions inside the pool are granted, however
// the give-backs of the other lanes interleave.  A pushed value is readable once the kernel ends.
// ---------------------------------------------------------------------------------------------
struct DevPool {
  PoolHeader* hdr;
  int32_t* stack;
};

// Whether the value was stored (false: the pool was at capacity, CT_ERR_POOL set).
__device__ inline bool dev_push_back(const DevPool& p, int32_t value) {
  const uint64_t m = __ballot(1);
  const int leader = __builtin_ctzll(m);
  const int64_t rank = (int64_t)__builtin_popcountll(m & ((1ull << wave_lane()) - 1ull));
  const int64_t cap = p.hdr->cap;
  int64_t old = 0;
  if (wave_lane() == leader) {
    const int64_t want = (int64_t)__builtin_popcountll(m);
    old = __hip_atomic_fetch_add(&p.hdr->top, want, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    const int64_t room = old < cap ? cap - (old < 0 ? 0 : old) : 0;
    if (want > room) {
      __hip_atomic_fetch_sub(&p.hdr->top, want - room, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      __hip_atomic_fetch_or(&p.hdr->err, kErrPool, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
  }
  old = __shfl(old, leader, 64);
  const int64_t pos = old + rank;
  if (old < 0 || pos >= cap) return false;
  p.stack[ring_pos(p.hdr->head, cap, pos)] = value;
  return true;
}

// Whether a value was removed into *value (false: the pool was empty, CT_ERR_POOL set).
__device__ inline bool dev_pop_back(const DevPool& p, int32_t* value) {
  const uint64_t m = __ballot(1);
  const int leader = __builtin_ctzll(m);
  const int64_t rank = (int64_t)__builtin_popcountll(m & ((1ull << wave_lane()) - 1ull));
  int64_t old = 0;
  if (wave_lane() == leader) {
    const int64_t want = (int64_t)__builtin_popcountll(m);
    old = __hip_atomic_fetch_sub(&p.hdr->top, want, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    const int64_t avail = old > 0 ? old : 0;
    if (want > avail) {
      __hip_atomic_fetch_add(&p.hdr->top, want - avail, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      __hip_atomic_fetch_or(&p.hdr->err, kErrPool, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
  }
  old = __shfl(old, leader, 64);
  if (rank >= old) return false;
  *value = p.stack[ring_pos(p.hdr->head, p.hdr->cap, old - 1 - rank)];
  return true;
}

// Insert whose new key takes pop_back() of the pool as its value (the block map of Section 4.1
// fed by the free list); a present key reports its value.  kPresent / kInserted / kFull (no
// capacity or an empty pool: the claim is undone).  *out gets the key's value, -1 on FULL.
__device__ inline uint8_t dev_insert_alloc(const DevView& v, const DevPool& p, uint64_t key,
                                           int32_t* out) {
  int32_t got = -1;
  const uint8_t st = dev_insert_with(v, key, [&](uint64_t* val) {
    if (!dev_pop_back(p, &got)) return false;
    *val = (uint64_t)(uint32_t)got;
    return true;
  });
  if (st == kPresent) {
    uint64_t val = 0;
    *out = dev_find(v, key, &val) ? (int32_t)(uint32_t)val : -1;
  } else {
    *out = st == kInserted ? got : -1;
  }
  return st;
}

}  // namespace ct
