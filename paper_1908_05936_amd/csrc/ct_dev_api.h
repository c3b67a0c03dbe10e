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
//
// Inserts and erases never share a kernel.  The live count stays exact throughout: an insert
// reserves capacity before it claims a slot (one compare-and-swap loop per wave), and gives it
// back when another thread stored the same key first; FULL means the table held its capacity.
// Key words are read with agent-scope atomic loads, which see other compute units' claims.
#pragma once

#include "ct_device.h"

namespace ct {

enum : int32_t { kDevRead = 0, kDevInsert = 1, kDevErase = 2 };

struct DevView {
  TableView t;
  int32_t mode;
  int32_t pad;
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
    bool end = false;
    for (int c = c0; c < kSlots; ++c) {
      const uint64_t k = dev_key(t, b * kSlots + (uint64_t)c);
      if (k == key) return b * kSlots + (uint64_t)c;
      if (k == kEmpty && !end) {
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

// One compare-and-swap loop per wave over the live count: lanes of the wave that arrive together
// reserve one unit each, in lane order, while capacity lasts.  Returns whether this lane got one.
__device__ __forceinline__ bool dev_reserve(const TableView& t) {
  const uint64_t m = __ballot(1);
  const int leader = __builtin_ctzll(m);
  const uint32_t rank = (uint32_t)__builtin_popcountll(m & ((1ull << wave_lane()) - 1ull));
  uint64_t granted = 0;
  if (wave_lane() == leader) {
    const uint64_t want = (uint64_t)__builtin_popcountll(m);
    uint64_t cur = __hip_atomic_load(&t.hdr->size, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    for (;;) {
      const uint64_t room = cur < t.cap ? t.cap - cur : 0;
      granted = want < room ? want : room;
      if (granted == 0) break;
      if (__hip_atomic_compare_exchange_strong(&t.hdr->size, &cur, cur + granted, __ATOMIC_RELAXED,
                                               __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT))
        break;
    }
  }
  granted = __shfl(granted, leader, 64);
  return rank < granted;
}

// Every lane that reaches this call takes one from the live count: one atomic per wave.
__device__ __forceinline__ void dev_uncount(const TableView& t) {
  const uint64_t m = __ballot(1);
  if (wave_lane() == __builtin_ctzll(m))
    __hip_atomic_fetch_sub(&t.hdr->size, (uint64_t)__builtin_popcountll(m), __ATOMIC_RELAXED,
                           __HIP_MEMORY_SCOPE_AGENT);
}

// kPresent, kInserted or kFull.
__device__ inline uint8_t dev_insert(const DevView& v, uint64_t key, uint64_t val) {
  const TableView& t = v.t;
  if (key >= kTomb) {  // out-of-band keys live in the header
    const int s = (int)(key - kTomb);
    if (__hip_atomic_load(&t.hdr->spec_live[s], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) return kPresent;
    if (!dev_reserve(t)) return kFull;
    uint32_t expected = 0;
    if (__hip_atomic_compare_exchange_strong(&t.hdr->spec_live[s], &expected, 1u, __ATOMIC_RELAXED,
                                             __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) {
      t.hdr->spec_val[s] = val;
      return kInserted;
    }
    dev_uncount(t);
    return kPresent;
  }
  const Seq sq = probe_seq(t, key);
  uint64_t empty;
  if (dev_probe(t, key, sq, sq.home, 0, &empty) != kNoPos) return kPresent;
  if (empty == kNoPos) return kFull;  // every bucket holds keys or tombstones
  if (!dev_reserve(t)) return kFull;
  for (;;) {
    uint64_t expected = kEmpty;
    if (cas64(&t.bk[empty >> 3].s[empty & 7].key, expected, key)) {
      t.bk[empty >> 3].s[empty & 7].val = val;
      return kInserted;
    }
    if (expected == key) {  // another thread stored this key in the same first empty slot
      dev_uncount(t);
      return kPresent;
    }
    // another key took the slot: go on from the next slot of the sequence
    uint64_t b = empty >> 3;
    int c = (int)(empty & 7) + 1;
    if (c == kSlots) {
      c = 0;
      b = next_bucket(t, b, sq.step);
    }
    if (dev_probe(t, key, sq, b, c, &empty) != kNoPos) {
      dev_uncount(t);
      return kPresent;
    }
    if (empty == kNoPos) {
      dev_uncount(t);
      return kFull;
    }
  }
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
    dev_uncount(t);
    return true;
  }
  const Seq sq = probe_seq(t, key);
  uint64_t empty;
  const uint64_t pos = dev_probe(t, key, sq, sq.home, 0, &empty);
  if (pos == kNoPos) return false;
  // an empty slot only where the bucket already holds one
  bool has_empty = false;
  for (int c = 0; c < kSlots; ++c) has_empty |= dev_key(t, (pos & ~7ull) + (uint64_t)c) == kEmpty;
  uint64_t expected = key;
  if (!cas64(&t.bk[pos >> 3].s[pos & 7].key, expected, has_empty ? kEmpty : kTomb)) return false;
  dev_uncount(t);
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
  const uint64_t pos = dev_probe(t, key, sq, sq.home, 0, &empty);
  if (pos == kNoPos) return false;
  if (val) *val = t.bk[pos >> 3].s[pos & 7].val;
  return true;
}

__device__ inline bool dev_contains(const DevView& v, uint64_t key) {
  return dev_find(v, key, nullptr);
}

}  // namespace ct
