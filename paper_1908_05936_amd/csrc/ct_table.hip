// ct_table.hip -- gfx950 kernels and the C ABI of the batch hash containers and index pool.
//
// Operation pipelines (every kernel on the caller's stream, in this order):
//   find           : k_find                                    one launch, read-only, lock-free
//   insert (chunk) : k_prologue -> k_dedup -> k_insert [-> k_tile_count -> k_tile_scan -> k_final]
//                    -> k_fix
//   insert_alloc   : k_prologue -> k_dedup -> k_insert -> k_tile_count -> k_tile_scan -> k_final
//                    -> k_fix
//   erase          : k_prologue -> k_dedup -> k_erase
//   erase_release  : k_prologue -> k_dedup -> k_erase -> k_tile_count -> k_tile_scan -> k_final
//
// Index-order semantics.  k_dedup records, per distinct key of the chunk, the lowest chunk index
// holding it (an atomic min in a cache-resident scratch table).  Only that element (the "actor")
// touches the table; later copies are resolved afterwards from its outcome (k_fix), which gives
// exactly the results of a sequential replay.  Distinct actors never race on one key, so a claim
// CAS can only fail because another key took the slot.  When a chunk might reach capacity or
// empty the pool, or when values come from a pool, the new actors are ranked by an exclusive scan
// in index order (k_tile_count / k_tile_scan) and k_final hands out capacity and pool entries by
// rank, so the k-th new key of the chunk is the k-th to be stored, as in the sequential replay.
#include <hip/hip_cooperative_groups.h>
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdint>
#include <cstdlib>
#include <cstring>
#include <mutex>
#include <new>
#include <vector>

#include "ct.h"
#include "ct_device.h"
#include "ct_dev_api.h"

using namespace ct;

namespace {

// ---------------------------------------------------------------------------------------------
// value I/O by value kind (0 none, 1 u32, 2 u64); table slots always hold 64-bit values
// ---------------------------------------------------------------------------------------------
template <int VK>
__device__ __forceinline__ uint64_t load_val(const void* vals, int64_t i) {
  if constexpr (VK == 1) return (uint64_t)static_cast<const uint32_t*>(vals)[i];
  else if constexpr (VK == 2) return static_cast<const uint64_t*>(vals)[i];
  else return 0;
}
template <int VK>
__device__ __forceinline__ void store_val(void* out, int64_t i, uint64_t v) {
  if constexpr (VK == 1) static_cast<uint32_t*>(out)[i] = (uint32_t)v;
  else if constexpr (VK == 2) static_cast<uint64_t*>(out)[i] = v;
}
template <int VK>
__device__ __forceinline__ uint64_t sentinel() {
  return VK == 1 ? 0xFFFFFFFFull : ~0ull;
}

// ---------------------------------------------------------------------------------------------
// group-cooperative probes of the home table (8 lanes, converged within the group)
// ---------------------------------------------------------------------------------------------
struct Probe {
  bool found;
  bool had_empty;    // the bucket where the key was found holds a kEmpty slot
  uint64_t val;
  uint64_t pos;      // slot index b*8+c of the key when found
  uint64_t free_b;   // first bucket with a free slot on the probe path (when !found)
  bool has_free;
};

__device__ __forceinline__ Probe probe(const TableView& t, uint64_t key, int sub, bool want_free) {
  Probe r;
  r.found = false;
  r.had_empty = false;
  r.val = 0;
  r.pos = kNoPos;
  r.free_b = 0;
  r.has_free = false;
  const Seq q = probe_seq(t, key);
  uint64_t b = q.home;
  for (uint64_t step = 0; step < t.nb; ++step) {
    const Slot s = t.bk[b].s[sub];
    const uint32_t m = group_bits(__ballot(s.key == key));
    const uint32_t e = group_bits(__ballot(s.key == kEmpty));
    if (m) {
      const int c = lowest(m);
      r.found = true;
      r.had_empty = e != 0;
      r.val = __shfl(s.val, group_base() + c, 64);
      r.pos = b * kSlots + (uint64_t)c;
      return r;
    }
    if (want_free && !r.has_free) {
      const uint32_t f = e | group_bits(__ballot(s.key == kTomb));
      if (f) {
        r.has_free = true;
        r.free_b = b;
      }
    }
    if (e) return r;
    b = next_bucket(t, b, q.step);
  }
  return r;
}

// Claim a free slot for an absent `key`, scanning forward from bucket `b`.  Returns the slot
// index, or kNoPos when every bucket was tried (only possible when the table is physically full).
// A stale view can only show a slot as free when it is not: the CAS then fails and reports the
// truth, so the scan always makes progress.
__device__ __forceinline__ uint64_t claim(const TableView& t, uint64_t key, uint64_t b,
                                          uint64_t stride, int sub) {
  for (uint64_t step = 0; step < t.nb; ++step) {
    const uint64_t cur = t.bk[b].s[sub].key;
    uint32_t f = group_bits(__ballot(cur == kEmpty || cur == kTomb));
    while (f) {
      const int c = lowest(f);
      int won = 0;
      if (sub == c) {
        uint64_t expected = cur;
        won = cas64(&t.bk[b].s[c].key, expected, key) ? 1 : 0;
      }
      if (group_bits(__ballot(won))) return b * kSlots + (uint64_t)c;
      f &= f - 1;
    }
    b = next_bucket(t, b, stride);
  }
  return kNoPos;
}

// Per lane: lowest chunk index of a key that k_dedup marked as repeated.  The entry is always
// there; the scan is bounded anyway, and a miss makes the element act for itself and raises
// kErrInternal.
__device__ __forceinline__ uint32_t dedup_lookup(const TableView& t, const uint64_t* keys,
                                                 uint64_t key, uint32_t dmask, uint32_t self) {
  const uint64_t mix = dedup_mix(key);
  const uint64_t tag = mix & 0xFFFFFFFF00000000ull;
  uint32_t h = (uint32_t)mix & dmask;
  for (uint32_t step = 0; step <= dmask; ++step) {
    const uint64_t e = t.dd[h];
    if (e == kEmpty) break;
    if ((e & 0xFFFFFFFF00000000ull) == tag && keys[(uint32_t)e] == key) return (uint32_t)e;
    h = (h + 1) & dmask;
  }
  aor32(&t.hdr->err, kErrInternal);
  return self;
}

// ---------------------------------------------------------------------------------------------
// kernels
// ---------------------------------------------------------------------------------------------
// Empty every slot in [lo, hi) (thread-strided by `step`); `header` also resets the counters.
// Slots are written as 16-byte words, U per thread and round (the stores of a round issue
// back to back; a round that would pass `hi` takes a bounds test per word).
__device__ __forceinline__ void reset_range(const TableView& t, int64_t lo, int64_t hi,
                                            int64_t step, bool header, int zero_err) {
  constexpr int U = 4;
  const uint4 empty = make_uint4(0xFFFFFFFFu, 0xFFFFFFFFu, 0u, 0u);
  uint4* slots = reinterpret_cast<uint4*>(t.bk);
  int64_t j = lo * U + threadIdx.x;
  const int64_t span = step * U;
  const int64_t width = blockDim.x;
  for (; j + (U - 1) * width < hi; j += span) {
#pragma unroll
    for (int u = 0; u < U; ++u) slots[j + u * width] = empty;
  }
  for (int u = 0; u < U; ++u)
    if (j + u * width < hi) slots[j + u * width] = empty;
  if (header && threadIdx.x == 0) {
    Header* h = t.hdr;
    h->size = 0;
    h->size0 = 0;
    h->spec_val[0] = h->spec_val[1] = 0;
    h->spec_live[0] = h->spec_live[1] = 0;
    h->spec_first[0] = h->spec_first[1] = kNone;
    if (zero_err) {
      h->err = 0;
      h->inject = 0;
    }
    // an empty table starts a fresh history: its next insert and erase chunks speculate
    h->fbd[0] = h->fbd[1] = 0;
    if (t.fb) {
      __hip_atomic_store(t.fb, (uint64_t)0, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
      __hip_atomic_store(t.fb + 1, (uint64_t)0, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
    }
    h->fast = 0;
    h->spec = 0;
    h->ndup = 0;
    h->nnew = 0;
    h->dump_count = 0;
    h->live_count = 0;
    h->violations = 0;
    h->dagg = 0;
    h->dskew = 0;
    h->dskew_age = 0;
  }
}

__global__ __launch_bounds__(kBlock) void k_table_reset(TableView t, int zero_header) {
  reset_range(t, (int64_t)blockIdx.x * blockDim.x, (int64_t)t.nb * kSlots,
              (int64_t)gridDim.x * blockDim.x, blockIdx.x == 0, zero_header);
}

// Per chunk: clear the dedup scratch, snapshot the counters, decide whether the chunk can reach
// capacity (or empty the pool).
// Units [lo, hi) of a chunk's scratch clear: the first dslots/2 units are 16-byte dedup-entry
// pairs, the rest 16-byte groups of repeated-key marks.  `header`: snapshot the counters and
// decide whether the chunk can reach capacity (or empty the pool).
__device__ __forceinline__ int64_t prologue_units(uint32_t dslots, int64_t q) {
  return (int64_t)dslots / 2 + (q + 15) / 16;
}

// Per-chunk counters: snapshot size (and pool top), reset the chunk's lists, decide whether the
// chunk can reach capacity (or empty the pool), and record how repeated keys are resolved.
__device__ __forceinline__ void chunk_header(const TableView& t, PoolHeader* pool, int64_t q,
                                             uint32_t dmode) {
  Header* h = t.hdr;
  h->size0 = h->size;
  h->spec_first[0] = h->spec_first[1] = kNone;
  h->ndup = 0;
  h->nnew = 0;
  bool fast = h->size + (uint64_t)q <= t.cap;
  if (pool) {
    pool->top0 = pool->top;
    fast = fast && pool->top >= q;
  }
  h->fast = fast ? 1u : 0u;
  h->spec = 0u;
  h->dmode = dmode;
  h->dovf = 0;
  // binned chunks of a table whose keys recently overflowed the bins fold each tile's repeated
  // keys before scattering; every 16th such chunk tries without, and ends the hint if it fits
  uint32_t agg = 0;
  if (dmode && h->dskew) agg = (++h->dskew_age & 15u) != 0u ? 1u : 0u;
  h->dagg = agg;
}

__device__ __forceinline__ void prologue_range(const TableView& t, PoolHeader* pool,
                                               uint32_t dslots, int64_t q, int64_t lo, int64_t hi,
                                               int64_t step, bool header) {
  const uint4 empty = make_uint4(0xFFFFFFFFu, 0xFFFFFFFFu, 0xFFFFFFFFu, 0xFFFFFFFFu);
  const int64_t nd = (int64_t)dslots / 2;
  for (int64_t j = lo + threadIdx.x; j < hi; j += step) {
    if (j < nd) reinterpret_cast<uint4*>(t.dd)[j] = empty;
    else reinterpret_cast<uint4*>(t.dmark)[j - nd] = make_uint4(0, 0, 0, 0);
  }
  if (header && threadIdx.x == 0) chunk_header(t, pool, q, 0u);
}

// zero_tiles: also zero the chunk's tile sums, for an insert kernel that counts its tiles itself.
__global__ __launch_bounds__(kBlock) void k_prologue(TableView t, PoolHeader* pool,
                                                     uint32_t dslots, int64_t q, int zero_tiles) {
  prologue_range(t, pool, dslots, q, (int64_t)blockIdx.x * blockDim.x, prologue_units(dslots, q),
                 (int64_t)gridDim.x * blockDim.x, blockIdx.x == 0);
  if (zero_tiles)
    for (int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; j < (q + kTile - 1) / kTile;
         j += (int64_t)gridDim.x * blockDim.x)
      t.tsum[j] = 0;
}

// Lowest index per distinct key of the chunk.  The block takes 256 consecutive elements at a time
// and first resolves them among themselves in LDS: every element of a key repeated inside the
// window is marked, and only the window's lowest copy of each key (its representative) goes on
// to the chunk-wide table dd.  There the first representative to arrive claims an empty entry
// with one CAS; a later one marks itself and the holder, and lowers the entry's index with an
// atomic min when its own index is lower (the index only decreases, so a representative above
// the index it reads cannot lower it).  Every element of a key that occurs more than once ends
// up marked, unique keys stay unmarked, and the entry ends at the key's lowest index.  All
// indices held by one entry belong to one key, so the fingerprint plus one look at that
// element's key identifies the entry exactly.  A key repeated many times therefore costs one
// global operation per window, not per copy.  Needs blockDim.x == kBlock.
// `skip` (nullable): elements with a nonzero byte there take no part (a masked insert).
__device__ __forceinline__ void dedup_range(const TableView& t, const uint64_t* __restrict__ keys,
                                            const uint8_t* __restrict__ skip, uint32_t dmask,
                                            int64_t lo, int64_t hi, int64_t step) {
  constexpr uint32_t kW = 2 * kBlock;  // LDS slots of a window's table
  __shared__ unsigned long long wk[kW];
  __shared__ uint32_t wmin[kW], wcnt[kW];
  for (int64_t b0 = lo; b0 < hi; b0 += step) {  // uniform trip count: barriers below
    for (uint32_t j = threadIdx.x; j < kW; j += kBlock) {
      wk[j] = kEmpty;
      wmin[j] = kNone;
      wcnt[j] = 0;
    }
    __syncthreads();
    const int64_t i = b0 + threadIdx.x;
    const bool valid = i < hi && !(skip && skip[i]);
    const uint64_t key = valid ? keys[i] : kEmpty;
    const bool normal = valid && key < kTomb;
    if (valid && !normal) amin32(&t.hdr->spec_first[key - kTomb], (uint32_t)i);
    const uint64_t mix = dedup_mix(key);
    uint32_t s = (uint32_t)(mix >> 32) & (kW - 1);
    if (normal) {
      for (;;) {  // at most kBlock keys in kW slots: a free or matching slot exists
        const unsigned long long old = atomicCAS(&wk[s], (unsigned long long)kEmpty,
                                                 (unsigned long long)key);
        if (old == kEmpty || old == key) break;
        s = (s + 1) & (kW - 1);
      }
      atomicMin(&wmin[s], (uint32_t)i);
      atomicAdd(&wcnt[s], 1u);
    }
    __syncthreads();
    if (normal) {
      if (wcnt[s] > 1) t.dmark[i] = 1;
      if (wmin[s] == (uint32_t)i) {  // the window's representative of this key
        const uint64_t tag = mix & 0xFFFFFFFF00000000ull;
        const uint64_t mine = tag | (uint64_t)i;
        uint32_t h = (uint32_t)mix & dmask;
        for (uint32_t probe = 0; probe <= dmask; ++probe) {
          uint64_t e = t.dd[h];
          if (e == kEmpty) {
            uint64_t expected = kEmpty;
            if (cas64(&t.dd[h], expected, mine)) break;
            e = expected;
          }
          if ((e & 0xFFFFFFFF00000000ull) == tag && keys[(uint32_t)e] == key) {
            const uint32_t held = (uint32_t)e;
            uint32_t prev = held;
            if ((uint32_t)i < held) prev = (uint32_t)amin64(&t.dd[h], mine);
            t.dmark[i] = 1;
            if (!t.dmark[prev]) t.dmark[prev] = 1;
            break;
          }
          h = (h + 1) & dmask;
        }
      }
    }
    __syncthreads();  // the window's LDS table is reused by the next window
  }
}

__global__ __launch_bounds__(kBlock) void k_dedup(TableView t, const uint64_t* __restrict__ keys,
                                                  const uint8_t* __restrict__ skip, int64_t q,
                                                  uint32_t dmask) {
  dedup_range(t, keys, skip, dmask, (int64_t)blockIdx.x * kBlock, q, (int64_t)gridDim.x * kBlock);
}

// ---------------------------------------------------------------------------------------------
// Binned dedup: the same marks as dedup_range (every element of a key that occurs more than once
// in the chunk), plus each marked element's first occurrence in dfirst, without a device-scope
// atomic per element.  Keys move into 64 coarse bins and then into P fine bins by the high bits
// of dedup_mix, so all copies of a key share a fine bin; each fine bin (about 1024 elements)
// finds its repeated keys in an LDS hash table.  The only global atomics reserve room in a bin,
// one per block and non-empty bin.  A bin that would overflow its capacity sets dovf; the chunk
// then clears dd and runs dedup_range instead, so results never depend on the key distribution.
// ---------------------------------------------------------------------------------------------
// Exclusive block-wide scan of one value per thread (kBlock threads); returns the prefix and
// writes the block total to *total.
__device__ __forceinline__ uint32_t block_exclusive_scan(uint32_t v, uint32_t* total) {
  __shared__ uint32_t wsum[kBlock / 64];
  const int lane = wave_lane();
  uint32_t x = v;
  for (int off = 1; off < 64; off <<= 1) {
    const uint32_t y = __shfl_up(x, off, 64);
    if (lane >= off) x += y;
  }
  if (lane == 63) wsum[threadIdx.x >> 6] = x;
  __syncthreads();
  uint32_t before = 0, all = 0;
  for (int w = 0; w < kBlock / 64; ++w) {
    if (w < (int)(threadIdx.x >> 6)) before += wsum[w];
    all += wsum[w];
  }
  *total = all;
  __syncthreads();
  return before + x - v;
}

// The chunk's overflow flag and one fill count, read once for the whole block.  Other blocks of
// the same launch may raise the flag while this block starts, so a per-wave read could let some
// waves of a block leave and others stay; the staying waves would then meet the block's barriers
// and scans without the leavers' contributions (the scan words those waves never wrote hold stale
// LDS contents).  One reader and a barrier make the decision uniform across the block.
__device__ __forceinline__ bool block_overflowed(const TableView& t, const uint32_t* count,
                                                 uint32_t* fill) {
  __shared__ uint32_t flag_and_fill[2];
  if (threadIdx.x == 0) {
    const uint32_t o = t.hdr->dovf;
    const uint32_t f = *count;
    flag_and_fill[0] = o;
    flag_and_fill[1] = f;
  }
  __syncthreads();
  *fill = flag_and_fill[1];
  return flag_and_fill[0] != 0;
}

__device__ __forceinline__ uint32_t fine_bin(const TableView& t, uint64_t mix) {
  return (uint32_t)(mix >> (64 - t.lp));
}

// Units [lo, hi) of a binned chunk's prologue: the marks (16 per unit), then the bin counts
// (4 per unit); `header` also takes the chunk's counter snapshot.
__device__ __forceinline__ int64_t bin_prologue_units(const TableView& t, int64_t q) {
  return (q + 15) / 16 + ((int64_t)kCoarseCtrWords + ((int64_t)1 << t.lp)) / 4;
}

__global__ __launch_bounds__(kBlock) void k_bin_prologue(TableView t, PoolHeader* pool, int64_t q) {
  const int64_t nm = (q + 15) / 16;
  const int64_t hi = bin_prologue_units(t, q);
  const uint4 zero = make_uint4(0, 0, 0, 0);
  for (int64_t j = (int64_t)blockIdx.x * kBlock + threadIdx.x; j < hi; j += (int64_t)gridDim.x * kBlock) {
    if (j < nm) reinterpret_cast<uint4*>(t.dmark)[j] = zero;
    else reinterpret_cast<uint4*>(t.bcur)[j - nm] = zero;
  }
  if (blockIdx.x == 0 && threadIdx.x == 0) chunk_header(t, pool, q, 1u);
}

// Both scatters: the block's elements, ranked within their bin (code = rank << 8 | bin, or ~0 for
// none), are staged in LDS in bin order and each bin's run is written by consecutive threads, so
// the stores of a wave go to consecutive positions of one bin.  cnt[b] holds the block's count
// for bin b; this reserves the runs (bin b's fill count at bcur[cur0 + b * cur_stride]), flags an
// overflow of `cap`, and writes bin b of the block to out[(gbin0 + b * gstride) * cap + position].
struct BinStage {
  uint64_t k[kBinTile];
  uint32_t i[kBinTile];
  uint8_t b[kBinTile];
  uint32_t cnt[kMaxFinePerCoarse];
  uint32_t base[kMaxFinePerCoarse];
  uint32_t loc[kMaxFinePerCoarse];
};

template <int PER>
__device__ __forceinline__ void bin_write(const TableView& t, BinStage& S, uint32_t nbins,
                                          const uint64_t (&k)[PER], const uint32_t (&ix)[PER],
                                          const uint32_t (&code)[PER], uint32_t cur0,
                                          uint32_t cur_stride, uint32_t gbin0, uint32_t gstride,
                                          uint32_t cap, uint64_t* __restrict__ outk,
                                          uint32_t* __restrict__ outi) {
  const uint32_t c = threadIdx.x < nbins ? S.cnt[threadIdx.x] : 0u;
  uint32_t total;
  const uint32_t pre = block_exclusive_scan(c, &total);
  if (threadIdx.x < nbins) {
    uint32_t o = 0;
    if (c) {
      o = aadd32(&t.bcur[cur0 + threadIdx.x * cur_stride], c);
      if (o + c > cap) t.hdr->dovf = 1u;
    }
    S.base[threadIdx.x] = o;
    S.loc[threadIdx.x] = pre;
  }
  __syncthreads();
#pragma unroll
  for (int e = 0; e < PER; ++e) {
    if (code[e] == ~0u) continue;
    const uint32_t b = code[e] & 0xFFu;
    const uint32_t p = S.loc[b] + (code[e] >> 8);
    S.k[p] = k[e];
    S.i[p] = ix[e];
    S.b[p] = (uint8_t)b;
  }
  __syncthreads();
  // a block stages at most kBinTile elements; the bound also keeps p from wrapping
  const uint32_t staged = min(total, (uint32_t)kBinTile);
  for (uint32_t p = threadIdx.x; p < staged; p += kBlock) {
    const uint32_t b = S.b[p];
    const uint32_t pos = S.base[b] + (p - S.loc[b]);
    if (pos < cap) {
      const int64_t at = (int64_t)(gbin0 + b * gstride) * cap + pos;
      outk[at] = S.k[p];
      outi[at] = S.i[p];
    }
  }
}

// Coarse scatter: block b takes elements [b * kBinTile, (b + 1) * kBinTile) into segment
// b mod kBinSub of the 64 coarse bins.  The out-of-band keys take their lowest index directly, as
// in dedup_range.
// When the chunk folds (dagg: its table's recent chunks overflowed the bins, i.e. skewed keys),
// the tile first finds its own repeated keys in an LDS table.  Only each key's first copy in the
// tile goes to the bins; when the tile holds other copies it is marked with dfirst = itself (the
// fine bins replace that if an earlier tile holds the key), and every other copy is marked with
// dfirst = kIndirect | that first copy.  A key repeated thousands of times then reaches its fine
// bin once per tile instead of once per copy.  A copy that finds no slot within kFoldProbe probes
// simply goes to the bins unfolded: the fine bins resolve whatever reaches them exactly.
constexpr int kFoldProbe = 32;

__global__ __launch_bounds__(kBlock) void k_bin_scatter1(TableView t, const uint64_t* __restrict__ keys,
                                                         int64_t q) {
  constexpr int kPer = kBinTile / kBlock;
  constexpr uint32_t kFolded = ~0u - 1u;  // hs entry of a copy that stays out of the bins
  __shared__ BinStage S;
  const int64_t t0 = (int64_t)blockIdx.x * kBinTile;
  uint64_t k[kPer];
  uint32_t ix[kPer], code[kPer], hs[kPer];
  // all loads first, from clamped (in-bounds) positions: a load under a branch would make the
  // compiler wait for it before the next one is issued.  The chunk's mode comes with them.
#pragma unroll
  for (int e = 0; e < kPer; ++e) k[e] = keys[min(t0 + e * kBlock + (int64_t)threadIdx.x, q - 1)];
  const uint32_t agg = t.hdr->dagg;
  if (threadIdx.x < kBinCoarse) S.cnt[threadIdx.x] = 0;
#pragma unroll
  for (int e = 0; e < kPer; ++e) hs[e] = ~0u;
  if (agg) {
    // H[s] (in S.i): tile position of a copy of slot s's key, the lowest once all have arrived;
    // D[s] (in S.b): the key occurs more than once in the tile.  S.k holds the tile's keys by
    // position.  All three are free until the bins are written.
    uint32_t* H = S.i;
    uint8_t* D = S.b;
    for (uint32_t j = threadIdx.x; j < (uint32_t)kBinTile; j += kBlock) {
      H[j] = ~0u;
      D[j] = 0;
    }
#pragma unroll
    for (int e = 0; e < kPer; ++e) S.k[e * kBlock + threadIdx.x] = k[e];
    __syncthreads();
#pragma unroll
    for (int e = 0; e < kPer; ++e) {
      const uint32_t local = e * kBlock + threadIdx.x;
      if (t0 + local < q && k[e] < kTomb) {
        uint32_t s = (uint32_t)dedup_mix(k[e]) & (kBinTile - 1u);
        for (int probe = 0; probe < kFoldProbe; ++probe) {
          const uint32_t prev = atomicCAS(&H[s], ~0u, local);
          if (prev == ~0u) {
            hs[e] = s;
            break;
          }
          if (S.k[prev] == k[e]) {
            atomicMin(&H[s], local);
            D[s] = 1;
            hs[e] = s;
            break;
          }
          s = (s + 1u) & (kBinTile - 1u);
        }
      }
    }
    __syncthreads();
#pragma unroll
    for (int e = 0; e < kPer; ++e) {
      if (hs[e] == ~0u || !D[hs[e]]) continue;
      const uint32_t local = e * kBlock + threadIdx.x;
      const uint32_t i = (uint32_t)(t0 + local);
      const uint32_t rep = H[hs[e]];
      t.dmark[i] = 1;
      if (rep == local) {
        t.dfirst[i] = i;
      } else {
        t.dfirst[i] = kIndirect | (uint32_t)(t0 + rep);
        hs[e] = kFolded;
      }
    }
  }
  __syncthreads();
#pragma unroll
  for (int e = 0; e < kPer; ++e) {
    const int64_t i = t0 + e * kBlock + threadIdx.x;
    code[e] = ~0u;
    ix[e] = (uint32_t)i;
    if (i < q) {
      if (k[e] >= kTomb) {
        amin32(&t.hdr->spec_first[k[e] - kTomb], (uint32_t)i);
      } else if (hs[e] != kFolded) {
        const uint32_t b = (uint32_t)(dedup_mix(k[e]) >> (64 - t.lp1));
        code[e] = (atomicAdd(&S.cnt[b], 1u) << 8) | b;
      }
    }
  }
  __syncthreads();
  const uint32_t seg = blockIdx.x % kBinSub;
  bin_write<kPer>(t, S, kBinCoarse, k, ix, code, seg * kCtrStride, kBinSub * kCtrStride, seg,
                  kBinSub, t.c1, t.r1k, t.r1i);
}

// Fine scatter: the blocks of segment g of coarse bin c = g / kBinSub take its tiles in turn
// (tile r, r + blocks_per_seg, ...) and move each into the 2^(lp - lp1) fine bins of c, the same
// way.
__global__ __launch_bounds__(kBlock) void k_bin_scatter2(TableView t, int blocks_per_seg) {
  constexpr int kPer = kBinTile / kBlock;
  __shared__ BinStage S;
  const int g = (int)blockIdx.x / blocks_per_seg;
  const int c = g / kBinSub;
  uint32_t fill;
  if (block_overflowed(t, &t.bcur[g * kCtrStride], &fill)) return;
  const uint32_t n1 = min(fill, t.c1);
  const int lp2 = t.lp - t.lp1;
  const uint32_t p2 = 1u << lp2;
  const int64_t src = (int64_t)g * t.c1;
  for (uint32_t j0 = (uint32_t)((int)blockIdx.x % blocks_per_seg) * kBinTile; j0 < n1;
       j0 += (uint32_t)blocks_per_seg * kBinTile) {
    uint64_t k[kPer];
    uint32_t ix[kPer], code[kPer];
#pragma unroll
    for (int e = 0; e < kPer; ++e) {   // loads first, clamped (n1 > j0 >= 0)
      const uint32_t j = min(j0 + e * kBlock + threadIdx.x, n1 - 1u);
      k[e] = t.r1k[src + j];
      ix[e] = t.r1i[src + j];
    }
    // (the previous tile's writes read S.k, S.i, S.b, S.base and S.loc only: cnt is free)
    for (uint32_t j = threadIdx.x; j < p2; j += kBlock) S.cnt[j] = 0;
    __syncthreads();
#pragma unroll
    for (int e = 0; e < kPer; ++e) {
      const uint32_t j = j0 + e * kBlock + threadIdx.x;
      code[e] = ~0u;
      if (j < n1) {
        const uint32_t f2 = fine_bin(t, dedup_mix(k[e])) & (p2 - 1u);
        code[e] = (atomicAdd(&S.cnt[f2], 1u) << 8) | f2;
      }
    }
    __syncthreads();
    bin_write<kPer>(t, S, p2, k, ix, code, kCoarseCtrWords + ((uint32_t)c << lp2), 1u,
                    (uint32_t)c << lp2, 1u, t.c2, t.r2k, t.r2i);
  }
}

// One fine bin per block: insert its keys into an LDS table (CAS on the key word, atomic min on
// the index, a flag when a key arrives again), then mark every element of a repeated key and
// give it the key's lowest index.  A bin holds up to c2 entries but the table has kBinLds slots:
// it needs fewer distinct keys than slots, which the bins of folded (skewed) chunks meet by far.
// A bin with more distinct keys (no probe finds a free or matching slot) flags an overflow, and
// the chunk takes the exact fallback.
__global__ __launch_bounds__(kBlock) void k_bin_dedup(TableView t) {
  __shared__ unsigned long long hk[kBinLds];
  __shared__ uint32_t hm[kBinLds];
  __shared__ uint8_t hx[kBinLds];
  const uint32_t f = blockIdx.x;
  uint32_t fill;
  if (block_overflowed(t, &t.bcur[kCoarseCtrWords + f], &fill)) return;
  const uint32_t n = min(fill, t.c2);
  if (n == 0) return;
  const uint64_t* rk = t.r2k + (int64_t)f * t.c2;
  const uint32_t* ri = t.r2i + (int64_t)f * t.c2;
  // a bin holds at most c2 <= kPer * kBlock elements: each thread keeps its own in registers.
  // The loads are issued first, from clamped positions, and overlap the table's initialisation.
  // The first kPer0 rows cover any bin of uniform keys (1.75 x the mean); the rest are loaded
  // only when the fill reaches them (a uniform test).
  constexpr int kPer = (kBinFineCap + kBlock - 1) / kBlock;
  constexpr int kPer0 = 7;
  uint64_t kk[kPer];
  uint32_t slot[kPer], idx[kPer];
#pragma unroll
  for (int e = 0; e < kPer0; ++e) {
    const uint32_t j = min(threadIdx.x + e * kBlock, n - 1u);
    kk[e] = rk[j];
    idx[e] = ri[j];
  }
#pragma unroll
  for (int e = kPer0; e < kPer; ++e) {
    kk[e] = kEmpty;
    idx[e] = 0;
  }
  if (n > (uint32_t)(kPer0 * kBlock)) {
#pragma unroll
    for (int e = kPer0; e < kPer; ++e) {
      const uint32_t j = min(threadIdx.x + e * kBlock, n - 1u);
      kk[e] = rk[j];
      idx[e] = ri[j];
    }
  }
  for (uint32_t j = threadIdx.x; j < (uint32_t)kBinLds; j += kBlock) {
    hk[j] = kEmpty;
    hm[j] = kNone;
    hx[j] = 0;
  }
  __syncthreads();
#pragma unroll
  for (int e = 0; e < kPer; ++e) {
    const uint32_t j = threadIdx.x + e * kBlock;
    slot[e] = kNone;
    if (j < n) {
      const uint64_t key = kk[e];
      uint32_t s = (uint32_t)dedup_mix(key) & (kBinLds - 1);
      for (int probe = 0; probe < kBinLds; ++probe) {
        const unsigned long long old = atomicCAS(&hk[s], (unsigned long long)kEmpty,
                                                 (unsigned long long)key);
        if (old == kEmpty || old == key) {
          if (old == key) hx[s] = 1;
          atomicMin(&hm[s], idx[e]);
          slot[e] = s;
          break;
        }
        s = (s + 1) & (kBinLds - 1);
      }
      if (slot[e] == kNone) t.hdr->dovf = 1u;  // every slot holds another key
    }
  }
  __syncthreads();
#pragma unroll
  for (int e = 0; e < kPer; ++e) {
    if (slot[e] != kNone && hx[slot[e]]) {
      t.dmark[idx[e]] = 1;
      t.dfirst[idx[e]] = hm[slot[e]];
    }
  }
}

// Overflow path: clear dd (it aliases the coarse bins) and switch the chunk to dedup_range.
__global__ __launch_bounds__(kBlock) void k_bin_fallback_clear(TableView t, uint32_t dslots) {
  if (!t.hdr->dovf) {
    // the bins held: a chunk scattered without folding ends the skew hint
    if (blockIdx.x == 0 && threadIdx.x == 0 && !t.hdr->dagg) t.hdr->dskew = 0;
    return;
  }
  const uint4 empty = make_uint4(0xFFFFFFFFu, 0xFFFFFFFFu, 0xFFFFFFFFu, 0xFFFFFFFFu);
  for (int64_t j = (int64_t)blockIdx.x * kBlock + threadIdx.x; j < (int64_t)dslots / 2;
       j += (int64_t)gridDim.x * kBlock)
    reinterpret_cast<uint4*>(t.dd)[j] = empty;
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    t.hdr->dmode = 0;
    t.hdr->dskew = 1;   // later chunks of this table fold each tile's repeats first
    t.hdr->dskew_age = 0;
  }
}

__global__ __launch_bounds__(kBlock) void k_bin_fallback_dedup(TableView t,
                                                               const uint64_t* __restrict__ keys,
                                                               int64_t q, uint32_t dmask) {
  if (!t.hdr->dovf) return;
  dedup_range(t, keys, nullptr, dmask, (int64_t)blockIdx.x * kBlock, q, (int64_t)gridDim.x * kBlock);
}

// Index-order role of this lane's element: its own index when it is the first copy of its key in
// the chunk, else the index of that first copy.  `mark` is dmark[i], which the caller loads
// together with the key (one memory round trip instead of two).
__device__ __forceinline__ uint32_t first_copy(const TableView& t, const uint64_t* keys,
                                               uint64_t key, int64_t i, uint32_t dmask,
                                               uint32_t mark) {
  if (key >= kTomb) return t.hdr->spec_first[key - kTomb];
  if (mark) {
    if (!t.hdr->dmode) return dedup_lookup(t, keys, key, dmask, (uint32_t)i);
    const uint32_t f = t.dfirst[i];
    return (f & kIndirect) ? t.dfirst[f & ~kIndirect] : f;
  }
  return (uint32_t)i;
}

// Group probe of up to 8 keys at once.  Key u of the group (held by lane u, broadcast here) is
// probed when bit u of `A` is set.  All bucket loads of a round are issued before any is
// resolved.  Results: bit u of *found / *hadE / *freeb, and on lane u for its own key: the slot
// and value when found; with WANT_FREE, the first free slot on the probe path (bucket *myfb, slot
// *myc) and the key word seen there (*myexp, the expected value of a claim).
template <bool WANT_FREE>
__device__ __forceinline__ void group_probe(const TableView& t, uint64_t key, uint32_t A, int sub,
                                            uint32_t* found, uint32_t* hadE, uint32_t* freeb,
                                            uint64_t* mypos, uint64_t* myval, uint64_t* myfb,
                                            int* myc, uint64_t* myexp, uint64_t* mystep) {
  const int gb = group_base();
  // bucket indices and strides fit 32 bits (fewer than 2^31 buckets): half the registers and
  // shuffles of 64-bit copies
  uint64_t kk[kSlots];
  uint32_t b[kSlots], st[kSlots];
  Slot sl[kSlots];
  Seq mine = {0, 0};
  if ((A >> sub) & 1) mine = probe_seq(t, key);  // each lane hashes its own key once
  const uint32_t nb32 = (uint32_t)t.nb;
#pragma unroll
  for (int u = 0; u < kSlots; ++u) {
    kk[u] = __shfl(key, gb + u, 64);
    b[u] = (uint32_t)__shfl((uint32_t)mine.home, gb + u, 64);
    st[u] = (uint32_t)__shfl((uint32_t)mine.step, gb + u, 64);
  }
  uint32_t live = A, fnd = 0, he = 0, frb = 0;
  for (uint64_t round = 0; live && round < t.nb; ++round) {
    // unconditional: a branch around each load would make the compiler drain the load queue
    // before the next one; a finished key re-reads its last bucket (an L1 hit)
#pragma unroll
    for (int u = 0; u < kSlots; ++u) sl[u] = t.bk[b[u]].s[sub];
#pragma unroll
    for (int u = 0; u < kSlots; ++u) {
      if (!((live >> u) & 1)) continue;
      const uint32_t m = group_bits(__ballot(sl[u].key == kk[u]));
      const uint32_t e = group_bits(__ballot(sl[u].key == kEmpty));
      if (m) {
        const int c = lowest(m);
        const uint64_t v = __shfl(sl[u].val, gb + c, 64);
        if (sub == u) {
          *mypos = (uint64_t)b[u] * kSlots + (uint64_t)c;
          *myval = v;
        }
        fnd |= 1u << u;
        if (e) he |= 1u << u;
        live &= ~(1u << u);
        continue;
      }
      if (WANT_FREE && !((frb >> u) & 1)) {
        const uint32_t f = e | group_bits(__ballot(sl[u].key == kTomb));
        if (f) {
          const int c = lowest(f);
          const uint64_t seen = __shfl(sl[u].key, gb + c, 64);
          frb |= 1u << u;
          if (sub == u) {
            *myfb = b[u];
            *myc = c;
            *myexp = seen;
          }
        }
      }
      if (e) {
        live &= ~(1u << u);
      } else {
        const uint32_t nx = b[u] + st[u];   // < 2^32: both terms are below 2^31
        b[u] = nx >= nb32 ? nx - nb32 : nx;
      }
    }
  }
  *found = fnd;
  *hadE = he;
  *freeb = frb;
  *mystep = mine.step;
}

// Claims for the keys of the lanes in `want` (bit u: lane u's key is new and its probe saw a free
// slot first at bucket myfb, slot myc, holding myexp): every lane claims for its own key, one CAS
// instruction for the whole group; a key that lost its slot to another key scans on, one key at a
// time.  Returns this lane's claimed slot (meaningful on `want` lanes), kNoPos when none is left.
__device__ __forceinline__ uint64_t claim_group(const TableView& t, uint64_t key, uint32_t want,
                                                int sub, uint64_t myfb, int myc, uint64_t myexp,
                                                uint64_t mystep, uint32_t inject, uint64_t id) {
  uint64_t mypos = kNoPos;
  int won = 0;
  if ((want >> sub) & 1) {
    uint64_t expected = myexp;
    if (!inject || id % inject != 0) won = cas64(&t.bk[myfb].s[myc].key, expected, key) ? 1 : 0;
  }
  if (won) mypos = myfb * kSlots + (uint64_t)myc;
  const uint32_t retry = want & ~group_bits(__ballot(won));
  if (retry) {
    const int gb = group_base();
#pragma unroll
    for (int u = 0; u < kSlots; ++u) {
      if (!((retry >> u) & 1)) continue;
      const uint64_t ku = __shfl(key, gb + u, 64);
      const uint64_t fbu = __shfl(myfb, gb + u, 64);
      const uint64_t stu = __shfl(mystep, gb + u, 64);
      const uint64_t pos = claim(t, ku, fbu, stu, sub);
      if (sub == u) mypos = pos;
    }
  }
  return mypos;
}

// Insert actors, 8 elements per group and one per lane.  fast: claim directly with one CAS per
// new key (all CASes of the group in flight together; a lost race retries one key at a time).
// Otherwise (or with a pool) flag new keys for the ranked completion.
// Elements [lo, hi) of a chunk, 8 per group, the block's groups striding by `step` elements.
// `skip` (nullable): elements with a nonzero byte there take no part and keep their outputs.
// Returns this thread's count of stored keys.
template <int VK, bool ALLOC>
__device__ __forceinline__ int64_t insert_range(const TableView& t, const uint64_t* __restrict__ keys,
                                                const uint8_t* __restrict__ skip,
                                                const void* __restrict__ vals, uint32_t dmask,
                                                uint8_t* __restrict__ status,
                                                int32_t* __restrict__ vout, int64_t lo, int64_t hi,
                                                int64_t step) {
  const int sub = threadIdx.x & 7;
  const bool fast = t.hdr->fast != 0;
  const uint32_t inject = t.hdr->inject;
  const bool flags = ALLOC || !fast;
  int64_t ins = 0;
  for (int64_t g0 = lo + (int64_t)(threadIdx.x >> 3) * kSlots; g0 < hi; g0 += step) {
    const int64_t i = g0 + sub;
    const bool valid = i < hi;
    const uint64_t key = valid ? keys[i] : kEmpty;
    // the value is loaded with the key (coalesced) so that its latency hides behind the probe
    const uint64_t val = (!ALLOC && valid) ? load_val<VK>(vals, i) : 0;
    const uint32_t mark = t.dmark[min(i, hi - 1)];
    asm volatile("" ::"v"(mark));  // keep the load here, issued with the key's
    const bool active = valid && !(skip && skip[i]);
    const uint32_t first = active ? first_copy(t, keys, key, i, dmask, mark) : 0u;
    const bool actor = active && first == (uint32_t)i;
    const bool dup = active && !actor;
    const uint32_t slot = wave_append(dup, &t.hdr->ndup);
    if (dup) t.dup[slot] = make_uint2((uint32_t)i, first);

    uint8_t st = kNoStatus;
    uint8_t newf = 0;
    uint64_t ref = 0;
    if (actor && key >= kTomb) {  // out-of-band key: this lane alone
      const int s = (int)(key - kTomb);
      if (t.hdr->spec_live[s]) {
        st = kPresent;
        if (ALLOC && vout) vout[i] = (int32_t)(uint32_t)t.hdr->spec_val[s];
      } else if (!fast) {
        newf = 1;
      } else if (ALLOC) {
        t.hdr->spec_live[s] = 1;
        ref = kSpecRef + (uint64_t)s;
        newf = 1;
      } else {
        t.hdr->spec_live[s] = 1;
        t.hdr->spec_val[s] = val;
        st = kInserted;
        ++ins;
      }
    }
    const uint32_t A = group_bits(__ballot(actor && key < kTomb));
    if (A) {
      uint32_t found, hadE, freeb;
      uint64_t mypos = kNoPos, myval = 0, myfb = 0, myexp = 0;
      int myc = 0;
      uint64_t mystep = 0;
      group_probe<true>(t, key, A, sub, &found, &hadE, &freeb, &mypos, &myval, &myfb, &myc, &myexp,
                        &mystep);
      const uint32_t want = fast ? (A & ~found & freeb) : 0u;
      if (want) {
        // every lane claims for its own key: one CAS instruction for the whole group
        int won = 0;
        if ((want >> sub) & 1) {
          uint64_t expected = myexp;
          // (test hook: an injected loss leaves the slot free, so the retry below claims it)
          if (!inject || (uint64_t)i % inject != 0)
            won = cas64(&t.bk[myfb].s[myc].key, expected, key) ? 1 : 0;
        }
        if (won) mypos = myfb * kSlots + (uint64_t)myc;
        const uint32_t retry = want & ~group_bits(__ballot(won));
        if (retry) {  // lost a race for the slot to another key: scan on, one key at a time
          const int gb = group_base();
#pragma unroll
          for (int u = 0; u < kSlots; ++u) {
            if (!((retry >> u) & 1)) continue;
            const uint64_t ku = __shfl(key, gb + u, 64);
            const uint64_t fbu = __shfl(myfb, gb + u, 64);
            const uint64_t stu = __shfl(mystep, gb + u, 64);
            const uint64_t pos = claim(t, ku, fbu, stu, sub);
            if (sub == u) mypos = pos;
          }
        }
      }
      if ((A >> sub) & 1) {
        if ((found >> sub) & 1) {
          st = kPresent;
          if (ALLOC && vout) vout[i] = (int32_t)(uint32_t)myval;
        } else if (!fast) {
          newf = 1;
        } else if (!((want >> sub) & 1) || mypos == kNoPos) {
          st = kFull;  // no free slot anywhere: cannot happen while size + chunk <= capacity
          aor32(&t.hdr->err, kErrFull);
        } else if (ALLOC) {
          ref = mypos;
          newf = 1;
        } else {
          t.bk[mypos >> 3].s[mypos & 7].val = val;
          st = kInserted;
          ++ins;
        }
      }
    }
    if (valid) {
      if (flags) t.flag[i] = newf;
      if (ALLOC && newf) t.ref[i] = ref;
      if (status && st != kNoStatus) status[i] = st;
    }
  }
  return ins;
}

// Map inserts are held to 96 VGPRs (5 waves per SIMD); the set and allocating variants need more
// and keep the compiler's choice.
template <int VK, bool ALLOC>
__global__ __launch_bounds__(kBlock) __attribute__((amdgpu_waves_per_eu((ALLOC || VK == 0) ? 1 : 5))) void k_insert(TableView t, const uint64_t* __restrict__ keys,
                                                   const void* __restrict__ vals, int64_t q,
                                                   uint32_t dmask, uint8_t* __restrict__ status,
                                                   int32_t* __restrict__ vout,
                                                   const uint8_t* __restrict__ skip,
                                                   int count_tiles) {
  const int64_t ins = insert_range<VK, ALLOC>(t, keys, skip, vals, dmask, status, vout,
                                              (int64_t)blockIdx.x * kBlock, q,
                                              (int64_t)gridDim.x * kBlock);
  // one partial per block, summed by k_apply_count: no same-address atomics across the grid
  const int64_t tot = block_sum(ins);
  if (threadIdx.x == 0) t.bcnt[blockIdx.x] = tot;
  if (ALLOC && count_tiles) {
    // the rank flags per tile (what k_tile_count computes): each pass of the block covers 256
    // consecutive elements, all in one tile, and each thread re-reads the flag it wrote itself;
    // the tile sums were zeroed by the chunk's prologue
    for (int64_t b0 = (int64_t)blockIdx.x * kBlock; b0 < q; b0 += (int64_t)gridDim.x * kBlock) {
      __syncthreads();  // block_sum's partials are reused
      const int64_t i = b0 + threadIdx.x;
      const int64_t c = block_sum((int64_t)(i < q ? t.flag[i] : 0));
      if (threadIdx.x == 0 && c) aadd32(&t.tsum[b0 / kTile], (uint32_t)c);
    }
  }
}

// Host-side resizing (a table's capacity is fixed when it is created, Section 4; it grows by a
// copy into a larger table): every live pair of src is inserted into dst.  One 8-lane group per
// src bucket, its 8 slots as the group's keys.  The keys of src are distinct and the host has
// checked that dst has room for all of them, so a new key claims a slot directly; a key dst
// already holds stays unchanged.  Counts per block, summed by k_apply_count.
__global__ __launch_bounds__(kBlock) void k_rehash(TableView src, TableView dst) {
  const int sub = threadIdx.x & 7;
  const int64_t nbk = (int64_t)src.nb;
  const int64_t gpb = kBlock / 8;
  const int64_t ngroups = (int64_t)gridDim.x * gpb;
  const int64_t span = ((nbk + ngroups - 1) / ngroups) * ngroups;  // equal trips for all lanes
  const uint32_t inject = dst.hdr->inject;
  int64_t ins = 0;
  for (int64_t g = (int64_t)blockIdx.x * gpb + (threadIdx.x >> 3); g < span; g += ngroups) {
    Slot sl;
    sl.key = kEmpty;
    sl.val = 0;
    if (g < nbk) sl = src.bk[g].s[sub];
    const bool live = sl.key != kEmpty && sl.key != kTomb;
    const uint64_t key = live ? sl.key : kEmpty;
    const uint32_t A = group_bits(__ballot(live));
    if (!A) continue;
    uint32_t found, hadE, freeb;
    uint64_t mypos = kNoPos, myval = 0, myfb = 0, myexp = 0;
    int myc = 0;
    uint64_t mystep = 0;
    group_probe<true>(dst, key, A, sub, &found, &hadE, &freeb, &mypos, &myval, &myfb, &myc, &myexp,
                      &mystep);
    const uint32_t want = A & ~found & freeb;
    uint64_t pos = kNoPos;
    if (want)
      pos = claim_group(dst, key, want, sub, myfb, myc, myexp, mystep, inject,
                        (uint64_t)g * kSlots + (uint64_t)sub);
    if (live && !((found >> sub) & 1)) {
      if (((want >> sub) & 1) && pos != kNoPos) {
        dst.bk[pos >> 3].s[pos & 7].val = sl.val;
        ++ins;
      } else {
        aor32(&dst.hdr->err, kErrFull);  // not reached while dst has the room the host checked
      }
    }
  }
  if (blockIdx.x == 0 && threadIdx.x == 0) {  // the out-of-band keys
    for (int s = 0; s < 2; ++s) {
      if (src.hdr->spec_live[s] && !dst.hdr->spec_live[s]) {
        dst.hdr->spec_live[s] = 1;
        dst.hdr->spec_val[s] = src.hdr->spec_val[s];
        ++ins;
      }
    }
  }
  const int64_t tot = block_sum(ins);
  if (threadIdx.x == 0) dst.bcnt[blockIdx.x] = tot;
}

// Erase actors, 8 elements per group.  RELEASE: the removed value is kept for the ordered push.
template <bool RELEASE>
__device__ __forceinline__ int64_t erase_range(const TableView& t, const uint64_t* __restrict__ keys,
                                               uint32_t dmask, uint8_t* __restrict__ erased,
                                               int64_t lo, int64_t hi, int64_t step) {
  const int sub = threadIdx.x & 7;
  int64_t del = 0;
  for (int64_t g0 = lo + (int64_t)(threadIdx.x >> 3) * kSlots; g0 < hi; g0 += step) {
    const int64_t i = g0 + sub;
    const bool valid = i < hi;
    const uint64_t key = valid ? keys[i] : kEmpty;
    const uint32_t mark = t.dmark[min(i, hi - 1)];
    asm volatile("" ::"v"(mark));  // keep the load here, issued with the key's
    const bool actor = valid && first_copy(t, keys, key, i, dmask, mark) == (uint32_t)i;
    uint8_t hit = 0;
    uint64_t val = 0;
    if (actor && key >= kTomb) {
      const int s = (int)(key - kTomb);
      if (t.hdr->spec_live[s]) {
        t.hdr->spec_live[s] = 0;
        val = t.hdr->spec_val[s];
        hit = 1;
      }
    }
    const uint32_t A = group_bits(__ballot(actor && key < kTomb));
    if (A) {
      uint32_t found, hadE, freeb;
      uint64_t mypos = kNoPos, myval = 0, myfb = 0, myexp = 0;
      int myc = 0;
      uint64_t mystep = 0;
      group_probe<false>(t, key, A, sub, &found, &hadE, &freeb, &mypos, &myval, &myfb, &myc, &myexp,
                         &mystep);
      if ((found >> sub) & 1) {
        // kEmpty only where the bucket already holds one: no probe sequence runs through it
        t.bk[mypos >> 3].s[mypos & 7].key = ((hadE >> sub) & 1) ? kEmpty : kTomb;
        val = myval;
        hit = 1;
      }
    }
    if (valid) {
      if (erased) erased[i] = hit;
      if (RELEASE) {
        t.flag[i] = hit;
        t.ref[i] = val;
      }
      del += hit;
    }
  }
  return del;
}

template <bool RELEASE>
__global__ __launch_bounds__(kBlock) void k_erase(TableView t, const uint64_t* __restrict__ keys,
                                                  int64_t q, uint32_t dmask,
                                                  uint8_t* __restrict__ erased) {
  const int64_t del = erase_range<RELEASE>(t, keys, dmask, erased, (int64_t)blockIdx.x * kBlock, q,
                                           (int64_t)gridDim.x * kBlock);
  const int64_t tot = block_sum(del);
  if (threadIdx.x == 0) t.bcnt[blockIdx.x] = -tot;
}

// Add the per-block partials of the preceding insert/erase kernel to the live count.
// Returns the change (valid on thread 0).
__device__ __forceinline__ int64_t apply_count_block(const TableView& t, int nparts) {
  int64_t v = 0;
  for (int j = threadIdx.x; j < nparts; j += blockDim.x) v += t.bcnt[j];
  v = (int64_t)wave_sum((uint64_t)v);
  __shared__ int64_t part[16];
  if (wave_lane() == 0) part[threadIdx.x >> 6] = v;
  __syncthreads();
  int64_t s = 0;
  if (threadIdx.x == 0) {
    for (int w = 0; w < (int)(blockDim.x >> 6); ++w) s += part[w];
    if (s) t.hdr->size = (uint64_t)((int64_t)t.hdr->size + s);
  }
  __syncthreads();
  return s;
}

// The host's view of how an insert chunk of q keys went: q and the keys it stored, one 64-bit
// store to host-mapped memory (read without synchronising; a stale or torn read only changes
// which path the next chunk takes, never a result).
// Word 0 reports insert chunks (keys stored), word 1 erase chunks (keys removed).
__device__ __forceinline__ void chunk_feedback(const TableView& t, int word, int64_t q,
                                               int64_t changed) {
  if (q <= 0) return;
  const uint64_t w = ((uint64_t)q << 32) | (uint64_t)(uint32_t)(changed < 0 ? 0 : changed);
  t.hdr->fbd[word] = w;
  if (t.fb) __hip_atomic_store(t.fb + word, w, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
}

// fb_q > 0: the partials are the count changes of an insert (fb_word 0) or erase (fb_word 1)
// chunk of fb_q keys: report how many keys the chunk stored or removed.
__global__ __launch_bounds__(1024) void k_apply_count(TableView t, int nblocks, int64_t fb_q,
                                                      int fb_word) {
  const int64_t s = apply_count_block(t, nblocks);
  if (threadIdx.x == 0 && fb_q) chunk_feedback(t, fb_word, fb_q, fb_word ? -s : s);
}

// ---------------------------------------------------------------------------------------------
// Speculative insert: repeated keys resolved after the table update instead of before it.
//
// When the host can prove that a chunk cannot reach capacity, no element can meet FULL and the
// index order matters only among copies of one key.  Every element then probes and claims for
// itself.  Claims only turn free slots into keys during the kernel, and every copy of a key takes
// the first free slot of the same probe sequence, so a key is stored at most once: a copy either
// claims the slot, sees the key in a bucket, or loses its CAS to the key (the rescan after a lost
// CAS looks for the key as well as for free slots).  The claimer is whichever copy got there
// first, not necessarily the lowest index, and a copy that sees the key cannot tell whether it
// was there before the chunk.  Such elements are "listed" (flag 2; claimers have flag 1): they
// report PRESENT.  After the kernel, a key needs a fix only when it has a claimer and a listed
// copy of lower index; that copy becomes the inserter (its value goes into the slot, the statuses
// swap).  A listed key without a claimer was present before the chunk, so PRESENT was right.
//
// The resolution pairs claimers with listed copies through the dd table, in the direction that
// puts fewer keys into it: with few listed elements (a batch of mostly new keys), the listed keys
// enter dd with their lowest index and the claimers look themselves up; with mostly listed
// elements (keys that are mostly present already), the claimers enter dd and each listed copy
// lowers the index beside its claimer's entry, which the claimer checks afterwards.  The
// out-of-band keys are always listed and resolved by one thread.  With distinct keys absent from
// the table nothing is listed, and the resolution kernels return at once.
// ---------------------------------------------------------------------------------------------
constexpr int kListStripes = 32;          // listed-count stripes, one per 128-byte line
constexpr int kListStripeWords = 32;      // u32 words between stripes
enum : uint8_t { kFlagNone = 0, kFlagClaimed = 1, kFlagListed = 2 };

// The listed-count stripes sit behind the block partials of the table's bcnt region.
__device__ __forceinline__ uint32_t* list_stripes(const TableView& t) {
  return reinterpret_cast<uint32_t*>(t.bcnt + kMaxGroupBlocks);
}

__device__ __forceinline__ uint32_t listed_total(const TableView& t) {
  const uint32_t* st = list_stripes(t);
  uint32_t n = 0;
  for (int j = 0; j < kListStripes; ++j) n += st[j * kListStripeWords];
  return n;
}

// Claim for an absent key from bucket b on (the retry after a lost CAS), watching for the key
// itself: *seen is set when a copy of the key holds a slot on the way.  Returns the claimed slot,
// or kNoPos (also when seen).
__device__ __forceinline__ uint64_t claim_watch(const TableView& t, uint64_t key, uint64_t b,
                                                uint64_t stride, int sub, bool* seen) {
  for (uint64_t step = 0; step < t.nb; ++step) {
    const uint64_t cur = t.bk[b].s[sub].key;
    if (group_bits(__ballot(cur == key))) {
      *seen = true;
      return kNoPos;
    }
    uint32_t f = group_bits(__ballot(cur == kEmpty || cur == kTomb));
    while (f) {
      const int c = lowest(f);
      int won = 0, same = 0;
      if (sub == c) {
        uint64_t expected = cur;
        won = cas64(&t.bk[b].s[c].key, expected, key) ? 1 : 0;
        same = !won && expected == key;
      }
      if (group_bits(__ballot(won))) return b * kSlots + (uint64_t)c;
      if (group_bits(__ballot(same))) {
        *seen = true;
        return kNoPos;
      }
      f &= f - 1;
    }
    b = next_bucket(t, b, stride);
  }
  return kNoPos;
}

// Elements [lo, hi) of a chunk, 8 per group.  Returns this thread's (stored, listed) counts.
template <int VK>
__device__ __forceinline__ uint2 insert_spec_range(const TableView& t,
                                                   const uint64_t* __restrict__ keys,
                                                   const void* __restrict__ vals,
                                                   uint8_t* __restrict__ status, int64_t lo,
                                                   int64_t hi, int64_t step) {
  const int sub = threadIdx.x & 7;
  const uint32_t inject = t.hdr->inject;
  uint32_t ins = 0, listed = 0;
  for (int64_t g0 = lo + (int64_t)(threadIdx.x >> 3) * kSlots; g0 < hi; g0 += step) {
    const int64_t i = g0 + sub;
    const bool valid = i < hi;
    const uint64_t key = valid ? keys[i] : kEmpty;
    const uint64_t val = valid ? load_val<VK>(vals, i) : 0;
    bool amb = valid && key >= kTomb;  // out-of-band keys: resolved after the kernel
    uint8_t st = kPresent;
    uint8_t claimed = 0;
    const uint32_t A = group_bits(__ballot(valid && key < kTomb));
    if (A) {
      uint32_t found, hadE, freeb;
      uint64_t mypos = kNoPos, myval = 0, myfb = 0, myexp = 0;
      int myc = 0;
      uint64_t mystep = 0;
      group_probe<true>(t, key, A, sub, &found, &hadE, &freeb, &mypos, &myval, &myfb, &myc, &myexp,
                        &mystep);
      const uint32_t want = A & ~found & freeb;
      bool seen = false;
      if (want) {
        int won = 0;
        if ((want >> sub) & 1) {
          uint64_t expected = myexp;
          // (test hook: an injected loss leaves the slot free, so the retry below claims it)
          if (!inject || (uint64_t)i % inject != 0) {
            won = cas64(&t.bk[myfb].s[myc].key, expected, key) ? 1 : 0;
            seen = !won && expected == key;
          }
        }
        if (won) mypos = myfb * kSlots + (uint64_t)myc;
        const uint32_t retry = want & ~group_bits(__ballot(won || seen));
        if (retry) {  // lost the slot to another key: scan on, one key at a time
          const int gb = group_base();
#pragma unroll
          for (int u = 0; u < kSlots; ++u) {
            if (!((retry >> u) & 1)) continue;
            const uint64_t ku = __shfl(key, gb + u, 64);
            const uint64_t fbu = __shfl(myfb, gb + u, 64);
            const uint64_t stu = __shfl(mystep, gb + u, 64);
            bool su = false;
            const uint64_t pos = claim_watch(t, ku, fbu, stu, sub, &su);
            if (sub == u) {
              mypos = pos;
              seen = su;
            }
          }
        }
      }
      if ((A >> sub) & 1) {
        if (((found >> sub) & 1) || seen) {
          amb = true;
        } else if (!((want >> sub) & 1) || mypos == kNoPos) {
          st = kFull;  // no free slot anywhere: cannot happen while size + chunk <= capacity
          aor32(&t.hdr->err, kErrFull);
        } else {
          if (VK) t.bk[mypos >> 3].s[mypos & 7].val = val;
          st = kInserted;
          claimed = 1;
          ++ins;
        }
      }
    }
    if (valid) {
      t.flag[i] = claimed ? kFlagClaimed : (amb ? kFlagListed : kFlagNone);
      if (status) status[i] = st;
      listed += amb ? 1u : 0u;
    }
  }
  return make_uint2(ins, listed);
}

template <int VK>
__global__ __launch_bounds__(kBlock) __attribute__((amdgpu_waves_per_eu(VK == 0 ? 1 : 5))) void k_insert_spec(TableView t, const uint64_t* __restrict__ keys,
                                                        const void* __restrict__ vals, int64_t q,
                                                        uint8_t* __restrict__ status) {
  const uint2 c = insert_spec_range<VK>(t, keys, vals, status, (int64_t)blockIdx.x * kBlock, q,
                                        (int64_t)gridDim.x * kBlock);
  // both counts in one reduction: stored in the low half, listed in the high half
  const int64_t tot = block_sum((int64_t)c.x + ((int64_t)c.y << 32));
  if (threadIdx.x == 0) {
    t.bcnt[blockIdx.x] = tot & 0xFFFFFFFFll;
    const uint32_t nl = (uint32_t)(tot >> 32);
    // one atomic per block with listed elements, spread over the stripes
    if (nl) aadd32(&list_stripes(t)[(blockIdx.x % kListStripes) * kListStripeWords], nl);
  }
}

// Speculative erase: every element probes; a found key is removed with one CAS (key -> kEmpty
// where its bucket holds an empty slot, else kTomb), so of several copies exactly one removes it
// (flag 1, reports 1).  A copy that loses that CAS or finds no key is listed (flag 2, reports 0):
// afterwards the lowest listed copy takes the removal over from a higher remover.  A copy cannot
// miss a key that is still there: an erase writes kEmpty only into buckets that already hold one,
// so no probe sequence is cut short.  Out-of-band keys are always listed.
__device__ __forceinline__ uint2 erase_spec_range(const TableView& t, const uint64_t* __restrict__ keys,
                                                  uint8_t* __restrict__ erased, int64_t lo,
                                                  int64_t hi, int64_t step) {
  const int sub = threadIdx.x & 7;
  uint32_t del = 0, listed = 0;
  for (int64_t g0 = lo + (int64_t)(threadIdx.x >> 3) * kSlots; g0 < hi; g0 += step) {
    const int64_t i = g0 + sub;
    const bool valid = i < hi;
    const uint64_t key = valid ? keys[i] : kEmpty;
    bool amb = valid && key >= kTomb;
    uint8_t hit = 0;
    const uint32_t A = group_bits(__ballot(valid && key < kTomb));
    if (A) {
      uint32_t found, hadE, freeb;
      uint64_t mypos = kNoPos, myval = 0, myfb = 0, myexp = 0;
      int myc = 0;
      uint64_t mystep = 0;
      group_probe<false>(t, key, A, sub, &found, &hadE, &freeb, &mypos, &myval, &myfb, &myc, &myexp,
                         &mystep);
      if ((A >> sub) & 1) {
        if ((found >> sub) & 1) {
          uint64_t expected = key;
          const uint64_t gone = ((hadE >> sub) & 1) ? kEmpty : kTomb;
          if (cas64(&t.bk[mypos >> 3].s[mypos & 7].key, expected, gone)) hit = 1;
          else amb = true;
        } else {
          amb = true;
        }
      }
    }
    if (valid) {
      t.flag[i] = hit ? kFlagClaimed : (amb ? kFlagListed : kFlagNone);
      if (erased) erased[i] = hit;
      del += hit;
      listed += amb ? 1u : 0u;
    }
  }
  return make_uint2(del, listed);
}

__global__ __launch_bounds__(kBlock) void k_erase_spec(TableView t, const uint64_t* __restrict__ keys,
                                                       int64_t q, uint8_t* __restrict__ erased) {
  const uint2 c = erase_spec_range(t, keys, erased, (int64_t)blockIdx.x * kBlock, q,
                                   (int64_t)gridDim.x * kBlock);
  const int64_t tot = block_sum((int64_t)c.x + ((int64_t)c.y << 32));
  if (threadIdx.x == 0) {
    t.bcnt[blockIdx.x] = -(tot & 0xFFFFFFFFll);
    const uint32_t nl = (uint32_t)(tot >> 32);
    if (nl) aadd32(&list_stripes(t)[(blockIdx.x % kListStripes) * kListStripeWords], nl);
  }
}

// The host's size bound has proved that the chunk cannot reach capacity; a live count that
// says otherwise is a library bug and raises kErrInternal.  Also zeroes the listed counts.
__global__ void k_spec_prologue(TableView t, int64_t q, int insert) {
  if (threadIdx.x < kListStripes) list_stripes(t)[threadIdx.x * kListStripeWords] = 0;
  if (threadIdx.x == 0) {
    Header* h = t.hdr;
    h->size0 = h->size;
    h->spec_first[0] = h->spec_first[1] = kNone;
    h->ndup = 0;
    h->nnew = 0;
    h->fast = 1u;
    h->spec = 1u;
    h->dmode = 0u;
    if (insert && h->size + (uint64_t)q > t.cap) h->err |= kErrInternal;
  }
}

// Resolution direction and dd entries for `nd` listed elements of a q-element chunk.
struct SpecPlan {
  bool by_claimers;  // claimers enter dd (mostly listed elements)
  uint32_t slots;    // dd entries in use: a power of two >= 2 x the keys entering dd
};

__device__ __forceinline__ SpecPlan spec_plan(uint32_t nd, int64_t q) {
  SpecPlan p;
  p.by_claimers = 2 * (int64_t)nd > q;
  const uint32_t enter = p.by_claimers ? (uint32_t)(q - nd) : nd;
  uint32_t s = 2;
  while (s < 2 * enter) s <<= 1;
  p.slots = s;
  return p;
}

// In the claimer direction, the lowest listed index per claimer entry sits behind the entries.
__device__ __forceinline__ uint32_t* spec_low(const TableView& t, const SpecPlan& p) {
  return reinterpret_cast<uint32_t*>(t.dd + p.slots);
}

// One block: the count change of the insert or erase kernel (`nblocks` partials) goes into the
// live count and the feedback word; the listed counts are summed into the header for the
// kernels that follow.
__global__ __launch_bounds__(1024) void k_spec_sum(TableView t, int nblocks, int64_t q, int erase) {
  const int64_t change = apply_count_block(t, nblocks);
  if (threadIdx.x == 0) {
    chunk_feedback(t, erase, q, erase ? -change : change);
    t.hdr->ndup = listed_total(t);
  }
}

// Clears the dd entries (and, in the claimer direction, the lowest-index words) the resolution
// uses; nothing when no element is listed.
// (The resolution stages take their block b of nb as arguments, so that the grouped plan can run
// them per step; the single-table kernels pass blockIdx.x and gridDim.x.)
__device__ __forceinline__ void spec_clear_range(const TableView& t, int64_t q, int64_t b, int64_t nb) {
  const uint32_t nd = t.hdr->ndup;
  if (nd == 0) return;
  const SpecPlan p = spec_plan(nd, q);
  const int64_t units = p.slots / 2;
  const uint4 ones = make_uint4(0xFFFFFFFFu, 0xFFFFFFFFu, 0xFFFFFFFFu, 0xFFFFFFFFu);
  for (int64_t j = b * kBlock + threadIdx.x; j < units; j += nb * kBlock) {
    reinterpret_cast<uint4*>(t.dd)[j] = ones;
    if (p.by_claimers && j < units / 2) reinterpret_cast<uint4*>(spec_low(t, p))[j] = ones;
  }
  if (p.by_claimers && units == 1 && b == 0 && threadIdx.x == 0) {
    spec_low(t, p)[0] = kNone;
    spec_low(t, p)[1] = kNone;
  }
}

__global__ __launch_bounds__(kBlock) void k_spec_clear(TableView t, int64_t q) {
  spec_clear_range(t, q, blockIdx.x, gridDim.x);
}

// dd slot of `key` among entries (tag | chunk index); kNone when absent.
__device__ __forceinline__ uint32_t dd_find(const TableView& t, const uint64_t* keys, uint64_t key,
                                           uint32_t dmask, uint32_t* idx) {
  const uint64_t mix = dedup_mix(key);
  const uint64_t tag = mix & 0xFFFFFFFF00000000ull;
  uint32_t h = (uint32_t)mix & dmask;
  for (uint32_t probe = 0; probe <= dmask; ++probe) {
    const uint64_t e = t.dd[h];
    if (e == kEmpty) return kNone;
    if ((e & 0xFFFFFFFF00000000ull) == tag && keys[(uint32_t)e] == key) {
      *idx = (uint32_t)e;
      return h;
    }
    h = (h + 1) & dmask;
  }
  return kNone;
}

// Build: the keys that enter dd.  Listed direction: windows of 256 elements first resolve their
// listed keys in LDS, so a key listed many times costs one CAS or atomic min per window (skipped
// when the held index is already lower).  Claimer direction: every claimer's key is distinct, so
// each takes an empty entry with one CAS.  Out-of-band listed copies take an atomic min on their
// header word in both directions.
__device__ __forceinline__ void spec_build_range(const TableView& t, const uint64_t* __restrict__ keys,
                                                 int64_t q, int64_t blk, int64_t nblk) {
  const uint32_t nd = t.hdr->ndup;  // written by k_spec_sum
  if (nd == 0) return;
  const SpecPlan p = spec_plan(nd, q);
  const uint32_t dmask = p.slots - 1;
  constexpr uint32_t kW = 2 * kBlock;
  __shared__ unsigned long long wk[kW];
  __shared__ uint32_t wmin[kW];
  for (int64_t b0 = blk * kBlock; b0 < q; b0 += nblk * kBlock) {
    const int64_t i = b0 + threadIdx.x;
    const uint8_t f = i < q ? t.flag[i] : kFlagNone;
    const uint64_t key = f != kFlagNone ? keys[i] : kEmpty;
    if (f == kFlagListed && key >= kTomb) amin32(&t.hdr->spec_first[key - kTomb], (uint32_t)i);
    const uint64_t mix = dedup_mix(key);
    const uint64_t tag = mix & 0xFFFFFFFF00000000ull;
    if (p.by_claimers) {
      if (f == kFlagClaimed) {
        uint32_t h = (uint32_t)mix & dmask;
        for (uint32_t probe = 0; probe <= dmask; ++probe) {
          uint64_t expected = kEmpty;
          if (cas64(&t.dd[h], expected, tag | (uint64_t)i)) break;
          h = (h + 1) & dmask;
        }
      }
      continue;
    }
    // listed direction (uniform per block: p depends only on nd and q)
    for (uint32_t j = threadIdx.x; j < kW; j += kBlock) {
      wk[j] = kEmpty;
      wmin[j] = kNone;
    }
    __syncthreads();
    const bool normal = f == kFlagListed && key < kTomb;
    uint32_t s = (uint32_t)(mix >> 32) & (kW - 1);
    if (normal) {
      for (;;) {  // at most kBlock keys in kW slots: a free or matching slot exists
        const unsigned long long old = atomicCAS(&wk[s], (unsigned long long)kEmpty,
                                                 (unsigned long long)key);
        if (old == kEmpty || old == key) break;
        s = (s + 1) & (kW - 1);
      }
      atomicMin(&wmin[s], (uint32_t)i);
    }
    __syncthreads();
    if (normal && wmin[s] == (uint32_t)i) {
      const uint64_t mine = tag | (uint64_t)i;
      uint32_t h = (uint32_t)mix & dmask;
      for (uint32_t probe = 0; probe <= dmask; ++probe) {
        uint64_t e = t.dd[h];
        if (e == kEmpty) {
          uint64_t expected = kEmpty;
          if (cas64(&t.dd[h], expected, mine)) break;
          e = expected;
        }
        if ((e & 0xFFFFFFFF00000000ull) == tag && keys[(uint32_t)e] == key) {
          if ((uint32_t)i < (uint32_t)e) amin64(&t.dd[h], mine);
          break;
        }
        h = (h + 1) & dmask;
      }
    }
    __syncthreads();  // the window's LDS table is reused by the next window
  }
}

__global__ __launch_bounds__(kBlock) void k_spec_build(TableView t, const uint64_t* __restrict__ keys,
                                                       int64_t q) {
  spec_build_range(t, keys, q, blockIdx.x, gridDim.x);
}

// Slot of a key that is known to be stored (one lane alone, eight key loads per bucket).
__device__ __forceinline__ uint64_t lane_slot_of(const TableView& t, uint64_t key) {
  const Seq q = probe_seq(t, key);
  uint64_t b = q.home;
  for (uint64_t step = 0; step < t.nb; ++step) {
    for (int c = 0; c < kSlots; ++c)
      if (t.bk[b].s[c].key == key) return b * kSlots + (uint64_t)c;
    b = next_bucket(t, b, q.step);
  }
  return kNoPos;
}

// Claimer c hands the insert of its key to listed copy m < c: m's value into the slot, statuses
// swapped.
// An erase only moves the outcome: m reports the removal, c reports none (both statuses are the
// insert's INSERTED / PRESENT values, 1 / 0).
template <int VK, bool ERASE>
__device__ __forceinline__ void hand_over(const TableView& t, const void* __restrict__ vals,
                                          uint8_t* __restrict__ status, uint64_t key, uint32_t c,
                                          uint32_t m) {
  if (ERASE) {
    if (status) {
      status[m] = 1;
      status[c] = 0;
    }
    return;
  }
  const uint64_t pos = lane_slot_of(t, key);
  if (pos == kNoPos) {
    aor32(&t.hdr->err, kErrInternal);
    return;
  }
  if (VK) t.bk[pos >> 3].s[pos & 7].val = load_val<VK>(vals, m);
  if (status) {
    status[m] = kInserted;
    status[c] = kPresent;
  }
}

// Probe: listed direction: every claimer looks its key up and hands over to a lower listed copy.
// Claimer direction: every listed copy of a claimed key lowers the index word beside the entry
// (windows of 256 elements combine copies of one entry in LDS first; skipped when the word is
// already lower).
template <int VK, bool ERASE>
__device__ __forceinline__ void spec_probe_range(const TableView& t, const uint64_t* __restrict__ keys,
                                                 const void* __restrict__ vals, int64_t q,
                                                 uint8_t* __restrict__ status, int64_t blk,
                                                 int64_t nblk) {
  const uint32_t nd = t.hdr->ndup;  // written by k_spec_sum
  if (nd == 0) return;
  const SpecPlan p = spec_plan(nd, q);
  const uint32_t dmask = p.slots - 1;
  uint32_t* low = spec_low(t, p);
  constexpr uint32_t kW = 2 * kBlock;
  __shared__ uint32_t wh[kW], wmin[kW];
  for (int64_t b0 = blk * kBlock; b0 < q; b0 += nblk * kBlock) {
    const int64_t i = b0 + threadIdx.x;
    const uint8_t f = i < q ? t.flag[i] : kFlagNone;
    if (!p.by_claimers) {
      if (f == kFlagClaimed) {
        const uint64_t key = keys[i];
        uint32_t m = 0;
        if (dd_find(t, keys, key, dmask, &m) != kNone && m < (uint32_t)i)
          hand_over<VK, ERASE>(t, vals, status, key, (uint32_t)i, m);
      }
      continue;
    }
    for (uint32_t j = threadIdx.x; j < kW; j += kBlock) {
      wh[j] = kNone;
      wmin[j] = kNone;
    }
    __syncthreads();
    uint32_t h = kNone, s = 0;
    if (f == kFlagListed) {
      const uint64_t key = keys[i];
      uint32_t c = 0;
      if (key < kTomb) {
        h = dd_find(t, keys, key, dmask, &c);
        if (h != kNone && (uint32_t)i > c) h = kNone;  // the claimer is lower: nothing to do
      }
    }
    if (h != kNone) {
      s = (h * 2654435761u) & (kW - 1);
      for (;;) {  // at most kBlock entries in kW slots
        const uint32_t old = atomicCAS(&wh[s], kNone, h);
        if (old == kNone || old == h) break;
        s = (s + 1) & (kW - 1);
      }
      atomicMin(&wmin[s], (uint32_t)i);
    }
    __syncthreads();
    if (h != kNone && wmin[s] == (uint32_t)i && (uint32_t)i < low[h]) amin32(&low[h], (uint32_t)i);
    __syncthreads();
  }
}

template <int VK, bool ERASE>
__global__ __launch_bounds__(kBlock) void k_spec_probe(TableView t, const uint64_t* __restrict__ keys,
                                                       const void* __restrict__ vals, int64_t q,
                                                       uint8_t* __restrict__ status) {
  spec_probe_range<VK, ERASE>(t, keys, vals, q, status, blockIdx.x, gridDim.x);
}

// Swap (claimer direction): a claimer whose entry holds a lower listed index hands over.  Thread
// 0 of the first block settles each out-of-band key on its lowest copy (an insert stores it when
// it was absent, an erase removes it when it was there).
template <int VK, bool ERASE>
__device__ __forceinline__ void spec_swap_range(const TableView& t, const uint64_t* __restrict__ keys,
                                                const void* __restrict__ vals, int64_t q,
                                                uint8_t* __restrict__ status, int64_t blk,
                                                int64_t nblk) {
  const uint32_t nd = t.hdr->ndup;  // written by k_spec_sum
  if (nd == 0) return;
  if (blk == 0 && threadIdx.x == 0) {
    Header* h = t.hdr;
    for (int s = 0; s < 2; ++s) {
      const uint32_t m = h->spec_first[s];
      if (m == kNone) continue;
      if (ERASE) {  // the lowest copy removes the key when it was there
        if (!h->spec_live[s]) continue;
        h->spec_live[s] = 0;
        h->size -= 1;
        if (status) status[m] = 1;
      } else {      // the lowest copy stores the key when it was absent
        if (h->spec_live[s]) continue;
        h->spec_live[s] = 1;
        h->spec_val[s] = load_val<VK>(vals, m);
        h->size += 1;
        if (status) status[m] = kInserted;
      }
    }
  }
  const SpecPlan p = spec_plan(nd, q);
  if (!p.by_claimers) return;
  const uint32_t dmask = p.slots - 1;
  const uint32_t* low = spec_low(t, p);
  for (int64_t c = blk * kBlock + threadIdx.x; c < q; c += nblk * kBlock) {
    if (t.flag[c] != kFlagClaimed) continue;
    const uint64_t key = keys[c];
    uint32_t self = 0;
    const uint32_t h = dd_find(t, keys, key, dmask, &self);
    if (h == kNone) {
      aor32(&t.hdr->err, kErrInternal);
      continue;
    }
    const uint32_t m = low[h];
    if (m < (uint32_t)c) hand_over<VK, ERASE>(t, vals, status, key, (uint32_t)c, m);
  }
}

template <int VK, bool ERASE>
__global__ __launch_bounds__(kBlock) void k_spec_swap(TableView t, const uint64_t* __restrict__ keys,
                                                      const void* __restrict__ vals, int64_t q,
                                                      uint8_t* __restrict__ status) {
  spec_swap_range<VK, ERASE>(t, keys, vals, q, status, blockIdx.x, gridDim.x);
}

// Flagged count per tile of kTile elements.
__global__ __launch_bounds__(kBlock) void k_tile_count(TableView t, int64_t q, int only_slow) {
  if (only_slow && t.hdr->fast) return;
  __shared__ uint32_t part[kBlock / 64];
  const int64_t t0 = (int64_t)blockIdx.x * kTile;
  uint64_t c = 0;
  for (int j = threadIdx.x; j < kTile; j += kBlock) {
    const int64_t i = t0 + j;
    if (i < q) c += t.flag[i];
  }
  c = wave_sum(c);
  if (wave_lane() == 0) part[threadIdx.x >> 6] = (uint32_t)c;
  __syncthreads();
  if (threadIdx.x == 0) {
    uint32_t s = 0;
    for (int w = 0; w < kBlock / 64; ++w) s += part[w];
    t.tsum[blockIdx.x] = s;
  }
}


// One block of NT threads: exclusive scan of the tile counts, then the counter updates the ranks
// imply.  mode 0: insert near capacity; 1: insert with pool values; 2: erase releasing to the pool.
// A chunk's totals once its nnew new actors are ranked: the live count, the pool top and the
// error bits (mode 0 insert near capacity, 1 insert with pool values, 2 erase releasing to the
// pool).  One thread.
__device__ __forceinline__ void rank_totals(const TableView& t, PoolHeader* pool, uint64_t nnew,
                                            int mode) {
  Header* h = t.hdr;
  h->nnew = (uint32_t)nnew;
  const uint64_t room = t.cap - h->size0;
  if (mode == 0) {
    const uint64_t ins = nnew < room ? nnew : room;
    h->size = h->size0 + ins;
    if (nnew > room) h->err |= kErrFull;
  } else if (mode == 1) {
    const uint64_t avail = (uint64_t)pool->top0;
    const uint64_t lim = room < avail ? room : avail;
    const uint64_t ins = nnew < lim ? nnew : lim;
    h->size = h->size0 + ins;
    pool->top = pool->top0 - (int64_t)ins;
    if (nnew > lim) {
      if (room <= avail) h->err |= kErrFull;
      else h->err |= kErrPool;
    }
  } else {
    const uint64_t room_p = (uint64_t)(pool->cap - pool->top0);
    const uint64_t pushed = nnew < room_p ? nnew : room_p;
    pool->top = pool->top0 + (int64_t)pushed;
    if (nnew > room_p) pool->err |= kErrPool;
  }
}

template <int NT>
__device__ __forceinline__ void scan_tiles_block(const TableView& t, PoolHeader* pool, int ntiles,
                                                 int mode) {
  __shared__ uint32_t carry;
  __shared__ uint32_t ws[NT / 64];
  if (threadIdx.x == 0) carry = 0;
  __syncthreads();
  for (int base = 0; base < ntiles; base += NT) {
    const int j = base + (int)threadIdx.x;
    const uint32_t v = j < ntiles ? t.tsum[j] : 0u;
    const int lane = wave_lane();
    uint32_t x = v;
    for (int off = 1; off < 64; off <<= 1) {
      const uint32_t y = __shfl_up(x, off, 64);
      if (lane >= off) x += y;
    }
    if (lane == 63) ws[threadIdx.x >> 6] = x;
    __syncthreads();
    uint32_t before = 0, all = 0;
    for (int w = 0; w < NT / 64; ++w) {
      if (w < (int)(threadIdx.x >> 6)) before += ws[w];
      all += ws[w];
    }
    if (j < ntiles) t.tsum[j] = carry + before + x - v;
    __syncthreads();
    if (threadIdx.x == 0) carry += all;
    __syncthreads();
  }
  if (threadIdx.x == 0) rank_totals(t, pool, carry, mode);
  __syncthreads();
}

__global__ __launch_bounds__(1024) void k_tile_scan(TableView t, PoolHeader* pool, int ntiles,
                                                    int mode) {
  if (mode == 0 && t.hdr->fast) return;
  scan_tiles_block<1024>(t, pool, ntiles, mode);
}

// Ranked completion of flagged elements, one tile per block.
// MODE 0: insert near capacity (rank < room -> claim, else FULL)
// MODE 1: insert with pool values (rank < min(room, pool) -> value = pool element top0-1-rank)
// MODE 2: erase releasing to the pool (pool element top0+rank = value)
// (the batch moves only the back of the pool: head is fixed while it runs)
template <int VK, int MODE>
__device__ __forceinline__ void final_tile(const TableView& t, PoolHeader* pool,
                                           int32_t* __restrict__ pstack,
                                           const uint64_t* __restrict__ keys,
                                           const void* __restrict__ vals, int64_t q,
                                           uint8_t* __restrict__ status,
                                           int32_t* __restrict__ vout, int64_t tile,
                                           int inline_tiles) {
  const bool fast = t.hdr->fast != 0;
  if (MODE == 0 && fast) return;
  __shared__ uint16_t list[kTile];
  const int64_t t0 = tile * kTile;
  uint32_t f[kTile / kBlock];
  uint32_t cnt = 0;
#pragma unroll
  for (int k = 0; k < kTile / kBlock; ++k) {
    const int64_t i = t0 + (int64_t)threadIdx.x * (kTile / kBlock) + k;
    f[k] = i < q ? t.flag[i] : 0u;
    cnt += f[k];
  }
  uint32_t total;
  uint32_t o = block_exclusive_scan(cnt, &total);
#pragma unroll
  for (int k = 0; k < kTile / kBlock; ++k)
    if (f[k]) list[o++] = (uint16_t)(threadIdx.x * (kTile / kBlock) + k);
  __syncthreads();
  // inline_tiles == 0: the tile sums hold the rank scan's exclusive prefixes.  inline_tiles = n > 0
  // (small chunks, no scan launched): they hold the n tiles' counts; each block adds those before
  // its tile, and the block of tile 0 also settles the chunk's totals as the scan would.
  uint64_t rbase;
  if (inline_tiles > 0) {
    __shared__ uint64_t rb_shared;
    uint64_t before = 0, all = 0;
    for (int j = threadIdx.x; j < inline_tiles; j += kBlock) {
      const uint64_t c = t.tsum[j];
      all += c;
      if (j < tile) before += c;
    }
    before = (uint64_t)block_sum((int64_t)before);
    __syncthreads();  // block_sum's partials are reused
    all = (uint64_t)block_sum((int64_t)all);
    if (threadIdx.x == 0) {
      rb_shared = before;
      if (tile == 0) rank_totals(t, pool, all, MODE);
    }
    __syncthreads();
    rbase = rb_shared;
  } else {
    rbase = t.tsum[tile];
  }
  const Header* h = t.hdr;
  const uint64_t room = t.cap - h->size0;
  const int sub = threadIdx.x & 7;
  for (uint32_t j = threadIdx.x >> 3; j < total; j += kBlock / 8) {
    const int64_t i = t0 + list[j];
    const uint64_t rank = rbase + j;
    if constexpr (MODE == 2) {
      if (sub == 0) {
        const int64_t pos = pool->top0 + (int64_t)rank;
        if (pos < pool->cap)
          pstack[ring_pos(pool->head, pool->cap, pos)] = (int32_t)(uint32_t)t.ref[i];
      }
      continue;
    } else {
      uint64_t lim = room;
      if constexpr (MODE == 1) {
        const uint64_t avail = (uint64_t)pool->top0;
        lim = room < avail ? room : avail;
      }
      if (rank >= lim) {
        if (sub == 0) {
          if (status) status[i] = kFull;
          if (MODE == 1 && vout) vout[i] = -1;
        }
        continue;
      }
      const uint64_t key = keys[i];
      uint64_t v = 0;
      if constexpr (MODE == 1)
        v = (uint64_t)(uint32_t)pstack[ring_pos(pool->head, pool->cap, pool->top0 - 1 - (int64_t)rank)];
      else v = load_val<VK>(vals, i);
      uint64_t pos;
      if (MODE == 1 && fast) {
        pos = t.ref[i];
      } else if (key >= kTomb) {
        pos = kSpecRef + (key - kTomb);
        if (sub == 0) t.hdr->spec_live[key - kTomb] = 1;
      } else {
        const Probe p = probe(t, key, sub, true);
        pos = p.has_free ? claim(t, key, p.free_b, probe_seq(t, key).step, sub) : kNoPos;
      }
      if (pos >= kSpecRef && pos != kNoPos) {
        if (sub == 0) t.hdr->spec_val[pos - kSpecRef] = v;
      } else if (pos != kNoPos) {
        if (sub == (int)(pos & 7)) t.bk[pos >> 3].s[pos & 7].val = v;
      }
      if (sub == 0) {
        if (status) status[i] = pos == kNoPos ? kFull : kInserted;
        if (MODE == 1 && vout) vout[i] = pos == kNoPos ? -1 : (int32_t)(uint32_t)v;
      }
    }
  }
  __syncthreads();  // the tile list is reused by the caller's next tile
}

template <int VK, int MODE>
__global__ __launch_bounds__(kBlock) void k_final(TableView t, PoolHeader* pool,
                                                  int32_t* __restrict__ pstack,
                                                  const uint64_t* __restrict__ keys,
                                                  const void* __restrict__ vals, int64_t q,
                                                  uint8_t* __restrict__ status,
                                                  int32_t* __restrict__ vout, int inline_tiles) {
  final_tile<VK, MODE>(t, pool, pstack, keys, vals, q, status, vout, blockIdx.x, inline_tiles);
}

// Later copies of a key take the outcome of its first occurrence: PRESENT (or its value), unless
// the first occurrence met FULL, which a later copy meets again.
__device__ __forceinline__ void fix_range(const TableView& t, uint8_t* __restrict__ status,
                                          int32_t* __restrict__ vout, int64_t lo, int64_t step) {
  const int64_t nd = t.hdr->ndup;
  for (int64_t j = lo + threadIdx.x; j < nd; j += step) {
    const uint2 d = t.dup[j];
    if (vout) vout[d.x] = vout[d.y];
    if (status) status[d.x] = status[d.y] == kFull ? kFull : kPresent;
  }
}

__global__ __launch_bounds__(kBlock) void k_fix(TableView t, uint8_t* __restrict__ status,
                                                int32_t* __restrict__ vout) {
  fix_range(t, status, vout, (int64_t)blockIdx.x * blockDim.x, (int64_t)gridDim.x * blockDim.x);
}

// find / contains, 8 keys per group and one per lane for loading and storing (coalesced).  The
// group probes its keys together in rounds: every pending bucket load of a round is issued before
// the first ballot, so a lane has up to 8 independent 16-byte loads in flight.
template <int VK>
__device__ __forceinline__ void find_range(const TableView& t, const uint64_t* __restrict__ keys,
                                           void* __restrict__ out, uint8_t* __restrict__ found_out,
                                           int64_t lo, int64_t hi, int64_t step) {
  const int sub = threadIdx.x & 7;
  for (int64_t g0 = lo + (int64_t)(threadIdx.x >> 3) * kSlots; g0 < hi; g0 += step) {
    const int64_t i = g0 + sub;
    const bool valid = i < hi;
    const uint64_t key = valid ? keys[i] : kEmpty;
    bool hit = false;
    uint64_t v = 0;
    if (valid && key >= kTomb) {
      hit = t.hdr->spec_live[key - kTomb] != 0;
      v = t.hdr->spec_val[key - kTomb];
    }
    const uint32_t A = group_bits(__ballot(valid && key < kTomb));
    if (A) {
      uint32_t found, hadE, freeb;
      uint64_t mypos = kNoPos, myval = 0, myfb = 0, myexp = 0;
      int myc = 0;
      uint64_t mystep = 0;
      group_probe<false>(t, key, A, sub, &found, &hadE, &freeb, &mypos, &myval, &myfb, &myc, &myexp,
                         &mystep);
      if ((A >> sub) & 1) {
        hit = (found >> sub) & 1;
        v = myval;
      }
    }
    if (valid) {
      if (out) store_val<VK>(out, i, hit ? v : sentinel<VK>());
      if (found_out) found_out[i] = hit ? 1 : 0;
    }
  }
}

template <int VK>
__global__ __launch_bounds__(kBlock) void k_find(TableView t, const uint64_t* __restrict__ keys,
                                                 int64_t n, void* __restrict__ out,
                                                 uint8_t* __restrict__ found_out) {
  find_range<VK>(t, keys, out, found_out, (int64_t)blockIdx.x * kBlock, n,
                 (int64_t)gridDim.x * kBlock);
}

// Range selection (Section 3.6: a range of the container becomes a vector through a copy_if),
// and the dump, which selects every live pair.  Appending through one shared counter serialises
// (every append is an atomic on the same address), so block b owns a contiguous slot range:
// k_sel_count writes its count to bcnt[b], k_sel_scan turns the counts into offsets (and the
// total, out-of-band keys included, into dump_count), and k_sel_write reads the range again and
// writes each accepted pair at its block's offset plus its rank in the block.  The out-of-band
// keys go last.  Predicates see the key only.
struct AllKeys {
  __device__ bool operator()(uint64_t) const { return true; }
};
struct KeyRange {
  uint64_t lo, hi;  // lo <= key < hi, unsigned
  __device__ bool operator()(uint64_t key) const { return key >= lo && key < hi; }
};
struct VoxelBox {
  int32_t lo[3], hi[3];  // packed block coordinates in [lo, hi], bounds included
  __device__ bool operator()(uint64_t key) const {
    if (key >> 63) return false;  // packs no block
#pragma unroll
    for (int d = 0; d < 3; ++d) {
      const uint32_t f = (uint32_t)(key >> (21 * d)) & 0x1FFFFFu;
      const int32_t c = (int32_t)(f << 11) >> 11;  // sign-extend the 21-bit field
      if (c < lo[d] || c > hi[d]) return false;
    }
    return true;
  }
};

constexpr int kSelPer = 8;                       // slots per thread and round
constexpr int64_t kSelRound = (int64_t)kBlock * kSelPer;

template <class Pred>
__device__ __forceinline__ uint32_t sel_round(const TableView& t, const Pred& pred, int64_t r0,
                                              int64_t hi, Slot (&sl)[kSelPer]) {
  uint32_t take = 0;
#pragma unroll
  for (int e = 0; e < kSelPer; ++e) {   // loads first (clamped), then the tests
    const int64_t j = min(r0 + e * kBlock + (int64_t)threadIdx.x, hi - 1);
    sl[e] = t.bk[j >> 3].s[j & 7];
  }
#pragma unroll
  for (int e = 0; e < kSelPer; ++e) {
    const int64_t j = r0 + e * kBlock + (int64_t)threadIdx.x;
    if (j < hi && sl[e].key != kEmpty && sl[e].key != kTomb && pred(sl[e].key)) take |= 1u << e;
  }
  return take;
}

template <class Pred>
__global__ __launch_bounds__(kBlock) void k_sel_count(TableView t, Pred pred, int64_t per) {
  const int64_t nslots = (int64_t)t.nb * kSlots;
  const int64_t lo = (int64_t)blockIdx.x * per;
  const int64_t hi = min(lo + per, nslots);
  int64_t c = 0;
  Slot sl[kSelPer];
  for (int64_t r0 = lo; r0 < hi; r0 += kSelRound) c += __builtin_popcount(sel_round(t, pred, r0, hi, sl));
  const int64_t tot = block_sum(c);
  if (threadIdx.x == 0) t.bcnt[blockIdx.x] = tot;
}

template <class Pred>
__global__ __launch_bounds__(1024) void k_sel_scan(TableView t, Pred pred, int nblocks) {
  __shared__ int64_t wsum[16];
  const int per = (nblocks + 1023) / 1024;
  const int b0 = (int)threadIdx.x * per;
  int64_t loc = 0;
  for (int j = 0; j < per; ++j)
    if (b0 + j < nblocks) loc += t.bcnt[b0 + j];
  const int lane = wave_lane();
  int64_t x = loc;
  for (int off = 1; off < 64; off <<= 1) {
    const int64_t y = __shfl_up(x, off, 64);
    if (lane >= off) x += y;
  }
  if (lane == 63) wsum[threadIdx.x >> 6] = x;
  __syncthreads();
  int64_t before = 0, total = 0;
  for (int w = 0; w < (int)(blockDim.x >> 6); ++w) {
    if (w < (int)(threadIdx.x >> 6)) before += wsum[w];
    total += wsum[w];
  }
  int64_t run = before + x - loc;
  for (int j = 0; j < per; ++j) {
    if (b0 + j >= nblocks) break;
    const int64_t c = t.bcnt[b0 + j];
    t.bcnt[b0 + j] = run;
    run += c;
  }
  if (threadIdx.x == 0) {
    for (int sp = 0; sp < 2; ++sp)
      if (t.hdr->spec_live[sp] && pred(kTomb + (uint64_t)sp)) ++total;
    t.hdr->dump_count = (uint64_t)total;
  }
}

template <class Pred>
__global__ __launch_bounds__(kBlock) void k_sel_write(TableView t, Pred pred, int64_t per,
                                                      uint64_t* __restrict__ kout,
                                                      uint64_t* __restrict__ vout, int64_t cap) {
  const int64_t nslots = (int64_t)t.nb * kSlots;
  const int64_t lo = (int64_t)blockIdx.x * per;
  const int64_t hi = min(lo + per, nslots);
  int64_t off = t.bcnt[blockIdx.x];
  Slot sl[kSelPer];
  for (int64_t r0 = lo; r0 < hi; r0 += kSelRound) {
    const uint32_t take = sel_round(t, pred, r0, hi, sl);
    uint32_t total;
    uint32_t p = block_exclusive_scan((uint32_t)__builtin_popcount(take), &total);
#pragma unroll
    for (int e = 0; e < kSelPer; ++e) {
      if (!((take >> e) & 1u)) continue;
      const int64_t at = off + p++;
      if (at < cap) {
        kout[at] = sl[e].key;
        if (vout) vout[at] = sl[e].val;
      }
    }
    off += total;
  }
  if (blockIdx.x == 0 && threadIdx.x == 0) {  // the out-of-band keys, after every bucket's
    int64_t at = (int64_t)t.hdr->dump_count;
    for (int sp = 0; sp < 2; ++sp)
      if (t.hdr->spec_live[sp] && pred(kTomb + (uint64_t)sp)) --at;
    for (int sp = 0; sp < 2; ++sp) {
      if (!t.hdr->spec_live[sp] || !pred(kTomb + (uint64_t)sp)) continue;
      if (at < cap) {
        kout[at] = kTomb + (uint64_t)sp;
        if (vout) vout[at] = t.hdr->spec_val[sp];
      }
      ++at;
    }
  }
}

// Set-up and fold of a striped launch of the reference kernels below: zero the stripes and decide
// whether the launch can meet the capacity (the live count plus `maxins` inserts), then add the
// stripes to the live count.  The decision is one word that every wave of the launch reads.
__global__ __launch_bounds__(64) void k_dev_prep(TableView t, uint64_t maxins) {
  t.bcnt[threadIdx.x * kStripeStride] = 0;
  if (threadIdx.x == 0) {
    const uint64_t n = t.hdr->size;
    t.bcnt[kStripeFlag] = (n <= t.cap && maxins <= t.cap - n) ? 1 : 0;
  }
}

__global__ __launch_bounds__(64) void k_dev_fold(TableView t) {
  if (!t.bcnt[kStripeFlag]) return;
  const uint64_t s = wave_sum((uint64_t)t.bcnt[threadIdx.x * kStripeStride]);
  if (threadIdx.x == 0) t.hdr->size += s;
}

// One element of the reference kernels below: operation `op` on keys[i] through the device
// functions, its status (and found value) written at i.
__device__ __forceinline__ void dev_apply_one(const DevView& v, int32_t op, int64_t i, uint64_t key,
                                              const void* __restrict__ vals, int32_t vk,
                                              void* __restrict__ vout, uint8_t* __restrict__ status) {
  if (op == CT_OP_INSERT) {
    const uint64_t val = vk == 2 ? static_cast<const uint64_t*>(vals)[i]
                         : vk == 1 ? (uint64_t)static_cast<const uint32_t*>(vals)[i] : 0ull;
    const uint8_t st = dev_insert(v, key, val);
    if (status) status[i] = st;
  } else if (op == CT_OP_ERASE) {
    const bool hit = dev_erase(v, key);
    if (status) status[i] = hit ? 1 : 0;
  } else {
    uint64_t val = 0;
    const bool hit = dev_find(v, key, &val);
    if (status) status[i] = hit ? 1 : 0;
    if (vout) {
      if (vk == 2) static_cast<uint64_t*>(vout)[i] = hit ? val : ~0ull;
      else if (vk == 1) static_cast<uint32_t*>(vout)[i] = hit ? (uint32_t)val : ~0u;
    }
  }
}

// Per-thread operations through the device-side API (ct_dev_api.h): element i is handled by one
// thread, all concurrently and in no particular order.  The reference user kernel, and what the
// tests drive the device API with.
__global__ __launch_bounds__(kBlock) void k_dev_apply(DevView v, int32_t op, const uint64_t* __restrict__ keys,
                                                      const void* __restrict__ vals, int32_t vk,
                                                      int64_t n, void* __restrict__ vout,
                                                      uint8_t* __restrict__ status) {
  if (v.striped) v.striped = (int32_t)v.t.bcnt[kStripeFlag];
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x)
    dev_apply_one(v, op, i, keys[i], vals, vk, vout, status);
}

// The mixed-mode reference kernel: element i does operation ops[i], every element concurrently.
// A workgroup takes a window of kSortWin elements and sorts their indices by operation into LDS
// queues, then runs each queue on consecutive threads, so most waves call one device function
// with all 64 lanes and their probes go as a team.  An unknown code leaves the table alone and
// reports kNoStatus; non-find elements get the absent sentinel as their value.
constexpr int kSortWin = 4 * kBlock;

__global__ __launch_bounds__(kBlock) void k_dev_apply_sorted(DevView v, const uint8_t* __restrict__ ops,
                                                             const uint64_t* __restrict__ keys,
                                                             const void* __restrict__ vals, int32_t vk,
                                                             int64_t n, void* __restrict__ vout,
                                                             uint8_t* __restrict__ status) {
  constexpr int32_t kKind[3] = {CT_OP_FIND, CT_OP_INSERT, CT_OP_ERASE};
  __shared__ uint16_t q[3][kSortWin];
  __shared__ uint32_t qn[3];
  if (v.striped) v.striped = (int32_t)v.t.bcnt[kStripeFlag];
  const uint64_t below = (1ull << wave_lane()) - 1ull;
  const int64_t nwin = (n + kSortWin - 1) / kSortWin;
  for (int64_t w = blockIdx.x; w < nwin; w += gridDim.x) {  // the same trips for the whole block
    if (threadIdx.x < 3) qn[threadIdx.x] = 0;
    __syncthreads();
#pragma unroll
    for (int r = 0; r < kSortWin / kBlock; ++r) {
      const int slot = r * kBlock + (int)threadIdx.x;
      const int64_t i = w * kSortWin + slot;
      int kind = -1;
      if (i < n) {
        const int32_t op = ops[i];
        kind = op == CT_OP_FIND ? 0 : op == CT_OP_INSERT ? 1 : op == CT_OP_ERASE ? 2 : -1;
        if (vout && op != CT_OP_FIND) {
          if (vk == 2) static_cast<uint64_t*>(vout)[i] = ~0ull;
          else if (vk == 1) static_cast<uint32_t*>(vout)[i] = ~0u;
        }
        if (kind < 0 && status) status[i] = kNoStatus;
      }
      // one LDS add per wave and kind; order inside the wave by rank among the kind's lanes
#pragma unroll
      for (int k = 0; k < 3; ++k) {
        const uint64_t m = __ballot(kind == k);
        if (!m) continue;
        uint32_t base = 0;
        if (wave_lane() == __builtin_ctzll(m)) base = atomicAdd(&qn[k], (uint32_t)__builtin_popcountll(m));
        base = __shfl(base, __builtin_ctzll(m), 64);
        if (kind == k) q[k][base + (uint32_t)__builtin_popcountll(m & below)] = (uint16_t)slot;
      }
    }
    __syncthreads();
#pragma unroll
    for (int k = 0; k < 3; ++k) {
      const uint32_t cnt = qn[k];
      for (uint32_t j = threadIdx.x; j < cnt; j += kBlock) {
        const int64_t e = w * kSortWin + q[k][j];
        dev_apply_one(v, kKind[k], e, keys[e], vals, vk, vout, status);
      }
    }
    __syncthreads();  // the queues are read before the next window refills them
  }
}

// The neighbour update of a block map (the allocation step of the reconstruction workload behind
// Section 4.1's voxel-block example): every block of `blocks` makes sure that its 6 face
// neighbours (ndirs 6) or all 26 neighbours (ndirs 26) are in the table, each new one with the
// index of a block that asked for it as its value, or (ALLOC) with pop_back() of the index pool,
// as a reconstruction allocates voxel blocks.  Coordinates wrap in their 21-bit fields.
template <bool ALLOC>
__global__ __launch_bounds__(kBlock) void k_voxel_neighbours(DevView v, DevPool pool,
                                                             const uint64_t* __restrict__ blocks,
                                                             int64_t n, int32_t ndirs) {
  if (v.striped) v.striped = (int32_t)v.t.bcnt[kStripeFlag];
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x) {
    const uint64_t b = blocks[i];
    const int32_t x = sfield21(b), y = sfield21(b >> 21), z = sfield21(b >> 42);
    for (int d = 0; d < 27; ++d) {
      const int dx = d % 3 - 1, dy = (d / 3) % 3 - 1, dz = d / 9 - 1;
      const int nz = (dx != 0) + (dy != 0) + (dz != 0);
      if (nz == 0 || (ndirs == 6 && nz != 1)) continue;
      const uint64_t k = ((uint64_t)(uint32_t)(x + dx) & 0x1FFFFFull) |
                         (((uint64_t)(uint32_t)(y + dy) & 0x1FFFFFull) << 21) |
                         (((uint64_t)(uint32_t)(z + dz) & 0x1FFFFFull) << 42);
      if (dev_contains(v, k)) continue;
      if constexpr (ALLOC) {
        int32_t got;
        dev_insert_alloc(v, pool, k, &got);
      } else {
        dev_insert(v, k, (uint64_t)(uint32_t)i);
      }
    }
  }
}

// The two-container step of the reconstruction example of Section 4.1: every thread asks the
// block map whether its key is there (contains, read-only on `map`) and, if so, inserts the key
// into the update set `set` (an unordered_set, many threads may insert the same key).  status[i]:
// kNoStatus when the map lacks the key, else the set insert's PRESENT / INSERTED / FULL.
__global__ __launch_bounds__(kBlock) void k_dev_update_set(DevView map, DevView set,
                                                           const uint64_t* __restrict__ keys,
                                                           int64_t n, uint8_t* __restrict__ status) {
  if (set.striped) set.striped = (int32_t)set.t.bcnt[kStripeFlag];
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x) {
    const uint64_t key = keys[i];
    uint8_t st = kNoStatus;
    if (dev_contains(map, key)) st = dev_insert(set, key, 0);
    if (status) status[i] = st;
  }
}

// Per-thread push_back / pop_back through the device-side API: element i by one thread, all
// concurrently.
__global__ __launch_bounds__(kBlock) void k_dev_pool_apply(DevPool p, int32_t op,
                                                           const int32_t* __restrict__ in, int64_t n,
                                                           int32_t* __restrict__ out,
                                                           uint8_t* __restrict__ status) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x) {
    bool ok;
    if (op == CT_DEV_PUSH_BACK) {
      ok = dev_push_back(p, in[i]);
    } else {
      int32_t v = -1;
      ok = dev_pop_back(p, &v);
      if (out) out[i] = ok ? v : -1;
    }
    if (status) status[i] = ok ? 1 : 2;
  }
}

__global__ void k_check_begin(TableView t) {
  Header* h = t.hdr;
  h->live_count = 0;
  h->violations = 0;
  h->dup_count = 0;
  h->pool_bad = 0;
  h->pool_count = 0;
  h->pool_h1 = 0;
  h->pool_h2 = 0;
}

// Two independent 64-bit fingerprints of a pool index.  Sums of them over a multiset (wrapping)
// are equal for equal multisets; a multiset that differs from {0 .. P-1} (an index missing,
// repeated, or replaced) changes both sums except with probability about 2^-64 each.
__device__ __forceinline__ uint64_t check_h1(uint64_t v) { return fmix64(v + 0x9E3779B97F4A7C15ull); }
__device__ __forceinline__ uint64_t check_h2(uint64_t v) {
  return fmix64(v * 0xD1B54A32D192ED03ull + 0x632BE59BD9B4E019ull);
}

struct CheckSums {
  uint64_t live = 0, unreach = 0, dup = 0, pbad = 0, h1 = 0, h2 = 0;
  int64_t pcnt = 0;
};

__device__ __forceinline__ void check_pool_value(CheckSums& c, uint64_t v, int64_t pool_cap) {
  if (v >= (uint64_t)pool_cap) {
    ++c.pbad;
  } else {
    ++c.pcnt;
    c.h1 += check_h1(v);
    c.h2 += check_h2(v);
  }
}

__device__ __forceinline__ void check_flush(const TableView& t, CheckSums c) {
  c.live = wave_sum(c.live);
  c.unreach = wave_sum(c.unreach);
  c.dup = wave_sum(c.dup);
  c.pbad = wave_sum(c.pbad);
  c.h1 = wave_sum(c.h1);
  c.h2 = wave_sum(c.h2);
  c.pcnt = (int64_t)wave_sum((uint64_t)c.pcnt);
  if (wave_lane() == 0) {
    Header* h = t.hdr;
    if (c.live) aadd64(&h->live_count, c.live);
    if (c.unreach) aadd64(&h->violations, c.unreach);
    if (c.dup) aadd64(&h->dup_count, c.dup);
    if (c.pbad) aadd64(&h->pool_bad, c.pbad);
    if (c.pcnt) aadd64(reinterpret_cast<uint64_t*>(&h->pool_count), (uint64_t)c.pcnt);
    if (c.h1) aadd64(&h->pool_h1, c.h1);
    if (c.h2) aadd64(&h->pool_h2, c.h2);
  }
}

// Every live key must be reachable (no bucket between its home and its own bucket holds a kEmpty
// slot, so a lookup finds it) and stored once: a second copy of a key lies on the same probe
// path, so the walk of the later copy passes the earlier one (or an earlier slot of its own
// bucket).  With pool_cap > 0 the live values are pool indices and enter the fingerprint sums.
__global__ __launch_bounds__(kBlock) void k_check(TableView t, int64_t pool_cap) {
  const int64_t tid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t nt = (int64_t)gridDim.x * blockDim.x;
  const int64_t nslots = (int64_t)t.nb * kSlots;
  CheckSums c;
  for (int64_t j = tid; j < nslots; j += nt) {
    const Slot sl = t.bk[j >> 3].s[j & 7];
    if (sl.key == kEmpty || sl.key == kTomb) continue;
    ++c.live;
    const uint64_t at = (uint64_t)(j >> 3);
    const int own = (int)(j & 7);
    const Seq q = probe_seq(t, sl.key);
    uint64_t b = q.home;
    bool unreachable = false, dup = false;
    for (uint64_t step = 0;; ++step) {
      if (step >= t.nb) { unreachable = true; break; }
      const bool last = b == at;
      bool has_empty = false;
      for (int s = 0; s < kSlots; ++s) {
        const uint64_t k2 = t.bk[b].s[s].key;
        has_empty |= k2 == kEmpty;
        dup |= k2 == sl.key && (!last || s < own);
      }
      if (last) break;
      if (has_empty) { unreachable = true; break; }
      b = next_bucket(t, b, q.step);
    }
    c.unreach += unreachable;
    c.dup += dup;
    if (pool_cap > 0) check_pool_value(c, sl.val, pool_cap);
  }
  if (pool_cap > 0 && tid == 0) {
    for (int s = 0; s < 2; ++s)
      if (t.hdr->spec_live[s]) check_pool_value(c, t.hdr->spec_val[s], pool_cap);
  }
  check_flush(t, c);
}

// The pool's entries enter the fingerprint sums, and every index 0 .. cap-1 leaves them once: the
// sums and the count end at zero exactly when the pool and the table's live values together hold
// each index once.
__global__ __launch_bounds__(kBlock) void k_check_pool(TableView t, const PoolHeader* ph,
                                                       const int32_t* __restrict__ stack) {
  const int64_t tid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t nt = (int64_t)gridDim.x * blockDim.x;
  const int64_t top = ph->top, head = ph->head, cap = ph->cap;
  CheckSums c;
  for (int64_t j = tid; j < cap; j += nt) {
    if (j < top) {
      const int32_t v = stack[ring_pos(head, cap, j)];
      check_pool_value(c, v < 0 ? ~0ull : (uint64_t)v, cap);
    }
    --c.pcnt;
    c.h1 -= check_h1((uint64_t)j);
    c.h2 -= check_h2((uint64_t)j);
  }
  check_flush(t, c);
}

// ---------------------------------------------------------------------------------------------
// table health and purge.  An erase leaves a tombstone where its bucket holds no empty slot, and
// inserts turn tombstones back into keys; nothing turns a tombstone back into an empty slot, so
// under long churn the buckets without an empty slot grow in number, and lookups of absent keys
// walk past more of them.  The purge reopens every bucket that no live key's probe path passes:
// its tombstones become empty slots.  A bucket that some live key passes (one before that key's
// own bucket on its path) keeps its tombstones, so every live key stays reachable.
// ---------------------------------------------------------------------------------------------
// Buckets without an empty slot, and tombstones; 8 lanes per bucket.
__global__ __launch_bounds__(kBlock) void k_health(TableView t) {
  const int sub = threadIdx.x & 7;
  const int64_t ngroups = (int64_t)gridDim.x * (kBlock / 8);
  uint64_t closed = 0, tombs = 0;
  const int64_t nbk = (int64_t)t.nb;
  const int64_t span = ((nbk + ngroups - 1) / ngroups) * ngroups;   // equal trips: ballots below
  for (int64_t b = (int64_t)blockIdx.x * (kBlock / 8) + (threadIdx.x >> 3); b < span; b += ngroups) {
    const uint64_t key = b < nbk ? t.bk[b].s[sub].key : 0;
    const uint32_t e = group_bits(__ballot(b < nbk && key == kEmpty));
    if (b < nbk && sub == 0 && !e) ++closed;
    if (b < nbk && key == kTomb) ++tombs;
  }
  closed = wave_sum(closed);
  tombs = wave_sum(tombs);
  if (wave_lane() == 0) {
    if (closed) aadd64(&t.hdr->closed_count, closed);
    if (tombs) aadd64(&t.hdr->tomb_count, tombs);
  }
}

__global__ void k_health_begin(TableView t) {
  t.hdr->closed_count = 0;
  t.hdr->tomb_count = 0;
}

__global__ __launch_bounds__(kBlock) void k_purge_clear(uint32_t* __restrict__ bits, int64_t words) {
  for (int64_t j = (int64_t)blockIdx.x * kBlock + threadIdx.x; j < words;
       j += (int64_t)gridDim.x * kBlock)
    bits[j] = 0;
}

// Bit (b - w0) for every bucket b in [w0, w1) that a live key's probe path passes before the
// key's own bucket.
__global__ __launch_bounds__(kBlock) void k_purge_mark(TableView t, uint32_t* __restrict__ bits,
                                                       int64_t w0, int64_t w1) {
  const int64_t nslots = (int64_t)t.nb * kSlots;
  for (int64_t j = (int64_t)blockIdx.x * kBlock + threadIdx.x; j < nslots;
       j += (int64_t)gridDim.x * kBlock) {
    const uint64_t key = t.bk[j >> 3].s[j & 7].key;
    if (key == kEmpty || key == kTomb) continue;
    const uint64_t at = (uint64_t)(j >> 3);
    const Seq q = probe_seq(t, key);
    uint64_t b = q.home;
    for (uint64_t step = 0; b != at && step < t.nb; ++step) {
      if ((int64_t)b >= w0 && (int64_t)b < w1) {
        const uint64_t r = b - (uint64_t)w0;
        atomicOr(&bits[r >> 5], 1u << (r & 31));
      }
      b = next_bucket(t, b, q.step);
    }
  }
}

// Every bucket of [w0, w1) that no live key passes: its tombstones become empty slots.
__global__ __launch_bounds__(kBlock) void k_purge_reopen(TableView t, const uint32_t* __restrict__ bits,
                                                         int64_t w0, int64_t w1) {
  const int64_t nslots = (w1 - w0) * kSlots;
  for (int64_t j = (int64_t)blockIdx.x * kBlock + threadIdx.x; j < nslots;
       j += (int64_t)gridDim.x * kBlock) {
    const uint64_t r = (uint64_t)(j >> 3);
    if ((bits[r >> 5] >> (r & 31)) & 1u) continue;
    uint64_t* k = &t.bk[(uint64_t)w0 + r].s[j & 7].key;
    if (*k == kTomb) *k = kEmpty;
  }
}

// ---------------------------------------------------------------------------------------------
// pool kernels
// ---------------------------------------------------------------------------------------------
__global__ __launch_bounds__(kBlock) void k_pool_init(PoolHeader* ph, int32_t* stack, int64_t cap) {
  const int64_t tid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t nt = (int64_t)gridDim.x * blockDim.x;
  for (int64_t j = tid; j < cap; j += nt) stack[j] = (int32_t)(cap - 1 - j);
  if (tid == 0) {
    ph->top = cap;
    ph->top0 = cap;
    ph->cap = cap;
    ph->err = 0;
    ph->head = 0;
    ph->head0 = 0;
  }
}

__global__ void k_pool_snapshot(PoolHeader* ph) {
  ph->top0 = ph->top;
  ph->head0 = ph->head;
}

__global__ __launch_bounds__(kBlock) void k_pool_pop(PoolHeader* ph, const int32_t* __restrict__ stack,
                                                     int64_t n, int32_t* __restrict__ out,
                                                     uint8_t* __restrict__ status) {
  const int64_t tid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t nt = (int64_t)gridDim.x * blockDim.x;
  const int64_t top0 = ph->top0, head0 = ph->head0, cap = ph->cap;
  for (int64_t i = tid; i < n; i += nt) {
    const bool ok = i < top0;
    if (out) out[i] = ok ? stack[ring_pos(head0, cap, top0 - 1 - i)] : -1;
    if (status) status[i] = ok ? 1 : 2;
  }
  if (tid == 0) {
    ph->top = n < top0 ? top0 - n : 0;
    if (n > top0) ph->err |= kErrPool;
  }
}

__global__ __launch_bounds__(kBlock) void k_pool_push(PoolHeader* ph, int32_t* __restrict__ stack,
                                                      const int32_t* __restrict__ in, int64_t n,
                                                      uint8_t* __restrict__ status) {
  const int64_t tid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t nt = (int64_t)gridDim.x * blockDim.x;
  const int64_t top0 = ph->top0, head0 = ph->head0, cap = ph->cap;
  for (int64_t i = tid; i < n; i += nt) {
    const bool ok = top0 + i < cap;
    if (ok) stack[ring_pos(head0, cap, top0 + i)] = in[i];
    if (status) status[i] = ok ? 1 : 2;
  }
  if (tid == 0) {
    ph->top = (top0 + n < cap) ? top0 + n : cap;
    if (top0 + n > cap) ph->err |= kErrPool;
  }
}

__global__ __launch_bounds__(kBlock) void k_pool_copy(const PoolHeader* ph, const int32_t* __restrict__ stack,
                                                      int32_t* __restrict__ out, int64_t cap) {
  const int64_t tid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t nt = (int64_t)gridDim.x * blockDim.x;
  const int64_t m = ph->top < cap ? ph->top : cap;
  for (int64_t j = tid; j < m; j += nt) out[j] = stack[ring_pos(ph->head, ph->cap, j)];
}

// Deque front operations (Section 4.3).  pop_front: element i of the batch removes pool element i
// (front first), -1 once the pool is empty.  push_front: element i goes just in front of the
// previous one, so the last value pushed ends up first.
__global__ __launch_bounds__(kBlock) void k_pool_pop_front(PoolHeader* ph, const int32_t* __restrict__ stack,
                                                           int64_t n, int32_t* __restrict__ out,
                                                           uint8_t* __restrict__ status) {
  const int64_t tid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t nt = (int64_t)gridDim.x * blockDim.x;
  const int64_t top0 = ph->top0, head0 = ph->head0, cap = ph->cap;
  for (int64_t i = tid; i < n; i += nt) {
    const bool ok = i < top0;
    if (out) out[i] = ok ? stack[ring_pos(head0, cap, i)] : -1;
    if (status) status[i] = ok ? 1 : 2;
  }
  if (tid == 0) {
    const int64_t m = n < top0 ? n : top0;
    ph->head = m ? ring_pos(head0, cap, m) : head0;
    ph->top = top0 - m;
    if (n > top0) ph->err |= kErrPool;
  }
}

__global__ __launch_bounds__(kBlock) void k_pool_push_front(PoolHeader* ph, int32_t* __restrict__ stack,
                                                            const int32_t* __restrict__ in, int64_t n,
                                                            uint8_t* __restrict__ status) {
  const int64_t tid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t nt = (int64_t)gridDim.x * blockDim.x;
  const int64_t top0 = ph->top0, head0 = ph->head0, cap = ph->cap;
  for (int64_t i = tid; i < n; i += nt) {
    const bool ok = top0 + i < cap;
    if (ok) stack[ring_pos(head0, cap, -1 - i)] = in[i];
    if (status) status[i] = ok ? 1 : 2;
  }
  if (tid == 0) {
    const int64_t room = cap - top0;
    const int64_t m = n < room ? n : room;
    ph->head = m ? ring_pos(head0, cap, -m) : head0;
    ph->top = top0 + m;
    if (n > room) ph->err |= kErrPool;
  }
}

// ---------------------------------------------------------------------------------------------
// grouped execution of a plan: one launch per pipeline stage covers the same stage of many
// tables.  A plan is cut into levels holding at most one chunk-step per table (the k-th step of
// every table); within a level the steps touch disjoint tables, scratch and arrays, so a stage's
// blocks of all steps can run in one grid.  Block b of a stage launch finds its step from the
// launch's entry list (first block of each step, ascending) and then runs exactly the range code
// of the single-table kernel with the step's own block index and block count.
// ---------------------------------------------------------------------------------------------
// Plan operation kinds (the CT_OP_* values).
enum : int32_t { kOpClear = 0, kOpInsert = 1, kOpFind = 2, kOpErase = 3 };

// Stages of the grouped pipeline, in launch order within a level.
enum GStage : int32_t {
  gReset, gPro, gDedup, gFind, gInsert, gErase, gApply,
  gSClear, gSBuild, gSProbe, gSSwap,  // resolution of speculative steps
  gCount, gScan, gFinal, gFix, gStages,
  gCopy = 100  // copy stage of merged operations (before the first and after the last level)
};

struct GStep {
  TableView v;
  const uint64_t* keys;
  const void* vals;
  void* vout;
  uint8_t* flags;
  int64_t q;      // elements of this step (at most the table's chunk for insert and erase)
  uint32_t db;    // dedup slots of the step's chunk
  int32_t vk;     // value kind of the table
  int32_t type;   // plan operation
  int32_t gb;     // blocks of the step's insert / erase / find stage
  int32_t ntiles; // rank-scan tiles
  int32_t spath;  // insert or erase: 0 resolve repeated keys first; 1 speculate when the table's
                  // last chunk of the kind changed at least half its keys; 2 speculate always
                  // (an insert only when it cannot reach capacity)
};

struct GEntry {
  int32_t first;  // first block of the step in this launch
  int32_t step;   // index into the step array
};

struct GLoc {
  int32_t step, lb, nblk;
};

// Step of block b of a launch of nb blocks: the last entry whose first block is <= b.  Uniform per
// block.
__device__ __forceinline__ GLoc g_locate_at(const GEntry* __restrict__ e, int32_t n, int32_t b,
                                            int32_t nb) {
  int32_t lo = 0, hi = n - 1;
  while (lo < hi) {
    const int32_t mid = (lo + hi + 1) >> 1;
    if (e[mid].first <= b) lo = mid;
    else hi = mid - 1;
  }
  const int32_t end = lo + 1 < n ? e[lo + 1].first : nb;
  return GLoc{e[lo].step, b - e[lo].first, end - e[lo].first};
}

__device__ __forceinline__ GLoc g_locate(const GEntry* __restrict__ e, int32_t n) {
  return g_locate_at(e, n, (int32_t)blockIdx.x, (int32_t)gridDim.x);
}

__device__ __forceinline__ void g_reset_body(const GStep* __restrict__ st, const GLoc L) {
  const TableView t = st[L.step].v;
  reset_range(t, (int64_t)L.lb * kBlock, (int64_t)t.nb * kSlots, (int64_t)L.nblk * kBlock,
              L.lb == 0, 0);
}

// Whether an insert or erase step speculates, decided on the device from the table's state when
// the step starts, so that a plan replayed later decides afresh.  Every block of the prologue
// stage computes it from words that no block of the stage writes, so all agree.
__device__ __forceinline__ bool g_speculates(const GStep& g) {
  if (g.spath == 0 || g.q <= 0 || (g.type != kOpInsert && g.type != kOpErase)) return false;
  const Header* h = g.v.hdr;
  const bool ins = g.type == kOpInsert;
  if (ins && h->size + (uint64_t)g.q > g.v.cap) return false;   // FULL must be ranked
  if (g.spath == 2) return true;
  const uint64_t f = h->fbd[ins ? 0 : 1];
  const uint64_t fq = f >> 32, changed = f & 0xFFFFFFFFull;
  return fq == 0 || 2 * changed >= fq;
}

// Prologue: a speculative step needs only its header snapshot and zeroed listed counts (the dd
// entries are cleared after the claims, and only when something is listed); otherwise the
// dedup scratch is cleared and the header decides as for a single-table chunk.
__device__ __forceinline__ void g_prologue_body(const GStep* __restrict__ st, const GLoc L) {
  const GStep& g = st[L.step];
  const TableView t = g.v;
  if (g_speculates(g)) {
    if (L.lb != 0) return;
    if (threadIdx.x < kListStripes) list_stripes(t)[threadIdx.x * kListStripeWords] = 0;
    if (threadIdx.x == 0) {
      Header* h = t.hdr;
      h->size0 = h->size;
      h->spec_first[0] = h->spec_first[1] = kNone;
      h->ndup = 0;
      h->nnew = 0;
      h->fast = 1u;
      h->spec = 1u;
      h->dmode = 0u;
    }
    return;
  }
  prologue_range(t, nullptr, g.db, g.q, (int64_t)L.lb * kBlock, prologue_units(g.db, g.q),
                 (int64_t)L.nblk * kBlock, L.lb == 0);
}

__device__ __forceinline__ void g_dedup_body(const GStep* __restrict__ st, const GLoc L) {
  const GStep& g = st[L.step];
  const TableView t = g.v;
  if (t.hdr->spec) return;
  dedup_range(t, g.keys, nullptr, g.db - 1, (int64_t)L.lb * kBlock, g.q, (int64_t)L.nblk * kBlock);
}

// Block totals of a speculative insert or erase: the count change into the block's partial, the
// listed elements onto one of the listed-count stripes.
template <int BS>
__device__ __forceinline__ void g_spec_counts(const TableView& t, uint2 c, int32_t lb, bool erase) {
  const int64_t tot = block_sum<BS>((int64_t)c.x + ((int64_t)c.y << 32));
  if (threadIdx.x == 0) {
    const int64_t changed = tot & 0xFFFFFFFFll;
    t.bcnt[lb] = erase ? -changed : changed;
    const uint32_t nl = (uint32_t)(tot >> 32);
    if (nl) aadd32(&list_stripes(t)[(lb % kListStripes) * kListStripeWords], nl);
  }
}

// The grouped find / insert / erase stages run with BS threads per block (the plan's block size):
// the range code strides by the step's blocks times BS, 8 lanes per key group as always.
template <int BS>
__device__ __forceinline__ void g_insert_body(const GStep* __restrict__ st, const GLoc L) {
  const GStep& g = st[L.step];
  const TableView t = g.v;
  const int64_t lo = (int64_t)L.lb * BS, step = (int64_t)L.nblk * BS;
  if (t.hdr->spec) {
    uint2 c;
    if (g.vk == 1) c = insert_spec_range<1>(t, g.keys, g.vals, g.flags, lo, g.q, step);
    else if (g.vk == 2) c = insert_spec_range<2>(t, g.keys, g.vals, g.flags, lo, g.q, step);
    else c = insert_spec_range<0>(t, g.keys, nullptr, g.flags, lo, g.q, step);
    g_spec_counts<BS>(t, c, L.lb, false);
    return;
  }
  int64_t ins;
  if (g.vk == 1)
    ins = insert_range<1, false>(t, g.keys, nullptr, g.vals, g.db - 1, g.flags, nullptr, lo, g.q, step);
  else if (g.vk == 2)
    ins = insert_range<2, false>(t, g.keys, nullptr, g.vals, g.db - 1, g.flags, nullptr, lo, g.q, step);
  else
    ins = insert_range<0, false>(t, g.keys, nullptr, nullptr, g.db - 1, g.flags, nullptr, lo, g.q, step);
  const int64_t tot = block_sum<BS>(ins);
  if (threadIdx.x == 0) t.bcnt[L.lb] = tot;
}

template <int BS>
__device__ __forceinline__ void g_erase_body(const GStep* __restrict__ st, const GLoc L) {
  const GStep& g = st[L.step];
  const TableView t = g.v;
  if (t.hdr->spec) {
    const uint2 c = erase_spec_range(t, g.keys, g.flags, (int64_t)L.lb * BS, g.q,
                                     (int64_t)L.nblk * BS);
    g_spec_counts<BS>(t, c, L.lb, true);
    return;
  }
  const int64_t del = erase_range<false>(t, g.keys, g.db - 1, g.flags, (int64_t)L.lb * BS,
                                         g.q, (int64_t)L.nblk * BS);
  const int64_t tot = block_sum<BS>(del);
  if (threadIdx.x == 0) t.bcnt[L.lb] = -tot;
}

template <int BS>
__device__ __forceinline__ void g_find_body(const GStep* __restrict__ st, const GLoc L) {
  const GStep& g = st[L.step];
  const TableView t = g.v;
  const int64_t lo = (int64_t)L.lb * BS, step = (int64_t)L.nblk * BS;
  if (g.vk == 1) find_range<1>(t, g.keys, g.vout, g.flags, lo, g.q, step);
  else if (g.vk == 2) find_range<2>(t, g.keys, g.vout, g.flags, lo, g.q, step);
  else find_range<0>(t, g.keys, nullptr, g.flags, lo, g.q, step);
}

// The count change into the live count and the feedback words; for a speculative step also the
// listed total, which the resolution stages read.
__device__ __forceinline__ void g_apply_body(const GStep* __restrict__ st, const GLoc L) {
  const GStep& g = st[L.step];
  const TableView t = g.v;
  const int64_t change = apply_count_block(t, g.gb);
  if (threadIdx.x == 0) {
    const bool erase = g.type == kOpErase;
    chunk_feedback(t, erase ? 1 : 0, g.q, erase ? -change : change);
    if (t.hdr->spec) t.hdr->ndup = listed_total(t);
  }
}

// Resolution of a speculative step (the single-table kernels' range code, per step).
__device__ __forceinline__ void g_sclear_body(const GStep* __restrict__ st, const GLoc L) {
  const GStep& g = st[L.step];
  if (!g.v.hdr->spec) return;
  spec_clear_range(g.v, g.q, L.lb, L.nblk);
}

__device__ __forceinline__ void g_sbuild_body(const GStep* __restrict__ st, const GLoc L) {
  const GStep& g = st[L.step];
  if (!g.v.hdr->spec) return;
  spec_build_range(g.v, g.keys, g.q, L.lb, L.nblk);
}

template <bool SWAP>
__device__ __forceinline__ void g_sfix_body(const GStep* __restrict__ st, const GLoc L) {
  const GStep& g = st[L.step];
  const TableView t = g.v;
  if (!t.hdr->spec) return;
  if (g.type == kOpErase) {
    if (SWAP) spec_swap_range<0, true>(t, g.keys, nullptr, g.q, g.flags, L.lb, L.nblk);
    else spec_probe_range<0, true>(t, g.keys, nullptr, g.q, g.flags, L.lb, L.nblk);
  } else if (g.vk == 1) {
    if (SWAP) spec_swap_range<1, false>(t, g.keys, g.vals, g.q, g.flags, L.lb, L.nblk);
    else spec_probe_range<1, false>(t, g.keys, g.vals, g.q, g.flags, L.lb, L.nblk);
  } else if (g.vk == 2) {
    if (SWAP) spec_swap_range<2, false>(t, g.keys, g.vals, g.q, g.flags, L.lb, L.nblk);
    else spec_probe_range<2, false>(t, g.keys, g.vals, g.q, g.flags, L.lb, L.nblk);
  } else {
    if (SWAP) spec_swap_range<0, false>(t, g.keys, nullptr, g.q, g.flags, L.lb, L.nblk);
    else spec_probe_range<0, false>(t, g.keys, nullptr, g.q, g.flags, L.lb, L.nblk);
  }
}

__device__ __forceinline__ void g_tile_count_body(const GStep* __restrict__ st, const GLoc L) {
  const GStep& g = st[L.step];
  const TableView t = g.v;
  if (t.hdr->fast) return;
  __shared__ uint32_t part[kBlock / 64];
  const int64_t t0 = (int64_t)L.lb * kTile;
  uint64_t c = 0;
  for (int j = threadIdx.x; j < kTile; j += kBlock) {
    const int64_t i = t0 + j;
    if (i < g.q) c += t.flag[i];
  }
  c = wave_sum(c);
  if (wave_lane() == 0) part[threadIdx.x >> 6] = (uint32_t)c;
  __syncthreads();
  if (threadIdx.x == 0) {
    uint32_t sum = 0;
    for (int w = 0; w < kBlock / 64; ++w) sum += part[w];
    t.tsum[L.lb] = sum;
  }
}

template <int NT>
__device__ __forceinline__ void g_tile_scan_body(const GStep* __restrict__ st, const GLoc L) {
  const TableView t = st[L.step].v;
  if (t.hdr->fast) return;
  scan_tiles_block<NT>(t, nullptr, st[L.step].ntiles, 0);
}

__device__ __forceinline__ void g_final_body(const GStep* __restrict__ st, const GLoc L) {
  const GStep& g = st[L.step];
  const TableView t = g.v;
  if (t.hdr->fast) return;   // nothing to rank: leave before any of the tile code
  if (g.vk == 1)
    final_tile<1, 0>(t, nullptr, nullptr, g.keys, g.vals, g.q, g.flags, nullptr, L.lb, 0);
  else if (g.vk == 2)
    final_tile<2, 0>(t, nullptr, nullptr, g.keys, g.vals, g.q, g.flags, nullptr, L.lb, 0);
  else
    final_tile<0, 0>(t, nullptr, nullptr, g.keys, nullptr, g.q, g.flags, nullptr, L.lb, 0);
}

// A byte range moved by the grouped plan's copy stages (operations merged into one step).
struct GCopy {
  const void* src;
  void* dst;
  int64_t bytes;
};

// Segment of this block's entry, copied by the entry's blocks in the widest aligned unit.
__device__ __forceinline__ void g_copy_body(const GCopy* __restrict__ segs, const GLoc L) {
  const GCopy g = segs[L.step];
  const uintptr_t a = reinterpret_cast<uintptr_t>(g.src) | reinterpret_cast<uintptr_t>(g.dst) |
                      (uintptr_t)g.bytes;
  const int64_t first = (int64_t)L.lb * kBlock + threadIdx.x;
  const int64_t stride = (int64_t)L.nblk * kBlock;
  if ((a & 15) == 0) {
    const uint4* s = static_cast<const uint4*>(g.src);
    uint4* d = static_cast<uint4*>(g.dst);
    for (int64_t i = first; i < g.bytes / 16; i += stride) d[i] = s[i];
  } else if ((a & 7) == 0) {
    const uint64_t* s = static_cast<const uint64_t*>(g.src);
    uint64_t* d = static_cast<uint64_t*>(g.dst);
    for (int64_t i = first; i < g.bytes / 8; i += stride) d[i] = s[i];
  } else {
    const uint8_t* s = static_cast<const uint8_t*>(g.src);
    uint8_t* d = static_cast<uint8_t*>(g.dst);
    for (int64_t i = first; i < g.bytes; i += stride) d[i] = s[i];
  }
}

__device__ __forceinline__ void g_fix_body(const GStep* __restrict__ st, const GLoc L) {
  const GStep& g = st[L.step];
  const TableView t = g.v;
  if (t.hdr->spec) return;   // (ndup counts listed elements there, not repeated keys)
  fix_range(t, g.flags, nullptr, (int64_t)L.lb * kBlock, (int64_t)L.nblk * kBlock);
}

// One launch per stage: block b of the launch runs the stage's body for its own step.
__global__ __launch_bounds__(kBlock) void k_g_reset(const GStep* __restrict__ st,
                                                    const GEntry* __restrict__ e, int32_t n) {
  g_reset_body(st, g_locate(e, n));
}
__global__ __launch_bounds__(kBlock) void k_g_prologue(const GStep* __restrict__ st,
                                                       const GEntry* __restrict__ e, int32_t n) {
  g_prologue_body(st, g_locate(e, n));
}
__global__ __launch_bounds__(kBlock) void k_g_dedup(const GStep* __restrict__ st,
                                                    const GEntry* __restrict__ e, int32_t n) {
  g_dedup_body(st, g_locate(e, n));
}
template <int BS>
__global__ __launch_bounds__(BS) void k_g_insert(const GStep* __restrict__ st,
                                                 const GEntry* __restrict__ e, int32_t n) {
  g_insert_body<BS>(st, g_locate(e, n));
}
template <int BS>
__global__ __launch_bounds__(BS) void k_g_erase(const GStep* __restrict__ st,
                                                const GEntry* __restrict__ e, int32_t n) {
  g_erase_body<BS>(st, g_locate(e, n));
}
template <int BS>
__global__ __launch_bounds__(BS) void k_g_find(const GStep* __restrict__ st,
                                               const GEntry* __restrict__ e, int32_t n) {
  g_find_body<BS>(st, g_locate(e, n));
}
__global__ __launch_bounds__(1024) void k_g_apply(const GStep* __restrict__ st,
                                                  const GEntry* __restrict__ e, int32_t n) {
  g_apply_body(st, g_locate(e, n));
}
__global__ __launch_bounds__(kBlock) void k_g_tile_count(const GStep* __restrict__ st,
                                                         const GEntry* __restrict__ e, int32_t n) {
  g_tile_count_body(st, g_locate(e, n));
}
__global__ __launch_bounds__(1024) void k_g_tile_scan(const GStep* __restrict__ st,
                                                      const GEntry* __restrict__ e, int32_t n) {
  g_tile_scan_body<1024>(st, g_locate(e, n));
}
__global__ __launch_bounds__(kBlock) void k_g_final(const GStep* __restrict__ st,
                                                    const GEntry* __restrict__ e, int32_t n) {
  g_final_body(st, g_locate(e, n));
}
__global__ __launch_bounds__(kBlock) void k_g_copy(const GCopy* __restrict__ segs,
                                                   const GEntry* __restrict__ e, int32_t n) {
  g_copy_body(segs, g_locate(e, n));
}
__global__ __launch_bounds__(kBlock) void k_g_fix(const GStep* __restrict__ st,
                                                  const GEntry* __restrict__ e, int32_t n) {
  g_fix_body(st, g_locate(e, n));
}
__global__ __launch_bounds__(kBlock) void k_g_sclear(const GStep* __restrict__ st,
                                                     const GEntry* __restrict__ e, int32_t n) {
  g_sclear_body(st, g_locate(e, n));
}
__global__ __launch_bounds__(kBlock) void k_g_sbuild(const GStep* __restrict__ st,
                                                     const GEntry* __restrict__ e, int32_t n) {
  g_sbuild_body(st, g_locate(e, n));
}
template <bool SWAP>
__global__ __launch_bounds__(kBlock) void k_g_sfix(const GStep* __restrict__ st,
                                                   const GEntry* __restrict__ e, int32_t n) {
  g_sfix_body<SWAP>(st, g_locate(e, n));
}

// The whole grouped schedule in one cooperative launch.  Every workgroup of the grid is resident
// at once (the runtime refuses a cooperative launch that cannot be), so a grid-wide barrier
// between stages cannot wait for a workgroup that never runs.  Stage by stage, the grid's blocks
// take the stage's blocks in turn (block b runs b, b + grid, ...) with the same bodies as the
// per-stage launches, 256 threads each, then meet at the barrier, whose device-scope fences make
// the stage's stores visible to every XCD before the next stage reads them.  No workgroup waits
// for another in any other way, and every workgroup reaches every barrier.
struct GLaunchDev {
  int32_t stage, n, blocks, pad;
  int64_t entry_off;
};

__global__ __launch_bounds__(kBlock) void k_g_persistent(const GLaunchDev* __restrict__ ls,
                                                         int32_t nl, const GStep* __restrict__ st,
                                                         const GEntry* __restrict__ en,
                                                         const GCopy* __restrict__ cp) {
  cooperative_groups::grid_group grid = cooperative_groups::this_grid();
  for (int32_t l = 0; l < nl; ++l) {
    const GLaunchDev L = ls[l];
    const GEntry* e = en + L.entry_off;
    for (int32_t b = (int32_t)blockIdx.x; b < L.blocks; b += (int32_t)gridDim.x) {
      const GLoc g = g_locate_at(e, L.n, b, L.blocks);
      switch (L.stage) {
        case gReset: g_reset_body(st, g); break;
        case gPro: g_prologue_body(st, g); break;
        case gDedup: g_dedup_body(st, g); break;
        case gFind: g_find_body<kBlock>(st, g); break;
        case gInsert: g_insert_body<kBlock>(st, g); break;
        case gErase: g_erase_body<kBlock>(st, g); break;
        case gApply: g_apply_body(st, g); break;
        case gCount: g_tile_count_body(st, g); break;
        case gScan: g_tile_scan_body<kBlock>(st, g); break;
        case gFinal: g_final_body(st, g); break;
        case gFix: g_fix_body(st, g); break;
        case gSClear: g_sclear_body(st, g); break;
        case gSBuild: g_sbuild_body(st, g); break;
        case gSProbe: g_sfix_body<false>(st, g); break;
        case gSSwap: g_sfix_body<true>(st, g); break;
        case gCopy: g_copy_body(cp, g); break;
        default: break;
      }
      __syncthreads();  // the next block's body reuses this workgroup's LDS
    }
    grid.sync();
  }
}

}  // namespace

// =============================================================================================
// host side
// =============================================================================================
// Per-table kernel timing: while enabled, each kernel launched for the table is bracketed by two
// HIP events recorded on the caller's stream; read-out waits for them and sums per kernel kind.
struct Profiler {
  bool on = false;
  std::vector<hipEvent_t> events;  // pairs (start, end)
  std::vector<int> kinds;          // kind of each recorded pair
  size_t used = 0;
  double total_ms[CT_KERNEL_KINDS] = {};
  int64_t launches[CT_KERNEL_KINDS] = {};
};

struct ct_table {
  Profiler prof;
  ct_table_desc desc;
  uint8_t* base;
  int64_t bytes;
  TableView v;
  int64_t chunk;      // Q: elements per chunk (power of two)
  uint64_t size_ub;   // upper bound of the live count known to the host
  int64_t dd_bytes;   // bytes of the dedup scratch region at v.dd (the purge's bitmap)
  int32_t insert_path = CT_INSERT_AUTO;  // how insert chunks resolve repeated keys
  uint64_t* fb_host = nullptr;           // host side of v.fb (pinned, mapped), or null
};

struct ct_pool {
  uint8_t* base;
  int64_t cap;
  PoolHeader* hdr;
  int32_t* stack;
};

namespace {

constexpr int64_t kAlign = 256;

int64_t align_up(int64_t x) { return (x + kAlign - 1) / kAlign * kAlign; }

bool is_prime(int64_t x) {
  if (x < 2) return false;
  if (x % 2 == 0) return x == 2;
  for (int64_t d = 3; d * d <= x; d += 2)
    if (x % d == 0) return false;
  return true;
}

// Smallest prime >= x (x >= 1); a prime bucket count lets every probe step visit all buckets.
int64_t next_prime(int64_t x) {
  if (x <= 2) return 2;
  while (!is_prime(x)) ++x;
  return x;
}

int64_t pow2ceil(int64_t x) {
  int64_t p = 1;
  while (p < x) p <<= 1;
  return p;
}

struct Layout {
  int64_t nb, chunk, dslots, ntiles;
  int64_t off_bk, off_dd, off_dmark, off_dup, off_flag, off_ref, off_tsum, off_bcnt, total;
  // binned dedup (chunk >= kBinMinChunk; otherwise bins == false and the offsets are unused)
  bool bins;
  int64_t nfine, c1, c2;
  int lp, lp1;
  int64_t off_r1k, off_r1i, off_r2k, off_r2i, off_bcur, off_dfirst;
};

static_assert(kBinFineCap % kBlock == 0, "fine-bin entries are held kBlock per register row");

bool make_layout(const ct_table_desc* d, Layout* L) {
  if (!d || d->capacity < 0) return false;
  if (d->val_kind < 0 || d->val_kind > 2 || d->hash_kind < 0 || d->hash_kind > 1) return false;
  int64_t nb = d->bucket_count;
  if (nb == 0) nb = next_prime(std::max<int64_t>(1, (d->capacity + kSlots - 1) / kSlots));
  if (nb < 1) nb = 1;
  if (nb >= ((int64_t)1 << 31)) return false;  // 32-bit bucket arithmetic in the probes
  if (nb * kSlots < d->capacity) return false;
  int64_t q = d->chunk;
  if (q == 0) {
    // one chunk per ~capacity/8 keys: long kernels amortise launch and drain, and the scratch
    // (about 82 bytes per chunk element at these sizes) stays below two thirds of the buckets'
    // 16 bytes per slot
    int64_t f = 1024;
    while (f * 2 <= d->capacity / 8 && f < ((int64_t)1 << 23)) f *= 2;
    q = f;
  }
  if (q < 1024 || q > ((int64_t)1 << 24) || (q & (q - 1))) return false;
  L->nb = nb;
  L->chunk = q;
  L->dslots = 2 * q;
  L->ntiles = (q + kTile - 1) / kTile;
  int64_t off = align_up((int64_t)sizeof(Header));
  L->off_bk = off;
  off = align_up(off + nb * (int64_t)sizeof(Bucket));
  L->bins = q >= kBinMinChunk;
  if (L->bins) {
    L->nfine = q / kBinFine;
    L->lp = 0;
    while (((int64_t)1 << L->lp) < L->nfine) ++L->lp;
    L->lp1 = 0;
    while ((1 << L->lp1) < kBinCoarse) ++L->lp1;
    const int64_t nseg = (int64_t)kBinCoarse * kBinSub;
    L->c1 = 2 * (q / nseg) + 256;
    L->c2 = kBinFineCap;
    if (L->nfine / kBinCoarse > kMaxFinePerCoarse) return false;
    if (nseg * L->c1 < L->dslots) return false;  // dd (8 bytes per slot) must fit in r1k
    L->off_r1k = off;
    L->off_dd = off;
    off = align_up(off + nseg * L->c1 * 8);
    L->off_r1i = off;
    off = align_up(off + nseg * L->c1 * 4);
    L->off_r2k = off;
    off = align_up(off + L->nfine * L->c2 * 8);
    L->off_r2i = off;
    off = align_up(off + L->nfine * L->c2 * 4);
    L->off_bcur = off;
    off = align_up(off + (kCoarseCtrWords + L->nfine) * 4);
    L->off_dfirst = off;
    off = align_up(off + q * 4);
  } else {
    L->off_dd = off;
    off = align_up(off + L->dslots * 8);
  }
  L->off_dmark = off;
  off = align_up(off + q);
  L->off_dup = off;
  off = align_up(off + q * (int64_t)sizeof(uint2));
  L->off_flag = off;
  off = align_up(off + q);
  L->off_ref = off;
  off = align_up(off + q * 8);
  L->off_tsum = off;
  off = align_up(off + L->ntiles * 4);
  L->off_bcnt = off;
  off = align_up(off + kMaxGroupBlocks * 8 + kStripeRegion);
  L->total = off;
  return true;
}

inline hipStream_t S(void* s) { return reinterpret_cast<hipStream_t>(s); }

// Sum the recorded pairs into the per-kind totals (waits for the last recorded event).
ct_status prof_drain(Profiler& P) {
  ct_status r = CT_OK;
  for (size_t j = 0; j < P.kinds.size(); ++j) {
    float ms = 0.f;
    if (hipEventSynchronize(P.events[2 * j + 1]) != hipSuccess ||
        hipEventElapsedTime(&ms, P.events[2 * j], P.events[2 * j + 1]) != hipSuccess) {
      r = CT_E_HIP;
      continue;
    }
    P.total_ms[P.kinds[j]] += ms;
    P.launches[P.kinds[j]] += 1;
  }
  P.kinds.clear();
  P.used = 0;
  return r;
}

// Launch `f` (a kernel launch on stream s) for table t, timed when profiling is on.
template <typename F>
void launch(ct_table* t, int kind, hipStream_t s, F&& f) {
  hipEvent_t end = nullptr;
  if (t && t->prof.on) {
    Profiler& P = t->prof;
    if (P.used + 2 > P.events.size()) prof_drain(P);
    if (hipEventRecord(P.events[P.used], s) == hipSuccess) {  // else this launch goes untimed
      end = P.events[P.used + 1];
      P.kinds.push_back(kind);
      P.used += 2;
    }
  }
  f();
  if (end && hipEventRecord(end, s) != hipSuccess) {  // drop the half-recorded pair
    t->prof.kinds.pop_back();
    t->prof.used -= 2;
  }
}

int64_t bin_prologue_units_host(const TableView& v, int64_t q) {
  return (q + 15) / 16 + ((int64_t)kCoarseCtrWords + ((int64_t)1 << v.lp)) / 4;
}

// Blocks of `bs` threads for n key groups of 8 lanes (at most kMaxGroupBlocks: the count
// partials of one launch).
int group_blocks(int64_t n, int bs = kBlock) {
  const int64_t b = (n + (bs / 8) - 1) / (bs / 8);
  return (int)std::max<int64_t>(1, std::min<int64_t>(b, kMaxGroupBlocks));
}

// Chunks of at most this many rank tiles skip the one-block rank scan: each ranked-completion
// block sums the tile counts before its own tile (at most 256 loads), and the first settles the
// chunk's totals.
constexpr int kInlineRankTiles = 256;

int flat_blocks(int64_t n) {
  const int64_t b = (n + kBlock - 1) / kBlock;
  return (int)std::max<int64_t>(1, std::min<int64_t>(b, 8192));
}

ct_status launched() { return hipGetLastError() == hipSuccess ? CT_OK : CT_E_HIP; }

// dedup entries for a chunk of q elements: a power of two >= 2q (load at most one half)
uint32_t dedup_slots_for(int64_t q) { return (uint32_t)std::max<int64_t>(2, pow2ceil(2 * q)); }

template <typename T>
ct_status read_back(const T* dev, T* host, hipStream_t s) {
  if (hipMemcpyAsync(host, dev, sizeof(T), hipMemcpyDeviceToHost, s) != hipSuccess) return CT_E_HIP;
  return hipStreamSynchronize(s) == hipSuccess ? CT_OK : CT_E_HIP;
}

// ---------------------------------------------------------------------------------------------
// insert / erase drivers
// ---------------------------------------------------------------------------------------------
// Resolve the repeated keys of one chunk: binned for large chunks, dd otherwise.
void dedup_chunk(ct_table* t, const TableView& v, PoolHeader* pool, const uint64_t* kc, int64_t q,
                 hipStream_t s) {
  const uint32_t db = dedup_slots_for(q);
  if (v.r1k && q >= kBinMinChunk) {
    // blocks per coarse segment: enough for its expected fill (about c1 / 2) in one tile each
    const int blocks_per_seg = (int)std::max<int64_t>(1, (v.c1 / 2 + kBinTile - 1) / kBinTile);
    const int nfine = 1 << v.lp;
    launch(t, CT_KERNEL_PROLOGUE, s, [&] { k_bin_prologue<<<flat_blocks(bin_prologue_units_host(v, q)), kBlock, 0, s>>>(v, pool, q); });
    launch(t, CT_KERNEL_DEDUP, s, [&] { k_bin_scatter1<<<(int)((q + kBinTile - 1) / kBinTile), kBlock, 0, s>>>(v, kc, q); });
    launch(t, CT_KERNEL_DEDUP, s, [&] { k_bin_scatter2<<<kBinCoarse * kBinSub * blocks_per_seg, kBlock, 0, s>>>(v, blocks_per_seg); });
    launch(t, CT_KERNEL_DEDUP, s, [&] { k_bin_dedup<<<nfine, kBlock, 0, s>>>(v); });
    launch(t, CT_KERNEL_DEDUP, s, [&] { k_bin_fallback_clear<<<flat_blocks(db / 2), kBlock, 0, s>>>(v, db); });
    launch(t, CT_KERNEL_DEDUP, s, [&] { k_bin_fallback_dedup<<<flat_blocks(q), kBlock, 0, s>>>(v, kc, q, db - 1); });
  } else {
    launch(t, CT_KERNEL_PROLOGUE, s, [&] { k_prologue<<<flat_blocks(db / 2), kBlock, 0, s>>>(v, pool, db, q, 0); });
    launch(t, CT_KERNEL_DEDUP, s, [&] { k_dedup<<<flat_blocks(q), kBlock, 0, s>>>(v, kc, nullptr, q, db - 1); });
  }
}

// Whether a chunk that cannot reach capacity is inserted speculatively.  AUTO follows the
// table's last insert chunk (reported through the mapped feedback word, possibly stale): keys
// mostly new -> speculative; mostly present or repeated -> repeated keys resolved first, where
// only one copy of each key probes the table.
bool use_speculation(const ct_table* t, int word) {
  if (t->insert_path == CT_INSERT_RESOLVE_FIRST) return false;
  if (t->insert_path == CT_INSERT_SPECULATIVE || !t->fb_host) return true;
  const uint64_t f = __atomic_load_n(t->fb_host + word, __ATOMIC_RELAXED);
  const uint64_t fq = f >> 32, changed = f & 0xFFFFFFFFull;
  return fq == 0 || 2 * changed >= fq;
}

// The resolution kernels of a speculative chunk (after its insert or erase kernel).
// The resolution kernels stride over their elements with at most kSpecGrid blocks: they read one
// header word and leave when nothing is listed, and a small grid keeps that cheap.
constexpr int kSpecGrid = 1024;

template <int VK, bool ERASE>
void spec_resolve(ct_table* t, const TableView& v, const uint64_t* kc, const void* vc, int64_t q,
                  uint8_t* sc, int gb, uint32_t db, hipStream_t s) {
  const int g = std::min(flat_blocks(q), kSpecGrid);
  launch(t, CT_KERNEL_APPLY, s, [&] { k_spec_sum<<<1, 1024, 0, s>>>(v, gb, q, ERASE ? 1 : 0); });
  launch(t, CT_KERNEL_APPLY, s, [&] { k_spec_clear<<<std::min(flat_blocks(db / 2), kSpecGrid), kBlock, 0, s>>>(v, q); });
  launch(t, CT_KERNEL_DEDUP, s, [&] { k_spec_build<<<g, kBlock, 0, s>>>(v, kc, q); });
  launch(t, CT_KERNEL_FIX, s, [&] { k_spec_probe<VK, ERASE><<<g, kBlock, 0, s>>>(v, kc, vc, q, sc); });
  launch(t, CT_KERNEL_FIX, s, [&] { k_spec_swap<VK, ERASE><<<g, kBlock, 0, s>>>(v, kc, vc, q, sc); });
}

// Insert of n keys in chunks of at most `chunk`, with the per-chunk scratch that view `v` names
// (the table's own, or another region holding the same arrays).
template <int VK>
ct_status insert_chunks(ct_table* t, const TableView& v, int64_t chunk, const uint64_t* keys,
                        const void* vals, int64_t n, uint8_t* status, hipStream_t s) {
  const int vb = VK == 1 ? 4 : 8;
  for (int64_t c0 = 0; c0 < n; c0 += chunk) {
    const int64_t q = std::min<int64_t>(chunk, n - c0);
    const uint32_t db = dedup_slots_for(q);
    const uint64_t* kc = keys + c0;
    const void* vc = VK ? static_cast<const void*>(static_cast<const uint8_t*>(vals) + c0 * vb) : nullptr;
    uint8_t* sc = status ? status + c0 : nullptr;
    const int gb = group_blocks((q + kSlots - 1) / kSlots);
    const int ntiles = (int)((q + kTile - 1) / kTile);
    // the host bound proves that no element can meet FULL: the rank pass is not needed
    const bool surely_fast = t->size_ub + (uint64_t)q <= (uint64_t)t->desc.capacity;
    if (surely_fast && use_speculation(t, 0)) {
      // speculative: insert first, then resolve the copies of keys listed as ambiguous
      launch(t, CT_KERNEL_PROLOGUE, s, [&] { k_spec_prologue<<<1, 64, 0, s>>>(v, q, 1); });
      launch(t, CT_KERNEL_INSERT, s, [&] { k_insert_spec<VK><<<gb, kBlock, 0, s>>>(v, kc, vc, q, sc); });
      spec_resolve<VK, false>(t, v, kc, vc, q, sc, gb, db, s);
      t->size_ub = std::min<uint64_t>(t->size_ub + (uint64_t)q, (uint64_t)t->desc.capacity);
      ct_status r = launched();
      if (r != CT_OK) return r;
      continue;
    }
    dedup_chunk(t, v, nullptr, kc, q, s);
    launch(t, CT_KERNEL_INSERT, s, [&] { k_insert<VK, false><<<gb, kBlock, 0, s>>>(v, kc, vc, q, db - 1, sc, nullptr, nullptr, 0); });
    // a chunk that may meet capacity stores more keys in its ranked pass: no report
    launch(t, CT_KERNEL_APPLY, s, [&] { k_apply_count<<<1, 1024, 0, s>>>(v, gb, surely_fast ? q : 0, 0); });
    if (!surely_fast) {
      launch(t, CT_KERNEL_RANK, s, [&] { k_tile_count<<<ntiles, kBlock, 0, s>>>(v, q, 1); });
      const int inl = ntiles <= kInlineRankTiles ? ntiles : 0;
      if (!inl) launch(t, CT_KERNEL_RANK, s, [&] { k_tile_scan<<<1, 1024, 0, s>>>(v, nullptr, ntiles, 0); });
      launch(t, CT_KERNEL_FINAL, s, [&] { k_final<VK, 0><<<ntiles, kBlock, 0, s>>>(v, nullptr, nullptr, kc, vc, q, sc, nullptr, inl); });
    }
    if (sc) launch(t, CT_KERNEL_FIX, s, [&] { k_fix<<<flat_blocks(q), kBlock, 0, s>>>(v, sc, nullptr); });
    t->size_ub = std::min<uint64_t>(t->size_ub + (uint64_t)q, (uint64_t)t->desc.capacity);
    ct_status r = launched();
    if (r != CT_OK) return r;
  }
  return CT_OK;
}

template <int VK>
ct_status insert_chunks(ct_table* t, const uint64_t* keys, const void* vals, int64_t n,
                        uint8_t* status, hipStream_t s) {
  return insert_chunks<VK>(t, t->v, t->chunk, keys, vals, n, status, s);
}

template <bool RELEASE>
ct_status erase_chunks(ct_table* t, ct_pool* p, const uint64_t* keys, int64_t n, uint8_t* erased,
                       hipStream_t s) {
  for (int64_t c0 = 0; c0 < n; c0 += t->chunk) {
    const int64_t q = std::min<int64_t>(t->chunk, n - c0);
    const uint32_t db = dedup_slots_for(q);
    const uint64_t* kc = keys + c0;
    uint8_t* ec = erased ? erased + c0 : nullptr;
    const int gb = group_blocks((q + kSlots - 1) / kSlots);
    const int ntiles = (int)((q + kTile - 1) / kTile);
    if (!RELEASE && use_speculation(t, 1)) {
      // speculative: remove first, then move each removal to the lowest copy of its key
      launch(t, CT_KERNEL_PROLOGUE, s, [&] { k_spec_prologue<<<1, 64, 0, s>>>(t->v, q, 0); });
      launch(t, CT_KERNEL_ERASE, s, [&] { k_erase_spec<<<gb, kBlock, 0, s>>>(t->v, kc, q, ec); });
      spec_resolve<0, true>(t, t->v, kc, nullptr, q, ec, gb, db, s);
      ct_status r = launched();
      if (r != CT_OK) return r;
      continue;
    }
    dedup_chunk(t, t->v, RELEASE ? p->hdr : nullptr, kc, q, s);
    launch(t, CT_KERNEL_ERASE, s, [&] { k_erase<RELEASE><<<gb, kBlock, 0, s>>>(t->v, kc, q, db - 1, ec); });
    launch(t, CT_KERNEL_APPLY, s, [&] { k_apply_count<<<1, 1024, 0, s>>>(t->v, gb, RELEASE ? 0 : q, 1); });
    if (RELEASE) {
      launch(t, CT_KERNEL_RANK, s, [&] { k_tile_count<<<ntiles, kBlock, 0, s>>>(t->v, q, 0); });
      const int inl = ntiles <= kInlineRankTiles ? ntiles : 0;
      if (!inl) launch(t, CT_KERNEL_RANK, s, [&] { k_tile_scan<<<1, 1024, 0, s>>>(t->v, p->hdr, ntiles, 2); });
      launch(t, CT_KERNEL_FINAL, s, [&] { k_final<0, 2><<<ntiles, kBlock, 0, s>>>(t->v, p->hdr, p->stack, kc, nullptr, q, nullptr, nullptr, inl); });
    }
    ct_status r = launched();
    if (r != CT_OK) return r;
  }
  return CT_OK;
}

ct_status check_batch(const ct_table* t, const void* keys, int64_t n) {
  if (!t || n < 0) return CT_E_INVALID;
  if (n > 0 && !keys) return CT_E_INVALID;
  return CT_OK;
}

}  // namespace

namespace {
template <class Pred>
ct_status select_into(ct_table* t, const Pred& pred, uint64_t* keys_out, uint64_t* vals_out,
                      int64_t cap, int64_t* h_count, void* stream) {
  if (!t || !h_count || cap < 0 || (cap > 0 && !keys_out)) return CT_E_INVALID;
  if (t->desc.val_kind == CT_VAL_NONE) vals_out = nullptr;
  hipStream_t s = S(stream);
  const int64_t nslots = (int64_t)t->v.nb * kSlots;
  const int64_t rounds = (nslots + kSelRound - 1) / kSelRound;
  const int64_t g0 = std::max<int64_t>(1, std::min<int64_t>(rounds, kMaxGroupBlocks));
  const int64_t per = ((rounds + g0 - 1) / g0) * kSelRound;   // whole rounds per block
  const int grid = (int)((nslots + per - 1) / per);
  k_sel_count<Pred><<<grid, kBlock, 0, s>>>(t->v, pred, per);
  k_sel_scan<Pred><<<1, 1024, 0, s>>>(t->v, pred, grid);
  k_sel_write<Pred><<<grid, kBlock, 0, s>>>(t->v, pred, per, keys_out, vals_out, cap);
  if (launched() != CT_OK) return CT_E_HIP;
  uint64_t c = 0;
  ct_status r = read_back(&t->v.hdr->dump_count, &c, s);
  if (r != CT_OK) return r;
  *h_count = (int64_t)c;
  return CT_OK;
}
}  // namespace

extern "C" {

const char* ct_status_str(ct_status s) {
  switch (s) {
    case CT_OK: return "ok";
    case CT_E_INVALID: return "invalid argument";
    case CT_E_FULL: return "capacity exhausted";
    case CT_E_EMPTY: return "pool empty";
    case CT_E_NOMEM: return "host allocation failed";
    case CT_E_HIP: return "HIP runtime error";
  }
  return "unknown status";
}

ct_status ct_table_bytes(const ct_table_desc* d, int64_t* bytes) {
  Layout L;
  if (!bytes || !make_layout(d, &L)) return CT_E_INVALID;
  *bytes = L.total;
  return CT_OK;
}

ct_status ct_table_init(void* d_buf, int64_t bytes, const ct_table_desc* d, void* stream,
                        ct_table** out) {
  Layout L;
  if (!out || !d_buf || !make_layout(d, &L) || bytes < L.total) return CT_E_INVALID;
  if (reinterpret_cast<uintptr_t>(d_buf) % kAlign) return CT_E_INVALID;
  ct_table* t = new (std::nothrow) ct_table;
  if (!t) return CT_E_NOMEM;
  uint8_t* base = static_cast<uint8_t*>(d_buf);
  t->desc = *d;
  t->desc.bucket_count = L.nb;
  t->desc.chunk = L.chunk;
  t->base = base;
  t->bytes = bytes;
  t->chunk = L.chunk;
  t->size_ub = 0;
  t->dd_bytes = L.bins ? (int64_t)kBinCoarse * kBinSub * L.c1 * 8 : L.dslots * 8;
  TableView& v = t->v;
  v.hdr = reinterpret_cast<Header*>(base);
  v.bk = reinterpret_cast<Bucket*>(base + L.off_bk);
  v.nb = (uint64_t)L.nb;
  v.cap = (uint64_t)d->capacity;
  v.dd = reinterpret_cast<uint64_t*>(base + L.off_dd);
  v.dmark = base + L.off_dmark;
  v.dup = reinterpret_cast<uint2*>(base + L.off_dup);
  v.flag = base + L.off_flag;
  v.ref = reinterpret_cast<uint64_t*>(base + L.off_ref);
  v.tsum = reinterpret_cast<uint32_t*>(base + L.off_tsum);
  v.bcnt = reinterpret_cast<int64_t*>(base + L.off_bcnt);
  v.r1k = L.bins ? reinterpret_cast<uint64_t*>(base + L.off_r1k) : nullptr;
  v.r1i = L.bins ? reinterpret_cast<uint32_t*>(base + L.off_r1i) : nullptr;
  v.r2k = L.bins ? reinterpret_cast<uint64_t*>(base + L.off_r2k) : nullptr;
  v.r2i = L.bins ? reinterpret_cast<uint32_t*>(base + L.off_r2i) : nullptr;
  v.bcur = L.bins ? reinterpret_cast<uint32_t*>(base + L.off_bcur) : nullptr;
  v.dfirst = L.bins ? reinterpret_cast<uint32_t*>(base + L.off_dfirst) : nullptr;
  v.c1 = L.bins ? (uint32_t)L.c1 : 0u;
  v.c2 = L.bins ? (uint32_t)L.c2 : 0u;
  v.lp = L.bins ? L.lp : 0;
  v.lp1 = L.bins ? L.lp1 : 0;
  v.hash = d->hash_kind;
  v.nb_pow2 = (L.nb & (L.nb - 1)) == 0;
  v.step_mode = v.nb_pow2 ? 1 : (is_prime(L.nb) ? 2 : 0);
  // the insert-path feedback word; without it every provable chunk is speculative
  v.fb = nullptr;
  void* fbh = nullptr;
  if (hipHostMalloc(&fbh, 64, hipHostMallocMapped) == hipSuccess) {
    void* fbd = nullptr;
    if (hipHostGetDevicePointer(&fbd, fbh, 0) == hipSuccess) {
      t->fb_host = static_cast<uint64_t*>(fbh);
      *t->fb_host = 0;
      v.fb = static_cast<uint64_t*>(fbd);
    } else {
      (void)hipHostFree(fbh);
    }
  }
  (void)hipGetLastError();  // a failed pinned allocation only disables the feedback
  k_table_reset<<<flat_blocks(L.nb * kSlots), kBlock, 0, S(stream)>>>(v, 1);
  if (launched() != CT_OK) {
    if (t->fb_host) (void)hipHostFree(t->fb_host);
    delete t;
    return CT_E_HIP;
  }
  *out = t;
  return CT_OK;
}

ct_status ct_table_destroy(ct_table* t) {
  if (!t) return CT_E_INVALID;
  for (hipEvent_t e : t->prof.events) (void)hipEventDestroy(e);
  if (t->fb_host) (void)hipHostFree(t->fb_host);
  delete t;
  return CT_OK;
}

ct_status ct_table_set_profiling(ct_table* t, int enable) {
  if (!t) return CT_E_INVALID;
  Profiler& P = t->prof;
  if (enable && !P.on) {
    if (P.events.empty()) {
      P.events.resize(8192);
      for (hipEvent_t& e : P.events)
        if (hipEventCreate(&e) != hipSuccess) return CT_E_HIP;
    }
    P.on = true;
  } else if (!enable && P.on) {
    P.on = false;
    return prof_drain(P);
  }
  return CT_OK;
}

ct_status ct_table_profile(ct_table* t, int32_t kind, double* total_ms, int64_t* launches) {
  if (!t || kind < 0 || kind >= CT_KERNEL_KINDS) return CT_E_INVALID;
  ct_status r = prof_drain(t->prof);
  if (total_ms) *total_ms = t->prof.total_ms[kind];
  if (launches) *launches = t->prof.launches[kind];
  return r;
}

ct_status ct_table_profile_reset(ct_table* t) {
  if (!t) return CT_E_INVALID;
  ct_status r = prof_drain(t->prof);
  for (int k = 0; k < CT_KERNEL_KINDS; ++k) {
    t->prof.total_ms[k] = 0.0;
    t->prof.launches[k] = 0;
  }
  return r;
}

ct_status ct_table_info(const ct_table* t, int64_t* bucket_count, int64_t* chunk) {
  if (!t) return CT_E_INVALID;
  if (bucket_count) *bucket_count = (int64_t)t->v.nb;
  if (chunk) *chunk = t->chunk;
  return CT_OK;
}

ct_status ct_table_value_bytes(const ct_table* t, int32_t* bytes) {
  if (!t || !bytes) return CT_E_INVALID;
  *bytes = t->desc.val_kind == CT_VAL_U64 ? 8 : t->desc.val_kind == CT_VAL_U32 ? 4 : 0;
  return CT_OK;
}

ct_status ct_insert_batch(ct_table* t, const uint64_t* keys, const void* vals, int64_t n,
                          uint8_t* status, void* stream) {
  ct_status r = check_batch(t, keys, n);
  if (r != CT_OK) return r;
  if (n == 0) return CT_OK;
  const int vk = t->desc.val_kind;
  if (vk != CT_VAL_NONE && !vals) return CT_E_INVALID;
  if (vk == CT_VAL_U32) return insert_chunks<1>(t, keys, vals, n, status, S(stream));
  if (vk == CT_VAL_U64) return insert_chunks<2>(t, keys, vals, n, status, S(stream));
  return insert_chunks<0>(t, keys, nullptr, n, status, S(stream));
}

ct_status ct_find_batch(ct_table* t, const uint64_t* keys, int64_t n, void* vals_out,
                        uint8_t* found, void* stream) {
  ct_status r = check_batch(t, keys, n);
  if (r != CT_OK) return r;
  const int vk = t->desc.val_kind;
  if (vk == CT_VAL_NONE && vals_out) return CT_E_INVALID;
  if (n == 0) return CT_OK;
  const int gb = group_blocks((n + kSlots - 1) / kSlots);
  hipStream_t s = S(stream);
  launch(t, CT_KERNEL_FIND, s, [&] {
    if (vk == CT_VAL_U32) k_find<1><<<gb, kBlock, 0, s>>>(t->v, keys, n, vals_out, found);
    else if (vk == CT_VAL_U64) k_find<2><<<gb, kBlock, 0, s>>>(t->v, keys, n, vals_out, found);
    else k_find<0><<<gb, kBlock, 0, s>>>(t->v, keys, n, nullptr, found);
  });
  return launched();
}

ct_status ct_erase_batch(ct_table* t, const uint64_t* keys, int64_t n, uint8_t* erased,
                         void* stream) {
  ct_status r = check_batch(t, keys, n);
  if (r != CT_OK) return r;
  if (n == 0) return CT_OK;
  return erase_chunks<false>(t, nullptr, keys, n, erased, S(stream));
}

ct_status ct_size(ct_table* t, int64_t* h_size, void* stream) {
  if (!t || !h_size) return CT_E_INVALID;
  uint64_t v = 0;
  ct_status r = read_back(&t->v.hdr->size, &v, S(stream));
  if (r != CT_OK) return r;
  *h_size = (int64_t)v;
  t->size_ub = v;
  return CT_OK;
}

ct_status ct_clear(ct_table* t, void* stream) {
  if (!t) return CT_E_INVALID;
  launch(t, CT_KERNEL_CLEAR, S(stream), [&] { k_table_reset<<<flat_blocks((int64_t)t->v.nb * kSlots), kBlock, 0, S(stream)>>>(t->v, 0); });
  t->size_ub = 0;
  return launched();
}

ct_status ct_table_device_view(ct_table* t, int32_t mode, void* out, int64_t bytes) {
  if (!t || !out || bytes < (int64_t)sizeof(DevView) || mode < kDevRead || mode > kDevMixed)
    return CT_E_INVALID;
  DevView v{};
  v.t = t->v;
  v.mode = mode;
  std::memcpy(out, &v, sizeof(v));
  // device inserts grow the table behind the host's back
  if (mode == kDevInsert || mode == kDevMixed) t->size_ub = (uint64_t)t->desc.capacity;
  return CT_OK;
}

ct_status ct_dev_apply(ct_table* t, int32_t op, const uint64_t* keys, const void* vals, int64_t n,
                       void* vals_out, uint8_t* status, void* stream) {
  if (!t || n < 0 || (n > 0 && !keys)) return CT_E_INVALID;
  if (op != CT_OP_INSERT && op != CT_OP_FIND && op != CT_OP_ERASE) return CT_E_INVALID;
  const int32_t vk = t->desc.val_kind;
  if (op == CT_OP_INSERT && vk != CT_VAL_NONE && n > 0 && !vals) return CT_E_INVALID;
  if (n == 0) return CT_OK;
  DevView v{};
  v.t = t->v;
  v.mode = op == CT_OP_INSERT ? kDevInsert : op == CT_OP_ERASE ? kDevErase : kDevRead;
  if (op == CT_OP_INSERT)
    t->size_ub = std::min<uint64_t>(t->size_ub + (uint64_t)n, (uint64_t)t->desc.capacity);
  v.striped = op != CT_OP_FIND;
  if (v.striped) k_dev_prep<<<1, kStripes, 0, S(stream)>>>(t->v, op == CT_OP_INSERT ? (uint64_t)n : 0);
  k_dev_apply<<<flat_blocks(n), kBlock, 0, S(stream)>>>(v, op, keys, vals, vk, n, vals_out, status);
  if (v.striped) k_dev_fold<<<1, kStripes, 0, S(stream)>>>(t->v);
  return launched();
}

ct_status ct_dev_apply_mixed(ct_table* t, const uint8_t* ops, const uint64_t* keys, const void* vals,
                             int64_t n, void* vals_out, uint8_t* status, void* stream) {
  if (!t || n < 0 || (n > 0 && (!keys || !ops))) return CT_E_INVALID;
  const int32_t vk = t->desc.val_kind;
  if (vk != CT_VAL_NONE && n > 0 && !vals) return CT_E_INVALID;
  if (n == 0) return CT_OK;
  DevView v{};
  v.t = t->v;
  v.mode = kDevMixed;
  t->size_ub = std::min<uint64_t>(t->size_ub + (uint64_t)n, (uint64_t)t->desc.capacity);
  v.striped = 1;
  k_dev_prep<<<1, kStripes, 0, S(stream)>>>(t->v, (uint64_t)n);
  const int sorted_blocks = (int)std::max<int64_t>(1, std::min<int64_t>((n + kSortWin - 1) / kSortWin, 8192));
  k_dev_apply_sorted<<<sorted_blocks, kBlock, 0, S(stream)>>>(v, ops, keys, vals, vk, n, vals_out,
                                                               status);
  k_dev_fold<<<1, kStripes, 0, S(stream)>>>(t->v);
  return launched();
}

ct_status ct_voxel_insert_neighbours(ct_table* t, const uint64_t* blocks, int64_t n, int32_t ndirs,
                                     void* stream) {
  if (!t || n < 0 || (n > 0 && !blocks) || (ndirs != 6 && ndirs != 26)) return CT_E_INVALID;
  if (t->desc.val_kind == CT_VAL_NONE) return CT_E_INVALID;
  if (n == 0) return CT_OK;
  DevView v{};
  v.t = t->v;
  v.mode = kDevInsert;
  t->size_ub = std::min<uint64_t>(t->size_ub + (uint64_t)n * (uint64_t)ndirs,
                                  (uint64_t)t->desc.capacity);
  v.striped = 1;
  k_dev_prep<<<1, kStripes, 0, S(stream)>>>(t->v, (uint64_t)n * (uint64_t)ndirs);
  k_voxel_neighbours<false><<<flat_blocks(n), kBlock, 0, S(stream)>>>(v, DevPool{}, blocks, n, ndirs);
  k_dev_fold<<<1, kStripes, 0, S(stream)>>>(t->v);
  return launched();
}

ct_status ct_voxel_insert_neighbours_alloc(ct_table* t, ct_pool* p, const uint64_t* blocks,
                                           int64_t n, int32_t ndirs, void* stream) {
  if (!t || !p || n < 0 || (n > 0 && !blocks) || (ndirs != 6 && ndirs != 26)) return CT_E_INVALID;
  if (t->desc.val_kind == CT_VAL_NONE) return CT_E_INVALID;
  if (n == 0) return CT_OK;
  DevView v{};
  v.t = t->v;
  v.mode = kDevInsert;
  t->size_ub = std::min<uint64_t>(t->size_ub + (uint64_t)n * (uint64_t)ndirs,
                                  (uint64_t)t->desc.capacity);
  v.striped = 1;
  k_dev_prep<<<1, kStripes, 0, S(stream)>>>(t->v, (uint64_t)n * (uint64_t)ndirs);
  k_voxel_neighbours<true><<<flat_blocks(n), kBlock, 0, S(stream)>>>(v, DevPool{p->hdr, p->stack},
                                                                     blocks, n, ndirs);
  k_dev_fold<<<1, kStripes, 0, S(stream)>>>(t->v);
  return launched();
}

ct_status ct_dev_update_set(ct_table* map, ct_table* set, const uint64_t* keys, int64_t n,
                            uint8_t* status, void* stream) {
  if (!map || !set || map == set || n < 0 || (n > 0 && !keys)) return CT_E_INVALID;
  if (n == 0) return CT_OK;
  hipStream_t s = S(stream);
  DevView mv{};
  mv.t = map->v;
  mv.mode = kDevRead;
  DevView sv{};
  sv.t = set->v;
  sv.mode = kDevInsert;
  sv.striped = 1;
  set->size_ub = std::min<uint64_t>(set->size_ub + (uint64_t)n, (uint64_t)set->desc.capacity);
  k_dev_prep<<<1, kStripes, 0, s>>>(set->v, (uint64_t)n);
  k_dev_update_set<<<flat_blocks(n), kBlock, 0, s>>>(mv, sv, keys, n, status);
  k_dev_fold<<<1, kStripes, 0, s>>>(set->v);
  return launched();
}

ct_status ct_pool_device_view(ct_pool* p, void* out, int64_t bytes) {
  if (!p || !out || bytes < (int64_t)sizeof(DevPool)) return CT_E_INVALID;
  const DevPool d{p->hdr, p->stack};
  std::memcpy(out, &d, sizeof(d));
  return CT_OK;
}

ct_status ct_dev_pool_apply(ct_pool* p, int32_t op, const int32_t* in, int64_t n, int32_t* out,
                            uint8_t* status, void* stream) {
  if (!p || n < 0 || (op != CT_DEV_PUSH_BACK && op != CT_DEV_POP_BACK)) return CT_E_INVALID;
  if (op == CT_DEV_PUSH_BACK && n > 0 && !in) return CT_E_INVALID;
  if (n == 0) return CT_OK;
  k_dev_pool_apply<<<flat_blocks(n), kBlock, 0, S(stream)>>>(DevPool{p->hdr, p->stack}, op, in, n,
                                                             out, status);
  return launched();
}

ct_status ct_table_rehash(ct_table* src, ct_table* dst, void* stream) {
  if (!src || !dst || src == dst || src->desc.val_kind != dst->desc.val_kind) return CT_E_INVALID;
  int64_t ns = 0, nd = 0;
  ct_status r = ct_size(src, &ns, stream);
  if (r == CT_OK) r = ct_size(dst, &nd, stream);
  if (r != CT_OK) return r;
  if (nd + ns > dst->desc.capacity) return CT_E_FULL;
  if (ns == 0) return CT_OK;
  const int grid = (int)std::max<int64_t>(1, std::min<int64_t>(((int64_t)src->v.nb + kBlock / 8 - 1) / (kBlock / 8), kMaxGroupBlocks));
  hipStream_t s = S(stream);
  launch(dst, CT_KERNEL_INSERT, s, [&] { k_rehash<<<grid, kBlock, 0, s>>>(src->v, dst->v); });
  launch(dst, CT_KERNEL_APPLY, s, [&] { k_apply_count<<<1, 1024, 0, s>>>(dst->v, grid, 0, 0); });
  dst->size_ub = (uint64_t)(nd + ns);
  return launched();
}

ct_status ct_dump(ct_table* t, uint64_t* keys_out, uint64_t* vals_out, int64_t cap,
                  int64_t* h_count, void* stream) {
  return select_into(t, AllKeys{}, keys_out, vals_out, cap, h_count, stream);
}

ct_status ct_select_key_range(ct_table* t, uint64_t lo, uint64_t hi, uint64_t* keys_out,
                              uint64_t* vals_out, int64_t cap, int64_t* h_count, void* stream) {
  return select_into(t, KeyRange{lo, hi}, keys_out, vals_out, cap, h_count, stream);
}

ct_status ct_select_voxel_box(ct_table* t, const int32_t* h_lo3, const int32_t* h_hi3,
                              uint64_t* keys_out, uint64_t* vals_out, int64_t cap, int64_t* h_count,
                              void* stream) {
  if (!h_lo3 || !h_hi3) return CT_E_INVALID;
  VoxelBox box;
  for (int d = 0; d < 3; ++d) {
    box.lo[d] = h_lo3[d];
    box.hi[d] = h_hi3[d];
  }
  return select_into(t, box, keys_out, vals_out, cap, h_count, stream);
}

ct_status ct_check_invariants_detail(ct_table* t, const ct_pool* p, int64_t* h_violations,
                                     uint32_t* h_what, void* stream) {
  if (!t || !h_violations) return CT_E_INVALID;
  if (p && t->desc.val_kind != CT_VAL_U32) return CT_E_INVALID;
  hipStream_t s = S(stream);
  const int64_t pool_cap = p ? std::max<int64_t>(p->cap, 1) : 0;
  k_check_begin<<<1, 1, 0, s>>>(t->v);
  k_check<<<flat_blocks((int64_t)t->v.nb * kSlots), kBlock, 0, s>>>(t->v, pool_cap);
  if (p) k_check_pool<<<flat_blocks(p->cap), kBlock, 0, s>>>(t->v, p->hdr, p->stack);
  if (launched() != CT_OK) return CT_E_HIP;
  Header h;
  if (hipMemcpyAsync(&h, t->v.hdr, sizeof(Header), hipMemcpyDeviceToHost, s) != hipSuccess)
    return CT_E_HIP;
  if (hipStreamSynchronize(s) != hipSuccess) return CT_E_HIP;
  const uint64_t specs = (uint64_t)(h.spec_live[0] != 0) + (uint64_t)(h.spec_live[1] != 0);
  int64_t bad = 0;
  uint32_t what = 0;
  if (h.live_count + specs != h.size || h.size > t->v.cap) {
    ++bad;
    what |= CT_CHECK_SIZE;
  }
  if (h.dup_count) {
    bad += (int64_t)h.dup_count;
    what |= CT_CHECK_DUPLICATE;
  }
  if (h.violations) {
    bad += (int64_t)h.violations;
    what |= CT_CHECK_REACH;
  }
  if (p && (h.pool_bad || h.pool_count != 0 || h.pool_h1 != 0 || h.pool_h2 != 0)) {
    bad += h.pool_bad ? (int64_t)h.pool_bad : 1;
    what |= CT_CHECK_POOL;
  }
  *h_violations = bad;
  if (h_what) *h_what = what;
  return CT_OK;
}

ct_status ct_check_invariants(ct_table* t, const ct_pool* p, int64_t* h_violations, void* stream) {
  return ct_check_invariants_detail(t, p, h_violations, nullptr, stream);
}

ct_status ct_table_health(ct_table* t, int64_t* h_closed, int64_t* h_tombstones, void* stream) {
  if (!t || (!h_closed && !h_tombstones)) return CT_E_INVALID;
  hipStream_t s = S(stream);
  k_health_begin<<<1, 1, 0, s>>>(t->v);
  k_health<<<group_blocks((int64_t)t->v.nb), kBlock, 0, s>>>(t->v);
  if (launched() != CT_OK) return CT_E_HIP;
  Header h;
  if (hipMemcpyAsync(&h, t->v.hdr, sizeof(Header), hipMemcpyDeviceToHost, s) != hipSuccess)
    return CT_E_HIP;
  if (hipStreamSynchronize(s) != hipSuccess) return CT_E_HIP;
  if (h_closed) *h_closed = (int64_t)h.closed_count;
  if (h_tombstones) *h_tombstones = (int64_t)h.tomb_count;
  return CT_OK;
}

ct_status ct_table_purge(ct_table* t, void* stream) {
  if (!t) return CT_E_INVALID;
  hipStream_t s = S(stream);
  uint32_t* bits = reinterpret_cast<uint32_t*>(t->v.dd);
  const int64_t window = t->dd_bytes / 4 * 32;   // buckets per pass: one bit each
  const int64_t nb = (int64_t)t->v.nb;
  for (int64_t w0 = 0; w0 < nb; w0 += window) {
    const int64_t w1 = std::min(nb, w0 + window);
    const int64_t words = (w1 - w0 + 31) / 32;
    k_purge_clear<<<flat_blocks(words), kBlock, 0, s>>>(bits, words);
    k_purge_mark<<<flat_blocks(nb * kSlots), kBlock, 0, s>>>(t->v, bits, w0, w1);
    k_purge_reopen<<<flat_blocks((w1 - w0) * kSlots), kBlock, 0, s>>>(t->v, bits, w0, w1);
    if (launched() != CT_OK) return CT_E_HIP;
  }
  return CT_OK;
}

ct_status ct_get_error(ct_table* t, uint32_t* h_err, void* stream) {
  if (!t || !h_err) return CT_E_INVALID;
  uint32_t e = 0;
  ct_status r = read_back(&t->v.hdr->err, &e, S(stream));
  if (r != CT_OK) return r;
  *h_err = e;
  const uint32_t zero = 0;
  if (hipMemcpyAsync(&t->v.hdr->err, &zero, sizeof(zero), hipMemcpyHostToDevice, S(stream)) != hipSuccess)
    return CT_E_HIP;
  return hipStreamSynchronize(S(stream)) == hipSuccess ? CT_OK : CT_E_HIP;
}

__global__ void k_set_inject(TableView t, uint32_t every) { t.hdr->inject = every; }

ct_status ct_table_debug_inject_claim_losses(ct_table* t, uint32_t every, void* stream) {
  if (!t) return CT_E_INVALID;
  k_set_inject<<<1, 1, 0, S(stream)>>>(t->v, every);
  return launched();
}

ct_status ct_table_dedup_skewed(ct_table* t, int32_t* h_skewed, void* stream) {
  if (!t || !h_skewed) return CT_E_INVALID;
  uint32_t v = 0;
  ct_status r = read_back(&t->v.hdr->dskew, &v, S(stream));
  if (r != CT_OK) return r;
  *h_skewed = v ? 1 : 0;
  return CT_OK;
}

ct_status ct_table_set_insert_path(ct_table* t, int32_t path) {
  if (!t || path < CT_INSERT_AUTO || path > CT_INSERT_SPECULATIVE) return CT_E_INVALID;
  t->insert_path = path;
  return CT_OK;
}

// --- pools -------------------------------------------------------------------------------------
ct_status ct_pool_bytes(int64_t capacity, int64_t* bytes) {
  if (!bytes || capacity < 0 || capacity > 0x7FFFFFFFll) return CT_E_INVALID;
  *bytes = align_up((int64_t)sizeof(PoolHeader)) + align_up(capacity * 4);
  return CT_OK;
}

ct_status ct_pool_init(void* d_buf, int64_t bytes, int64_t capacity, void* stream, ct_pool** out) {
  int64_t need = 0;
  if (!out || !d_buf || ct_pool_bytes(capacity, &need) != CT_OK || bytes < need) return CT_E_INVALID;
  if (reinterpret_cast<uintptr_t>(d_buf) % kAlign) return CT_E_INVALID;
  ct_pool* p = new (std::nothrow) ct_pool;
  if (!p) return CT_E_NOMEM;
  p->base = static_cast<uint8_t*>(d_buf);
  p->cap = capacity;
  p->hdr = reinterpret_cast<PoolHeader*>(p->base);
  p->stack = reinterpret_cast<int32_t*>(p->base + align_up((int64_t)sizeof(PoolHeader)));
  k_pool_init<<<flat_blocks(capacity), kBlock, 0, S(stream)>>>(p->hdr, p->stack, capacity);
  if (launched() != CT_OK) {
    delete p;
    return CT_E_HIP;
  }
  *out = p;
  return CT_OK;
}

ct_status ct_pool_destroy(ct_pool* p) {
  if (!p) return CT_E_INVALID;
  delete p;
  return CT_OK;
}

ct_status ct_pool_pop_batch(ct_pool* p, int64_t n, int32_t* out, uint8_t* status, void* stream) {
  if (!p || n < 0) return CT_E_INVALID;
  if (n == 0) return CT_OK;
  k_pool_snapshot<<<1, 1, 0, S(stream)>>>(p->hdr);
  k_pool_pop<<<flat_blocks(n), kBlock, 0, S(stream)>>>(p->hdr, p->stack, n, out, status);
  return launched();
}

ct_status ct_pool_pop_front_batch(ct_pool* p, int64_t n, int32_t* out, uint8_t* status,
                                  void* stream) {
  if (!p || n < 0) return CT_E_INVALID;
  if (n == 0) return CT_OK;
  k_pool_snapshot<<<1, 1, 0, S(stream)>>>(p->hdr);
  k_pool_pop_front<<<flat_blocks(n), kBlock, 0, S(stream)>>>(p->hdr, p->stack, n, out, status);
  return launched();
}

ct_status ct_pool_push_front_batch(ct_pool* p, const int32_t* in, int64_t n, uint8_t* status,
                                   void* stream) {
  if (!p || n < 0 || (n > 0 && !in)) return CT_E_INVALID;
  if (n == 0) return CT_OK;
  k_pool_snapshot<<<1, 1, 0, S(stream)>>>(p->hdr);
  k_pool_push_front<<<flat_blocks(n), kBlock, 0, S(stream)>>>(p->hdr, p->stack, in, n, status);
  return launched();
}

ct_status ct_pool_push_batch(ct_pool* p, const int32_t* in, int64_t n, uint8_t* status,
                             void* stream) {
  if (!p || n < 0 || (n > 0 && !in)) return CT_E_INVALID;
  if (n == 0) return CT_OK;
  k_pool_snapshot<<<1, 1, 0, S(stream)>>>(p->hdr);
  k_pool_push<<<flat_blocks(n), kBlock, 0, S(stream)>>>(p->hdr, p->stack, in, n, status);
  return launched();
}

ct_status ct_pool_size(ct_pool* p, int64_t* h_size, void* stream) {
  if (!p || !h_size) return CT_E_INVALID;
  return read_back(&p->hdr->top, h_size, S(stream));
}

ct_status ct_pool_dump(ct_pool* p, int32_t* out, int64_t cap, int64_t* h_count, void* stream) {
  if (!p || !h_count || cap < 0 || (cap > 0 && !out)) return CT_E_INVALID;
  if (cap > 0) k_pool_copy<<<flat_blocks(cap), kBlock, 0, S(stream)>>>(p->hdr, p->stack, out, cap);
  if (launched() != CT_OK) return CT_E_HIP;
  return read_back(&p->hdr->top, h_count, S(stream));
}

ct_status ct_pool_get_error(ct_pool* p, uint32_t* h_err, void* stream) {
  if (!p || !h_err) return CT_E_INVALID;
  uint32_t e = 0;
  ct_status r = read_back(&p->hdr->err, &e, S(stream));
  if (r != CT_OK) return r;
  *h_err = e;
  const uint32_t zero = 0;
  if (hipMemcpyAsync(&p->hdr->err, &zero, sizeof(zero), hipMemcpyHostToDevice, S(stream)) != hipSuccess)
    return CT_E_HIP;
  return hipStreamSynchronize(S(stream)) == hipSuccess ? CT_OK : CT_E_HIP;
}

}  // extern "C"

namespace {

// Pool-valued insert of n keys; with `skip`, only the elements whose byte there is zero take part,
// in index order among themselves (masked batches are sparse: their repeated keys are resolved
// through dd, whatever the chunk size).
ct_status insert_alloc_chunks(ct_table* t, ct_pool* p, const uint64_t* keys, const uint8_t* skip,
                              int64_t n, int32_t* vals_out, uint8_t* status, hipStream_t s) {
  ct_status r = CT_OK;
  for (int64_t c0 = 0; c0 < n; c0 += t->chunk) {
    const int64_t q = std::min<int64_t>(t->chunk, n - c0);
    const uint32_t db = dedup_slots_for(q);
    const uint64_t* kc = keys + c0;
    const uint8_t* mc = skip ? skip + c0 : nullptr;
    uint8_t* sc = status ? status + c0 : nullptr;
    int32_t* vc = vals_out ? vals_out + c0 : nullptr;
    const int gb = group_blocks((q + kSlots - 1) / kSlots);
    const int ntiles = (int)((q + kTile - 1) / kTile);
    // a masked chunk's prologue also zeroes the tile sums, and its insert kernel counts the
    // rank flags per tile itself: one launch fewer for the small chunks of a reconstruction frame
    if (mc) {
      launch(t, CT_KERNEL_PROLOGUE, s, [&] { k_prologue<<<flat_blocks(db / 2), kBlock, 0, s>>>(t->v, p->hdr, db, q, 1); });
      launch(t, CT_KERNEL_DEDUP, s, [&] { k_dedup<<<flat_blocks(q), kBlock, 0, s>>>(t->v, kc, mc, q, db - 1); });
    } else {
      dedup_chunk(t, t->v, p->hdr, kc, q, s);
    }
    launch(t, CT_KERNEL_INSERT, s, [&] { k_insert<1, true><<<gb, kBlock, 0, s>>>(t->v, kc, nullptr, q, db - 1, sc, vc, mc, mc ? 1 : 0); });
    if (!mc) launch(t, CT_KERNEL_RANK, s, [&] { k_tile_count<<<ntiles, kBlock, 0, s>>>(t->v, q, 0); });
    const int inl = ntiles <= kInlineRankTiles ? ntiles : 0;
    if (!inl) launch(t, CT_KERNEL_RANK, s, [&] { k_tile_scan<<<1, 1024, 0, s>>>(t->v, p->hdr, ntiles, 1); });
    launch(t, CT_KERNEL_FINAL, s, [&] { k_final<1, 1><<<ntiles, kBlock, 0, s>>>(t->v, p->hdr, p->stack, kc, nullptr, q, sc, vc, inl); });
    if (sc || vc) launch(t, CT_KERNEL_FIX, s, [&] { k_fix<<<flat_blocks(q), kBlock, 0, s>>>(t->v, sc, vc); });
    t->size_ub = std::min<uint64_t>(t->size_ub + (uint64_t)q, (uint64_t)t->desc.capacity);
    r = launched();
    if (r != CT_OK) return r;
  }
  return CT_OK;
}

}  // namespace

extern "C" {

ct_status ct_insert_alloc_batch(ct_table* t, ct_pool* p, const uint64_t* keys, int64_t n,
                                int32_t* vals_out, uint8_t* status, void* stream) {
  ct_status r = check_batch(t, keys, n);
  if (r != CT_OK || !p) return CT_E_INVALID;
  if (t->desc.val_kind != CT_VAL_U32) return CT_E_INVALID;
  if (n == 0) return CT_OK;
  return insert_alloc_chunks(t, p, keys, nullptr, n, vals_out, status, S(stream));
}

ct_status ct_insert_alloc_batch_masked(ct_table* t, ct_pool* p, const uint64_t* keys,
                                       const uint8_t* skip, int64_t n, int32_t* vals_out,
                                       uint8_t* status, void* stream) {
  ct_status r = check_batch(t, keys, n);
  if (r != CT_OK || !p || (n > 0 && !skip)) return CT_E_INVALID;
  if (t->desc.val_kind != CT_VAL_U32) return CT_E_INVALID;
  if (n == 0) return CT_OK;
  return insert_alloc_chunks(t, p, keys, skip, n, vals_out, status, S(stream));
}

ct_status ct_erase_release_batch(ct_table* t, ct_pool* p, const uint64_t* keys, int64_t n,
                                 uint8_t* erased, void* stream) {
  ct_status r = check_batch(t, keys, n);
  if (r != CT_OK || !p) return CT_E_INVALID;
  if (t->desc.val_kind != CT_VAL_U32) return CT_E_INVALID;
  if (n == 0) return CT_OK;
  return erase_chunks<true>(t, p, keys, n, erased, S(stream));
}

}  // extern "C"

// --- multi-table plans ----------------------------------------------------------------------
// A plan replays a schedule of single-table operations.  Tables are spread over `lanes` side
// streams forked from the caller's stream (a table's operations stay on one stream, so their
// order holds) and joined back at the end; each operation runs the same kernel pipeline as the
// single-table call.  The whole fork/join sequence captures into one HIP graph.
namespace {
struct PlanOp {
  ct_table* t;
  int32_t type;
  const uint64_t* keys;
  const void* vals;
  void* vout;
  uint8_t* flags;
  int64_t n;
};
}  // namespace

namespace ct_group {
// One kernel launch of a grouped plan: `n` entries from `entry_off` of the entry array.
struct Launch {
  int32_t stage, n, blocks;
  int64_t entry_off;
};
}  // namespace ct_group

struct ct_plan {
  std::vector<PlanOp> ops;
  std::vector<ct_table*> tables;  // distinct tables in first-use order
  std::vector<hipStream_t> side;
  std::vector<hipEvent_t> ev;     // fork event + one join event per side stream
  // grouped form (ct_plan_group): valid while the plan still has `grouped_ops` operations
  std::vector<ct_group::Launch> glaunch;
  const void* gsteps = nullptr;    // device: GStep[]
  const void* gentries = nullptr;  // device: GEntry[]
  const void* gcopies = nullptr;   // device: GCopy[] of the merged operations' copy stages
  size_t grouped_ops = (size_t)-1;
  int gblock = kBlock;             // threads per block of its find / insert / erase stages
  const void* glaunch_dev = nullptr;  // device: GLaunchDev[] for the single-launch form
  int32_t gwidest = 1;             // most blocks of any one stage launch
};

namespace {

ct_status plan_streams(ct_plan* p, int32_t lanes) {
  while ((int32_t)p->side.size() < lanes) {
    hipStream_t s;
    if (hipStreamCreateWithFlags(&s, hipStreamNonBlocking) != hipSuccess) return CT_E_HIP;
    p->side.push_back(s);
  }
  while (p->ev.size() < p->side.size() + 1) {
    hipEvent_t e;
    if (hipEventCreateWithFlags(&e, hipEventDisableTiming) != hipSuccess) return CT_E_HIP;
    p->ev.push_back(e);
  }
  return CT_OK;
}

ct_status run_op(const PlanOp& o, hipStream_t s) {
  ct_table* t = o.t;
  const int vk = t->desc.val_kind;
  switch (o.type) {
    case kOpClear:
      launch(t, CT_KERNEL_CLEAR, s, [&] { k_table_reset<<<flat_blocks((int64_t)t->v.nb * kSlots), kBlock, 0, s>>>(t->v, 0); });
      return launched();
    case kOpInsert:
      if (vk == CT_VAL_U32) return insert_chunks<1>(t, o.keys, o.vals, o.n, o.flags, s);
      if (vk == CT_VAL_U64) return insert_chunks<2>(t, o.keys, o.vals, o.n, o.flags, s);
      return insert_chunks<0>(t, o.keys, nullptr, o.n, o.flags, s);
    case kOpErase:
      return erase_chunks<false>(t, nullptr, o.keys, o.n, o.flags, s);
    default: {
      const int gb = group_blocks((o.n + kSlots - 1) / kSlots);
      launch(t, CT_KERNEL_FIND, s, [&] {
        if (vk == CT_VAL_U32) k_find<1><<<gb, kBlock, 0, s>>>(t->v, o.keys, o.n, o.vout, o.flags);
        else if (vk == CT_VAL_U64) k_find<2><<<gb, kBlock, 0, s>>>(t->v, o.keys, o.n, o.vout, o.flags);
        else k_find<0><<<gb, kBlock, 0, s>>>(t->v, o.keys, o.n, nullptr, o.flags);
      });
      return launched();
    }
  }
}

// Copy-stage blocks for a segment: enough 256-thread blocks for 16-byte units, at most 2048.
int copy_blocks(int64_t bytes) {
  const int64_t b = (bytes / 16 + kBlock - 1) / kBlock;
  return (int)std::max<int64_t>(1, std::min<int64_t>(b, 2048));
}

bool inserts_or_erases(const GStep& g) { return g.type == kOpInsert || g.type == kOpErase; }

// Blocks of a grouped stage whose blocks stride over n units of work and usually find little
// or nothing to do (the resolution of a speculative step, the repeated-key outcomes, the
// prologue's scratch clear): 8 units per thread, at most 1024 blocks per step.
int spec_blocks(int64_t n) {
  const int64_t b = (n + 8 * kBlock - 1) / (8 * kBlock);
  return (int)std::max<int64_t>(1, std::min<int64_t>(b, 1024));
}

// Units of a chunk's scratch clear (as prologue_units on the device).
int64_t prologue_units_host(uint32_t dslots, int64_t q) { return (int64_t)dslots / 2 + (q + 15) / 16; }

// Blocks of step `g` in stage `stage` (0: the step has no such stage); the same grids as the
// single-table pipeline.
int stage_blocks(int stage, const GStep& g) {
  switch (stage) {
    case gReset: return g.type == kOpClear ? flat_blocks((int64_t)g.v.nb * kSlots) : 0;
    case gPro: return inserts_or_erases(g) ? spec_blocks(prologue_units_host(g.db, g.q)) : 0;
    case gDedup: return inserts_or_erases(g) ? flat_blocks(g.q) : 0;
    case gFind: return g.type == kOpFind ? g.gb : 0;
    case gInsert: return g.type == kOpInsert ? g.gb : 0;
    case gErase: return g.type == kOpErase ? g.gb : 0;
    case gApply: return inserts_or_erases(g) ? 1 : 0;
    // resolution of a speculative step: a few elements per thread when something is listed; the
    // blocks leave at once otherwise
    case gSClear: return inserts_or_erases(g) && g.spath ? spec_blocks((int64_t)g.db / 2) : 0;
    case gSBuild:
    case gSProbe:
    case gSSwap: return inserts_or_erases(g) && g.spath ? spec_blocks(g.q) : 0;
    case gCount: return g.type == kOpInsert ? g.ntiles : 0;
    case gScan: return g.type == kOpInsert ? 1 : 0;
    case gFinal: return g.type == kOpInsert ? g.ntiles : 0;
    case gFix: return g.type == kOpInsert && g.flags ? spec_blocks(g.q) : 0;
  }
  return 0;
}

// The grouped form of a plan, built on the host.  `base` is the device buffer the form will live
// in (null while only sizing it): steps, entries, copy segments, then the merge area.
struct GroupForm {
  std::vector<GStep> steps;
  std::vector<GEntry> entries;
  std::vector<GCopy> copies;
  std::vector<ct_group::Launch> launches;
  int64_t merge_bytes = 0;
  int64_t steps_off = 0, entries_off = 0, copies_off = 0, launches_off = 0, merge_off = 0,
          total = 0;
};

// Cut the plan into chunk-steps, assign each the per-table ordinal as its level, and lay out one
// launch per (level, stage) that has steps.  With CT_GROUP_MERGE_RUNS, a run of consecutive
// operations of one kind on one table becomes one operation over a contiguous copy of its arrays
// in the merge area (a batch equals its parts applied in order), gathered before the first level
// and scattered back after the last.  Host only.
// Threads per block of the grouped find / insert / erase stages encoded in `options`.
int group_block_size(int32_t options) {
  const int code = (options >> CT_GROUP_BLOCK_SHIFT) & 0xF;
  return code ? (1 << code) : kBlock;
}

bool group_options_valid(int32_t options) {
  if (options & ~(CT_GROUP_MERGE_RUNS | (0xF << CT_GROUP_BLOCK_SHIFT))) return false;
  const int code = (options >> CT_GROUP_BLOCK_SHIFT) & 0xF;
  return code == 0 || (code >= 7 && code <= 10);   // 128 .. 1024 threads
}

ct_status group_build(const ct_plan* p, int32_t options, uint8_t* base, GroupForm& F) {
  const bool merge = (options & CT_GROUP_MERGE_RUNS) != 0;
  const int bs = group_block_size(options);
  struct Eff {  // an operation of one table as it will be cut into steps
    PlanOp op;
    size_t first, count;  // its run of plan operations
  };
  std::vector<std::vector<Eff>> per(p->tables.size());
  for (size_t k = 0; k < p->ops.size(); ++k) {
    const PlanOp& o = p->ops[k];
    const size_t ti = (size_t)(std::find(p->tables.begin(), p->tables.end(), o.t) - p->tables.begin());
    std::vector<Eff>& v = per[ti];
    if (merge && o.type != kOpClear && !v.empty() && v.back().op.type == o.type) {
      v.back().count += 1;
      v.back().op.n += o.n;
    } else {
      v.push_back(Eff{o, k, 1});
    }
  }
  // merge area: contiguous arrays for every run of two or more operations
  std::vector<GCopy> copy_out;
  int64_t moff = 0;
  auto take = [&](int64_t bytes) {
    const int64_t o = moff;
    moff += align_up(bytes);
    return o;
  };
  struct Fix {  // device addresses of a merged run's arrays, as offsets into the merge area
    int64_t keys = -1, vals = -1, flags = -1, vout = -1;
  };
  std::vector<std::vector<Fix>> fixes(per.size());
  for (size_t ti = 0; ti < per.size(); ++ti) {
    fixes[ti].resize(per[ti].size());
    for (size_t r = 0; r < per[ti].size(); ++r) {
      const Eff& e = per[ti][r];
      if (e.count < 2) continue;
      const ct_table* t = e.op.t;
      const int vk = t->desc.val_kind;
      const int64_t vb = vk == CT_VAL_U32 ? 4 : 8;
      bool want_flags = false, want_vout = false;
      for (size_t k = e.first, c = 0; c < e.count; ++k) {
        const PlanOp& o = p->ops[k];
        if (o.t != t) continue;
        want_flags = want_flags || o.flags;
        want_vout = want_vout || o.vout;
        ++c;
      }
      Fix& f = fixes[ti][r];
      f.keys = take(e.op.n * 8);
      if (e.op.type == kOpInsert && vk != CT_VAL_NONE) f.vals = take(e.op.n * vb);
      if (want_flags) f.flags = take(e.op.n);
      if (e.op.type == kOpFind && vk != CT_VAL_NONE && want_vout) f.vout = take(e.op.n * vb);
    }
  }
  F.merge_bytes = moff;
  // device layout: steps | entries | copies | merge area (filled in below once counts are known)
  // while only sizing, a placeholder base keeps every merged array non-null, so the steps and
  // their stages (a fix stage needs a status array) are the same as when building
  uint8_t* const b0 = base ? base : reinterpret_cast<uint8_t*>((uintptr_t)kAlign);
  auto dev = [&](int64_t merge_off) -> uint8_t* { return b0 + F.merge_off + merge_off; };

  std::vector<int32_t> level;
  std::vector<GCopy> copy_in;
  // first pass only counts steps and copies so the layout offsets are known; the second fills
  for (int pass = 0; pass < 2; ++pass) {
    F.steps.clear();
    level.clear();
    copy_in.clear();
    copy_out.clear();
    for (size_t ti = 0; ti < per.size(); ++ti) {
      int32_t lev = 0;
      for (size_t r = 0; r < per[ti].size(); ++r) {
        const Eff& e = per[ti][r];
        PlanOp o = e.op;
        ct_table* t = o.t;
        const int vk = t->desc.val_kind;
        const int64_t vb = vk == CT_VAL_U32 ? 4 : 8;
        if (e.count >= 2) {
          const Fix& f = fixes[ti][r];
          uint8_t* mk = dev(f.keys);
          uint8_t* mv = f.vals >= 0 ? dev(f.vals) : nullptr;
          uint8_t* mf = f.flags >= 0 ? dev(f.flags) : nullptr;
          uint8_t* mo = f.vout >= 0 ? dev(f.vout) : nullptr;
          int64_t pos = 0;
          for (size_t k = e.first, c = 0; c < e.count; ++k) {
            const PlanOp& part = p->ops[k];
            if (part.t != t) continue;
            ++c;
            copy_in.push_back(GCopy{part.keys, mk + pos * 8, part.n * 8});
            if (mv) copy_in.push_back(GCopy{part.vals, mv + pos * vb, part.n * vb});
            if (mf && part.flags) copy_out.push_back(GCopy{mf + pos, part.flags, part.n});
            if (mo && part.vout) copy_out.push_back(GCopy{mo + pos * vb, part.vout, part.n * vb});
            pos += part.n;
          }
          o.keys = reinterpret_cast<const uint64_t*>(mk);
          o.vals = mv;
          o.flags = mf;
          o.vout = mo;
        }
        const bool ie = o.type == kOpInsert || o.type == kOpErase;
        const int64_t span = ie ? t->chunk : std::max<int64_t>(o.n, 1);
        for (int64_t c0 = 0; c0 < std::max<int64_t>(o.n, 1); c0 += span) {
          const int64_t q = o.type == kOpClear ? 0 : std::min<int64_t>(span, o.n - c0);
          GStep g{};
          g.v = t->v;
          g.type = o.type;
          g.vk = vk;
          g.q = q;
          g.keys = o.keys ? o.keys + c0 : nullptr;
          g.vals = (o.type == kOpInsert && vk != CT_VAL_NONE)
                       ? static_cast<const uint8_t*>(o.vals) + c0 * vb : nullptr;
          g.vout = (o.type == kOpFind && o.vout) ? static_cast<uint8_t*>(o.vout) + c0 * vb : nullptr;
          g.flags = o.flags ? o.flags + c0 : nullptr;
          g.db = ie ? dedup_slots_for(q) : 0u;
          g.spath = !ie || t->insert_path == CT_INSERT_RESOLVE_FIRST ? 0
                    : t->insert_path == CT_INSERT_SPECULATIVE ? 2 : 1;
          g.gb = group_blocks((q + kSlots - 1) / kSlots, bs);
          g.ntiles = (int32_t)((q + kTile - 1) / kTile);
          F.steps.push_back(g);
          level.push_back(lev++);
        }
      }
    }
    F.copies = copy_in;
    F.copies.insert(F.copies.end(), copy_out.begin(), copy_out.end());
    F.steps_off = 0;
    F.entries_off = align_up((int64_t)(F.steps.size() * sizeof(GStep)));
    // entries: one per (level, stage, step) plus one per copy segment (bounded by a count pass)
    int64_t nent = (int64_t)F.copies.size();
    for (const GStep& g : F.steps)
      for (int stage = 0; stage < gStages; ++stage) nent += stage_blocks(stage, g) ? 1 : 0;
    F.copies_off = F.entries_off + align_up(nent * (int64_t)sizeof(GEntry));
    // launch list for the single-launch form: at most a copy launch on each side of the levels
    int32_t nlev_max = 0;
    for (int32_t l : level) nlev_max = std::max(nlev_max, l + 1);
    const int64_t max_launches = 2 + (int64_t)nlev_max * gStages;
    F.launches_off = F.copies_off + align_up((int64_t)(F.copies.size() * sizeof(GCopy)));
    F.merge_off = F.launches_off + align_up(max_launches * (int64_t)sizeof(GLaunchDev));
    F.total = std::max<int64_t>(kAlign, F.merge_off + F.merge_bytes);
  }
  // Keys per thread of the find / insert / erase stages, per level: a level with much work runs
  // its steps with fewer, longer-running blocks (each block pays its step lookup and partial count
  // once), as long as the level still offers about 2^20 threads; at most 16 keys per thread.
  {
    int32_t nl = 0;
    for (int32_t l : level) nl = std::max(nl, l + 1);
    std::vector<int64_t> keys_at(nl, 0);
    auto probes = [](const GStep& g) {
      return g.type == kOpInsert || g.type == kOpErase || g.type == kOpFind;
    };
    for (size_t i = 0; i < F.steps.size(); ++i)
      if (probes(F.steps[i])) keys_at[level[i]] += F.steps[i].q;
    for (size_t i = 0; i < F.steps.size(); ++i) {
      GStep& g = F.steps[i];
      if (!probes(g)) continue;
      int64_t per = 1;
      while (per < 16 && keys_at[level[i]] >= (per * 2) << 20) per *= 2;
      g.gb = group_blocks((g.q + kSlots * per - 1) / (kSlots * per), bs);
    }
  }
  // launches: copy in, the levels, copy out
  F.entries.clear();
  F.launches.clear();
  auto copy_launch = [&](size_t from, size_t to) {
    if (from == to) return CT_OK;
    int64_t blocks = 0;
    const int64_t off = (int64_t)F.entries.size();
    for (size_t i = from; i < to; ++i) {
      F.entries.push_back(GEntry{(int32_t)blocks, (int32_t)i});
      blocks += copy_blocks(F.copies[i].bytes);
      if (blocks > (int64_t)INT32_MAX / 2) return CT_E_INVALID;
    }
    F.launches.push_back(ct_group::Launch{gCopy, (int32_t)(to - from), (int32_t)blocks, off});
    return CT_OK;
  };
  if (copy_launch(0, copy_in.size()) != CT_OK) return CT_E_INVALID;
  int32_t nlev = 0;
  for (int32_t l : level) nlev = std::max(nlev, l + 1);
  std::vector<std::vector<int32_t>> by_level(nlev);
  for (size_t i = 0; i < F.steps.size(); ++i) by_level[level[i]].push_back((int32_t)i);
  for (int32_t l = 0; l < nlev; ++l) {
    for (int stage = 0; stage < gStages; ++stage) {
      int64_t blocks = 0;
      const int64_t off = (int64_t)F.entries.size();
      for (int32_t i : by_level[l]) {
        const int b = stage_blocks(stage, F.steps[i]);
        if (!b) continue;
        F.entries.push_back(GEntry{(int32_t)blocks, i});
        blocks += b;
        if (blocks > (int64_t)INT32_MAX / 2) return CT_E_INVALID;
      }
      const int64_t n = (int64_t)F.entries.size() - off;
      if (n) F.launches.push_back(ct_group::Launch{stage, (int32_t)n, (int32_t)blocks, off});
    }
  }
  if (copy_launch(copy_in.size(), F.copies.size()) != CT_OK) return CT_E_INVALID;
  return CT_OK;
}

// One launch of a grouped find / insert / erase stage with BS threads per block.
template <int BS>
void probe_stage(int32_t stage, hipStream_t s, const ct_group::Launch& L, const GStep* st,
                 const GEntry* e) {
  if (stage == gFind) k_g_find<BS><<<L.blocks, BS, 0, s>>>(st, e, L.n);
  else if (stage == gInsert) k_g_insert<BS><<<L.blocks, BS, 0, s>>>(st, e, L.n);
  else k_g_erase<BS><<<L.blocks, BS, 0, s>>>(st, e, L.n);
}

}  // namespace

extern "C" {

ct_status ct_plan_group_bytes(ct_plan* p, int32_t options, int64_t* bytes) {
  if (!p || !bytes || !group_options_valid(options)) return CT_E_INVALID;
  GroupForm F;
  ct_status r = group_build(p, options, nullptr, F);
  if (r != CT_OK) return r;
  *bytes = F.total;
  return CT_OK;
}

ct_status ct_plan_group(ct_plan* p, int32_t options, void* d_buf, int64_t bytes) {
  if (!p || !d_buf || reinterpret_cast<uintptr_t>(d_buf) % kAlign) return CT_E_INVALID;
  if (!group_options_valid(options)) return CT_E_INVALID;
  uint8_t* base = static_cast<uint8_t*>(d_buf);
  GroupForm F;
  ct_status r = group_build(p, options, base, F);
  if (r != CT_OK) return r;
  if (bytes < F.total) return CT_E_INVALID;
  if (!F.steps.empty() && hipMemcpy(base + F.steps_off, F.steps.data(), F.steps.size() * sizeof(GStep),
                                    hipMemcpyHostToDevice) != hipSuccess)
    return CT_E_HIP;
  if (!F.entries.empty() && hipMemcpy(base + F.entries_off, F.entries.data(),
                                      F.entries.size() * sizeof(GEntry), hipMemcpyHostToDevice) != hipSuccess)
    return CT_E_HIP;
  if (!F.copies.empty() && hipMemcpy(base + F.copies_off, F.copies.data(),
                                     F.copies.size() * sizeof(GCopy), hipMemcpyHostToDevice) != hipSuccess)
    return CT_E_HIP;
  std::vector<GLaunchDev> ld;
  int32_t widest = 1;
  for (const ct_group::Launch& L : F.launches) {
    ld.push_back(GLaunchDev{L.stage, L.n, L.blocks, 0, L.entry_off});
    widest = std::max(widest, L.blocks);
  }
  if (!ld.empty() && hipMemcpy(base + F.launches_off, ld.data(), ld.size() * sizeof(GLaunchDev),
                               hipMemcpyHostToDevice) != hipSuccess)
    return CT_E_HIP;
  p->glaunch_dev = base + F.launches_off;
  p->gwidest = widest;
  p->glaunch = std::move(F.launches);
  p->gsteps = base + F.steps_off;
  p->gentries = base + F.entries_off;
  p->gcopies = base + F.copies_off;
  p->grouped_ops = p->ops.size();
  p->gblock = group_block_size(options);
  return CT_OK;
}

ct_status ct_plan_launch_grouped(ct_plan* p, void* stream) {
  if (!p || p->grouped_ops != p->ops.size()) return CT_E_INVALID;
  hipStream_t s = S(stream);
  const GStep* st = static_cast<const GStep*>(p->gsteps);
  const GEntry* en = static_cast<const GEntry*>(p->gentries);
  for (const ct_group::Launch& L : p->glaunch) {
    const GEntry* e = en + L.entry_off;
    switch (L.stage) {
      case gReset: k_g_reset<<<L.blocks, kBlock, 0, s>>>(st, e, L.n); break;
      case gPro: k_g_prologue<<<L.blocks, kBlock, 0, s>>>(st, e, L.n); break;
      case gDedup: k_g_dedup<<<L.blocks, kBlock, 0, s>>>(st, e, L.n); break;
      case gFind:
      case gInsert:
      case gErase:
        if (p->gblock == 128) probe_stage<128>(L.stage, s, L, st, e);
        else if (p->gblock == 512) probe_stage<512>(L.stage, s, L, st, e);
        else if (p->gblock == 1024) probe_stage<1024>(L.stage, s, L, st, e);
        else probe_stage<kBlock>(L.stage, s, L, st, e);
        break;
      case gApply: k_g_apply<<<L.blocks, 1024, 0, s>>>(st, e, L.n); break;
      case gCount: k_g_tile_count<<<L.blocks, kBlock, 0, s>>>(st, e, L.n); break;
      case gScan: k_g_tile_scan<<<L.blocks, 1024, 0, s>>>(st, e, L.n); break;
      case gFinal: k_g_final<<<L.blocks, kBlock, 0, s>>>(st, e, L.n); break;
      case gFix: k_g_fix<<<L.blocks, kBlock, 0, s>>>(st, e, L.n); break;
      case gSClear: k_g_sclear<<<L.blocks, kBlock, 0, s>>>(st, e, L.n); break;
      case gSBuild: k_g_sbuild<<<L.blocks, kBlock, 0, s>>>(st, e, L.n); break;
      case gSProbe: k_g_sfix<false><<<L.blocks, kBlock, 0, s>>>(st, e, L.n); break;
      case gSSwap: k_g_sfix<true><<<L.blocks, kBlock, 0, s>>>(st, e, L.n); break;
      case gCopy:
        k_g_copy<<<L.blocks, kBlock, 0, s>>>(static_cast<const GCopy*>(p->gcopies), e, L.n);
        break;
      default: return CT_E_INVALID;
    }
    if (launched() != CT_OK) return CT_E_HIP;
  }
  return CT_OK;
}

ct_status ct_plan_launch_single(ct_plan* p, int32_t max_blocks, void* stream) {
  if (!p || p->grouped_ops != p->ops.size() || p->gblock != kBlock || max_blocks < 0)
    return CT_E_INVALID;
  if (p->glaunch.empty()) return CT_OK;
  int dev = 0, coop = 0, ncu = 0, per_cu = 0;
  hipStream_t s = S(stream);
  if (s) {
    if (hipStreamGetDevice(s, &dev) != hipSuccess) return CT_E_HIP;
  } else if (hipGetDevice(&dev) != hipSuccess) {
    return CT_E_HIP;
  }
  if (hipDeviceGetAttribute(&coop, hipDeviceAttributeCooperativeLaunch, dev) != hipSuccess ||
      hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess ||
      hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k_g_persistent, kBlock, 0) != hipSuccess)
    return CT_E_HIP;
  if (!coop || per_cu < 1 || ncu < 1) return CT_E_HIP;
  // every workgroup must be resident at once: at most what the device holds, and no more than
  // the widest stage can use
  int64_t grid = std::min<int64_t>((int64_t)per_cu * ncu, p->gwidest);
  if (max_blocks > 0) grid = std::min<int64_t>(grid, max_blocks);
  grid = std::max<int64_t>(grid, 1);
  const GLaunchDev* ls = static_cast<const GLaunchDev*>(p->glaunch_dev);
  int32_t nl = (int32_t)p->glaunch.size();
  const GStep* st = static_cast<const GStep*>(p->gsteps);
  const GEntry* en = static_cast<const GEntry*>(p->gentries);
  const GCopy* cp = static_cast<const GCopy*>(p->gcopies);
  void* args[] = {&ls, &nl, &st, &en, &cp};
  if (hipLaunchCooperativeKernel(reinterpret_cast<const void*>(k_g_persistent), dim3((unsigned)grid),
                                 dim3(kBlock), args, 0, s) != hipSuccess) {
    (void)hipGetLastError();  // a refused launch must not fail the caller's next call
    return CT_E_HIP;
  }
  return CT_OK;
}

ct_status ct_plan_group_info(ct_plan* p, int64_t* nlaunches, int64_t* nsteps) {
  if (!p || p->grouped_ops != p->ops.size()) return CT_E_INVALID;
  if (nlaunches) *nlaunches = (int64_t)p->glaunch.size();
  if (nsteps) {
    int64_t m = 0;
    for (const ct_group::Launch& L : p->glaunch)
      if (L.stage == gReset || L.stage == gPro || L.stage == gFind) m += L.n;
    *nsteps = m;
  }
  return CT_OK;
}

ct_status ct_plan_create(ct_plan** out) {
  if (!out) return CT_E_INVALID;
  ct_plan* p = new (std::nothrow) ct_plan;
  if (!p) return CT_E_NOMEM;
  *out = p;
  return CT_OK;
}

ct_status ct_plan_destroy(ct_plan* p) {
  if (!p) return CT_E_INVALID;
  for (hipStream_t s : p->side) (void)hipStreamDestroy(s);
  for (hipEvent_t e : p->ev) (void)hipEventDestroy(e);
  delete p;
  return CT_OK;
}

ct_status ct_plan_add(ct_plan* p, ct_table* t, int32_t op, const uint64_t* keys, const void* vals,
                      void* vals_out, uint8_t* flags_out, int64_t n) {
  if (!p || !t || n < 0) return CT_E_INVALID;
  if (op < kOpClear || op > kOpErase) return CT_E_INVALID;
  const int vk = t->desc.val_kind;
  if (op != kOpClear && n > 0 && !keys) return CT_E_INVALID;
  if (op == kOpInsert && vk != CT_VAL_NONE && n > 0 && !vals) return CT_E_INVALID;
  if (op == kOpFind && vk == CT_VAL_NONE && vals_out) return CT_E_INVALID;
  if (op != kOpClear && n == 0) return CT_OK;
  p->ops.push_back(PlanOp{t, op, keys, vals, vals_out, flags_out, op == kOpClear ? 0 : n});
  if (std::find(p->tables.begin(), p->tables.end(), t) == p->tables.end()) p->tables.push_back(t);
  // the plan may run any number of times later: the host no longer bounds this table's size
  t->size_ub = (uint64_t)t->desc.capacity;
  return CT_OK;
}

ct_status ct_plan_info(ct_plan* p, int64_t* nops, int64_t* ntables) {
  if (!p) return CT_E_INVALID;
  if (nops) *nops = (int64_t)p->ops.size();
  if (ntables) *ntables = (int64_t)p->tables.size();
  return CT_OK;
}

ct_status ct_plan_launch(ct_plan* p, int32_t lanes, void* stream) {
  if (!p || lanes < 1 || lanes > 8) return CT_E_INVALID;
  ct_status r = plan_streams(p, lanes);
  if (r != CT_OK) return r;
  hipStream_t s = S(stream);
  if (hipEventRecord(p->ev[0], s) != hipSuccess) return CT_E_HIP;
  for (int32_t i = 0; i < lanes; ++i)
    if (hipStreamWaitEvent(p->side[i], p->ev[0], 0) != hipSuccess) return CT_E_HIP;
  for (const PlanOp& o : p->ops) {
    const size_t ti = (size_t)(std::find(p->tables.begin(), p->tables.end(), o.t) - p->tables.begin());
    r = run_op(o, p->side[ti % (size_t)lanes]);
    if (r != CT_OK) return r;
  }
  for (int32_t i = 0; i < lanes; ++i) {
    if (hipEventRecord(p->ev[1 + i], p->side[i]) != hipSuccess) return CT_E_HIP;
    if (hipStreamWaitEvent(s, p->ev[1 + i], 0) != hipSuccess) return CT_E_HIP;
  }
  return CT_OK;
}

ct_status ct_plan_capture(ct_plan* p, int32_t lanes, void* stream, void** graph_exec) {
  if (!p || !graph_exec || !stream || lanes < 1 || lanes > 8) return CT_E_INVALID;
  ct_status r = plan_streams(p, lanes);
  if (r != CT_OK) return r;
  hipStream_t s = S(stream);
  if (hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal) != hipSuccess) return CT_E_HIP;
  r = ct_plan_launch(p, lanes, stream);
  hipGraph_t g = nullptr;
  const hipError_t e = hipStreamEndCapture(s, &g);
  if (r != CT_OK || e != hipSuccess) {
    if (g) (void)hipGraphDestroy(g);
    return r != CT_OK ? r : CT_E_HIP;
  }
  hipGraphExec_t x = nullptr;
  const hipError_t ie = hipGraphInstantiate(&x, g, nullptr, nullptr, 0);
  (void)hipGraphDestroy(g);
  if (ie != hipSuccess) return CT_E_HIP;
  *graph_exec = x;
  return CT_OK;
}

ct_status ct_plan_capture_grouped(ct_plan* p, void* stream, void** graph_exec) {
  if (!p || !graph_exec || !stream || p->grouped_ops != p->ops.size()) return CT_E_INVALID;
  hipStream_t s = S(stream);
  if (hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal) != hipSuccess) return CT_E_HIP;
  ct_status r = ct_plan_launch_grouped(p, stream);
  hipGraph_t g = nullptr;
  const hipError_t e = hipStreamEndCapture(s, &g);
  if (r != CT_OK || e != hipSuccess) {
    if (g) (void)hipGraphDestroy(g);
    return r != CT_OK ? r : CT_E_HIP;
  }
  hipGraphExec_t x = nullptr;
  const hipError_t ie = hipGraphInstantiate(&x, g, nullptr, nullptr, 0);
  (void)hipGraphDestroy(g);
  if (ie != hipSuccess) return CT_E_HIP;
  *graph_exec = x;
  return CT_OK;
}

ct_status ct_graph_launch(void* graph_exec, void* stream) {
  if (!graph_exec) return CT_E_INVALID;
  return hipGraphLaunch(static_cast<hipGraphExec_t>(graph_exec), S(stream)) == hipSuccess ? CT_OK : CT_E_HIP;
}

ct_status ct_graph_destroy(void* graph_exec) {
  if (!graph_exec) return CT_E_INVALID;
  return hipGraphExecDestroy(static_cast<hipGraphExec_t>(graph_exec)) == hipSuccess ? CT_OK : CT_E_HIP;
}

}  // extern "C"

// ---------------------------------------------------------------------------------------------
// Allocation-free insert: the per-chunk scratch lives in a static device array, not in the
// table's buffer.  One array per GPU (each device holds its own copy), shared by every call on
// that GPU: calls that overlap on one GPU race on it.  Every kernel that needs part of it cleared
// clears it itself at the start of each chunk (the prologue kernels), so a call never depends on
// what the previous call left there.
// ---------------------------------------------------------------------------------------------
namespace {

constexpr int64_t kStaticChunk = 1 << 15;  // elements per chunk: below the binned-dedup size

struct StaticScratch {
  int64_t dd, dmark, dup, flag, ref, tsum, bcnt, total;
};

constexpr StaticScratch static_scratch_layout() {
  StaticScratch L{};
  int64_t off = 0;
  L.dd = off;
  off += 2 * kStaticChunk * 8;
  L.dmark = off;
  off += kStaticChunk;
  L.dup = off;
  off += kStaticChunk * 8;
  L.flag = off;
  off += kStaticChunk;
  L.ref = off;
  off += kStaticChunk * 8;
  L.tsum = off;
  off += 256;  // kStaticChunk / kTile tile sums, 4 bytes each
  L.bcnt = off;
  off += (int64_t)kMaxGroupBlocks * 8 + kStripeRegion;
  L.total = off;
  return L;
}

constexpr StaticScratch kStaticLayout = static_scratch_layout();
static_assert(kStaticChunk / kTile * 4 <= 256, "tile sums fit their region");
static_assert(kStaticLayout.dd % 256 == 0 && kStaticLayout.dmark % 256 == 0 &&
                  kStaticLayout.dup % 256 == 0 && kStaticLayout.flag % 256 == 0 &&
                  kStaticLayout.ref % 256 == 0 && kStaticLayout.tsum % 256 == 0 &&
                  kStaticLayout.bcnt % 256 == 0,
              "every region starts on a 256-byte boundary");

}  // namespace

static __device__ __align__(256) uint8_t scratch[kStaticLayout.total];

namespace {

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
uint8_t* g_scratch_ptr[kMaxDevices] = {};

// Device address of `scratch` on the device that runs `s`, looked up once per device with that
// device current.  The array's name is a host-side stand-in and never reaches a kernel.
ct_status scratch_for_stream(hipStream_t s, uint8_t** out) {
  int dev = -1;
  if (s) {
    if (hipStreamGetDevice(s, &dev) != hipSuccess) return CT_E_HIP;
  } else if (hipGetDevice(&dev) != hipSuccess) {
    return CT_E_HIP;
  }
  if (dev < 0 || dev >= kMaxDevices) return CT_E_INVALID;
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    int prev = -1;
    if (hipGetDevice(&prev) != hipSuccess) return CT_E_HIP;
    if (prev != dev && hipSetDevice(dev) != hipSuccess) return CT_E_HIP;
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (prev != dev) (void)hipSetDevice(prev);
    if (e != hipSuccess || !p) return CT_E_HIP;
    g_scratch_ptr[dev] = static_cast<uint8_t*>(p);
  }
  *out = g_scratch_ptr[dev];
  return CT_OK;
}

}  // namespace

extern "C" {

ct_status ct_insert_batch_noalloc(ct_table* t, const uint64_t* keys, const void* vals, int64_t n,
                                  uint8_t* status, void* stream) {
  ct_status r = check_batch(t, keys, n);
  if (r != CT_OK) return r;
  const int vk = t->desc.val_kind;
  if (vk != CT_VAL_NONE && !vals) return CT_E_INVALID;
  if (n == 0) return CT_OK;
  hipStream_t s = S(stream);
  uint8_t* base = nullptr;
  r = scratch_for_stream(s, &base);
  if (r != CT_OK) return r;
  TableView w = t->v;  // the table's slots and header, the static array's scratch
  w.dd = reinterpret_cast<uint64_t*>(base + kStaticLayout.dd);
  w.dmark = base + kStaticLayout.dmark;
  w.dup = reinterpret_cast<uint2*>(base + kStaticLayout.dup);
  w.flag = base + kStaticLayout.flag;
  w.ref = reinterpret_cast<uint64_t*>(base + kStaticLayout.ref);
  w.tsum = reinterpret_cast<uint32_t*>(base + kStaticLayout.tsum);
  w.bcnt = reinterpret_cast<int64_t*>(base + kStaticLayout.bcnt);
  w.r1k = nullptr;  // chunks below the binned size resolve repeats through dd
  w.r1i = nullptr;
  w.r2k = nullptr;
  w.r2i = nullptr;
  w.bcur = nullptr;
  w.dfirst = nullptr;
  const int64_t chunk = std::min<int64_t>(t->chunk, kStaticChunk);
  if (vk == CT_VAL_U32) return insert_chunks<1>(t, w, chunk, keys, vals, n, status, s);
  if (vk == CT_VAL_U64) return insert_chunks<2>(t, w, chunk, keys, vals, n, status, s);
  return insert_chunks<0>(t, w, chunk, keys, nullptr, n, status, s);
}

}  // extern "C"
