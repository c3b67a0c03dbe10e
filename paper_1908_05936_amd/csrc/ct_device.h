// ct_device.h -- device-side layout and wave64 helpers of the batch hash containers (gfx950).
//
// Layout of a table buffer (one caller-owned device allocation):
//   [Header, 256 B][buckets: nb x 128 B][dedup scratch, or the bins of the binned dedup with the
//   dedup scratch aliasing the coarse bins][marks][dup list][flags][refs][tile sums][block sums]
//
// Buckets.  A bucket is one 128-byte line of 8 slots {u64 key, u64 value}.  A key's probe
// sequence starts at its home bucket and steps by a key-dependent stride (double hashing) that
// visits all nb buckets, so every one of the 8*nb slots can hold any key and the fixed capacity
// of Section 4 is a hard guarantee.  Occupancy is kept in the key word with two reserved bit
// patterns, kEmpty and kTomb; the two keys that share those patterns are stored out of band in
// the header (spec_*), so every 2^64 key value stays legal (the indicator principle of
// Section 5.1 without a separate bitset).
//
// Probe rule.  A lookup scans its probe sequence and stops at the first bucket holding the key or
// holding a kEmpty slot.  Inserts claim the first free (kEmpty or kTomb) slot at or before the
// first bucket that holds a kEmpty slot, so every live key is reachable.  Erase writes kEmpty
// when its bucket already holds a kEmpty slot (no probe sequence passes such a bucket) and kTomb
// otherwise.
//
// Cooperation.  Eight lanes of a wave64 probe one key: lane j loads slot j of the bucket (one
// 16-byte load per lane, one 128-byte line per group), a ballot answers "which slot matches /
// is empty", and a shuffle broadcasts the matching value.  A wave therefore has eight keys in
// flight per step.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace ct {

constexpr uint64_t kEmpty = ~0ull;      // slot never held a key since the last clear
constexpr uint64_t kTomb = ~0ull - 1;   // slot held a key that was erased
constexpr int kSlots = 8;               // slots per bucket (one 128-byte line)
constexpr uint32_t kNone = 0xFFFFFFFFu;
constexpr uint64_t kNoPos = ~0ull;
constexpr uint64_t kSpecRef = ~0ull - 3;  // refs kSpecRef+0/+1 name the out-of-band keys
constexpr int kTile = 1024;             // elements per tile of the rank scan
constexpr int kBlock = 256;             // threads per block of every group kernel
constexpr int64_t kBinMinChunk = 1 << 16; // chunks at least this large dedup through bins
constexpr int kBinFine = 1024;          // mean elements per fine bin
constexpr uint32_t kIndirect = 0x80000000u;  // dfirst entry: names a copy whose dfirst is final
constexpr int kBinCoarse = 64;          // coarse bins
constexpr int kBinSub = 8;              // segments per coarse bin, each with its own fill count
constexpr int kCtrStride = 32;          // u32 words between coarse fill counts (one 128-byte line)
constexpr int kCoarseCtrWords = kBinCoarse * kBinSub * kCtrStride;  // fine counts follow
constexpr int kBinTile = 2048;          // elements per block of the scatter kernels
constexpr int kBinFineCap = 3072;       // entries of a fine bin (3 x the mean; more overflows)
constexpr int kBinLds = 2048;           // LDS hash slots of the fine-bin dedup: distinct keys of a
                                        // bin must be fewer (else the chunk takes the fallback)
constexpr int kMaxFinePerCoarse = 256;  // fine bins per coarse bin at the largest chunk (2^24)
constexpr int kMaxGroupBlocks = 16384;  // blocks of one insert/erase launch: its count partials
constexpr int kStripeRegion = 4096;     // behind the partials: the speculative insert's listed
                                        // counts, 32 words on separate 128-byte lines

enum : uint8_t { kPresent = 0, kInserted = 1, kFull = 2, kNoStatus = 0xFF };
enum : uint32_t { kErrFull = 1u, kErrPool = 2u, kErrInternal = 0x80000000u };

struct alignas(16) Slot {
  uint64_t key;
  uint64_t val;
};
struct alignas(128) Bucket {
  Slot s[kSlots];
};

struct alignas(256) Header {
  uint64_t size;           // live keys, out-of-band keys included
  uint64_t size0;          // size when the current chunk started
  uint64_t spec_val[2];    // values of the keys kTomb (index 0) and kEmpty (index 1)
  uint32_t spec_live[2];
  uint32_t spec_first[2];  // lowest chunk index of each out-of-band key in the current chunk
  uint32_t err;            // sticky CT_ERR_* bits
  uint32_t fast;           // 1 when the current chunk cannot reach capacity or empty the pool
  uint32_t ndup;           // duplicate elements listed for the current chunk
  uint32_t nnew;           // flagged elements of the current chunk (set by the rank scan)
  uint64_t dump_count;
  uint64_t live_count;
  uint64_t violations;
  uint32_t dmode;          // 1: the chunk's repeated keys were resolved by bins (dfirst valid)
  uint32_t dovf;           // 1: a bin of the current chunk overflowed; the chunk uses dd instead
  uint32_t dagg;           // 1: the current chunk's coarse scatter folds each tile's repeats first
  uint32_t dskew;          // 1: a recent chunk overflowed its bins (skewed keys): aggregate
  uint32_t dskew_age;      // binned chunks since dskew was set; every 16th tries without folding
  // invariant check (ct_check_invariants): duplicate keys found, pool values out of range, and
  // the multiset fingerprint of (pool entries + live values - {0 .. pool capacity - 1})
  uint64_t dup_count;
  uint64_t pool_bad;
  int64_t pool_count;
  uint64_t pool_h1, pool_h2;
  uint32_t inject;         // test hook: when nonzero, the first claim of every chunk element whose
                           // index is a multiple of it is treated as lost to another key
  uint64_t closed_count;   // health scan: buckets without an empty slot
  uint64_t tomb_count;     //              tombstone slots
  uint64_t fbd[2];         // the last insert (0) and erase (1) chunk: keys << 32 | keys stored
                           // or removed (the device copy of the feedback words)
  uint32_t spec;           // 1: the current chunk resolves repeated keys after its claims
};
static_assert(sizeof(Header) == 256, "the header fills one 256-byte line");

// A pool is a deque of int32 in a ring of `cap` entries: element x (0 = front, top - 1 = back)
// sits at stack[(head + x) mod cap].  Back operations move top; front operations move head too.
struct alignas(256) PoolHeader {
  int64_t top;   // entries in the pool
  int64_t top0;  // top when the current batch started
  int64_t cap;
  uint32_t err;
  int64_t head;  // ring position of the front element
  int64_t head0; // head when the current batch started
};

// Ring position of pool element x, for head in [0, cap) and x in [-cap, 2 cap - head).
__device__ __forceinline__ int64_t ring_pos(int64_t head, int64_t cap, int64_t x) {
  int64_t p = head + x;
  if (p >= cap) p -= cap;
  else if (p < 0) p += cap;
  return p;
}

// Everything a kernel needs to reach a table; passed by value (a shallow copy, Section 3.7).
struct TableView {
  Bucket* bk;
  uint64_t nb;
  uint64_t cap;
  Header* hdr;
  uint64_t* dd;      // dedup scratch: (fingerprint << 32 | lowest chunk index), kEmpty = free
  uint8_t* dmark;   // per chunk element: 1 = its key occurs more than once in the chunk
  uint2* dup;       // (chunk index, index of its first occurrence)
  uint8_t* flag;    // per chunk element: 1 = takes part in the rank scan
  uint64_t* ref;    // per chunk element: claimed slot, or the value an erase releases
  uint32_t* tsum;   // per tile: flagged count, then its exclusive prefix
  int64_t* bcnt;    // per block of the last insert/erase kernel: change of the live count
  // binned dedup (chunks of at least kBinMinChunk elements): elements are scattered by a hash of
  // their key into P1 coarse bins, then into P = P1 * P2 fine bins, and each fine bin resolves its
  // repeated keys in LDS.  A coarse bin is kBinSub segments: scatter block b appends to segment
  // b mod kBinSub, so each fill count takes 1/kBinSub of the blocks' reservations.  dd aliases
  // r1k: it is needed only when a bin overflows.
  uint64_t* r1k;    // coarse bin segments: keys, (P1 x kBinSub) x c1
  uint32_t* r1i;    //                      chunk indices
  uint64_t* r2k;    // fine bins: keys, P x c2
  uint32_t* r2i;
  uint32_t* bcur;   // fill counts: P1 x kBinSub coarse, kCtrStride words apart; then P fine
  uint32_t* dfirst; // per repeated element: index of its key's first occurrence
  uint32_t c1, c2;  // capacities of a coarse segment and of a fine bin
  int lp1, lp;      // log2 of P1 and of P
  uint64_t* fb;     // host-mapped word (or null): (keys << 32 | keys newly stored) of the table's
                    // last insert chunk, which the host reads to pick the next chunk's path
  int hash;         // 0 mix64, 1 voxel21
  int nb_pow2;
  int step_mode;    // probe step between buckets: 0 linear (1), 1 odd (nb a power of two),
                    // 2 any in [1, nb) (nb prime); every mode visits all nb buckets
};

// ---------------------------------------------------------------------------------------------
// hashes
// ---------------------------------------------------------------------------------------------
__device__ __forceinline__ uint64_t fmix64(uint64_t k) {  // MurmurHash3 finaliser (Appleby)
  k ^= k >> 33;
  k *= 0xff51afd7ed558ccdull;
  k ^= k >> 33;
  k *= 0xc4ceb9fe1a85ec53ull;
  k ^= k >> 33;
  return k;
}

__device__ __forceinline__ int32_t sfield21(uint64_t v) {  // low 21 bits, sign-extended
  return ((int32_t)((uint32_t)v << 11)) >> 11;
}

// Spatial hash of Section 4.1 on a packed int3 key, as the 64-bit size_t the listing returns.
__device__ __forceinline__ uint64_t voxel21(uint64_t key) {
  const uint32_t x = (uint32_t)sfield21(key);
  const uint32_t y = (uint32_t)sfield21(key >> 21);
  const uint32_t z = (uint32_t)sfield21(key >> 42);
  const uint32_t h = (x * 73856093u) ^ (y * 19349669u) ^ (z * 83492791u);
  return (uint64_t)(int64_t)(int32_t)h;
}

// Home bucket and probe step of a key.  The probe sequence is home, home+step, home+2*step, ...
// (mod nb): double hashing, so displaced keys of neighbouring homes do not pile up into long
// runs, and a step coprime with nb visits every bucket (the capacity guarantee).
struct Seq {
  uint64_t home;
  uint64_t step;
};

__device__ __forceinline__ Seq probe_seq(const TableView& t, uint64_t key) {
  const uint64_t mix = fmix64(key);
  Seq r;
  if (t.hash == 1) {
    const uint64_t h = voxel21(key);
    r.home = t.nb_pow2 ? (h & (t.nb - 1)) : (h % t.nb);
  } else {
    r.home = __umul64hi(mix, t.nb);
  }
  const uint64_t rot = (mix << 32) | (mix >> 32);
  if (t.step_mode == 1) r.step = (rot | 1ull) & (t.nb - 1);
  else if (t.step_mode == 2) r.step = 1 + __umul64hi(rot, t.nb - 1);
  else r.step = 1;
  if (t.nb == 1) r.step = 0;
  return r;
}

__device__ __forceinline__ uint64_t dedup_mix(uint64_t key) {
  return fmix64(key ^ 0x9E3779B97F4A7C15ull);
}

__device__ __forceinline__ uint64_t next_bucket(const TableView& t, uint64_t b, uint64_t step) {
  b += step;
  return b >= t.nb ? b - t.nb : b;
}

// ---------------------------------------------------------------------------------------------
// wave64 group helpers: 8 groups of 8 lanes per wave
// ---------------------------------------------------------------------------------------------
__device__ __forceinline__ int wave_lane() { return (int)(threadIdx.x & 63); }
__device__ __forceinline__ int group_base() { return wave_lane() & ~7; }
__device__ __forceinline__ uint32_t group_bits(uint64_t ballot) {
  return (uint32_t)(ballot >> group_base()) & 0xFFu;
}
__device__ __forceinline__ int lowest(uint32_t m) { return __builtin_ctz(m); }

// ---------------------------------------------------------------------------------------------
// atomics with explicit order and scope.  Claims are relaxed at agent scope: a claim only has to
// be unique, and the results of a batch are read after the kernel boundary that ends it.
// ---------------------------------------------------------------------------------------------
__device__ __forceinline__ bool cas64(uint64_t* p, uint64_t& expected, uint64_t desired) {
  return __hip_atomic_compare_exchange_strong(p, &expected, desired, __ATOMIC_RELAXED,
                                              __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ uint32_t amin32(uint32_t* p, uint32_t v) {
  return __hip_atomic_fetch_min(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ uint64_t amin64(uint64_t* p, uint64_t v) {
  return __hip_atomic_fetch_min(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ uint32_t aadd32(uint32_t* p, uint32_t v) {
  return __hip_atomic_fetch_add(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ uint64_t aadd64(uint64_t* p, uint64_t v) {
  return __hip_atomic_fetch_add(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ uint32_t aor32(uint32_t* p, uint32_t v) {
  return __hip_atomic_fetch_or(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Reserve a position in an append-only list for every active lane with `pred`, one atomic per wave.
__device__ __forceinline__ uint32_t wave_append(bool pred, uint32_t* counter) {
  const uint64_t m = __ballot(pred);
  uint32_t base = 0;
  if (m) {
    const int leader = __builtin_ctzll(m);
    if (wave_lane() == leader) base = aadd32(counter, (uint32_t)__builtin_popcountll(m));
    base = __shfl(base, leader, 64);
  }
  return base + (uint32_t)__builtin_popcountll(m & ((1ull << wave_lane()) - 1ull));
}

// Sum of `v` over the wave; call with every lane of the wave active.
__device__ __forceinline__ uint64_t wave_sum(uint64_t v) {
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}

// Sum of `v` over a block of NT threads, returned to thread 0; call with every thread active.
template <int NT = kBlock>
__device__ __forceinline__ int64_t block_sum(int64_t v) {
  __shared__ int64_t part[NT / 64];
  v = (int64_t)wave_sum((uint64_t)v);
  if (wave_lane() == 0) part[threadIdx.x >> 6] = v;
  __syncthreads();
  int64_t s = 0;
  if (threadIdx.x == 0)
    for (int w = 0; w < NT / 64; ++w) s += part[w];
  return s;
}

}  // namespace ct
