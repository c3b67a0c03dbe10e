/*
 * ct.h -- C ABI of the batch hash containers and index pool for AMD MI355X (gfx950).
 *
 * The containers follow the paper's STL-like containers: unordered_map / unordered_set
 * (Section 4.1) and the vector / deque back operations (Sections 4.2 and 4.3), whose design
 * decisions are given at the start of Section 4 (fixed capacity; insert and erase as the central
 * operations; lock-free, non-blocking lookups; inserting beyond capacity as the only failure).
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 *  * Counts are int64_t (the paper's signed index type, Section 3.2).  A negative count is an
 *    argument error; a zero count is a no-op that returns CT_OK.
 *  * Key, value, status and index arrays are DEVICE pointers owned by the caller.  Inputs must not
 *    alias outputs.  Output pointers documented as nullable may be NULL to skip that output.
 *  * `stream` is a hipStream_t passed as void* (NULL = the default stream).  Batch calls only
 *    enqueue work and return; calls documented as "synchronises" wait for `stream`.
 *  * Calls on one table (or pool) must be ordered on one stream by the caller; different tables
 *    are independent and may run concurrently on different streams.
 *  * Argument errors are detected on the host before anything is enqueued and return
 *    CT_E_INVALID; a failed HIP launch returns CT_E_HIP.  Per-element outcomes (FULL, pool empty)
 *    are reported in the status arrays and OR-ed into a sticky device error word (ct_get_error).
 *  * Every 2^64 key value is a legal key: occupancy is kept without reserving key values
 *    (the indicator principle of Section 5.1).
 *  * Memory order: inside a batch, slots are claimed with relaxed compare-and-swap at device
 *    (agent) scope; a claim only has to be unique.  Equal keys of one batch are resolved to their
 *    lowest index either before any claim, or (speculative inserts, ct_table_set_insert_path)
 *    after the claiming kernel has ended, from the copies that met their key; in both cases the
 *    order comes from kernel boundaries, not from fences.  Batches are ordered by the stream: the
 *    outputs of a call, and the table state it leaves, are visible to work enqueued after it on
 *    the same stream (or after an event that follows it); the host sees them after synchronising.
 *
 * Batch semantics
 * ---------------
 * A batch of n elements gives exactly the results of n single-element calls made one after the
 * other in index order.  So among equal keys in one batch the lowest index acts first and later
 * copies see the state it left; a key that is already present is never modified by insert.
 *
 * Memory
 * ------
 * A table or pool lives in one caller-provided device buffer of the size reported by
 * ct_table_bytes / ct_pool_bytes, at least 256-byte aligned.  The buffer holds the slots, the
 * counters and the per-batch scratch; the library allocates no device memory.  The handle returned
 * by the init call is host memory owned by the library until the matching destroy call.
 */
#ifndef CT_H
#define CT_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum ct_status {
    CT_OK = 0,
    CT_E_INVALID = 1, /* bad argument; nothing was enqueued */
    CT_E_FULL = 2,    /* ct_table_rehash: the destination lacks room; otherwise reserved for
                         callers mapping the sticky error word */
    CT_E_EMPTY = 3,   /* reserved for callers mapping the sticky error word */
    CT_E_NOMEM = 4,   /* host allocation of a handle failed */
    CT_E_HIP = 5      /* a HIP runtime call or kernel launch failed */
} ct_status;

/* Per-element insert status (status arrays of ct_insert_batch / ct_insert_alloc_batch). */
#define CT_PRESENT 0u  /* key was already present; nothing modified (Section 4.1, insert) */
#define CT_INSERTED 1u /* key stored */
#define CT_FULL 2u     /* capacity (or the pool) exhausted: the only failure case (Section 4) */

/* Bits of the sticky device error word. */
#define CT_ERR_FULL 1u      /* an insert met a full table */
#define CT_ERR_POOL 2u      /* a pool ran empty (pop) or over capacity (push) */
#define CT_ERR_INTERNAL 0x80000000u /* an internal consistency check failed (a library bug) */

typedef enum ct_val_kind {
    CT_VAL_NONE = 0, /* unordered_set: keys only */
    CT_VAL_U32 = 1,  /* unordered_map with 32-bit mapped values */
    CT_VAL_U64 = 2   /* unordered_map with 64-bit mapped values */
} ct_val_kind;

typedef enum ct_hash_kind {
    CT_HASH_MIX64 = 0,  /* MurmurHash3 64-bit finaliser, multiply-high reduction: generic keys */
    CT_HASH_VOXEL21 = 1 /* spatial hash of Section 4.1 on packed signed 21-bit int3 keys:
                           (x*73856093 ^ y*19349669 ^ z*83492791) in 32-bit wrapping int
                           arithmetic, sign-extended to 64 bits, modulo bucket_count.
                           Packing: x bits 0-20, y bits 21-41, z bits 42-62. */
} ct_hash_kind;

/* Table description. */
typedef struct ct_table_desc {
    int64_t capacity;     /* C: number of distinct keys guaranteed storable whatever their hashes
                             (the fixed capacity of Section 4).  C >= 0. */
    int32_t val_kind;     /* ct_val_kind */
    int32_t hash_kind;    /* ct_hash_kind */
    int64_t bucket_count; /* buckets of 8 slots each (one 128-byte line); 0 = the smallest prime
                             >= ceil(C / 8).  Must satisfy 8 * bucket_count >= C and
                             bucket_count >= 1.  Probing steps between buckets by a per-key
                             stride (double hashing) when the count is prime or a power of two,
                             and by 1 otherwise. */
    int64_t chunk;        /* keys handled per internal insert/erase chunk; a power of two in
                             [1024, 2^24]; 0 = the largest power of two <= C/8, clamped to
                             [1024, 2^23].  Batches larger than a chunk run as consecutive chunks
                             (same results).  The table buffer holds about 34 bytes of scratch
                             per chunk element below 2^16, and 82-109 for larger chunks, which
                             resolve repeated keys through bins (ct_table_bytes is exact). */
} ct_table_desc;

typedef struct ct_table ct_table;
typedef struct ct_pool ct_pool;

/* --- tables ------------------------------------------------------------------------------- */

/* Bytes of device memory a table with description `d` needs.  Host only. */
ct_status ct_table_bytes(const ct_table_desc *d, int64_t *bytes);

/* Create an empty table in `d_buf` (device, `bytes` >= ct_table_bytes, 256-byte aligned) and
   return its handle in *out.  Enqueues the initialisation on `stream` (createDeviceObject,
   Section 3.7). */
ct_status ct_table_init(void *d_buf, int64_t bytes, const ct_table_desc *d, void *stream,
                        ct_table **out);

/* Release the host handle (destroyDeviceObject, Section 3.7).  The device buffer stays owned by
   the caller; work already enqueued must have finished before the buffer is reused. */
ct_status ct_table_destroy(ct_table *t);

/* Geometry of a table: home buckets and chunk size (host only, either pointer nullable). */
ct_status ct_table_info(const ct_table *t, int64_t *bucket_count, int64_t *chunk);

/* Bytes per mapped value: 0 for a set, 4 for CT_VAL_U32, 8 for CT_VAL_U64.  Host only. */
ct_status ct_table_value_bytes(const ct_table *t, int32_t *bytes);

/* Iterator-based insert of an array (Section 4.1, insert).  keys[n] u64; vals[n] u32 or u64 by the
   table's value kind (ignored and nullable for sets, required otherwise).  status[n] (nullable):
   CT_PRESENT, CT_INSERTED or CT_FULL per element. */
ct_status ct_insert_batch(ct_table *t, const uint64_t *keys, const void *vals, int64_t n,
                          uint8_t *status, void *stream);

/* ct_insert_batch for callers that cannot allocate device memory, or must not do so while they
   run (code under HIP graph capture, tight serving loops, harnesses that forbid allocation).  Same
   arguments, same results and the same table as ct_insert_batch, but the per-chunk scratch
   (repeated-key table, marks, lists, rank sums, count partials: about 1.2 MiB) lives in one static
   device array per GPU instead of the table buffer, and no call allocates anything.  The batch
   runs in chunks of at most 2^15 elements, the largest the array holds, so every batch size is
   accepted.  Every call on one GPU shares that GPU's array: calls that overlap on one GPU (other
   streams, other threads, other tables) race on it and must be serialised by the caller.  The
   array keeps the last call's contents; each chunk clears what it needs itself.  CT_E_HIP when
   the array's device address cannot be obtained. */
ct_status ct_insert_batch_noalloc(ct_table *t, const uint64_t *keys, const void *vals, int64_t n,
                                  uint8_t *status, void *stream);

/* find / contains (Section 4.1) for an array.  vals_out[n] (nullable; u32 or u64 by value kind;
   not allowed for sets) receives the mapped value, or all-ones of the value width when the key is
   absent; found[n] (nullable) receives 1 when present, else 0.  Read-only and lock-free. */
ct_status ct_find_batch(ct_table *t, const uint64_t *keys, int64_t n, void *vals_out,
                        uint8_t *found, void *stream);

/* erase (Section 4.1) for an array.  erased[n] (nullable): 1 if the key was present before this
   element, else 0. */
ct_status ct_erase_batch(ct_table *t, const uint64_t *keys, int64_t n, uint8_t *erased,
                         void *stream);

/* Number of live keys.  Synchronises `stream`. */
ct_status ct_size(ct_table *t, int64_t *h_size, void *stream);

/* Remove every key (capacity unchanged; Section 4 "Capacity").  The pool, if any, is untouched. */
ct_status ct_clear(ct_table *t, void *stream);

/* Copy the live (key, value) pairs in unspecified order into keys_out/vals_out (device,
   `cap` entries; vals_out nullable, ignored for sets; values written as u64) and return the live
   count in *h_count (which may exceed `cap`; only `cap` pairs are written).  Synchronises.  The
   range-to-vector selection of Section 3.6. */
ct_status ct_dump(ct_table *t, uint64_t *keys_out, uint64_t *vals_out, int64_t cap,
                  int64_t *h_count, void *stream);

/* Range selection (Section 3.6: a range of the container turned into a vector with a copy_if):
   copy the live (key, value) pairs whose key the predicate accepts into keys_out / vals_out
   (device, `cap` entries; vals_out nullable, ignored for sets; values as u64), in unspecified
   order, and return the number selected in *h_count (only `cap` pairs are written).
   Synchronises.
   ct_select_key_range: lo <= key < hi, unsigned.
   ct_select_voxel_box: the key packs signed 21-bit block coordinates (x bits 0-20, y 21-41,
   z 42-62, bit 63 clear) and each lies in [h_lo3[d], h_hi3[d]] (host arrays of 3, bounds
   included); a key with bit 63 set packs no block and is never selected. */
ct_status ct_select_key_range(ct_table *t, uint64_t lo, uint64_t hi, uint64_t *keys_out,
                              uint64_t *vals_out, int64_t cap, int64_t *h_count, void *stream);
ct_status ct_select_voxel_box(ct_table *t, const int32_t *h_lo3, const int32_t *h_hi3,
                              uint64_t *keys_out, uint64_t *vals_out, int64_t cap,
                              int64_t *h_count, void *stream);

/* Check the table's invariants on the device (the uniqueness of Section 4.1 and the contracts of
   Section 3.3 stated for this layout) and return the number of failures in *h_violations
   (0 = consistent).  Checked:
     CT_CHECK_SIZE       the size counter equals the number of live slots (out-of-band keys
                         included) and does not exceed the capacity;
     CT_CHECK_DUPLICATE  no key is stored twice (a second copy of a key lies on the same probe
                         path, so the walk from a copy's home bucket would pass the other);
     CT_CHECK_REACH      every live key is reachable: no bucket between its home bucket and its
                         own holds an empty slot, so find would see it;
     CT_CHECK_POOL       with `p` (nullable; only for CT_VAL_U32 tables whose values are pool
                         indices, as insert_alloc / erase_release keep them): the pool's entries
                         and the table's live values together hold every index 0 .. capacity(p)-1
                         exactly once (no leaked or duplicated index).  This is tested with two
                         independent 64-bit multiset fingerprints and a count, which any missing,
                         repeated or foreign index changes except with probability about 2^-64.
   Uses the table's header words only: no scratch.  Synchronises `stream`.  CT_E_INVALID for a
   pool with a table that is not CT_VAL_U32. */
#define CT_CHECK_SIZE 1u
#define CT_CHECK_DUPLICATE 2u
#define CT_CHECK_REACH 12u  /* an unreachable key is also not findable: two bits, as the oracle */
#define CT_CHECK_POOL 32u
ct_status ct_check_invariants(ct_table *t, const ct_pool *p, int64_t *h_violations, void *stream);

/* The same check, with the CT_CHECK_* bits of the failed invariants in *h_what (nullable). */
ct_status ct_check_invariants_detail(ct_table *t, const ct_pool *p, int64_t *h_violations,
                                     uint32_t *h_what, void *stream);

/* Table health: *h_closed (nullable) = buckets without an empty slot, *h_tombstones (nullable) =
   slots holding a tombstone.  An erase leaves a tombstone where its bucket holds no empty slot;
   inserts reuse tombstones, but nothing else turns them back into empty slots, so after long
   churn near full load more buckets close, and a lookup of an absent key walks past closed
   buckets until it meets an open one (every bucket when none is open).  Synchronises. */
ct_status ct_table_health(ct_table *t, int64_t *h_closed, int64_t *h_tombstones, void *stream);

/* Reopen buckets in place: every bucket that no live key's probe path passes (no live key lies
   further along a path that runs through it) gets its tombstones turned into empty slots.  Keys,
   values, size and every result are unchanged; lookups of absent keys and inserts stop earlier
   afterwards.  Uses the table's per-batch scratch as a bitmap of buckets (several passes over the
   slots when that scratch holds fewer bits than buckets).  Asynchronous on `stream`; must not
   overlap other calls on the table. */
ct_status ct_table_purge(ct_table *t, void *stream);

/* Host-side resizing (a capacity is fixed at creation, Section 4; growth is a copy into a larger
   table): insert every live (key, value) of `src` into `dst`, which must have the same value kind
   and room for all of them (capacity(dst) >= size(dst) + size(src), else CT_E_FULL and nothing
   is enqueued).  Keys `dst` already holds keep their value there.  `src` is unchanged.  Reads both
   sizes (synchronises `stream`), then runs asynchronously on `stream`.  With a new empty `dst`
   this is a rehash into a larger table; with a dump and an insert it is also how a table is
   snapshot and restored. */
ct_status ct_table_rehash(ct_table *src, ct_table *dst, void *stream);

/* --- device-side per-thread operations (Section 4.1: container functions called inside
   kernels, one element per thread; Section 4: concurrency across the operations) ------------ */

#define CT_DEV_READ 0   /* find / contains only */
#define CT_DEV_INSERT 1 /* insert, find, contains; the same key from several threads allowed */
#define CT_DEV_ERASE 2  /* erase, find, contains */
#define CT_DEV_MIXED 3  /* insert, erase, find, contains together; erases leave tombstones only */

/* Fill `out` (at least `bytes` bytes, host memory) with the by-value view a user kernel passes to
   the device functions of paper_1908_05936_amd/csrc/ct_dev_api.h (dev_insert, dev_erase,
   dev_find, dev_contains), for one kernel that uses the table in `mode`.  Inserts and erases share
   a kernel only in CT_DEV_MIXED; within a mode every operation may run concurrently from any
   thread (the header states the guarantees).  Host only; CT_E_INVALID if `bytes` is too small or
   `mode` unknown. */
ct_status ct_table_device_view(ct_table *t, int32_t mode, void *out, int64_t bytes);

/* The reference user kernel of the device functions: element i of keys[n] is handled by one
   thread, all concurrently, in no particular order.  op CT_OP_INSERT (vals in the table's value
   width; status[i] 0 PRESENT / 1 INSERTED / 2 FULL: each new key is INSERTED by exactly one of
   its elements, whose value it keeps), CT_OP_ERASE (status[i] 1 for exactly one element of each
   present key), CT_OP_FIND (status[i] found; vals_out as ct_find_batch).  status and vals_out
   nullable.  Asynchronous on `stream`. */
ct_status ct_dev_apply(ct_table *t, int32_t op, const uint64_t *keys, const void *vals, int64_t n,
                       void *vals_out, uint8_t *status, void *stream);

/* The same reference kernel in CT_DEV_MIXED (Section 4: concurrency across all operations):
   element i does operation ops[i] (device array of CT_OP_INSERT / CT_OP_FIND / CT_OP_ERASE) on
   keys[i], every element concurrently, the same key under several operations included.  vals
   (device, the table's value width; required for a map) is read at insert elements; status[i] as
   in ct_dev_apply for the element's operation, 255 for an unknown code (the table untouched);
   vals_out[i] (nullable) holds the found value at find elements and the absent sentinel
   elsewhere.  Per key, INSERTED results and successful erases alternate, starting from the key's
   state before the kernel.  Erases leave tombstones, which later batch inserts reuse.  The live
   count is exact when the kernel ends; at capacity it can pass the capacity by the number of
   keys that an erase removed between their insert's claim and its count.  Asynchronous on
   `stream`. */
ct_status ct_dev_apply_mixed(ct_table *t, const uint8_t *ops, const uint64_t *keys, const void *vals,
                             int64_t n, void *vals_out, uint8_t *status, void *stream);

/* Neighbour update of a voxel-block map through the device functions (the allocation step of the
   reconstruction workload behind Section 4.1's block map): every packed block of blocks[n] makes
   sure that its 6 face neighbours (ndirs 6) or all 26 neighbours (ndirs 26) are in the table, a
   new one with the index of a block that asked for it as its value (which one is not fixed).
   Coordinates wrap in their 21-bit fields.  The table needs room for every new key (else some
   are left out and the size stays at capacity).  Asynchronous on `stream`. */
ct_status ct_voxel_insert_neighbours(ct_table *t, const uint64_t *blocks, int64_t n, int32_t ndirs,
                                     void *stream);

/* The same with the index pool: a new neighbour block takes pop_back() of `p` as its value (the
   block map of Section 4.1 fed by the free list, as a reconstruction allocates blocks).  A block
   that finds no capacity or an empty pool is left out (CT_ERR_POOL set when the pool ran out). */
ct_status ct_voxel_insert_neighbours_alloc(ct_table *t, ct_pool *p, const uint64_t *blocks,
                                           int64_t n, int32_t ndirs, void *stream);

/* The two-container step of Section 4.1's reconstruction example, through the device functions
   in one kernel: for every key of keys[n] (device), one thread asks `map` whether it holds the key
   (dev_contains, read-only) and, if so, inserts it into `set` (dev_insert; many threads may insert
   one key, it is stored once).  status[n] (nullable): 255 when `map` lacks the key, else the set
   insert's CT_PRESENT / CT_INSERTED / CT_FULL (exactly one element of each new key reads
   CT_INSERTED).  `map` and `set` must be different tables; `set` may be of any value kind (values
   are stored as 0).  Asynchronous on `stream`. */
ct_status ct_dev_update_set(ct_table *map, ct_table *set, const uint64_t *keys, int64_t n,
                            uint8_t *status, void *stream);

/* Device-side vector / deque back operations on a pool (Sections 4.2-4.3: push_back / pop_back
   from threads).  ct_pool_device_view fills the by-value pool view of the device functions
   dev_push_back / dev_pop_back (paper_1908_05936_amd/csrc/ct_dev_api.h); a kernel either pushes
   or pops.  ct_dev_pool_apply is their reference kernel: element i by one thread, all
   concurrently; status[i] 1 done / 2 full or empty; popped values in out[i] (-1 when empty): the
   pops together take the pool's last min(n, size) entries, in no fixed order. */
#define CT_DEV_PUSH_BACK 0
#define CT_DEV_POP_BACK 1
ct_status ct_pool_device_view(ct_pool *p, void *out, int64_t bytes);
ct_status ct_dev_pool_apply(ct_pool *p, int32_t op, const int32_t *in, int64_t n, int32_t *out,
                            uint8_t *status, void *stream);

/* Read and clear the sticky error word (CT_ERR_* bits).  Synchronises. */
ct_status ct_get_error(ct_table *t, uint32_t *h_err, void *stream);

/* Test hook, not for production use: from now on (clear keeps it, 0 switches it off), the first
   claim attempt of every insert element whose index within its chunk is a multiple of `every` is
   treated as lost to another key, as when a concurrent insert took the slot first (the rare
   failed attempt of Section 4 that further attempts resolve).  The slot stays free, so the
   element's retry path claims it; results are unchanged.  Also applies to ct_table_rehash into
   this table (by source slot).  Enqueued on `stream`. */
ct_status ct_table_debug_inject_claim_losses(ct_table *t, uint32_t every, void *stream);

/* Diagnostic: *h_skewed = 1 when a recent chunk of this table overflowed its dedup bins (keys
   repeated thousands of times), so its large chunks fold each tile's repeated keys before binning;
   0 otherwise.  Results never depend on it.  Synchronises. */
ct_status ct_table_dedup_skewed(ct_table *t, int32_t *h_skewed, void *stream);

/* How insert and erase chunks resolve repeated keys (the index order of the batch semantics
   above).  For inserts, only chunks that the host can prove cannot reach capacity have a choice;
   the others, ct_insert_alloc_batch and ct_erase_release_batch always resolve repeated keys
   first.
   CT_INSERT_SPECULATIVE: every element acts for itself (an insert claims a slot with one CAS, an
   erase removes the key it finds with one CAS), and only the elements that met their key in the
   table, lost that CAS to a copy of their key, or (erase) found nothing are resolved afterwards,
   by lowest index.  A batch of distinct new keys to insert, or of distinct present keys to erase,
   then needs no resolution pass at all.
   CT_INSERT_RESOLVE_FIRST: repeated keys are resolved before the table is touched, so only one
   copy of each key probes it (cheaper when most keys are present or repeated, or absent from an
   erase).
   CT_INSERT_AUTO (the default): speculative while the table's last chunk of the same operation
   stored (erase: removed) at least half of its keys, else resolve first; the table reports each
   chunk through a word of pinned host memory that the host reads without synchronising.  A clear
   starts a fresh history (the next chunks speculate).  Results are identical on every path.
   Host only: applies to calls enqueued afterwards, and to grouped plans built afterwards
   (ct_plan_group records each table's path; the grouped steps then decide on the device, from the
   table's size and last chunks when the step starts, so replays decide afresh). */
#define CT_INSERT_AUTO 0
#define CT_INSERT_RESOLVE_FIRST 1
#define CT_INSERT_SPECULATIVE 2
ct_status ct_table_set_insert_path(ct_table *t, int32_t path);

/* --- index pool: vector/deque of int32 used as a LIFO free list (Sections 4.2, 4.3) -------- */

/* Bytes of device memory a pool of `capacity` int32 entries needs.  Host only. */
ct_status ct_pool_bytes(int64_t capacity, int64_t *bytes);

/* Create a full pool in `d_buf`: it holds 0 .. capacity-1 and pops return 0, 1, 2, ... */
ct_status ct_pool_init(void *d_buf, int64_t bytes, int64_t capacity, void *stream, ct_pool **out);

ct_status ct_pool_destroy(ct_pool *p);

/* pop_back n times (Section 4.2: pop_back returns the removed value).  out[n] (nullable) gets the
   value or -1 once the pool is empty; status[n] (nullable) 1 = popped, 2 = empty. */
ct_status ct_pool_pop_batch(ct_pool *p, int64_t n, int32_t *out, uint8_t *status, void *stream);

/* push_back in[0..n) in order (Section 4.2).  status[n] (nullable) 1 = stored, 2 = the pool was
   at capacity (value dropped, CT_ERR_POOL set). */
ct_status ct_pool_push_batch(ct_pool *p, const int32_t *in, int64_t n, uint8_t *status,
                             void *stream);

/* Deque front operations (Section 4.3: the deque also inserts and removes at its front).  The
   pool is a double-ended queue whose back the operations above use; a fresh pool's front holds
   capacity-1.  pop_front n times: out[n] (nullable) gets the removed first element or -1 once the
   pool is empty; status[n] (nullable) 1 = popped, 2 = empty (CT_ERR_POOL set).  With push_back
   this is a first-in first-out free list. */
ct_status ct_pool_pop_front_batch(ct_pool *p, int64_t n, int32_t *out, uint8_t *status,
                                  void *stream);

/* push_front in[0..n) in order: each value goes in front of the previous one, so in[n-1] ends
   up first.  status[n] (nullable) 1 = stored, 2 = the pool was at capacity (value dropped,
   CT_ERR_POOL set). */
ct_status ct_pool_push_front_batch(ct_pool *p, const int32_t *in, int64_t n, uint8_t *status,
                                   void *stream);

/* Number of entries in the pool.  Synchronises. */
ct_status ct_pool_size(ct_pool *p, int64_t *h_size, void *stream);

/* Copy the pool front first (the stack bottom first) into out (device, `cap` entries) and return
   the entry count in *h_count.  Synchronises. */
ct_status ct_pool_dump(ct_pool *p, int32_t *out, int64_t cap, int64_t *h_count, void *stream);

/* Read and clear the pool's sticky error word.  Synchronises. */
ct_status ct_pool_get_error(ct_pool *p, uint32_t *h_err, void *stream);

/* --- tables whose values come from a pool (block map of Section 4.1: key -> block index) --- */

/* Insert of an array into a CT_VAL_U32 table where every new key takes pop_back() of `p` as its
   value, new keys taking pool entries in batch order.  vals_out[n] (nullable, int32): the new or
   existing value, -1 on FULL.  status[n] (nullable): CT_PRESENT / CT_INSERTED / CT_FULL, FULL
   when the table is at capacity or the pool is empty. */
ct_status ct_insert_alloc_batch(ct_table *t, ct_pool *p, const uint64_t *keys, int64_t n,
                                int32_t *vals_out, uint8_t *status, void *stream);

/* ct_insert_alloc_batch of the elements i with skip[i] == 0 only (skip[n], device, required):
   the same results as ct_insert_alloc_batch of those keys gathered in index order, written back to
   their positions; vals_out[i] and status[i] of skipped elements are left untouched.  Passing the
   `found` array of a ct_find_batch of the same keys inserts the keys the find missed (the
   allocation step of the reconstruction use of Section 4.1), with no host round trip to count
   or compact them. */
ct_status ct_insert_alloc_batch_masked(ct_table *t, ct_pool *p, const uint64_t *keys,
                                       const uint8_t *skip, int64_t n, int32_t *vals_out,
                                       uint8_t *status, void *stream);

/* Erase of an array where each removed key's value is pushed back to `p`, in batch order.
   erased[n] nullable as for ct_erase_batch. */
ct_status ct_erase_release_batch(ct_table *t, ct_pool *p, const uint64_t *keys, int64_t n,
                                 uint8_t *erased, void *stream);

/* --- multi-table plans: a schedule of operations over many tables ------------------------- */
/* A plan records operations on many tables in schedule order and replays them: operations on one
   table keep their order (the results equal those of the single-table calls made in that order)
   and tables are spread over up to 8 side streams forked from the caller's stream and joined
   back, so operations on different tables overlap on the device.  Each operation runs the same
   kernel pipeline as its single-table call.  The fork/join sequence captures into one HIP graph
   that replays the whole schedule with one call.  The caller keeps every table and array a plan
   names alive and unchanged in place until the last run of the plan ends. */

#define CT_OP_CLEAR 0  /* remove every key of the table (no arrays) */
#define CT_OP_INSERT 1 /* keys, vals (in), flags_out = status */
#define CT_OP_FIND 2   /* keys, vals_out, flags_out = found */
#define CT_OP_ERASE 3  /* keys, flags_out = erased */

typedef struct ct_plan ct_plan;

ct_status ct_plan_create(ct_plan **out);
ct_status ct_plan_destroy(ct_plan *p);

/* Append one operation (host only; arrays as in the single-table calls, nullable outputs as
   there). */
ct_status ct_plan_add(ct_plan *p, ct_table *t, int32_t op, const uint64_t *keys, const void *vals,
                      void *vals_out, uint8_t *flags_out, int64_t n);

/* Number of recorded operations and of distinct tables. */
ct_status ct_plan_info(ct_plan *p, int64_t *nops, int64_t *ntables);

/* Run the plan after the work already on `stream`, with tables spread over `lanes` (1..8) side
   streams; `stream` waits for all of it.  Enqueues only. */
ct_status ct_plan_launch(ct_plan *p, int32_t lanes, void *stream);

/* Capture ct_plan_launch(p, lanes) on `stream` (a non-default stream) into an executable HIP
   graph returned in *graph_exec; replay it with ct_graph_launch and free it with
   ct_graph_destroy. */
ct_status ct_plan_capture(ct_plan *p, int32_t lanes, void *stream, void **graph_exec);
ct_status ct_graph_launch(void *graph_exec, void *stream);
ct_status ct_graph_destroy(void *graph_exec);

/* Grouped form of a plan: one kernel launch per pipeline stage covers that stage for many tables.
   Insert and erase operations are cut into chunk-steps of their table's chunk; the k-th step of
   every table forms level k, and each level runs the pipeline stages (reset, prologue, dedup,
   find / insert / erase, count update, rank scan, ranked completion, repeated-key outcomes) as
   one launch each over all of its steps.  Steps of one level touch different tables, so a table's
   steps still run in schedule order and every result equals that of the single-table calls.
   The step descriptors live in a caller-provided device buffer. */

/* Options of the grouped form. */
#define CT_GROUP_MERGE_RUNS 1 /* a run of consecutive operations of one kind on one table runs as
                                 one operation over a contiguous copy of its arrays (gathered from
                                 the operations' arrays before the first level and scattered back
                                 after the last): fewer, larger steps and levels, for up to
                                 (8 + 2 value widths + 1) bytes per merged element of device
                                 memory in the grouped form's buffer */

#define CT_GROUP_BLOCK_SHIFT 8  /* options bits 8-11: log2 of the threads per block of the
                                  find / insert / erase stages, 7 .. 10 (128 .. 1024); 0 = 256 */
#define CT_GROUP_BLOCK(threads) ((threads) == 128 ? (7 << 8) : (threads) == 512 ? (9 << 8) : \
                                 (threads) == 1024 ? (10 << 8) : 0)

/* Bytes of device memory the grouped form of `p` with `options` needs (host only). */
ct_status ct_plan_group_bytes(ct_plan *p, int32_t options, int64_t *bytes);

/* Build the grouped form of `p` into `d_buf` (device, `bytes` >= ct_plan_group_bytes with the
   same options, 256-byte aligned, owned by the caller and kept alive and unmodified while the
   grouped form is used).  Copies synchronously.  Adding an operation to `p` afterwards
   invalidates the grouped form (launching it then returns CT_E_INVALID until it is built again). */
ct_status ct_plan_group(ct_plan *p, int32_t options, void *d_buf, int64_t bytes);

/* Launches and steps of the grouped form (either pointer nullable). */
ct_status ct_plan_group_info(ct_plan *p, int64_t *nlaunches, int64_t *nsteps);

/* Run the grouped form on `stream` after the work already there.  Enqueues only. */
ct_status ct_plan_launch_grouped(ct_plan *p, void *stream);

/* Capture ct_plan_launch_grouped(p) on `stream` (a non-default stream) into an executable HIP
   graph, replayed with ct_graph_launch and freed with ct_graph_destroy. */
ct_status ct_plan_capture_grouped(ct_plan *p, void *stream, void **graph_exec);

/* The grouped form of `p` as ONE kernel launch (a cooperative launch: every workgroup of its grid
   is resident at once).  The grid runs the stage launches of ct_plan_launch_grouped in order:
   within a stage its workgroups take the stage's blocks in turn, and a grid-wide barrier (with
   device-scope fences) separates consecutive stages.  Results equal ct_plan_launch_grouped's.
   The plan must have been grouped with 256-thread stages (the default block size); the grid is at
   most what the device keeps resident, capped by the widest stage and by `max_blocks` when it is
   positive.  Asynchronous on `stream`; CT_E_INVALID for a plan that is not grouped (or grouped
   with another block size), CT_E_HIP when the device cannot launch cooperatively. */
ct_status ct_plan_launch_single(ct_plan *p, int32_t max_blocks, void *stream);

/* --- kernel timing (tracing) ---------------------------------------------------------------- */

/* Kernel kinds the library launches for a table. */
#define CT_KERNEL_CLEAR 0    /* table reset */
#define CT_KERNEL_PROLOGUE 1 /* per-chunk scratch clear and counter snapshot */
#define CT_KERNEL_DEDUP 2    /* lowest index per distinct key of a chunk */
#define CT_KERNEL_INSERT 3   /* insert probe and claim */
#define CT_KERNEL_ERASE 4    /* erase probe and release */
#define CT_KERNEL_APPLY 5    /* live-count update */
#define CT_KERNEL_RANK 6     /* index-order rank scan (capacity or pool limits) */
#define CT_KERNEL_FINAL 7    /* ranked completion */
#define CT_KERNEL_FIX 8      /* outcomes of repeated keys */
#define CT_KERNEL_FIND 9     /* find / contains */
#define CT_KERNEL_KINDS 10

/* While enabled, every kernel launched for `t` is bracketed by two HIP events recorded on the
   stream of the call that launched it.  Disabling folds the pending records into the totals. */
ct_status ct_table_set_profiling(ct_table *t, int enable);

/* Total device time (ms) and launch count of kernel kind `kind` recorded for `t` since profiling
   was first enabled or last reset.  Waits for the recorded events.  Either output nullable. */
ct_status ct_table_profile(ct_table *t, int32_t kind, double *total_ms, int64_t *launches);

/* Zero the per-kind totals (after waiting for pending records). */
ct_status ct_table_profile_reset(ct_table *t);

/* Static description of a status code. */
const char *ct_status_str(ct_status s);

#ifdef __cplusplus
}
#endif

#endif /* CT_H */
