/*
 * oracle.c -- plain, slow, sequential CPU reference for the batch operations of the hash
 * containers (unordered_map / unordered_set, Section 4.1) and of the index pool (vector / deque
 * back operations used as a stack, Sections 4.2 and 4.3).
 *
 * TEST INFRASTRUCTURE.  Only the test suite, the smoke check and the CPU-baseline leg of the
 * benchmark load this file's library.  It shares no code, header, table or constant with the GPU
 * library: every hash, every status code and every rule below is written out again here.
 *
 * What it computes: a batch is replayed one element at a time in batch-index order, exactly as a
 * loop of single-element container calls would run on the host:
 *   insert : a key already present is left unmodified (the paper's insert reports the end
 *            position for an already inserted value, Section 4.1); a new key is stored if fewer
 *            than `capacity` keys are live, else the element fails with FULL (inserting beyond the
 *            fixed capacity is the only failure case, Section 4 "Capacity" and "Guarantees").
 *   find   : the mapped value or "not found" (find / contains, Section 4.1).
 *   erase  : removes the key, reporting whether it was present (Section 4.1).
 *   pool   : push_back appends, pop_back removes and returns the last element (Sections 4.2-4.3);
 *            used as a last-in first-out free list of int32 indices.  The deque's front
 *            operations (Section 4.3) remove or insert at the other end: pop_front then
 *            push_back is a first-in first-out free list.
 * Duplicates inside one batch therefore resolve in index order: the lowest index acts first and
 * later copies see the state it left.
 *
 * Storage is the textbook chained hash map: a bucket array of list heads and an entry array of
 * exactly `capacity` entries whose unused members sit on a LIFO free list.  A table is FULL exactly
 * when that free list is empty.  Occupancy is the list membership itself, so no key value is
 * reserved as a placeholder (Section 5.1) and every 2^64 key value is legal.
 *
 * Hashes (they decide bucket membership only; results never depend on them):
 *   mix64   : the 64-bit finaliser of MurmurHash3 (Appleby), a "basic hash function" in the sense
 *             of Section 5.3, reduced modulo the bucket count.
 *   voxel21 : the spatial hash of Section 4.1, x*73856093 XOR y*19349669 XOR z*83492791, on
 *             block coordinates packed as three signed 21-bit fields (x bits 0-20, y 21-41,
 *             z 42-62).  Products and XOR wrap in 32-bit two's complement (the int arithmetic of
 *             the listing); the int result converts to a 64-bit size_t by sign extension, then is
 *             reduced modulo the bucket count.
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define OR_PRESENT 0
#define OR_INSERTED 1
#define OR_FULL 2

#define OR_HASH_MIX64 0
#define OR_HASH_VOXEL21 1

typedef struct {
    int64_t capacity;     /* number of keys the table can hold, fixed at creation */
    int hash_kind;
    int64_t nbuckets;
    int64_t *head;        /* head[b]: first entry of bucket b's list, -1 when empty */
    uint64_t *key;        /* entry storage, `capacity` entries */
    uint64_t *val;
    int64_t *next;        /* next entry of the same list, -1 at the end */
    int64_t *free_stack;  /* indices of unused entries; the top is free_stack[free_top - 1] */
    int64_t free_top;
    int64_t size;         /* number of live keys */
    int error;            /* sticky: 1 = an insert hit FULL, 2 = a pool ran empty or over */
} or_table;

typedef struct {
    int64_t capacity;
    int32_t *stack;       /* stack[0 .. top-1]; pop_back returns stack[top-1] */
    int64_t top;
} or_pool;

/* ---------------------------------------------------------------------------------------- */
/* hashes                                                                                    */
/* ---------------------------------------------------------------------------------------- */
uint64_t or_fmix64(uint64_t k)
{
    k ^= k >> 33;
    k *= 0xff51afd7ed558ccdULL;
    k ^= k >> 33;
    k *= 0xc4ceb9fe1a85ec53ULL;
    k ^= k >> 33;
    return k;
}

static int32_t field21(uint64_t key, int shift)
{
    uint32_t f = (uint32_t)((key >> shift) & 0x1FFFFFu);
    if (f & 0x100000u) f |= 0xFFE00000u;   /* sign-extend 21 -> 32 bits */
    return (int32_t)f;
}

/* The spatial hash as a size_t value (before the bucket reduction). */
uint64_t or_voxel21_hash(uint64_t key)
{
    uint32_t x = (uint32_t)field21(key, 0);
    uint32_t y = (uint32_t)field21(key, 21);
    uint32_t z = (uint32_t)field21(key, 42);
    uint32_t h = (x * 73856093u) ^ (y * 19349669u) ^ (z * 83492791u);
    return (uint64_t)(int64_t)(int32_t)h;
}

int64_t or_bucket_of(const or_table *t, uint64_t key)
{
    uint64_t h = (t->hash_kind == OR_HASH_VOXEL21) ? or_voxel21_hash(key) : or_fmix64(key);
    return (int64_t)(h % (uint64_t)t->nbuckets);
}

/* ---------------------------------------------------------------------------------------- */
/* table                                                                                     */
/* ---------------------------------------------------------------------------------------- */
static void table_reset(or_table *t)
{
    for (int64_t b = 0; b < t->nbuckets; ++b) t->head[b] = -1;
    /* free list holds every entry; entry 0 is handed out first */
    for (int64_t j = 0; j < t->capacity; ++j) t->free_stack[j] = t->capacity - 1 - j;
    t->free_top = t->capacity;
    t->size = 0;
}

or_table *or_table_new(int64_t capacity, int hash_kind, int64_t nbuckets)
{
    if (capacity < 0 || nbuckets <= 0) return NULL;
    or_table *t = (or_table *)calloc(1, sizeof(or_table));
    if (!t) return NULL;
    t->capacity = capacity;
    t->hash_kind = hash_kind;
    t->nbuckets = nbuckets;
    size_t c = (size_t)(capacity > 0 ? capacity : 1);
    t->head = (int64_t *)malloc(sizeof(int64_t) * (size_t)nbuckets);
    t->key = (uint64_t *)malloc(sizeof(uint64_t) * c);
    t->val = (uint64_t *)malloc(sizeof(uint64_t) * c);
    t->next = (int64_t *)malloc(sizeof(int64_t) * c);
    t->free_stack = (int64_t *)malloc(sizeof(int64_t) * c);
    if (!t->head || !t->key || !t->val || !t->next || !t->free_stack) {
        free(t->head); free(t->key); free(t->val); free(t->next); free(t->free_stack); free(t);
        return NULL;
    }
    table_reset(t);
    return t;
}

void or_table_free(or_table *t)
{
    if (!t) return;
    free(t->head); free(t->key); free(t->val); free(t->next); free(t->free_stack);
    free(t);
}

/* Entry index holding `key`, or -1. */
static int64_t lookup(const or_table *t, uint64_t key)
{
    for (int64_t e = t->head[or_bucket_of(t, key)]; e >= 0; e = t->next[e])
        if (t->key[e] == key) return e;
    return -1;
}

/* Store a key that is known to be absent; the caller checked that an entry is free. */
static void store_new(or_table *t, uint64_t key, uint64_t val)
{
    int64_t e = t->free_stack[--t->free_top];
    int64_t b = or_bucket_of(t, key);
    t->key[e] = key;
    t->val[e] = val;
    t->next[e] = t->head[b];
    t->head[b] = e;
    t->size += 1;
}

/* Unlink the entry holding `key` (known present) and return its value. */
static uint64_t remove_key(or_table *t, uint64_t key)
{
    int64_t b = or_bucket_of(t, key);
    int64_t prev = -1;
    int64_t e = t->head[b];
    while (t->key[e] != key) { prev = e; e = t->next[e]; }
    if (prev < 0) t->head[b] = t->next[e];
    else t->next[prev] = t->next[e];
    t->free_stack[t->free_top++] = e;
    t->size -= 1;
    return t->val[e];
}

int64_t or_size(const or_table *t) { return t->size; }
int or_error(const or_table *t) { return t->error; }
void or_clear(or_table *t) { table_reset(t); t->error = 0; }

void or_insert(or_table *t, const uint64_t *keys, const uint64_t *vals, int64_t n, uint8_t *status)
{
    for (int64_t i = 0; i < n; ++i) {
        uint8_t st;
        if (lookup(t, keys[i]) >= 0) {
            st = OR_PRESENT;
        } else if (t->size == t->capacity) {
            st = OR_FULL;
            t->error |= 1;
        } else {
            store_new(t, keys[i], vals ? vals[i] : 0);
            st = OR_INSERTED;
        }
        if (status) status[i] = st;
    }
}

void or_find(const or_table *t, const uint64_t *keys, int64_t n, uint64_t *vals_out,
             uint64_t sentinel, uint8_t *found)
{
    for (int64_t i = 0; i < n; ++i) {
        int64_t e = lookup(t, keys[i]);
        if (vals_out) vals_out[i] = (e >= 0) ? t->val[e] : sentinel;
        if (found) found[i] = (e >= 0) ? 1 : 0;
    }
}

void or_erase(or_table *t, const uint64_t *keys, int64_t n, uint8_t *erased)
{
    for (int64_t i = 0; i < n; ++i) {
        int hit = lookup(t, keys[i]) >= 0;
        if (hit) remove_key(t, keys[i]);
        if (erased) erased[i] = (uint8_t)hit;
    }
}

/* ---------------------------------------------------------------------------------------- */
/* index pool: a fixed-capacity stack of int32                                               */
/* ---------------------------------------------------------------------------------------- */
or_pool *or_pool_new(int64_t capacity)
{
    if (capacity < 0) return NULL;
    or_pool *p = (or_pool *)calloc(1, sizeof(or_pool));
    if (!p) return NULL;
    p->capacity = capacity;
    p->stack = (int32_t *)malloc(sizeof(int32_t) * (size_t)(capacity > 0 ? capacity : 1));
    if (!p->stack) { free(p); return NULL; }
    /* a fresh pool holds every index; pops return 0, 1, 2, ... */
    for (int64_t j = 0; j < capacity; ++j) p->stack[j] = (int32_t)(capacity - 1 - j);
    p->top = capacity;
    return p;
}

void or_pool_free(or_pool *p)
{
    if (!p) return;
    free(p->stack);
    free(p);
}

int64_t or_pool_size(const or_pool *p) { return p->top; }

/* Copy the live stack, bottom first; returns the element count. */
int64_t or_pool_dump(const or_pool *p, int32_t *out, int64_t cap)
{
    int64_t m = p->top < cap ? p->top : cap;
    if (out) memcpy(out, p->stack, sizeof(int32_t) * (size_t)m);
    return p->top;
}

/* pop_back n times: out[i] is the removed value, or -1 (status 2) once the pool is empty. */
void or_pool_pop(or_pool *p, int64_t n, int32_t *out, uint8_t *status)
{
    for (int64_t i = 0; i < n; ++i) {
        if (p->top == 0) {
            if (out) out[i] = -1;
            if (status) status[i] = 2;
        } else {
            int32_t v = p->stack[--p->top];
            if (out) out[i] = v;
            if (status) status[i] = 1;
        }
    }
}

/* push_back n values in order: status 1 stored, 2 when the pool is already at capacity. */
void or_pool_push(or_pool *p, const int32_t *in, int64_t n, uint8_t *status)
{
    for (int64_t i = 0; i < n; ++i) {
        if (p->top == p->capacity) {
            if (status) status[i] = 2;
        } else {
            p->stack[p->top++] = in[i];
            if (status) status[i] = 1;
        }
    }
}

/* pop_front n times (a deque front operation, Section 4.3): out[i] is the removed first
   element, or -1 (status 2) once the pool is empty.  The stack's bottom is the deque's front. */
void or_pool_pop_front(or_pool *p, int64_t n, int32_t *out, uint8_t *status)
{
    for (int64_t i = 0; i < n; ++i) {
        if (p->top == 0) {
            if (out) out[i] = -1;
            if (status) status[i] = 2;
        } else {
            int32_t v = p->stack[0];
            memmove(p->stack, p->stack + 1, sizeof(int32_t) * (size_t)(p->top - 1));
            --p->top;
            if (out) out[i] = v;
            if (status) status[i] = 1;
        }
    }
}

/* push_front n values in order (the last one ends up first): status 1 stored, 2 when the pool is
   already at capacity. */
void or_pool_push_front(or_pool *p, const int32_t *in, int64_t n, uint8_t *status)
{
    for (int64_t i = 0; i < n; ++i) {
        if (p->top == p->capacity) {
            if (status) status[i] = 2;
        } else {
            memmove(p->stack + 1, p->stack, sizeof(int32_t) * (size_t)p->top);
            p->stack[0] = in[i];
            ++p->top;
            if (status) status[i] = 1;
        }
    }
}

/* Insert whose values are pool indices: a new key takes pop_back() of the pool. */
void or_insert_alloc(or_table *t, or_pool *p, const uint64_t *keys, int64_t n, int32_t *vals_out,
                     uint8_t *status)
{
    for (int64_t i = 0; i < n; ++i) {
        int64_t e = lookup(t, keys[i]);
        uint8_t st;
        int32_t v;
        if (e >= 0) {
            v = (int32_t)(uint32_t)t->val[e];
            st = OR_PRESENT;
        } else if (t->size == t->capacity || p->top == 0) {
            v = -1;
            st = OR_FULL;
            t->error |= (t->size == t->capacity) ? 1 : 2;
        } else {
            v = p->stack[--p->top];
            store_new(t, keys[i], (uint64_t)(uint32_t)v);
            st = OR_INSERTED;
        }
        if (vals_out) vals_out[i] = v;
        if (status) status[i] = st;
    }
}

/* Erase whose freed values go back to the pool with push_back, in batch order. */
void or_erase_release(or_table *t, or_pool *p, const uint64_t *keys, int64_t n, uint8_t *erased)
{
    for (int64_t i = 0; i < n; ++i) {
        int hit = lookup(t, keys[i]) >= 0;
        if (hit) {
            int32_t v = (int32_t)(uint32_t)remove_key(t, keys[i]);
            if (p->top == p->capacity) t->error |= 2;
            else p->stack[p->top++] = v;
        }
        if (erased) erased[i] = (uint8_t)hit;
    }
}

/* ---------------------------------------------------------------------------------------- */
/* dump and invariants                                                                       */
/* ---------------------------------------------------------------------------------------- */
static int cmp_pair(const void *a, const void *b)
{
    uint64_t x = ((const uint64_t *)a)[0], y = ((const uint64_t *)b)[0];
    return (x > y) - (x < y);
}

/* Live (key, value) pairs sorted by key; returns the live count (copies at most `cap`). */
int64_t or_dump(const or_table *t, uint64_t *keys_out, uint64_t *vals_out, int64_t cap)
{
    uint64_t *pairs = (uint64_t *)malloc(sizeof(uint64_t) * 2 * (size_t)(t->size > 0 ? t->size : 1));
    int64_t m = 0;
    for (int64_t b = 0; b < t->nbuckets; ++b)
        for (int64_t e = t->head[b]; e >= 0 && m < t->size; e = t->next[e]) {
            pairs[2 * m] = t->key[e];
            pairs[2 * m + 1] = t->val[e];
            ++m;
        }
    qsort(pairs, (size_t)m, 2 * sizeof(uint64_t), cmp_pair);
    for (int64_t j = 0; j < m && j < cap; ++j) {
        if (keys_out) keys_out[j] = pairs[2 * j];
        if (vals_out) vals_out[j] = pairs[2 * j + 1];
    }
    free(pairs);
    return m;
}

/*
 * Neighbour keys of voxel blocks (the allocation step of the reconstruction workload behind the
 * voxel-block example of Section 4.1): for block i, in direction order d = 0 .. 26 (offsets
 * dx = d mod 3 - 1, dy = (d / 3) mod 3 - 1, dz = d / 9 - 1, the zero offset skipped, and with
 * ndirs 6 only the offsets along one axis), out[i * ndirs + j] is the j-th neighbour's key.  Each
 * coordinate is the block's signed 21-bit field plus the offset, taken modulo 2^21 when packed.
 * Returns the number of keys written (n * ndirs), or -1 for an ndirs other than 6 or 26.
 */
static int64_t sign21(uint64_t f) { return (f & 0x100000u) ? (int64_t)f - 0x200000 : (int64_t)f; }

int64_t or_voxel_neighbour_keys(const uint64_t *blocks, int64_t n, int ndirs, uint64_t *out)
{
    if (ndirs != 6 && ndirs != 26) return -1;
    int64_t m = 0;
    for (int64_t i = 0; i < n; ++i) {
        int64_t c[3];
        for (int a = 0; a < 3; ++a) c[a] = sign21((blocks[i] >> (21 * a)) & 0x1FFFFFu);
        for (int d = 0; d < 27; ++d) {
            int64_t o[3] = {d % 3 - 1, (d / 3) % 3 - 1, d / 9 - 1};
            int nz = (o[0] != 0) + (o[1] != 0) + (o[2] != 0);
            if (nz == 0 || (ndirs == 6 && nz != 1)) continue;
            uint64_t k = 0;
            for (int a = 0; a < 3; ++a)
                k |= ((uint64_t)(c[a] + o[a]) & 0x1FFFFFu) << (21 * a);
            out[m++] = k;
        }
    }
    return m;
}

/*
 * Range selection (Section 3.6: a range of the container turned into a vector with a copy_if):
 * the live pairs whose key a predicate accepts, sorted by key.  Returns the number selected;
 * at most `cap` pairs are written.
 *   kind 0 (key range) : lo <= key < hi, unsigned.
 *   kind 1 (voxel box) : the key packs three signed 21-bit block coordinates (x bits 0-20, y 21-41,
 *                        z 42-62, bit 63 clear) and each lies in [lo3[d], hi3[d]], bounds included.
 *                        A key with bit 63 set packs no block and is never selected.
 */

static int select_accepts(int kind, uint64_t key, uint64_t lo, uint64_t hi, const int32_t *lo3,
                          const int32_t *hi3)
{
    if (kind == 0) return key >= lo && key < hi;
    if (key >> 63) return 0;
    for (int d = 0; d < 3; ++d) {
        int64_t c = sign21((key >> (21 * d)) & 0x1FFFFFu);
        if (c < lo3[d] || c > hi3[d]) return 0;
    }
    return 1;
}

int64_t or_select(const or_table *t, int kind, uint64_t lo, uint64_t hi, const int32_t *lo3,
                  const int32_t *hi3, uint64_t *keys_out, uint64_t *vals_out, int64_t cap)
{
    uint64_t *pairs = (uint64_t *)malloc(sizeof(uint64_t) * 2 * (size_t)(t->size > 0 ? t->size : 1));
    int64_t m = 0;
    for (int64_t b = 0; b < t->nbuckets; ++b)
        for (int64_t e = t->head[b]; e >= 0; e = t->next[e]) {
            if (!select_accepts(kind, t->key[e], lo, hi, lo3, hi3)) continue;
            pairs[2 * m] = t->key[e];
            pairs[2 * m + 1] = t->val[e];
            ++m;
        }
    qsort(pairs, (size_t)m, 2 * sizeof(uint64_t), cmp_pair);
    for (int64_t j = 0; j < m && j < cap; ++j) {
        if (keys_out) keys_out[j] = pairs[2 * j];
        if (vals_out) vals_out[j] = pairs[2 * j + 1];
    }
    free(pairs);
    return m;
}

/*
 * Count invariant violations; `what` (nullable) receives a bit per failed invariant:
 *   1  size equals the number of entries reachable from the buckets, and size <= capacity
 *   2  no key occurs twice among the reachable entries
 *   4  every reachable entry's key is found by lookup, with the entry's value
 *   8  every entry lies in the list of its own bucket; links stay in range; lists are acyclic
 *      and no entry is on two lists
 *  16  reachable entries and free-list entries partition {0 .. capacity-1}: every entry is in
 *      exactly one of the two (no leaked entry, no entry both live and free)
 *  32  (with a pool) pool stack entries are in range and distinct; when `values_from_pool`, the
 *      pool stack and the live values partition {0 .. pool capacity - 1}
 * These are the uniqueness guarantee of Section 4.1 (a key is stored at most once), the fixed
 * capacity of Section 4 and the contracts of Section 3.3 written out for the chained layout; each
 * bit is computed from its own evidence, so a single broken invariant sets a single bit (a key
 * filed under another bucket sets 8 and, since lookup then misses it, 4).
 */
/* lookup() that stops at a link out of range or after `capacity` steps (a damaged list). */
static int64_t checked_lookup(const or_table *t, uint64_t key)
{
    int64_t steps = 0;
    for (int64_t e = t->head[or_bucket_of(t, key)]; e >= 0 && e < t->capacity && steps <= t->capacity;
         e = t->next[e], ++steps)
        if (t->key[e] == key) return e;
    return -1;
}

int64_t or_check(const or_table *t, const or_pool *p, int values_from_pool, int *what)
{
    int64_t bad = 0;
    int w = 0;
    int64_t C = t->capacity;
    uint8_t *mark = (uint8_t *)calloc((size_t)(C > 0 ? C : 1), 1);
    uint64_t *ks = (uint64_t *)malloc(sizeof(uint64_t) * (size_t)(C > 0 ? C : 1));
    int64_t reach = 0;
    for (int64_t b = 0; b < t->nbuckets; ++b) {
        for (int64_t e = t->head[b]; e >= 0; e = t->next[e]) {
            if (e >= C) { ++bad; w |= 8; break; }    /* link out of range */
            if (mark[e]) { ++bad; w |= 8; break; }   /* a cycle, or an entry on two lists */
            mark[e] = 1;
            ks[reach++] = t->key[e];
            if (or_bucket_of(t, t->key[e]) != b) { ++bad; w |= 8; }
            int64_t f = checked_lookup(t, t->key[e]);
            if (f < 0 || t->val[f] != t->val[e]) { ++bad; w |= 4; }
        }
    }
    if (reach != t->size || t->size > C) { ++bad; w |= 1; }
    for (int64_t j = 0; j < t->free_top; ++j) {
        int64_t e = t->free_stack[j];
        if (e < 0 || e >= C || mark[e]) { ++bad; w |= 16; continue; }
        mark[e] = 2;
    }
    for (int64_t e = 0; e < C; ++e)
        if (!mark[e]) { ++bad; w |= 16; }
    free(mark);

    qsort(ks, (size_t)reach, sizeof(uint64_t), cmp_pair);  /* cmp_pair reads the first u64 only */
    for (int64_t j = 1; j < reach; ++j)
        if (ks[j] == ks[j - 1]) { ++bad; w |= 2; }
    free(ks);

    if (p) {
        int64_t P = p->capacity;
        uint8_t *pm = (uint8_t *)calloc((size_t)(P > 0 ? P : 1), 1);
        for (int64_t j = 0; j < p->top; ++j) {
            int32_t v = p->stack[j];
            if (v < 0 || v >= P || pm[v]) { ++bad; w |= 32; continue; }
            pm[v] = 1;
        }
        if (values_from_pool) {
            for (int64_t b = 0; b < t->nbuckets; ++b) {
                int64_t steps = 0;
                for (int64_t e = t->head[b]; e >= 0 && e < C && steps <= C; e = t->next[e], ++steps) {
                    int64_t v = (int64_t)(int32_t)(uint32_t)t->val[e];
                    if (v < 0 || v >= P || pm[v]) { ++bad; w |= 32; continue; }
                    pm[v] = 2;
                }
            }
            for (int64_t v = 0; v < P; ++v)
                if (!pm[v]) { ++bad; w |= 32; }
        }
        free(pm);
    }
    if (what) *what = w;
    return bad;
}

/*
 * TEST HOOK, not an operation of the containers: break exactly one invariant of a table (and
 * pool) so that the tests can show that or_check reports it.  Returns 0 when the corruption was
 * applied, -1 when the state has no room for it (for example an empty table, or no free entry).
 *   1  size counter off by one (invariant 1)
 *   2  a free entry made a second copy of a live key, with the same value, on the same list (2)
 *   3  a live entry moved to the list of another bucket (8, and 4 through the failed lookup)
 *   4  a list made cyclic: its last entry links back to its first (8)
 *   5  a link pointing past the entry array (8)
 *   6  a free entry dropped from the free list without being linked anywhere (16)
 *   7  an entry both live and on the free list (16)
 *   8  (pool) an index duplicated inside the pool stack (32)
 *   9  (pool, values from the pool) an index dropped from the pool stack (32)
 */
static int64_t first_nonempty_bucket(const or_table *t, int64_t from)
{
    for (int64_t b = from; b < t->nbuckets; ++b)
        if (t->head[b] >= 0) return b;
    return -1;
}

int or_corrupt(or_table *t, or_pool *p, int kind)
{
    int64_t b = first_nonempty_bucket(t, 0);
    switch (kind) {
    case 1:
        t->size += 1;
        return 0;
    case 2: {
        if (b < 0 || t->free_top == 0) return -1;
        int64_t e = t->head[b];
        int64_t d = t->free_stack[--t->free_top];
        t->key[d] = t->key[e];
        t->val[d] = t->val[e];
        t->next[d] = t->head[b];
        t->head[b] = d;
        t->size += 1;
        return 0;
    }
    case 3: {
        if (b < 0 || t->nbuckets < 2) return -1;
        int64_t e = t->head[b];
        t->head[b] = t->next[e];
        int64_t o = (b + 1) % t->nbuckets;
        t->next[e] = t->head[o];
        t->head[o] = e;
        return 0;
    }
    case 4: {
        if (b < 0) return -1;
        int64_t e = t->head[b];
        while (t->next[e] >= 0) e = t->next[e];
        t->next[e] = t->head[b];
        return 0;
    }
    case 5: {
        if (b < 0) return -1;
        int64_t e = t->head[b];
        while (t->next[e] >= 0) e = t->next[e];
        t->next[e] = t->capacity + 5;
        return 0;
    }
    case 6:
        if (t->free_top == 0) return -1;
        --t->free_top;
        return 0;
    case 7:
        if (b < 0 || t->free_top == 0) return -1;
        t->free_stack[0] = t->head[b];
        return 0;
    case 8:
        if (!p || p->top < 2) return -1;
        p->stack[1] = p->stack[0];
        return 0;
    case 9:
        if (!p || p->top < 1) return -1;
        --p->top;
        return 0;
    }
    return -1;
}
