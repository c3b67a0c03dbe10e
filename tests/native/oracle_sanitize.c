/*
 * oracle_sanitize.c -- drives every entry point of the CPU oracle (oracle.c, partitioned.c) on
 * random batches so that the test suite can run it under AddressSanitizer and
 * UndefinedBehaviorSanitizer (host code only; built with gcc, see tests/test_oracle_sanitize.py).
 *
 * Tables of several capacities and bucket counts, both hashes, keys from a small universe that
 * includes the all-ones and all-ones-minus-one patterns; after every batch the invariant checker
 * must report nothing, and every planted corruption must be reported.  Everything allocated is
 * freed, so the leak checker sees a clean exit.
 */
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>

typedef struct or_table or_table;
typedef struct or_pool or_pool;
typedef struct or_part or_part_opaque;

or_table *or_table_new(int64_t capacity, int hash_kind, int64_t nbuckets);
void or_table_free(or_table *t);
int64_t or_size(const or_table *t);
void or_clear(or_table *t);
void or_insert(or_table *t, const uint64_t *keys, const uint64_t *vals, int64_t n, uint8_t *status);
void or_find(const or_table *t, const uint64_t *keys, int64_t n, uint64_t *vals_out,
             uint64_t sentinel, uint8_t *found);
void or_erase(or_table *t, const uint64_t *keys, int64_t n, uint8_t *erased);
or_pool *or_pool_new(int64_t capacity);
void or_pool_free(or_pool *p);
int64_t or_pool_size(const or_pool *p);
int64_t or_pool_dump(const or_pool *p, int32_t *out, int64_t cap);
void or_pool_pop(or_pool *p, int64_t n, int32_t *out, uint8_t *status);
void or_pool_push(or_pool *p, const int32_t *in, int64_t n, uint8_t *status);
void or_pool_pop_front(or_pool *p, int64_t n, int32_t *out, uint8_t *status);
void or_pool_push_front(or_pool *p, const int32_t *in, int64_t n, uint8_t *status);
void or_insert_alloc(or_table *t, or_pool *p, const uint64_t *keys, int64_t n, int32_t *vals_out,
                     uint8_t *status);
void or_erase_release(or_table *t, or_pool *p, const uint64_t *keys, int64_t n, uint8_t *erased);
int64_t or_dump(const or_table *t, uint64_t *keys_out, uint64_t *vals_out, int64_t cap);
int64_t or_voxel_neighbour_keys(const uint64_t *blocks, int64_t n, int ndirs, uint64_t *out);
int64_t or_select(const or_table *t, int kind, uint64_t lo, uint64_t hi, const int32_t *lo3,
                  const int32_t *hi3, uint64_t *keys_out, uint64_t *vals_out, int64_t cap);
int64_t or_check(const or_table *t, const or_pool *p, int values_from_pool, int *what);
int or_corrupt(or_table *t, or_pool *p, int kind);
void *or_part_new(int64_t capacity, int parts, double slack);
void or_part_free(void *p);
int or_part_insert(void *p, const uint64_t *keys, const uint64_t *vals, int64_t n, uint8_t *status);
int or_part_find(void *p, const uint64_t *keys, int64_t n, uint64_t *vals_out, uint64_t absent,
                 uint8_t *found);
int or_part_erase(void *p, const uint64_t *keys, int64_t n, uint8_t *erased);

static uint64_t rng_state = 0x243F6A8885A308D3ull;
static uint64_t next_u64(void) {  /* splitmix64 (Steele, Lea, Flood) */
    uint64_t z = (rng_state += 0x9E3779B97F4A7C15ull);
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

static int failures = 0;
#define EXPECT(c)                                                        \
    do {                                                                 \
        if (!(c)) {                                                      \
            fprintf(stderr, "line %d: expectation failed: %s\n", __LINE__, #c); \
            ++failures;                                                  \
        }                                                                \
    } while (0)

static uint64_t pick_key(const uint64_t *universe, int64_t u) { return universe[next_u64() % (uint64_t)u]; }

static void one_table(int64_t cap, int hash_kind, int64_t nb, int64_t pool_cap) {
    enum { U = 600, N = 900 };
    uint64_t universe[U];
    for (int i = 0; i < U; ++i) universe[i] = next_u64();
    universe[0] = ~0ull;
    universe[1] = ~0ull - 1;
    universe[2] = 0;
    or_table *t = or_table_new(cap, hash_kind, nb);   /* plain values */
    or_table *ta = or_table_new(cap, hash_kind, nb);  /* values from the pool */
    or_pool *p = or_pool_new(pool_cap);
    uint64_t keys[N], vals[N], out[N];
    uint8_t st[N];
    int32_t iv[N];
    int32_t *fill = (int32_t *)malloc(sizeof(int32_t) * (size_t)(pool_cap > 0 ? pool_cap : 1));
    for (int64_t i = 0; i < pool_cap; ++i) fill[i] = (int32_t)(pool_cap - 1 - i);
    uint8_t *pst = (uint8_t *)malloc((size_t)(pool_cap > 0 ? pool_cap : 1));
    or_pool_push(p, fill, pool_cap, pst);
    for (int round = 0; round < 40; ++round) {
        const int64_t n = (int64_t)(next_u64() % N);
        for (int64_t i = 0; i < n; ++i) {
            keys[i] = pick_key(universe, U);
            vals[i] = next_u64();
        }
        int what = 0;
        switch (round % 5) {
        case 0: or_insert(t, keys, vals, n, st); break;
        case 1: or_find(t, keys, n, out, ~0ull, st); break;
        case 2: or_erase(t, keys, n, st); break;
        case 3: or_insert_alloc(ta, p, keys, n, iv, st); break;
        default: or_erase_release(ta, p, keys, n, st); break;
        }
        EXPECT(or_check(t, NULL, 0, &what) == 0);
        EXPECT(or_check(ta, p, 1, &what) == 0);
        uint64_t *dk = (uint64_t *)malloc(sizeof(uint64_t) * (size_t)(or_size(t) + 1));
        uint64_t *dv = (uint64_t *)malloc(sizeof(uint64_t) * (size_t)(or_size(t) + 1));
        EXPECT(or_dump(t, dk, dv, or_size(t)) == or_size(t));
        const int32_t lo3[3] = {-100, -100, -100}, hi3[3] = {100, 100, 100};
        EXPECT(or_select(t, 1, 0, ~0ull >> 1, lo3, hi3, dk, dv, or_size(t)) >= 0);
        EXPECT(or_select(t, 2, 0, 0, lo3, hi3, dk, dv, or_size(t)) >= 0);
        free(dk);
        free(dv);
    }
    int32_t pout[64];
    uint8_t pst2[64];
    or_pool_pop_front(p, 17, pout, pst2);
    or_pool_push_front(p, pout, 17, pst2);
    int32_t *pd = (int32_t *)malloc(sizeof(int32_t) * (size_t)(or_pool_size(p) + 1));
    EXPECT(or_pool_dump(p, pd, or_pool_size(p)) == or_pool_size(p));
    free(pd);
    or_pool_pop(p, 64, pout, pst2);
    or_clear(t);
    EXPECT(or_size(t) == 0);
    free(fill);
    free(pst);
    or_pool_free(p);
    or_table_free(ta);
    or_table_free(t);
}

/* Every planted corruption of a pool-valued table is reported (kinds 1-7 break the map, 8-9 the
   pool; or_corrupt returns 0 when it planted one). */
static void planted(void) {
    for (int kind = 1; kind <= 9; ++kind) {
        or_table *t = or_table_new(256, 0, 31);
        or_pool *p = or_pool_new(300);
        int32_t in[300];
        uint8_t pst[300];
        for (int i = 0; i < 300; ++i) in[i] = 299 - i;
        or_pool_push(p, in, 300, pst);
        uint64_t keys[200];
        int32_t got[200];
        uint8_t st[200];
        for (int i = 0; i < 200; ++i) keys[i] = next_u64();
        or_insert_alloc(t, p, keys, 200, got, st);
        int what = 0;
        EXPECT(or_check(t, p, 1, &what) == 0);
        EXPECT(or_corrupt(t, p, kind) == 0);
        EXPECT(or_check(t, p, 1, &what) != 0 && what != 0);
        or_pool_free(p);
        or_table_free(t);
    }
}

static void neighbours(void) {
    uint64_t blocks[50], out[50 * 26];
    for (int i = 0; i < 50; ++i) blocks[i] = next_u64() & ((1ull << 63) - 1);
    EXPECT(or_voxel_neighbour_keys(blocks, 50, 6, out) == 300);
    EXPECT(or_voxel_neighbour_keys(blocks, 50, 26, out) == 1300);
    EXPECT(or_voxel_neighbour_keys(blocks, 50, 5, out) == -1);
}

static void partitioned(void) {
    enum { N = 5000 };
    void *pp = or_part_new(4000, 4, 1.5);
    uint64_t keys[N], vals[N];
    uint8_t st[N];
    for (int i = 0; i < N; ++i) {
        keys[i] = next_u64() % 3000;
        vals[i] = (uint64_t)i;
    }
    EXPECT(or_part_insert(pp, keys, vals, N, st) == 0);
    EXPECT(or_part_find(pp, keys, N, vals, ~0ull, st) == 0);
    EXPECT(or_part_erase(pp, keys, N / 2, st) == 0);
    or_part_free(pp);
}

int main(void) {
    const int64_t caps[] = {0, 1, 7, 300, 2000};
    const int64_t nbs[] = {1, 7, 13, 4096};
    for (int c = 0; c < 5; ++c)
        for (int b = 0; b < 4; ++b)
            for (int h = 0; h < 2; ++h) one_table(caps[c], h, nbs[b], caps[c] + 5);
    planted();
    neighbours();
    partitioned();
    if (failures) {
        fprintf(stderr, "%d expectation(s) failed\n", failures);
        return 1;
    }
    printf("oracle sanitize run passed\n");
    return 0;
}
