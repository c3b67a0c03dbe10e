/*
 * partitioned.c -- multi-core CPU baseline for timing the batch operations on the host.
 *
 * TEST INFRASTRUCTURE (benchmark context only; the definition of the results is oracle.c).
 * Keys are split into P partitions by the high half of or_fmix64(key).  Each partition is an independent
 * oracle table replayed by its own thread over the batch in index order, so every partition sees
 * its keys in the same order as the sequential replay.  Because the operations of different keys
 * never interact (Section 4.1 semantics are per key), the results equal the sequential oracle's
 * whenever no partition reaches its own capacity; each partition is given `slack` times its share
 * of the capacity so that this holds for the workloads it is timed on.
 */
#define _POSIX_C_SOURCE 200809L
#include <pthread.h>
#include <stdint.h>
#include <stdlib.h>

typedef struct or_table or_table;
uint64_t or_fmix64(uint64_t k);
or_table *or_table_new(int64_t capacity, int hash_kind, int64_t nbuckets);
void or_table_free(or_table *t);
int64_t or_size(const or_table *t);
void or_insert(or_table *t, const uint64_t *keys, const uint64_t *vals, int64_t n, uint8_t *status);
void or_find(const or_table *t, const uint64_t *keys, int64_t n, uint64_t *vals_out,
             uint64_t absent, uint8_t *found);
void or_erase(or_table *t, const uint64_t *keys, int64_t n, uint8_t *erased);

typedef struct {
  int parts;
  or_table **t;
  uint16_t *part;   /* partition of each batch element (scratch, grown on demand) */
  int64_t part_cap;
} or_part;

enum { OP_INSERT, OP_FIND, OP_ERASE };

typedef struct {
  or_part *p;
  int id, op;
  const uint64_t *keys;
  const uint64_t *vals;
  int64_t n;
  uint8_t *flags;
  uint64_t *vals_out;
  uint64_t absent;
  pthread_barrier_t *bar;
} job;

or_part *or_part_new(int64_t capacity, int parts, double slack) {
  if (parts < 1 || parts > 4096) return NULL;
  or_part *p = calloc(1, sizeof(or_part));
  if (!p) return NULL;
  p->parts = parts;
  p->t = calloc((size_t)parts, sizeof(or_table *));
  const int64_t share = (int64_t)((double)capacity / parts * slack) + 16;
  for (int i = 0; p->t && i < parts; ++i) p->t[i] = or_table_new(share, 0, share);
  return p;
}

void or_part_free(or_part *p) {
  if (!p) return;
  for (int i = 0; p->t && i < p->parts; ++i)
    if (p->t[i]) or_table_free(p->t[i]);
  free(p->t);
  free(p->part);
  free(p);
}

int64_t or_part_size(const or_part *p) {
  int64_t s = 0;
  for (int i = 0; i < p->parts; ++i) s += or_size(p->t[i]);
  return s;
}

static void *run(void *arg) {
  job *j = arg;
  or_part *p = j->p;
  /* phase 1: this thread's slice of the partition ids */
  const int64_t lo = j->n * j->id / p->parts, hi = j->n * (j->id + 1) / p->parts;
  /* the high half of the hash picks the partition; the tables' buckets use the whole hash */
  for (int64_t i = lo; i < hi; ++i)
    p->part[i] = (uint16_t)(((or_fmix64(j->keys[i]) >> 32) * (uint64_t)p->parts) >> 32);
  pthread_barrier_wait(j->bar);
  /* phase 2: this thread's partition, in index order */
  or_table *t = p->t[j->id];
  for (int64_t i = 0; i < j->n; ++i) {
    if (p->part[i] != j->id) continue;
    if (j->op == OP_INSERT)
      or_insert(t, &j->keys[i], j->vals ? &j->vals[i] : NULL, 1, &j->flags[i]);
    else if (j->op == OP_FIND)
      or_find(t, &j->keys[i], 1, &j->vals_out[i], j->absent, &j->flags[i]);
    else
      or_erase(t, &j->keys[i], 1, &j->flags[i]);
  }
  return NULL;
}

static int batch(or_part *p, int op, const uint64_t *keys, const uint64_t *vals, int64_t n,
                 uint8_t *flags, uint64_t *vals_out, uint64_t absent) {
  if (n > p->part_cap) {
    uint16_t *q = realloc(p->part, (size_t)n * sizeof(uint16_t));
    if (!q) return -1;
    p->part = q;
    p->part_cap = n;
  }
  pthread_barrier_t bar;
  pthread_barrier_init(&bar, NULL, (unsigned)p->parts);
  job *js = calloc((size_t)p->parts, sizeof(job));
  pthread_t *th = calloc((size_t)p->parts, sizeof(pthread_t));
  if (!js || !th) {
    free(js);
    free(th);
    pthread_barrier_destroy(&bar);
    return -1;
  }
  for (int i = 0; i < p->parts; ++i) {
    js[i] = (job){p, i, op, keys, vals, n, flags, vals_out, absent, &bar};
    pthread_create(&th[i], NULL, run, &js[i]);
  }
  for (int i = 0; i < p->parts; ++i) pthread_join(th[i], NULL);
  pthread_barrier_destroy(&bar);
  free(js);
  free(th);
  return 0;
}

int or_part_insert(or_part *p, const uint64_t *keys, const uint64_t *vals, int64_t n,
                   uint8_t *status) {
  return batch(p, OP_INSERT, keys, vals, n, status, NULL, 0);
}

int or_part_find(or_part *p, const uint64_t *keys, int64_t n, uint64_t *vals_out, uint64_t absent,
                 uint8_t *found) {
  return batch(p, OP_FIND, keys, NULL, n, found, vals_out, absent);
}

int or_part_erase(or_part *p, const uint64_t *keys, int64_t n, uint8_t *erased) {
  return batch(p, OP_ERASE, keys, NULL, n, erased, NULL, 0);
}
