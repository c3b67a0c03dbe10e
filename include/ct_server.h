/*
 * ct_server.h -- continuous-batching request server over device-resident tables (ct.h).
 *
 * The paper's containers are driven by host code that hands them whole batches; a server sits in
 * front of them when requests of uneven sizes arrive over time.  A request is one insert, find or
 * erase batch for one table, with its keys, values and result arrays in host memory.  A worker
 * thread owned by the server
 *   1. takes submitted requests into one FIFO per table, stamped with their submission time;
 *   2. admits work in arrival order of the tables' head requests: a head, merged with the
 *      requests of the same kind queued right behind it on its table (up to max_batch_keys keys),
 *      is admitted when its staging space fits in the caller's device staging buffer and a batch
 *      slot is free; otherwise admission waits (back-pressure; nothing is dropped or reordered);
 *   3. runs an admitted batch on its table's stream: copies of every request's inputs into the
 *      batch's staging space, the table's batch call, copies of the results back into every
 *      request's host result arrays, and a completion event;
 *   4. retires a batch when its event has completed: the staging space and the slot are freed and
 *      each request is reported complete with its completion time.
 * Merging consecutive same-kind requests of one table keeps every request's sequential result,
 * because a batch gives the results of its elements applied one after the other in index order
 * (ct.h, batch semantics).  A table's batches run in admission order on one stream, so each
 * request sees exactly the state left by the requests of its table submitted before it.
 *
 * Staging space of a batch of n keys: n * (8 + in_value_bytes + out_value_bytes + 1), each array
 * rounded up to 256 bytes, where the value widths are the table's (ct_table_value_bytes) and
 * in/out apply to insert/find respectively.  The staging buffer is the HBM admission budget.
 *
 * Conventions: as in ct.h (int64_t counts, ct_status results).  Host arrays passed to submit must
 * stay valid and unmodified until the request is reported complete; they should be pinned
 * (hipHostMalloc) so that the copies are asynchronous.  While a server exists, its worker is the
 * only caller of its tables: the caller must not use them directly until ct_server_destroy
 * returns.  All entry points may be called from any one host thread at a time.
 */
#ifndef CT_SERVER_H
#define CT_SERVER_H

#include <stdint.h>

#include "ct.h"

#ifdef __cplusplus
extern "C" {
#endif

typedef struct ct_server ct_server;

typedef struct ct_server_desc {
    int32_t streams;        /* 1..16 streams (default priority); table i runs on stream i % streams */
    int32_t max_inflight;   /* 1..4096 batch slots in flight */
    int64_t max_batch_keys; /* >= 1: keys merged into one batch (a single larger request still runs
                               alone) */
} ct_server_desc;

typedef struct ct_server_stats {
    int64_t submitted, completed, batches;
    int64_t peak_staging_bytes; /* most staging bytes in flight at once */
    int64_t peak_inflight;      /* most batches in flight at once */
    int64_t dispatch_ns;        /* worker time spent enqueueing batches (copies, kernels, events) */
    int64_t retire_ns;          /* worker time spent polling events and retiring batches */
    int32_t error;              /* first ct_status other than CT_OK met by the worker */
} ct_server_stats;

/* Create a server over `tables[ntables]` (their handles stay owned by the caller and must outlive
   the server) with the device staging buffer `d_staging` (`staging_bytes` bytes, 256-byte
   aligned, owned by the caller) as its admission budget.  Starts the worker thread on the current
   device. */
ct_status ct_server_create(ct_table *const *tables, int32_t ntables, const ct_server_desc *d,
                           void *d_staging, int64_t staging_bytes, ct_server **out);

/* Queue request: `op` is CT_OP_INSERT, CT_OP_FIND or CT_OP_ERASE (ct.h) on table index `table`.
   h_keys[n] u64; h_vals[n] values of the table's width (insert into a map; else ignored);
   h_vals_out[n] (find on a map, nullable) receives the value or all-ones; h_flags_out[n]
   (nullable) receives the status, found or erased flag as the table's batch calls do.  All host
   memory.  *ticket receives the request's number (0, 1, 2, ... in submission order).  A request
   whose staging space exceeds the whole buffer is rejected with CT_E_INVALID. */
ct_status ct_server_submit(ct_server *s, int32_t table, int32_t op, const uint64_t *h_keys,
                           const void *h_vals, int64_t n, void *h_vals_out, uint8_t *h_flags_out,
                           int64_t *ticket);

/* Move up to `max` completed requests, oldest completion first, into tickets[], with their
   submission and completion times in nanoseconds since the server was created (each output
   array nullable) and their status (CT_OK, or the error that ended their batch).  *count gets
   the number moved.  Does not wait. */
ct_status ct_server_poll(ct_server *s, int64_t *tickets, int64_t *submit_ns, int64_t *done_ns,
                         int32_t *status, int64_t max, int64_t *count);

/* Wait until every submitted request has completed (results in host memory). */
ct_status ct_server_wait_idle(ct_server *s);

/* Counters since creation (ct_server_stats above). */
ct_status ct_server_get_stats(ct_server *s, ct_server_stats *out);

/* Nanoseconds since the server was created, on the clock of the submit and completion times. */
ct_status ct_server_now(ct_server *s, int64_t *ns);

/* Wait until idle, stop the worker and free the server's host state and streams. */
ct_status ct_server_destroy(ct_server *s);

#ifdef __cplusplus
}
#endif

#endif /* CT_SERVER_H */
