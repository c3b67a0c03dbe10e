/*
 * ct_roofline.h -- random-access and streaming microbenchmarks that give the measured ceilings
 * the batch container kernels are compared with on the same chip.  They run the same access
 * shapes as the containers with none of the container logic:
 *
 *   ctr_gather     : per key, read the 8-byte key, pick a line by the key's hash, read that whole
 *                    line with `line_bytes`/16 cooperating lanes, write 8 bytes (the traffic of a
 *                    find that always hits its home bucket).
 *   ctr_gather_cas : the same plus one 64-bit compare-and-swap on the line (the read-modify-write
 *                    of an insert or erase that claims or clears a slot).
 *   ctr_gather_cas_store : the same plus an 8-byte store to the word after the swapped one (the
 *                    claim and value store of an insert into one 16-byte slot; 64 bits is the
 *                    widest compare-and-swap, so a slot takes both).
 *   ctr_cas        : one 64-bit compare-and-swap per key on a random 8-byte word, nothing else.
 *   ctr_amin       : one 64-bit atomic min per key on a random 8-byte word, result not returned.
 *   ctr_copy       : stream copy of `bytes` bytes (16-byte vector loads and stores).
 *
 * Arguments follow include/ct.h: device pointers owned by the caller, int64_t counts, `stream` a
 * hipStream_t passed as void*, CT_E_INVALID for bad arguments with nothing enqueued.
 * `lines` must be 128-byte aligned and hold `nlines` lines of `line_bytes` (64 or 128) bytes.
 */
#ifndef CT_ROOFLINE_H
#define CT_ROOFLINE_H

#include <stdint.h>

#include "ct.h"

#ifdef __cplusplus
extern "C" {
#endif

ct_status ctr_gather(const void *lines, int64_t nlines, int32_t line_bytes, const uint64_t *keys,
                     int64_t n, uint64_t *out, void *stream);
ct_status ctr_gather_cas(void *lines, int64_t nlines, int32_t line_bytes, const uint64_t *keys,
                         int64_t n, uint64_t *out, void *stream);
ct_status ctr_gather_cas_store(void *lines, int64_t nlines, int32_t line_bytes,
                               const uint64_t *keys, int64_t n, uint64_t *out, void *stream);
ct_status ctr_cas(void *words, int64_t nwords, const uint64_t *keys, int64_t n, void *stream);
ct_status ctr_amin(void *words, int64_t nwords, const uint64_t *keys, int64_t n, void *stream);
ct_status ctr_copy(const void *src, void *dst, int64_t bytes, void *stream);

#ifdef __cplusplus
}
#endif

#endif /* CT_ROOFLINE_H */
