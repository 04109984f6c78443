/*
 * hm_roofline.h -- random-access rate probe for MI355X (gfx950).
 *
 * k-mer analysis spends its time in random, fine-grained reads and atomic
 * updates of a large hash table and Bloom filter (arXiv 1705.11147, section
 * "Parallel k-mer analysis": hash-table counting; section "Summary of
 * communication patterns and costs": fine-grained irregular lookups and
 * atomics are latency-bound).  This probe measures what one GPU sustains for
 * each access kind over a buffer of a chosen size, so the counting kernels
 * can be placed against a measured random-access ceiling as well as against
 * the HBM spec peak.
 *
 * hm_random_access: n_ops accesses of `kind` at uniformly random 8-byte words
 * (HM_RA_LINE_RMW: random 64-byte lines) of buf[0 .. n_words), n_words a
 * power of two >= 16.  The buffer is device memory owned by the caller; its
 * contents are modified by the atomic kinds.  `sink` (device, 1 word) keeps
 * loads from being optimized away.  Asynchronous on `stream`; time it with
 * events.  Returns 0 or a negative HM_E* code (hm_kmer.h).
 *   HM_RA_COPY: streaming copy of the first n_words/2 words onto the second
 *   half (n_ops ignored), the reference kernel for byte-counter scaling.
 *   Each thread keeps four independent accesses in flight, or one with
 *   HM_RA_SERIAL, so the probe also shows how much the rate depends on
 *   memory-level parallelism.
 */
#ifndef HM_ROOFLINE_H
#define HM_ROOFLINE_H

#include <stdint.h>

#include <hip/hip_runtime_api.h>

#ifdef __cplusplus
extern "C" {
#endif

#define HM_RA_LOAD 0          /* plain 8-byte load (cacheable) */
#define HM_RA_LOAD_COHERENT 1 /* device-scope relaxed atomic load */
#define HM_RA_ATOMIC_ADD 2    /* device-scope atomic add, result unused */
#define HM_RA_ATOMIC_OR_RET 3 /* device-scope atomic OR, result used (Bloom test-and-set) */
#define HM_RA_LINE_RMW 4      /* coherent load + two atomic adds on one 64-byte line (a table hit) */
#define HM_RA_COPY 5          /* streaming copy, for counter calibration */
#define HM_RA_PROBE_CAS 6     /* 16-byte load of a random 64-byte line, then a CAS of its second word with the
                                 loaded value (the counting pass's table hit) */
#define HM_RA_SERIAL 0x100    /* flag OR-ed into kind: one access in flight per thread instead of four */

int hm_random_access(uint64_t *buf, uint64_t n_words, int32_t kind, uint64_t n_ops, uint64_t seed, uint64_t *sink,
                     hipStream_t stream);

#ifdef __cplusplus
}
#endif

#endif /* HM_ROOFLINE_H */
