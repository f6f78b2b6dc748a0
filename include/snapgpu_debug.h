/*
 * snapgpu test hooks: host-side evaluations of the library's own index layout
 * and seed order (checkable without a GPU), and copies of device memory for the
 * GPU tests. Not part of the alignment path.
 */
#ifndef SNAPGPU_DEBUG_H
#define SNAPGPU_DEBUG_H

#include <stdint.h>

#include "snapgpu.h"

#ifdef __cplusplus
extern "C" {
#endif

/*
 * Builds the seed table of snap_index_build (Section 3.1) in host memory and
 * looks up nq seeds of seed_len ASCII bases each (queries, back to back) with
 * the probe sequence the device uses. Per query: fwd = windows equal to the seed,
 * rev = windows equal to its reverse complement (Section 3.2, omitted aspect 2),
 * first_fwd = smallest forward position or -1; -1/-1/-1 for a seed holding an N.
 * windows (may be NULL) receives the number of N-free windows. Host pointers
 * only. Returns SNAP_OK, SNAP_EINVAL or SNAP_ENOMEM.
 */
int snap_debug_host_lookup(const uint8_t *genome, uint64_t len, int32_t seed_len, const uint8_t *queries,
                           int64_t nq, int64_t *fwd, int64_t *rev, int64_t *first_fwd, uint64_t *windows);

/*
 * Offsets of the first n seeds tried for a read of length L with seed length s
 * (Section 3.2, omitted aspect 3). out holds at least n entries (n <= 64).
 * Returns the number written (fewer than n when the read holds fewer seeds).
 */
int32_t snap_debug_seed_offsets(int32_t L, int32_t s, int32_t n, int32_t *out);

/*
 * Copies `bytes` (a multiple of 4) from device src to device dst on `stream`
 * (hipStream_t) with a plain load/store kernel: a transfer of known size for
 * calibrating hardware byte counters. Returns SNAP_OK, SNAP_EINVAL, SNAP_EDEVICE.
 */
int snap_debug_copy(const void *src, void *dst, uint64_t bytes, void *stream);

/* Random-line gather microbenchmark (the access pattern of the seed probe and the
 * position reads): `threads` threads (a multiple of 256 and of line_bytes / 16) read, in
 * groups of line_bytes / 16 lanes, one line_bytes-byte line (32, 64 or 128) at a
 * pseudo-random line-aligned place of the device buffer `buf` (`bytes` long, 128-byte
 * aligned), `rounds` times each; each thread writes one uint32 to device `sink`.
 * Algorithmic bytes: threads * rounds * 16. Async on `stream`. Errors: SNAP_EINVAL,
 * SNAP_EDEVICE. */
int snap_debug_gather_lines(const void *buf, uint64_t bytes, int32_t line_bytes, int32_t rounds, uint64_t threads,
                            uint64_t seed, void *sink, void *stream);

/* Copy one device array of an index to host memory (for checks): which = 0 packed
 * genome (uint32 words), 1 N mask (uint32 words), 2 table (two uint64 per slot),
 * 3 positions (uint32). `bytes` must equal the array's size (from snap_index_info: G,
 * table_slots, position_entries). Synchronous. Errors: SNAP_EINVAL, SNAP_EDEVICE. */
int snap_debug_index_download(const snap_index *ix, int32_t which, void *host_dst, uint64_t bytes);

/* Copy the index's exact-duplicate class array (count = genome length entries of
 * uint32) to host memory. SNAP_EINVAL when the index has no classes or count differs. */
int snap_debug_dup_download(const snap_index *ix, uint32_t *host_dst, uint64_t count);

#ifdef __cplusplus
}
#endif

#endif /* SNAPGPU_DEBUG_H */
