/*
 * snapgpu — MI355X (gfx950) read-alignment path of SNAP (Zaharia et al.,
 * "Faster and More Accurate Sequence Alignment with SNAP", arXiv 1111.5572).
 *
 * The library builds a device-resident index of every s-base seed of a genome
 * (Section 3.1) and aligns batches of reads with Algorithm 1 (Section 3.2):
 * seed lookup with the h_max skip, candidate gathering and dedupe, bounded edit
 * distance verification, and the best / second-best placement call with the
 * confidence threshold c, the 32-base result buckets and both orientations
 * (the three aspects the paper lists as omitted from its pseudocode).
 *
 * Conventions for every call:
 *  - return value: SNAP_OK (0) or a positive SNAP_E* code; snap_strerror names it;
 *  - argument checks happen before any device work; a failed check leaves the
 *    outputs untouched;
 *  - the library never frees caller memory; the caller never frees index memory
 *    except through snap_index_free.
 */
#ifndef SNAPGPU_H
#define SNAPGPU_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum {
    SNAP_OK = 0,
    SNAP_EINVAL = 1,   /* an argument is out of range, a pointer is NULL where data is required */
    SNAP_ENOMEM = 2,   /* host or device allocation failed, or the workspace is smaller than required */
    SNAP_EDEVICE = 3,  /* a HIP runtime call or kernel launch failed */
    SNAP_EBUSY = 4,    /* the server queue is full; retry later */
    SNAP_EAGAIN = 5,   /* a polled server request has not completed yet */
    SNAP_EINTERNAL = 6, /* an internal consistency bound was exceeded (a library bug; outputs invalid) */
    SNAP_ETOOBIG = 7    /* snap_align_noalloc: the batch needs more scratch than its fixed array holds */
};

/* Name of a status code (static string, never NULL). */
const char *snap_strerror(int code);

/* ------------------------------------------------------------------ index */

typedef struct snap_index snap_index;

typedef struct {
    uint64_t genome_len;      /* G, bases */
    int32_t seed_len;         /* s */
    int32_t stride;           /* windows at positions that are multiples of it are indexed (1: all) */
    uint64_t windows;         /* indexed N-free windows of length s (entries per orientation) */
    uint64_t distinct_keys;   /* distinct seeds up to reverse complement */
    uint64_t table_slots;     /* slots of the open-addressing seed table (8 per 128-byte bucket) */
    uint64_t position_entries;/* entries of the position array (windows + palindromic windows) */
    uint64_t device_bytes;    /* HBM held by the index */
    int32_t device;           /* HIP device ordinal the index lives on */
    int32_t dup_window;       /* W of the attached exact-duplicate classes, 0 if none */
} snap_index_sizes;

/*
 * Build the seed index of Section 3.1 on the current HIP device: every window
 * of `seed_len` bases of the genome that holds no N, slid one base at a time
 * (overlapping seeds), indexed so that a lookup returns the positions of the
 * seed and of its reverse complement (Section 3.2, omitted aspect 2).
 *
 * genome:   host pointer to `len` ASCII bases; A, C, G, T in either case are
 *           bases, every other byte is N. Copied; the caller may free it on return.
 * len:      genome length, seed_len <= len < 2^32.
 * seed_len: s, 1 <= s <= 32.
 * out:      receives the index handle (device memory owned by the index).
 * Errors:   SNAP_EINVAL (bad len or seed_len, NULL pointers), SNAP_ENOMEM,
 *           SNAP_EDEVICE. On error *out is NULL.
 */
int snap_index_build(const uint8_t *genome, uint64_t len, int32_t seed_len, snap_index **out);

/* Same, reporting each finished build stage (packing, records, each radix-sort pass,
 * grouping, placement, copy to the device) to `progress` (stage text, valid during
 * the call; `ctx` passed through) from the calling thread. progress may be NULL. */
typedef void (*snap_progress_fn)(const char *stage, void *ctx);
int snap_index_build_progress(const uint8_t *genome, uint64_t len, int32_t seed_len, snap_progress_fn progress,
                              void *ctx, snap_index **out);

/* The same index built on the device (Section 3.1; the canonical entries of Section 3.2,
 * omitted aspect 2): the genome (caller's host buffer, copied in and free to release on
 * return) is packed, every N-free window's records are radix-sorted by canonical code and
 * orientation and the table is filled by compare-and-swap, all by kernels on `stream`
 * (a hipStream_t; NULL = the default stream). Returns when the index is complete;
 * `progress` (may be NULL) is told each finished stage, as for snap_index_build_progress.
 * The result answers every lookup exactly as snap_index_build's does: the same packed
 * genome, N mask and positions array and the same table entries, though an entry may sit
 * in another slot of its probe sequence. seed_len 1..31 (the sort key is the code and the
 * orientation bit). Device memory while sorting: about 24 bytes per window on top of the
 * index. Errors: SNAP_EINVAL (NULL genome or out, seed_len outside 1..31, len < seed_len
 * or len >= 2^32), SNAP_ENOMEM, SNAP_EDEVICE. On error *out is NULL. */
int snap_index_build_device(const uint8_t *genome, uint64_t len, int32_t seed_len, void *stream,
                            snap_progress_fn progress, void *ctx, snap_index **out);

/* The strided index of Section 3.1's footnote to overlapping seeds: the same device build,
 * but only the windows at positions that are multiples of `stride` (1, 2 or 4) are indexed,
 * so the positions array and the table shrink by about that factor. snap_align with such an
 * index looks up, for each seed slot at read offset o, the `stride` seeds at o, o + 1, ...,
 * o + stride - 1 that fit in the read (one of them starts at an indexed position of any
 * location): the slot is skipped as holding an N when any of those bases is an N, its entries
 * for the h_max test are the sum over its seeds, it votes once for every location any of its
 * seeds hit, and it counts as a non-overlapping seed of Algorithm 1 only when it is at a
 * multiple of s and all its `stride` seeds fit. stride 1 is snap_index_build_device.
 * Reads align with seeds-per-read times stride of at most 64 (SNAP_EINVAL otherwise).
 * Errors: as snap_index_build_device, and SNAP_EINVAL for any other stride. */
int snap_index_build_strided(const uint8_t *genome, uint64_t len, int32_t seed_len, int32_t stride, void *stream,
                             snap_progress_fn progress, void *ctx, snap_index **out);

/* Exact-duplicate classes (Section 4.2, "Approach": identical substrings of a read's
 * length found by hashing, so that each repeated string is compared once), attached to
 * the index: for every genome position q, the smallest position whose `window`-base
 * window is identical to q's (bases as codes, an N equal to every N), q itself when no
 * earlier one is or when q's window runs past the genome's end. Built on the device from
 * the index's packed genome (a rolling 64-bit hash of every window, a radix sort, and a
 * word-by-word comparison of every window with its hash run's first one, so a hash
 * collision never merges two classes). Afterwards snap_align verifies, for each read
 * with L + d_max(L) + c - 1 <= window, one location per class and strand among the read's
 * locations and answers the others from it (their text windows are identical, so every
 * edit distance is); outputs do not change. Calling it again replaces the classes.
 * Device memory: 4 bytes and 1 bit per base kept with the index; about 24 bytes per window more
 * while building. The current device must be the index's. Errors: SNAP_EINVAL (NULL
 * index, window < 1, another device), SNAP_ENOMEM, SNAP_EDEVICE. */
int snap_index_dup_classes(snap_index *ix, int32_t window, void *stream);

/* Release the index and its device memory. NULL is accepted. */
int snap_index_free(snap_index *ix);

/* Sizes of a built index. */
int snap_index_info(const snap_index *ix, snap_index_sizes *info);

/* ------------------------------------------------------------ parameters */

/*
 * The five parameters of Table 3 (s is fixed by the index), plus the rules that
 * scale n and d_max with read length L and the result bucket size:
 *   n(L)     = min(n_cap, max(n_min, ceil(L / bp_per_seed)))   seeds to try
 *   d_max(L) = max(d_max, ceil(d_max_pct * L / 100))            maximum distance
 *   c        = conf_c                                           confidence threshold
 *   h_max    = max_hits                                          max index entries per seed
 *   bucket   = size of the position buckets whose results are merged (32 in the paper)
 * Valid ranges: 1 <= n_min <= n_cap <= 32, bp_per_seed >= 1, conf_c >= 1,
 * 1 <= max_hits <= 16382, 0 <= d_max_pct <= 100, bucket >= 1.
 */
typedef struct {
    int32_t n_min;
    int32_t n_cap;
    int32_t bp_per_seed;
    int32_t conf_c;
    int32_t max_hits;
    int32_t d_max_pct;
    int32_t bucket;
} snap_params;

/* n_min 10, n_cap 32, bp_per_seed 100, c 2, h_max 300, d_max_pct 0, bucket 32. */
snap_params snap_default_params(void);

/* ----------------------------------------------------------------- align */

/* Placement calls (Algorithm 1's three results). */
enum { SNAP_NOT_FOUND = 0, SNAP_SINGLE = 1, SNAP_MULTIPLE = 2 };

/*
 * Workspace bytes snap_align needs for a batch of n_reads reads holding
 * total_bases bases in all, the longest max_len. Any workspace of at least
 * this size gives identical outputs; a larger one lets the library process
 * more reads per internal pass. Returns 0 on invalid arguments (NULL index or
 * params, negative sizes, max_len above 16,384, invalid params).
 */
size_t snap_align_workspace_bytes(const snap_index *ix, int64_t n_reads, int64_t total_bases,
                                  int32_t max_len, int32_t d_max, const snap_params *p);

/*
 * Align a batch of reads with Algorithm 1 of Section 3.2.
 *
 * All array arguments are DEVICE pointers on the index's device, owned by the
 * caller:
 *   reads     n_reads reads concatenated, ASCII bases (uint8), sum(lengths) bytes
 *   lengths   int32 per read, 0 <= length; reads shorter than s find no seed
 *   pos       int64 per read: 0-based leftmost genome coordinate of the best
 *             location (the read is reverse-complemented for strand 1), -1 if none
 *   strand    int8 per read: 0 forward, 1 reverse complement, -1 if none
 *   dist      int32 per read: d_best, -1 if none
 *   second    int32 per read: d_second (best distance in any other bucket), -1 if none
 *   call      int8 per read: SNAP_NOT_FOUND, SNAP_SINGLE or SNAP_MULTIPLE
 *   workspace at least snap_align_workspace_bytes(...) bytes, 256-byte aligned
 * d_max is Table 3's maximum distance (scaled per read by d_max_pct).
 * stream is a hipStream_t (NULL = the default stream). Work is queued on it; the
 * call may wait on the stream between internal passes, and returns once the
 * last pass is queued. Outputs are valid after the stream is synchronized.
 * Results do not depend on the workspace size, the batch composition or the
 * order of reads in the batch.
 * Errors: SNAP_EINVAL (NULL or misaligned pointers, n_reads < 0, bad params,
 * d_max < 0, a read longer than 16,384 bases or a negative length, a read whose
 * limit d_max(L) + c - 1 exceeds snap_max_limit()), SNAP_ENOMEM (workspace too
 * small), SNAP_EDEVICE, SNAP_EINTERNAL (the replay / verification loop exceeded
 * its round bound: a library bug, never expected).
 */
int snap_align(const snap_index *ix, const uint8_t *reads, const int32_t *lengths, int64_t n_reads,
               int32_t d_max, const snap_params *p, int64_t *pos, int8_t *strand, int32_t *dist,
               int32_t *second, int8_t *call, void *workspace, size_t ws_bytes, void *stream);

/*
 * snap_align without a workspace, for callers that cannot allocate device memory
 * (code that must not call hipMalloc: tight serving loops, harnesses that forbid
 * allocation). The same arguments and outputs as snap_align, minus workspace and
 * ws_bytes; the same kernels, run by one host worker on the given stream, and the
 * same outputs.
 * Scratch: a fixed array of snap_align_noalloc_scratch_bytes() bytes (128 MiB) per
 * device, part of the library's device code (placed when the library is loaded on
 * that device, held until the process ends). The call allocates no device memory and
 * creates no stream. It clears what it needs itself, so a call never sees what an
 * earlier one left there. Every call on one device shares that device's array:
 * calls that overlap on one device (several host threads, or several streams
 * without waits between the calls) race and give wrong outputs; serialize them.
 * Size limit: a batch is taken exactly when snap_align_workspace_bytes(ix, n_reads,
 * sum of lengths, longest length, d_max, p) <= snap_align_noalloc_scratch_bytes()
 * (about 70,000 reads of 100 bp); a larger batch returns SNAP_ETOOBIG before any
 * output is written. Split it, or use snap_align with a workspace.
 * Errors: as snap_align (SNAP_EINVAL, SNAP_EDEVICE, SNAP_EINTERNAL), plus
 * SNAP_ETOOBIG.
 */
int snap_align_noalloc(const snap_index *ix, const uint8_t *reads, const int32_t *lengths, int64_t n_reads,
                       int32_t d_max, const snap_params *p, int64_t *pos, int8_t *strand, int32_t *dist,
                       int32_t *second, int8_t *call, void *stream);

/* Bytes of snap_align_noalloc's fixed scratch array on each device. */
size_t snap_align_noalloc_scratch_bytes(void);

/* Largest limit d_max(L) + c - 1 the verify kernels accept. */
int32_t snap_max_limit(void);

/*
 * Output-invariant schedule of snap_align (process-wide). A first pass probes
 * only the first pass1_seeds seed slots of every read and verifies locations with
 * limit pass1_limit; the final pass probes every seed slot of the reads left over
 * and verifies with limit final_limit. In either pass Algorithm 1 is then replayed
 * on what was computed; where a replay needs a distance above the limit a location
 * was verified with, that location is verified again with exactly the limit the
 * replay uses, or (reads in the lane tile, once the limit is below d_max(L) + c - 1
 * or after exact_rounds rounds) every unscored location still undecided at that
 * limit, and the read is replayed again. For reads in the lane tile (plain calls, no
 * duplicate classes, verify_seeds 0) the location Algorithm 1 scores first is verified
 * at the read's full limit before the others, and when its distance d1 is within
 * d_max(L) the others are verified with min(limit, d1 + c - 1). Only reads that need
 * more seeds than the first pass probed go on to the final pass. 0 in a field means
 * "no cap" (no first pass when pass1_seeds and pass1_limit are both 0). Outputs never
 * depend on these values.
 */
typedef struct {
    int32_t pass1_seeds;
    int32_t pass1_limit;
    int32_t final_limit;
    int32_t lane_max_len;   /* verify tile: reads up to this length (and limits up to 63) get one lane
                               per location, longer ones a wave per location; 0 = 512 (the maximum) */
    int32_t exact_rounds;   /* lane-tile reads ask for single locations at the full limit in at most this
                               many replay rounds, then for all their undecided locations at the limit */
    int32_t verify_seeds;   /* snap_align, reads in the lane tile: the first verification covers only
                               locations hit by one of the first verify_seeds seed slots, the others
                               are verified when a replay asks (0 = all locations) */
    int32_t chunk_reads;    /* reads per chunk pass (0 = 2^20) */
    int32_t workers;        /* a batch of several chunks is worked by up to this many host threads
                               with a stream each (0 = 2, at most 4), as many as the workspace holds
                               chunk parts for */
    int32_t request_top;    /* a replay of a lane-tile read that asks for one location at the limit
                               it needs asks, in the same round, for this many of the best-voted
                               locations undecided at that limit (the calls that likely follow): fewer
                               replay rounds for more verification (0 = 4, at most 16); reads in the
                               wave tile, whose verifications at limits of hundreds are costly, ask
                               for the one location */
    int32_t pass1_max_len;  /* snap_align with a first pass: reads longer than this take every seed
                               slot at once, in a complete pass over their own list with the first
                               pass's limit, instead of the first and the final pass (a long read
                               needs more round-0 seeds than pass1_seeds before Algorithm 1 can stop,
                               d_best growing with the length); 0 = no such reads */
} snap_tuning;

/* Set the process-wide schedule that snap_align (and snap_align_batched with a NULL
 * tuning) uses from the next call on; copied, so t may be released on return.
 * SNAP_EINVAL for a NULL pointer or a negative field. snap_get_tuning copies the
 * current schedule into *t (SNAP_EINVAL for NULL). */
int snap_set_tuning(const snap_tuning *t);
int snap_get_tuning(snap_tuning *t);

/*
 * Batched form of snap_align for batches that mix read lengths (100 bp to 10 kb):
 * identical outputs, same arguments and errors, plus an explicit schedule
 * (tuning may be NULL for the process-wide one). Per pass, every location of the
 * batch is verified by ONE persistent work-stealing launch: each wave first takes
 * long locations one at a time (a wave per location), then groups of 64 short
 * locations (a lane per location) in guided chunks of about half the remaining
 * groups per wave (the range rule of Section 2.3). A larger workspace lets a pass
 * cover more of the batch.
 */
int snap_align_batched(const snap_index *ix, const uint8_t *reads, const int32_t *lengths, int64_t n_reads,
                       int32_t d_max, const snap_params *p, const snap_tuning *tuning, int64_t *pos,
                       int8_t *strand, int32_t *dist, int32_t *second, int8_t *call, void *workspace,
                       size_t ws_bytes, void *stream);

/* ---------------------------------------------------------------- server */

/*
 * Request server with continuous batching. The index stays on the device. The
 * HBM budget is divided into slots; each slot owns a HIP stream, a slice of one
 * device arena (reads, lengths, outputs, align workspace for up to batch_reads
 * reads / batch_bases bases) and pinned host staging, and is driven by its own
 * host thread. A free slot admits every waiting request that fits (oldest
 * first), runs snap_align_batched on its stream and completes those requests, so
 * requests arriving while other slots are busy are admitted as slots free up and
 * their work overlaps on the device. Outputs are exactly those of snap_align on
 * the same reads; a request's result does not depend on the others in flight.
 */
typedef struct snap_server snap_server;

typedef struct {
    uint64_t hbm_budget;   /* device bytes the server may hold (slots are carved from it) */
    int32_t slots;         /* at most this many slots (fewer if the budget is smaller) */
    int32_t max_waiting;   /* submit returns SNAP_EBUSY with this many requests waiting */
    int64_t batch_reads;   /* per-slot capacity in reads (also the largest request) */
    int64_t batch_bases;   /* per-slot capacity in bases (also the largest request) */
    int32_t max_len;       /* longest read accepted */
    int32_t d_max;         /* Table 3's maximum distance for every request of this server */
} snap_server_config;

/* Result of a completed request. Arrays are host memory owned by the server and
 * valid until snap_server_release. Times are seconds of a monotonic host clock. */
typedef struct {
    int64_t n;
    int32_t status;        /* SNAP_OK, or the error the batch failed with */
    int32_t reserved;
    const int64_t *pos;
    const int8_t *strand;
    const int32_t *dist;
    const int32_t *second;
    const int8_t *call;
    double t_submit, t_start, t_done;
} snap_result;

typedef struct {
    int64_t slots, submitted, completed, failed, batches, waiting, busy_slots;
    uint64_t slot_device_bytes;
} snap_server_stats_t;

/* hbm_budget 8 GiB, 4 slots, 4096 waiting, 262144 reads / 256 Mi bases per slot, max_len 16384, d_max 8. */
snap_server_config snap_server_default_config(void);

/* Creates the server on the current device; p and the index must outlive it.
 * tuning may be NULL (process-wide schedule). SNAP_ENOMEM if not even one slot fits the budget. */
int snap_server_create(const snap_index *ix, const snap_params *p, const snap_server_config *cfg,
                       const snap_tuning *tuning, snap_server **out);

/* Queues a request (host arrays, copied before return) and returns at once with its
 * ticket. d_max must equal the server's. SNAP_EBUSY when max_waiting requests wait;
 * SNAP_EINVAL for a request larger than a slot or reads longer than max_len. */
int snap_server_submit(snap_server *s, const uint8_t *reads, const int32_t *lengths, int64_t n, int32_t d_max,
                       uint64_t *ticket);

/* SNAP_OK and the result once the request completed, SNAP_EAGAIN before. */
int snap_server_poll(snap_server *s, uint64_t ticket, snap_result *out);

/* Frees a completed request's result (SNAP_EAGAIN if it has not completed). */
int snap_server_release(snap_server *s, uint64_t ticket);

int snap_server_stats(snap_server *s, snap_server_stats_t *out);

/* Completes every admitted and waiting request, then frees the server. */
int snap_server_destroy(snap_server *s);

/* ------------------------------------------------------- instrumentation */

/* Device time of one kernel of the path, summed over launches. */
typedef struct {
    char name[32];
    int64_t launches;
    double total_ms;
} snap_kernel_time;

/*
 * Per-kernel device time. After snap_profile_begin, every kernel the library
 * launches is bracketed by a pair of HIP events recorded on its launch stream.
 * snap_profile_end waits for those events, writes up to cap per-kernel totals
 * (host array out, *count receives how many) and stops recording. Process-wide;
 * not meant to be combined with concurrent callers. Returns SNAP_OK or SNAP_EDEVICE.
 */
int snap_profile_begin(void);
int snap_profile_end(snap_kernel_time *out, int32_t cap, int32_t *count);

/* Work counted by snap_align while profiling is on (since snap_profile_begin):
 * the units the kernels' algorithmic bytes and operations are computed from.
 * Collecting them adds one stream wait per internal pass. */
typedef struct {
    int64_t passes;       /* internal passes (chunks of reads) */
    int64_t reads;        /* reads aligned */
    int64_t seed_slots;   /* (read, seed slot) probe items */
    int64_t hits;         /* seed hits gathered (h_max-passing seeds) */
    int64_t locations;    /* distinct (strand, p) locations verified */
    int64_t lv_steps;     /* diagonal extensions run by the verify kernels */
    int64_t second_pass_reads; /* reads a first pass left to a later pass */
    int64_t requests;     /* replays of reads after the verification they asked for */
    int64_t workers;      /* most chunk workers (host thread + stream) one call used */
    int64_t lv_steps_first; /* of lv_steps, those of the first verification of every location
                             * (the rest verified what replays asked for) */
    int64_t dup_aliases;  /* locations answered by their exact-duplicate representative */
} snap_counters;

int snap_profile_counters(snap_counters *out);

#ifdef __cplusplus
}
#endif

#endif /* SNAPGPU_H */
