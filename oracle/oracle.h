/*
 * CPU oracle for the SNAP read-alignment path — TEST INFRASTRUCTURE ONLY.
 *
 * Plain, slow, deliberately literal C: the hash index of Section 3.1 as a sorted
 * array of (s-mer, position) pairs, the seed order of Section 3.2 (omitted
 * aspect 3), the bounded edit distance of Section 3.2 as the textbook dynamic
 * program, and Algorithm 1 step by step with the bucket merge (omitted aspect 1)
 * and the two-orientation lookup (omitted aspect 2).
 *
 * Only the tests, the smoke check and the benchmark's CPU-baseline leg may load
 * this library. It shares no code with the GPU path.
 */
#ifndef SNAP_ORACLE_H
#define SNAP_ORACLE_H
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define ORC_INF 0x3FFFFFFF

typedef struct orc_index orc_index;

typedef struct {
    int32_t seed_len;     /* s */
    int32_t n_min, n_cap, bp_per_seed;   /* n(L) = min(n_cap, max(n_min, ceil(L/bp_per_seed))) */
    int32_t conf_c;       /* c */
    int32_t max_hits;     /* h_max */
    int32_t d_max;        /* d_max(L) = max(d_max, ceil(d_max_pct * L / 100)) */
    int32_t d_max_pct;
    int32_t bucket;       /* bucket size of the result merge */
} orc_params;

typedef struct {
    int64_t seeds_looked_up;   /* index lookups performed */
    int64_t seeds_over_limit;  /* lookups with more than h_max entries */
    int64_t seeds_with_n;      /* seed slots skipped because the seed holds an N */
    int64_t candidates;        /* distinct (strand, p) locations that received a vote */
    int64_t ed_calls;          /* EditDistance calls */
    int64_t ed_over_limit;     /* calls that returned the special value */
    int64_t lv_extensions;     /* sum over calls of (min(D, limit) + 1)^2: the diagonal extensions a
                                  furthest-reaching-diagonal evaluation runs at each call's own limit */
    int64_t index_lookups;     /* seeds looked up in the index (stride per seed slot with a strided index) */
    int64_t select_visits;     /* statistic: sum over selections of "the unscored location with the most
                                  seeds hitting" of the candidate locations looked at (the scan's length) */
} orc_stats;

/* Index: every N-free window of length s, as sorted (key, position) pairs. */
orc_index *orc_index_build(const uint8_t *genome, int64_t len, int32_t s);
/* The same index (identical sorted array) built by `threads` threads with a bucket sort;
 * threads <= 1 is orc_index_build. */
orc_index *orc_index_build_threads(const uint8_t *genome, int64_t len, int32_t s, int32_t threads);
/* Strided index (Section 3.1, footnote to "Overlapping Seeds"): only the windows at positions
 * q with q % stride == 0; stride 1 is orc_index_build_threads. Alignment with such an index
 * looks up `stride` consecutive seeds per seed slot (see orc_align). */
orc_index *orc_index_build_strided(const uint8_t *genome, int64_t len, int32_t s, int32_t stride,
                                   int32_t threads);
int32_t orc_index_stride(const orc_index *ix);
/* Copies up to cap (window key, position) pairs of the sorted array; returns the count. */
int64_t orc_index_entries(const orc_index *ix, uint64_t *keys, int64_t *qs, int64_t cap);
void orc_index_free(orc_index *ix);
int64_t orc_index_windows(const orc_index *ix);
/* Positions q with genome[q, q+s) == the s bases at `seed` (ASCII); -1 if the seed holds an N.
 * Writes up to `cap` positions (ascending) into `out` and returns the total count. */
int64_t orc_index_occ(const orc_index *ix, const uint8_t *seed, int64_t *out, int64_t cap);

/* Seed order: offsets of the seeds tried for a read of length L (up to n of them). */
int32_t orc_seed_offsets(int32_t L, int32_t s, int32_t n, int32_t *out);
int32_t orc_seeds_for_length(const orc_params *p, int32_t L);
int32_t orc_dmax_for_length(const orc_params *p, int32_t L);

/* Bounded edit distance on ASCII strings: D = min over j of Lev(read, text[0, j)),
 * N matching nothing. Returns D if D <= lim, else ORC_INF. */
int32_t orc_edit_distance(const uint8_t *read, int32_t L, const uint8_t *text, int32_t T, int32_t lim);

/* Algorithm 1 over reads [0, n). offsets has n+1 entries (byte offsets into reads).
 * Outputs per read: pos (-1 if none), strand (0 forward, 1 reverse complement, -1 none),
 * dist and second (-1 for none), call (0 not found, 1 single, 2 multiple).
 * stats may be NULL. threads <= 0 uses every online core. Returns the threads used. */
int32_t orc_align(const orc_index *ix, const uint8_t *reads, const int64_t *offsets, const int32_t *lengths,
                  int64_t n, const orc_params *p, int64_t *pos, int8_t *strand, int32_t *dist,
                  int32_t *second, int8_t *call, orc_stats *stats, int32_t threads);

/* Scored-location log of one read, for invariant checks: up to cap entries of
 * (p, strand, returned distance or ORC_INF, d_limit used). Returns entries written. */
int32_t orc_align_log(const orc_index *ix, const uint8_t *read, int32_t L, const orc_params *p,
                      int64_t *log_p, int8_t *log_strand, int32_t *log_d, int32_t *log_lim, int32_t cap);

/* Exact-duplicate classes of the genome's W-base windows (Section 4.2, "Approach"): rep[p]
 * (len entries) = the smallest position whose W-base window equals p's, or p itself (also for
 * positions whose window runs past the end). Not thread-safe. Returns 0, or -1 for bad sizes. */
int32_t orc_dup_classes(const uint8_t *genome, int64_t len, int64_t W, int64_t *rep);

#ifdef __cplusplus
}
#endif
#endif
