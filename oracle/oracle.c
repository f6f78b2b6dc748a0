/*
 * CPU oracle for the SNAP read-alignment path — TEST INFRASTRUCTURE ONLY.
 *
 * Written from the paper (Zaharia et al., "Faster and More Accurate Sequence
 * Alignment with SNAP", arXiv 1111.5572): Section 3.1 (hash index), Section 3.2
 * (local alignment, Algorithm 1, Table 3 parameters, and the three aspects the
 * pseudocode omits). Points the paper leaves open are settled by the readings
 * listed beside each function. Nothing here is shared with the GPU path, and
 * only tests, the smoke check and the benchmark's CPU-baseline leg load it.
 *
 * Parity status: every function below is pinned by the CPU test suite (worked
 * examples of the paper, closed forms, brute force on tiny inputs, invariants).
 */
#define _GNU_SOURCE
#include "oracle.h"

#include <pthread.h>
#include <stdlib.h>
#include <string.h>
#include <unistd.h>

/* ------------------------------------------------------------- alphabet */

/* A, C, G, T in either case are the bases 0..3; every other byte is N (4). */
static int code_of(uint8_t b) {
    switch (b) {
        case 'A': case 'a': return 0;
        case 'C': case 'c': return 1;
        case 'G': case 'g': return 2;
        case 'T': case 't': return 3;
        default: return 4;
    }
}

/* Complement A<->T, C<->G, N<->N. */
static int comp_code(int c) { return c < 4 ? 3 - c : 4; }

/* ---------------------------------------------------------------- index */

/*
 * Section 3.1: the index maps every seed string of length s to the list of
 * genome positions where it occurs, over overlapping windows (a window slid one
 * base at a time). Here it is the plainest form of that map: all (window, q)
 * pairs sorted by window then position, searched by binary search. Windows that
 * hold an N are not seeds and are left out. The reverse-complement orientation
 * (omitted aspect 2 of Section 3.2) is handled at lookup time by also searching
 * the reverse complement of the seed.
 */
typedef struct { uint64_t key; int64_t q; } entry;

struct orc_index {
    int32_t s;
    int32_t stride;   /* windows at positions q with q % stride == 0 are indexed */
    int64_t G;
    uint8_t *codes;   /* genome as codes 0..4 */
    int64_t n;        /* number of N-free windows */
    entry *e;         /* sorted by (key, q) */
};

/* A seed as a base-4 number, first base most significant; -1 if it holds an N. */
static int64_t key_of_codes(const uint8_t *c, int32_t s) {
    uint64_t k = 0;
    for (int32_t i = 0; i < s; i++) {
        if (c[i] > 3) return -1;
        k = (k << 2) | c[i];
    }
    return (int64_t)k;
}

/* The same, for a seed that must hold no N (full 64-bit range for s = 32). */
static uint64_t key_u64(const uint8_t *c, int32_t s) {
    uint64_t k = 0;
    for (int32_t i = 0; i < s; i++) k = (k << 2) | c[i];
    return k;
}

static int has_n(const uint8_t *c, int32_t s) {
    for (int32_t i = 0; i < s; i++) if (c[i] > 3) return 1;
    return 0;
}

static int cmp_entry(const void *a, const void *b) {
    const entry *x = (const entry *)a, *y = (const entry *)b;
    if (x->key != y->key) return x->key < y->key ? -1 : 1;
    if (x->q != y->q) return x->q < y->q ? -1 : 1;
    return 0;
}

/*
 * Strided index (the footnote to "Overlapping Seeds" in Section 3.1): a window slid
 * `stride` bases at a time instead of one, i.e. only the windows at positions that are
 * multiples of the stride are indexed; stride 1 is the index of every overlapping window.
 */
static orc_index *build_plain(const uint8_t *genome, int64_t len, int32_t s, int32_t stride) {
    if (s < 1 || s > 32 || len < 0 || stride < 1) return NULL;
    orc_index *ix = (orc_index *)calloc(1, sizeof(orc_index));
    ix->s = s;
    ix->stride = stride;
    ix->G = len;
    ix->codes = (uint8_t *)malloc(len > 0 ? (size_t)len : 1);
    for (int64_t i = 0; i < len; i++) ix->codes[i] = (uint8_t)code_of(genome[i]);
    int64_t m = 0;
    for (int64_t q = 0; q + s <= len; q++) if (q % stride == 0 && !has_n(ix->codes + q, s)) m++;
    ix->e = (entry *)malloc((size_t)(m > 0 ? m : 1) * sizeof(entry));
    m = 0;
    for (int64_t q = 0; q + s <= len; q++) {
        if (q % stride != 0 || has_n(ix->codes + q, s)) continue;
        ix->e[m].key = key_u64(ix->codes + q, s);
        ix->e[m].q = q;
        m++;
    }
    ix->n = m;
    qsort(ix->e, (size_t)m, sizeof(entry), cmp_entry);
    return ix;
}

orc_index *orc_index_build(const uint8_t *genome, int64_t len, int32_t s) { return build_plain(genome, len, s, 1); }

/*
 * The same index built by `threads` threads; the result is the same sorted array of
 * (window, position) pairs, byte for byte. Plain bucket sort: the windows are split
 * into contiguous ranges, one per thread; each thread counts its windows per bucket
 * (the leading bits of the window), every (bucket, thread) pair gets its place from a
 * prefix sum, each thread writes its pairs there, and the buckets are then sorted one
 * by one with qsort, threads taking the next unsorted bucket in turn.
 */
typedef struct {
    orc_index *ix;
    int64_t q0, q1;        /* window range of this thread */
    int32_t shift;         /* bucket = key >> shift */
    int64_t *cnt;          /* per bucket: windows of this thread, then its write cursor */
    int phase;             /* 0 count, 1 scatter */
} build_part;

typedef struct {
    orc_index *ix;
    const int64_t *boff;   /* bucket b spans [boff[b], boff[b+1]) */
    int64_t nbuckets;
    int64_t next;
    pthread_mutex_t mu;
} sort_job;

/* Windows [q0, q1): the key of each is kept rolling (two bits in, two bits out) and a
 * window holds an N exactly when the last N seen lies inside it. */
static void *build_pass(void *arg) {
    build_part *bp = (build_part *)arg;
    orc_index *ix = bp->ix;
    const int32_t s = ix->s;
    const uint64_t mask = s >= 32 ? ~0ull : ((1ull << (2 * s)) - 1);
    if (bp->q1 <= bp->q0) return NULL;
    uint64_t key = 0;
    int64_t last_n = bp->q0 - 1;
    for (int64_t i = bp->q0; i < bp->q1 + s - 1; i++) {
        int c = ix->codes[i];
        if (c > 3) { last_n = i; c = 0; }
        key = ((key << 2) | (uint64_t)c) & mask;
        const int64_t q = i - s + 1;
        if (q < bp->q0 || last_n >= q || q % ix->stride != 0) continue;
        const int64_t b = (int64_t)(key >> bp->shift);
        if (bp->phase == 0) {
            bp->cnt[b]++;
        } else {
            entry *e = &ix->e[bp->cnt[b]++];
            e->key = key;
            e->q = q;
        }
    }
    return NULL;
}

typedef struct { const uint8_t *genome; uint8_t *codes; int64_t a, b; } code_part;

static void *code_pass(void *arg) {
    code_part *cp = (code_part *)arg;
    for (int64_t i = cp->a; i < cp->b; i++) cp->codes[i] = (uint8_t)code_of(cp->genome[i]);
    return NULL;
}

static void *sort_buckets(void *arg) {
    sort_job *sj = (sort_job *)arg;
    for (;;) {
        pthread_mutex_lock(&sj->mu);
        const int64_t b = sj->next++;
        pthread_mutex_unlock(&sj->mu);
        if (b >= sj->nbuckets) break;
        const int64_t n = sj->boff[b + 1] - sj->boff[b];
        if (n > 1) qsort(sj->ix->e + sj->boff[b], (size_t)n, sizeof(entry), cmp_entry);
    }
    return NULL;
}

orc_index *orc_index_build_strided(const uint8_t *genome, int64_t len, int32_t s, int32_t stride,
                                   int32_t threads) {
    if (threads <= 1) return build_plain(genome, len, s, stride);
    if (s < 1 || s > 32 || len < 0 || stride < 1) return NULL;
    if (threads > 256) threads = 256;
    orc_index *ix = (orc_index *)calloc(1, sizeof(orc_index));
    ix->s = s;
    ix->stride = stride;
    ix->G = len;
    ix->codes = (uint8_t *)malloc(len > 0 ? (size_t)len : 1);
    code_part cp[256];
    pthread_t th[256];
    for (int32_t t = 0; t < threads; t++) {
        cp[t].genome = genome;
        cp[t].codes = ix->codes;
        cp[t].a = len * t / threads;
        cp[t].b = len * (t + 1) / threads;
        pthread_create(&th[t], NULL, code_pass, &cp[t]);
    }
    for (int32_t t = 0; t < threads; t++) pthread_join(th[t], NULL);
    const int64_t nwin = len >= s ? len - s + 1 : 0;
    const int32_t bits = 2 * s < 16 ? 2 * s : 16;
    const int64_t nb = (int64_t)1 << bits;
    build_part *bp = (build_part *)calloc((size_t)threads, sizeof(build_part));
    for (int32_t t = 0; t < threads; t++) {
        bp[t].ix = ix;
        bp[t].q0 = nwin * t / threads;
        bp[t].q1 = nwin * (t + 1) / threads;
        bp[t].shift = 2 * s - bits;
        bp[t].cnt = (int64_t *)calloc((size_t)nb, sizeof(int64_t));
        bp[t].phase = 0;
        pthread_create(&th[t], NULL, build_pass, &bp[t]);
    }
    for (int32_t t = 0; t < threads; t++) pthread_join(th[t], NULL);
    /* bucket b, thread t writes from boff[b] + (windows of b in threads before t) */
    int64_t *boff = (int64_t *)malloc(sizeof(int64_t) * (size_t)(nb + 1));
    int64_t m = 0;
    for (int64_t b = 0; b < nb; b++) {
        boff[b] = m;
        for (int32_t t = 0; t < threads; t++) {
            const int64_t c = bp[t].cnt[b];
            bp[t].cnt[b] = m;
            m += c;
        }
    }
    boff[nb] = m;
    ix->n = m;
    ix->e = (entry *)malloc((size_t)(m > 0 ? m : 1) * sizeof(entry));
    for (int32_t t = 0; t < threads; t++) {
        bp[t].phase = 1;
        pthread_create(&th[t], NULL, build_pass, &bp[t]);
    }
    for (int32_t t = 0; t < threads; t++) pthread_join(th[t], NULL);
    sort_job sj;
    sj.ix = ix;
    sj.boff = boff;
    sj.nbuckets = nb;
    sj.next = 0;
    pthread_mutex_init(&sj.mu, NULL);
    for (int32_t t = 0; t < threads; t++) pthread_create(&th[t], NULL, sort_buckets, &sj);
    for (int32_t t = 0; t < threads; t++) pthread_join(th[t], NULL);
    pthread_mutex_destroy(&sj.mu);
    for (int32_t t = 0; t < threads; t++) free(bp[t].cnt);
    free(bp);
    free(boff);
    return ix;
}

orc_index *orc_index_build_threads(const uint8_t *genome, int64_t len, int32_t s, int32_t threads) {
    return orc_index_build_strided(genome, len, s, 1, threads);
}

int32_t orc_index_stride(const orc_index *ix) { return ix->stride; }

int64_t orc_index_entries(const orc_index *ix, uint64_t *keys, int64_t *qs, int64_t cap) {
    for (int64_t i = 0; i < ix->n && i < cap; i++) {
        keys[i] = ix->e[i].key;
        qs[i] = ix->e[i].q;
    }
    return ix->n;
}

void orc_index_free(orc_index *ix) {
    if (!ix) return;
    free(ix->codes);
    free(ix->e);
    free(ix);
}

int64_t orc_index_windows(const orc_index *ix) { return ix->n; }

/* [lo, hi) range of entries whose window equals key. */
static void occ_range(const orc_index *ix, uint64_t key, int64_t *lo_out, int64_t *hi_out) {
    int64_t lo = 0, hi = ix->n;
    while (lo < hi) { int64_t mid = lo + (hi - lo) / 2; if (ix->e[mid].key < key) lo = mid + 1; else hi = mid; }
    int64_t a = lo;
    hi = ix->n;
    while (lo < hi) { int64_t mid = lo + (hi - lo) / 2; if (ix->e[mid].key <= key) lo = mid + 1; else hi = mid; }
    *lo_out = a;
    *hi_out = lo;
}

int64_t orc_index_occ(const orc_index *ix, const uint8_t *seed, int64_t *out, int64_t cap) {
    uint8_t c[32];
    for (int32_t i = 0; i < ix->s; i++) c[i] = (uint8_t)code_of(seed[i]);
    int64_t k = key_of_codes(c, ix->s);
    if (k < 0 && has_n(c, ix->s)) return -1;
    int64_t lo, hi;
    occ_range(ix, key_u64(c, ix->s), &lo, &hi);
    for (int64_t i = lo; i < hi && i - lo < cap; i++) out[i - lo] = ix->e[i].q;
    return hi - lo;
}

/* --------------------------------------------------------- seed order */

/*
 * Omitted aspect 3 of Section 3.2: first as many back-to-back, non-overlapping
 * seeds as fit (offsets 0, s, 2s, ...), then the same again shifted by s/2, then
 * by s/4 and 3s/4, and so on. Reading of the "etc.": level k contributes the
 * shifts floor(j*s/2^k) for odd j in ascending order, a shift already used is
 * dropped, and levels continue until every shift 0..s-1 has appeared. Each shift
 * contributes the seeds shift, shift+s, ... that fit in the read. The first n
 * seeds of this sequence are tried.
 */
int32_t orc_seed_offsets(int32_t L, int32_t s, int32_t n, int32_t *out) {
    if (s < 1 || n <= 0) return 0;
    int32_t shifts[64];
    uint8_t seen[64];
    memset(seen, 0, sizeof(seen));
    int32_t ns = 0;
    shifts[ns++] = 0;
    seen[0] = 1;
    for (int32_t level = 1; ns < s && level < 31; level++) {
        int64_t den = (int64_t)1 << level;
        for (int64_t j = 1; j < den && ns < s; j += 2) {
            int32_t sh = (int32_t)(((int64_t)s * j) / den);
            if (!seen[sh]) { seen[sh] = 1; shifts[ns++] = sh; }
        }
    }
    int32_t cnt = 0;
    for (int32_t k = 0; k < ns && cnt < n; k++)
        for (int32_t o = shifts[k]; o + s <= L && cnt < n; o += s) out[cnt++] = o;
    return cnt;
}

/* Table 3 "seeds to try": n grows with read length (reading: one seed per
 * bp_per_seed bases, clamped to [n_min, n_cap]). */
int32_t orc_seeds_for_length(const orc_params *p, int32_t L) {
    int32_t want = (L + p->bp_per_seed - 1) / p->bp_per_seed;
    if (want < p->n_min) want = p->n_min;
    if (want > p->n_cap) want = p->n_cap;
    return want;
}

/* Table 3 "maximum distance", optionally a percentage of the read length
 * (integer ceiling, no floating point). */
int32_t orc_dmax_for_length(const orc_params *p, int32_t L) {
    int32_t pct = (int32_t)(((int64_t)p->d_max_pct * L + 99) / 100);
    return pct > p->d_max ? pct : p->d_max;
}

/* ---------------------------------------------------- edit distance */

/*
 * Section 3.2: EditDistance(Read, Reference[p], d_limit) returns the distance if
 * it is at most d_limit and a special value otherwise. Reading of what is
 * measured: unit-cost Levenshtein distance between the whole read and a prefix
 * of the reference text starting at p (start anchored at p, end free), N
 * matching nothing. This is the definition written out as the textbook table:
 * C[i][j] = distance between the first i read bases and the first j text bases,
 * C[0][j] = j, C[i][0] = i, and D = min over j of C[L][j]. The table is filled
 * in full; no band or early exit.
 */
static int32_t ed_codes(const uint8_t *R, int32_t L, const uint8_t *T, int32_t Tn, int32_t lim) {
    if (lim < 0) return ORC_INF;
    int32_t *prev = (int32_t *)malloc(sizeof(int32_t) * (size_t)(Tn + 1));
    int32_t *cur = (int32_t *)malloc(sizeof(int32_t) * (size_t)(Tn + 1));
    for (int32_t j = 0; j <= Tn; j++) prev[j] = j;
    for (int32_t i = 1; i <= L; i++) {
        cur[0] = i;
        for (int32_t j = 1; j <= Tn; j++) {
            int32_t match = (R[i - 1] < 4 && R[i - 1] == T[j - 1]) ? 0 : 1;
            int32_t v = prev[j - 1] + match;
            if (prev[j] + 1 < v) v = prev[j] + 1;
            if (cur[j - 1] + 1 < v) v = cur[j - 1] + 1;
            cur[j] = v;
        }
        int32_t *t = prev; prev = cur; cur = t;
    }
    int32_t D = prev[0];
    for (int32_t j = 1; j <= Tn; j++) if (prev[j] < D) D = prev[j];
    free(prev);
    free(cur);
    return D <= lim ? D : ORC_INF;
}

int32_t orc_edit_distance(const uint8_t *read, int32_t L, const uint8_t *text, int32_t T, int32_t lim) {
    uint8_t *r = (uint8_t *)malloc((size_t)L + 1), *t = (uint8_t *)malloc((size_t)T + 1);
    for (int32_t i = 0; i < L; i++) r[i] = (uint8_t)code_of(read[i]);
    for (int32_t i = 0; i < T; i++) t[i] = (uint8_t)code_of(text[i]);
    int32_t d = ed_codes(r, L, t, T, lim);
    free(r);
    free(t);
    return d;
}

/* ------------------------------------------------------- Algorithm 1 */

typedef struct { int64_t p; int32_t strand; int32_t hits; int32_t scored; } cand;
typedef struct { int32_t strand; int64_t bkey; int32_t d; int64_t p; } bucket;

typedef struct { int64_t p; int32_t strand; } vkey;

typedef struct {
    cand *c; int64_t nc, capc;
    vkey *v; int64_t nv, capv;   /* one slot's locations before they are voted */
    bucket *b; int64_t nb, capb;
    uint8_t *fwd, *rc; int32_t capL;
    int32_t offs[64];
} work;

typedef struct {
    int32_t d_best, d_second;
    int64_t best_p;
    int32_t best_strand;
} state;

static void work_free(work *w) { free(w->c); free(w->v); free(w->b); free(w->fwd); free(w->rc); }

static void slot_add(work *w, int64_t p, int32_t strand) {
    if (w->nv == w->capv) {
        w->capv = w->capv ? 2 * w->capv : 64;
        w->v = (vkey *)realloc(w->v, sizeof(vkey) * (size_t)w->capv);
    }
    w->v[w->nv].p = p;
    w->v[w->nv].strand = strand;
    w->nv++;
}

static int cmp_vkey(const void *a, const void *b) {
    const vkey *x = (const vkey *)a, *y = (const vkey *)b;
    if (x->p != y->p) return x->p < y->p ? -1 : 1;
    return (x->strand > y->strand) - (x->strand < y->strand);
}

/* SeedsHitting[(strand, p)] += 1, the map kept sorted by (p, strand). */
static void vote(work *w, int64_t p, int32_t strand) {
    int64_t lo = 0, hi = w->nc;
    while (lo < hi) {
        int64_t mid = lo + (hi - lo) / 2;
        const cand *m = &w->c[mid];
        if (m->p < p || (m->p == p && m->strand < strand)) lo = mid + 1; else hi = mid;
    }
    if (lo < w->nc && w->c[lo].p == p && w->c[lo].strand == strand) { w->c[lo].hits++; return; }
    if (w->nc == w->capc) {
        w->capc = w->capc ? 2 * w->capc : 64;
        w->c = (cand *)realloc(w->c, sizeof(cand) * (size_t)w->capc);
    }
    memmove(&w->c[lo + 1], &w->c[lo], sizeof(cand) * (size_t)(w->nc - lo));
    w->c[lo].p = p; w->c[lo].strand = strand; w->c[lo].hits = 1; w->c[lo].scored = 0;
    w->nc++;
}

/* "unscored location with the most seeds hitting"; ties go to the smaller p,
 * then to the forward strand (the map order). -1 if every location is scored. */
static int64_t select_unscored(const work *w) {
    int64_t k = -1;
    for (int64_t i = 0; i < w->nc; i++) {
        if (w->c[i].scored) continue;
        if (k < 0 || w->c[i].hits > w->c[k].hits) k = i;
    }
    return k;
}

/* The three-case d_limit rule of Algorithm 1. */
static int32_t d_limit(const state *st, int32_t dmax, int32_t c) {
    if (st->d_best > dmax) return dmax + c - 1;
    if (st->d_second >= st->d_best + c) return st->d_best + c - 1;
    return st->d_best - 1;
}

/*
 * Omitted aspect 1 of Section 3.2 (bucket merge): locations are grouped into
 * buckets of `bsize` positions per strand and only the best result of each
 * bucket is kept (the lowest distance, then the lowest p). d_best and the best
 * location are the lowest (distance, p, strand) over buckets; d_second is the
 * lowest distance among the other buckets. A result above the limit marks the
 * location scored and is not kept.
 */
static void record(work *w, state *st, int64_t p, int32_t strand, int32_t d, int32_t bsize) {
    if (d >= ORC_INF) return;
    int64_t bk = p / bsize;
    int64_t j;
    for (j = 0; j < w->nb; j++) if (w->b[j].strand == strand && w->b[j].bkey == bk) break;
    if (j == w->nb) {
        if (w->nb == w->capb) {
            w->capb = w->capb ? 2 * w->capb : 16;
            w->b = (bucket *)realloc(w->b, sizeof(bucket) * (size_t)w->capb);
        }
        w->b[j].strand = strand; w->b[j].bkey = bk; w->b[j].d = d; w->b[j].p = p;
        w->nb++;
    } else if (d < w->b[j].d || (d == w->b[j].d && p < w->b[j].p)) {
        w->b[j].d = d; w->b[j].p = p;
    }
    int64_t bi = -1;
    for (j = 0; j < w->nb; j++) {
        const bucket *x = &w->b[j];
        if (bi < 0) { bi = j; continue; }
        const bucket *y = &w->b[bi];
        if (x->d < y->d || (x->d == y->d && (x->p < y->p || (x->p == y->p && x->strand < y->strand)))) bi = j;
    }
    st->d_best = w->b[bi].d;
    st->best_p = w->b[bi].p;
    st->best_strand = w->b[bi].strand;
    st->d_second = ORC_INF;
    for (j = 0; j < w->nb; j++) if (j != bi && w->b[j].d < st->d_second) st->d_second = w->b[j].d;
}

typedef struct {
    int64_t *p; int8_t *strand; int32_t *d; int32_t *lim; int32_t cap; int32_t n;
} scorelog;

/* Score location k with the current d_limit: EditDistance(Read, Reference[p], d_limit). */
static void score(const orc_index *ix, work *w, state *st, int64_t k, int32_t L, int32_t dmax,
                  const orc_params *pr, orc_stats *stt, scorelog *lg) {
    cand *cd = &w->c[k];
    int32_t lim = d_limit(st, dmax, pr->conf_c);
    const uint8_t *R = cd->strand ? w->rc : w->fwd;
    int64_t tn = ix->G - cd->p;
    int64_t want = (int64_t)L + (lim > 0 ? lim : 0);
    if (tn > want) tn = want;
    int32_t d = ed_codes(R, L, ix->codes + cd->p, (int32_t)tn, lim);
    cd->scored = 1;
    stt->ed_calls++;
    if (d >= ORC_INF) stt->ed_over_limit++;
    if (lim >= 0) {
        /* statistic only: the diagonal extensions a furthest-reaching-diagonal evaluation
         * of this call runs at its own limit (rounds e = 0 .. min(D, lim), 2e + 1 diagonals
         * each); the distance above comes from the full table */
        const int64_t e = d < lim ? d : lim;
        stt->lv_extensions += (e + 1) * (e + 1);
    }
    if (lg && lg->n < lg->cap) {
        lg->p[lg->n] = cd->p; lg->strand[lg->n] = (int8_t)cd->strand; lg->d[lg->n] = d; lg->lim[lg->n] = lim;
        lg->n++;
    }
    record(w, st, cd->p, cd->strand, d, pr->bucket);
}

/*
 * Algorithm 1 for one read, with the readings for the points it leaves open:
 *  - a seed holding an N is not looked up and skips its iteration (it still uses
 *    up one of the n seed slots);
 *  - "# of index entries for S" counts both orientations (omitted aspect 2):
 *    positions of S plus positions of its reverse complement;
 *  - a forward hit at q of the seed at offset o votes for (+, q - o); a reverse
 *    hit votes for (-, q - (L - o - s)), the leftmost coordinate of the
 *    reverse-complemented read; locations with p < 0 or p + L > G are dropped;
 *  - "# non-overlapping seeds tested" counts the seeds at offsets that are
 *    multiples of s that were looked up and not over h_max;
 *  - when no unscored location exists the edit distance is skipped but both
 *    tests still run;
 *  - "score remaining locations" repeats the selection rule, recomputes d_limit
 *    before each call, and does not apply the early multiple-hits return;
 *  - "all seeds had > h_max entries" means at least one seed was looked up and
 *    every looked-up seed was over h_max.
 * With a strided index (stride > 1, Section 3.1's footnote) a seed slot at offset o
 * looks up the seeds at o, o + 1, ..., o + stride - 1 that fit the read: whatever the
 * location, one of them starts at an indexed position of it. The slot is skipped as a
 * seed with an N if any of those bases is an N; its entries for the h_max test are the
 * sum over its seeds; it votes once for each location any of its seeds hit; and it
 * counts in t only if it is a round-0 slot all of whose stride seeds fit (then the
 * round-0 slots cover disjoint stretches of the read for any one location, as with the
 * full index). With stride 1 every rule above is the plain one.
 * The state at termination is reported: best location, strand, d_best, d_second.
 */
static void align_one(const orc_index *ix, work *w, const uint8_t *read, int32_t L, const orc_params *pr,
                      int64_t *o_pos, int8_t *o_strand, int32_t *o_dist, int32_t *o_second, int8_t *o_call,
                      orc_stats *stt, scorelog *lg) {
    const int32_t s = ix->s, c = pr->conf_c, hmax = pr->max_hits;
    const int32_t dmax = orc_dmax_for_length(pr, L);
    if (L + 1 > w->capL) {
        w->capL = L + 1;
        w->fwd = (uint8_t *)realloc(w->fwd, (size_t)w->capL);
        w->rc = (uint8_t *)realloc(w->rc, (size_t)w->capL);
    }
    for (int32_t i = 0; i < L; i++) w->fwd[i] = (uint8_t)code_of(read[i]);
    for (int32_t i = 0; i < L; i++) w->rc[i] = (uint8_t)comp_code(w->fwd[L - 1 - i]);
    w->nc = 0;
    w->nb = 0;
    const int32_t nseeds = orc_seed_offsets(L, s, orc_seeds_for_length(pr, L), w->offs);

    state st = {ORC_INF, ORC_INF, -1, -1};
    int32_t t = 0, looked = 0, all_over = 1, call = -1;
    uint8_t rcseed[32];
    const int32_t stride = ix->stride;
    for (int32_t i = 0; i < nseeds && call < 0; i++) {
        const int32_t o = w->offs[i];
        /* the slot's seeds: offsets o, o + 1, ..., o + stride - 1, those that fit the read
         * (with stride 1, the one seed at o); one of them is aligned with the index's
         * stride for any location */
        int32_t np = 0;
        while (np < stride && o + np + s <= L) np++;
        if (has_n(w->fwd + o, s + np - 1)) { stt->seeds_with_n++; continue; }
        int64_t entries = 0;
        w->nv = 0;
        for (int32_t j = 0; j < np; j++) {
            const uint8_t *S = w->fwd + o + j;
            for (int32_t k = 0; k < s; k++) rcseed[k] = (uint8_t)comp_code(S[s - 1 - k]);
            int64_t flo, fhi, rlo, rhi;
            occ_range(ix, key_u64(S, s), &flo, &fhi);
            occ_range(ix, key_u64(rcseed, s), &rlo, &rhi);
            stt->index_lookups++;
            entries += (fhi - flo) + (rhi - rlo);
            for (int64_t e = flo; e < fhi; e++) {
                int64_t p = ix->e[e].q - (o + j);
                if (p >= 0 && p + L <= ix->G) slot_add(w, p, 0);
            }
            for (int64_t e = rlo; e < rhi; e++) {
                int64_t p = ix->e[e].q - (L - (o + j) - s);
                if (p >= 0 && p + L <= ix->G) slot_add(w, p, 1);
            }
        }
        looked = 1;
        stt->seeds_looked_up++;
        if (entries > hmax) { stt->seeds_over_limit++; continue; }
        all_over = 0;
        /* one vote per location per slot */
        qsort(w->v, (size_t)w->nv, sizeof(vkey), cmp_vkey);
        for (int64_t e = 0; e < w->nv; e++)
            if (e == 0 || cmp_vkey(&w->v[e], &w->v[e - 1]) != 0) vote(w, w->v[e].p, w->v[e].strand);
        if (o % s == 0 && np == stride) t++;
        int64_t k = select_unscored(w);
        stt->select_visits += w->nc;
        if (k >= 0) score(ix, w, &st, k, L, dmax, pr, stt, lg);
        if (st.d_best < c && st.d_second < st.d_best + c) {
            call = 2;   /* multiple hits: no better hit could be confident */
        } else if (st.d_best < ORC_INF && t >= st.d_best + c) {
            /* any location not yet found is at least t edits away */
            for (;;) {
                k = select_unscored(w);
                stt->select_visits += w->nc;
                if (k < 0) break;
                score(ix, w, &st, k, L, dmax, pr, stt, lg);
            }
            break;
        }
    }
    if (call < 0) {
        if (st.d_best <= dmax && st.d_second >= st.d_best + c) call = 1;
        else if (st.d_best <= dmax || (looked && all_over)) call = 2;
        else call = 0;
    }
    stt->candidates += w->nc;
    *o_pos = st.d_best < ORC_INF ? st.best_p : -1;
    *o_strand = (int8_t)(st.d_best < ORC_INF ? st.best_strand : -1);
    *o_dist = st.d_best < ORC_INF ? st.d_best : -1;
    *o_second = st.d_second < ORC_INF ? st.d_second : -1;
    *o_call = (int8_t)call;
}

int32_t orc_align_log(const orc_index *ix, const uint8_t *read, int32_t L, const orc_params *p,
                      int64_t *log_p, int8_t *log_strand, int32_t *log_d, int32_t *log_lim, int32_t cap) {
    work w;
    memset(&w, 0, sizeof(w));
    orc_stats stt;
    memset(&stt, 0, sizeof(stt));
    scorelog lg = {log_p, log_strand, log_d, log_lim, cap, 0};
    int64_t pos; int8_t strand, call; int32_t dist, second;
    align_one(ix, &w, read, L, p, &pos, &strand, &dist, &second, &call, &stt, &lg);
    work_free(&w);
    return lg.n;
}

/* ----------------------------------------------- exact-duplicate classes */

/*
 * Section 4.2, "Approach": regions of exact duplication are found by looking for
 * identical substrings of a read's length, so that a read is compared with each
 * repeated string only once. Reading: the string a read of length L is compared with at
 * location p is the text window G[p, p + L + K) (the edit distance of Section 3.2 at any
 * limit up to K = d_max + c - 1 never looks further), so two locations whose windows of
 * W >= L + K bases are identical give the same distance at every limit, and the
 * distance needs computing once per class of identical windows. Here the classes are
 * the definition written out: rep[p] is the smallest p' whose W-base window equals p's
 * (bases compared as codes, every N equal to every N; a window is identical only as a
 * whole), found by sorting the positions by window content; a position whose window
 * would run past the genome's end is its own class.
 */
static const uint8_t *dup_codes;
static int64_t dup_W;

static int cmp_window(const void *a, const void *b) {
    const int64_t x = *(const int64_t *)a, y = *(const int64_t *)b;
    const int c = memcmp(dup_codes + x, dup_codes + y, (size_t)dup_W);
    if (c) return c;
    return (x > y) - (x < y);
}

int32_t orc_dup_classes(const uint8_t *genome, int64_t len, int64_t W, int64_t *rep) {
    if (len < 0 || W < 1) return -1;
    uint8_t *codes = (uint8_t *)malloc(len > 0 ? (size_t)len : 1);
    for (int64_t i = 0; i < len; i++) codes[i] = (uint8_t)code_of(genome[i]);
    for (int64_t p = 0; p < len; p++) rep[p] = p;
    const int64_t n = len >= W ? len - W + 1 : 0;
    int64_t *order = (int64_t *)malloc((size_t)(n > 0 ? n : 1) * sizeof(int64_t));
    for (int64_t p = 0; p < n; p++) order[p] = p;
    dup_codes = codes;   /* qsort has no context argument; the oracle's callers are serial */
    dup_W = W;
    qsort(order, (size_t)n, sizeof(int64_t), cmp_window);
    for (int64_t k = 1; k < n; k++)
        if (memcmp(codes + order[k], codes + order[k - 1], (size_t)W) == 0) rep[order[k]] = rep[order[k - 1]];
    free(order);
    free(codes);
    return 0;
}

/* ------------------------------------------------------ multi-core driver */

/*
 * Section 2.3: a core takes a range of the input, processes all of it, then
 * takes another; a range is about half of the remaining work divided by the
 * number of cores, with a minimum size.
 */
typedef struct {
    const orc_index *ix; const uint8_t *reads; const int64_t *offsets; const int32_t *lengths;
    int64_t n; const orc_params *p;
    int64_t *pos; int8_t *strand; int32_t *dist; int32_t *second; int8_t *call;
    pthread_mutex_t mu; int64_t next; int32_t threads; int64_t min_chunk;
    orc_stats total;
} job;

static void *worker(void *arg) {
    job *jb = (job *)arg;
    work w;
    memset(&w, 0, sizeof(w));
    orc_stats stt;
    memset(&stt, 0, sizeof(stt));
    for (;;) {
        pthread_mutex_lock(&jb->mu);
        int64_t rem = jb->n - jb->next, lo = jb->next, take = rem / (2 * jb->threads);
        if (take < jb->min_chunk) take = jb->min_chunk;
        if (take > rem) take = rem;
        jb->next += take;
        pthread_mutex_unlock(&jb->mu);
        if (take <= 0) break;
        for (int64_t r = lo; r < lo + take; r++)
            align_one(jb->ix, &w, jb->reads + jb->offsets[r], jb->lengths[r], jb->p, jb->pos + r, jb->strand + r,
                      jb->dist + r, jb->second + r, jb->call + r, &stt, NULL);
    }
    pthread_mutex_lock(&jb->mu);
    jb->total.seeds_looked_up += stt.seeds_looked_up;
    jb->total.seeds_over_limit += stt.seeds_over_limit;
    jb->total.seeds_with_n += stt.seeds_with_n;
    jb->total.candidates += stt.candidates;
    jb->total.ed_calls += stt.ed_calls;
    jb->total.ed_over_limit += stt.ed_over_limit;
    jb->total.lv_extensions += stt.lv_extensions;
    jb->total.index_lookups += stt.index_lookups;
    jb->total.select_visits += stt.select_visits;
    pthread_mutex_unlock(&jb->mu);
    work_free(&w);
    return NULL;
}

int32_t orc_align(const orc_index *ix, const uint8_t *reads, const int64_t *offsets, const int32_t *lengths,
                  int64_t n, const orc_params *p, int64_t *pos, int8_t *strand, int32_t *dist,
                  int32_t *second, int8_t *call, orc_stats *stats, int32_t threads) {
    if (threads <= 0) threads = (int32_t)sysconf(_SC_NPROCESSORS_ONLN);
    if (threads < 1) threads = 1;
    if (threads > 256) threads = 256;
    job jb;
    memset(&jb, 0, sizeof(jb));
    jb.ix = ix; jb.reads = reads; jb.offsets = offsets; jb.lengths = lengths; jb.n = n; jb.p = p;
    jb.pos = pos; jb.strand = strand; jb.dist = dist; jb.second = second; jb.call = call;
    jb.threads = threads;
    jb.min_chunk = 64;
    pthread_mutex_init(&jb.mu, NULL);
    pthread_t th[256];
    for (int32_t i = 0; i < threads; i++) pthread_create(&th[i], NULL, worker, &jb);
    for (int32_t i = 0; i < threads; i++) pthread_join(th[i], NULL);
    pthread_mutex_destroy(&jb.mu);
    if (stats) *stats = jb.total;
    return threads;
}
