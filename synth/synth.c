/*
 * Seeded synthetic inputs: genomes and simulated reads.
 *
 * This module generates inputs only. It holds none of the alignment method's
 * arithmetic (no seeds, no index, no edit distance, no placement call), and is
 * shared by the CPU oracle's tests and by the GPU path's tests and benchmark.
 *
 * Stand-ins for the paper's workloads (Section 2: reads simulated from a human
 * reference with substitutions and indels; Table 1 short reads, Table 2 long
 * reads with a high share of indels):
 *   - uniform genome: i.i.d. A/C/G/T;
 *   - repeat genome: blocks of unique sequence, segmental duplicates of earlier
 *     sequence (optionally reverse-complemented, diverged), and tandem arrays,
 *     optionally overlaid with runs of N;
 *   - reads: a window sampled uniformly from either strand, walked base by base
 *     with per-base substitution and indel events.
 *
 * Random numbers: xoshiro256** (Blackman and Vigna, "Scrambled linear
 * pseudorandom number generators", 2018), seeded through splitmix64 (Steele,
 * Lea and Flood, "Fast splittable pseudorandom number generators", 2014).
 * Every read has its own stream, keyed by (seed, read index), so reads can be
 * generated in parallel or one at a time with identical results.
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#include <math.h>

typedef struct { uint64_t s[4]; } rng_t;

static uint64_t splitmix64(uint64_t *x) {
    uint64_t z = (*x += 0x9E3779B97F4A7C15ull);
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

static inline uint64_t rotl(uint64_t x, int k) { return (x << k) | (x >> (64 - k)); }

static uint64_t rng_next(rng_t *r) {
    uint64_t *s = r->s;
    uint64_t result = rotl(s[1] * 5, 7) * 9;
    uint64_t t = s[1] << 17;
    s[2] ^= s[0]; s[3] ^= s[1]; s[1] ^= s[2]; s[0] ^= s[3];
    s[2] ^= t; s[3] = rotl(s[3], 45);
    return result;
}

static void rng_seed(rng_t *r, uint64_t seed, uint64_t stream) {
    uint64_t x = seed ^ (stream * 0xD1B54A32D192ED03ull);
    x = splitmix64(&x) ^ stream;
    for (int i = 0; i < 4; i++) r->s[i] = splitmix64(&x);
}

/* uniform double in [0, 1) with 53 random bits */
static double rng_unif(rng_t *r) { return (double)(rng_next(r) >> 11) * (1.0 / 9007199254740992.0); }

/* uniform integer in [0, n), n >= 1 (rejection removes modulo bias) */
static uint64_t rng_below(rng_t *r, uint64_t n) {
    if (n <= 1) return 0;
    uint64_t lim = UINT64_MAX - (UINT64_MAX % n);
    uint64_t x;
    do { x = rng_next(r); } while (x >= lim);
    return x % n;
}

/* uniform integer in [lo, hi] */
static int64_t rng_range(rng_t *r, int64_t lo, int64_t hi) { return lo + (int64_t)rng_below(r, (uint64_t)(hi - lo + 1)); }

static const uint8_t BASES[4] = {'A', 'C', 'G', 'T'};

static inline uint8_t comp_base(uint8_t b) {
    switch (b) {
        case 'A': return 'T'; case 'C': return 'G'; case 'G': return 'C'; case 'T': return 'A';
        default: return 'N';
    }
}

static inline uint8_t other_base(rng_t *r, uint8_t b) {
    /* one of the three bases different from b (uniform); N is replaced by any base */
    uint8_t o;
    do { o = BASES[rng_below(r, 4)]; } while (o == b);
    return o;
}

/* truncated geometric(1/2) on 1..maxlen: P(l) = 2^-l for l < maxlen, the tail folded into maxlen */
static int trunc_geom(rng_t *r, int maxlen) {
    int l = 1;
    while (l < maxlen && (rng_next(r) >> 63)) l++;
    return l;
}

/* ---------------------------------------------------------------- genomes */

int64_t synth_genome_uniform(uint8_t *out, int64_t G, uint64_t seed) {
    rng_t r; rng_seed(&r, seed, 0);
    int64_t i = 0;
    while (i < G) {
        uint64_t x = rng_next(&r);
        for (int k = 0; k < 32 && i < G; k++, i++) { out[i] = BASES[x & 3]; x >>= 2; }
    }
    return G;
}

/*
 * Repeat genome. Blocks are appended until G bases exist; the block type is
 * the one furthest below its target share of bases so far (deterministic).
 *   unique:  length U{1000..10000}, i.i.d. bases
 *   segdup:  length U{1000..5000}, copy of earlier sequence (source start
 *            uniform), reverse-complemented with probability 1/2, diverged at
 *            rate U[div_lo, div_hi] per base (90% substitutions, 10% indels of
 *            length U{1..3}, insertion or deletion with equal odds)
 *   tandem:  unit U{2..50} random bases, array length U{100..2000}, each copied
 *            base mutated (substituted) with probability tandem_mut
 * Then runs of N of log-uniform length in [n_run_lo, n_run_hi] are written at
 * uniform positions until at least n_frac*G bases are N.
 */
int64_t synth_genome_repeats(uint8_t *out, int64_t G, uint64_t seed,
                             double f_unique, double f_segdup, double f_tandem,
                             double div_lo, double div_hi, double tandem_mut,
                             double n_frac, int64_t n_run_lo, int64_t n_run_hi) {
    rng_t r; rng_seed(&r, seed, 0);
    double target[3] = {f_unique, f_segdup, f_tandem};
    double have[3] = {0, 0, 0};
    int64_t cur = 0;
    uint8_t *tmp = (uint8_t *)malloc(16384);
    uint8_t unit[64];
    while (cur < G) {
        int type = 0; double best = -1e300;
        for (int k = 0; k < 3; k++) {
            double deficit = target[k] * (double)(cur + 1) - have[k];
            if (target[k] > 0 && deficit > best) { best = deficit; type = k; }
        }
        if (cur < 10000) type = 0; /* copies need earlier sequence */
        int64_t added = 0;
        if (type == 0) {
            int64_t len = rng_range(&r, 1000, 10000);
            for (int64_t k = 0; k < len && cur < G; k++) { out[cur++] = BASES[rng_below(&r, 4)]; added++; }
        } else if (type == 1) {
            int64_t len = rng_range(&r, 1000, 5000);
            if (len > cur) len = cur;
            int64_t src = (int64_t)rng_below(&r, (uint64_t)(cur - len + 1));
            int rc = (int)rng_below(&r, 2);
            for (int64_t k = 0; k < len; k++) tmp[k] = rc ? comp_base(out[src + len - 1 - k]) : out[src + k];
            double div = div_lo + (div_hi - div_lo) * rng_unif(&r);
            for (int64_t k = 0; k < len && cur < G;) {
                if (rng_unif(&r) < div) {
                    if (rng_unif(&r) < 0.9) { out[cur++] = other_base(&r, tmp[k]); added++; k++; }
                    else {
                        int l = (int)rng_range(&r, 1, 3);
                        if (rng_below(&r, 2)) { for (int j = 0; j < l && cur < G; j++) { out[cur++] = BASES[rng_below(&r, 4)]; added++; } }
                        else k += l;
                    }
                } else { out[cur++] = tmp[k]; added++; k++; }
            }
        } else {
            int ulen = (int)rng_range(&r, 2, 50);
            for (int k = 0; k < ulen; k++) unit[k] = BASES[rng_below(&r, 4)];
            int64_t len = rng_range(&r, 100, 2000);
            for (int64_t k = 0; k < len && cur < G; k++) {
                uint8_t b = unit[k % ulen];
                if (rng_unif(&r) < tandem_mut) b = other_base(&r, b);
                out[cur++] = b; added++;
            }
        }
        have[type] += (double)added;
    }
    free(tmp);
    if (n_frac > 0 && n_run_hi >= n_run_lo && n_run_lo > 0) {
        int64_t want = (int64_t)ceil(n_frac * (double)G), got = 0;
        double llo = log((double)n_run_lo), lhi = log((double)n_run_hi);
        int guard = 0;
        while (got < want && guard++ < 100000000) {
            int64_t len = (int64_t)exp(llo + (lhi - llo) * rng_unif(&r));
            if (len > G) len = G;
            int64_t at = (int64_t)rng_below(&r, (uint64_t)(G - len + 1));
            for (int64_t k = at; k < at + len; k++) { if (out[k] != 'N') { out[k] = 'N'; got++; } }
        }
    }
    return G;
}

/* ------------------------------------------------------------------ reads */

/*
 * Read lengths.
 *   mode 0: every read has length a
 *   mode 1: length a or b with equal odds
 *   mode 2: floor(a * (b/a)^u), u ~ U[0,1) (log-uniform on [a, b))
 */
void synth_read_lengths(int64_t n, uint64_t seed, int mode, int32_t a, int32_t b, int32_t *lengths) {
    #pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < n; i++) {
        rng_t r; rng_seed(&r, seed ^ 0x5EEDull, (uint64_t)i);
        int32_t L = a;
        if (mode == 1) L = rng_below(&r, 2) ? b : a;
        else if (mode == 2) {
            double u = rng_unif(&r);
            L = (int32_t)floor((double)a * pow((double)b / (double)a, u));
            if (L < a) L = a;
            if (L >= b) L = b - 1;
        }
        lengths[i] = L;
    }
}

/*
 * Error model for one read. Per source base: with probability p_indel an indel
 * event (insertion or deletion with equal odds, length truncated geometric(1/2)
 * on 1..indel_max; inserted bases uniform), else with probability p_sub a
 * substitution (uniform among the three other bases), else a copy. Reads of
 * length <= long_thr use the first set, longer reads the second.
 */
typedef struct {
    double p_sub, p_indel; int32_t indel_max;
    double p_sub_long, p_indel_long; int32_t indel_max_long;
    int32_t long_thr;
} synth_err;

static int make_read(const uint8_t *g, int64_t G, int32_t L, rng_t *r, const synth_err *e,
                     uint8_t *out, int64_t *tpos, int8_t *tstrand, int32_t *tedits) {
    double ps = e->p_sub, pi = e->p_indel; int imax = e->indel_max;
    if (L > e->long_thr) { ps = e->p_sub_long; pi = e->p_indel_long; imax = e->indel_max_long; }
    int64_t W = (int64_t)L + (int64_t)L / 2 + 64;
    if (W > G) W = G;
    for (int attempt = 0; attempt < 1000; attempt++) {
        int64_t a = (int64_t)rng_below(r, (uint64_t)(G - W + 1));
        int strand = (int)rng_below(r, 2);
        int32_t olen = 0, edits = 0; int64_t k = 0; int bad = 0;
        while (olen < L) {
            if (k >= W) { bad = 1; break; }
            double u = rng_unif(r);
            if (u < pi) {
                int l = trunc_geom(r, imax);
                if (rng_below(r, 2)) {
                    for (int j = 0; j < l && olen < L; j++) out[olen++] = BASES[rng_below(r, 4)];
                    edits += l;
                } else { k += l; edits += l; }
                continue;
            }
            uint8_t b = strand ? comp_base(g[a + W - 1 - k]) : g[a + k];
            if (b == 'N') { bad = 1; break; }
            k++;
            if (u < pi + ps) { b = other_base(r, b); edits++; }
            out[olen++] = b;
        }
        if (bad) continue;
        /* reject windows whose consumed span holds an N (deleted bases included) */
        int64_t lo = strand ? a + W - k : a, hi = strand ? a + W : a + k;
        for (int64_t q = lo; q < hi && !bad; q++) if (g[q] != 'A' && g[q] != 'C' && g[q] != 'G' && g[q] != 'T') bad = 1;
        if (bad) continue;
        *tpos = lo; *tstrand = (int8_t)strand; *tedits = edits;
        return 0;
    }
    /* genome too small or too N-rich: emit an all-N read flagged by strand -1 */
    memset(out, 'N', (size_t)L);
    *tpos = -1; *tstrand = -1; *tedits = -1;
    return -1;
}

/*
 * Fill reads. offsets[i] is the byte offset of read i in `bases` (caller
 * computes the exclusive sum of lengths). Returns the number of reads that
 * could not be placed (0 on any reasonable genome).
 */
int64_t synth_reads_fill(const uint8_t *genome, int64_t G, int64_t n, uint64_t seed,
                         const int32_t *lengths, const int64_t *offsets, const synth_err *e,
                         uint8_t *bases, int64_t *tpos, int8_t *tstrand, int32_t *tedits) {
    int64_t failed = 0;
    #pragma omp parallel for schedule(dynamic, 1024) reduction(+ : failed)
    for (int64_t i = 0; i < n; i++) {
        rng_t r; rng_seed(&r, seed, (uint64_t)i);
        if (lengths[i] <= 0) { tpos[i] = -1; tstrand[i] = -1; tedits[i] = 0; continue; }
        if (make_read(genome, G, lengths[i], &r, e, bases + offsets[i], tpos + i, tstrand + i, tedits + i)) failed++;
    }
    return failed;
}

/* Poisson arrivals: exponential inter-arrival gaps of mean 1/rate (seconds), and
 * request sizes floor(10^(dec*u)) for u ~ U[0,1) (at least 1). */
void synth_arrivals(int64_t n, uint64_t seed, double rate, double dec, double *t_arrive, int32_t *n_reads) {
    rng_t r; rng_seed(&r, seed, 0xA11ull);
    double t = 0;
    for (int64_t i = 0; i < n; i++) {
        double u = rng_unif(&r);
        t += -log(1.0 - u) / rate;
        t_arrive[i] = t;
        int32_t k = (int32_t)floor(pow(10.0, dec * rng_unif(&r)));
        n_reads[i] = k < 1 ? 1 : k;
    }
}
