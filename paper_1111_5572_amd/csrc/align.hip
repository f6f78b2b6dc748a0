// Alignment path of Algorithm 1 (Section 3.2) on gfx950, as a pipeline of kernels
// per pass over a chunk of reads:
//
//   pack       ASCII reads -> 2-bit stream + 1-bit N mask (once per batch)
//   probe      every seed slot of every read: seed code, reverse complement,
//              canonical code, one 128-byte bucket read by 8 cooperating lanes,
//              h_max test; writes the forward / reverse hit lists of the seed
//   hitcount   per read: hits of the seeds that pass the h_max test
//   candidates per read: hits -> locations (strand, p), deduplicated into a
//              sorted list with one bit per seed that voted for it
//   compact    per read: sorted lists packed back to back
//   verify     per location: bounded edit distance with limit K = d_max + c - 1
//              (Landau-Vishkin furthest-reaching diagonals, one lane per
//              location, read and window staged in LDS)
//   replay     per read: Algorithm 1's control flow over the seed masks and the
//              capped distances, with the exact d_limit of every step
//
// Why verifying every location once with limit K and replaying gives the same
// result as the sequential algorithm: every d_limit Algorithm 1 can use is at most
// K (d_max + c - 1 when d_best > d_max; d_best + c - 1 <= K when d_best <= d_max;
// d_best - 1 < K otherwise), so EditDistance(p, limit) equals min(D, K+1) when
// that is at most the limit and the special value otherwise. The seed masks give
// the vote count of a location after seeds 1..i as popcount(mask & prefix_i).
#include <hip/hip_runtime.h>
#include <hipcub/hipcub.hpp>

#include <algorithm>
#include <atomic>
#include <cstring>
#include <memory>
#include <mutex>
#include <string>
#include <thread>
#include <vector>

#include "../../include/snapgpu.h"
#include "../../include/snapgpu_debug.h"
#include "snap_internal.h"

using namespace snapgpu;

namespace {

constexpr int ST_NONE = 0;   // slot beyond the read's seeds
constexpr int ST_N = 1;      // seed holds an N: not looked up
constexpr int ST_OVER = 2;   // more than h_max index entries: skipped
constexpr int ST_OK = 3;     // looked up (possibly with no hits)
static_assert(ST_OK < 4 && MAX_SEEDS <= 32, "a read's seed statuses pack into 64 bits, 2 each");
constexpr int DINF = 0x3FFF;
constexpr int STREAM_GUARD = 32;   // bases of padding before the packed read stream
constexpr int64_t CHUNK_READS = 1 << 20;
constexpr int VERIFY_KMAX = 1023;   // largest limit d_max(L) + c - 1
constexpr int VERIFY_LMAX = 16384;  // longest read
constexpr int LANE_KMAX = 63;       // lane-per-location verify: limit and read length bounds
constexpr int LANE_LMAX = 512;
constexpr int REQUEST_TOP_DEFAULT = 4;   // locations a single-location request takes (snap_tuning.request_top)
constexpr int REQUEST_TOP_MAX = 16;
// Verification requests live in one int16 per location: the limit, tagged for the
// wave tile when the read is verified a wave per location; -1 = none.
constexpr int REQ_WAVE = 0x4000;
constexpr int REQ_LIMIT_MASK = 0x3FFF;
constexpr uint32_t REQ_WAVE_READ = 0x80000000u;
// Replay of reads with more than 64 locations: a wave stages up to HEAVY_LDS_LOCS of
// them in LDS (seed mask, capped distance | verified limit << 16, scored bit, and
// for the phase that scores every remaining location the vote count); a read with
// more works in global memory. 512 keeps the LDS of a 4-wave workgroup at 18.7 KB
// (1024: 37.4 KB); the kernel's registers hold it at 12 waves a CU either way (measured
// 104.2 against 102.9 M reads/s at human scale with 512).
constexpr int HEAVY_LDS_LOCS = 512;
__host__ __device__ constexpr int heavy_lds_words(int cap) { return 2 * cap + cap / 32 + cap / 4; }
// Outcome of a read's replay in a pass.
constexpr uint8_t RF_DONE = 0;      // outputs written
constexpr uint8_t RF_PENDING = 1;   // needs a seed this pass did not probe
constexpr uint8_t RF_REPLAY = 2;    // asked for verification; replay again

struct ProbeRec {
    uint64_t off_f;   // first forward hit (positions index)
    uint64_t off_r;   // first reverse hit
    uint32_t nf;      // forward hits of the seed
    uint32_t nr;      // reverse hits of the seed
    uint16_t o;       // seed offset in the read
    uint8_t status;
    uint8_t pad[5];
};
static_assert(sizeof(ProbeRec) == 32, "probe record is two 16-byte words");

struct Shifts {
    int32_t n;
    int8_t v[32];
};

struct Rule {
    int32_t s, n_min, n_cap, bp_per_seed, c, hmax, dmax, dmax_pct, bucket;
};

__host__ __device__ inline int seeds_for_length(const Rule &r, int L) {
    int want = (L + r.bp_per_seed - 1) / r.bp_per_seed;
    return want < r.n_min ? r.n_min : (want > r.n_cap ? r.n_cap : want);
}

__host__ __device__ inline int dmax_for_length(const Rule &r, int L) {
    int pct = (int)(((int64_t)r.dmax_pct * L + 99) / 100);
    return pct > r.dmax ? pct : r.dmax;
}

// Offset of seed i (0-based) of a read of length L under the shift order, or -1.
__host__ __device__ inline int seed_offset(const Shifts &sh, int s, int L, int i) {
    for (int k = 0; k < sh.n; k++) {
        int phi = sh.v[k];
        int cnt = (phi + s <= L) ? (L - s - phi) / s + 1 : 0;
        if (i < cnt) return phi + i * s;
        i -= cnt;
    }
    return -1;
}

// Shift order of the seed schedule (Section 3.2, omitted aspect 3): 0, s/2, then
// s/4 and 3s/4, then odd multiples of s/8 ..., floored, repeats dropped.
Shifts make_shifts(int s) {
    Shifts sh{};
    bool used[32] = {false};
    sh.v[sh.n++] = 0;
    used[0] = true;
    for (int level = 1; sh.n < s && level < 31; level++) {
        int64_t den = 1ll << level;
        for (int64_t j = 1; j < den && sh.n < s; j += 2) {
            int v = (int)((int64_t)s * j / den);
            if (!used[v]) { used[v] = true; sh.v[sh.n++] = (int8_t)v; }
        }
    }
    return sh;
}

// ------------------------------------------------------------ bit helpers

__device__ inline uint32_t funnel(uint32_t hi, uint32_t lo, uint32_t sh) {
    return __builtin_amdgcn_alignbit(hi, lo, sh);   // (hi:lo) >> sh, sh in [0, 31]
}

// 16 bases from a 2-bit array starting at base x
__device__ inline uint32_t ext_code16(const uint32_t *a, int64_t x) {
    int64_t w = x >> 4;
    return funnel(a[w + 1], a[w], (uint32_t)(x & 15) * 2);
}

// 16 N flags from a 1-bit array starting at base x
__device__ inline uint32_t ext_mask16(const uint32_t *a, int64_t x) {
    int64_t w = x >> 5;
    return funnel(a[w + 1], a[w], (uint32_t)(x & 31)) & 0xFFFFu;
}

// Whether any of the n >= 1 bits [x, x + n) of a 1-bit array is set (nonzero if so).
__device__ inline uint32_t any_n(const uint32_t *a, int64_t x, int n) {
    const int64_t m0 = x >> 5, m1 = (x + n - 1) >> 5;
    uint32_t acc = 0;
    for (int64_t m = m0; m <= m1; m++) {
        uint32_t v = a[m];
        if (m == m0) v &= 0xFFFFFFFFu << (x & 31);
        if (m == m1) v &= 0xFFFFFFFFu >> (31 - ((x + n - 1) & 31));
        acc |= v;
    }
    return acc;
}

// bit k of a 16-bit mask -> bit 2k
__device__ inline uint32_t spread16(uint32_t m) {
    m = (m | (m << 8)) & 0x00FF00FFu;
    m = (m | (m << 4)) & 0x0F0F0F0Fu;
    m = (m | (m << 2)) & 0x33333333u;
    m = (m | (m << 1)) & 0x55555555u;
    return m;
}

// reverse complement of 16 bases in a word
__device__ inline uint32_t rc16(uint32_t w) {
    uint32_t r = __builtin_bitreverse32(w);
    r = ((r >> 1) & 0x55555555u) | ((r & 0x55555555u) << 1);
    return ~r;
}

__device__ inline int base_code(uint8_t b) {
    switch (b) {
        case 'A': case 'a': return 0;
        case 'C': case 'c': return 1;
        case 'G': case 'g': return 2;
        case 'T': case 't': return 3;
        default: return 4;
    }
}

// ------------------------------------------------------------------ pack

// Stream base x (x = STREAM_GUARD + global base index). Block t of 32 bases owns
// code words 2t, 2t+1 and mask word t. Bases outside the reads are N.
// A, C, G, T in either case to 0..3 and every other byte to N, four bytes of a 32-bit
// word at once: bits 1-2 of an ASCII letter xor-folded give the code (A 0, C 1, G 2,
// T 3, either case), and a byte is a base when it equals a, c, g or t once bit 5 is set
// (an exact zero-byte test on the difference). p: the four 2-bit codes (N as 0),
// nb: the four N flags.
__device__ inline void decode4(uint32_t w, uint32_t &p, uint32_t &nb) {
    auto zero_bytes = [](uint32_t v) { return ~(((v & 0x7F7F7F7Fu) + 0x7F7F7F7Fu) | v) & 0x80808080u; };
    const uint32_t x = w | 0x20202020u;
    const uint32_t valid = zero_bytes(x ^ 0x61616161u) | zero_bytes(x ^ 0x63636363u) |
                           zero_bytes(x ^ 0x67676767u) | zero_bytes(x ^ 0x74747474u);
    const uint32_t c = ((x >> 1) ^ (x >> 2)) & 0x03030303u & ((valid >> 7) * 3u);
    const uint32_t n = ~valid & 0x80808080u;
    p = (c & 3u) | ((c >> 6) & 0xCu) | ((c >> 12) & 0x30u) | ((c >> 18) & 0xC0u);
    nb = ((n >> 7) & 1u) | ((n >> 14) & 2u) | ((n >> 21) & 4u) | ((n >> 28) & 8u);
}

// One thread per 32-base block of the packed stream (block t holds batch bytes
// [32 (t - 1), 32 t); block 0 is the guard). A block wholly inside the batch reads its
// 32 bytes as two 16-byte loads (vec: the batch is 16-byte aligned) and decodes a word
// at a time; the guard and a partial last block go byte by byte.
__global__ void k_pack(const uint8_t *reads, int64_t B, uint32_t *rcode, uint32_t *rmask, int64_t nblk, int vec) {
    int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= nblk) return;
    const int64_t g0 = t * 32 - STREAM_GUARD;
    uint32_t c0 = 0, c1 = 0, m = 0;
    if (vec && g0 >= 0 && g0 + 32 <= B) {
        const uint4 a = *reinterpret_cast<const uint4 *>(reads + g0);
        const uint4 b = *reinterpret_cast<const uint4 *>(reads + g0 + 16);
        const uint32_t w[8] = {a.x, a.y, a.z, a.w, b.x, b.y, b.z, b.w};
#pragma unroll
        for (int q = 0; q < 8; q++) {
            uint32_t p, nb;
            decode4(w[q], p, nb);
            if (q < 4) c0 |= p << (8 * q); else c1 |= p << (8 * (q - 4));
            m |= nb << (4 * q);
        }
    } else {
        for (int k = 0; k < 32; k++) {
            const int64_t g = g0 + k;
            int c = (g >= 0 && g < B) ? base_code(reads[g]) : 4;
            if (c > 3) { m |= 1u << k; c = 0; }
            if (k < 16) c0 |= (uint32_t)c << (2 * k); else c1 |= (uint32_t)c << (2 * (k - 16));
        }
    }
    rcode[2 * t] = c0;
    rcode[2 * t + 1] = c1;
    rmask[t] = m;
}

__global__ void k_maxlen(const int32_t *len, int64_t n, uint32_t *out) {
    __shared__ uint32_t red[256];
    uint32_t m = 0;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        int v = len[i];
        uint32_t u = v < 0 ? 0x80000000u : (uint32_t)v;   // negative lengths flagged
        m = m > u ? m : u;
    }
    red[threadIdx.x] = m;
    __syncthreads();
    for (int s = 128; s > 0; s >>= 1) {
        if ((int)threadIdx.x < s) red[threadIdx.x] = max(red[threadIdx.x], red[threadIdx.x + s]);
        __syncthreads();
    }
    if (threadIdx.x == 0) atomicMax(out, red[0]);
}

__global__ void k_fill_u32(uint32_t *p, int64_t n, uint32_t v) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = v;
}

// ----------------------------------------------------------------- probe

// A pass works on a list of reads: entry r0 + r of `ridx` (or read r0 + r when
// there is no list) for r in [0, nr).
struct Pass {
    const uint32_t *ridx;
    int64_t r0, nr;
    int32_t NS;        // seed slots probed in this pass
    int32_t Kcap;      // verify limit cap: distances above min(Kcap, K(L)) stay unknown
    int32_t final_pass;
    int32_t ST;        // seeds per slot: the index's stride (one probe record each)
};

__device__ inline int64_t gid(const Pass &p, int64_t r) {
    return p.ridx ? (int64_t)p.ridx[p.r0 + r] : p.r0 + r;
}


struct ProbeArgs {
    DevIndex ix;
    const uint32_t *rcode, *rmask;
    const int64_t *roff;   // read offsets (bases) in the packed stream
    const int32_t *len;
    Pass ps;
    Rule rule;
    Shifts sh;
    ProbeRec *out;         // nr * NS * ST records
    uint32_t *hits;        // per read: hits of its looked-up seeds (zeroed before the launch)
};

// A wave takes 64 (read, seed slot, seed of the slot) items; a slot has one seed, or
// with a strided index ST seeds at consecutive offsets (consecutive lanes). First each
// lane computes one item's seed (offset, 2s-bit code, N test, canonical code); then in 8
// rounds every group of eight lanes probes one item, each lane reading one 16-byte slot
// of the seed's 128-byte bucket (one coalesced cache line per probe step); results come
// back to the item's lane through LDS. The lanes of a slot then combine their N tests and
// entry counts (the slot is skipped for an N in any of its seeds, over h_max on the sum),
// and each lane writes its own record. A read's hits (the counts of its looked-up seeds
// within h_max) are summed over its lanes by a segmented scan; a read split between two
// waves adds its two parts atomically.
__global__ __launch_bounds__(256) void k_probe(ProbeArgs a) {
    __shared__ uint64_t res_val[4][64];
    __shared__ uint8_t res_found[4][64];
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const int sub = lane & 7, grp = lane >> 3;
    const int s = a.ix.s;
    const int NS = a.ps.NS, ST = a.ps.ST;
    const int NI = NS * ST;                       // items per read (at most 64)
    const int64_t nitems = a.ps.nr * (int64_t)NI;
    const int64_t item = (((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6) * 64 + lane;
    const bool valid = item < nitems;
    // item = r * NI + k (32-bit division when the pass's items fit 32 bits, as they do
    // for any chunk of up to 2^26 reads); slot i = k / ST, seed j = k % ST of the slot
    int64_t r = 0;
    int k = 0;
    if (valid) {
        if (nitems <= 0xFFFFFFFFll) {
            const uint32_t r32 = (uint32_t)item / (uint32_t)NI;
            r = r32;
            k = (int)((uint32_t)item - r32 * (uint32_t)NI);
        } else {
            r = item / NI;
            k = (int)(item - r * NI);
        }
    }
    const int i = k / ST, j = k - i * ST;
    const int64_t g = valid ? gid(a.ps, r) : 0;
    const int L = valid ? a.len[g] : 0;
    int o = -1;
    if (valid && i < seeds_for_length(a.rule, L)) {
        const int os = seed_offset(a.sh, s, L, i);
        if (os >= 0 && os + j + s <= L) o = os + j;   // the slot's seed j, if it fits the read
    }
    int status = ST_NONE;
    uint64_t key = 0, canon = 0;
    if (o >= 0) {
        const int64_t x = STREAM_GUARD + a.roff[g] + o;
        const int64_t w = x >> 4;
        const uint32_t sh = (uint32_t)(x & 15) * 2;
        uint64_t lo = (uint64_t)a.rcode[w] | ((uint64_t)a.rcode[w + 1] << 32);
        uint64_t hi = a.rcode[w + 2];
        key = (lo >> sh) | (sh ? (hi << (64 - sh)) : 0);
        key &= seed_mask(s);
        const int64_t mw = x >> 5;
        uint64_t m64 = (uint64_t)a.rmask[mw] | ((uint64_t)a.rmask[mw + 1] << 32);
        uint64_t nbits = (m64 >> (x & 31)) & (s >= 32 ? 0xFFFFFFFFull : ((1ull << s) - 1));
        if (nbits) status = ST_N;
        else {
            status = ST_OK;
            uint64_t rc = rc_code(key, s);
            canon = key < rc ? key : rc;
        }
    }
    const int g0 = lane & ~7;
    for (int j = 0; j < 8; j++) {
        // group grp probes the item of lane src
        const int src = j * 8 + grp;
        const bool ok = __shfl(status, src, 64) == ST_OK;
        const uint32_t clo = (uint32_t)__shfl((int)(uint32_t)canon, src, 64);
        const uint32_t chi = (uint32_t)__shfl((int)(uint32_t)(canon >> 32), src, 64);
        const uint64_t ckey = ((uint64_t)chi << 32) | clo;
        bool pending = ok;
        uint64_t b = pending ? home_bucket(ckey, a.ix.log2_buckets) : 0;
        uint64_t steps = 0;
        bool found = false;
        uint64_t val = 0;
        // every group runs until its probe ends; the loop is uniform over the wave.
        // The table is at most 70% full, so an empty slot ends every probe; the step
        // bound only guarantees termination on a corrupted table.
        for (;;) {
            uint64_t k0 = EMPTY_KEY, v0 = 0;
            if (pending) {
                const uint64_t slot = b * SLOTS_PER_BUCKET + sub;
                const ulonglong2 e = *reinterpret_cast<const ulonglong2 *>(a.ix.table + 2 * slot);
                k0 = e.x;
                v0 = e.y;
            }
            const uint64_t hit = __ballot(pending && k0 == ckey);
            const uint64_t emp = __ballot(pending && k0 == EMPTY_KEY);
            const uint32_t ghit = (uint32_t)(hit >> g0) & 0xFFu, gemp = (uint32_t)(emp >> g0) & 0xFFu;
            if (pending) {
                if (ghit) {
                    if (sub == __builtin_ctz(ghit)) { found = true; val = v0; }
                    pending = false;
                } else if (gemp) {
                    pending = false;
                } else {
                    b = (b + 1) & (a.ix.nbuckets - 1);
                    if (++steps >= a.ix.nbuckets) pending = false;
                }
            }
            if (__ballot(pending) == 0) break;
        }
        // the lane that found the key reports it; sub 0 clears the flag first
        if (sub == 0) res_found[wv][src] = 0;
        __builtin_amdgcn_wave_barrier();
        if (found) {
            res_val[wv][src] = val;
            res_found[wv][src] = 1;
        }
    }
    __builtin_amdgcn_wave_barrier();
    const bool found = valid && res_found[wv][lane] != 0;
    const uint64_t val = res_val[wv][lane];
    const uint32_t nf = found ? (uint32_t)((val >> 36) & CNT_SAT) : 0u;
    const uint32_t nrv = found ? (uint32_t)((val >> 50) & CNT_SAT) : 0u;
    // the slot's entries (occ(S) + occ(RC S), summed over its seeds) and N test; a slot's
    // ST lanes are an aligned group of the wave (64 is a multiple of ST)
    uint32_t entries = status == ST_OK ? nf + nrv : 0u;
    int any_n = status == ST_N ? 1 : 0;
    for (int m = 1; m < ST; m <<= 1) {
        entries += (uint32_t)__shfl_xor((int)entries, m, 64);
        any_n |= __shfl_xor(any_n, m, 64);
    }
    if (status != ST_NONE) status = any_n ? ST_N : ((int64_t)entries > a.rule.hmax ? ST_OVER : ST_OK);
    ProbeRec rec{};
    rec.status = (uint8_t)status;
    rec.o = (uint16_t)(o < 0 ? 0 : o);
    if (status == ST_OK && found) {
        const uint64_t off = val & OFF_MASK;
        if (key == canon) {
            rec.off_f = off; rec.nf = nf; rec.off_r = off + nf; rec.nr = nrv;
        } else {   // the seed is the reverse complement of the stored key
            rec.off_f = off + nf; rec.nf = nrv; rec.off_r = off; rec.nr = nf;
        }
    }
    if (valid) a.out[item] = rec;
    // per-read hit sums
    const uint32_t rkey = valid ? (uint32_t)r : 0xFFFFFFFFu;
    uint32_t cnt = (valid && rec.status == ST_OK) ? rec.nf + rec.nr : 0u, len = valid ? 1u : 0u;
    for (int d = 1; d < 64; d <<= 1) {
        const uint32_t c2 = (uint32_t)__shfl_up((int)cnt, d, 64), l2 = (uint32_t)__shfl_up((int)len, d, 64);
        const uint32_t k2 = (uint32_t)__shfl_up((int)rkey, d, 64);
        if (lane >= d && k2 == rkey) { cnt += c2; len += l2; }
    }
    const uint32_t knext = (uint32_t)__shfl_down((int)rkey, 1, 64);
    if (valid && (lane == 63 || knext != rkey)) {
        if (len == (uint32_t)NI) a.hits[r] = cnt;
        else atomicAdd(&a.hits[r], cnt);
    }
}

// ------------------------------------------------------------ candidates


constexpr uint64_t HIT_NONE = ~0ull;

struct GatherArgs {
    const ProbeRec *pr;
    const uint32_t *positions;
    uint64_t G;
    int32_t s;
    const int32_t *len;
    Pass ps;
    const int64_t *hoff;
    uint64_t *hk;      // per hit: ((p << 1 | strand) << 5) | seed slot, or HIT_NONE
};

// Algorithm 1's vote loop. A wave takes 64 / NI whole reads at a time (NI = NS * ST probe
// records a read), lane k holding record k of them (the reads' hit regions are then one
// contiguous range of the hit array); a hit carries its seed slot, k / ST, so that the
// seeds of one slot of a strided index vote once for a location between them. A wave prefix sum of the slots' hit counts places every slot's hits, slot
// by slot and forward before reverse within a slot; then the lanes take 64 hits of the
// range at a time (coalesced position reads and hit writes), each finding its slot by
// a binary search over the slots' starts in LDS. A forward hit q of the seed at offset
// o votes for (+, q - o), a reverse hit for (-, q - (L - o - s)); locations outside
// [0, G - L] are dropped.
__global__ __launch_bounds__(256) void k_gather(GatherArgs a) {
    __shared__ uint32_t s_start[4][64];
    __shared__ uint32_t s_nf[4][64];
    __shared__ uint64_t s_offf[4][64], s_offr[4][64];
    __shared__ int32_t s_ofs[4][64], s_len[4][64];
    const int NI = a.ps.NS * a.ps.ST, ST = a.ps.ST;
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const int64_t wave = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6;
    const int64_t nwaves = ((int64_t)gridDim.x * blockDim.x) >> 6;
    const int rpw = 64 / NI;                       // reads per wave step
    const int nitems = rpw * NI;
    for (int64_t r0 = wave * rpw; r0 < a.ps.nr; r0 += nwaves * rpw) {
        const int nrd = (int)min((int64_t)rpw, a.ps.nr - r0);
        const int rl = lane / NI, i = lane - rl * NI;
        const bool mine = lane < nrd * NI;
        const int64_t r = r0 + rl;
        uint32_t cnt = 0, nf = 0;
        uint64_t offf = 0, offr = 0;
        int o = 0, L = 0;
        if (mine) {
            const ProbeRec p = a.pr[r * NI + i];
            L = a.len[gid(a.ps, r)];
            if (p.status == ST_OK) {
                cnt = p.nf + p.nr;
                nf = p.nf;
                o = p.o;
                offf = p.off_f;
                offr = p.off_r;
            }
        }
        uint32_t incl = cnt;
        for (int d = 1; d < 64; d <<= 1) {
            const uint32_t v = (uint32_t)__shfl_up((int)incl, d, 64);
            if (lane >= d) incl += v;
        }
        const uint32_t H = (uint32_t)__shfl((int)incl, 63, 64);
        if (lane < nitems) {
            s_start[wv][lane] = incl - cnt;
            s_nf[wv][lane] = nf;
            s_offf[wv][lane] = offf;
            s_offr[wv][lane] = offr;
            s_ofs[wv][lane] = o;
            s_len[wv][lane] = L;
        }
        const int64_t base = a.hoff[r0];
        __builtin_amdgcn_wave_barrier();
        for (uint32_t h0 = 0; h0 < H; h0 += 64) {
            const uint32_t h = h0 + lane;
            if (h < H) {
                // the last slot whose start is at most h (it holds h: the next start is above it)
                int lo = 0, hi = nitems - 1;
                while (lo < hi) {
                    const int mid = (lo + hi + 1) >> 1;
                    if (s_start[wv][mid] <= h) lo = mid; else hi = mid - 1;
                }
                const uint32_t k = h - s_start[wv][lo];
                const uint32_t snf = s_nf[wv][lo];
                const int64_t so = s_ofs[wv][lo], sl = s_len[wv][lo];
                const uint64_t slot = (uint64_t)((lo % NI) / ST);
                uint64_t hv;
                if (k < snf) {
                    const int64_t pp = (int64_t)a.positions[s_offf[wv][lo] + k] - so;
                    hv = (pp >= 0 && pp + sl <= (int64_t)a.G) ? (((uint64_t)pp << 1) << 5) | slot : HIT_NONE;
                } else {
                    const int64_t pp = (int64_t)a.positions[s_offr[wv][lo] + (k - snf)] - (sl - so - a.s);
                    hv = (pp >= 0 && pp + sl <= (int64_t)a.G) ? ((((uint64_t)pp << 1) | 1) << 5) | slot : HIT_NONE;
                }
                a.hk[base + h] = hv;
            }
        }
        __builtin_amdgcn_wave_barrier();
    }
}

struct DedupeArgs {
    const uint64_t *hk;
    const uint32_t *hits;
    const int64_t *hoff;
    int64_t nr;
    uint64_t *key;     // distinct locations (p << 1 | strand), ascending, at hoff[r]
    uint32_t *mask;    // the seed slots that voted for each
    uint32_t *count;
    const uint32_t *rlist;     // the reads of this tier (null: every read of the chunk)
    const int64_t *rlist_n;
};

__device__ inline uint64_t shfl_xor64(uint64_t v, int m) {
    const uint32_t lo = __shfl_xor((unsigned)(uint32_t)v, m, 64);
    const uint32_t hi = __shfl_xor((unsigned)(uint32_t)(v >> 32), m, 64);
    return ((uint64_t)hi << 32) | lo;
}
__device__ inline uint64_t shfl_up64(uint64_t v, int d) {
    const uint32_t lo = __shfl_up((unsigned)(uint32_t)v, d, 64);
    const uint32_t hi = __shfl_up((unsigned)(uint32_t)(v >> 32), d, 64);
    return ((uint64_t)hi << 32) | lo;
}
__device__ inline uint64_t shfl_down64(uint64_t v, int d) {
    const uint32_t lo = __shfl_down((unsigned)(uint32_t)v, d, 64);
    const uint32_t hi = __shfl_down((unsigned)(uint32_t)(v >> 32), d, 64);
    return ((uint64_t)hi << 32) | lo;
}

// Reads with at most 64 hits: one wave per read, one hit per lane, a 64-lane
// bitonic sort in registers, then equal locations merged (their seed bits OR-ed)
// and written in ascending order.
__global__ __launch_bounds__(256) void k_dedupe_light(DedupeArgs a) {
    const int lane = threadIdx.x & 63;
    const int64_t wave = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6;
    const int64_t nwaves = ((int64_t)gridDim.x * blockDim.x) >> 6;
    const int64_t n = a.rlist ? *a.rlist_n : a.nr;
    for (int64_t ri = wave; ri < n; ri += nwaves) {
        const int64_t r = a.rlist ? (int64_t)a.rlist[ri] : ri;
        if (r >= a.nr) continue;
        const uint32_t H = a.hits[r];
        if (H > 64) continue;
        const int64_t base = a.hoff[r];
        if (H == 0) {
            if (lane == 0) a.count[r] = 0;
            continue;
        }
        uint64_t v = (uint32_t)lane < H ? a.hk[base + lane] : HIT_NONE;
        for (int k = 2; k <= 64; k <<= 1)
            for (int j = k >> 1; j > 0; j >>= 1) {
                const uint64_t o = shfl_xor64(v, j);
                const bool up = (lane & k) == 0;
                const bool lower = (lane & j) == 0;
                const uint64_t mn = v < o ? v : o, mx = v < o ? o : v;
                v = (lower == up) ? mn : mx;
            }
        const bool valid = v != HIT_NONE;
        const uint64_t loc = v >> 5;
        const uint64_t prev = shfl_up64(loc, 1);
        const bool first = valid && (lane == 0 || prev != loc);
        uint32_t acc = valid ? (1u << (v & 31)) : 0u;
        // a location's run spans up to 32 lanes (one hit per seed slot), 64 with the two
        // seeds a slot of a stride-2 index has
        for (int d = 1; d < 64; d <<= 1) {
            const uint32_t nb = __shfl_down(acc, d, 64);
            const uint64_t nloc = shfl_down64(loc, d);
            if (lane + d < 64 && nloc == loc) acc |= nb;
        }
        const uint64_t fb = __ballot(first);
        const int rank = __popcll(fb & ((1ull << lane) - 1));
        if (first) {
            a.key[base + rank] = loc;
            a.mask[base + rank] = acc;
        }
        if (lane == 0) a.count[r] = (uint32_t)__popcll(fb);
    }
}

// Reads with at most 8 hits (most reads): one lane per read, a 19-comparator sorting
// network over registers, then the same merge of equal locations.
__global__ __launch_bounds__(256) void k_dedupe_tiny(DedupeArgs a) {
    constexpr int N = 8;
    for (int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; r < a.nr; r += (int64_t)gridDim.x * blockDim.x) {
        const uint32_t H = a.hits[r];
        if (H > (uint32_t)N) continue;
        const int64_t base = a.hoff[r];
        uint64_t v[N];
#pragma unroll
        for (int k = 0; k < N; k++) v[k] = (uint32_t)k < H ? a.hk[base + k] : HIT_NONE;
        constexpr int net[19][2] = {{0, 1}, {2, 3}, {4, 5}, {6, 7}, {0, 2}, {1, 3}, {4, 6}, {5, 7}, {1, 2}, {5, 6},
                                    {0, 4}, {1, 5}, {2, 6}, {3, 7}, {2, 4}, {3, 5}, {1, 2}, {3, 4}, {5, 6}};
#pragma unroll
        for (int q = 0; q < 19; q++) {
            const uint64_t x = v[net[q][0]], y = v[net[q][1]];
            v[net[q][0]] = x < y ? x : y;
            v[net[q][1]] = x < y ? y : x;
        }
        uint32_t n = 0, acc = 0;
        uint64_t cur = 0;
#pragma unroll
        for (int k = 0; k < N; k++) {
            if (v[k] == HIT_NONE) continue;
            const uint64_t loc = v[k] >> 5;
            if (n > 0 && loc == cur) {
                acc |= 1u << (v[k] & 31);
            } else {
                if (n > 0) { a.key[base + n - 1] = cur; a.mask[base + n - 1] = acc; }
                cur = loc;
                acc = 1u << (v[k] & 31);
                n++;
            }
        }
        if (n > 0) { a.key[base + n - 1] = cur; a.mask[base + n - 1] = acc; }
        a.count[r] = n;
    }
}

// Reads with more than 64 hits: one 256-thread workgroup per read, bitonic sort
// of the hits in LDS (ascending network with the padding beyond H left in
// place), then the same merge of equal locations, 256 hits at a time.
// Reads with more hits than fit in LDS sort in place in a global scratch region
// of their own (the same code with IN_LDS false).
// NT threads per read; the kernel takes reads with lo < H <= hi hits.
template <bool IN_LDS, int NT>
__global__ __launch_bounds__(NT) void k_dedupe_heavy(DedupeArgs a, uint64_t *gscratch, uint32_t lo_h, uint32_t hi_h) {
    extern __shared__ uint64_t lds_keys[];
    __shared__ uint32_t wcnt[NT / 64];
    const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
    const int64_t n = a.rlist ? *a.rlist_n : a.nr;
    for (int64_t ri = blockIdx.x; ri < n; ri += gridDim.x) {
        const int64_t r = a.rlist ? (int64_t)a.rlist[ri] : ri;
        if (r >= a.nr) continue;
        const uint32_t H = a.hits[r];
        if (H <= lo_h || H > hi_h) continue;
        const int64_t base = a.hoff[r];
        uint64_t *sk = IN_LDS ? lds_keys : gscratch + base;
        uint32_t N = 1;
        while (N < H) N <<= 1;
        for (uint32_t i = tid; i < H; i += NT) sk[i] = a.hk[base + i];
        __syncthreads();
        // k, half and j are powers of two: indices by shifts and masks
        for (uint32_t lk = 1; (1u << lk) <= N; lk++) {
            const uint32_t k = 1u << lk, lh = lk - 1, half = k >> 1;
            for (uint32_t i = tid; i < N / 2; i += NT) {
                const uint32_t blk = i >> lh, off = i & (half - 1);
                const uint32_t lo = (blk << lk) + off, hi = (blk << lk) + k - 1 - off;
                if (hi < H) {
                    const uint64_t x = sk[lo], y = sk[hi];
                    if (y < x) { sk[lo] = y; sk[hi] = x; }
                }
            }
            __syncthreads();
            for (int lj = (int)lk - 2; lj >= 0; lj--) {
                const uint32_t j = 1u << lj;
                for (uint32_t i = tid; i < N / 2; i += NT) {
                    const uint32_t lo = ((i >> lj) << (lj + 1)) + (i & (j - 1)), hi = lo + j;
                    if (hi < H) {
                        const uint64_t x = sk[lo], y = sk[hi];
                        if (y < x) { sk[lo] = y; sk[hi] = x; }
                    }
                }
                __syncthreads();
            }
        }
        uint32_t run = 0;
        for (uint32_t c0 = 0; c0 < H; c0 += NT) {
            const uint32_t i = c0 + tid;
            bool first = false;
            uint32_t acc = 0;
            uint64_t loc = 0;
            if (i < H && sk[i] != HIT_NONE) {
                loc = sk[i] >> 5;
                first = (i == 0) || ((sk[i - 1] >> 5) != loc);
                if (first)
                    for (uint32_t j = i; j < H && (sk[j] >> 5) == loc; j++) acc |= 1u << (sk[j] & 31);
            }
            const uint64_t fb = __ballot(first);
            if (lane == 0) wcnt[w] = (uint32_t)__popcll(fb);
            __syncthreads();
            uint32_t before = run, tot = 0;
            for (int q = 0; q < NT / 64; q++) {
                if (q < w) before += wcnt[q];
                tot += wcnt[q];
            }
            if (first) {
                const uint32_t rank = before + (uint32_t)__popcll(fb & ((1ull << lane) - 1));
                a.key[base + rank] = loc;
                a.mask[base + rank] = acc;
            }
            run += tot;
            __syncthreads();
        }
        if (tid == 0) a.count[r] = run;
        __syncthreads();
    }
}

// A wave takes 64 consecutive reads (lane l: read r0 + l's first hit slot and first
// location slot). Their kept locations fill one contiguous range of the compacted
// arrays; the lanes take 64 of them at a time, each finding its read by a binary
// search over the reads' first location slots in LDS, and copy location o of read r
// from slot hoff[r] + (o - coff[r]).
// With `lead` set, each read's lead location is recorded too: the location of Algorithm 1's
// first EditDistance call. That call comes after the first seed slot that has a hit, when
// each of that slot's locations has one vote, so it takes the smallest (p, strand) among
// them: the first location in key order whose lowest seed bit is the lowest of the read.
constexpr uint32_t LEAD_NONE = 0xFFFFFFFFu;
__global__ __launch_bounds__(256) void k_compact(const int64_t *hoff, const int64_t *coff, int64_t nr,
                                                 const uint64_t *key_in, const uint32_t *mask_in, uint64_t *key_out,
                                                 uint32_t *mask_out, uint32_t *cread, uint32_t *lead) {
    __shared__ int64_t s_src[4][64], s_dst[4][64];
    __shared__ unsigned long long s_lead[4][64];   // (lowest seed bit << 40) | location, minimum per read
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const int64_t wave = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6;
    const int64_t nwaves = ((int64_t)gridDim.x * blockDim.x) >> 6;
    for (int64_t r0 = wave * 64; r0 < nr; r0 += nwaves * 64) {
        const int nrd = (int)min((int64_t)64, nr - r0);
        const int64_t d1 = coff[r0 + nrd];
        if (lane < nrd) {
            s_src[wv][lane] = hoff[r0 + lane];
            s_dst[wv][lane] = coff[r0 + lane];
            s_lead[wv][lane] = ~0ull;
        }
        const int64_t d0 = coff[r0];
        __builtin_amdgcn_wave_barrier();
        for (int64_t o0 = d0; o0 < d1; o0 += 64) {
            const int64_t o = o0 + lane;
            if (o < d1) {
                // the last read whose first location slot is at most o holds o
                int lo = 0, hi = nrd - 1;
                while (lo < hi) {
                    const int mid = (lo + hi + 1) >> 1;
                    if (s_dst[wv][mid] <= o) lo = mid; else hi = mid - 1;
                }
                const int64_t src = s_src[wv][lo] + (o - s_dst[wv][lo]);
                const uint32_t m = mask_in[src];
                key_out[o] = key_in[src];
                mask_out[o] = m;
                cread[o] = (uint32_t)(r0 + lo);
                if (lead) {
                    const unsigned long long bit = m ? (unsigned long long)__builtin_ctz(m) : 63ull;
                    atomicMin(&s_lead[wv][lo], (bit << 40) | (unsigned long long)o);
                }
            }
        }
        __builtin_amdgcn_wave_barrier();
        if (lead && lane < nrd) {
            const unsigned long long v = s_lead[wv][lane];
            lead[r0 + lane] = v == ~0ull ? LEAD_NONE : (uint32_t)(v & ((1ull << 40) - 1));
        }
        __builtin_amdgcn_wave_barrier();
    }
}

// ----------------------------------------------------------------- verify

struct VerifyArgs {
    const uint32_t *gcode, *gmask;
    uint64_t G;
    const uint32_t *rcode, *rmask;
    const int64_t *roff;
    const int32_t *len;
    Pass ps;
    const uint64_t *key;
    const uint32_t *cread;
    const int64_t *ncand_ptr;   // number of locations (device scalar)
    Rule rule;
    int32_t RW, TW;             // staged words per lane (read, text), guard word included
    uint16_t *dcap;
    int16_t *vlim;              // the limit each location was verified with
    uint32_t *steps;            // per-location diagonal extensions (profiling only, else null)
    const uint32_t *list;       // locations routed to this kernel (null: all)
    const int64_t *nlist_ptr;   // their number when list is set
    int16_t *rq;                // requested limit per location (null: the read's limit); cleared once verified
    const uint32_t *lead = nullptr;   // per read (chunk index): its lead location, verified on its own
    const int16_t *rlim = nullptr;    // per read: a further cap on the limit (with lead)
};

// Per-lane LDS arrays are laid out [word][lane], so a wave's accesses to its
// lanes' arrays hit 64 distinct banks whatever word each lane needs.
// Only the read' and window codes are staged; the rare read or window that holds
// an N takes its N flags from the packed 1-bit masks in global memory.
struct Stage {
    uint32_t *RC, *TC;
    int16_t *FR;
    int lane;
    const uint32_t *rmask, *gmask;
    int64_t xb, p;   // read start in the packed stream, window start in the genome
    int L, strand;
    // 16 bases of read' and of the window from bit offset b (base b / 2; the funnel
    // shift takes b mod 32)
    __device__ inline uint32_t rb(int b) const {
        int w = b >> 5;
        return funnel(RC[(w + 1) * 64 + lane], RC[w * 64 + lane], (uint32_t)b);
    }
    __device__ inline uint32_t tb(int b) const {
        int w = b >> 5;
        return funnel(TC[(w + 1) * 64 + lane], TC[w * 64 + lane], (uint32_t)b);
    }
    // N flags of read' bases [i, i + 16) and window bases [j, j + 16), one per 2-bit slot
    // (bases past the read or the window may carry any value: the caller masks them)
    __device__ inline uint32_t rn16(int i) const {
        if (strand == 0) return spread16(ext_mask16(rmask, xb + i));
        return spread16(__builtin_bitreverse32(ext_mask16(rmask, xb + L - 16 - i)) >> 16);
    }
    __device__ inline uint32_t tn16(int j) const { return spread16(ext_mask16(gmask, p + j)); }
};

// Rows are kept in bit units (2 bits a base) from here on: the staged words are then
// indexed by the row itself, and the lowest set bit of the mismatch mask is already
// an offset in bits (every flag sits on an even bit).
// Extend a diagonal: from row b on diagonal d (d2 = 2d), advance while read and text
// bases are equal (N equals nothing), 16 bases per step, up to lim2 = 2 min(L, Tn - d).
// Bases past the end of the read or window are compared like any others (the staged
// guard words hold something there); the result is cut back to lim2 instead.
// HAS_N false: neither the read nor the window holds an N, so the N masks are skipped.
template <bool HAS_N>
__device__ __forceinline__ int slide2(const Stage &st, int b, int d2, int lim2) {
    if (b < lim2) {
        uint32_t run;
        do {
            const uint32_t x = st.rb(b) ^ st.tb(b + d2);
            uint32_t m = (x | (x >> 1)) & 0x55555555u;
            if (HAS_N) m |= st.rn16(b >> 1) | st.tn16((b + d2) >> 1);
            run = m ? (uint32_t)__builtin_ctz(m) : 32u;
            b += (int)run;
        } while (run == 32u && b < lim2);
    }
    return min(b, lim2);
}

// Furthest-reaching rows per diagonal for e = 0, 1, ..., K (the rows of the previous
// round kept in LDS, updated in place left to right). Returns D if D <= K, else K + 1.
template <int KMAX, bool HAS_N>
__device__ inline int lv_lane(const Stage &st, int L, int Tn, int K, uint32_t &nsteps) {
    constexpr int NEG = -30000;
    const int lane = st.lane;
    const int L2 = 2 * L, T2 = 2 * Tn;
    const int b0 = slide2<HAS_N>(st, 0, 0, min(L2, T2));
    if (b0 >= L2) return 0;
    for (int t = 0; t < 2 * KMAX + 3; t++) st.FR[t * 64 + lane] = (int16_t)NEG;
    st.FR[(KMAX + 1) * 64 + lane] = (int16_t)b0;
    for (int e = 1; e <= K; e++) {
        int left = NEG;   // previous round's value on diagonal d - 1
        for (int d = -e; d <= e; d++) {
            const int idx = d + KMAX + 1;
            const int od = st.FR[idx * 64 + lane], orr = st.FR[(idx + 1) * 64 + lane];
            const int lim2 = min(L2, T2 - 2 * d);
            int b = max(left, max(od, orr) + 2);
            left = od;
            b = min(b, lim2);
            if (b >= max(0, -2 * d)) {
                nsteps++;
                b = slide2<HAS_N>(st, b, 2 * d, lim2);
                if (b >= L2) return e;
            } else {
                b = NEG;
            }
            st.FR[idx * 64 + lane] = (int16_t)b;
        }
    }
    return K + 1;
}

// The same with the furthest rows in registers, for limits up to KM (every diagonal
// index is a compile-time constant once the rounds are unrolled).
template <int KM, bool HAS_N>
__device__ __forceinline__ int lv_lane_reg(const Stage &st, int L, int Tn, int K, uint32_t &nsteps) {
    constexpr int NEG = -30000;
    const int L2 = 2 * L, T2 = 2 * Tn;
    const int b0 = slide2<HAS_N>(st, 0, 0, min(L2, T2));
    if (b0 >= L2) return 0;
    int fr[2 * KM + 3];
#pragma unroll
    for (int t = 0; t < 2 * KM + 3; t++) fr[t] = NEG;
    fr[KM + 1] = b0;
    int D = K + 1;
#pragma unroll
    for (int e = 1; e <= KM; e++) {
        if (e <= K && D > K) {
            int left = NEG;   // previous round's value on diagonal d - 1
#pragma unroll
            for (int d = -e; d <= e; d++) {
                const int idx = d + KM + 1;
                const int od = fr[idx], orr = fr[idx + 1];
                const int lim2 = min(L2, T2 - 2 * d);
                int b = max(left, max(od, orr) + 2);
                left = od;
                b = min(b, lim2);
                // diagonals after one that reached the end in this round are still
                // extended (harmless: D stays e, and no later round runs)
                if (b >= max(0, -2 * d)) {
                    nsteps++;
                    b = slide2<HAS_N>(st, b, 2 * d, lim2);
                    if (b >= L2) D = e;
                } else {
                    b = NEG;
                }
                fr[idx] = b;
            }
        }
    }
    return D;
}

// Bounded edit distance (Section 3.2): D = min over j of Lev(read', text[0, j)),
// start anchored at p, end free, read' the read or its reverse complement.
// Furthest-reaching rows per diagonal, e = 0, 1, ..., limit; returns D if D <= K,
// else K + 1.
template <int KMAX>
__device__ __forceinline__ void verify_lane(const VerifyArgs &a, int64_t k, uint32_t *sm) {
    const int lane = threadIdx.x & 63;
    Stage st;
    st.lane = lane;
    st.RC = sm;
    st.TC = st.RC + a.RW * 64;
    st.FR = reinterpret_cast<int16_t *>(st.TC + a.TW * 64);

    const uint64_t key = a.key[k];
    const int64_t p = (int64_t)(key >> 1);
    const int strand = (int)(key & 1);
    const uint32_t cr = a.cread[k];
    if (a.lead && a.lead[cr] == (uint32_t)k) return;   // verified at the full limit already
    const int64_t g = gid(a.ps, cr);
    const int L = a.len[g];
    int K = a.rq ? (int)a.rq[k] : min(dmax_for_length(a.rule, L) + a.rule.c - 1, a.ps.Kcap);
    if (a.rlim) K = min(K, (int)a.rlim[cr]);
    const int64_t xb = STREAM_GUARD + a.roff[g];
    const int Tn = (int)min((int64_t)a.G - p, (int64_t)L + K);

    // read' and window, 16 bases per word, each raw word loaded once
    const int nrw = (L + 15) >> 4;
    if (strand == 0) {
        const int64_t q = xb >> 4;
        const uint32_t sh = (uint32_t)(xb & 15) * 2;
        uint32_t lo = a.rcode[q];
        for (int w = 0; w < nrw; w++) {
            const uint32_t hi = a.rcode[q + w + 1];
            st.RC[w * 64 + lane] = funnel(hi, lo, sh);
            lo = hi;
        }
    } else {
        // word w of the reverse complement holds bases [xe - 16(w+1), xe - 16w) of the stream
        const int64_t xe = xb + L;
        const int64_t q = xe >> 4;
        const uint32_t sh = (uint32_t)(xe & 15) * 2;
        uint32_t hi = a.rcode[q];
        for (int w = 0; w < nrw; w++) {
            const uint32_t lo = a.rcode[q - w - 1];
            st.RC[w * 64 + lane] = rc16(funnel(hi, lo, sh));
            hi = lo;
        }
    }
    st.RC[nrw * 64 + lane] = 0;
    const int ntw = (Tn + 15) >> 4;
    {
        const int64_t q = p >> 4;
        const uint32_t sh = (uint32_t)(p & 15) * 2;
        uint32_t lo = a.gcode[q];
        for (int w = 0; w < ntw; w++) {
            const uint32_t hi = a.gcode[q + w + 1];
            st.TC[w * 64 + lane] = funnel(hi, lo, sh);
            lo = hi;
        }
    }
    st.TC[ntw * 64 + lane] = 0;
    const uint32_t anyn = any_n(a.rmask, xb, L) | any_n(a.gmask, p, Tn);
    st.rmask = a.rmask;
    st.gmask = a.gmask;
    st.xb = xb;
    st.p = p;
    st.L = L;
    st.strand = strand;

    uint32_t nsteps = 1;
    int D;
    if constexpr (KMAX <= 17)
        D = anyn ? lv_lane_reg<KMAX, true>(st, L, Tn, K, nsteps) : lv_lane_reg<KMAX, false>(st, L, Tn, K, nsteps);
    else
        D = anyn ? lv_lane<KMAX, true>(st, L, Tn, K, nsteps) : lv_lane<KMAX, false>(st, L, Tn, K, nsteps);
    a.dcap[k] = (uint16_t)D;
    a.vlim[k] = (int16_t)K;
    if (a.steps) a.steps[k] = (a.rq ? a.steps[k] : 0u) + nsteps;
}


template <int KMAX>
__device__ __forceinline__ void verify_lanes(const VerifyArgs &a, uint32_t *sm) {
    const int lane = threadIdx.x;
    const int64_t n = a.list ? *a.nlist_ptr : *a.ncand_ptr;
    for (int64_t idx = (int64_t)blockIdx.x * 64 + lane; idx < n; idx += (int64_t)gridDim.x * 64)
        verify_lane<KMAX>(a, a.list ? (int64_t)a.list[idx] : idx, sm);
}

template <int KMAX>
__global__ __launch_bounds__(64) void k_verify(VerifyArgs a) {
    extern __shared__ uint32_t sm[];
    verify_lanes<KMAX>(a, sm);
}

// The same lane tile over the locations replays asked for (each at its requested
// limit); a kernel of its own so that profiles tell the two apart.
template <int KMAX>
__global__ __launch_bounds__(64) void k_verify_requested(VerifyArgs a) {
    extern __shared__ uint32_t sm[];
    verify_lanes<KMAX>(a, sm);
}

// Lane per read: its lead location (Algorithm 1's first call) at the read's full limit
// (a.ps.Kcap set above every limit), then the cap on its other locations' limits for the
// first verification. After a first call at distance d1 <= d_max(L), every later call of
// the replay runs at limit d1 + c - 1 or below (the best distance only falls, and a
// second location within c lowers the limit to d_best - 1), so verifying the others at
// min(Kpass, d1 + c - 1) answers as many calls as verifying them at Kpass does.
template <int KMAX>
__global__ __launch_bounds__(64) void k_verify_lead(VerifyArgs a, const uint32_t *lead, int16_t *rlim, int Kpass) {
    extern __shared__ uint32_t sm[];
    for (int64_t r = (int64_t)blockIdx.x * 64 + threadIdx.x; r < a.ps.nr; r += (int64_t)gridDim.x * 64) {
        const uint32_t k = lead[r];
        int lim = Kpass;
        if (k != LEAD_NONE) {
            verify_lane<KMAX>(a, (int64_t)k, sm);
            const int d1 = (int)a.dcap[k];
            const int dm = dmax_for_length(a.rule, a.len[gid(a.ps, r)]);
            if (d1 <= dm) lim = min(Kpass, d1 + a.rule.c - 1);
        }
        rlim[r] = (int16_t)lim;
    }
}

// Locations whose read or limit is too large for one lane: one wave per location.
// Lanes take diagonals (64 per step, as many steps as the round needs), the
// previous round's furthest rows are read from one LDS buffer and the new ones
// written to the other, and the read' and text window are staged in LDS once.
struct WaveVerifyArgs {
    const uint32_t *gcode, *gmask;
    uint64_t G;
    const uint32_t *rcode, *rmask;
    const int64_t *roff;
    const int32_t *len;
    Pass ps;
    const uint64_t *key;
    const uint32_t *cread;
    Rule rule;
    int32_t RW, TW, KL;         // staged words (guard included) and the largest limit
    uint16_t *dcap;
    int16_t *vlim;
    uint32_t *steps;
    unsigned long long *next;   // shared work counter (work-stealing launches), null: static stride
    int16_t *rq;                // requested limit per location, tagged REQ_WAVE (null: the read's limit);
                                // cleared once verified
};

// 16 bases of a staged array from bit offset b (base b / 2)
__device__ inline uint32_t lds_b32(const uint32_t *A, int b) {
    const int w = b >> 5;
    return funnel(A[w + 1], A[w], (uint32_t)b);
}

// Extend diagonal d from read row i (text column i + d) while bases are equal, 16 per
// step; the read' and window codes are in LDS, and when either holds an N (HAS_N)
// the N flags come from the packed 1-bit masks in global memory.
struct WaveText {
    const uint32_t *RC, *TC;
    const uint32_t *rmask, *gmask;
    int64_t xb, p;
    int L, Tn, strand;
};

// Rows in bit units as in the lane tile: from row b on diagonal d (d2 = 2d) up to
// lim2 = 2 min(L, Tn - d), bases past the ends compared like any others and the
// result cut back to lim2.
template <bool HAS_N>
__device__ inline int wave_slide2(const WaveText &w, int b, int d2, int lim2) {
    if (b < lim2) {
        uint32_t run;
        do {
            const uint32_t x = lds_b32(w.RC, b) ^ lds_b32(w.TC, b + d2);
            uint32_t m = (x | (x >> 1)) & 0x55555555u;
            if (HAS_N) {
                const int i = b >> 1, j = (b + d2) >> 1;
                const uint32_t rn = w.strand == 0 ? ext_mask16(w.rmask, w.xb + i)
                                                  : __builtin_bitreverse32(ext_mask16(w.rmask, w.xb + w.L - 16 - i)) >> 16;
                m |= spread16(rn) | spread16(ext_mask16(w.gmask, w.p + j));
            }
            run = m ? (uint32_t)__builtin_ctz(m) : 32u;
            b += (int)run;
        } while (run == 32u && b < lim2);
    }
    return min(b, lim2);
}

// Furthest rows per diagonal for e = 0, 1, ..., K with lanes over diagonals (64 per
// step), the previous round's rows read from one LDS buffer and the new ones written to
// the other (16-bit: rows never exceed the read length). D if D <= K, else K + 1.
template <bool HAS_N>
__device__ inline int lv_wave(const WaveText &w, int K, int16_t *F0, int16_t *F1, uint32_t &nsteps) {
    constexpr int NEG = -30000;
    const int lane = threadIdx.x;
    const int L = w.L, Tn = w.Tn;
    // rows are stored in bases (reads up to 16384 bases fit 16 bits), slid in bits
    for (int t = lane; t < 2 * max(K, 0) + 3; t += 64) { F0[t] = (int16_t)NEG; F1[t] = (int16_t)NEG; }
    int i0 = 0;
    if (lane == 0) i0 = wave_slide2<HAS_N>(w, 0, 0, 2 * min(L, Tn)) >> 1;
    i0 = __shfl(i0, 0, 64);
    if (i0 >= L) return 0;
    if (lane == 0) F0[K + 1] = (int16_t)i0;
    __syncthreads();
    int16_t *prev = F0, *nxt = F1;
    for (int e = 1; e <= K; e++) {
        bool hit = false;
        for (int d = -e + lane; d <= e; d += 64) {
            const int idx = d + K + 1;
            const int lim = min(L, Tn - d);
            int i = max((int)prev[idx - 1], max((int)prev[idx], (int)prev[idx + 1]) + 1);
            i = min(i, lim);
            if (i >= max(0, -d)) {
                nsteps++;
                i = wave_slide2<HAS_N>(w, 2 * i, 2 * d, 2 * lim) >> 1;
                if (i >= L) hit = true;
            } else {
                i = NEG;
            }
            nxt[idx] = (int16_t)i;
        }
        const bool done = __ballot(hit) != 0;
        __syncthreads();
        if (done) return e;
        int16_t *t = prev; prev = nxt; nxt = t;
    }
    return K + 1;
}

__device__ inline void verify_loc_wave(const WaveVerifyArgs &a, int64_t k, uint32_t *sm) {
    const int lane = threadIdx.x;
    uint32_t *RC = sm, *TC = RC + a.RW;
    int16_t *F0 = reinterpret_cast<int16_t *>(TC + a.TW), *F1 = F0 + (2 * a.KL + 3);
    const uint64_t key = a.key[k];
    const int64_t p = (int64_t)(key >> 1);
    const int strand = (int)(key & 1);
    const int64_t g = gid(a.ps, a.cread[k]);
    const int L = a.len[g];
    const int K = a.rq ? ((int)a.rq[k] & REQ_LIMIT_MASK) : min(dmax_for_length(a.rule, L) + a.rule.c - 1, a.ps.Kcap);
    const int64_t xb = STREAM_GUARD + a.roff[g];
    const int Tn = (int)min((int64_t)a.G - p, (int64_t)L + max(K, 0));
    const int nrw = (L + 15) >> 4, ntw = (Tn + 15) >> 4;
    for (int w = lane; w < nrw; w += 64) {
        if (strand == 0) {
            RC[w] = ext_code16(a.rcode, xb + 16 * w);
        } else {
            RC[w] = rc16(ext_code16(a.rcode, xb + L - 16 * (w + 1)));
        }
    }
    for (int w = lane; w < ntw; w += 64) TC[w] = ext_code16(a.gcode, p + 16 * w);
    if (lane == 0) { RC[nrw] = 0; TC[ntw] = 0; }
    // any N in the read or the window (32 flags per word, each lane a few words)
    uint32_t nn = 0;
    for (int64_t m = (xb >> 5) + lane; m <= (xb + L - 1) >> 5; m += 64) nn |= a.rmask[m];
    for (int64_t m = (p >> 5) + lane; m <= (p + Tn - 1) >> 5; m += 64) nn |= a.gmask[m];
    // the end words may hold flags of neighbouring bases: then the N path is taken for
    // nothing (same result, slower)
    const bool has_n = __ballot(nn != 0) != 0;
    __syncthreads();
    const WaveText w{RC, TC, a.rmask, a.gmask, xb, p, L, Tn, strand};
    uint32_t nsteps = 1;
    const int D = has_n ? lv_wave<true>(w, K, F0, F1, nsteps) : lv_wave<false>(w, K, F0, F1, nsteps);
    if (a.steps) {
        for (int d = 32; d >= 1; d >>= 1) nsteps += __shfl_xor(nsteps, d, 64);
    }
    if (lane == 0) {
        a.dcap[k] = (uint16_t)D;
        a.vlim[k] = (int16_t)K;
        if (a.steps) a.steps[k] = (a.rq ? a.steps[k] : 0u) + nsteps;
    }
    __syncthreads();
}

// Verification requests of the reads being replayed.
struct RequestArgs {
    const uint32_t *rlist;      // chunk reads being replayed
    const int64_t *n_ptr;       // how many
    const uint32_t *reqcount;   // per read: locations asked for (REQ_WAVE_READ: wave tile)
    const uint32_t *req_area;   // the locations, listed at the read's first location slot
    const int64_t *coff;        // first location slot of each read
};

// Requested locations per replayed read for the lane tile (0 for wave-tile reads).
struct LaneReqCount {
    const uint32_t *rlist, *reqcount;
    int64_t n;
    __host__ __device__ int64_t operator()(int64_t i) const {
        if (i >= n) return 0;
        const uint32_t c = reqcount[rlist[i]];
        return (c & REQ_WAVE_READ) ? 0 : (int64_t)c;
    }
};

// Lane tile: the requested locations of all replayed reads, one list (a wave per
// read copies its own at its offset; the last offset is the total).
__global__ __launch_bounds__(256) void k_flatten_requests(RequestArgs q, const int64_t *offs, uint32_t *out) {
    const int lane = threadIdx.x & 63;
    const int64_t n = *q.n_ptr;
    for (int64_t i = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6; i < n;
         i += ((int64_t)gridDim.x * blockDim.x) >> 6) {
        const uint32_t r = q.rlist[i];
        const uint32_t c = q.reqcount[r];
        if (c & REQ_WAVE_READ) continue;
        const int64_t base = q.coff[r], dst = offs[i];
        for (uint32_t k = lane; k < c; k += 64) out[dst + k] = q.req_area[base + k];
    }
}

// Wave tile: one wave per read of the replay list, its requested locations one at a
// time (work stealing over reads when `next` is set).
__global__ __launch_bounds__(64) void k_verify_requests_wave(WaveVerifyArgs a, RequestArgs q) {
    extern __shared__ uint32_t wsm[];
    const int64_t n = *q.n_ptr;
    for (int64_t idx = blockIdx.x;;) {
        if (a.next) {
            unsigned long long f = 0;
            if (threadIdx.x == 0) f = atomicAdd(a.next, 1ull);
            idx = (int64_t)__shfl((unsigned long long)f, 0, 64);
        }
        if (idx >= n) break;
        const uint32_t r = q.rlist[idx];
        const uint32_t c = q.reqcount[r];
        if (c & REQ_WAVE_READ) {
            const int64_t base = q.coff[r];
            for (uint32_t i = 0; i < (c & ~REQ_WAVE_READ); i++) verify_loc_wave(a, (int64_t)q.req_area[base + i], wsm);
        }
        if (!a.next) idx += gridDim.x;
    }
}

// Batched form: one persistent launch gives every short location of a pass its first
// verification (long reads' locations are verified on request). Each wave takes
// groups of 64 locations (lane tile) in guided chunks of about half the remaining
// groups divided by the number of waves, at least one (the range rule of Section 2.3).
struct StealArgs {
    VerifyArgs va;               // lane tile over the short list
    unsigned long long *next;    // [1]: group cursor
    int32_t nwaves;
};

template <int KMAX>
__global__ __launch_bounds__(64) void k_verify_steal(StealArgs a) {
    extern __shared__ uint32_t ssm[];
    const int lane = threadIdx.x;
    const int64_t nshort = *a.va.nlist_ptr;
    const int64_t ngroups = (nshort + 63) / 64;
    for (;;) {
        unsigned long long first = 0, take = 1;
        if (lane == 0) {
            const long long seen = (long long)*(volatile unsigned long long *)&a.next[1];
            const long long rem = (long long)ngroups - seen;
            take = rem > 2ll * a.nwaves ? (unsigned long long)(rem / (2ll * a.nwaves)) : 1ull;
            first = atomicAdd(&a.next[1], take);
        }
        first = __shfl(first, 0, 64);
        take = __shfl(take, 0, 64);
        if ((int64_t)first >= ngroups) break;
        const int64_t last = min((int64_t)(first + take), ngroups);
        for (int64_t gi = (int64_t)first; gi < last; gi++) {
            const int64_t idx = gi * 64 + lane;
            if (idx < nshort) verify_lane<KMAX>(a.va, (int64_t)a.va.list[idx], ssm);
        }
    }
}

// Locations hit by none of the first seed slots (`bits`): left for verification on
// request (capped distance unknown above -1).
// Exact-duplicate classes (Section 4.2): for a read whose text window L + d_max(L) + c - 1
// fits the class window, location k's representative is the read's location on the same
// strand at the first position of k's class. That location exists whenever k's class is
// not its own: the two W-base windows are identical, so every seed that hits k hits it at
// the same offset, with the same counts (with a strided index the other position may not
// be indexed; then k stays its own). k itself otherwise. An alias is left unverified: its
// representative's results answer it (the replays take them). *nalias (profiling only,
// else null) counts aliases, one atomic add per workgroup.
__global__ __launch_bounds__(256) void k_dup_alias(DevIndex ix, const uint64_t *key, const uint32_t *cread,
                                                   const int64_t *coff, const int32_t *len, Pass ps, Rule rule,
                                                   const int64_t *ncand_ptr, uint32_t *alias, uint16_t *dcap,
                                                   int16_t *vlim, uint32_t *steps, unsigned long long *nalias) {
    const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t n = *ncand_ptr;
    uint32_t al = (uint32_t)k;
    if (k < n) {
        const uint32_t r = cread[k];
        const int L = len[gid(ps, r)];
        if (L + dmax_for_length(rule, L) + rule.c - 1 <= ix.dup_w) {
            const uint64_t kk = key[k];
            const uint64_t p = kk >> 1;
            const uint64_t h = ((ix.repbits[p >> 5] >> (p & 31)) & 1u) ? ix.rep[p] : p;
            if (h != p) {
                const uint64_t want = (h << 1) | (kk & 1);
                int64_t lo = coff[r], hi = coff[r + 1];
                while (lo < hi) {
                    const int64_t mid = (lo + hi) >> 1;
                    if (key[mid] < want) lo = mid + 1; else hi = mid;
                }
                if (lo < coff[r + 1] && key[lo] == want) al = (uint32_t)lo;
            }
        }
        alias[k] = al;
        if (al != (uint32_t)k) {
            dcap[k] = 0xFFFF;
            vlim[k] = -1;
            if (steps) steps[k] = 0;
        }
    }
    if (nalias) {
        __shared__ uint32_t wsum[4];
        const uint64_t b = __ballot(k < n && al != (uint32_t)k);
        if ((threadIdx.x & 63) == 0) wsum[threadIdx.x >> 6] = (uint32_t)__popcll(b);
        __syncthreads();
        if (threadIdx.x == 0) {
            const uint32_t t = wsum[0] + wsum[1] + wsum[2] + wsum[3];
            if (t) atomicAdd(nalias, (unsigned long long)t);
        }
    }
}

__global__ void k_mark_late(const uint32_t *mask, const int64_t *ncand_ptr, uint32_t bits, uint16_t *dcap,
                            int16_t *vlim, uint32_t *steps) {
    const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= *ncand_ptr || (mask[k] & bits) != 0) return;
    dcap[k] = 0xFFFF;
    vlim[k] = -1;
    if (steps) steps[k] = 0;
}

// Locations left for verification on request: capped distance unknown above -1.
__global__ void k_mark_unverified(const uint32_t *list, const int64_t *n_ptr, uint16_t *dcap, int16_t *vlim,
                                  uint32_t *steps) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= *n_ptr) return;
    const uint32_t k = list[i];
    dcap[k] = 0xFFFF;
    vlim[k] = -1;
    if (steps) steps[k] = 0;
}

__global__ void k_sum_u32(const uint32_t *v, const int64_t *n_ptr, unsigned long long *out) {
    __shared__ unsigned long long red[256];
    const int64_t n = *n_ptr;
    unsigned long long acc = 0;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        acc += v[i];
    red[threadIdx.x] = acc;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) atomicAdd(out, red[0]);
}

// ----------------------------------------------------------------- replay

struct ReplayArgs {
    const ProbeRec *pr;
    const uint64_t *key;
    const uint32_t *mask;
    const uint16_t *dcap;
    const int16_t *vlim;
    const int64_t *coff;
    const uint32_t *count;
    uint64_t *bmin;
    uint8_t *scored;
    const int32_t *len;
    Pass ps;
    Rule rule;
    Shifts sh;
    const uint32_t *alias;      // per location: its exact-duplicate representative (null: no classes)
    uint8_t *rflag;             // per chunk read: RF_DONE / RF_PENDING / RF_REPLAY
    int16_t *rq;                // per location: requested verify limit (REQ_WAVE-tagged for long reads)
    uint32_t *req_area;         // per read, at its first location slot: the locations it asks for
    uint32_t *reqcount;         // per chunk read: how many (REQ_WAVE_READ set for the wave tile)
    const uint32_t *rlist;      // chunk reads to replay (null: all nr)
    const int64_t *rlist_n;
    int32_t round;              // 0 for the first replay of the chunk, then 1, 2, ...
    int32_t exact_rounds;       // short reads ask for single locations in rounds below this
    int32_t request_top;        // a single-location request of a lane-tile read takes this many best undecided locations
    int32_t lane_lmax;          // reads up to this length (limit <= 63) are verified one lane per location
    int64_t *pos;
    int8_t *strand;
    int32_t *dist, *second;
    int8_t *call;
};

// The best / second-best state of Algorithm 1 with the bucket merge (Section 3.2,
// omitted aspect 1). Held identically by every lane of the read's wave.
struct ReadState {
    int d_best, d_second;
    int64_t best_p;
    int best_s;
    int64_t best_rep;
};

__device__ inline bool lex_less(int d1, int64_t p1, int s1, int d2, int64_t p2, int s2) {
    return d1 < d2 || (d1 == d2 && (p1 < p2 || (p1 == p2 && s1 < s2)));
}

// Algorithm 1's three-case d_limit.
__device__ inline int d_limit(const ReadState &st, int dmax, int c) {
    if (st.d_best > dmax) return dmax + c - 1;
    if (st.d_second >= st.d_best + c) return st.d_best + c - 1;
    return st.d_best - 1;
}

// State update for a result at a location whose bucket now holds (vd, vp) (shared
// by both replay paths).
__device__ inline void state_update(ReadState &st, int64_t rep, int vd, int64_t vp, int s) {
    if (st.best_rep == rep) {
        st.d_best = vd;
        st.best_p = vp;
    } else if (st.best_rep < 0 || lex_less(vd, vp, s, st.d_best, st.best_p, st.best_s)) {
        st.d_second = st.best_rep < 0 ? DINF : st.d_best;
        st.d_best = vd;
        st.best_p = vp;
        st.best_s = s;
        st.best_rep = rep;
    } else if (vd < st.d_second) {
        st.d_second = vd;
    }
}

// A register's value in lane l, l the same in every lane: a scalar read of one lane
// (no LDS round trip, unlike a shuffle).
__device__ inline int lane_i32(int v, int l) { return __builtin_amdgcn_readlane(v, l); }
__device__ inline uint64_t lane_u64(uint64_t v, int l) {
    const uint32_t lo = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)v, l);
    const uint32_t hi = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)(v >> 32), l);
    return ((uint64_t)hi << 32) | lo;
}

// The lowest lane holding the largest v (0 <= v < 64, 0 = no candidate), or -1:
// one ballot per bit from the top, keeping the lanes that have it.
__device__ inline int wave_argmax6(uint32_t v) {
    uint64_t alive = __ballot(v != 0);
    if (!alive) return -1;
    for (int b = 5; b >= 0; b--) {
        const uint64_t hb = alive & __ballot((v >> b) & 1u);
        if (hb) alive = hb;
    }
    return __builtin_ctzll(alive);
}

// A read's verification requests: the locations whose `want` is set (all lanes of
// the wave call this together), each with limit `code`, listed at the read's first
// location slot.
//
// With exact-duplicate classes a location and its representative (an identical text
// window, see k_dup_alias) have the same distance, so a replay takes whichever of the two
// was verified with the higher limit, and a location does not ask for a verification
// when its representative asks in the same round.
__device__ inline uint32_t load_dv(const ReplayArgs &a, int64_t i) {
    uint32_t dc = a.dcap[i];
    int vl = a.vlim[i];
    if (a.alias) {
        const int64_t j = a.alias[i];
        if (j != i && a.vlim[j] > vl) {
            dc = a.dcap[j];
            vl = a.vlim[j];
        }
    }
    return dc | ((uint32_t)(uint16_t)vl << 16);
}
__device__ inline int dv_dc(uint32_t dv) { return (int)(dv & 0xFFFFu); }
__device__ inline int dv_vl(uint32_t dv) { return (int)(int16_t)(dv >> 16); }

__device__ inline void light_request(const ReplayArgs &a, int64_t base, int64_t r, bool want, int code,
                                     bool wave_tile, int lane) {
    if (a.alias) {
        const int64_t cnt = a.count[r];
        const int64_t j = lane < cnt ? (int64_t)a.alias[base + lane] - base : lane;
        const bool rep_wants = __shfl((int)want, (int)(j & 63), 64) != 0;
        if (j != lane && rep_wants) want = false;
    }
    const uint64_t b = __ballot(want);
    if (want) {
        a.rq[base + lane] = (int16_t)code;
        a.req_area[base + __popcll(b & ((1ull << lane) - 1))] = (uint32_t)(base + lane);
    }
    if (lane == 0) a.reqcount[r] = (uint32_t)__popcll(b) | (wave_tile ? REQ_WAVE_READ : 0u);
}

// Same for reads whose locations are in global memory: `want(k)` over all of them.
template <class Want>
__device__ inline void heavy_request(const ReplayArgs &a, int64_t base, int64_t C, int64_t r, Want want, int code,
                                     bool wave_tile, int lane) {
    uint32_t n = 0;
    for (int64_t k0 = 0; k0 < C; k0 += 64) {
        const int64_t k = k0 + lane;
        bool w = k < C && want(k);
        if (w && a.alias) {
            const int64_t j = (int64_t)a.alias[base + k] - base;
            if (j != k && want(j)) w = false;
        }
        const uint64_t b = __ballot(w);
        if (w) {
            a.rq[base + k] = (int16_t)code;
            a.req_area[base + n + __popcll(b & ((1ull << lane) - 1))] = (uint32_t)(base + k);
        }
        n += (uint32_t)__popcll(b);
    }
    if (lane == 0) a.reqcount[r] = n | (wave_tile ? REQ_WAVE_READ : 0u);
}

// Reads with at most 64 locations: location k lives in lane k's registers (key,
// seed mask, capped distance, verified limit, scored flag, bucket minimum when k is
// its bucket's representative), so the replay runs on shuffles and ballots.
__device__ inline void light_record(int j, int d, ReadState &st, uint64_t key, int rep, uint64_t &bmin, int lane) {
    const uint64_t kj = lane_u64(key, j);
    const int64_t p = (int64_t)(kj >> 1);
    const int s = (int)(kj & 1);
    const int rj = lane_i32(rep, j);
    const uint64_t bv = lane_u64(bmin, rj);
    const uint64_t nv0 = ((uint64_t)d << 32) | (uint64_t)p;
    const uint64_t nv = nv0 < bv ? nv0 : bv;
    if (lane == rj) bmin = nv;
    state_update(st, rj, (int)(nv >> 32), (int64_t)(nv & 0xFFFFFFFFull), s);
}

// A result d <= limit at location k: merge into its bucket and update the state.
// The bucket representative is the first location of the same strand and bucket
// in key order; a bucket spans at most 2 * bucket locations, so with a 32-base
// bucket it is found among the 64 keys ending at k.
__device__ inline void wave_record(const ReplayArgs &a, int64_t base, int64_t k, int d, ReadState &st, int lane) {
    const uint64_t kk = a.key[base + k];
    const int64_t p = (int64_t)(kk >> 1);
    const int s = (int)(kk & 1);
    const int64_t bk = p / a.rule.bucket;
    int64_t j = k;
    for (int64_t lo = k; ; lo -= 64) {
        const int64_t q = lo - lane;
        bool same = false;
        if (q >= 0) {
            const uint64_t kq = a.key[base + q];
            same = (int64_t)(kq >> 1) / a.rule.bucket == bk && (int)(kq & 1) == s;
        }
        const uint64_t m = __ballot(same);
        // keys are sorted, so the bucket's locations are contiguous: the highest
        // set lane is its first location in this window
        if (m) j = lo - (63 - __clzll(m));
        // the run continues below this window only if every lane matched in bucket
        const bool inb = (q >= 0) && (int64_t)(a.key[base + q] >> 1) / a.rule.bucket == bk;
        if (__ballot(inb) != ~0ull || lo - 64 < 0) break;
    }
    const uint64_t nv0 = ((uint64_t)d << 32) | (uint64_t)p;
    const uint64_t old = a.bmin[base + j];
    const uint64_t nv = nv0 < old ? nv0 : old;
    if (lane == 0) a.bmin[base + j] = nv;
    state_update(st, j, (int)(nv >> 32), (int64_t)(nv & 0xFFFFFFFFull), s);
}



// EditDistance(Read, Reference[p_k], lim) from what is known about location k: its
// capped distance dc = min(D, vl + 1) for the limit vl it was verified with.
// Seed slots that count as non-overlapping seeds of Algorithm 1 (t): the round-0 slots,
// at offsets that are multiples of s, i.e. the first L / s slots; with a strided index
// only those whose ST seeds all fit in the read, the first (L - ST + 1) / s of them.
__device__ inline int round0_slots(int L, int s, int ST) {
    return L >= ST - 1 ? (L - ST + 1) / s : 0;
}

// Returns the distance, -1 for the special value, or -2 when it is not known yet.
__device__ inline int ed_answer(int dc, int vl, int lim) {
    if (dc <= vl) return dc <= lim ? dc : -1;
    return lim <= vl ? -1 : -2;
}

// Algorithm 1's control flow over the seed masks and capped distances of one read,
// one wave per read. A call is answered from the location's capped distance; when
// that does not decide it (the location was verified with a limit below the one
// Algorithm 1 asks for), the read records a verification request and is replayed
// once it is answered. In the main loop a read asks for that one location at
// exactly that limit; a short read, in the lane tile, does so only while that limit
// is the full one, d_max + c - 1, and for at most exact_rounds rounds, and otherwise
// asks for every unscored location it has not decided at the current limit. In the
// phase that scores every remaining location it asks for every remaining undecided
// location at the current limit. The limit only shrinks as results come in (up to
// rare steps of one, answered by a further round), so a location verified at the
// current limit is decided for every later call. A read
// that needs a seed this pass did not probe is left to the next pass. The phase
// that scores every remaining location only changes state at calls that return a
// distance, so it scans for the next such location in selection order (vote count
// descending, then p, then strand) instead of visiting each one.
// CAP 0: reads with at most 64 locations (registers); otherwise reads with more,
// staged in LDS when they have at most CAP (global memory beyond).
template <int CAP>
__global__ __launch_bounds__(256) void k_replay(ReplayArgs a) {
    constexpr bool LIGHT = CAP == 0;
    extern __shared__ uint32_t rsm[];   // heavy instantiations: heavy_lds_words(CAP) per wave
    const int lane = threadIdx.x & 63;
    const int64_t wave = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6;
    const int64_t nwaves = ((int64_t)gridDim.x * blockDim.x) >> 6;
    const int64_t nlist = a.rlist ? *a.rlist_n : a.ps.nr;
    for (int64_t ri = wave; ri < nlist; ri += nwaves) {
        const int64_t r = a.rlist ? (int64_t)a.rlist[ri] : ri;
        const int64_t C = a.count[r];
        if (LIGHT != (C <= 64)) continue;
        const int64_t g = gid(a.ps, r);
        const int L = a.len[g];
        const int dmax = dmax_for_length(a.rule, L), c = a.rule.c;
        const int NS = a.ps.NS;
        const int64_t base = a.coff[r];
        const int Kfull = dmax + c - 1;
        const bool lane_class = L <= a.lane_lmax && Kfull <= LANE_KMAX;
        const bool all_undecided = lane_class && a.round >= a.exact_rounds;
        ReadState st{DINF, DINF, -1, -1, -1};
        const int round0 = round0_slots(L, a.rule.s, a.ps.ST);
        int t = 0, call = -1;
        bool looked = false, all_over = true, ended = false, unresolved = false;
        int64_t need_k = -1;
        uint32_t prefix = 0;
        // seed slot `lane`'s status, loaded once (the loops over seeds read it by lane)
        const int stat = lane < NS ? (int)a.pr[(r * NS + lane) * a.ps.ST].status : ST_NONE;
        if constexpr (LIGHT) {
            // ---- registers: location `lane`
            const bool have = lane < C;
            const uint64_t key = have ? a.key[base + lane] : ~0ull;
            const uint32_t mask = have ? a.mask[base + lane] : 0u;
            const uint32_t dv = have ? load_dv(a, base + lane) : 0u;
            const int dc = dv_dc(dv);
            const int vl = have ? dv_vl(dv) : 0;
            bool scored = false;
            uint64_t bmin = ~0ull;
            // bucket representative: first location of the same strand in the run of
            // equal buckets that ends here
            const int64_t bk = have ? (int64_t)(key >> 1) / a.rule.bucket : -1 - lane;
            const uint32_t bkl = __shfl((unsigned)(uint32_t)bk, (lane + 63) & 63, 64);
            const uint32_t bkh = __shfl((unsigned)(uint32_t)((uint64_t)bk >> 32), (lane + 63) & 63, 64);
            const int64_t bprev = (int64_t)(((uint64_t)bkh << 32) | bkl);
            const uint64_t starts = __ballot(lane == 0 || bprev != bk);
            const uint64_t upto = (lane == 63) ? ~0ull : ((2ull << lane) - 1);
            const int run0 = 63 - __clzll(starts & upto);
            const uint64_t same_s = __ballot(have && (key & 1)) ;
            const uint64_t mine = (key & 1) ? same_s : ~same_s;
            const uint64_t range = upto & ~((1ull << run0) - 1);
            const int rep = __builtin_ctzll(mine & range);
            for (int i = 0; i < NS; i++) {
                const int status = lane_i32(stat, i);
                if (status == ST_NONE) { ended = true; break; }
                if (status == ST_N) continue;
                looked = true;
                if (status == ST_OVER) continue;
                all_over = false;
                prefix |= 1u << i;
                if (i < round0) t++;
                const uint32_t m = mask & prefix;
                const int kb = wave_argmax6((have && m && !scored) ? (uint32_t)__builtin_popcount(m) : 0u);
                if (kb >= 0) {
                    const int lim = d_limit(st, dmax, c);
                    const int res = ed_answer(lane_i32(dc, kb), lane_i32(vl, kb), lim);
                    if (res == -2) {
                        unresolved = true;
                        need_k = kb;
                        if (lane_class && (all_undecided || lim < Kfull)) {
                            light_request(a, base, r, have && !scored && dc > vl && vl < lim, lim, false, lane);
                        } else {
                            // the request_top best locations undecided at this limit (one for a
                            // read of the wave tile: its verifications are costly)
                            bool pick = lane == kb;
                            const bool open = have && !scored && dc > vl && vl < lim && m != 0;
                            const int top = lane_class ? a.request_top : 1;
                            for (int q = 1; q < top; q++) {
                                const int k2 = wave_argmax6((open && !pick) ? (uint32_t)__builtin_popcount(m) : 0u);
                                if (k2 < 0) break;
                                pick |= lane == k2;
                            }
                            light_request(a, base, r, pick, lane_class ? lim : (REQ_WAVE | lim), !lane_class, lane);
                        }
                        break;
                    }
                    if (lane == kb) scored = true;
                    if (res >= 0) light_record(kb, res, st, key, rep, bmin, lane);
                }
                if (st.d_best < c && st.d_second < st.d_best + c) {
                    call = SNAP_MULTIPLE;
                    ended = true;
                    break;
                }
                if (st.d_best < DINF && t >= st.d_best + c) {
                    for (int lev = __builtin_popcount(prefix); lev >= 1 && !unresolved; lev--) {
                        bool in = have && !scored && __builtin_popcount(mask & prefix) == lev;
                        for (;;) {
                            const int lim = d_limit(st, dmax, c);
                            const int res = in ? ed_answer(dc, vl, lim) : -1;
                            const uint64_t bits = __ballot(res != -1);
                            if (!bits) break;
                            const int j = __builtin_ctzll(bits);
                            if ((__ballot(res == -2) >> j) & 1) {
                                unresolved = true;
                                need_k = j;
                                // every remaining location still undecided at the limit
                                const int lr = lim;
                                light_request(a, base, r, have && !scored && (mask & prefix) && dc > vl && vl < lr,
                                              lane_class ? lr : (REQ_WAVE | lr), !lane_class, lane);
                                break;
                            }
                            light_record(j, lane_i32(res, j), st, key, rep, bmin, lane);
                            if (lane <= j) in = false;
                        }
                    }
                    ended = true;
                    break;
                }
            }
        } else {
        // ---- reads with more than 64 locations: seed masks, capped distances, limits
        // and scored flags staged in this wave's LDS when they fit, else read in place
        constexpr int cap = CAP > 0 ? CAP : 32;
        const bool in_lds = C <= cap;
        uint32_t *Lmask = rsm + (threadIdx.x >> 6) * heavy_lds_words(cap);
        uint32_t *Ldv = Lmask + cap;
        uint32_t *Lsc = Ldv + cap;
        uint8_t *Llev = reinterpret_cast<uint8_t *>(Lsc + cap / 32);   // remaining phase: vote count
        if (in_lds) {
            for (int64_t k = lane; k < C; k += 64) {
                Lmask[k] = a.mask[base + k];
                Ldv[k] = load_dv(a, base + k);
            }
            for (int w = lane; w < cap / 32; w += 64) Lsc[w] = 0;
        } else {
            for (int64_t k = lane; k < C; k += 64) a.scored[base + k] = 0;
        }
        for (int64_t k = lane; k < C; k += 64) a.bmin[base + k] = ~0ull;
        __builtin_amdgcn_wave_barrier();
        auto mask_at = [&](int64_t k) -> uint32_t { return in_lds ? Lmask[k] : a.mask[base + k]; };
        auto dc_at = [&](int64_t k) -> int { return dv_dc(in_lds ? Ldv[k] : load_dv(a, base + k)); };
        auto vl_at = [&](int64_t k) -> int { return dv_vl(in_lds ? Ldv[k] : load_dv(a, base + k)); };
        auto scored_at = [&](int64_t k) -> bool {
            return in_lds ? ((Lsc[k >> 5] >> (k & 31)) & 1u) != 0 : a.scored[base + k] != 0;
        };
        for (int i = 0; i < NS; i++) {
            const int status = lane_i32(stat, i);
            if (status == ST_NONE) { ended = true; break; }
            if (status == ST_N) continue;
            looked = true;
            if (status == ST_OVER) continue;
            all_over = false;
            prefix |= 1u << i;
            if (i < round0) t++;
            // the unscored location with the most seeds hitting; ties to smaller p, then +:
            // each lane keeps the first best of its locations (k = lane + 64 j), then the wave
            // takes the highest vote and, among the lanes holding it, the lowest location
            // (one ballot per bit of each)
            uint32_t lv = 0, lk = 0xFFFFFFFFu;
            for (int64_t k = lane; k < C; k += 64) {
                if (!scored_at(k)) {
                    const uint32_t v = (uint32_t)__builtin_popcount(mask_at(k) & prefix);
                    if (v > lv) { lv = v; lk = (uint32_t)k; }
                }
            }
            int64_t kb = -1;
            uint64_t alive = __ballot(lv != 0);
            if (alive) {
                for (int b = 5; b >= 0; b--) {
                    const uint64_t hb = alive & __ballot((lv >> b) & 1u);
                    if (hb) alive = hb;
                }
                for (int b = 31 - __builtin_clz((uint32_t)C); b >= 0; b--) {
                    const uint64_t hb = alive & __ballot(((lk >> b) & 1u) == 0);
                    if (hb) alive = hb;
                }
                kb = (int64_t)(uint32_t)lane_i32((int)lk, __builtin_ctzll(alive));
            }
            if (kb >= 0) {
                const int lim = d_limit(st, dmax, c);
                const int res = ed_answer(dc_at(kb), vl_at(kb), lim);
                if (res == -2) {
                    unresolved = true;
                    need_k = kb;
                    if (lane_class && (all_undecided || lim < Kfull)) {
                        heavy_request(a, base, C, r, [&](int64_t k) {
                            const int dck = dc_at(k), vlk = vl_at(k);
                            return !scored_at(k) && dck > vlk && vlk < lim;
                        }, lim, false, lane);
                    } else {
                        // the request_top best locations undecided at this limit, in
                        // selection order (the next calls of this loop are likely among them;
                        // one for a read of the wave tile, whose verifications are costly)
                        int64_t pick[REQUEST_TOP_MAX];
                        int np = 0;
                        pick[np++] = kb;
                        const int top = lane_class ? a.request_top : 1;
                        for (int m = 1; m < top; m++) {
                            uint32_t bv = 0, bk = 0xFFFFFFFFu;
                            for (int64_t k = lane; k < C; k += 64) {
                                if (scored_at(k)) continue;
                                bool taken = false;
                                for (int q = 0; q < np; q++) taken |= pick[q] == k;
                                if (taken || ed_answer(dc_at(k), vl_at(k), lim) != -2) continue;
                                const uint32_t v = (uint32_t)__builtin_popcount(mask_at(k) & prefix);
                                if (v > bv) { bv = v; bk = (uint32_t)k; }
                            }
                            uint64_t alive2 = __ballot(bv != 0);
                            if (!alive2) break;
                            for (int b = 5; b >= 0; b--) {
                                const uint64_t hb = alive2 & __ballot((bv >> b) & 1u);
                                if (hb) alive2 = hb;
                            }
                            for (int b = 31 - __builtin_clz((uint32_t)C); b >= 0; b--) {
                                const uint64_t hb = alive2 & __ballot(((bk >> b) & 1u) == 0);
                                if (hb) alive2 = hb;
                            }
                            pick[np++] = (int64_t)(uint32_t)lane_i32((int)bk, __builtin_ctzll(alive2));
                        }
                        heavy_request(a, base, C, r, [&](int64_t k) {
                            bool w = false;
                            for (int q = 0; q < np; q++) w |= pick[q] == k;
                            return w;
                        }, lane_class ? lim : (REQ_WAVE | lim), !lane_class, lane);
                    }
                    break;
                }
                if (lane == 0) {
                    if (in_lds) Lsc[kb >> 5] |= 1u << (kb & 31);
                    else a.scored[base + kb] = 1;
                }
                __builtin_amdgcn_wave_barrier();
                if (res >= 0) wave_record(a, base, kb, res, st, lane);
            }
            if (st.d_best < c && st.d_second < st.d_best + c) {
                call = SNAP_MULTIPLE;
                ended = true;
                break;
            }
            if (st.d_best < DINF && t >= st.d_best + c) {
                // score every remaining location; vote counts are frozen now (kept per
                // location in LDS, 0 for a scored one). Only the vote levels some unscored
                // location has are visited (a bit per level, OR-ed over the wave).
                uint64_t levbits = 0;
                for (int64_t k = lane; k < C; k += 64) {
                    const int v = scored_at(k) ? 0 : __builtin_popcount(mask_at(k) & prefix);
                    if (in_lds) Llev[k] = (uint8_t)v;
                    levbits |= 1ull << v;
                }
                for (int m = 1; m < 64; m <<= 1) levbits |= shfl_xor64(levbits, m);
                if (in_lds) __builtin_amdgcn_wave_barrier();
                for (int lev = __builtin_popcount(prefix); lev >= 1 && !unresolved; lev--) {
                    if (!((levbits >> lev) & 1u)) continue;
                    for (int64_t c0 = 0; c0 < C && !unresolved; c0 += 64) {
                        const int64_t k = c0 + lane;
                        bool in = false;
                        int dc = 0, vl = 0;
                        if (k < C && (in_lds ? (int)Llev[k] == lev
                                             : !scored_at(k) && __builtin_popcount(mask_at(k) & prefix) == lev)) {
                            in = true;
                            dc = dc_at(k);
                            vl = vl_at(k);
                        }
                        for (;;) {
                            const int lim = d_limit(st, dmax, c);
                            const int res = in ? ed_answer(dc, vl, lim) : -1;
                            const bool un = res == -2;
                            const uint64_t bits = __ballot(res != -1);
                            if (!bits) break;
                            const int j = __builtin_ctzll(bits);
                            if ((__ballot(un) >> j) & 1) {
                                unresolved = true;
                                need_k = c0 + j;
                                // every remaining location still undecided at the limit
                                const int lr = lim;
                                heavy_request(a, base, C, r, [&](int64_t k2) {
                                    const int dck = dc_at(k2), vlk = vl_at(k2);
                                    return !scored_at(k2) && (mask_at(k2) & prefix) && dck > vlk && vlk < lr;
                                }, lane_class ? lr : (REQ_WAVE | lr), !lane_class, lane);
                                break;
                            }
                            const int dj = lane_i32(res, j);
                            wave_record(a, base, c0 + j, dj, st, lane);
                            // the calls before j returned the special value: scored, no effect
                            if (lane <= j) in = false;
                        }
                    }
                }
                ended = true;
                break;
            }
        }
        }   // locations in global memory
        // all slots of this pass used and the read still has seeds to try
        if (!ended && !unresolved && NS < seeds_for_length(a.rule, L) && seed_offset(a.sh, a.rule.s, L, NS) >= 0)
            unresolved = true;
        if (unresolved) {
            // a distance is missing (requests recorded above) or a seed is
            if (lane == 0) a.rflag[r] = need_k < 0 ? RF_PENDING : RF_REPLAY;
            continue;
        }
        if (call < 0) {
            if (st.d_best <= dmax && st.d_second >= st.d_best + c) call = SNAP_SINGLE;
            else if (st.d_best <= dmax || (looked && all_over)) call = SNAP_MULTIPLE;
            else call = SNAP_NOT_FOUND;
        }
        if (lane == 0) {
            const bool has = st.d_best < DINF;
            a.rflag[r] = RF_DONE;
            a.pos[g] = has ? st.best_p : -1;
            a.strand[g] = (int8_t)(has ? st.best_s : -1);
            a.dist[g] = has ? st.d_best : -1;
            a.second[g] = st.d_second < DINF ? st.d_second : -1;
            a.call[g] = (int8_t)call;
        }
    }
}

// Reads with at most TINY_LOCS locations (most reads: a unique region gives one or
// two): one lane per read, Algorithm 1's control flow run sequentially over
// registers (the same decisions as the wave paths, in the same order).
constexpr int TINY_LOCS = 8;

__global__ __launch_bounds__(256) void k_replay_tiny(ReplayArgs a) {
    const int64_t nlist = a.rlist ? *a.rlist_n : a.ps.nr;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t ri = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; ri < nlist; ri += stride) {
        const int64_t r = a.rlist ? (int64_t)a.rlist[ri] : ri;
        const int C = (int)a.count[r];
        if (C > TINY_LOCS) continue;
        const int64_t g = gid(a.ps, r);
        const int L = a.len[g];
        const int dmax = dmax_for_length(a.rule, L), c = a.rule.c;
        const int NS = a.ps.NS;
        const int64_t base = a.coff[r];
        const int Kfull = dmax + c - 1;
        const bool lane_class = L <= a.lane_lmax && Kfull <= LANE_KMAX;
        const bool all_undecided = lane_class && a.round >= a.exact_rounds;
        // location k: p, strand bit, seed mask, capped distance | verified limit << 16;
        // the bucket minimum is kept at the bucket's representative, the first location
        // of the same bucket and strand (a 4-bit index per location)
        uint32_t P[TINY_LOCS], M[TINY_LOCS], DV[TINY_LOCS];
        uint64_t BM[TINY_LOCS];
        uint32_t sbits = 0, repw = 0;
        {
            uint32_t BK[TINY_LOCS];
#pragma unroll
            for (int k = 0; k < TINY_LOCS; k++) {
                P[k] = 0; M[k] = 0; DV[k] = 0; BK[k] = 0xFFFFFFFFu - (uint32_t)k; BM[k] = ~0ull;
                if (k < C) {
                    const uint64_t key = a.key[base + k];
                    P[k] = (uint32_t)(key >> 1);
                    sbits |= (uint32_t)(key & 1) << k;
                    M[k] = a.mask[base + k];
                    DV[k] = load_dv(a, base + k);
                    BK[k] = P[k] / (uint32_t)a.rule.bucket;
                }
            }
#pragma unroll
            for (int k = 0; k < TINY_LOCS; k++) {
                int rk = k;
#pragma unroll
                for (int j = k - 1; j >= 0; j--)
                    if (BK[j] == BK[k] && ((sbits >> j) & 1u) == ((sbits >> k) & 1u)) rk = j;
                repw |= (uint32_t)rk << (4 * k);
            }
        }
        ReadState st{DINF, DINF, -1, -1, -1};
        // a distance d <= limit at location k
        auto record = [&](int k, int d) {
            const int rk = (int)((repw >> (4 * k)) & 15u);
            uint32_t pk = 0;
            uint64_t bv = 0;
#pragma unroll
            for (int j = 0; j < TINY_LOCS; j++) {
                if (j == k) pk = P[j];
                if (j == rk) bv = BM[j];
            }
            const uint64_t nv0 = ((uint64_t)d << 32) | pk;
            const uint64_t nv = nv0 < bv ? nv0 : bv;
#pragma unroll
            for (int j = 0; j < TINY_LOCS; j++)
                if (j == rk) BM[j] = nv;
            state_update(st, rk, (int)(nv >> 32), (int64_t)(nv & 0xFFFFFFFFull), (int)((sbits >> k) & 1u));
        };
        const int round0 = round0_slots(L, a.rule.s, a.ps.ST);
        int t = 0, call = -1, need_k = -1;
        int req_kind = 0, req_lim = 0;   // 0: location need_k at req_lim; 1: undecided at Kfull; 2: remaining at req_lim
        bool looked = false, all_over = true, ended = false, unresolved = false;
        uint32_t prefix = 0, scored = 0;
        // the seed slots' statuses (2 bits each), loaded together up front
        uint64_t stw = 0;
#pragma unroll 4
        for (int i = 0; i < NS; i++) stw |= (uint64_t)a.pr[(r * NS + i) * a.ps.ST].status << (2 * i);
        for (int i = 0; i < NS; i++) {
            const int status = (int)((stw >> (2 * i)) & 3u);
            if (status == ST_NONE) { ended = true; break; }
            if (status == ST_N) continue;
            looked = true;
            if (status == ST_OVER) continue;
            all_over = false;
            prefix |= 1u << i;
            if (i < round0) t++;
            // the unscored location with the most seeds hitting; ties to the lower index
            int kb = -1, bv = 0;
            uint32_t dvb = 0;
#pragma unroll
            for (int k = 0; k < TINY_LOCS; k++) {
                const int v = (k < C && !((scored >> k) & 1u)) ? __builtin_popcount(M[k] & prefix) : 0;
                if (v > bv) { bv = v; kb = k; dvb = DV[k]; }
            }
            if (kb >= 0) {
                const int lim = d_limit(st, dmax, c);
                const int res = ed_answer((int)(dvb & 0xFFFFu), (int)(int16_t)(dvb >> 16), lim);
                if (res == -2) {
                    unresolved = true;
                    need_k = kb;
                    req_kind = (lane_class && (all_undecided || lim < Kfull)) ? 1 : 0;
                    req_lim = lim;
                    break;
                }
                scored |= 1u << kb;
                if (res >= 0) record(kb, res);
            }
            if (st.d_best < c && st.d_second < st.d_best + c) {
                call = SNAP_MULTIPLE;
                ended = true;
                break;
            }
            if (st.d_best < DINF && t >= st.d_best + c) {
                // score every remaining location: vote count descending, then index
                for (int lev = __builtin_popcount(prefix); lev >= 1 && !unresolved; lev--) {
#pragma unroll
                    for (int k = 0; k < TINY_LOCS; k++) {
                        if (!unresolved && k < C && !((scored >> k) & 1u) && __builtin_popcount(M[k] & prefix) == lev) {
                            const int lim = d_limit(st, dmax, c);
                            const int res = ed_answer((int)(DV[k] & 0xFFFFu), (int)(int16_t)(DV[k] >> 16), lim);
                            if (res == -2) {
                                unresolved = true;
                                need_k = k;
                                req_kind = 2;
                                req_lim = lim;
                            } else if (res >= 0) {
                                record(k, res);
                            }
                        }
                    }
                }
                ended = true;
                break;
            }
        }
        // all slots of this pass used and the read still has seeds to try
        if (!ended && !unresolved && NS < seeds_for_length(a.rule, L) && seed_offset(a.sh, a.rule.s, L, NS) >= 0)
            unresolved = true;
        if (unresolved) {
            if (need_k >= 0) {
                // the locations asked for (see k_replay), listed at the read's first slot
                const int code = lane_class ? req_lim : (REQ_WAVE | req_lim);
                const int lr = req_lim;
                uint32_t n = 0, wbits = 0;
                if (req_kind == 0) {
                    // the request_top best locations undecided at this limit, in selection
                    // order: votes over the seeds so far descending, then index (one for a
                    // read of the wave tile)
                    wbits = 1u << need_k;
                    const int top = lane_class ? a.request_top : 1;
                    for (int q = 1; q < top; q++) {
                        int kb2 = -1, bv2 = 0;
#pragma unroll
                        for (int k = 0; k < TINY_LOCS; k++) {
                            const int dc = (int)(DV[k] & 0xFFFFu), vl = (int)(int16_t)(DV[k] >> 16);
                            const bool open = k < C && !((scored >> k) & 1u) && !((wbits >> k) & 1u) && dc > vl &&
                                              vl < lr;
                            const int v = open ? __builtin_popcount(M[k] & prefix) : 0;
                            if (v > bv2) { bv2 = v; kb2 = k; }
                        }
                        if (kb2 < 0) break;
                        wbits |= 1u << kb2;
                    }
                }
#pragma unroll
                for (int k = 0; k < TINY_LOCS; k++) {
                    const int dc = (int)(DV[k] & 0xFFFFu), vl = (int)(int16_t)(DV[k] >> 16);
                    bool want = false;
                    if (req_kind == 1) want = !((scored >> k) & 1u) && dc > vl && vl < lr;
                    else if (req_kind == 2) want = !((scored >> k) & 1u) && (M[k] & prefix) && dc > vl && vl < lr;
                    if (k < C && want) wbits |= 1u << k;
                }
#pragma unroll
                for (int k = 0; k < TINY_LOCS; k++) {
                    bool want = (wbits >> k) & 1u;
                    if (want && a.alias) {
                        // not when the location's representative asks in this round
                        const int64_t j = (int64_t)a.alias[base + k] - base;
                        if (j != k && j >= 0 && j < TINY_LOCS && ((wbits >> j) & 1u)) want = false;
                    }
                    if (want) {
                        a.rq[base + k] = (int16_t)code;
                        a.req_area[base + n] = (uint32_t)(base + k);
                        n++;
                    }
                }
                a.reqcount[r] = n | ((!lane_class) ? REQ_WAVE_READ : 0u);
            }
            a.rflag[r] = need_k < 0 ? RF_PENDING : RF_REPLAY;
            continue;
        }
        if (call < 0) {
            if (st.d_best <= dmax && st.d_second >= st.d_best + c) call = SNAP_SINGLE;
            else if (st.d_best <= dmax || (looked && all_over)) call = SNAP_MULTIPLE;
            else call = SNAP_NOT_FOUND;
        }
        const bool has = st.d_best < DINF;
        a.rflag[r] = RF_DONE;
        a.pos[g] = has ? st.best_p : -1;
        a.strand[g] = (int8_t)(has ? st.best_s : -1);
        a.dist[g] = has ? st.d_best : -1;
        a.second[g] = st.d_second < DINF ? st.d_second : -1;
        a.call[g] = (int8_t)call;
    }
}

// Chunk read indices -> global read ids (the list a later pass works on).
__global__ void k_map_gid(const uint32_t *in, const int64_t *n_ptr, Pass ps, uint32_t *out) {
    const int64_t n = *n_ptr;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        out[i] = (uint32_t)gid(ps, in[i]);
}

// For each read in the chunk, the largest prefix [0, k) whose reserved region fits.
__global__ void k_fit(const int64_t *hoff, int64_t nr, int64_t cap, int64_t *out) {
    int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= nr) return;
    if (hoff[k + 1] > cap && hoff[k] <= cap) *out = k;
}

// ------------------------------------------------------------------ host

struct CastLen {
    const int32_t *len;
    int64_t n;
    __host__ __device__ int64_t operator()(int64_t i) const { return i < n ? (int64_t)len[i] : 0; }
};
struct CastU32 {
    const uint32_t *v;
    int64_t n;
    __host__ __device__ int64_t operator()(int64_t i) const { return i < n ? (int64_t)v[i] : 0; }
};

template <class F>
hipError_t scan_excl(void *tmp, size_t &tmp_bytes, F f, int64_t items, int64_t *out, hipStream_t st) {
    hipcub::CountingInputIterator<int64_t> ci(0);
    hipcub::TransformInputIterator<int64_t, F, hipcub::CountingInputIterator<int64_t>> it(ci, f);
    return hipcub::DeviceScan::ExclusiveSum(tmp, tmp_bytes, it, out, (int)items, st);
}

// Stream compaction of indices [0, items) by a predicate on the index.
struct FlagPred {
    const uint8_t *f;
    uint8_t v;
    __host__ __device__ bool operator()(uint32_t r) const { return f[r] == v; }
};

template <class P>
hipError_t select_idx(void *tmp, size_t &tmp_bytes, int64_t items, P pred, uint32_t *out, int64_t *nsel,
                      hipStream_t st) {
    hipcub::CountingInputIterator<uint32_t> ci(0);
    return hipcub::DeviceSelect::If(tmp, tmp_bytes, ci, out, nsel, (int)items, pred, st);
}

// Locations (below the chunk's count) of the lane tile, or of the wave tile: a lane
// per location when the read and its limit fit one lane's LDS arrays.
struct TilePred {
    const uint32_t *cread;
    const int32_t *len;
    Pass ps;
    Rule rule;
    const int64_t *ncand;
    int32_t lane_lmax, lane_kmax;
    bool want_long;
    const uint32_t *alias;      // the lane tile's first verification takes representatives only
    __device__ bool operator()(uint32_t k) const {
        if ((int64_t)k >= *ncand) return false;
        if (alias && !want_long && alias[k] != k) return false;
        const int L = len[gid(ps, cread[k])];
        const int K = min(dmax_for_length(rule, L) + rule.c - 1, ps.Kcap);
        return (L > lane_lmax || K > lane_kmax) == want_long;
    }
};

// Reads whose hit count is in (lo, hi].
struct HitRangePred {
    const uint32_t *hits;
    uint32_t lo, hi;
    __host__ __device__ bool operator()(uint32_t r) const { return hits[r] > lo && hits[r] <= hi; }
};

// Reads longer than len_max (or, with `longer` false, the others).
struct LenPred {
    const int32_t *len;
    int32_t len_max;
    bool longer;
    __device__ bool operator()(uint32_t r) const { return (len[r] > len_max) == longer; }
};

// Locations hit by one of the first seed slots (`bits`), below the chunk's location count.
struct FirstSeedsPred {
    const uint32_t *mask;
    const int64_t *ncand;
    uint32_t bits;
    const uint32_t *alias;      // representatives only, when set
    __host__ __device__ bool operator()(uint32_t k) const {
        return (int64_t)k < *ncand && (mask[k] & bits) != 0 && (!alias || alias[k] == k);
    }
};

// Locations (below the chunk's count) that are their own exact-duplicate representative.
struct RepPred {
    const uint32_t *alias;
    const int64_t *ncand;
    __host__ __device__ bool operator()(uint32_t k) const { return (int64_t)k < *ncand && alias[k] == k; }
};

// Entries r of a read list (or reads [0, items) when it is null) with lo < count[r] <= hi.
struct ListAt {
    const uint32_t *list;
    __host__ __device__ uint32_t operator()(uint32_t i) const { return list ? list[i] : i; }
};
struct CountRangePred {
    const uint32_t *count;
    uint32_t lo, hi;
    __host__ __device__ bool operator()(uint32_t r) const { return count[r] > lo && count[r] <= hi; }
};

hipError_t select_count_range(void *tmp, size_t &tmp_bytes, int64_t items, const uint32_t *list, const uint32_t *count,
                              uint32_t lo, uint32_t hi, uint32_t *out, int64_t *nsel, hipStream_t st) {
    hipcub::CountingInputIterator<uint32_t> ci(0);
    hipcub::TransformInputIterator<uint32_t, ListAt, hipcub::CountingInputIterator<uint32_t>> it(ci, ListAt{list});
    return hipcub::DeviceSelect::If(tmp, tmp_bytes, it, out, nsel, (int)items, CountRangePred{count, lo, hi}, st);
}

size_t select_tmp_bytes(int64_t items) {
    size_t a = 0, b = 0, c = 0;
    (void)select_idx(nullptr, a, items, FlagPred{nullptr, 0}, nullptr, nullptr, 0);
    (void)select_count_range(nullptr, b, items, nullptr, nullptr, 0, 0, nullptr, nullptr, 0);
    (void)select_idx(nullptr, c, items, FirstSeedsPred{nullptr, nullptr, 0}, nullptr, nullptr, 0);
    size_t e = 0;
    (void)select_idx(nullptr, e, items, TilePred{}, nullptr, nullptr, 0);
    c = std::max(c, e);
    size_t d = 0;
    (void)select_idx(nullptr, d, items, HitRangePred{nullptr, 0, 0}, nullptr, nullptr, 0);
    return std::max(std::max(a, d), std::max(b, c));
}

size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

struct Layout {
    // batch part
    size_t off_roff, off_rcode, off_rmask, off_pending;
    // chunk part, one per worker, offsets from the start of a worker's part
    size_t off_misc, off_probe, off_hits, off_hoff, off_ccount, off_coff, off_scan, off_sel, off_req, off_pool;
    size_t chunk_base, chunk_bytes;
    int workers;
    int64_t R;             // reads per chunk
    int64_t pool_slots;    // hit / location slots per chunk
    size_t total;
};

// pool arrays per slot: hit 8, location key 8 + mask 4 (by read), compacted key 8 +
// mask 4 + read 4, bucket minimum 8, capped distance 2, verified limit 2, scored flag 1,
// verify routing lists / requests 4 + 4, requested limit 2
constexpr size_t POOL_SLOT_BYTES = 8 + 8 + 4 + 8 + 4 + 4 + 8 + 2 + 2 + 1 + 4 + 4 + 2 + 4;
constexpr int POOL_ARRAYS = 14;

size_t scan_tmp_bytes(int64_t items) {
    size_t b = 0;
    CastLen f{nullptr, 0};
    (void)scan_excl(nullptr, b, f, items, nullptr, 0);
    return b;
}

Layout make_layout(int64_t n, int64_t B, int NS, int hmax, int64_t R, int64_t pool_slots, int workers = 1) {
    Layout l{};
    size_t o = 0;
    l.off_roff = o; o = align256(o + sizeof(int64_t) * (size_t)(n + 1));
    const int64_t nblk = (B + STREAM_GUARD + 31) / 32 + 2;
    l.off_rcode = o; o = align256(o + sizeof(uint32_t) * 2 * (size_t)nblk);
    l.off_rmask = o; o = align256(o + sizeof(uint32_t) * (size_t)nblk);
    l.off_pending = o; o = align256(o + 2 * sizeof(uint32_t) * (size_t)n);
    l.chunk_base = o;
    l.R = R;
    l.workers = workers;
    o = 0;
    l.off_misc = o; o = align256(o + 256);
    l.off_probe = o; o = align256(o + sizeof(ProbeRec) * (size_t)R * NS);
    l.off_hits = o; o = align256(o + sizeof(uint32_t) * (size_t)R);
    l.off_hoff = o; o = align256(o + sizeof(int64_t) * (size_t)(R + 1));
    l.off_ccount = o; o = align256(o + sizeof(uint32_t) * (size_t)R);
    l.off_coff = o; o = align256(o + sizeof(int64_t) * (size_t)(R + 1));
    l.off_scan = o; o = align256(o + std::max(scan_tmp_bytes(R + 1), scan_tmp_bytes(n + 1)));
    // read flags; replay and next-pass lists, request counts, light-replay list; request offsets
    l.off_req = o; o = align256(o + (size_t)R); o = align256(o + 4 * sizeof(uint32_t) * (size_t)R);
    o = align256(o + sizeof(int64_t) * (size_t)(R + 1));
    // lead location and first-verification limit per read
    o = align256(o + sizeof(uint32_t) * (size_t)R);
    o = align256(o + sizeof(int16_t) * (size_t)R);
    const int64_t minslots = (int64_t)NS * hmax;
    if (pool_slots < minslots) pool_slots = minslots;
    l.pool_slots = pool_slots;
    l.off_sel = o; o = align256(o + select_tmp_bytes(std::max<int64_t>(R, pool_slots) + 1));
    l.off_pool = o; o = align256(o + POOL_SLOT_BYTES * (size_t)pool_slots + POOL_ARRAYS * 256);
    l.chunk_bytes = o;
    l.total = l.chunk_base + (size_t)workers * l.chunk_bytes;
    return l;
}

bool valid_params(const snap_params *p) {
    return p && p->n_min >= 1 && p->n_cap >= p->n_min && p->n_cap <= MAX_SEEDS && p->bp_per_seed >= 1 &&
           p->conf_c >= 1 && p->max_hits >= 1 && p->max_hits <= MAX_HITS_LIMIT && p->d_max_pct >= 0 &&
           p->d_max_pct <= 100 && p->bucket >= 1;
}

Rule make_rule(const snap_index *ix, int32_t d_max, const snap_params *p) {
    return Rule{ix->d.s, p->n_min, p->n_cap, p->bp_per_seed, p->conf_c, p->max_hits, d_max, p->d_max_pct, p->bucket};
}

#define HIP_OK(x) do { if ((x) != hipSuccess) return SNAP_EDEVICE; } while (0)

// Optional per-kernel device time: an event pair recorded on the launch stream
// around every kernel while profiling is on.
struct ProfRec {
    const char *name;
    hipEvent_t a, b;
};
std::mutex g_prof_mu;
std::vector<ProfRec> g_prof;
bool g_prof_on = false;
snap_counters g_ctr;

template <class Launch>
void timed(const char *name, hipStream_t st, Launch launch) {
    if (!g_prof_on) { launch(); return; }
    ProfRec r{name, nullptr, nullptr};
    (void)hipEventCreate(&r.a);
    (void)hipEventCreate(&r.b);
    (void)hipEventRecord(r.a, st);
    launch();
    (void)hipEventRecord(r.b, st);
    std::lock_guard<std::mutex> g(g_prof_mu);
    g_prof.push_back(r);
}

// Output-invariant schedule of the passes: the first pass probes pass1_seeds seed
// slots and verifies with limit pass1_limit; reads it cannot settle go to a
// complete second pass.
std::mutex g_tune_mu;
snap_tuning g_tune = {5, 6, 6, 0, 1, 0, 0, 0, 0, 0};   // stage-1 seeds and first limit, final first limit, lane-tile
                                           // read bound, exact-request rounds, first-verification seeds, ...


constexpr int KCAP_NONE = 1 << 20;
constexpr int MAX_WORKERS = 4;   // chunk workers of one call (host thread + stream each)

// Streams (default priority, non-blocking) kept per device for the second worker of
// snap_align calls; a call leases one with an event and returns both when it ends.
std::mutex g_stream_mu;
std::vector<std::pair<int, std::pair<hipStream_t, hipEvent_t>>> g_stream_free;

struct StreamLease {
    int dev = -1;
    hipStream_t s = nullptr;
    hipEvent_t ev = nullptr;
    explicit StreamLease(int device) : dev(device) {
        if (dev < 0) return;
        {
            std::lock_guard<std::mutex> g(g_stream_mu);
            for (size_t i = 0; i < g_stream_free.size(); i++) {
                if (g_stream_free[i].first == dev) {
                    s = g_stream_free[i].second.first;
                    ev = g_stream_free[i].second.second;
                    g_stream_free.erase(g_stream_free.begin() + (long)i);
                    return;
                }
            }
        }
        if (hipStreamCreateWithFlags(&s, hipStreamNonBlocking) != hipSuccess) { s = nullptr; return; }
        if (hipEventCreateWithFlags(&ev, hipEventDisableTiming) != hipSuccess) {
            (void)hipStreamDestroy(s);
            s = nullptr;
        }
    }
    ~StreamLease() {
        if (dev < 0 || !s) return;
        (void)hipStreamSynchronize(s);
        std::lock_guard<std::mutex> g(g_stream_mu);
        g_stream_free.push_back({dev, {s, ev}});
    }
    StreamLease(const StreamLease &) = delete;
    StreamLease &operator=(const StreamLease &) = delete;
};

}  // namespace

extern "C" snap_params snap_default_params(void) {
    snap_params p;
    p.n_min = 10; p.n_cap = 32; p.bp_per_seed = 100; p.conf_c = 2; p.max_hits = 300; p.d_max_pct = 0; p.bucket = 32;
    return p;
}

extern "C" int32_t snap_max_limit(void) { return VERIFY_KMAX; }

extern "C" int snap_set_tuning(const snap_tuning *t) {
    if (!t || t->pass1_seeds < 0 || t->pass1_limit < 0 || t->final_limit < 0 || t->lane_max_len < 0 || t->exact_rounds < 0 || t->verify_seeds < 0 || t->chunk_reads < 0 || t->workers < 0 || t->request_top < 0 || t->request_top > REQUEST_TOP_MAX || t->pass1_max_len < 0) return SNAP_EINVAL;
    std::lock_guard<std::mutex> g(g_tune_mu);
    g_tune = *t;
    return SNAP_OK;
}

extern "C" int snap_get_tuning(snap_tuning *t) {
    if (!t) return SNAP_EINVAL;
    std::lock_guard<std::mutex> g(g_tune_mu);
    *t = g_tune;
    return SNAP_OK;
}

namespace {

// The workspace a batch is sized for: one chunk of up to CHUNK_READS reads with 24 hit
// slots a read (a chunk shrinks to fit a smaller workspace; outputs do not change).
size_t workspace_bytes_for(const Rule &rule, int ST, int64_t n_reads, int64_t total_bases, int32_t max_len) {
    const int NS = seeds_for_length(rule, max_len);
    const int64_t R = std::max<int64_t>(1, std::min<int64_t>(n_reads, CHUNK_READS));
    return make_layout(n_reads, total_bases, NS * ST, rule.hmax, R, R * 24).total;
}

}  // namespace

extern "C" size_t snap_align_workspace_bytes(const snap_index *ix, int64_t n_reads, int64_t total_bases,
                                             int32_t max_len, int32_t d_max, const snap_params *p) {
    if (!ix || n_reads < 0 || total_bases < 0 || max_len < 0 || max_len > VERIFY_LMAX || d_max < 0 ||
        !valid_params(p))
        return 0;
    return workspace_bytes_for(make_rule(ix, d_max, p), std::max(1, ix->d.stride), n_reads, total_bases, max_len);
}

namespace {

int align_impl(const snap_index *ix, const uint8_t *reads, const int32_t *lengths, int64_t n_reads, int32_t d_max,
               const snap_params *p, int64_t *pos, int8_t *strand, int32_t *dist, int32_t *second, int8_t *call,
               void *workspace, size_t ws_bytes, void *stream, bool batched, const snap_tuning *tuning,
               bool fixed_scratch = false) {
    if (!ix || n_reads < 0 || d_max < 0 || !valid_params(p)) return SNAP_EINVAL;
    if (n_reads == 0) return SNAP_OK;
    if (!reads || !lengths || !pos || !strand || !dist || !second || !call || !workspace) return SNAP_EINVAL;
    if (((uintptr_t)workspace & 255) != 0 || n_reads >= (1ll << 32)) return SNAP_EINVAL;
    hipStream_t st = (hipStream_t)stream;
    const Rule rule = make_rule(ix, d_max, p);
    const Shifts sh = make_shifts(ix->d.s);
    snap_tuning tune;
    if (tuning) {
        tune = *tuning;
    } else {
        std::lock_guard<std::mutex> g(g_tune_mu);
        tune = g_tune;
    }
    if (tune.pass1_seeds < 0 || tune.pass1_limit < 0 || tune.final_limit < 0 || tune.lane_max_len < 0 || tune.exact_rounds < 0 || tune.verify_seeds < 0 || tune.chunk_reads < 0 || tune.workers < 0 || tune.request_top < 0 || tune.request_top > REQUEST_TOP_MAX || tune.pass1_max_len < 0) return SNAP_EINVAL;
    const int request_top = tune.request_top > 0 ? tune.request_top : REQUEST_TOP_DEFAULT;
    const int lane_lmax = tune.lane_max_len > 0 ? std::min(tune.lane_max_len, LANE_LMAX) : LANE_LMAX;
    const int exact_rounds = tune.exact_rounds;
    const int verify_seeds = tune.verify_seeds;
    int dev = 0, lds_max = 0;
    HIP_OK(hipGetDevice(&dev));
    HIP_OK(hipDeviceGetAttribute(&lds_max, hipDeviceAttributeMaxSharedMemoryPerBlock, dev));
    // hits that one workgroup can sort in LDS
    uint32_t cape = 64;
    while ((size_t)cape * 2 * 8 + 1024 <= (size_t)lds_max) cape *= 2;

    // read offsets, total bases and longest read (one wait for two scalars)
    const int too_small = fixed_scratch ? SNAP_ETOOBIG : SNAP_ENOMEM;
    Layout l0 = make_layout(n_reads, 0, 1, 1, 1, 0);
    if (ws_bytes < l0.chunk_base + 4096) return too_small;
    char *ws = (char *)workspace;
    int64_t *roff = (int64_t *)(ws + l0.off_roff);
    // until the layout is known (it needs the total), two scalars live at the tail
    uint64_t *tmp_scalars = (uint64_t *)(ws + ((ws_bytes - 64) & ~(size_t)255));
    {
        size_t tb = scan_tmp_bytes(n_reads + 1);
        size_t scan_at = align256(l0.off_roff + sizeof(int64_t) * (size_t)(n_reads + 1));
        if (scan_at + tb > ((ws_bytes - 64) & ~(size_t)255)) return too_small;
        CastLen f{lengths, n_reads};
        HIP_OK(scan_excl(ws + scan_at, tb, f, n_reads + 1, roff, st));
        hipLaunchKernelGGL(k_fill_u32, dim3(1), dim3(64), 0, st, (uint32_t *)tmp_scalars, 2, 0u);
        hipLaunchKernelGGL(k_maxlen, dim3(256), dim3(256), 0, st, lengths, n_reads, (uint32_t *)tmp_scalars);
        HIP_OK(hipMemcpyAsync(tmp_scalars + 1, roff + n_reads, 8, hipMemcpyDeviceToDevice, st));
    }
    uint64_t host_sc[2];
    HIP_OK(hipMemcpyAsync(host_sc, tmp_scalars, 16, hipMemcpyDeviceToHost, st));
    HIP_OK(hipStreamSynchronize(st));
    const uint32_t maxlen_u = (uint32_t)host_sc[0];
    const int64_t B = (int64_t)host_sc[1];
    if (maxlen_u & 0x80000000u) return SNAP_EINVAL;
    const int maxL = (int)maxlen_u;
    const int NS = std::max(1, seeds_for_length(rule, maxL));
    const int ST = std::max(1, ix->d.stride);   // probe records per seed slot
    const int Kmax = dmax_for_length(rule, maxL) + rule.c - 1;
    if (Kmax > VERIFY_KMAX || maxL > VERIFY_LMAX || NS * ST > 64) return SNAP_EINVAL;
    // the fixed scratch takes exactly the batches snap_align_workspace_bytes sizes within it
    if (fixed_scratch && workspace_bytes_for(rule, ST, n_reads, B, maxL) > ws_bytes) return SNAP_ETOOBIG;

    // chunk size and pool from the workspace
    int64_t R = std::min<int64_t>(n_reads, tune.chunk_reads > 0 ? tune.chunk_reads : CHUNK_READS);
    Layout l = make_layout(n_reads, B, NS * ST, rule.hmax, R, 0);
    while (l.total > ws_bytes && R > 1) {
        R = std::max<int64_t>(1, R / 2);
        l = make_layout(n_reads, B, NS * ST, rule.hmax, R, 0);
    }
    if (l.total > ws_bytes) return SNAP_ENOMEM;
    {
        int64_t extra = (int64_t)((ws_bytes - l.total) / POOL_SLOT_BYTES);
        l = make_layout(n_reads, B, NS * ST, rule.hmax, R, l.pool_slots + extra);
        while (l.total > ws_bytes) {
            const int64_t over = (int64_t)((l.total - ws_bytes) / POOL_SLOT_BYTES) + 64;
            l = make_layout(n_reads, B, NS * ST, rule.hmax, R, l.pool_slots - over);
        }
    }
    // two workers (a host thread and a stream each, and a chunk part of the workspace
    // each) when the batch spans several chunks and the workspace holds two parts
    // with room for the hits of a typical chunk: one worker's host waits and small
    // kernels then overlap the other's work
    int workers = 1;
    // the fixed-scratch form runs one worker: the others' streams come from a pool that
    // may have to create them
    const int max_workers = fixed_scratch ? 1 : std::min<int64_t>(tune.workers > 0 ? tune.workers : 2,
                                                                  (n_reads + R - 1) / R);
    for (int w = std::min(max_workers, MAX_WORKERS); w >= 2; w--) {
        Layout lw = make_layout(n_reads, B, NS * ST, rule.hmax, R, 0, w);
        if (lw.total > ws_bytes) continue;
        const int64_t extra = (int64_t)((ws_bytes - lw.total) / ((size_t)w * POOL_SLOT_BYTES));
        lw = make_layout(n_reads, B, NS * ST, rule.hmax, R, lw.pool_slots + extra, w);
        while (lw.total > ws_bytes) {
            const int64_t over = (int64_t)((lw.total - ws_bytes) / ((size_t)w * POOL_SLOT_BYTES)) + 64;
            lw = make_layout(n_reads, B, NS * ST, rule.hmax, R, lw.pool_slots - over, w);
        }
        if (lw.pool_slots >= 16 * R) {
            l = lw;
            workers = w;
            break;
        }
    }
    uint32_t *rcode = (uint32_t *)(ws + l.off_rcode);
    uint32_t *rmask = (uint32_t *)(ws + l.off_rmask);
    uint32_t *pending_out = nullptr;
    int64_t pend_count = 0;
    std::mutex pend_mu;
    uint32_t *pending = (uint32_t *)(ws + l.off_pending);
    const size_t sel_tb_all = select_tmp_bytes(std::max<int64_t>(R, l.pool_slots) + 1);
    const int64_t PS = l.pool_slots;
    struct Worker {
        hipStream_t st;
        int64_t *misc;
        ProbeRec *probe;
        uint32_t *hits;
        int64_t *hoff;
        uint32_t *ccount;
        int64_t *coff;
        void *scan_tmp, *sel_tmp;
        uint8_t *rflag;
        uint32_t *replay_list, *pend_local, *reqcount, *light_list;
        int64_t *req_off;
        uint64_t *hk, *key_res;
        uint32_t *mask_res;
        uint64_t *key_c;
        uint32_t *mask_c, *cread;
        uint64_t *bmin;
        uint16_t *dcap;
        int16_t *vlim;
        uint8_t *scored;
        uint32_t *short_list, *long_list;
        int16_t *rq;
        uint32_t *alias;
        uint32_t *lead;
        int16_t *rlim;
    };
    Worker wk[MAX_WORKERS];
    for (int w = 0; w < workers; w++) {
        char *cb = ws + l.chunk_base + (size_t)w * l.chunk_bytes;
        Worker &W = wk[w];
        W.misc = (int64_t *)(cb + l.off_misc);
        W.probe = (ProbeRec *)(cb + l.off_probe);
        W.hits = (uint32_t *)(cb + l.off_hits);
        W.hoff = (int64_t *)(cb + l.off_hoff);
        W.ccount = (uint32_t *)(cb + l.off_ccount);
        W.coff = (int64_t *)(cb + l.off_coff);
        W.scan_tmp = cb + l.off_scan;
        W.sel_tmp = cb + l.off_sel;
        W.rflag = (uint8_t *)(cb + l.off_req);
        W.replay_list = (uint32_t *)(cb + align256(l.off_req + (size_t)R));
        W.pend_local = W.replay_list + R;
        W.reqcount = W.pend_local + R;
        W.light_list = W.reqcount + R;
        W.req_off = (int64_t *)(cb + align256(l.off_req + (size_t)R) + align256(4 * sizeof(uint32_t) * (size_t)R));
        W.lead = (uint32_t *)((char *)W.req_off + align256(sizeof(int64_t) * (size_t)(R + 1)));
        W.rlim = (int16_t *)((char *)W.lead + align256(sizeof(uint32_t) * (size_t)R));
        char *pool = cb + l.off_pool;
        auto carve = [&](size_t bytes) { char *q = pool; pool += align256(bytes); return (void *)q; };
        W.hk = (uint64_t *)carve(8 * (size_t)PS);
        W.key_res = (uint64_t *)carve(8 * (size_t)PS);
        W.mask_res = (uint32_t *)carve(4 * (size_t)PS);
        W.key_c = (uint64_t *)carve(8 * (size_t)PS);
        W.mask_c = (uint32_t *)carve(4 * (size_t)PS);
        W.cread = (uint32_t *)carve(4 * (size_t)PS);
        W.bmin = (uint64_t *)carve(8 * (size_t)PS);
        W.dcap = (uint16_t *)carve(2 * (size_t)PS);
        W.vlim = (int16_t *)carve(2 * (size_t)PS);
        W.scored = (uint8_t *)carve((size_t)PS);
        W.short_list = (uint32_t *)carve(4 * (size_t)PS);
        W.long_list = (uint32_t *)carve(4 * (size_t)PS);
        W.rq = (int16_t *)carve(2 * (size_t)PS);
        W.alias = (uint32_t *)carve(4 * (size_t)PS);
        if ((size_t)(pool - ws) > ws_bytes) return SNAP_ENOMEM;
    }
    int64_t steal_waves = 2048;
    int cus = 256;
    {
        int c = 0;
        if (hipDeviceGetAttribute(&c, hipDeviceAttributeMultiprocessorCount, dev) == hipSuccess && c > 0) cus = c;
        steal_waves = (int64_t)cus * 16;
    }
    // the other workers' streams, from a pool of the device's streams; they start once
    // the read stream is packed on the caller's stream
    wk[0].st = st;
    if (g_prof_on) {
        std::lock_guard<std::mutex> g(g_prof_mu);
        g_ctr.workers = std::max<int64_t>(g_ctr.workers, workers);
    }
    std::vector<std::unique_ptr<StreamLease>> leases;
    for (int w = 1; w < workers; w++) {
        leases.emplace_back(new StreamLease(dev));
        if (!leases.back()->s) return SNAP_EDEVICE;
        wk[w].st = leases.back()->s;
    }

    for (int w = 0; w < workers; w++) hipLaunchKernelGGL(k_fill_u32, dim3(1), dim3(64), 0, st, (uint32_t *)wk[w].misc, 64, 0u);
    {
        const int64_t nblk = (B + STREAM_GUARD + 31) / 32 + 2;
        const int vec = ((uintptr_t)reads & 15) == 0 ? 1 : 0;
        timed("pack", st, [&] { hipLaunchKernelGGL(k_pack, dim3((unsigned)((nblk + 255) / 256)), dim3(256), 0, st, reads, B, rcode, rmask, nblk, vec); });
    }
    for (int w = 1; w < workers; w++) {
        HIP_OK(hipEventRecord(leases[w - 1]->ev, st));
        HIP_OK(hipStreamWaitEvent(wk[w].st, leases[w - 1]->ev, 0));
    }
    // one pass over a list of reads (all reads, or the ones an earlier pass left); `first`:
    // a pass of the first stage (its reads counted as the batch's, else as reads a first
    // pass left to a later one)
    auto run_pass = [&](const uint32_t *ridx, int64_t list_len, int NSp, int Kcap, int final_pass, bool first) -> int {
        const int Kp = std::min(Kmax, Kcap);
        // lane-per-location tile: reads up to LANE_LMAX bases with limits up to LANE_KMAX
        const int lane_L = std::min(maxL, lane_lmax), lane_K = std::min(Kp, LANE_KMAX);
        // every read of the batch is in the lane class exactly when the replay puts it
        // there: it classifies a read by its full limit d_max(L) + c - 1, not by the
        // pass's cap, so the test here uses the uncapped Kmax too (a read whose full
        // limit is above LANE_KMAX asks for the wave tile even in a capped pass)
        const bool all_lane = !batched && maxL <= lane_lmax && Kmax <= LANE_KMAX;
        const int RW = (std::max(lane_L, 1) + 15) / 16 + 1;
        const int TW = (std::max(lane_L, 1) + lane_K + 15) / 16 + 1;
        const int kmax_t = lane_K <= 7 ? 7 : (lane_K <= 15 ? 15 : (lane_K <= 31 ? 31 : 63));
        // furthest rows in LDS only above limit 7 (registers below)
        const size_t lds = (size_t)64 * 4 * (RW + TW) + (kmax_t > 7 ? (size_t)64 * 2 * (2 * kmax_t + 3) : 0);
        // wave-per-location tile: any read, any limit (requests go up to the full limit)
        const int Kw = Kmax;
        const int RWL = (std::max(maxL, 1) + 15) / 16 + 1;
        const int TWL = (std::max(maxL, 1) + Kw + 15) / 16 + 1;
        const size_t lds_wave = (size_t)4 * (RWL + TWL) + (size_t)4 * (2 * Kw + 3);
        if (lds > (size_t)lds_max || (!all_lane && lds_wave > (size_t)lds_max)) return SNAP_EINVAL;
        // workers take ranges of R reads of the list in turn; a range whose hits do not
        // fit the pool is done in several chunks
        std::atomic<int64_t> next_range{0};
        auto work = [&](Worker &W) -> int {
        hipStream_t st = W.st;
        int64_t *misc = W.misc;
        ProbeRec *probe = W.probe;
        uint32_t *hits = W.hits;
        int64_t *hoff = W.hoff;
        uint32_t *ccount = W.ccount;
        int64_t *coff = W.coff;
        void *scan_tmp = W.scan_tmp, *sel_tmp = W.sel_tmp;
        size_t sel_tb = sel_tb_all;
        uint8_t *rflag = W.rflag;
        uint32_t *replay_list = W.replay_list, *pend_local = W.pend_local, *reqcount = W.reqcount,
                 *light_list = W.light_list;
        uint32_t *heavy_list = pend_local;   // free while a chunk replays (the next-pass list is made after)
        int64_t *req_off = W.req_off;
        uint64_t *hk = W.hk, *key_res = W.key_res;
        uint32_t *mask_res = W.mask_res;
        uint64_t *key_c = W.key_c;
        uint32_t *mask_c = W.mask_c, *cread = W.cread;
        uint64_t *bmin = W.bmin;
        uint16_t *dcap = W.dcap;
        int16_t *vlim = W.vlim;
        uint8_t *scored = W.scored;
        uint32_t *short_list = W.short_list, *long_list = W.long_list;
        int16_t *rq = W.rq;
        // representatives of exact-duplicate classes, when the index has classes
        uint32_t *alias = (ix->d.rep != nullptr && ix->d.dup_w > 0) ? W.alias : nullptr;
        // lead verification: each read's first call at its full limit, then the first
        // verification of its other locations at the limit that call leaves
        const bool lead_mode = all_lane && !batched && !alias && !(verify_seeds > 0 && verify_seeds < NSp);
        uint32_t *lead = W.lead;
        int16_t *rlim = W.rlim;
        unsigned long long *nalias = (unsigned long long *)(misc + 12);
        unsigned long long *steps_sum = (unsigned long long *)(misc + 6);
        unsigned long long *steps_first = (unsigned long long *)(misc + 7);
        int64_t *sel_n = misc + 20;   // selected counts: [2] reads to replay, [3] reads for the next pass, ...
        unsigned long long *route_cnt = (unsigned long long *)(misc + 8);   // two counters
        unsigned long long *steal_next = (unsigned long long *)(misc + 10);  // two cursors
        // per-location step counts reuse the hit array, dead once locations are compacted
        uint32_t *steps = g_prof_on ? (uint32_t *)hk : nullptr;
        for (;;) {
          const int64_t a0 = next_range.fetch_add(R);
          if (a0 >= list_len) break;
          const int64_t b0 = std::min<int64_t>(a0 + R, list_len);
          for (int64_t r0 = a0; r0 < b0;) {
            int64_t nr = std::min<int64_t>(R, b0 - r0);
            Pass ps{ridx, r0, nr, NSp, Kcap, final_pass, ST};
            ProbeArgs pa{ix->d, rcode, rmask, roff, lengths, ps, rule, sh, probe, hits};
            const int64_t pthreads = nr * NSp * ST;   // one lane per (read, seed slot, seed of the slot)
            hipLaunchKernelGGL(k_fill_u32, dim3((unsigned)((nr + 255) / 256)), dim3(256), 0, st, hits, nr, 0u);
            timed("probe", st, [&] { hipLaunchKernelGGL(k_probe, dim3((unsigned)((pthreads + 255) / 256)), dim3(256), 0, st, pa); });
            size_t tb = scan_tmp_bytes(nr + 1);
            HIP_OK(scan_excl(scan_tmp, tb, CastU32{hits, nr}, nr + 1, hoff, st));
            // total hits, the largest per-read count and the reads of the two sorting
            // tiers above 64 hits (one wait per chunk)
            hipLaunchKernelGGL(k_fill_u32, dim3(1), dim3(64), 0, st, (uint32_t *)misc, 2, 0u);
            hipLaunchKernelGGL(k_maxlen, dim3(256), dim3(256), 0, st, (const int32_t *)hits, nr, (uint32_t *)misc);
            HIP_OK(hipMemcpyAsync(misc + 1, hoff + nr, 8, hipMemcpyDeviceToDevice, st));
            HIP_OK(select_idx(sel_tmp, sel_tb, nr, HitRangePred{hits, 64u, 512u}, replay_list, sel_n + 6, st));
            HIP_OK(select_idx(sel_tmp, sel_tb, nr, HitRangePred{hits, 512u, 0xFFFFFFFFu}, pend_local, sel_n + 7, st));
            HIP_OK(select_idx(sel_tmp, sel_tb, nr, HitRangePred{hits, 8u, 64u}, light_list, sel_n + 9, st));
            int64_t sc[2], ntier[3];
            HIP_OK(hipMemcpyAsync(sc, misc, 16, hipMemcpyDeviceToHost, st));
            HIP_OK(hipMemcpyAsync(ntier, sel_n + 6, 16, hipMemcpyDeviceToHost, st));
            HIP_OK(hipMemcpyAsync(ntier + 2, sel_n + 9, 8, hipMemcpyDeviceToHost, st));
            HIP_OK(hipStreamSynchronize(st));
            const uint32_t maxH = (uint32_t)(sc[0] & 0x7FFFFFFF);
            int64_t total = sc[1];
            if (total > PS) {
                // keep the longest prefix of reads whose hits fit; the rest go to the next chunk
                hipLaunchKernelGGL(k_fit, dim3((unsigned)((nr + 255) / 256)), dim3(256), 0, st, hoff, nr, PS, misc + 2);
                int64_t fit = 0;
                HIP_OK(hipMemcpyAsync(&fit, misc + 2, 8, hipMemcpyDeviceToHost, st));
                HIP_OK(hipStreamSynchronize(st));
                if (fit <= 0) return SNAP_ENOMEM;
                nr = fit;
                ps.nr = nr;
                HIP_OK(hipMemcpyAsync(&total, hoff + nr, 8, hipMemcpyDeviceToHost, st));
                HIP_OK(hipStreamSynchronize(st));
            }
            if (total > 0) {
                GatherArgs ga{probe, ix->d.positions, ix->d.G, ix->d.s, lengths, ps, hoff, hk};
                const int64_t rpb = 4 * (64 / (NSp * ST));   // reads per block step (4 waves)
                const unsigned gb = (unsigned)std::max<int64_t>(1, std::min<int64_t>((nr + rpb - 1) / rpb, 8192));
                timed("gather", st, [&] { hipLaunchKernelGGL(k_gather, dim3(gb), dim3(256), 0, st, ga); });
            }
            DedupeArgs da{hk, hits, hoff, nr, key_res, mask_res, ccount, nullptr, nullptr};
            {
                // up to 8 hits: a lane per read; up to 64: a wave per read, from its own list
                const unsigned tb = (unsigned)std::max<int64_t>(1, std::min<int64_t>((nr + 255) / 256, (int64_t)cus * 32));
                timed("dedupe_tiny", st, [&] { hipLaunchKernelGGL(k_dedupe_tiny, dim3(tb), dim3(256), 0, st, da); });
                if (ntier[2] > 0) {
                    DedupeArgs dl = da;
                    dl.rlist = light_list;
                    dl.rlist_n = sel_n + 9;
                    const unsigned lb = (unsigned)std::min<int64_t>((ntier[2] + 3) / 4, 8192);
                    timed("dedupe_light", st, [&] { hipLaunchKernelGGL(k_dedupe_light, dim3(lb), dim3(256), 0, st, dl); });
                }
            }
            // reads beyond 64 hits sort from their own lists (a chunk that shrank to fit the
            // pool keeps the lists of the whole chunk: the entries past nr are skipped)
            DedupeArgs dm = da, dh = da;
            dm.rlist = replay_list;
            dm.rlist_n = sel_n + 6;
            dh.rlist = pend_local;
            dh.rlist_n = sel_n + 7;
            if (ntier[0] > 0) {
                // 64 < H <= 512: one wave per read
                const unsigned mb = (unsigned)std::min<int64_t>(ntier[0], 8192);
                timed("dedupe_medium", st, [&] { hipLaunchKernelGGL((k_dedupe_heavy<true, 64>), dim3(mb), dim3(64), (size_t)512 * 8, st, dm, key_c, 64u, 512u); });
            }
            if (ntier[1] > 0) {
                // up to cape: a workgroup; beyond: global scratch
                const unsigned hb = (unsigned)std::min<int64_t>(ntier[1], 2048);
                uint32_t N = 1;
                while (N < std::min(maxH, cape)) N <<= 1;
                timed("dedupe_heavy", st, [&] { hipLaunchKernelGGL((k_dedupe_heavy<true, 256>), dim3(hb), dim3(256), (size_t)N * 8, st, dh, key_c, 512u, cape); });
                if (maxH > cape)
                    timed("dedupe_huge", st, [&] { hipLaunchKernelGGL((k_dedupe_heavy<false, 256>), dim3(hb), dim3(256), 0, st, dh, key_c, cape, 0xFFFFFFFFu); });
            }
            tb = scan_tmp_bytes(nr + 1);
            HIP_OK(scan_excl(scan_tmp, tb, CastU32{ccount, nr}, nr + 1, coff, st));
            if (total > 0) {
                const unsigned cb = (unsigned)std::max<int64_t>(1, std::min<int64_t>((nr + 255) / 256, 8192));
                timed("compact", st, [&] { hipLaunchKernelGGL(k_compact, dim3(cb), dim3(256), 0, st, hoff, coff, nr,
                                   key_res, mask_res, key_c, mask_c, cread, lead_mode ? lead : nullptr); });
            }
            if (total > 0) {
                const int64_t *ncand = coff + nr;
                const uint32_t *slist = nullptr;
                const int64_t *nshort = ncand;
                if (alias) {
                    hipLaunchKernelGGL(k_fill_u32, dim3(1), dim3(64), 0, st, (uint32_t *)nalias, 2, 0u);
                    timed("dup_alias", st, [&] { hipLaunchKernelGGL(k_dup_alias, dim3((unsigned)((total + 255) / 256)), dim3(256), 0, st, ix->d, key_c, cread, coff, lengths, ps, rule, ncand, alias, dcap, vlim, steps, g_prof_on ? nalias : nullptr); });
                }
                if (!all_lane) {
                    int64_t *rc64 = (int64_t *)route_cnt;
                    HIP_OK(select_idx(sel_tmp, sel_tb, total, TilePred{cread, lengths, ps, rule, ncand, lane_lmax, LANE_KMAX, false, alias},
                                      short_list, rc64, st));
                    HIP_OK(select_idx(sel_tmp, sel_tb, total, TilePred{cread, lengths, ps, rule, ncand, lane_lmax, LANE_KMAX, true, nullptr},
                                      long_list, rc64 + 1, st));
                    slist = short_list;
                    nshort = rc64;
                } else if (alias && !(verify_seeds > 0 && verify_seeds < NSp)) {
                    // the first verification takes the representatives only
                    HIP_OK(select_idx(sel_tmp, sel_tb, total, RepPred{alias, ncand}, short_list, sel_n + 5, st));
                    slist = short_list;
                    nshort = sel_n + 5;
                }
                VerifyArgs va{ix->d.gcode, ix->d.gmask, ix->d.G, rcode, rmask, roff, lengths, ps, key_c, cread, ncand,
                              rule, RW, TW, dcap, vlim, steps, slist, nshort};
                // long locations are verified on request, with the exact limit
                if (!all_lane) {
                    const int64_t *nlong = (const int64_t *)(route_cnt + 1);
                    timed("mark", st, [&] { hipLaunchKernelGGL(k_mark_unverified, dim3((unsigned)((total + 255) / 256)), dim3(256), 0, st, long_list, nlong, dcap, vlim, steps); });
                }
                if (batched) {
                    // one persistent work-stealing launch over the short locations
                    hipLaunchKernelGGL(k_fill_u32, dim3(1), dim3(64), 0, st, (uint32_t *)steal_next, 4, 0u);
                    const int nwaves = (int)std::min<int64_t>(std::max<int64_t>((total + 63) / 64, 1), steal_waves);
                    StealArgs sa{va, steal_next, nwaves};
                    const size_t lds_s = lds;
                    timed("verify_steal", st, [&] {
                        if (kmax_t == 7)
                            hipLaunchKernelGGL(k_verify_steal<7>, dim3(nwaves), dim3(64), lds_s, st, sa);
                        else if (kmax_t == 15)
                            hipLaunchKernelGGL(k_verify_steal<15>, dim3(nwaves), dim3(64), lds_s, st, sa);
                        else if (kmax_t == 31)
                            hipLaunchKernelGGL(k_verify_steal<31>, dim3(nwaves), dim3(64), lds_s, st, sa);
                        else
                            hipLaunchKernelGGL(k_verify_steal<63>, dim3(nwaves), dim3(64), lds_s, st, sa);
                    });
                } else {
                    const unsigned vb = (unsigned)((total + 63) / 64);
                    if (all_lane && verify_seeds > 0 && verify_seeds < NSp) {
                        // first verification only for locations hit by the first seed slots;
                        // the others wait for a replay to ask
                        const uint32_t bits = (1u << verify_seeds) - 1u;
                        const unsigned mb = (unsigned)((total + 255) / 256);
                        timed("mark", st, [&] { hipLaunchKernelGGL(k_mark_late, dim3(mb), dim3(256), 0, st, mask_c, ncand, bits, dcap, vlim, steps); });
                        HIP_OK(select_idx(sel_tmp, sel_tb, total, FirstSeedsPred{mask_c, ncand, bits, alias}, short_list, sel_n + 5, st));
                        va.list = short_list;
                        va.nlist_ptr = sel_n + 5;
                    }
                    if (lead_mode) {
                        // the lead locations at the full limit, a lane per read (the lane tile
                        // of the requested verification), and each read's cap for the others
                        const int kfull = std::min(Kmax, LANE_KMAX);
                        const int TWf = (std::max(lane_L, 1) + kfull + 15) / 16 + 1;
                        const int kmf = kfull <= 7 ? 7 : (kfull <= 11 ? 11 : (kfull <= 15 ? 15 : (kfull <= 17 ? 17 :
                                        (kfull <= 31 ? 31 : 63))));
                        const size_t ldsf = (size_t)64 * 4 * (RW + TWf) + (kmf > 17 ? (size_t)64 * 2 * (2 * kmf + 3) : 0);
                        VerifyArgs vl = va;
                        vl.ps.Kcap = 1 << 14;
                        vl.TW = TWf;
                        vl.list = nullptr;
                        vl.rq = nullptr;
                        const unsigned lb = (unsigned)std::max<int64_t>(1, std::min<int64_t>((nr + 63) / 64, (int64_t)cus * 16));
                        timed("verify_lead", st, [&] {
                            if (kmf == 7)
                                hipLaunchKernelGGL(k_verify_lead<7>, dim3(lb), dim3(64), ldsf, st, vl, lead, rlim, Kp);
                            else if (kmf == 11)
                                hipLaunchKernelGGL(k_verify_lead<11>, dim3(lb), dim3(64), ldsf, st, vl, lead, rlim, Kp);
                            else if (kmf == 15)
                                hipLaunchKernelGGL(k_verify_lead<15>, dim3(lb), dim3(64), ldsf, st, vl, lead, rlim, Kp);
                            else if (kmf == 17)
                                hipLaunchKernelGGL(k_verify_lead<17>, dim3(lb), dim3(64), ldsf, st, vl, lead, rlim, Kp);
                            else if (kmf == 31)
                                hipLaunchKernelGGL(k_verify_lead<31>, dim3(lb), dim3(64), ldsf, st, vl, lead, rlim, Kp);
                            else
                                hipLaunchKernelGGL(k_verify_lead<63>, dim3(lb), dim3(64), ldsf, st, vl, lead, rlim, Kp);
                        });
                        va.lead = lead;
                        va.rlim = rlim;
                    }
                    timed("verify", st, [&] {
                        if (kmax_t == 7)
                            hipLaunchKernelGGL(k_verify<7>, dim3(vb), dim3(64), lds, st, va);
                        else if (kmax_t == 15)
                            hipLaunchKernelGGL(k_verify<15>, dim3(vb), dim3(64), lds, st, va);
                        else if (kmax_t == 31)
                            hipLaunchKernelGGL(k_verify<31>, dim3(vb), dim3(64), lds, st, va);
                        else
                            hipLaunchKernelGGL(k_verify<63>, dim3(vb), dim3(64), lds, st, va);
                    });
                }
                if (g_prof_on) {
                    // profiling: the first verification's own diagonal extensions, before
                    // requests add theirs to the same per-location counts
                    hipLaunchKernelGGL(k_fill_u32, dim3(1), dim3(64), 0, st, (uint32_t *)steps_first, 2, 0u);
                    hipLaunchKernelGGL(k_sum_u32, dim3(256), dim3(256), 0, st, steps, coff + nr, steps_first);
                }
            }
            ReplayArgs ra{probe, key_c, mask_c, dcap, vlim, coff, ccount, bmin, scored, lengths, ps, rule, sh,
                          alias, rflag, rq, short_list, reqcount, nullptr, nullptr, 0, exact_rounds, request_top,
                          lane_lmax,
                          pos, strand, dist, second, call};
            const unsigned rb = (unsigned)std::min<int64_t>((nr + 3) / 4, 8192);
            // reads with up to TINY_LOCS locations replay a lane each; the others, a wave
            // each, from their own lists (up to 64 locations in registers, more in LDS)
            auto replay = [&](const ReplayArgs &x, unsigned blocks, int64_t items) {
                const unsigned tb = (unsigned)std::max<int64_t>(1, std::min<int64_t>((items + 255) / 256, (int64_t)cus * 32));
                timed("replay_tiny", st, [&] { hipLaunchKernelGGL(k_replay_tiny, dim3(tb), dim3(256), 0, st, x); });
                if (maxH > TINY_LOCS) {
                    (void)select_count_range(sel_tmp, sel_tb, items, x.rlist, ccount, TINY_LOCS, 64u, light_list, sel_n + 8, st);
                    ReplayArgs l = x;
                    l.rlist = light_list;
                    l.rlist_n = sel_n + 8;
                    timed("replay", st, [&] { hipLaunchKernelGGL(k_replay<0>, dim3(blocks), dim3(256), 0, st, l); });
                }
                if (maxH > 64) {
                    (void)select_count_range(sel_tmp, sel_tb, items, x.rlist, ccount, 64u, 0xFFFFFFFFu, heavy_list,
                                             sel_n + 4, st);
                    ReplayArgs h = x;
                    h.rlist = heavy_list;
                    h.rlist_n = sel_n + 4;
                    const unsigned hb = (unsigned)std::min<int64_t>((items + 3) / 4, 1024);
                    timed("replay_heavy", st, [&] { hipLaunchKernelGGL(k_replay<HEAVY_LDS_LOCS>, dim3(hb), dim3(256), (size_t)4 * 4 * heavy_lds_words(HEAVY_LDS_LOCS), st, h); });
                }
            };
            replay(ra, rb, nr);
            // verify what the replays asked for, replay those reads, until nothing is asked.
            // A location is asked for again only at a higher limit than it was verified
            // with, and a read's limit rises by at most c - 1 per better location found,
            // so a read needs about NS + exact_rounds + a few times (Kmax + 1) rounds; the
            // bound below is far above that and turns a broken invariant into an error
            // instead of an endless loop.
            const int max_rounds = 16 * (NSp + Kmax + 16) + exact_rounds;
            for (int round = 1;; round++) {
                if (round > max_rounds) return SNAP_EINTERNAL;
                int64_t nrep = 0;
                HIP_OK(select_idx(sel_tmp, sel_tb, nr, FlagPred{rflag, RF_REPLAY}, replay_list, sel_n + 2, st));
                HIP_OK(hipMemcpyAsync(&nrep, sel_n + 2, 8, hipMemcpyDeviceToHost, st));
                HIP_OK(hipStreamSynchronize(st));
                if (nrep == 0) break;
                RequestArgs qa{replay_list, sel_n + 2, reqcount, short_list, coff};
                {
                    // lane tile: one list of every requested location, each verified at the
                    // limit its read asked for
                    size_t tb = scan_tmp_bytes(nrep + 1);
                    HIP_OK(scan_excl(scan_tmp, tb, LaneReqCount{replay_list, reqcount, nrep}, nrep + 1, req_off, st));
                    const unsigned fb = (unsigned)std::min<int64_t>((nrep + 3) / 4, 8192);
                    hipLaunchKernelGGL(k_flatten_requests, dim3(fb), dim3(256), 0, st, qa, req_off, long_list);
                    const int kfull = std::min(Kmax, LANE_KMAX);
                    const int TWf = (std::max(lane_L, 1) + kfull + 15) / 16 + 1;
                    // requested limits up to 17 keep their rows in registers too (17: the
                    // limits of d_max 15-16 reads)
                    const int kmf = kfull <= 7 ? 7 : (kfull <= 11 ? 11 : (kfull <= 15 ? 15 : (kfull <= 17 ? 17 :
                                    (kfull <= 31 ? 31 : 63))));
                    const size_t ldsf = (size_t)64 * 4 * (RW + TWf) + (kmf > 17 ? (size_t)64 * 2 * (2 * kmf + 3) : 0);
                    VerifyArgs vq{ix->d.gcode, ix->d.gmask, ix->d.G, rcode, rmask, roff, lengths, ps, key_c, cread,
                                  coff + nr, rule, RW, TWf, dcap, vlim, steps, long_list, req_off + nrep, rq};
                    // as many waves as fit the device (the count is on the device): rows of
                    // limits up to 11 in registers leave room for 24 a CU (71 VGPRs), of 15 and
                    // 17 for 16 (88-98 VGPRs), rows in LDS for 16
                    const int64_t per_cu = kmf <= 11 ? 24 : 16;
                    const unsigned vb = (unsigned)std::max<int64_t>(1, std::min<int64_t>((total + 63) / 64, (int64_t)cus * per_cu));
                    timed("verify_request", st, [&] {
                        if (kmf == 7)
                            hipLaunchKernelGGL(k_verify_requested<7>, dim3(vb), dim3(64), ldsf, st, vq);
                        else if (kmf == 11)
                            hipLaunchKernelGGL(k_verify_requested<11>, dim3(vb), dim3(64), ldsf, st, vq);
                        else if (kmf == 15)
                            hipLaunchKernelGGL(k_verify_requested<15>, dim3(vb), dim3(64), ldsf, st, vq);
                        else if (kmf == 17)
                            hipLaunchKernelGGL(k_verify_requested<17>, dim3(vb), dim3(64), ldsf, st, vq);
                        else if (kmf == 31)
                            hipLaunchKernelGGL(k_verify_requested<31>, dim3(vb), dim3(64), ldsf, st, vq);
                        else
                            hipLaunchKernelGGL(k_verify_requested<63>, dim3(vb), dim3(64), ldsf, st, vq);
                    });
                }
                if (!all_lane) {
                    // wave tile, each location at exactly the limit its read uses there
                    WaveVerifyArgs wq{ix->d.gcode, ix->d.gmask, ix->d.G, rcode, rmask, roff, lengths, ps, key_c, cread,
                                      rule, RWL, TWL, Kw, dcap, vlim, steps, batched ? steal_next : nullptr, rq};
                    if (batched) hipLaunchKernelGGL(k_fill_u32, dim3(1), dim3(64), 0, st, (uint32_t *)steal_next, 2, 0u);
                    const unsigned wb = (unsigned)std::min<int64_t>(nrep, steal_waves);
                    timed("verify_request_wave", st, [&] { hipLaunchKernelGGL(k_verify_requests_wave, dim3(wb), dim3(64), lds_wave, st, wq, qa); });
                }
                ReplayArgs rr = ra;
                rr.rlist = replay_list;
                rr.rlist_n = sel_n + 2;
                rr.round = round;
                const unsigned rqb = (unsigned)std::min<int64_t>((nrep + 3) / 4, 8192);
                replay(rr, rqb, nrep);
                if (g_prof_on) {
                    std::lock_guard<std::mutex> g(g_prof_mu);
                    g_ctr.requests += nrep;
                }
            }
            // reads that need more seeds go to the next pass (at a place of the shared
            // list reserved once their number is known)
            if (!final_pass) {
                HIP_OK(select_idx(sel_tmp, sel_tb, nr, FlagPred{rflag, RF_PENDING}, pend_local, sel_n + 3, st));
                int64_t np = 0;
                HIP_OK(hipMemcpyAsync(&np, sel_n + 3, 8, hipMemcpyDeviceToHost, st));
                HIP_OK(hipStreamSynchronize(st));
                int64_t at = 0;
                {
                    std::lock_guard<std::mutex> g(pend_mu);
                    at = pend_count;
                    pend_count += np;
                }
                if (np > 0)
                    hipLaunchKernelGGL(k_map_gid, dim3(256), dim3(256), 0, st, pend_local, sel_n + 3, ps, pending_out + at);
            }
            HIP_OK(hipGetLastError());
            if (g_prof_on) {
                // counters for the roofline: one extra wait per chunk, profiling only
                unsigned long long zero = 0, ssum = 0, sfirst = 0, nal = 0;
                int64_t ncand = 0;
                if (total > 0) {
                    HIP_OK(hipMemcpyAsync(steps_sum, &zero, 8, hipMemcpyHostToDevice, st));
                    hipLaunchKernelGGL(k_sum_u32, dim3(256), dim3(256), 0, st, steps, coff + nr, steps_sum);
                    HIP_OK(hipMemcpyAsync(&ssum, steps_sum, 8, hipMemcpyDeviceToHost, st));
                    HIP_OK(hipMemcpyAsync(&sfirst, steps_first, 8, hipMemcpyDeviceToHost, st));
                    if (alias) HIP_OK(hipMemcpyAsync(&nal, nalias, 8, hipMemcpyDeviceToHost, st));
                }
                HIP_OK(hipMemcpyAsync(&ncand, coff + nr, 8, hipMemcpyDeviceToHost, st));
                HIP_OK(hipStreamSynchronize(st));
                std::lock_guard<std::mutex> g(g_prof_mu);
                g_ctr.passes += 1;
                g_ctr.reads += first ? nr : 0;
                g_ctr.seed_slots += nr * NSp;
                g_ctr.hits += total;
                g_ctr.locations += ncand;
                g_ctr.lv_steps += (int64_t)ssum;
                g_ctr.lv_steps_first += (int64_t)sfirst;
                g_ctr.dup_aliases += (int64_t)nal;
                if (!first) g_ctr.second_pass_reads += nr;
            }
            r0 += nr;
          }
        }
        HIP_OK(hipStreamSynchronize(st));
        HIP_OK(hipGetLastError());
        return SNAP_OK;
        };
        if (workers == 1) return work(wk[0]);
        int rcs[MAX_WORKERS] = {};
        std::vector<std::thread> threads;
        for (int w = 1; w < workers; w++) {
            threads.emplace_back([&, w] {
                if (hipSetDevice(dev) != hipSuccess) {
                    rcs[w] = SNAP_EDEVICE;
                    return;
                }
                rcs[w] = work(wk[w]);
            });
        }
        rcs[0] = work(wk[0]);
        for (auto &t : threads) t.join();
        for (int w = 0; w < workers; w++)
            if (rcs[w] != SNAP_OK) return rcs[w];
        return SNAP_OK;
    };

    // stage 1 (when it is not complete): the first pass1_seeds seeds, locations
    // verified first with limit pass1_limit; final stage: every seed, first limit
    // final_limit. In both, the replay asks for whatever more it needs (short reads:
    // their undecided locations at the full limit; long reads in the final stage:
    // single locations at the exact limit) and only reads that need more seeds
    // leave stage 1.
    struct Stage { int seeds, cap; };
    Stage stages[2];
    int nst = 0;
    {
        const int s1 = tune.pass1_seeds > 0 ? std::min(NS, tune.pass1_seeds) : NS;
        const int k1 = tune.pass1_limit > 0 && tune.pass1_limit < Kmax ? tune.pass1_limit : KCAP_NONE;
        if (!(s1 >= NS && k1 == KCAP_NONE)) stages[nst++] = Stage{s1, k1};
        const int kf = tune.final_limit > 0 && tune.final_limit < Kmax ? tune.final_limit : KCAP_NONE;
        stages[nst++] = Stage{NS, kf};
    }
    uint32_t *plist[2] = {pending, pending + n_reads};
    const uint32_t *list = nullptr;
    int64_t list_len = n_reads;
    const int32_t split_len = tune.pass1_max_len;
    if (nst == 2 && !batched && split_len > 0 && maxL > split_len && select_tmp_bytes(n_reads + 1) <= 8 * (size_t)PS) {
        // reads longer than split_len need more round-0 seeds than the first stage probes
        // before Algorithm 1 can stop: they take every seed slot in one complete pass over
        // their own list (the first stage's limit); the others take the two stages
        int64_t *cnt = wk[0].misc + 14;
        size_t tb = select_tmp_bytes(n_reads + 1);
        HIP_OK(select_idx(wk[0].hk, tb, n_reads, LenPred{lengths, split_len, false}, plist[0], cnt, st));
        int64_t nshort = 0;
        HIP_OK(hipMemcpyAsync(&nshort, cnt, 8, hipMemcpyDeviceToHost, st));
        HIP_OK(hipStreamSynchronize(st));
        HIP_OK(select_idx(wk[0].hk, tb, n_reads, LenPred{lengths, split_len, true}, plist[0] + nshort, cnt + 1, st));
        HIP_OK(hipStreamSynchronize(st));
        pending_out = nullptr;
        pend_count = 0;
        int rc = run_pass(plist[0] + nshort, n_reads - nshort, NS, stages[0].cap, 1, true);
        if (rc != SNAP_OK) return rc;
        list = plist[0];
        list_len = nshort;
        pending_out = plist[1];
        pend_count = 0;
        if (list_len > 0) {
            rc = run_pass(list, list_len, stages[0].seeds, stages[0].cap, 0, true);
            if (rc != SNAP_OK) return rc;
        }
        list = plist[1];
        list_len = pend_count;
        if (list_len > 0) return run_pass(list, list_len, stages[1].seeds, stages[1].cap, 1, false);
        return SNAP_OK;
    }
    for (int k = 0; k < nst && list_len > 0; k++) {
        const bool last = (k == nst - 1);
        pending_out = plist[k & 1];
        pend_count = 0;
        int rc = run_pass(list, list_len, stages[k].seeds, stages[k].cap, last ? 1 : 0, k == 0);
        if (rc != SNAP_OK) return rc;
        if (last) break;
        list = plist[k & 1];
        list_len = pend_count;
    }
    return SNAP_OK;
}

}  // namespace

extern "C" int snap_align(const snap_index *ix, const uint8_t *reads, const int32_t *lengths, int64_t n_reads,
                          int32_t d_max, const snap_params *p, int64_t *pos, int8_t *strand, int32_t *dist,
                          int32_t *second, int8_t *call, void *workspace, size_t ws_bytes, void *stream) {
    return align_impl(ix, reads, lengths, n_reads, d_max, p, pos, strand, dist, second, call, workspace, ws_bytes,
                      stream, false, nullptr);
}

extern "C" int snap_align_batched(const snap_index *ix, const uint8_t *reads, const int32_t *lengths, int64_t n_reads,
                                  int32_t d_max, const snap_params *p, const snap_tuning *tuning, int64_t *pos,
                                  int8_t *strand, int32_t *dist, int32_t *second, int8_t *call, void *workspace,
                                  size_t ws_bytes, void *stream) {
    return align_impl(ix, reads, lengths, n_reads, d_max, p, pos, strand, dist, second, call, workspace, ws_bytes,
                      stream, true, tuning);
}

// Scratch of snap_align_noalloc: one array per device, part of the code object (placed
// in device memory when the library is loaded on a device, held until the process
// ends). Host code reaches it only through the address hipGetSymbolAddress gives on
// each device; the array's name is not a device address in host code.
constexpr size_t NOALLOC_SCRATCH_BYTES = (size_t)128 << 20;
__device__ __align__(256) char scratch[NOALLOC_SCRATCH_BYTES];

namespace {

constexpr int MAX_DEVICES = 64;
std::mutex g_scratch_mu;
void *g_scratch_ptr[MAX_DEVICES] = {};

// The device address of the current device's scratch array, looked up once per device
// (with that device current) and kept.
int scratch_address(void **out) {
    int dev = -1;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= MAX_DEVICES) return SNAP_EDEVICE;
    std::lock_guard<std::mutex> g(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void *ptr = nullptr;
        if (hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)) != hipSuccess || !ptr) return SNAP_EDEVICE;
        g_scratch_ptr[dev] = ptr;
    }
    *out = g_scratch_ptr[dev];
    return SNAP_OK;
}

}  // namespace

extern "C" size_t snap_align_noalloc_scratch_bytes(void) { return NOALLOC_SCRATCH_BYTES; }

extern "C" int snap_align_noalloc(const snap_index *ix, const uint8_t *reads, const int32_t *lengths, int64_t n_reads,
                                  int32_t d_max, const snap_params *p, int64_t *pos, int8_t *strand, int32_t *dist,
                                  int32_t *second, int8_t *call, void *stream) {
    if (!ix || n_reads < 0 || d_max < 0 || !valid_params(p)) return SNAP_EINVAL;
    if (n_reads == 0) return SNAP_OK;
    void *ws = nullptr;
    const int rc = scratch_address(&ws);
    if (rc != SNAP_OK) return rc;
    return align_impl(ix, reads, lengths, n_reads, d_max, p, pos, strand, dist, second, call, ws,
                      NOALLOC_SCRATCH_BYTES, stream, false, nullptr, true);
}

// Seed offsets tried for a read of length L (host evaluation of the same
// functions the probe kernel uses).
extern "C" int32_t snap_debug_seed_offsets(int32_t L, int32_t s, int32_t n, int32_t *out) {
    if (!out || s < 1 || s > 32 || n < 0 || n > 64) return 0;
    const Shifts sh = make_shifts(s);
    int32_t k = 0;
    for (int i = 0; i < n; i++) {
        int o = seed_offset(sh, s, L, i);
        if (o < 0) break;
        out[k++] = o;
    }
    return k;
}

extern "C" int snap_profile_begin(void) {
    std::lock_guard<std::mutex> g(g_prof_mu);
    for (auto &r : g_prof) { (void)hipEventDestroy(r.a); (void)hipEventDestroy(r.b); }
    g_prof.clear();
    std::memset(&g_ctr, 0, sizeof(g_ctr));
    g_prof_on = true;
    return SNAP_OK;
}

extern "C" int snap_profile_counters(snap_counters *out) {
    if (!out) return SNAP_EINVAL;
    std::lock_guard<std::mutex> g(g_prof_mu);
    *out = g_ctr;
    return SNAP_OK;
}

extern "C" int snap_profile_end(snap_kernel_time *out, int32_t cap, int32_t *count) {
    std::lock_guard<std::mutex> g(g_prof_mu);
    g_prof_on = false;
    std::vector<std::string> names;
    std::vector<int64_t> launches;
    std::vector<double> ms;
    int rc = SNAP_OK;
    for (auto &r : g_prof) {
        float t = 0;
        if (hipEventSynchronize(r.b) != hipSuccess || hipEventElapsedTime(&t, r.a, r.b) != hipSuccess) rc = SNAP_EDEVICE;
        size_t k = 0;
        while (k < names.size() && names[k] != r.name) k++;
        if (k == names.size()) { names.push_back(r.name); launches.push_back(0); ms.push_back(0); }
        launches[k]++;
        ms[k] += t;
        (void)hipEventDestroy(r.a);
        (void)hipEventDestroy(r.b);
    }
    g_prof.clear();
    int32_t n = 0;
    for (size_t k = 0; k < names.size() && (int32_t)k < cap; k++, n++) {
        std::memset(&out[k], 0, sizeof(out[k]));
        std::strncpy(out[k].name, names[k].c_str(), sizeof(out[k].name) - 1);
        out[k].launches = launches[k];
        out[k].total_ms = ms[k];
    }
    if (count) *count = n;
    return rc;
}

// Plain device copy (one dword per lane per step), used to calibrate hardware
// byte counters against a transfer of known size.
__global__ void k_copy_u32(const uint32_t *__restrict__ src, uint32_t *__restrict__ dst, int64_t n) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        dst[i] = src[i];
}

// Random-line gather (the access pattern of the probe and the position reads): every
// group of `line / 16` lanes reads one `line`-byte line at a pseudo-random line-aligned
// place of the buffer (16 bytes a lane, one coalesced access), `rounds` times; the lines'
// words are summed so the loads stay, and each thread writes its sum once.
__global__ __launch_bounds__(256) void k_gather_lines(const uint4 *buf, uint64_t nlines, int lanes_per_line,
                                                      int rounds, uint64_t seed, uint32_t *sink) {
    const uint64_t t = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const uint64_t grp = t / (uint64_t)lanes_per_line;
    const int sub = (int)(t % (uint64_t)lanes_per_line);
    uint32_t acc = 0;
    for (int i = 0; i < rounds; i++) {
        const uint64_t line = mix64(seed ^ (grp * 0x9E3779B97F4A7C15ull + (uint64_t)i)) % nlines;
        const uint4 v = buf[line * (uint64_t)lanes_per_line + (uint64_t)sub];
        acc += v.x ^ v.y ^ v.z ^ v.w;
    }
    sink[t] = acc;
}

extern "C" int snap_debug_gather_lines(const void *buf, uint64_t bytes, int32_t line_bytes, int32_t rounds,
                                       uint64_t threads, uint64_t seed, void *sink, void *stream) {
    if (!buf || !sink || (line_bytes != 32 && line_bytes != 64 && line_bytes != 128) || rounds < 1 || threads == 0 ||
        bytes < (uint64_t)line_bytes || (threads % 256) != 0 || ((uintptr_t)buf & 127) != 0)
        return SNAP_EINVAL;
    const int lpl = line_bytes / 16;
    if (threads % (uint64_t)lpl != 0) return SNAP_EINVAL;
    hipStream_t st = (hipStream_t)stream;
    const uint64_t nlines = bytes / (uint64_t)line_bytes;
    timed("gather_lines", st, [&] {
        hipLaunchKernelGGL(k_gather_lines, dim3((unsigned)(threads / 256)), dim3(256), 0, st, (const uint4 *)buf, nlines,
                           lpl, rounds, seed, (uint32_t *)sink);
    });
    return hipGetLastError() == hipSuccess ? SNAP_OK : SNAP_EDEVICE;
}

extern "C" int snap_debug_copy(const void *src, void *dst, uint64_t bytes, void *stream) {
    if (!src || !dst || (bytes & 3)) return SNAP_EINVAL;
    hipStream_t st = (hipStream_t)stream;
    const int64_t n = (int64_t)(bytes / 4);
    timed("copy", st, [&] { hipLaunchKernelGGL(k_copy_u32, dim3(4096), dim3(256), 0, st, (const uint32_t *)src, (uint32_t *)dst, n); });
    return hipGetLastError() == hipSuccess ? SNAP_OK : SNAP_EDEVICE;
}
