// Seed index of Section 3.1: every N-free window of s bases, overlapping (slid one
// base at a time), looked up in both orientations (Section 3.2, omitted aspect 2).
//
// Built on the host in four passes, then copied to HBM:
//   1. pack the genome: 2-bit codes + 1-bit N mask;
//   2. emit one record (canonical code, orientation, q) per N-free window q, where
//      the canonical code is min(forward, reverse complement) and the orientation
//      says which of the two the window is (a palindromic window emits both);
//   3. stable LSD radix sort by (canonical code, orientation): positions come out
//      grouped per key, forward windows first, each group ascending in q;
//   4. fill the open-addressing table (keys placed in home-bucket order, linear
//      probing over 128-byte buckets) and the position array.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <cstdlib>
#include <cstring>
#include <new>
#include <thread>
#include <vector>

#include "../../include/snapgpu.h"
#include "../../include/snapgpu_debug.h"
#include "snap_internal.h"

using namespace snapgpu;

namespace {

inline int base_code(uint8_t b) {
    switch (b) {
        case 'A': case 'a': return 0;
        case 'C': case 'c': return 1;
        case 'G': case 'g': return 2;
        case 'T': case 't': return 3;
        default: return 4;
    }
}

struct Rec {
    uint64_t key;
    uint32_t q;
    uint32_t orient;
};

int num_threads() {
    unsigned t = std::thread::hardware_concurrency();
    if (t == 0) t = 1;
    if (t > 64) t = 64;
    return (int)t;
}

template <class F>
void parallel_for(int64_t n, int threads, F f) {
    if (threads <= 1 || n < 1 << 16) {
        f(0, n, 0);
        return;
    }
    std::vector<std::thread> th;
    int64_t per = (n + threads - 1) / threads;
    for (int t = 0; t < threads; t++) {
        int64_t lo = t * per, hi = std::min(n, lo + per);
        if (lo >= hi) break;
        th.emplace_back([=]() { f(lo, hi, t); });
    }
    for (auto &x : th) x.join();
}

// Stable LSD radix sort of records by (key, orient), 8-bit digits, parallel
// histogram + scatter over contiguous input slices.
void radix_sort(std::vector<Rec> &a, int key_bits, int threads) {
    const int64_t n = (int64_t)a.size();
    if (n <= 1) return;
    std::vector<Rec> b(n);
    Rec *src = a.data(), *dst = b.data();
    const int T = (n < (1 << 16)) ? 1 : threads;
    std::vector<int64_t> hist((size_t)T * 256);
    auto pass = [&](auto digit_of) {
        std::fill(hist.begin(), hist.end(), 0);
        parallel_for(n, T, [&](int64_t lo, int64_t hi, int t) {
            int64_t *h = &hist[(size_t)t * 256];
            for (int64_t i = lo; i < hi; i++) h[digit_of(src[i])]++;
        });
        int64_t run = 0;
        for (int d = 0; d < 256; d++)
            for (int t = 0; t < T; t++) {
                int64_t c = hist[(size_t)t * 256 + d];
                hist[(size_t)t * 256 + d] = run;
                run += c;
            }
        parallel_for(n, T, [&](int64_t lo, int64_t hi, int t) {
            int64_t *h = &hist[(size_t)t * 256];
            for (int64_t i = lo; i < hi; i++) dst[h[digit_of(src[i])]++] = src[i];
        });
        std::swap(src, dst);
    };
    pass([](const Rec &r) { return (int)r.orient; });
    for (int sh = 0; sh < key_bits; sh += 8) pass([sh](const Rec &r) { return (int)((r.key >> sh) & 0xFF); });
    if (src != a.data()) std::memcpy(a.data(), src, sizeof(Rec) * (size_t)n);
}

struct HostIndex {
    std::vector<uint32_t> gcode, gmask, positions;
    std::vector<uint64_t> table;
    uint64_t G = 0, nbuckets = 0, windows = 0, distinct = 0;
    int log2b = 0, s = 0;
};

int build_host(const uint8_t *genome, uint64_t G, int s, HostIndex &h) {
    const int T = num_threads();
    h.G = G;
    h.s = s;
    const uint64_t ncw = (G + 15) / 16 + GENOME_PAD_WORDS, nmw = (G + 31) / 32 + GENOME_PAD_WORDS;
    h.gcode.assign(ncw, 0);
    h.gmask.assign(nmw, 0);
    // 1. pack (each 32-base block owns 2 code words and 1 mask word)
    parallel_for((int64_t)((G + 31) / 32), T, [&](int64_t lo, int64_t hi, int) {
        for (int64_t blk = lo; blk < hi; blk++) {
            uint32_t c0 = 0, c1 = 0, m = 0;
            for (int k = 0; k < 32; k++) {
                uint64_t j = (uint64_t)blk * 32 + k;
                if (j >= G) break;
                int c = base_code(genome[j]);
                if (c > 3) { m |= 1u << k; c = 0; }
                if (k < 16) c0 |= (uint32_t)c << (2 * k); else c1 |= (uint32_t)c << (2 * (k - 16));
            }
            h.gcode[2 * blk] = c0;
            h.gcode[2 * blk + 1] = c1;
            h.gmask[blk] = m;
        }
    });
    // 2. records; windows split into T slices, each slice counted then filled
    const int64_t nwin = (G >= (uint64_t)s) ? (int64_t)(G - s + 1) : 0;
    const uint64_t km = seed_mask(s);
    auto window_has_n = [&](int64_t q) {
        for (int64_t j = q; j < q + s;) {
            int off = (int)(j & 31);
            int span = std::min<int64_t>(32 - off, q + s - j);
            uint32_t w = h.gmask[j >> 5] >> off;
            if (span < 32) w &= (1u << span) - 1;
            if (w) return true;
            j += span;
        }
        return false;
    };
    // returns records written (fill) or counted; *nfree receives N-free windows
    auto scan_slice = [&](int64_t lo, int64_t hi, Rec *out, int64_t *nfree) -> int64_t {
        int64_t m = 0, free_w = 0;
        uint64_t fw = 0;
        for (int64_t j = lo; j < lo + s - 1 && j < (int64_t)G; j++)
            fw = ((fw >> 2) | ((uint64_t)(base_code(genome[j]) & 3) << (2 * (s - 1)))) & km;
        for (int64_t q = lo; q < hi; q++) {
            fw = ((fw >> 2) | ((uint64_t)(base_code(genome[q + s - 1]) & 3) << (2 * (s - 1)))) & km;
            if (window_has_n(q)) continue;
            free_w++;
            uint64_t rc = rc_code(fw, s);
            uint64_t canon = fw < rc ? fw : rc;
            if (out) {
                if (fw == canon) out[m++] = Rec{canon, (uint32_t)q, 0};
                if (rc == canon) out[m++] = Rec{canon, (uint32_t)q, 1};
            } else {
                m += (fw == canon) + (rc == canon);
            }
        }
        if (nfree) *nfree = free_w;
        return m;
    };
    const int64_t per = (nwin + T - 1) / T;
    std::vector<int64_t> cnt(T + 1, 0), nfree(T, 0);
    {
        std::vector<std::thread> th;
        for (int t = 0; t < T; t++)
            th.emplace_back([&, t]() {
                int64_t lo = std::min<int64_t>(nwin, t * per), hi = std::min<int64_t>(nwin, lo + per);
                cnt[t + 1] = scan_slice(lo, hi, nullptr, &nfree[t]);
            });
        for (auto &x : th) x.join();
    }
    h.windows = 0;
    for (int t = 0; t < T; t++) { cnt[t + 1] += cnt[t]; h.windows += (uint64_t)nfree[t]; }
    const int64_t nrec = cnt[T];
    std::vector<Rec> recs;
    try { recs.resize((size_t)nrec); } catch (const std::bad_alloc &) { return SNAP_ENOMEM; }
    {
        std::vector<std::thread> th;
        for (int t = 0; t < T; t++)
            th.emplace_back([&, t]() {
                int64_t lo = std::min<int64_t>(nwin, t * per), hi = std::min<int64_t>(nwin, lo + per);
                scan_slice(lo, hi, recs.data() + cnt[t], nullptr);
            });
        for (auto &x : th) x.join();
    }
    // 3. sort
    radix_sort(recs, 2 * s, T);
    // 4. group: one table entry per distinct canonical code
    h.positions.resize((size_t)nrec);
    std::vector<uint64_t> keys, vals;
    for (int64_t i = 0; i < nrec;) {
        int64_t j = i;
        uint64_t nf = 0, nr = 0;
        while (j < nrec && recs[j].key == recs[i].key) {
            if (recs[j].orient == 0) nf++; else nr++;
            h.positions[j] = recs[j].q;
            j++;
        }
        keys.push_back(recs[i].key);
        vals.push_back(((uint64_t)i & OFF_MASK) | ((uint64_t)std::min<uint64_t>(nf, CNT_SAT) << 36) |
                       ((uint64_t)std::min<uint64_t>(nr, CNT_SAT) << 50));
        i = j;
    }
    h.distinct = keys.size();
    recs.clear();
    recs.shrink_to_fit();
    // table size: power-of-two buckets, load factor at most 0.7
    uint64_t need = (uint64_t)((double)h.distinct / (0.7 * SLOTS_PER_BUCKET)) + 1;
    h.log2b = 0;
    while ((1ull << h.log2b) < need) h.log2b++;
    h.nbuckets = 1ull << h.log2b;
    h.table.assign(h.nbuckets * SLOTS_PER_BUCKET * 2, 0);
    for (uint64_t i = 0; i < h.nbuckets * SLOTS_PER_BUCKET; i++) h.table[2 * i] = EMPTY_KEY;
    // place keys in home-bucket order (counting sort by home bucket); a key lands
    // in the first bucket at or after its home that still has a free slot, and
    // every bucket it passes over is full, which is what the lookup relies on
    std::vector<uint32_t> home(h.distinct);
    std::vector<uint64_t> start(h.nbuckets + 1, 0);
    for (uint64_t i = 0; i < h.distinct; i++) {
        uint64_t b = home_bucket(keys[i], h.log2b);
        home[i] = (uint32_t)b;
        start[b + 1]++;
    }
    for (uint64_t b = 0; b < h.nbuckets; b++) start[b + 1] += start[b];
    std::vector<uint64_t> order(h.distinct);
    {
        std::vector<uint64_t> fillp(start.begin(), start.end() - 1);
        for (uint64_t i = 0; i < h.distinct; i++) order[fillp[home[i]]++] = i;
    }
    uint64_t cur = 0, used = 0;
    std::vector<uint64_t> spill;
    for (uint64_t k = 0; k < h.distinct; k++) {
        uint64_t i = order[k], hb = home[i];
        if (hb > cur) { cur = hb; used = 0; }
        if (used == SLOTS_PER_BUCKET) { cur++; used = 0; }
        if (cur >= h.nbuckets) { spill.push_back(i); continue; }
        uint64_t slot = cur * SLOTS_PER_BUCKET + used++;
        h.table[2 * slot] = keys[i];
        h.table[2 * slot + 1] = vals[i];
    }
    // keys pushed past the last bucket wrap around to the front
    for (uint64_t i : spill) {
        for (uint64_t b = 0;; b++) {
            uint64_t s0 = b * SLOTS_PER_BUCKET, k;
            for (k = 0; k < SLOTS_PER_BUCKET; k++)
                if (h.table[2 * (s0 + k)] == EMPTY_KEY) break;
            if (k < SLOTS_PER_BUCKET) {
                h.table[2 * (s0 + k)] = keys[i];
                h.table[2 * (s0 + k) + 1] = vals[i];
                break;
            }
        }
    }
    return SNAP_OK;
}

// Host-side lookup with the same probe sequence as the device kernel.
bool host_lookup(const HostIndex &h, uint64_t canon, uint64_t *val) {
    uint64_t b = home_bucket(canon, h.log2b);
    for (uint64_t step = 0; step < h.nbuckets; step++) {
        bool empty = false;
        for (int k = 0; k < SLOTS_PER_BUCKET; k++) {
            uint64_t slot = b * SLOTS_PER_BUCKET + k;
            if (h.table[2 * slot] == canon) { *val = h.table[2 * slot + 1]; return true; }
            if (h.table[2 * slot] == EMPTY_KEY) empty = true;
        }
        if (empty) return false;
        b = (b + 1) & (h.nbuckets - 1);
    }
    return false;
}

template <class T>
int upload(const std::vector<T> &v, void **dptr) {
    size_t bytes = std::max<size_t>(v.size() * sizeof(T), 256);
    if (hipMalloc(dptr, bytes) != hipSuccess) { *dptr = nullptr; return SNAP_ENOMEM; }
    if (!v.empty() && hipMemcpy(*dptr, v.data(), v.size() * sizeof(T), hipMemcpyHostToDevice) != hipSuccess)
        return SNAP_EDEVICE;
    return SNAP_OK;
}

}  // namespace

extern "C" const char *snap_strerror(int code) {
    switch (code) {
        case SNAP_OK: return "ok";
        case SNAP_EINVAL: return "invalid argument";
        case SNAP_ENOMEM: return "out of memory or workspace too small";
        case SNAP_EDEVICE: return "HIP device error";
        case SNAP_EBUSY: return "queue full";
        case SNAP_EAGAIN: return "not complete yet";
        default: return "unknown status";
    }
}

extern "C" int snap_index_free(snap_index *ix) {
    if (!ix) return SNAP_OK;
    int dev = 0;
    (void)hipGetDevice(&dev);
    (void)hipSetDevice(ix->device);
    if (ix->alloc_gcode) (void)hipFree(ix->alloc_gcode);
    if (ix->alloc_gmask) (void)hipFree(ix->alloc_gmask);
    if (ix->alloc_table) (void)hipFree(ix->alloc_table);
    if (ix->alloc_pos) (void)hipFree(ix->alloc_pos);
    (void)hipSetDevice(dev);
    delete ix;
    return SNAP_OK;
}

extern "C" int snap_index_build(const uint8_t *genome, uint64_t len, int32_t seed_len, snap_index **out) {
    if (!out) return SNAP_EINVAL;
    *out = nullptr;
    if (!genome || seed_len < 1 || seed_len > 32 || len < (uint64_t)seed_len || len >= (1ull << 32))
        return SNAP_EINVAL;
    HostIndex h;
    int rc;
    try {
        rc = build_host(genome, len, seed_len, h);
    } catch (const std::bad_alloc &) {
        return SNAP_ENOMEM;
    }
    if (rc != SNAP_OK) return rc;
    snap_index *ix = new (std::nothrow) snap_index();
    if (!ix) return SNAP_ENOMEM;
    if (hipGetDevice(&ix->device) != hipSuccess) { delete ix; return SNAP_EDEVICE; }
    if ((rc = upload(h.gcode, &ix->alloc_gcode)) || (rc = upload(h.gmask, &ix->alloc_gmask)) ||
        (rc = upload(h.table, &ix->alloc_table)) || (rc = upload(h.positions, &ix->alloc_pos))) {
        snap_index_free(ix);
        return rc;
    }
    ix->d.gcode = (const uint32_t *)ix->alloc_gcode;
    ix->d.gmask = (const uint32_t *)ix->alloc_gmask;
    ix->d.table = (const uint64_t *)ix->alloc_table;
    ix->d.positions = (const uint32_t *)ix->alloc_pos;
    ix->d.G = h.G;
    ix->d.nbuckets = h.nbuckets;
    ix->d.log2_buckets = h.log2b;
    ix->d.s = seed_len;
    ix->windows = h.windows;
    ix->distinct_keys = h.distinct;
    ix->position_entries = h.positions.size();
    ix->device_bytes = h.gcode.size() * 4 + h.gmask.size() * 4 + h.table.size() * 8 + h.positions.size() * 4;
    *out = ix;
    return SNAP_OK;
}

extern "C" int snap_index_info(const snap_index *ix, snap_index_sizes *info) {
    if (!ix || !info) return SNAP_EINVAL;
    std::memset(info, 0, sizeof(*info));
    info->genome_len = ix->d.G;
    info->seed_len = ix->d.s;
    info->windows = ix->windows;
    info->distinct_keys = ix->distinct_keys;
    info->table_slots = ix->d.nbuckets * SLOTS_PER_BUCKET;
    info->position_entries = ix->position_entries;
    info->device_bytes = ix->device_bytes;
    info->device = ix->device;
    return SNAP_OK;
}

// Host-only check of the table layout (no device needed): builds the index in
// host memory and answers queries with the same probe sequence the device uses.
// For each ASCII seed of length s in `queries` (nq of them, back to back) writes
// the number of windows equal to the seed (fwd) and to its reverse complement
// (rev), or -1/-1 for a seed holding an N. Returns a status code.
extern "C" int snap_debug_host_lookup(const uint8_t *genome, uint64_t len, int32_t seed_len,
                                      const uint8_t *queries, int64_t nq, int64_t *fwd, int64_t *rev,
                                      int64_t *first_fwd, uint64_t *windows) {
    if (!genome || !queries || !fwd || !rev || seed_len < 1 || seed_len > 32 || len < (uint64_t)seed_len)
        return SNAP_EINVAL;
    HostIndex h;
    int rc = build_host(genome, len, seed_len, h);
    if (rc) return rc;
    if (windows) *windows = h.windows;
    for (int64_t i = 0; i < nq; i++) {
        const uint8_t *q = queries + i * seed_len;
        uint64_t k = 0;
        bool hasn = false;
        for (int j = 0; j < seed_len; j++) {
            int c = base_code(q[j]);
            if (c > 3) hasn = true;
            k |= (uint64_t)(c & 3) << (2 * j);
        }
        if (hasn) { fwd[i] = rev[i] = -1; if (first_fwd) first_fwd[i] = -1; continue; }
        uint64_t r = rc_code(k, seed_len), canon = k < r ? k : r, v = 0;
        if (!host_lookup(h, canon, &v)) { fwd[i] = rev[i] = 0; if (first_fwd) first_fwd[i] = -1; continue; }
        uint64_t off = v & OFF_MASK, nf = (v >> 36) & CNT_SAT, nr = (v >> 50) & CNT_SAT;
        bool flip = (k != canon);
        fwd[i] = (int64_t)(flip ? nr : nf);
        rev[i] = (int64_t)(flip ? nf : nr);
        if (first_fwd) {
            uint64_t o = flip ? off + nf : off;
            first_fwd[i] = fwd[i] > 0 ? (int64_t)h.positions[o] : -1;
        }
    }
    return SNAP_OK;
}
