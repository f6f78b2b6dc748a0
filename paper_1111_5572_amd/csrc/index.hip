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
#include <cstdio>
#include <cstring>
#include <memory>
#include <new>
#include <thread>
#include <type_traits>
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

// Progress of a long build: each finished stage is reported (stage name, null ctx ok).
struct Progress {
    snap_progress_fn fn;
    void *ctx;
    void operator()(const char *stage) const {
        if (fn) fn(stage, ctx);
    }
};

// Stable LSD radix sort of records by (key, orient), 8-bit digits, parallel
// histogram + scatter over contiguous input slices.
void radix_sort(std::vector<Rec> &a, int key_bits, int threads, const Progress &prog) {
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
    for (int sh = 0; sh < key_bits; sh += 8) {
        pass([sh](const Rec &r) { return (int)((r.key >> sh) & 0xFF); });
        char msg[64];
        std::snprintf(msg, sizeof(msg), "sorted records by key bits %d-%d", sh, std::min(sh + 8, key_bits) - 1);
        prog(msg);
    }
    if (src != a.data()) std::memcpy(a.data(), src, sizeof(Rec) * (size_t)n);
}

// Host array left uninitialised on allocation (the table is cleared in parallel).
template <class T>
struct HostArray {
    std::unique_ptr<T[]> p;
    size_t n = 0;
    void allocate(size_t count) {
        p.reset(new T[count]);
        n = count;
    }
    size_t size() const { return n; }
    T *data() { return p.get(); }
    const T *data() const { return p.get(); }
    T &operator[](size_t i) { return p[i]; }
    const T &operator[](size_t i) const { return p[i]; }
};

// Insert a key into the table: buckets are probed from the key's home bucket on
// (wrapping at the end) and the first empty slot is claimed with a compare-and-swap
// on its key word, so threads insert at once. Nothing is ever removed, so every
// bucket a key passed over is full for good, which is what a lookup relies on (it
// stops at the first bucket with an empty slot). Which slot a key lands in depends
// on the order of insertion; what a lookup returns does not.
void table_insert(uint64_t *table, uint64_t nb, int log2b, uint64_t key, uint64_t val) {
    uint64_t b = home_bucket(key, log2b);
    for (;;) {
        for (int k = 0; k < SLOTS_PER_BUCKET; k++) {
            uint64_t *slot = table + 2 * (b * SLOTS_PER_BUCKET + k);
            uint64_t expect = EMPTY_KEY;
            if (__atomic_load_n(slot, __ATOMIC_RELAXED) == EMPTY_KEY &&
                __atomic_compare_exchange_n(slot, &expect, key, false, __ATOMIC_RELAXED, __ATOMIC_RELAXED)) {
                slot[1] = val;
                return;
            }
        }
        b = (b + 1) & (nb - 1);
    }
}

struct HostIndex {
    std::vector<uint32_t> gcode, gmask, positions;
    HostArray<uint64_t> table;
    uint64_t G = 0, nbuckets = 0, windows = 0, distinct = 0;
    int log2b = 0, s = 0;
};

int build_host(const uint8_t *genome, uint64_t G, int s, HostIndex &h, const Progress &prog) {
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
    prog("packed the genome");
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
    prog("emitted window records");
    // 3. sort
    radix_sort(recs, 2 * s, T, prog);
    // 4. group: one table entry per distinct canonical code. The records are cut
    //    into T slices at key boundaries; each slice counts its distinct keys, the
    //    table is sized from the total, then each slice writes its positions and
    //    inserts its keys.
    h.positions.resize((size_t)nrec);
    std::vector<int64_t> cut(T + 1, nrec);
    cut[0] = 0;
    for (int t = 1; t < T; t++) {
        int64_t c = std::max<int64_t>(cut[t - 1], nrec * t / T);
        while (c > 0 && c < nrec && recs[c].key == recs[c - 1].key) c++;
        cut[t] = c;
    }
    std::vector<uint64_t> nkeys(T, 0);
    {
        std::vector<std::thread> th;
        for (int t = 0; t < T; t++)
            th.emplace_back([&, t]() {
                uint64_t n = 0;
                for (int64_t i = cut[t]; i < cut[t + 1]; i++)
                    if (i == cut[t] || recs[i].key != recs[i - 1].key) n++;
                nkeys[t] = n;
            });
        for (auto &x : th) x.join();
    }
    h.distinct = 0;
    for (int t = 0; t < T; t++) h.distinct += nkeys[t];
    // table size: power-of-two buckets, load factor at most 0.7
    uint64_t need = (uint64_t)((double)h.distinct / (0.7 * SLOTS_PER_BUCKET)) + 1;
    h.log2b = 0;
    while ((1ull << h.log2b) < need) h.log2b++;
    h.nbuckets = 1ull << h.log2b;
    h.table.allocate(h.nbuckets * SLOTS_PER_BUCKET * 2);
    uint64_t *table = h.table.data();
    parallel_for((int64_t)(h.nbuckets * SLOTS_PER_BUCKET), T, [&](int64_t lo, int64_t hi, int) {
        for (int64_t i = lo; i < hi; i++) {
            table[2 * i] = EMPTY_KEY;
            table[2 * i + 1] = 0;
        }
    });
    prog("counted distinct keys and cleared the table");
    {
        const uint64_t nb = h.nbuckets;
        const int log2b = h.log2b;
        std::vector<std::thread> th;
        for (int t = 0; t < T; t++)
            th.emplace_back([&, t]() {
                for (int64_t i = cut[t]; i < cut[t + 1];) {
                    int64_t j = i;
                    uint64_t nf = 0, nr = 0;
                    while (j < cut[t + 1] && recs[j].key == recs[i].key) {
                        if (recs[j].orient == 0) nf++; else nr++;
                        h.positions[j] = recs[j].q;
                        j++;
                    }
                    table_insert(table, nb, log2b, recs[i].key,
                                 ((uint64_t)i & OFF_MASK) | ((uint64_t)std::min<uint64_t>(nf, CNT_SAT) << 36) |
                                     ((uint64_t)std::min<uint64_t>(nr, CNT_SAT) << 50));
                    i = j;
                }
            });
        for (auto &x : th) x.join();
    }
    prog("grouped positions by key and filled the table");
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

template <class V>
int upload(const V &v, void **dptr) {
    using T = std::remove_cv_t<std::remove_reference_t<decltype(v[0])>>;
    size_t bytes = std::max<size_t>(v.size() * sizeof(T), 256);
    if (hipMalloc(dptr, bytes) != hipSuccess) { *dptr = nullptr; return SNAP_ENOMEM; }
    if (v.size() != 0 && hipMemcpy(*dptr, v.data(), v.size() * sizeof(T), hipMemcpyHostToDevice) != hipSuccess)
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
        case SNAP_EINTERNAL: return "internal consistency bound exceeded";
        case SNAP_ETOOBIG: return "batch needs more scratch than the fixed scratch array holds";
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
    if (ix->alloc_rep) (void)hipFree(ix->alloc_rep);
    if (ix->alloc_repbits) (void)hipFree(ix->alloc_repbits);
    (void)hipSetDevice(dev);
    delete ix;
    return SNAP_OK;
}

extern "C" int snap_index_build(const uint8_t *genome, uint64_t len, int32_t seed_len, snap_index **out) {
    return snap_index_build_progress(genome, len, seed_len, nullptr, nullptr, out);
}

extern "C" int snap_index_build_progress(const uint8_t *genome, uint64_t len, int32_t seed_len,
                                         snap_progress_fn progress, void *ctx, snap_index **out) {
    if (!out) return SNAP_EINVAL;
    const Progress prog{progress, ctx};
    *out = nullptr;
    if (!genome || seed_len < 1 || seed_len > 32 || len < (uint64_t)seed_len || len >= (1ull << 32))
        return SNAP_EINVAL;
    HostIndex h;
    int rc;
    try {
        rc = build_host(genome, len, seed_len, h, prog);
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
    prog("copied the index to the device");
    ix->d.gcode = (const uint32_t *)ix->alloc_gcode;
    ix->d.gmask = (const uint32_t *)ix->alloc_gmask;
    ix->d.table = (const uint64_t *)ix->alloc_table;
    ix->d.positions = (const uint32_t *)ix->alloc_pos;
    ix->d.G = h.G;
    ix->d.nbuckets = h.nbuckets;
    ix->d.log2_buckets = h.log2b;
    ix->d.s = seed_len;
    ix->d.stride = 1;
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
    info->stride = ix->d.stride;
    info->windows = ix->windows;
    info->distinct_keys = ix->distinct_keys;
    info->table_slots = ix->d.nbuckets * SLOTS_PER_BUCKET;
    info->position_entries = ix->position_entries;
    info->device_bytes = ix->device_bytes;
    info->device = ix->device;
    info->dup_window = ix->d.rep ? ix->d.dup_w : 0;
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
    int rc = build_host(genome, len, seed_len, h, Progress{nullptr, nullptr});
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
