// Seed index built on the device (Section 3.1: a hash table from every seed-length
// window of the genome to the positions where it occurs; Section 3.2, omitted aspect:
// forward and reverse-complement windows share one entry under the canonical code).
//
// Same result as the host build in index.hip (identical packed genome, N mask and
// positions array; the same table entries, each in the slot its compare-and-swap
// claimed), made with device kernels instead of host threads:
//   1. the genome is copied in and packed (2-bit codes, N mask);
//   2. every N-free window emits one record per orientation whose code is the canonical
//      one (two for a palindrome): sort key canonical << 1 | orientation, value the
//      window's position, in position order (counted per block, scanned, then written);
//   3. a stable device radix sort over the 2s + 1 key bits puts each key's forward
//      windows, then its reverse ones, in position order: the sorted values are the
//      positions array;
//   4. each run of equal canonical codes inserts one table entry (first record, forward
//      and reverse counts) by compare-and-swap on the slot's key word, probing buckets
//      linearly from the key's home bucket.
// Keys take 2s + 1 bits, so the device build takes seed lengths up to 31.

#include <algorithm>
#include <cstring>
#include <new>

#include <hip/hip_runtime.h>
#include <rocprim/device/device_radix_sort.hpp>
#include <rocprim/device/device_reduce.hpp>
#include <rocprim/device/device_scan.hpp>
#include <rocprim/iterator/transform_iterator.hpp>

#include "../../include/snapgpu.h"
#include "../../include/snapgpu_debug.h"
#include "snap_internal.h"

using namespace snapgpu;

namespace {

constexpr int EMIT_WPT = 16;                          // windows per thread
constexpr int EMIT_THREADS = 256;
constexpr int64_t EMIT_BLOCK = (int64_t)EMIT_WPT * EMIT_THREADS;

__device__ inline uint32_t dev_base_code(uint8_t b) {
    switch (b) {
        case 'A': case 'a': return 0;
        case 'C': case 'c': return 1;
        case 'G': case 'g': return 2;
        case 'T': case 't': return 3;
        default: return 4;
    }
}

// One thread per 4 bases (one 32-bit load of the genome), 8 threads per 32-base block:
// each contributes a byte of the two code words and 4 bits of the N-mask word, gathered
// by shuffles (N stored as 0). Bases past G are none.
__global__ __launch_bounds__(256) void k_pack_genome(const uint8_t *g, uint64_t G, uint32_t *gcode, uint32_t *gmask,
                                                     int64_t nblk) {
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;   // 4-base group
    const int64_t blk = t >> 3;
    const int part = (int)(t & 7);
    uint32_t code = 0, m = 0;
    if (blk < nblk) {
        const uint64_t j0 = (uint64_t)t * 4;
        uint32_t w = 0;
        if (j0 + 4 <= G) {
            w = *reinterpret_cast<const uint32_t *>(g + j0);   // the genome copy is 256-byte aligned
        } else {
            for (int k = 0; k < 4; k++) w |= (j0 + k < G ? (uint32_t)g[j0 + k] : (uint32_t)'A') << (8 * k);
        }
        for (int k = 0; k < 4; k++) {
            uint32_t c = dev_base_code((uint8_t)(w >> (8 * k)));
            const bool past = j0 + k >= G;
            if (c > 3 && !past) m |= 1u << k;
            if (c > 3 || past) c = 0;
            code |= c << (2 * k);
        }
    }
    // gather the 8 parts of a block (lanes 8b .. 8b+7 of the wave)
    const int lane = threadIdx.x & 63, b0 = lane & ~7;
    uint32_t c0 = 0, c1 = 0, mm = 0;
    for (int q = 0; q < 8; q++) {
        const uint32_t cq = (uint32_t)__shfl((int)code, b0 + q, 64), mq = (uint32_t)__shfl((int)m, b0 + q, 64);
        if (q < 4) c0 |= cq << (8 * q); else c1 |= cq << (8 * (q - 4));
        mm |= mq << (4 * q);
    }
    if (blk < nblk && part == 0) {
        gcode[2 * blk] = c0;
        gcode[2 * blk + 1] = c1;
        gmask[blk] = mm;
    }
}

// Forward code of the s bases at q (first base least significant) and whether any is N.
__device__ inline uint64_t window_code(const uint32_t *gcode, uint64_t q, int s) {
    const uint64_t w = q >> 4;
    const uint32_t sh = (uint32_t)(q & 15) * 2;
    const uint64_t lo = (uint64_t)gcode[w] | ((uint64_t)gcode[w + 1] << 32);
    const uint64_t hi = gcode[w + 2];
    const uint64_t v = sh ? ((lo >> sh) | (hi << (64 - sh))) : lo;
    return v & seed_mask(s);
}
__device__ inline bool window_has_n(const uint32_t *gmask, uint64_t q, int s) {
    const uint64_t w = q >> 5;
    const uint64_t v = ((uint64_t)gmask[w] | ((uint64_t)gmask[w + 1] << 32)) >> (q & 31);
    return (v & ((1ull << s) - 1)) != 0;
}

// The records window q gives: bit 0 forward (its code is canonical), bit 1 reverse
// (its reverse complement is), none if it holds an N, lies past the last window or is
// not at a multiple of the index's stride (Section 3.1's footnote: a window slid
// `stride` bases at a time; stride 1 indexes every overlapping window).
__device__ inline uint32_t window_records(const uint32_t *gcode, const uint32_t *gmask, uint64_t q, uint64_t nwin,
                                          int s, uint32_t stride, uint64_t &canon) {
    if (q >= nwin || (stride > 1 && q % stride != 0) || window_has_n(gmask, q, s)) return 0;
    const uint64_t fw = window_code(gcode, q, s), rc = rc_code(fw, s);
    canon = fw < rc ? fw : rc;
    return (fw == canon ? 1u : 0u) | (rc == canon ? 2u : 0u);
}

// A block's 4096 windows: wave w of the block takes windows [1024 w, 1024 (w + 1)) of
// it, 64 at a time, lane l the l-th (so a wave's loads and stores are contiguous).
__device__ inline uint64_t emit_window(int k) {
    return (uint64_t)blockIdx.x * EMIT_BLOCK + (uint64_t)(threadIdx.x >> 6) * (EMIT_WPT * 64) + (uint64_t)k * 64 +
           (threadIdx.x & 63);
}

// Pass 1: per block, the records its windows give (low 32 bits) and its N-free windows
// (high 32 bits).
__global__ __launch_bounds__(EMIT_THREADS) void k_count_records(const uint32_t *gcode, const uint32_t *gmask,
                                                                uint64_t nwin, int s, uint32_t stride,
                                                                uint64_t *block_counts) {
    uint32_t recs = 0, free_w = 0;
    for (int k = 0; k < EMIT_WPT; k++) {
        uint64_t canon = 0;
        const uint32_t f = window_records(gcode, gmask, emit_window(k), nwin, s, stride, canon);
        recs += (f & 1) + (f >> 1);
        free_w += f ? 1 : 0;
    }
    __shared__ uint32_t sr[EMIT_THREADS], sf[EMIT_THREADS];
    sr[threadIdx.x] = recs;
    sf[threadIdx.x] = free_w;
    __syncthreads();
    for (int o = EMIT_THREADS / 2; o > 0; o >>= 1) {
        if ((int)threadIdx.x < o) {
            sr[threadIdx.x] += sr[threadIdx.x + o];
            sf[threadIdx.x] += sf[threadIdx.x + o];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) block_counts[blockIdx.x] = (uint64_t)sr[0] | ((uint64_t)sf[0] << 32);
}

// Pass 2: the same windows write their records at the block's offset (exclusive scan
// of the block counts) in window order: waves in order, and within a wave 64 windows at
// a time, each lane's records placed after those of the lanes before it (ballots).
__global__ __launch_bounds__(EMIT_THREADS) void k_emit_records(const uint32_t *gcode, const uint32_t *gmask,
                                                               uint64_t nwin, int s, uint32_t stride,
                                                               const uint64_t *block_off, uint64_t *keys,
                                                               uint32_t *vals) {
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    uint32_t recs = 0;
    for (int k = 0; k < EMIT_WPT; k++) {
        uint64_t canon = 0;
        const uint32_t f = window_records(gcode, gmask, emit_window(k), nwin, s, stride, canon);
        recs += (f & 1) + (f >> 1);
    }
    for (int o = 32; o > 0; o >>= 1) recs += (uint32_t)__shfl_xor((int)recs, o, 64);
    __shared__ uint32_t wave_recs[EMIT_THREADS / 64];
    if (lane == 0) wave_recs[wv] = recs;
    __syncthreads();
    uint64_t at = block_off[blockIdx.x];
    for (int w = 0; w < wv; w++) at += wave_recs[w];
    const uint64_t below = (1ull << lane) - 1;
    for (int k = 0; k < EMIT_WPT; k++) {
        const uint64_t q = emit_window(k);
        uint64_t canon = 0;
        const uint32_t f = window_records(gcode, gmask, q, nwin, s, stride, canon);
        const uint64_t b0 = __ballot(f & 1), b1 = __ballot(f & 2);
        uint64_t my = at + __popcll(b0 & below) + __popcll(b1 & below);
        if (f & 1) { keys[my] = canon << 1; vals[my] = (uint32_t)q; my++; }
        if (f & 2) { keys[my] = (canon << 1) | 1; vals[my] = (uint32_t)q; }
        at += __popcll(b0) + __popcll(b1);
    }
}

// Record i starts a run of equal canonical codes.
__device__ inline bool run_start(const uint64_t *keys, uint64_t i) {
    return i == 0 || (keys[i] >> 1) != (keys[i - 1] >> 1);
}

__global__ void k_count_runs(const uint64_t *keys, uint64_t n, unsigned long long *runs) {
    uint32_t c = 0;
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (uint64_t)gridDim.x * blockDim.x)
        c += run_start(keys, i) ? 1u : 0u;
    for (int o = 32; o > 0; o >>= 1) c += __shfl_xor(c, o, 64);
    if ((threadIdx.x & 63) == 0 && c) atomicAdd(runs, (unsigned long long)c);
}

__global__ void k_clear_table(uint64_t *table, uint64_t nslots) {
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < nslots; i += (uint64_t)gridDim.x * blockDim.x) {
        table[2 * i] = EMPTY_KEY;
        table[2 * i + 1] = 0;
    }
}

// One thread per record; the first record of each run counts the run's forward and
// reverse records and inserts the entry. A probe that finds no free slot in every
// bucket (impossible at load 0.7, so a corrupted table) sets *fail and stops.
__global__ void k_insert_runs(const uint64_t *keys, uint64_t n, uint64_t *table, uint64_t nbuckets, int log2b,
                              unsigned int *fail) {
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (uint64_t)gridDim.x * blockDim.x) {
        if (!run_start(keys, i)) continue;
        const uint64_t key = keys[i] >> 1;
        uint64_t j = i;
        while (j < n && keys[j] == (key << 1)) j++;
        uint64_t e = j;
        while (e < n && keys[e] == ((key << 1) | 1)) e++;
        const uint64_t nf = j - i, nr = e - j;
        const uint64_t val = (i & OFF_MASK) | ((nf < CNT_SAT ? nf : (uint64_t)CNT_SAT) << 36) |
                             ((nr < CNT_SAT ? nr : (uint64_t)CNT_SAT) << 50);
        uint64_t b = home_bucket(key, log2b);
        bool done = false;
        for (uint64_t step = 0; step < nbuckets && !done; step++) {
            for (int k = 0; k < SLOTS_PER_BUCKET && !done; k++) {
                unsigned long long *slot = reinterpret_cast<unsigned long long *>(table + 2 * (b * SLOTS_PER_BUCKET + k));
                // a slot never goes back to empty, so a stale read can only send us to a
                // compare-and-swap that fails
                if (*slot == (unsigned long long)EMPTY_KEY &&
                    atomicCAS(slot, (unsigned long long)EMPTY_KEY, (unsigned long long)key) ==
                        (unsigned long long)EMPTY_KEY) {
                    slot[1] = val;
                    done = true;
                }
            }
            b = (b + 1) & (nbuckets - 1);
        }
        if (!done) atomicOr(fail, 1u);
    }
}

// The two counts packed in a block's word.
struct LowHalf {
    __host__ __device__ uint64_t operator()(uint64_t v) const { return v & 0xFFFFFFFFull; }
};
struct HighHalf {
    __host__ __device__ uint64_t operator()(uint64_t v) const { return v >> 32; }
};

// Device allocations of one build, freed on every exit unless handed to the index.
struct DevBuf {
    void *p = nullptr;
    ~DevBuf() { if (p) (void)hipFree(p); }
    int alloc(size_t bytes) {
        if (hipMalloc(&p, std::max<size_t>(bytes, 256)) != hipSuccess) { p = nullptr; return SNAP_ENOMEM; }
        return SNAP_OK;
    }
    void *release() { void *q = p; p = nullptr; return q; }
};

#define DEV_OK(x) do { if ((x) != hipSuccess) return SNAP_EDEVICE; } while (0)
#define RC_OK(x) do { const int rc_ = (x); if (rc_ != SNAP_OK) return rc_; } while (0)

// Stage reports of a build (stage text, null callback allowed).
struct DevProgress {
    snap_progress_fn fn;
    void *ctx;
    void operator()(const char *stage) const {
        if (fn) fn(stage, ctx);
    }
};

int build_device(const uint8_t *genome, uint64_t G, int s, uint32_t stride, hipStream_t st, const DevProgress &prog,
                 snap_index *ix) {
    const uint64_t ncw = (G + 15) / 16 + GENOME_PAD_WORDS, nmw = (G + 31) / 32 + GENOME_PAD_WORDS;
    const int64_t nblk = (int64_t)((G + 31) / 32);
    DevBuf dg, gcode, gmask;
    RC_OK(dg.alloc(G));
    RC_OK(gcode.alloc(ncw * 4));
    RC_OK(gmask.alloc(nmw * 4));
    DEV_OK(hipMemcpyAsync(dg.p, genome, G, hipMemcpyHostToDevice, st));
    DEV_OK(hipMemsetAsync(gcode.p, 0, ncw * 4, st));
    DEV_OK(hipMemsetAsync(gmask.p, 0, nmw * 4, st));
    hipLaunchKernelGGL(k_pack_genome, dim3((unsigned)((nblk * 8 + 255) / 256)), dim3(256), 0, st, (const uint8_t *)dg.p,
                       G, (uint32_t *)gcode.p, (uint32_t *)gmask.p, nblk);
    DEV_OK(hipGetLastError());
    DEV_OK(hipStreamSynchronize(st));
    (void)hipFree(dg.release());
    prog("copied the genome in and packed it");
    const uint32_t *gc = (const uint32_t *)gcode.p, *gm = (const uint32_t *)gmask.p;

    // records: count, scan, emit
    const uint64_t nwin = G - (uint64_t)s + 1;
    const uint64_t nb = (nwin + EMIT_BLOCK - 1) / EMIT_BLOCK;
    DevBuf bcnt, boff, total;
    RC_OK(bcnt.alloc(nb * 8));
    RC_OK(boff.alloc(nb * 8));
    RC_OK(total.alloc(16));
    hipLaunchKernelGGL(k_count_records, dim3((unsigned)nb), dim3(EMIT_THREADS), 0, st, gc, gm, nwin, s, stride,
                       (uint64_t *)bcnt.p);
    DEV_OK(hipGetLastError());
    uint64_t sums[2] = {0, 0};   // records, N-free windows
    {
        // exclusive scan of the record counts; the total of each field from a reduction
        const uint64_t *bc = (const uint64_t *)bcnt.p;
        auto recs = rocprim::make_transform_iterator(bc, LowHalf{});
        auto wins = rocprim::make_transform_iterator(bc, HighHalf{});
        size_t tb1 = 0, tb2 = 0;
        DEV_OK(rocprim::exclusive_scan(nullptr, tb1, recs, (uint64_t *)boff.p, (uint64_t)0, (size_t)nb,
                                       rocprim::plus<uint64_t>(), st));
        DEV_OK(rocprim::reduce(nullptr, tb2, wins, (uint64_t *)total.p + 1, (uint64_t)0, (size_t)nb,
                               rocprim::plus<uint64_t>(), st));
        DevBuf tmp;
        RC_OK(tmp.alloc(std::max(tb1, tb2)));
        DEV_OK(rocprim::exclusive_scan(tmp.p, tb1, recs, (uint64_t *)boff.p, (uint64_t)0, (size_t)nb,
                                       rocprim::plus<uint64_t>(), st));
        DEV_OK(rocprim::reduce(tmp.p, tb2, wins, (uint64_t *)total.p + 1, (uint64_t)0, (size_t)nb,
                               rocprim::plus<uint64_t>(), st));
        uint64_t last_off = 0, last_cnt = 0;
        DEV_OK(hipMemcpyAsync(&last_off, (uint64_t *)boff.p + (nb - 1), 8, hipMemcpyDeviceToHost, st));
        DEV_OK(hipMemcpyAsync(&last_cnt, bc + (nb - 1), 8, hipMemcpyDeviceToHost, st));
        DEV_OK(hipMemcpyAsync(&sums[1], (uint64_t *)total.p + 1, 8, hipMemcpyDeviceToHost, st));
        DEV_OK(hipStreamSynchronize(st));
        sums[0] = last_off + (last_cnt & 0xFFFFFFFFull);
    }
    const uint64_t nrec = sums[0];
    (void)hipFree(bcnt.release());
    DevBuf k0, k1, v0, v1;
    RC_OK(k0.alloc(nrec * 8));
    RC_OK(k1.alloc(nrec * 8));
    RC_OK(v0.alloc(nrec * 4));
    RC_OK(v1.alloc(nrec * 4));
    hipLaunchKernelGGL(k_emit_records, dim3((unsigned)nb), dim3(EMIT_THREADS), 0, st, gc, gm, nwin, s, stride,
                       (const uint64_t *)boff.p, (uint64_t *)k0.p, (uint32_t *)v0.p);
    DEV_OK(hipGetLastError());
    DEV_OK(hipStreamSynchronize(st));
    (void)hipFree(boff.release());
    prog("emitted the window records");

    // stable sort over the canonical code and orientation bits
    rocprim::double_buffer<uint64_t> kb((uint64_t *)k0.p, (uint64_t *)k1.p);
    rocprim::double_buffer<uint32_t> vb((uint32_t *)v0.p, (uint32_t *)v1.p);
    {
        size_t tb = 0;
        DEV_OK(rocprim::radix_sort_pairs(nullptr, tb, kb, vb, (size_t)nrec, 0u, (unsigned)(2 * s + 1), st));
        DevBuf tmp;
        RC_OK(tmp.alloc(tb));
        DEV_OK(rocprim::radix_sort_pairs(tmp.p, tb, kb, vb, (size_t)nrec, 0u, (unsigned)(2 * s + 1), st));
        DEV_OK(hipStreamSynchronize(st));
    }
    DevBuf *keys_buf = kb.current() == (uint64_t *)k0.p ? &k0 : &k1;
    DevBuf *pos_buf = vb.current() == (uint32_t *)v0.p ? &v0 : &v1;
    (void)hipFree((keys_buf == &k0 ? k1 : k0).release());
    (void)hipFree((pos_buf == &v0 ? v1 : v0).release());
    prog("sorted the records");
    const uint64_t *keys = (const uint64_t *)keys_buf->p;

    // distinct codes, table size as in the host build, then one insertion per run
    unsigned long long *runs = (unsigned long long *)total.p;
    DEV_OK(hipMemsetAsync(runs, 0, 8, st));
    hipLaunchKernelGGL(k_count_runs, dim3(4096), dim3(256), 0, st, keys, nrec, runs);
    DEV_OK(hipGetLastError());
    uint64_t distinct = 0;
    DEV_OK(hipMemcpyAsync(&distinct, runs, 8, hipMemcpyDeviceToHost, st));
    DEV_OK(hipStreamSynchronize(st));
    const uint64_t need = (uint64_t)((double)distinct / (0.7 * SLOTS_PER_BUCKET)) + 1;
    int log2b = 0;
    while ((1ull << log2b) < need) log2b++;
    const uint64_t nbuckets = 1ull << log2b;
    DevBuf table;
    RC_OK(table.alloc(nbuckets * SLOTS_PER_BUCKET * 16));
    hipLaunchKernelGGL(k_clear_table, dim3(8192), dim3(256), 0, st, (uint64_t *)table.p, nbuckets * SLOTS_PER_BUCKET);
    DEV_OK(hipGetLastError());
    unsigned int *fail = (unsigned int *)((uint64_t *)total.p + 1);
    DEV_OK(hipMemsetAsync(fail, 0, 4, st));
    hipLaunchKernelGGL(k_insert_runs, dim3(8192), dim3(256), 0, st, keys, nrec, (uint64_t *)table.p, nbuckets, log2b,
                       fail);
    DEV_OK(hipGetLastError());
    unsigned int failed = 0;
    DEV_OK(hipMemcpyAsync(&failed, fail, 4, hipMemcpyDeviceToHost, st));
    DEV_OK(hipStreamSynchronize(st));
    if (failed) return SNAP_EDEVICE;
    (void)hipFree(keys_buf->release());
    prog("filled the table");

    ix->d.G = G;
    ix->d.s = s;
    ix->d.stride = (int32_t)stride;
    ix->d.nbuckets = nbuckets;
    ix->d.log2_buckets = log2b;
    ix->windows = sums[1];
    ix->distinct_keys = distinct;
    ix->position_entries = nrec;
    ix->device_bytes = ncw * 4 + nmw * 4 + nbuckets * SLOTS_PER_BUCKET * 16 + nrec * 4;
    ix->alloc_gcode = gcode.release();
    ix->alloc_gmask = gmask.release();
    ix->alloc_table = table.release();
    ix->alloc_pos = pos_buf->release();
    ix->d.gcode = (const uint32_t *)ix->alloc_gcode;
    ix->d.gmask = (const uint32_t *)ix->alloc_gmask;
    ix->d.table = (const uint64_t *)ix->alloc_table;
    ix->d.positions = (const uint32_t *)ix->alloc_pos;
    return SNAP_OK;
}

}  // namespace

extern "C" int snap_index_build_strided(const uint8_t *genome, uint64_t len, int32_t seed_len, int32_t stride,
                                        void *stream, snap_progress_fn progress, void *ctx, snap_index **out) {
    if (!out) return SNAP_EINVAL;
    *out = nullptr;
    if (!genome || seed_len < 1 || seed_len > 31 || len < (uint64_t)seed_len || len >= (1ull << 32))
        return SNAP_EINVAL;
    if (stride != 1 && stride != 2 && stride != 4) return SNAP_EINVAL;
    snap_index *ix = new (std::nothrow) snap_index();
    if (!ix) return SNAP_ENOMEM;
    if (hipGetDevice(&ix->device) != hipSuccess) { delete ix; return SNAP_EDEVICE; }
    const int rc = build_device(genome, len, seed_len, (uint32_t)stride, (hipStream_t)stream,
                                DevProgress{progress, ctx}, ix);
    if (rc != SNAP_OK) {
        (void)hipStreamSynchronize((hipStream_t)stream);
        snap_index_free(ix);
        return rc;
    }
    *out = ix;
    return SNAP_OK;
}

extern "C" int snap_index_build_device(const uint8_t *genome, uint64_t len, int32_t seed_len, void *stream,
                                       snap_progress_fn progress, void *ctx, snap_index **out) {
    return snap_index_build_strided(genome, len, seed_len, 1, stream, progress, ctx, out);
}

extern "C" int snap_debug_index_download(const snap_index *ix, int32_t which, void *host_dst, uint64_t bytes) {
    if (!ix || !host_dst) return SNAP_EINVAL;
    const void *src = nullptr;
    uint64_t have = 0;
    const uint64_t G = ix->d.G;
    switch (which) {
        case 0: src = ix->d.gcode; have = ((G + 15) / 16 + GENOME_PAD_WORDS) * 4; break;
        case 1: src = ix->d.gmask; have = ((G + 31) / 32 + GENOME_PAD_WORDS) * 4; break;
        case 2: src = ix->d.table; have = ix->d.nbuckets * SLOTS_PER_BUCKET * 16; break;
        case 3: src = ix->d.positions; have = ix->position_entries * 4; break;
        default: return SNAP_EINVAL;
    }
    if (bytes != have) return SNAP_EINVAL;
    if (bytes && hipMemcpy(host_dst, src, bytes, hipMemcpyDeviceToHost) != hipSuccess) return SNAP_EDEVICE;
    return SNAP_OK;
}
