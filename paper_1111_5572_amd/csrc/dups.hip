// Exact-duplicate classes of the genome's W-base windows (Section 4.2, "Approach":
// identical substrings of a read's length are found by hashing them, so that a read is
// compared with each repeated string once).
//
// rep[q] is the smallest position whose W-base window is identical to q's (bases as
// codes, an N equal to every N; identical only as a whole window), q itself when no
// earlier one is, and q for a position whose window runs past the genome's end. Two
// locations of one read on one strand whose positions share a class have identical
// text windows for any read with L + limit <= W, so one edit distance answers both.
//
// Built on the device from the index's packed genome:
//   1. a 64-bit polynomial hash of every complete window (a thread hashes its first
//      window directly and rolls the hash over the next ones);
//   2. a stable radix sort of (hash, position): equal hashes form runs, each in
//      position order;
//   3. every element finds its run's first element (a max scan of run starts) and
//      compares its window with that one, word by word: equal windows take the run
//      head's position as their class;
//   4. elements whose window differs from their run head's (a hash collision) are
//      listed and each compared with the earlier listed members of its run: the first
//      identical one is its class, else it is its own. No hash collision is trusted.
// Memory while building: 24 bytes per window (keys and positions, double buffered),
// freed before returning; the class array (4 bytes per base) and a bit map of the
// positions whose class is another position (1 bit per base) stay with the index.

#include <algorithm>
#include <new>

#include <hip/hip_runtime.h>
#include <rocprim/device/device_radix_sort.hpp>
#include <rocprim/device/device_scan.hpp>
#include <rocprim/device/device_select.hpp>
#include <rocprim/iterator/counting_iterator.hpp>
#include <rocprim/iterator/transform_iterator.hpp>

#include "../../include/snapgpu.h"
#include "../../include/snapgpu_debug.h"
#include "snap_internal.h"

using namespace snapgpu;

namespace {

constexpr uint64_t HASH_BASE = 0x9E3779B97F4A7C15ull;   // odd multiplier of the polynomial hash
constexpr int HASH_RUN = 256;                              // windows hashed per thread

// Base q as a symbol: its 2-bit code, or 4 for an N.
__device__ inline uint64_t base_sym(const uint32_t *gcode, const uint32_t *gmask, uint64_t q) {
    if ((gmask[q >> 5] >> (q & 31)) & 1u) return 4;
    return (gcode[q >> 4] >> (2 * (q & 15))) & 3u;
}

// Hash of window q: sum of sym(q + i) * B^(W - 1 - i) mod 2^64, rolled from q to q + 1 by
// h' = (h - sym(q) * B^(W-1)) * B + sym(q + W).
__global__ void k_hash_windows(const uint32_t *gcode, const uint32_t *gmask, uint64_t nwin, int64_t W, uint64_t bw1,
                               uint64_t *keys, uint32_t *vals) {
    const uint64_t t = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const uint64_t q0 = t * HASH_RUN;
    if (q0 >= nwin) return;
    uint64_t h = 0;
    for (int64_t i = 0; i < W; i++) h = h * HASH_BASE + base_sym(gcode, gmask, q0 + (uint64_t)i);
    const uint64_t q1 = min(nwin, q0 + HASH_RUN);
    for (uint64_t q = q0;; q++) {
        keys[q] = h;
        vals[q] = (uint32_t)q;
        if (q + 1 >= q1) break;
        h = (h - base_sym(gcode, gmask, q) * bw1) * HASH_BASE + base_sym(gcode, gmask, q + (uint64_t)W);
    }
}

__global__ void k_identity(uint32_t *rep, uint64_t G) {
    for (uint64_t q = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; q < G; q += (uint64_t)gridDim.x * blockDim.x)
        rep[q] = (uint32_t)q;
}

// Element i starts a run of equal hashes: its own index, else 0 (a max scan then gives
// every element its run head).
struct RunStart {
    const uint64_t *keys;
    __host__ __device__ uint32_t operator()(uint32_t i) const { return (i == 0 || keys[i] != keys[i - 1]) ? i : 0u; }
};
struct MaxU32 {
    __host__ __device__ uint32_t operator()(uint32_t a, uint32_t b) const { return a > b ? a : b; }
};

// The W bases at a and at b are identical (codes and N flags).
__device__ inline bool same_window(const uint32_t *gcode, const uint32_t *gmask, uint64_t a, uint64_t b, int64_t W) {
    for (int64_t i = 0; i < W;) {
        // up to 16 bases at a time from each side (2-bit codes), and their N flags
        const int n = (int)min<int64_t>(16, W - i);
        const uint64_t pa = a + (uint64_t)i, pb = b + (uint64_t)i;
        auto codes = [&](uint64_t p) {
            const uint64_t w = p >> 4;
            const uint32_t sh = (uint32_t)(p & 15) * 2;
            const uint64_t v = (uint64_t)gcode[w] | ((uint64_t)gcode[w + 1] << 32);
            return (uint32_t)(v >> sh);
        };
        auto nbits = [&](uint64_t p) {
            const uint64_t w = p >> 5;
            const uint64_t v = (uint64_t)gmask[w] | ((uint64_t)gmask[w + 1] << 32);
            return (uint32_t)(v >> (p & 31));
        };
        const uint32_t cm = n == 16 ? 0xFFFFFFFFu : ((1u << (2 * n)) - 1u);
        const uint32_t nm = n == 32 ? 0xFFFFFFFFu : ((1u << n) - 1u);
        const uint32_t na = nbits(pa) & nm, nb = nbits(pb) & nm;
        if (na != nb) return false;
        // an N is stored as code 0 on both sides, so codes compare equal there
        if ((codes(pa) & cm) != (codes(pb) & cm)) return false;
        i += n;
    }
    return true;
}

// Every sorted element: equal to its run head's window -> the head's position is its
// class; otherwise it is flagged for the collision pass.
__global__ void k_classes(const uint32_t *gcode, const uint32_t *gmask, const uint32_t *vals, const uint32_t *head,
                          uint64_t n, int64_t W, uint32_t *rep, uint8_t *mismatch) {
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (uint64_t)gridDim.x * blockDim.x) {
        const uint32_t h = head[i];
        bool mis = false;
        if (h != (uint32_t)i) {
            const uint32_t q = vals[i], qh = vals[h];
            if (same_window(gcode, gmask, q, qh, W)) rep[q] = qh;
            else mis = true;
        }
        mismatch[i] = mis ? 1 : 0;
    }
}

// The listed elements (ascending), each compared with the earlier listed members of its
// run; the first identical one gives its class.
__global__ void k_collisions(const uint32_t *gcode, const uint32_t *gmask, const uint32_t *vals, const uint32_t *head,
                             const uint32_t *list, const uint32_t *nlist, int64_t W, uint32_t *rep) {
    const uint32_t m = *nlist;
    for (uint32_t u = blockIdx.x * blockDim.x + threadIdx.x; u < m; u += gridDim.x * blockDim.x) {
        const uint32_t i = list[u];
        for (uint32_t v = 0; v < u; v++) {
            const uint32_t j = list[v];
            if (head[j] == head[i] && same_window(gcode, gmask, vals[i], vals[j], W)) {
                rep[vals[i]] = vals[j];
                break;
            }
        }
    }
}

// Bit q of the map: position q's class is another position (rep[q] != q). The alignment
// reads this map first (32 times smaller than the class array, mostly cache-resident)
// and the class array only where the bit is set.
__global__ void k_dup_bits(const uint32_t *rep, uint64_t G, uint32_t *bits, uint64_t nwords) {
    for (uint64_t w = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; w < nwords; w += (uint64_t)gridDim.x * blockDim.x) {
        uint32_t v = 0;
        for (int b = 0; b < 32; b++) {
            const uint64_t q = w * 32 + (uint64_t)b;
            if (q < G && rep[q] != (uint32_t)q) v |= 1u << b;
        }
        bits[w] = v;
    }
}

struct Buf {
    void *p = nullptr;
    ~Buf() { if (p) (void)hipFree(p); }
    int alloc(size_t bytes) {
        if (hipMalloc(&p, std::max<size_t>(bytes, 256)) != hipSuccess) { p = nullptr; return SNAP_ENOMEM; }
        return SNAP_OK;
    }
    void *release() { void *q = p; p = nullptr; return q; }
};

#define DEV_OK(x) do { if ((x) != hipSuccess) return SNAP_EDEVICE; } while (0)
#define RC_OK(x) do { const int rc_ = (x); if (rc_ != SNAP_OK) return rc_; } while (0)

int build_classes(snap_index *ix, int64_t W, hipStream_t st) {
    const uint64_t G = ix->d.G;
    Buf rep;
    RC_OK(rep.alloc(G * 4));
    hipLaunchKernelGGL(k_identity, dim3(8192), dim3(256), 0, st, (uint32_t *)rep.p, G);
    DEV_OK(hipGetLastError());
    if ((uint64_t)W <= G) {
        const uint64_t nwin = G - (uint64_t)W + 1;
        Buf k0, k1, v0, v1;
        RC_OK(k0.alloc(nwin * 8));
        RC_OK(k1.alloc(nwin * 8));
        RC_OK(v0.alloc(nwin * 4));
        RC_OK(v1.alloc(nwin * 4));
        uint64_t bw1 = 1;
        for (int64_t i = 1; i < W; i++) bw1 *= HASH_BASE;
        const uint64_t nthr = (nwin + HASH_RUN - 1) / HASH_RUN;
        hipLaunchKernelGGL(k_hash_windows, dim3((unsigned)((nthr + 255) / 256)), dim3(256), 0, st, ix->d.gcode,
                           ix->d.gmask, nwin, W, bw1, (uint64_t *)k0.p, (uint32_t *)v0.p);
        DEV_OK(hipGetLastError());
        rocprim::double_buffer<uint64_t> kb((uint64_t *)k0.p, (uint64_t *)k1.p);
        rocprim::double_buffer<uint32_t> vb((uint32_t *)v0.p, (uint32_t *)v1.p);
        {
            size_t tb = 0;
            DEV_OK(rocprim::radix_sort_pairs(nullptr, tb, kb, vb, (size_t)nwin, 0u, 64u, st));
            Buf tmp;
            RC_OK(tmp.alloc(tb));
            DEV_OK(rocprim::radix_sort_pairs(tmp.p, tb, kb, vb, (size_t)nwin, 0u, 64u, st));
            DEV_OK(hipStreamSynchronize(st));
        }
        const uint64_t *keys = kb.current();
        const uint32_t *vals = vb.current();
        // run heads into the spare key buffer's memory (4 bytes per element of its 8)
        uint32_t *head = (uint32_t *)(keys == (const uint64_t *)k0.p ? k1.p : k0.p);
        uint8_t *mis = (uint8_t *)(vals == (const uint32_t *)v0.p ? v1.p : v0.p);
        {
            rocprim::counting_iterator<uint32_t> ci(0);
            auto starts = rocprim::make_transform_iterator(ci, RunStart{keys});
            size_t tb = 0;
            DEV_OK(rocprim::inclusive_scan(nullptr, tb, starts, head, (size_t)nwin, MaxU32{}, st));
            Buf tmp;
            RC_OK(tmp.alloc(tb));
            DEV_OK(rocprim::inclusive_scan(tmp.p, tb, starts, head, (size_t)nwin, MaxU32{}, st));
            hipLaunchKernelGGL(k_classes, dim3(16384), dim3(256), 0, st, ix->d.gcode, ix->d.gmask, vals, head, nwin, W,
                               (uint32_t *)rep.p, mis);
            DEV_OK(hipGetLastError());
            DEV_OK(hipStreamSynchronize(st));
        }
        {
            // the mismatched elements, in order; their list reuses the head buffer's tail
            Buf lst, cnt;
            RC_OK(lst.alloc(nwin * 4));
            RC_OK(cnt.alloc(16));
            rocprim::counting_iterator<uint32_t> ci(0);
            size_t tb = 0;
            DEV_OK(rocprim::select(nullptr, tb, ci, mis, (uint32_t *)lst.p, (uint32_t *)cnt.p, (size_t)nwin, st));
            Buf tmp;
            RC_OK(tmp.alloc(tb));
            DEV_OK(rocprim::select(tmp.p, tb, ci, mis, (uint32_t *)lst.p, (uint32_t *)cnt.p, (size_t)nwin, st));
            hipLaunchKernelGGL(k_collisions, dim3(64), dim3(256), 0, st, ix->d.gcode, ix->d.gmask, vals, head,
                               (const uint32_t *)lst.p, (const uint32_t *)cnt.p, W, (uint32_t *)rep.p);
            DEV_OK(hipGetLastError());
            uint32_t ncol = 0;
            DEV_OK(hipMemcpyAsync(&ncol, cnt.p, 4, hipMemcpyDeviceToHost, st));
            DEV_OK(hipStreamSynchronize(st));
            ix->dup_collisions = ncol;
        }
    } else {
        DEV_OK(hipStreamSynchronize(st));
        ix->dup_collisions = 0;
    }
    const uint64_t nwords = (G + 31) / 32;
    Buf bits;
    RC_OK(bits.alloc(nwords * 4));
    hipLaunchKernelGGL(k_dup_bits, dim3(8192), dim3(256), 0, st, (const uint32_t *)rep.p, G, (uint32_t *)bits.p, nwords);
    DEV_OK(hipGetLastError());
    DEV_OK(hipStreamSynchronize(st));
    if (ix->alloc_rep) (void)hipFree(ix->alloc_rep);
    if (ix->alloc_repbits) (void)hipFree(ix->alloc_repbits);
    ix->alloc_rep = rep.release();
    ix->alloc_repbits = bits.release();
    ix->d.rep = (const uint32_t *)ix->alloc_rep;
    ix->d.repbits = (const uint32_t *)ix->alloc_repbits;
    ix->d.dup_w = (int32_t)W;
    ix->device_bytes += ix->rep_bytes ? 0 : G * 4 + nwords * 4;
    ix->rep_bytes = G * 4 + nwords * 4;
    return SNAP_OK;
}

}  // namespace

extern "C" int snap_index_dup_classes(snap_index *ix, int32_t window, void *stream) {
    if (!ix || window < 1) return SNAP_EINVAL;
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return SNAP_EDEVICE;
    if (dev != ix->device) return SNAP_EINVAL;
    return build_classes(ix, window, (hipStream_t)stream);
}

extern "C" int snap_debug_dup_download(const snap_index *ix, uint32_t *host_dst, uint64_t count) {
    if (!ix || !host_dst || !ix->d.rep || count != ix->d.G) return SNAP_EINVAL;
    if (hipMemcpy(host_dst, ix->d.rep, count * 4, hipMemcpyDeviceToHost) != hipSuccess) return SNAP_EDEVICE;
    return SNAP_OK;
}
