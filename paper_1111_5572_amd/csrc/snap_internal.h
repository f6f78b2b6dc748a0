// Internal layout shared by the index builder and the alignment kernels.
//
// HBM layout of an index (all arrays device-resident for the index lifetime):
//   gcode     2-bit genome, 16 bases per uint32, base j at bits 2*(j%16) of word j/16
//             (A=0 C=1 G=2 T=3, N stored as 0), padded with 4 zero words
//   gmask     N mask, 1 bit per base, 32 bases per uint32, padded with 4 zero words
//   table     open-addressing seed table: 2^log2_buckets buckets of 8 slots of 16 bytes
//             (one 128-byte line per bucket), linear probing over buckets
//   positions uint32 genome positions; each key owns [off, off+nf) windows equal to the
//             key followed by [off+nf, off+nf+nr) windows equal to its reverse complement
//
// A table slot is two uint64 words:
//   key  the canonical seed, min(forward code, reverse-complement code), or EMPTY_KEY
//   val  off (bits 0..35) | min(nf, 16383) << 36 | min(nr, 16383) << 50
// A seed's code is base k at bits 2k (first base least significant).
#pragma once

#include <stdint.h>

namespace snapgpu {

constexpr uint64_t EMPTY_KEY = ~0ull;   // never canonical: RC of all-T is all-A
constexpr int SLOTS_PER_BUCKET = 8;
constexpr uint64_t OFF_MASK = (1ull << 36) - 1;
constexpr uint32_t CNT_SAT = 16383;
constexpr int GENOME_PAD_WORDS = 4;
constexpr int MAX_HITS_LIMIT = 16382;   // saturated counts stay above any allowed h_max
constexpr int MAX_SEEDS = 32;           // n_cap limit (one mask bit per seed slot)

struct DevIndex {
    const uint32_t *gcode;
    const uint32_t *gmask;
    const uint64_t *table;       // 2 words per slot
    const uint32_t *positions;
    uint64_t G;
    uint64_t nbuckets;
    int32_t log2_buckets;
    int32_t s;
    int32_t stride;              // windows at positions q with q % stride == 0 are indexed
    const uint32_t *rep;         // exact-duplicate class of each position's dup_w-base window, or null
    const uint32_t *repbits;     // bit q: rep[q] != q
    int32_t dup_w;
};

// 64-bit finalizer (MurmurHash3 fmix64, Appleby): spreads a seed code over the table.
#if defined(__HIPCC__)
__host__ __device__
#endif
inline uint64_t mix64(uint64_t k) {
    k ^= k >> 33;
    k *= 0xff51afd7ed558ccdull;
    k ^= k >> 33;
    k *= 0xc4ceb9fe1a85ec53ull;
    k ^= k >> 33;
    return k;
}

#if defined(__HIPCC__)
__host__ __device__
#endif
inline uint64_t home_bucket(uint64_t key, int log2_buckets) {
    return log2_buckets == 0 ? 0 : (mix64(key) >> (64 - log2_buckets));
}

#if defined(__HIPCC__)
__host__ __device__
#endif
inline uint64_t seed_mask(int s) { return s >= 32 ? ~0ull : ((1ull << (2 * s)) - 1); }

// Reverse complement of an s-base code (first base least significant).
#if defined(__HIPCC__)
__host__ __device__
#endif
inline uint64_t rc_code(uint64_t k, int s) {
    uint64_t x = ~k;                                   // complement: 3 - c == c ^ 3
    // reverse the 32 two-bit groups of the 64-bit word
    x = ((x >> 2) & 0x3333333333333333ull) | ((x & 0x3333333333333333ull) << 2);
    x = ((x >> 4) & 0x0F0F0F0F0F0F0F0Full) | ((x & 0x0F0F0F0F0F0F0F0Full) << 4);
    x = ((x >> 8) & 0x00FF00FF00FF00FFull) | ((x & 0x00FF00FF00FF00FFull) << 8);
    x = ((x >> 16) & 0x0000FFFF0000FFFFull) | ((x & 0x0000FFFF0000FFFFull) << 16);
    x = (x >> 32) | (x << 32);
    return x >> (64 - 2 * s);
}

}  // namespace snapgpu

struct snap_index {
    snapgpu::DevIndex d;
    int device;
    uint64_t windows;
    uint64_t distinct_keys;
    uint64_t position_entries;
    uint64_t device_bytes;
    void *alloc_gcode, *alloc_gmask, *alloc_table, *alloc_pos;
    void *alloc_rep;             // duplicate classes (snap_index_dup_classes), or null
    void *alloc_repbits;
    uint64_t rep_bytes;
    uint64_t dup_collisions;     // hash collisions the class build resolved by comparison
};
