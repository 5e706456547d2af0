// Device helpers shared by the join kernels (per-level and fused paths).
#pragma once

#include "gsi_internal.h"

namespace gsi {

// N(v,l) through PCSR (Sec. IV lookup): read the home group (8 x 16-byte
// loads = its 128 bytes), probe the 15 key slots in ascending key order,
// follow the GID chain.  Keys of a chain ascend, so meeting a larger key (or
// the empty marker) ends the search.  Returns (offset, length) in ci.
__device__ __forceinline__ uint2 pcsr_find(const uint32_t *gl, uint32_t G, uint32_t H, uint32_t v) {
    if (G == 0) return make_uint2(0, 0);
    uint32_t grp = pcsr_home(v, H);
    for (uint32_t hop = 0; hop < G; hop++) {
        const uint4 *p = reinterpret_cast<const uint4 *>(gl + (uint64_t)grp * GROUP_WORDS);
        uint32_t w[GROUP_WORDS];
#pragma unroll
        for (int i = 0; i < 8; i++) {
            uint4 t = p[i];
            w[4 * i] = t.x;
            w[4 * i + 1] = t.y;
            w[4 * i + 2] = t.z;
            w[4 * i + 3] = t.w;
        }
#pragma unroll
        for (uint32_t s = 0; s < KEYS_PER_GROUP; s++) {
            uint32_t key = w[2 * s];
            if (key == v) return make_uint2(w[2 * s + 1], w[2 * s + 3] - w[2 * s + 1]);
            if (key > v) return make_uint2(0, 0);
        }
        grp = w[2 * KEYS_PER_GROUP];
        if (grp == NONE32) break;
    }
    return make_uint2(0, 0);
}

__device__ __forceinline__ bool in_sorted(const uint32_t *list, uint32_t len, uint32_t x) {
    uint32_t lo = 0, hi = len;
    while (lo < hi) {
        uint32_t mid = (lo + hi) >> 1;
        if (list[mid] < x) lo = mid + 1;
        else hi = mid;
    }
    return lo < len && list[lo] == x;
}

// FNV-1a-64 over the four little-endian bytes of one 32-bit word
__device__ __forceinline__ uint64_t fnv_word(uint64_t h, uint32_t v) {
#pragma unroll
    for (int b = 0; b < 4; b++) {
        h ^= (v >> (8 * b)) & 0xFFu;
        h *= 1099511628211ull;
    }
    return h;
}
// SplitMix64 output mixing (Steele, Lea, Flood 2014)
__device__ __forceinline__ uint64_t mix64(uint64_t z) {
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

}  // namespace gsi
