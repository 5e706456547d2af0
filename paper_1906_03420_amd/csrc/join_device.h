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

// x in the ascending list[0, len)?  An 8-ary search: each step reads 7
// probes at once (independent loads) and keeps the eighth of the range that
// can hold x, then the last <= 8 elements are read at once, so a list of L
// elements costs about log8(L) + 1 dependent round trips to memory, not
// log2(L).
__host__ __device__ __forceinline__ bool in_sorted(const uint32_t *list, uint32_t len, uint32_t x) {
    uint32_t lo = 0, n = len;  // x, if present, is in [lo, lo + n)
    while (n > 8) {
        const uint32_t s = (n + 7) / 8;  // 8 segments of s (the last may be shorter)
        uint32_t v[7];
#pragma unroll
        for (uint32_t t = 1; t < 8; t++) v[t - 1] = s * t < n ? list[lo + s * t] : 0xFFFFFFFFu;
        uint32_t c = 0;  // segments whose first element is <= x, after the first
#pragma unroll
        for (uint32_t t = 1; t < 8; t++) c += (s * t < n && v[t - 1] <= x) ? 1u : 0u;
        lo += s * c;
        n = (n - s * c) < s ? (n - s * c) : s;
    }
    bool hit = false;
#pragma unroll
    for (uint32_t t = 0; t < 8; t++) hit |= t < n && list[lo + t] == x;
    return hit;
}

// in_sorted for U (list, x) pairs at once, with A-ary rounds (A - 1 probes
// each): list u is base[st[u] .. st[u] + len[u]).  Each round issues the probes of every pair before any
// is compared, so a thread waits for one chain of dependent loads instead
// of U.  A pair whose range is already down to 9 (or an empty list) probes
// base[lo] again, a valid address: base[0] when the list is empty, which
// every label holding an edge has.  With VEC (the per-level join), the
// last <= 9 elements are read as three aligned 16-byte words (12 elements
// from the 16-byte boundary at or below base + lo), 3 vector loads instead
// of 8 scalar ones: the join is bound by the address units, which pay per
// load instruction.  The window may read up to CI_PAD elements past the
// array's last list.  Without VEC the last <= 8 elements are read one by
// one (fewer registers: the engine's join holds four pairs).
template <uint32_t U, bool VEC = true, uint32_t A = 8>
__host__ __device__ __forceinline__ void in_sorted_many(const uint32_t *base, const uint32_t *st, const uint32_t *len,
                                               const uint32_t *x, bool *hit) {
    constexpr uint32_t TAIL = VEC ? 9u : 8u;  // elements the last round reads at most
    uint32_t lo[U], n[U];
#pragma unroll
    for (uint32_t u = 0; u < U; u++) {
        lo[u] = len[u] ? st[u] : 0u;
        n[u] = len[u];
    }
    for (;;) {
        bool more = false;
#pragma unroll
        for (uint32_t u = 0; u < U; u++) more |= n[u] > TAIL;
        if (!more) break;
        uint32_t v[U][A - 1];
#pragma unroll
        for (uint32_t u = 0; u < U; u++) {
            const uint32_t s = (n[u] + A - 1) / A;
#pragma unroll
            for (uint32_t t = 1; t < A; t++) v[u][t - 1] = base[lo[u] + (n[u] > TAIL && s * t < n[u] ? s * t : 0u)];
        }
#pragma unroll
        for (uint32_t u = 0; u < U; u++) {
            if (n[u] <= TAIL) continue;
            const uint32_t s = (n[u] + A - 1) / A;
            uint32_t c = 0;
#pragma unroll
            for (uint32_t t = 1; t < A; t++) c += (s * t < n[u] && v[u][t - 1] <= x[u]) ? 1u : 0u;
            lo[u] += s * c;
            n[u] = (n[u] - s * c) < s ? (n[u] - s * c) : s;
        }
    }
    if (!VEC) {
        uint32_t w[U][8];
#pragma unroll
        for (uint32_t u = 0; u < U; u++)
#pragma unroll
            for (uint32_t t = 0; t < 8; t++) w[u][t] = base[lo[u] + (t < n[u] ? t : 0u)];
#pragma unroll
        for (uint32_t u = 0; u < U; u++) {
            bool h = false;
#pragma unroll
            for (uint32_t t = 0; t < 8; t++) h |= t < n[u] && w[u][t] == x[u];
            hit[u] = h;
        }
        return;
    }
    uint4 w[U][3];
    uint32_t off[U];
#pragma unroll
    for (uint32_t u = 0; u < U; u++) {
        const uint32_t *p = base + lo[u];
        const uint4 *pa = reinterpret_cast<const uint4 *>(reinterpret_cast<uintptr_t>(p) & ~(uintptr_t)15);
        off[u] = (uint32_t)(p - reinterpret_cast<const uint32_t *>(pa));
#pragma unroll
        for (uint32_t t = 0; t < 3; t++) w[u][t] = pa[t];
    }
#pragma unroll
    for (uint32_t u = 0; u < U; u++) {
        bool h = false;
#pragma unroll
        for (uint32_t t = 0; t < 3; t++) {
            const uint32_t e[4] = {w[u][t].x, w[u][t].y, w[u][t].z, w[u][t].w};
#pragma unroll
            for (uint32_t q = 0; q < 4; q++) {
                const uint32_t d = 4 * t + q - off[u];  // position in [lo, lo + n) when < n (wraps below lo)
                h |= d < n[u] && e[q] == x[u];
            }
        }
        hit[u] = h;
    }
}

// One FNV-1a-64 step with a 32-bit value as the symbol (the tuple hash takes
// a row's k values as k symbols)
__device__ __forceinline__ uint64_t fnv_word(uint64_t h, uint32_t v) {
    h ^= v;
    h *= 1099511628211ull;
    return h;
}
// SplitMix64 output mixing (Steele, Lea, Flood 2014)
__device__ __forceinline__ uint64_t mix64(uint64_t z) {
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

}  // namespace gsi
