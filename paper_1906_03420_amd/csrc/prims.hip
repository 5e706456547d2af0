// Data-parallel primitives: fill, exclusive scan (u32 -> u64) and a stable
// LSD radix sort of tuples of uint32 arrays.  wave64 throughout.
#include "gsi_internal.h"

namespace gsi {

// ------------------------------------------------------------------- fill
template <typename T>
__global__ void k_fill(T *p, T v, uint64_t n) {
    uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    for (; i < n; i += stride) p[i] = v;
}

static uint32_t grid_for(uint64_t n, uint32_t per_block, uint32_t cap = 65536) {
    uint64_t b = (n + per_block - 1) / per_block;
    if (b == 0) b = 1;
    if (b > cap) b = cap;
    return (uint32_t)b;
}

void fill_u32(gsi_ctx *c, uint32_t *p, uint32_t v, uint64_t n) {
    if (!n) return;
    launch(c, "k_fill", 4.0 * n, k_fill<uint32_t>, grid_for(n, 1024), 256, p, v, n);
}
void fill_u64(gsi_ctx *c, uint64_t *p, uint64_t v, uint64_t n) {
    if (!n) return;
    launch(c, "k_fill", 8.0 * n, k_fill<uint64_t>, grid_for(n, 1024), 256, p, v, n);
}

// ------------------------------------------------------------------- scan
// Three passes: per-tile sums, one-workgroup scan of the tile sums, and a
// per-tile scan that adds the tile's offset.  A tile is 256 threads x 8
// consecutive items.
constexpr int SCAN_THREADS = 256;
constexpr int SCAN_ITEMS = 8;
constexpr int SCAN_TILE = SCAN_THREADS * SCAN_ITEMS;

template <int NT>
__device__ uint64_t block_exclusive_sum(uint64_t v, uint64_t *total) {
    __shared__ uint64_t s_w[NT / 64];
    uint64_t inc = wave_inclusive_sum(v);
    const uint32_t lane = lane_id(), w = threadIdx.x >> 6;
    if (lane == 63) s_w[w] = inc;
    __syncthreads();
    uint64_t off = 0, tot = 0;
#pragma unroll
    for (int i = 0; i < NT / 64; i++) {
        uint64_t x = s_w[i];
        off += (i < (int)w) ? x : 0;
        tot += x;
    }
    __syncthreads();
    *total = tot;
    return off + inc - v;
}

__global__ __launch_bounds__(SCAN_THREADS) void k_scan_reduce(const uint32_t *in, uint64_t n, uint64_t *part) {
    uint64_t base = (uint64_t)blockIdx.x * SCAN_TILE;
    uint64_t s = 0;
#pragma unroll
    for (int i = 0; i < SCAN_ITEMS; i++) {
        uint64_t idx = base + (uint64_t)i * SCAN_THREADS + threadIdx.x;
        if (idx < n) s += in[idx];
    }
    uint64_t tot;
    block_exclusive_sum<SCAN_THREADS>(s, &tot);
    if (threadIdx.x == 0) part[blockIdx.x] = tot;
}

__global__ __launch_bounds__(1024) void k_scan_partials(uint64_t *part, uint64_t nb, uint64_t *total,
                                                       uint64_t *total2, uint64_t *seqp, uint64_t seqv) {
    uint64_t carry = 0;
    for (uint64_t c0 = 0; c0 < nb; c0 += 1024) {
        uint64_t idx = c0 + threadIdx.x;
        uint64_t v = idx < nb ? part[idx] : 0;
        uint64_t tot;
        uint64_t ex = block_exclusive_sum<1024>(v, &tot);
        if (idx < nb) part[idx] = carry + ex;
        carry += tot;
    }
    if (threadIdx.x == 0) {
        *total = carry;
        if (total2) *total2 = carry;
        post_seq(seqp, seqv);
    }
}

__global__ __launch_bounds__(SCAN_THREADS) void k_scan_apply(const uint32_t *in, uint64_t n, const uint64_t *part,
                                                             uint64_t *out) {
    uint64_t base = (uint64_t)blockIdx.x * SCAN_TILE + (uint64_t)threadIdx.x * SCAN_ITEMS;
    uint32_t v[SCAN_ITEMS];
    uint64_t s = 0;
#pragma unroll
    for (int i = 0; i < SCAN_ITEMS; i++) {
        uint64_t idx = base + i;
        v[i] = idx < n ? in[idx] : 0;
        s += v[i];
    }
    uint64_t tot;
    uint64_t run = part[blockIdx.x] + block_exclusive_sum<SCAN_THREADS>(s, &tot);
#pragma unroll
    for (int i = 0; i < SCAN_ITEMS; i++) {
        uint64_t idx = base + i;
        if (idx < n) out[idx] = run;
        run += v[i];
    }
}

// whole scan in one workgroup (1024 threads x 8 consecutive items), for
// inputs of at most SMALL_SCAN items: one launch instead of three
constexpr int SMALL_SCAN = 1024 * SCAN_ITEMS;
__global__ __launch_bounds__(1024) void k_scan_small(const uint32_t *in, uint64_t n, uint64_t *out, uint64_t *total,
                                                    uint64_t *seqp, uint64_t seqv) {
    uint64_t base = (uint64_t)threadIdx.x * SCAN_ITEMS;
    uint32_t v[SCAN_ITEMS];
    uint64_t s = 0;
#pragma unroll
    for (int i = 0; i < SCAN_ITEMS; i++) {
        uint64_t idx = base + i;
        v[i] = idx < n ? in[idx] : 0;
        s += v[i];
    }
    uint64_t tot;
    uint64_t run = block_exclusive_sum<1024>(s, &tot);
#pragma unroll
    for (int i = 0; i < SCAN_ITEMS; i++) {
        uint64_t idx = base + i;
        if (idx < n) out[idx] = run;
        run += v[i];
    }
    if (threadIdx.x == 0) {
        out[n] = tot;
        if (total) *total = tot;
        post_seq(seqp, seqv);
    }
}

void exclusive_scan(gsi_ctx *c, const uint32_t *in, uint64_t n, uint64_t *out, Scratch &s, uint64_t *total) {
    if (n == 0) {
        fill_u64(c, out, 0, 1);
        if (total) fill_u64(c, total, 0, 1);
        return;
    }
    uint64_t seqv = 0;
    uint64_t *seqp = seq_slot(c, total, &seqv);
    if (n <= (uint64_t)SMALL_SCAN) {
        launch(c, "k_scan_small", 12.0 * n, k_scan_small, 1, 1024, in, n, out, total, seqp, seqv);
        c->seq_armed = seqp != nullptr;
        return;
    }
    uint64_t nb = (n + SCAN_TILE - 1) / SCAN_TILE;
    if (nb > 0x7FFFFFFFull) fail(GSI_E_INVALID, "scan too large");
    uint64_t *part = s.get<uint64_t>(nb, "scan partials");
    launch(c, "k_scan_reduce", 4.0 * n, k_scan_reduce, (uint32_t)nb, SCAN_THREADS, in, n, part);
    launch(c, "k_scan_partials", 16.0 * nb, k_scan_partials, 1, 1024, part, nb, out + n, total, seqp, seqv);
    launch(c, "k_scan_apply", 12.0 * n, k_scan_apply, (uint32_t)nb, SCAN_THREADS, in, n, (const uint64_t *)part, out);
    // the total is posted before the apply pass ends; a reader of it alone
    // need not wait for out[]: stream order makes later launches see out[]
    c->seq_armed = seqp != nullptr;
    s.drop(part);
}

// ------------------------------------------------------------ radix sort
// Tiles of 4096 tuples (256 threads x 16 rounds).  Stability: within a tile
// tuple r*256 + t is handled in round r by thread t, so (round, wave, lane)
// is the input order; ranks are counted in that order.
constexpr int RS_THREADS = 256;
constexpr int RS_ROUNDS = 16;
constexpr int RS_TILE = RS_THREADS * RS_ROUNDS;

// lanes of this wave holding the same 8-bit digit (valid lanes only)
__device__ __forceinline__ uint64_t digit_peers(uint32_t d, bool valid) {
    uint64_t peers = __ballot(valid);
#pragma unroll
    for (int b = 0; b < 8; b++) {
        bool bit = (d >> b) & 1u;
        uint64_t bb = __ballot(valid && bit);
        peers &= bit ? bb : ~bb;
    }
    return valid ? peers : 0ull;
}

__global__ __launch_bounds__(RS_THREADS) void k_radix_hist(const uint32_t *key, int shift, uint32_t n,
                                                          uint32_t ntiles, uint32_t *hist) {
    __shared__ uint32_t h[256];
    h[threadIdx.x] = 0;
    __syncthreads();
    uint64_t base = (uint64_t)blockIdx.x * RS_TILE;
    for (int r = 0; r < RS_ROUNDS; r++) {
        uint64_t idx = base + (uint64_t)r * RS_THREADS + threadIdx.x;
        bool valid = idx < n;
        uint32_t d = valid ? (key[idx] >> shift) & 255u : 0u;
        uint64_t peers = digit_peers(d, valid);
        if (valid && rank_below(peers) == 0) atomicAdd(&h[d], (uint32_t)__popcll(peers));
    }
    __syncthreads();
    hist[(uint64_t)threadIdx.x * ntiles + blockIdx.x] = h[threadIdx.x];
}

struct Arrays3 {
    uint32_t *p[3];
};

template <int NA>
__global__ __launch_bounds__(RS_THREADS) void k_radix_scatter(Arrays3 src, Arrays3 dst, int key_arr, int shift,
                                                             uint32_t n, uint32_t ntiles, const uint64_t *offs) {
    __shared__ uint64_t s_goff[256];
    __shared__ uint32_t s_run[256];
    __shared__ uint32_t s_wc[RS_THREADS / 64][256];
    const uint32_t t = threadIdx.x, w = t >> 6;
    s_goff[t] = offs[(uint64_t)t * ntiles + blockIdx.x];
    s_run[t] = 0;
    const uint32_t *key = src.p[key_arr];
    uint64_t base = (uint64_t)blockIdx.x * RS_TILE;
    for (int r = 0; r < RS_ROUNDS; r++) {
#pragma unroll
        for (int q = 0; q < RS_THREADS / 64; q++) s_wc[q][t] = 0;
        __syncthreads();
        uint64_t idx = base + (uint64_t)r * RS_THREADS + t;
        bool valid = idx < n;
        uint32_t vals[NA];
#pragma unroll
        for (int i = 0; i < NA; i++) vals[i] = valid ? src.p[i][idx] : 0u;
        uint32_t d = valid ? (key[idx] >> shift) & 255u : 0u;
        uint64_t peers = digit_peers(d, valid);
        uint32_t rk = rank_below(peers);
        if (valid && rk == 0) s_wc[w][d] = (uint32_t)__popcll(peers);
        __syncthreads();
        {
            uint32_t run = s_run[t];
#pragma unroll
            for (int q = 0; q < RS_THREADS / 64; q++) {
                uint32_t cnt = s_wc[q][t];
                s_wc[q][t] = run;
                run += cnt;
            }
            s_run[t] = run;
        }
        __syncthreads();
        if (valid) {
            uint64_t pos = s_goff[d] + s_wc[w][d] + rk;
            if (pos >= n) pos = n - 1;  // unreachable when the histogram matches; never write out of bounds
#pragma unroll
            for (int i = 0; i < NA; i++) dst.p[i][pos] = vals[i];
        }
        __syncthreads();
    }
}

bool radix_sort(gsi_ctx *c, uint32_t n, int na, uint32_t *const *a, uint32_t *const *tmp,
                const std::vector<SortPass> &passes, Scratch &s) {
    if (n <= 1 || passes.empty()) return false;
    if (na < 1 || na > 3) fail(GSI_E_INTERNAL, "radix_sort: 1..3 arrays");
    uint32_t ntiles = (uint32_t)(((uint64_t)n + RS_TILE - 1) / RS_TILE);
    uint64_t nh = 256ull * ntiles;
    uint32_t *hist = s.get<uint32_t>(nh, "radix histogram");
    uint64_t *offs = s.get<uint64_t>(nh + 1, "radix offsets");
    Arrays3 A{}, B{};
    for (int i = 0; i < na; i++) {
        A.p[i] = a[i];
        B.p[i] = tmp[i];
    }
    bool in_tmp = false;
    for (const SortPass &p : passes) {
        Arrays3 from = in_tmp ? B : A, to = in_tmp ? A : B;
        const uint32_t *key = from.p[p.key_arr];
        launch(c, "k_radix_hist", 4.0 * n, k_radix_hist, ntiles, RS_THREADS, key, p.shift, n, ntiles, hist);
        exclusive_scan(c, hist, nh, offs, s);
        double bytes = 8.0 * na * n;
        const uint64_t *co = offs;
        if (na == 1)
            launch(c, "k_radix_scatter", bytes, k_radix_scatter<1>, ntiles, RS_THREADS, from, to, p.key_arr, p.shift, n,
                   ntiles, co);
        else if (na == 2)
            launch(c, "k_radix_scatter", bytes, k_radix_scatter<2>, ntiles, RS_THREADS, from, to, p.key_arr, p.shift, n,
                   ntiles, co);
        else
            launch(c, "k_radix_scatter", bytes, k_radix_scatter<3>, ntiles, RS_THREADS, from, to, p.key_arr, p.shift, n,
                   ntiles, co);
        in_tmp = !in_tmp;
    }
    return in_tmp;
}

}  // namespace gsi
