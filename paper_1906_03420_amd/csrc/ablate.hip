// Join-step variants that reproduce the paper's ablations on this hardware
// (measurement and tests only).  Each one computes, for a join level, the
// same keep bit per |GBA| slot (slot p of row i is element p - F[i] of the
// row's scanned list) and the same survivor count per tile as k_join, so the
// per-level link (k_link) finishes the level unchanged:
//
//   naive set operations   (Sec. V, the "+SO" step of Table V) one kernel
//                          per set operation over the whole slot space: the
//                          subtraction of m_i writes a buffer of vertex ids
//                          in GBA, the C(u) intersection and one
//                          intersection per further linking edge each read
//                          and rewrite it, a last pass turns it into keep
//                          bits (no fusion, no LDS)
//   one wave per row       Algorithm 3 as written: the wave of row i scans
//                          the row's list; no load balance
//   4-layer balance        (Sec. VI-A) rows longer than W1 go to a separate
//                          launch spread over the whole chip; within a
//                          1024-thread workgroup, rows longer than W2 are run
//                          by the whole workgroup, rows longer than W3 join a
//                          pool in LDS divided equally among its threads, and
//                          the rest stay with their own wave
//   duplicate removal      (Sec. VI-B, Algorithm 5) with either of the two
//                          above: waves of a workgroup whose rows scan the
//                          same list share it: the first of them reads each
//                          batch of it into LDS, the others wait at the
//                          barrier and read the batch from there
#include <algorithm>
#include <cstring>

#include "level.h"

namespace gsi {

constexpr uint32_t AT = 1024;      // threads per workgroup (the paper's blocks of 1024)
constexpr uint32_t AW = AT / 64;   // waves per workgroup
// 4-layer thresholds: W2 is the workgroup size; W1 = 4 W2 = 16 W3 as in the
// paper's setting (W1 > W2 > W3 > wave size)
constexpr uint32_t W1 = 4 * AT, W2 = AT, W3 = AT / 4;
constexpr uint32_t DUP_BATCH = 256;  // elements per shared batch (Algorithm 5)
constexpr uint32_t NT = 256;         // threads of the slot-parallel kernels

// ORs the 64 keep bits of `mask` into the bitmap at bit positions pos..pos+63
__device__ __forceinline__ void or_bits(uint64_t *bm, uint64_t pos, uint64_t mask) {
    if (!mask) return;
    const uint64_t w = pos >> 6;
    const uint32_t sh = (uint32_t)(pos & 63);
    atomicOr(reinterpret_cast<unsigned long long *>(bm + w), (unsigned long long)(mask << sh));
    if (sh) {
        const uint64_t hi = mask >> (64 - sh);
        if (hi) atomicOr(reinterpret_cast<unsigned long long *>(bm + w + 1), (unsigned long long)hi);
    }
}

struct RowRef {
    uint64_t i, base;  // row, its first slot F[i]
    uint32_t start;    // its scanned list in ci_all
    uint32_t len;      // F[i+1] - F[i]
};

__device__ __forceinline__ RowRef row_ref(const LevelArgs &a, uint64_t i) {
    RowRef r;
    r.i = i;
    r.base = a.F[i];
    r.len = (uint32_t)(a.F[i + 1] - r.base);
    r.start = a.loc[(uint64_t)(2 * a.ne) * a.R + i];
    return r;
}

// one wave scans elements [t0, t1) of row r (t0 a multiple of 64 from the
// row's first element); `src` reads element t
template <typename Src>
__device__ __forceinline__ void wave_scan(const LevelArgs &a, const RowRef &r, uint32_t t0, uint32_t t1, Src src) {
    const uint32_t lane = lane_id();
    for (uint32_t t = t0; t < t1; t += 64) {
        const uint32_t tt = t + lane;
        bool keep = false;
        if (tt < t1) keep = slot_keep(a, r.i, src(tt));
        const uint64_t m = __ballot(keep);
        if (lane == 0) or_bits(a.bitmap, r.base + t, m);
    }
}

// The per-wave layer: wave w scans row `my` (len 0: nothing).  With `dup`,
// Algorithm 5: waves whose rows scan the same list (same start in ci_all)
// share it; the first such wave reads each batch into LDS, a barrier
// publishes it, and every sharing wave tests its own row's subtraction and
// intersections on the shared batch.
template <bool DUP>
__device__ __forceinline__ void wave_layer(const LevelArgs &a, const RowRef &my, bool valid) {
    const uint32_t w = threadIdx.x >> 6, lane = lane_id();
    if (!DUP) {
        if (valid) wave_scan(a, my, 0, my.len, [&](uint32_t t) { return a.ci_all[my.start + t]; });
        return;
    }
    __shared__ uint32_t s_id[AW], s_len[AW];
    __shared__ uint32_t s_buf[AW][DUP_BATCH];
    if (lane == 0) {
        s_id[w] = valid ? my.start : NONE32;
        s_len[w] = valid ? my.len : 0u;
    }
    __syncthreads();
    uint32_t addr = w, maxlen = 0;
    for (uint32_t q = 0; q < AW; q++) {
        maxlen = max(maxlen, s_len[q]);
        if (q < addr && valid && s_id[q] == my.start) addr = q;
    }
    const uint32_t nb = (maxlen + DUP_BATCH - 1) / DUP_BATCH;
    for (uint32_t b = 0; b < nb; b++) {
        const uint32_t t0 = b * DUP_BATCH;
        if (valid && addr == w)
            for (uint32_t x = lane; x < DUP_BATCH && t0 + x < my.len; x += 64) s_buf[w][x] = a.ci_all[my.start + t0 + x];
        __syncthreads();
        if (valid && t0 < my.len) {
            const uint32_t t1 = min(my.len, t0 + DUP_BATCH);
            wave_scan(a, my, t0, t1, [&](uint32_t t) { return s_buf[addr][t - t0]; });
        }
        __syncthreads();
    }
}

// one wave per row (Algorithm 3 without load balance)
template <bool DUP>
__global__ __launch_bounds__(AT) void k_abl_rows(LevelArgs a) {
    const uint64_t i = (uint64_t)blockIdx.x * AW + (threadIdx.x >> 6);
    const bool valid = i < a.R;
    RowRef r{};
    if (valid) r = row_ref(a, i);
    wave_layer<DUP>(a, r, valid && r.len > 0);
}

// rows longer than W1, listed for the separate launch (layer 1)
__global__ __launch_bounds__(NT) void k_abl_heavy_list(LevelArgs a, uint32_t *list, uint32_t *cnt) {
    const uint64_t i = (uint64_t)blockIdx.x * NT + threadIdx.x;
    if (i >= a.R) return;
    const uint64_t len = a.F[i + 1] - a.F[i];
    if (len > W1) {
        const uint32_t at = atomicAdd(cnt, 1u);
        list[at] = (uint32_t)i;
        atomicMax(cnt + 1, (uint32_t)((len + W1 - 1) / W1));
    }
}

// layer 1: workgroup (x, y) scans chunks y, y + gridDim.y, ... (W1 elements
// each) of heavy row list[x]
__global__ __launch_bounds__(AT) void k_abl_heavy(LevelArgs a, const uint32_t *list) {
    const RowRef r = row_ref(a, list[blockIdx.x]);
    const uint32_t w = threadIdx.x >> 6;
    for (uint64_t c0 = (uint64_t)blockIdx.y * W1; c0 < r.len; c0 += (uint64_t)gridDim.y * W1) {
        const uint32_t c1 = (uint32_t)min((uint64_t)r.len, c0 + W1);
        for (uint32_t t = (uint32_t)c0 + w * 64; t < c1; t += AT)
            wave_scan(a, r, t, min(c1, t + 64), [&](uint32_t tt) { return a.ci_all[r.start + tt]; });
    }
}

// layers 2-4 for the rows of one workgroup (one row per wave)
template <bool DUP>
__global__ __launch_bounds__(AT) void k_abl_4layer(LevelArgs a) {
    __shared__ uint32_t s_l2[AW], s_n2, s_n3;
    __shared__ uint32_t s_l3[AW], s_pre[AW + 1];
    const uint32_t w = threadIdx.x >> 6, lane = lane_id();
    const uint64_t i = (uint64_t)blockIdx.x * AW + w;
    const bool valid = i < a.R;
    RowRef my{};
    if (valid) my = row_ref(a, i);
    if (threadIdx.x == 0) s_n2 = s_n3 = 0;
    __syncthreads();
    // the waves vote: rows over W2 for the workgroup, over W3 for the pool
    if (lane == 0 && valid && my.len <= W1) {
        if (my.len > W2) s_l2[atomicAdd(&s_n2, 1u)] = w;
        else if (my.len > W3) s_l3[atomicAdd(&s_n3, 1u)] = w;
    }
    __syncthreads();
    const uint32_t n2 = s_n2, n3 = s_n3;
    // layer 2: the whole workgroup scans each such row
    for (uint32_t q = 0; q < n2; q++) {
        const RowRef r = row_ref(a, (uint64_t)blockIdx.x * AW + s_l2[q]);
        for (uint32_t t = w * 64; t < r.len; t += AT)
            wave_scan(a, r, t, min(r.len, t + 64), [&](uint32_t tt) { return a.ci_all[r.start + tt]; });
    }
    // layer 3: the pool's elements divided equally among all threads
    if (threadIdx.x == 0) {
        uint32_t run = 0;
        for (uint32_t q = 0; q < n3; q++) {
            s_pre[q] = run;
            run += (uint32_t)(a.F[(uint64_t)blockIdx.x * AW + s_l3[q] + 1] - a.F[(uint64_t)blockIdx.x * AW + s_l3[q]]);
        }
        s_pre[n3] = run;
    }
    __syncthreads();
    const uint32_t pool = s_pre[n3];
    for (uint32_t p = threadIdx.x; p < pool; p += AT) {
        uint32_t q = 0;
        while (q + 1 < n3 && s_pre[q + 1] <= p) q++;
        const RowRef r = row_ref(a, (uint64_t)blockIdx.x * AW + s_l3[q]);
        const uint32_t t = p - s_pre[q];
        if (slot_keep(a, r.i, a.ci_all[r.start + t])) {
            const uint64_t pos = r.base + t;
            atomicOr(reinterpret_cast<unsigned long long *>(a.bitmap + (pos >> 6)), 1ull << (pos & 63));
        }
    }
    // layer 4: short rows stay with their wave
    wave_layer<DUP>(a, my, valid && my.len > 0 && my.len <= W3);
}

// ------------------------------------------------- naive set operations
__global__ __launch_bounds__(NT) void k_abl_naive_sub(LevelArgs a, uint32_t *buf) {
    const uint64_t p = (uint64_t)blockIdx.x * NT + threadIdx.x;
    if (p >= a.gba) return;
    const uint64_t i = row_of(a.F, 0, a.R - 1, p);
    const uint32_t x = a.ci_all[a.loc[(uint64_t)(2 * a.ne) * a.R + i] + (uint32_t)(p - a.F[i])];
    bool in_m = false;
    for (uint32_t c = 0; !a.homo && c < a.j; c++) in_m |= a.M[(uint64_t)c * a.ldm + i] == x;
    buf[p] = in_m ? NONE32 : x;
}

__global__ __launch_bounds__(NT) void k_abl_naive_cand(LevelArgs a, uint32_t *buf) {
    const uint64_t p = (uint64_t)blockIdx.x * NT + threadIdx.x;
    if (p >= a.gba) return;
    const uint32_t x = buf[p];
    if (x != NONE32 && !((a.Cu[x >> 6] >> (x & 63)) & 1ull)) buf[p] = NONE32;
}

__global__ __launch_bounds__(NT) void k_abl_naive_isect(LevelArgs a, uint32_t *buf, uint32_t e) {
    const uint64_t p = (uint64_t)blockIdx.x * NT + threadIdx.x;
    if (p >= a.gba) return;
    const uint32_t x = buf[p];
    if (x == NONE32) return;
    const uint64_t i = row_of(a.F, 0, a.R - 1, p);
    const uint32_t be = a.ne > 1 ? a.loc[(uint64_t)(2 * a.ne + 1) * a.R + i] : a.e0;
    if (e == be) return;  // the row's scanned list
    const uint2 sl = loc_pair(a, e, i);
    if (!in_sorted(a.e[e].ci + sl.x, sl.y, x)) buf[p] = NONE32;
}

// keep bits from the buffer: one ballot word per wave (the grid covers every
// slot of every tile, the ones past |GBA| give 0 bits)
__global__ __launch_bounds__(NT) void k_abl_naive_keep(LevelArgs a, const uint32_t *buf) {
    const uint64_t p = (uint64_t)blockIdx.x * NT + threadIdx.x;
    const bool keep = p < a.gba && buf[p] != NONE32;
    const uint64_t m = __ballot(keep);
    if (lane_id() == 0) a.bitmap[p >> 6] = m;
}

// survivors per tile of ts slots
__global__ __launch_bounds__(NT) void k_abl_tile_count(const uint64_t *bm, uint64_t ntiles, uint32_t words,
                                                       uint32_t *cnt) {
    const uint64_t t = (uint64_t)blockIdx.x * NT + threadIdx.x;
    if (t >= ntiles) return;
    uint32_t s = 0;
    for (uint32_t q = 0; q < words; q++) s += (uint32_t)__popcll(bm[t * words + q]);
    cnt[t] = s;
}

static uint32_t grid_of(uint64_t n, uint64_t per) {
    const uint64_t b = (n + per - 1) / per;
    if (b > 0x7FFFFFFFull) fail(GSI_E_CAPACITY, "grid of %llu workgroups exceeds the launch limit", (unsigned long long)b);
    return (uint32_t)(b ? b : 1);
}

void run_join_ablation(gsi_ctx *c, const LevelArgs &a, uint32_t flags, uint64_t ntiles, uint32_t ts,
                       double join_bytes, Scratch &s) {
    const uint64_t words = ntiles * (ts / 64);
    const double G = (double)a.gba, R = (double)a.R;
    if (flags & GSI_ABL_NAIVE_SETOPS) {
        uint32_t *buf = s.get<uint32_t>(a.gba, "GBA buffer (naive set operations)");
        const uint32_t g = grid_of(a.gba, NT);
        launch(c, "k_abl_naive_sub", 8.0 * G + R * (4.0 * a.j + 12.0), k_abl_naive_sub, g, NT, a, buf);
        launch(c, "k_abl_naive_cand", 8.0 * G, k_abl_naive_cand, g, NT, a, buf);
        for (uint32_t e = 0; e < a.ne; e++)
            if (a.ne > 1 || e != a.e0)
                launch(c, "k_abl_naive_isect", 8.0 * G + R * 12.0, k_abl_naive_isect, g, NT, a, buf, e);
        launch(c, "k_abl_naive_keep", 4.0 * G + G / 8.0, k_abl_naive_keep, grid_of(ntiles * ts, NT), NT, a,
               (const uint32_t *)buf);
    } else {
        fill_u64(c, a.bitmap, 0, words);
        const bool dup = (flags & GSI_ABL_DUP_REMOVAL) != 0;
        const uint32_t g = grid_of(a.R, AW);
        if (flags & GSI_ABL_FOUR_LAYER) {
            uint32_t *cnt = s.get<uint32_t>(2, "heavy-row counters");
            uint32_t *list = s.get<uint32_t>(a.R, "heavy rows");
            fill_u32(c, cnt, 0, 2);
            launch(c, "k_abl_heavy_list", 16.0 * R, k_abl_heavy_list, grid_of(a.R, NT), NT, a, list, cnt);
            uint64_t hc[2];
            uint32_t h[2];
            read_scalars(c, reinterpret_cast<const uint64_t *>(cnt), hc, 1);
            memcpy(h, hc, 8);
            if (h[0])
                launch(c, "k_abl_heavy", join_bytes, k_abl_heavy, dim3(h[0], std::min<uint32_t>(h[1], 65535u)), AT, a,
                       (const uint32_t *)list);
            if (dup) launch(c, "k_abl_4layer", join_bytes, k_abl_4layer<true>, g, AT, a);
            else launch(c, "k_abl_4layer", join_bytes, k_abl_4layer<false>, g, AT, a);
        } else {
            if (dup) launch(c, "k_abl_rows", join_bytes, k_abl_rows<true>, g, AT, a);
            else launch(c, "k_abl_rows", join_bytes, k_abl_rows<false>, g, AT, a);
        }
    }
    launch(c, "k_abl_tile_count", 8.0 * words + 4.0 * ntiles, k_abl_tile_count, grid_of(ntiles, NT), NT,
           (const uint64_t *)a.bitmap, ntiles, (uint32_t)(ts / 64), a.tile_cnt);
}

}  // namespace gsi
