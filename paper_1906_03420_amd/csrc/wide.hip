// Level-synchronous joins of many queries at once.
//
// Every step advances each active query by one join level (Algorithm 3 with
// Algorithm 4's pre-allocation), all queries sharing the same launches:
//   rows      the tables of all active queries are one row space: query q
//             owns global rows [rbase_q, rbase_q + R_q)
//   k_wlocate one thread per global row: N(v, l) for every linking edge of
//             the row's own query; bound = |N(v', l0)|
//   scan      F over all rows -> one global slot space [0, |GBA|)
//   k_wjoin   256-slot tiles over the global slots: the same tests as the
//             single-query join, with each slot's query found from its row
//   scan      survivor offsets; k_wsurv turns them into each query's first
//             and last survivor, so every query's next table gets its exact
//             size (host readback)
//   k_wlink   (m_i, x) into the query's own next table, or, at a query's
//             last level, its rows in query-vertex order plus each row's
//             hash (digest summed per query by k_wdigest)
// Slots of a query are contiguous and ordered by its rows, so each query's
// result, row order included, equals the single-query path's.
#include <algorithm>
#include <chrono>
#include <cstring>

#include "join_device.h"
#include "scan_device.h"
#include "wide.h"

namespace gsi {

constexpr uint32_t WT = 256;

struct WEdge {
    const uint32_t *gl;
    const uint32_t *ci;
    uint32_t G, H, col;
    uint32_t ci_off;  // offset of its label's lists in the whole ci array
};

// Lookups of a query's rows at loc + locbase: start of linking edge e at
// [e*R + i], length at [(ne+e)*R + i], start (in the whole ci array) of the
// list the row scans at [2ne*R + i] and that list's edge at [(2ne+1)*R + i].
struct WQ {
    const uint32_t *M;  // table, column c at M + c*R
    uint64_t R, rbase, locbase;
    const uint64_t *Cu;
    uint32_t j, ne, e0, efirst, k, final_level;
    uint32_t *Mn;   // next table (inner level)
    uint32_t *out;  // result rows (last level)
    uint64_t S, sbase;
    uint32_t qcol[GSI_MAX_K];
    uint32_t mmask;  // columns of m_i whose query vertex has u's label
};

// candidates a join thread tests at once (wkeep_many)
constexpr uint32_t WU = 4;
// the last search round as vector loads (in_sorted_many): more registers,
// one wave fewer per SIMD for the engine's join
constexpr bool WVEC = false;
// search rounds split a range in WARITY parts (in_sorted_many)
constexpr uint32_t WARITY = 8;

// The costly tests of U candidates of query Q at once (rows i[u] of Q's
// table): keep[u] (on entry: candidate u is live) becomes x[u] not in the
// row's values and x[u] in every other linking list of the row.  Every step
// issues the loads of all U candidates before using any.
template <uint32_t U>
__device__ __forceinline__ void wkeep_many(const WQ &Q, const uint32_t *loc, const WEdge *edges, const uint32_t *x,
                                           const uint64_t *i, bool *keep) {
    // only the columns of u's label can hold x; four at a time, the last
    // one read again past the end
    uint32_t mm = Q.mmask;
    const uint32_t last = mm ? 31u - (uint32_t)__builtin_clz(mm) : 0u;
    while (mm) {
        uint32_t cq[4], m[U][4];
#pragma unroll
        for (uint32_t t = 0; t < 4; t++) {
            cq[t] = mm ? (uint32_t)__builtin_ctz(mm) : last;
            mm &= mm - 1;
        }
#pragma unroll
        for (uint32_t u = 0; u < U; u++)
#pragma unroll
            for (uint32_t t = 0; t < 4; t++) m[u][t] = Q.M[(uint64_t)cq[t] * Q.R + i[u]];
#pragma unroll
        for (uint32_t u = 0; u < U; u++)
#pragma unroll
            for (uint32_t t = 0; t < 4; t++) keep[u] = keep[u] && m[u][t] != x[u];
    }
    if (Q.ne < 2) return;
    uint32_t be[U];
#pragma unroll
    for (uint32_t u = 0; u < U; u++) be[u] = loc[Q.locbase + (uint64_t)(2 * Q.ne + 1) * Q.R + i[u]];
    for (uint32_t e2 = 0; e2 < Q.ne; e2++) {
        uint32_t st[U], len[U];
        bool act[U], hit[U];
#pragma unroll
        for (uint32_t u = 0; u < U; u++) {
            st[u] = loc[Q.locbase + (uint64_t)e2 * Q.R + i[u]];
            len[u] = loc[Q.locbase + (uint64_t)(Q.ne + e2) * Q.R + i[u]];
        }
#pragma unroll
        for (uint32_t u = 0; u < U; u++) {
            act[u] = keep[u] && e2 != be[u];
            if (!act[u]) len[u] = 0;
        }
        in_sorted_many<U, WVEC, WARITY>(edges[Q.efirst + e2].ci, st, len, x, hit);
#pragma unroll
        for (uint32_t u = 0; u < U; u++)
            if (act[u]) keep[u] = hit[u];
    }
}

static uint32_t wblocks(uint64_t n) {
    uint64_t b = (n + WT - 1) / WT;
    if (b == 0) b = 1;
    if (b > 0x7FFFFFFFull) fail(GSI_E_CAPACITY, "grid too large");
    return (uint32_t)b;
}

// largest q in [lo, hi] with qs[q].rbase <= r
__device__ __forceinline__ uint32_t query_of(const WQ *qs, uint32_t lo, uint32_t hi, uint64_t r) {
    while (lo < hi) {
        uint32_t mid = (lo + hi + 1) >> 1;
        if (qs[mid].rbase <= r) lo = mid;
        else hi = mid - 1;
    }
    return lo;
}

// Each row scans its shortest linking list (e0's on ties): the survivors,
// and their order, are those of the first edge of Algorithm 4.
__global__ __launch_bounds__(WT) void k_wlocate(const WQ *qs, uint32_t nq, const WEdge *edges, uint64_t Rtot,
                                               uint32_t *loc, uint32_t *bound, uint32_t *rowq) {
    __shared__ uint32_t s_q[2];
    const uint64_t r0 = (uint64_t)blockIdx.x * WT;
    if (threadIdx.x == 0) {
        const uint64_t rl = r0 + WT - 1 < Rtot ? r0 + WT - 1 : Rtot - 1;
        s_q[0] = query_of(qs, 0, nq - 1, r0);
        s_q[1] = query_of(qs, s_q[0], nq - 1, rl);
    }
    __syncthreads();
    const uint64_t r = r0 + threadIdx.x;
    if (r >= Rtot) return;
    const uint32_t qi = query_of(qs, s_q[0], s_q[1], r);
    rowq[r] = qi;  // the row's query, for the join and link of this step
    const WQ &Q = qs[qi];
    const uint64_t i = r - Q.rbase;
    uint32_t s0 = 0, l0 = 0, ob = NONE32, os = 0, ol = 0xFFFFFFFFu;
    for (uint32_t e = 0; e < Q.ne; e++) {
        const WEdge &ed = edges[Q.efirst + e];
        const uint32_t v = Q.M[(uint64_t)ed.col * Q.R + i];
        const uint2 f = pcsr_find(ed.gl, ed.G, ed.H, v);
        loc[Q.locbase + (uint64_t)e * Q.R + i] = f.x;
        loc[Q.locbase + (uint64_t)(Q.ne + e) * Q.R + i] = f.y;
        if (e == Q.e0) {
            s0 = f.x;
            l0 = f.y;
        } else if (f.y < ol) {
            ob = e;
            os = f.x;
            ol = f.y;
        }
    }
    uint32_t be = Q.e0, bs = s0, bl = l0;
    if (ob != NONE32 && ol < l0) {
        be = ob;
        bs = os;
        bl = ol;
    }
    bound[r] = bl;
    loc[Q.locbase + (uint64_t)(2 * Q.ne) * Q.R + i] = edges[Q.efirst + be].ci_off + bs;
    loc[Q.locbase + (uint64_t)(2 * Q.ne + 1) * Q.R + i] = be;
}

// The join of WJ_TILES consecutive 256-slot tiles per workgroup: each
// thread takes one slot of each tile and issues their loads together, and
// the set-up (rows staged in LDS, the query's descriptor) is paid once per
// WJ_TILES tiles.  Outputs stay per 256-slot tile: WT/64 bitmap words and
// one survivor count each.  When the rows fit (staged), each slot's row
// comes from a map built once per workgroup: each row after the first
// marks the slot where its slice starts (the largest row wins where empty
// rows share a start) and a max-scan carries the marks forward.
// (WJ_TILES by default; the batch schedule may pick 1, 2, 4 or 8, tuned)
constexpr uint32_t WJ_TILES = 4;

template <uint32_t TPW>
__global__ __launch_bounds__(WT) void k_wjoin(const WQ *qs, const uint32_t *rowq, const WEdge *edges,
                                             const uint32_t *ci_all, const uint64_t *F, const uint64_t *tile_row,
                                             uint64_t ntiles, uint64_t gba, const uint32_t *loc, uint64_t *bitmap,
                                             uint32_t *tile_cnt) {
    __shared__ uint64_t s_F[(TPW * WT)];
    __shared__ uint32_t s_st[(TPW * WT)];
    __shared__ uint32_t s_row[(TPW * WT)];  // row (from r_lo) of each slot, staged groups
    __shared__ uint32_t s_w[WT / 64];
    __shared__ WQ s_Q;
    __shared__ uint32_t s_q[2];
    __shared__ uint32_t s_x[(TPW * WT)];    // elements that passed the C(u) test, compacted
    __shared__ uint32_t s_r[(TPW * WT)];    // and their rows (from r_lo)
    __shared__ uint16_t s_slot[(TPW * WT)]; // and their slots in the group
    __shared__ uint64_t s_keep[(TPW * WT) / 64];
    __shared__ uint32_t s_n;
    const uint64_t t0 = (uint64_t)blockIdx.x * TPW;
    const uint64_t t1 = t0 + TPW < ntiles ? t0 + TPW : ntiles;
    const uint64_t p0 = t0 * WT;
    const uint64_t r_lo = tile_row[t0], r_hi = tile_row[t1];
    const uint64_t nr = r_hi - r_lo + 1;
    const bool staged = nr <= (TPW * WT);
    if (threadIdx.x == 0) {
        s_n = 0;
        s_q[0] = rowq[r_lo];
        s_q[1] = rowq[r_hi];
    }
    if (threadIdx.x < (TPW * WT) / 64) s_keep[threadIdx.x] = 0;
#pragma unroll
    for (uint32_t k = 0; k < TPW; k++) s_row[threadIdx.x * TPW + k] = 0;
    if (staged)
        for (uint32_t r = threadIdx.x; r < nr; r += WT) s_F[r] = F[r_lo + r];
    __syncthreads();
    const bool one = s_q[0] == s_q[1];
    if (one) {
        const WQ &Q = qs[s_q[0]];
        const uint32_t *src = reinterpret_cast<const uint32_t *>(&Q);
        uint32_t *dst = reinterpret_cast<uint32_t *>(&s_Q);
        for (uint32_t w = threadIdx.x; w < sizeof(WQ) / 4; w += WT) dst[w] = src[w];
        if (staged)
            for (uint32_t r = threadIdx.x; r < nr; r += WT)
                s_st[r] = loc[Q.locbase + (uint64_t)(2 * Q.ne) * Q.R + (r_lo + r - Q.rbase)];
    }
    if (staged)
        for (uint32_t r = threadIdx.x; r < nr; r += WT) {
            // rows after the first start past p0 (the first holds slot p0)
            const uint64_t pos = s_F[r] - p0;
            if (r > 0 && pos < (TPW * WT)) atomicMax(&s_row[pos], r);
        }
    __syncthreads();
    if (staged) block_max_scan<WT, TPW>(s_row, s_w);
    const uint32_t lane = lane_id();
    // x = N(v'_i, l0)[p - F[i]] for the thread's slot of each tile, then the
    // C(u) test; the slots that pass are compacted so that the costly tests
    // below run in dense waves
    uint32_t xs[TPW], rs[TPW];
    bool kp[TPW];
#pragma unroll
    for (uint32_t k = 0; k < TPW; k++) {
        const uint32_t sl = k * WT + threadIdx.x;
        const uint64_t p = p0 + sl;
        kp[k] = p < gba;
        xs[k] = 0;
        rs[k] = 0;
        if (kp[k]) {
            uint64_t r, Fr;
            uint32_t lr;
            if (staged) {
                lr = s_row[sl];
                r = r_lo + lr;
                Fr = s_F[lr];
            } else {
                uint64_t lo = r_lo, hi = r_hi;
                while (lo < hi) {
                    const uint64_t mid = lo + (hi - lo + 1) / 2;
                    if (F[mid] <= p) lo = mid;
                    else hi = mid - 1;
                }
                r = lo;
                Fr = F[lo];
                lr = 0;
            }
            rs[k] = (uint32_t)(r - r_lo);
            const WQ &Q = one ? s_Q : qs[rowq[r]];
            const uint64_t i = r - Q.rbase;
            const uint32_t st0 = (one && staged) ? s_st[lr] : loc[Q.locbase + (uint64_t)(2 * Q.ne) * Q.R + i];
            xs[k] = ci_all[st0 + (uint32_t)(p - Fr)];
        }
    }
    {
        // every slot's C(u) word is loaded before any is tested (a slot past
        // |GBA| has x = 0 and row r_lo: valid addresses)
        uint64_t cw[TPW];
#pragma unroll
        for (uint32_t k = 0; k < TPW; k++) {
            const uint64_t *Cu = one ? s_Q.Cu : qs[rowq[r_lo + rs[k]]].Cu;
            cw[k] = Cu[xs[k] >> 6];
        }
#pragma unroll
        for (uint32_t k = 0; k < TPW; k++) kp[k] = kp[k] && ((cw[k] >> (xs[k] & 63)) & 1ull);
    }
#pragma unroll
    for (uint32_t k = 0; k < TPW; k++) {
        const uint64_t pm = __ballot(kp[k]);
        if (pm) {
            uint32_t base = 0;
            if (lane == 0) base = atomicAdd(&s_n, (uint32_t)__popcll(pm));
            base = __shfl(base, 0, 64);
            if (kp[k]) {
                const uint32_t idx = base + rank_below(pm);
                s_slot[idx] = (uint16_t)(k * WT + threadIdx.x);
                s_x[idx] = xs[k];
                s_r[idx] = rs[k];
            }
        }
    }
    __syncthreads();
    const uint32_t n = __builtin_amdgcn_readfirstlane(s_n);
    if (one) {
        // one query in the tile: WU candidates per thread at a time, their
        // loads issued together
        for (uint32_t e0 = 0; e0 < n; e0 += WU * WT) {
            uint32_t xs2[WU], sl[WU];
            uint64_t is[WU];
            bool kq[WU];
#pragma unroll
            for (uint32_t u = 0; u < WU; u++) {
                const uint32_t e = e0 + u * WT + threadIdx.x;
                kq[u] = e < n;
                const uint32_t c = kq[u] ? e : 0u;  // a past-the-end thread reads candidate 0
                sl[u] = s_slot[c];
                xs2[u] = s_x[c];
                is[u] = r_lo + s_r[c] - s_Q.rbase;
            }
            wkeep_many<WU>(s_Q, loc, edges, xs2, is, kq);
#pragma unroll
            for (uint32_t u = 0; u < WU; u++)
                if (kq[u]) atomicOr(&s_keep[sl[u] >> 6], 1ull << (sl[u] & 63));
        }
    }
    for (uint32_t e = one ? n : threadIdx.x; e < n; e += WT) {
        const uint32_t slot = s_slot[e], xv = s_x[e];
        const uint64_t r = r_lo + s_r[e];
        const WQ &Q = one ? s_Q : qs[rowq[r]];
        const uint64_t i = r - Q.rbase;
        bool keep = true;
        // x not in m_i: the row's values eight at a time, every load issued
        // before the compares (a column past j re-reads column j - 1)
        for (uint32_t c = 0; keep && c < Q.j; c += 8) {
            uint32_t m[8];
#pragma unroll
            for (uint32_t q = 0; q < 8; q++) m[q] = Q.M[(uint64_t)(c + q < Q.j ? c + q : Q.j - 1) * Q.R + i];
#pragma unroll
            for (uint32_t q = 0; q < 8; q++) keep = keep && m[q] != xv;
        }
        const uint32_t be = (keep && Q.ne > 1) ? loc[Q.locbase + (uint64_t)(2 * Q.ne + 1) * Q.R + i] : Q.e0;
        for (uint32_t e2 = 0; keep && e2 < Q.ne; e2++) {
            if (e2 == be) continue;
            keep = in_sorted(edges[Q.efirst + e2].ci + loc[Q.locbase + (uint64_t)e2 * Q.R + i],
                             loc[Q.locbase + (uint64_t)(Q.ne + e2) * Q.R + i], xv);
        }
        if (keep) atomicOr(&s_keep[slot >> 6], 1ull << (slot & 63));
    }
    __syncthreads();
    // per 256-slot tile: its WT/64 bitmap words and their count
    if (threadIdx.x < 64) {
        const uint32_t tk = threadIdx.x / (WT / 64);  // tile of the group
        const uint64_t word = threadIdx.x < (TPW * WT) / 64 ? s_keep[threadIdx.x] : 0ull;
        if (threadIdx.x < (TPW * WT) / 64 && t0 + tk < t1) bitmap[p0 / 64 + threadIdx.x] = word;
        uint32_t c = (uint32_t)__popcll(word);
#pragma unroll
        for (uint32_t o = 1; o < WT / 64; o <<= 1) c += __shfl_xor(c, o, 64);
        if (threadIdx.x < (TPW * WT) / 64 && threadIdx.x % (WT / 64) == 0 && t0 + tk < t1) tile_cnt[t0 + tk] = c;
    }
}

// survivors before slot p
__device__ __forceinline__ uint64_t survivors_before(const uint64_t *bitmap, const uint64_t *tile_off, uint64_t gba,
                                                     uint64_t p) {
    const uint64_t ntiles = (gba + WT - 1) / WT;
    if (p >= gba) return tile_off[ntiles];
    const uint64_t t = p / WT;
    const uint32_t within = (uint32_t)(p - t * WT);
    uint64_t r = tile_off[t];
    for (uint32_t w = 0; w < within / 64; w++) r += (uint64_t)__popcll(bitmap[t * (WT / 64) + w]);
    const uint32_t b = within % 64;
    if (b) r += (uint64_t)__popcll(bitmap[t * (WT / 64) + within / 64] & ((1ull << b) - 1));
    return r;
}

// per query: first survivor, end of its survivors, first slot, end of slots
__global__ __launch_bounds__(WT) void k_wsurv(const WQ *qs, uint32_t nq, const uint64_t *F, const uint64_t *bitmap,
                                             const uint64_t *tile_off, uint64_t gba, uint64_t *sb) {
    const uint32_t q = blockIdx.x * WT + threadIdx.x;
    if (q >= nq) return;
    const WQ &Q = qs[q];
    const uint64_t f0 = F[Q.rbase], f1 = F[Q.rbase + Q.R];
    sb[4 * (uint64_t)q] = survivors_before(bitmap, tile_off, gba, f0);
    sb[4 * (uint64_t)q + 1] = survivors_before(bitmap, tile_off, gba, f1);
    sb[4 * (uint64_t)q + 2] = f0;
    sb[4 * (uint64_t)q + 3] = f1;
}

// last-level rows of a one-query tile are staged in LDS and written as one
// contiguous block when k is at most this
constexpr uint32_t WLINK_STAGE_K = 16;

// (m_i, x) of every survivor into its query's next table, or, at a query's
// last level, the row in query-vertex order and its hash.  A workgroup
// takes the same WJ_TILES consecutive tiles as the join: their kept slots
// are listed in slot order in LDS first, so that the waves that gather,
// write and hash are dense, and survivor q of the list is survivor
// tile_off[t0] + q of the step.  The row of a survivor's slot is found by a
// binary search over the group's rows in LDS (survivors are often few, so
// a map of every slot would not pay).
template <uint32_t TPW>
__global__ __launch_bounds__(WT) void k_wlink(const WQ *qs, const uint32_t *rowq, const uint32_t *ci_all,
                                             const uint64_t *F, const uint64_t *tile_row, uint64_t ntiles,
                                             const uint32_t *loc, const uint64_t *bitmap, const uint64_t *tile_off,
                                             uint64_t *hv) {
    __shared__ uint64_t s_F[(TPW * WT)];
    __shared__ uint32_t s_st[(TPW * WT)];
    __shared__ WQ s_Q;
    __shared__ uint32_t s_q[2];
    __shared__ uint32_t s_rows[WT * WLINK_STAGE_K];
    __shared__ uint16_t s_list[(TPW * WT)];          // the group's kept slots, in slot order
    __shared__ uint32_t s_pre[(TPW * WT) / 64 + 1];  // kept slots before each bitmap word
    const uint64_t t0 = (uint64_t)blockIdx.x * TPW;
    const uint64_t t1 = t0 + TPW < ntiles ? t0 + TPW : ntiles;
    const uint64_t gbase = tile_off[t0];
    if (tile_off[t1] == gbase) return;  // no survivor in the group (uniform)
    const uint64_t p0 = t0 * WT;
    const uint32_t nwords = (uint32_t)(t1 - t0) * (WT / 64);
    const uint64_t *words = bitmap + p0 / 64;
    const uint64_t r_lo = tile_row[t0], r_hi = tile_row[t1];
    const uint64_t nr = r_hi - r_lo + 1;
    const bool staged = nr <= (TPW * WT);
    if (threadIdx.x == 0) {
        s_q[0] = rowq[r_lo];
        s_q[1] = rowq[r_hi];
        uint32_t run = 0;
        for (uint32_t q = 0; q < (TPW * WT) / 64; q++) {
            s_pre[q] = run;
            if (q < nwords) run += (uint32_t)__popcll(words[q]);
        }
        s_pre[(TPW * WT) / 64] = run;
    }
    if (staged)
        for (uint32_t r = threadIdx.x; r < nr; r += WT) s_F[r] = F[r_lo + r];
    __syncthreads();
    const bool one = s_q[0] == s_q[1];
    if (one) {
        const WQ &Q = qs[s_q[0]];
        const uint32_t *src = reinterpret_cast<const uint32_t *>(&Q);
        uint32_t *dst = reinterpret_cast<uint32_t *>(&s_Q);
        for (uint32_t w = threadIdx.x; w < sizeof(WQ) / 4; w += WT) dst[w] = src[w];
        if (staged)
            for (uint32_t r = threadIdx.x; r < nr; r += WT)
                s_st[r] = loc[Q.locbase + (uint64_t)(2 * Q.ne) * Q.R + (r_lo + r - Q.rbase)];
    }
    {
        const uint32_t w = threadIdx.x >> 6, lane = lane_id();
#pragma unroll
        for (uint32_t k = 0; k < TPW; k++) {
            const uint32_t wi = k * (WT / 64) + w;
            const uint64_t word = wi < nwords ? words[wi] : 0ull;
            if ((word >> lane) & 1ull) s_list[s_pre[wi] + rank_below(word)] = (uint16_t)(k * WT + threadIdx.x);
        }
    }
    __syncthreads();
    // the same count in every lane (the loop holds barriers)
    const uint32_t n = __builtin_amdgcn_readfirstlane(s_pre[(TPW * WT) / 64]);
    const bool stage = one && s_Q.final_level && s_Q.out && s_Q.k <= WLINK_STAGE_K;
    for (uint32_t q0 = 0; q0 < n; q0 += WT) {
        const uint32_t local = threadIdx.x;  // survivor q0 + local of the group
        const uint32_t q = q0 + local;
        const uint64_t gpos = gbase + q;
        if (q < n) {
            const uint64_t p = p0 + s_list[q];
            uint64_t r, Fr;
            uint32_t lr = 0;
            if (staged) {
                uint32_t lo = 0, hi = (uint32_t)(nr - 1);
                while (lo < hi) {
                    const uint32_t mid = (lo + hi + 1) >> 1;
                    if (s_F[mid] <= p) lo = mid;
                    else hi = mid - 1;
                }
                lr = lo;
                r = r_lo + lo;
                Fr = s_F[lo];
            } else {
                uint64_t lo = r_lo, hi = r_hi;
                while (lo < hi) {
                    const uint64_t mid = lo + (hi - lo + 1) / 2;
                    if (F[mid] <= p) lo = mid;
                    else hi = mid - 1;
                }
                r = lo;
                Fr = F[lo];
            }
            const WQ &Q = one ? s_Q : qs[rowq[r]];
            const uint64_t i = r - Q.rbase;
            const uint64_t pos = gpos - Q.sbase;
            if (pos < Q.S) {  // always, when the survivor ranges are consistent
                const uint32_t st0 = (one && staged) ? s_st[lr] : loc[Q.locbase + (uint64_t)(2 * Q.ne) * Q.R + i];
                const uint32_t x = ci_all[st0 + (uint32_t)(p - Fr)];
                // the row's values are loaded eight at a time, every load
                // issued before any is used (clamped columns: valid
                // addresses), not one dependent round trip per column
                if (!Q.final_level) {
                    for (uint32_t c = 0; c < Q.j; c += 8) {
                        uint32_t m[8];
#pragma unroll
                        for (uint32_t k4 = 0; k4 < 8; k4++)
                            m[k4] = Q.M[(uint64_t)(c + k4 < Q.j ? c + k4 : Q.j - 1) * Q.R + i];
#pragma unroll
                        for (uint32_t k4 = 0; k4 < 8; k4++)
                            if (c + k4 < Q.j) Q.Mn[(uint64_t)(c + k4) * Q.S + pos] = m[k4];
                    }
                    Q.Mn[(uint64_t)Q.j * Q.S + pos] = x;
                } else {
                    uint64_t f = 14695981039346656037ull;
                    for (uint32_t u0 = 0; u0 < Q.k; u0 += 8) {
                        uint32_t val[8];
#pragma unroll
                        for (uint32_t k4 = 0; k4 < 8; k4++) {
                            const uint32_t qc = Q.qcol[u0 + k4 < GSI_MAX_K ? u0 + k4 : GSI_MAX_K - 1];
                            const uint32_t c = u0 + k4 < Q.k ? qc : Q.j;
                            const uint32_t mv = Q.M[(uint64_t)(c < Q.j ? c : 0u) * Q.R + i];
                            val[k4] = c < Q.j ? mv : x;
                        }
#pragma unroll
                        for (uint32_t k4 = 0; k4 < 8; k4++) {
                            const uint32_t u = u0 + k4;
                            if (u >= Q.k) break;
                            if (stage) s_rows[local * Q.k + u] = val[k4];
                            else if (Q.out) Q.out[pos * Q.k + u] = val[k4];
                            f = fnv_word(f, val[k4]);
                        }
                    }
                    hv[gpos] = mix64(f);
                }
            }
        }
        if (stage) {
            // the round's rows are one contiguous block of the query's result
            __syncthreads();
            const uint64_t first = gbase + q0 - s_Q.sbase;
            uint64_t end = gbase + (q0 + WT < n ? q0 + WT : n) - s_Q.sbase;
            if (end > s_Q.S) end = s_Q.S;
            const uint32_t nw = first < end ? (uint32_t)(end - first) * s_Q.k : 0u;
            uint32_t *dst = s_Q.out + first * s_Q.k;
            for (uint32_t v = threadIdx.x; v < nw; v += WT) dst[v] = s_rows[v];
            __syncthreads();
        }
    }
}

// (sum, xor) of hv[a, b) per item, one workgroup per item
__global__ __launch_bounds__(WT) void k_wdigest(const uint64_t *items, const uint64_t *hv, uint64_t *part) {
    __shared__ uint64_t s_s[WT / 64], s_x[WT / 64];
    const uint64_t a = items[2 * (uint64_t)blockIdx.x], b = items[2 * (uint64_t)blockIdx.x + 1];
    uint64_t sm = 0, xr = 0;
    for (uint64_t t = a + threadIdx.x; t < b; t += WT) {
        const uint64_t h = hv[t];
        sm += h;
        xr ^= h;
    }
    sm = wave_sum(sm);
    xr = wave_xor(xr);
    if (lane_id() == 0) {
        s_s[threadIdx.x >> 6] = sm;
        s_x[threadIdx.x >> 6] = xr;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        uint64_t ts = 0, tx = 0;
        for (int q = 0; q < WT / 64; q++) {
            ts += s_s[q];
            tx ^= s_x[q];
        }
        part[2 * (uint64_t)blockIdx.x] = ts;
        part[2 * (uint64_t)blockIdx.x + 1] = tx;
    }
}

// One join level for the queries in `act` (all of them, or none: on an
// allocation failure everything allocated for the step is given back and
// no query changes state).
static void wide_step(gsi_graph *g, const std::vector<WideQuery *> &act, bool count_only, uint32_t tpw) {
    gsi_ctx *c = g->ctx;
    constexpr uint64_t DIGEST_ITEM = 1u << 16;
    {
        const uint32_t nq = (uint32_t)act.size();
        Scratch s(c);
        std::vector<WQ> hq(nq);
        std::vector<WEdge> he;
        // per-step allocations of the queries, released unless the step
        // commits; declared after the host arrays so that, on a failure, the
        // stream has drained the copies out of them before they go
        struct Pending {
            std::vector<WideQuery *> q;
            bool commit = false;
            gsi_ctx *c;
            ~Pending() {
                if (commit) return;
                (void)hipStreamSynchronize(c->stream);
                for (auto *x : q) {
                    if (x->next) c->arena.release(x->next);
                    x->next = nullptr;
                    if (x->rows) c->arena.release(x->rows);
                    x->rows = nullptr;
                    x->digest[0] = x->digest[1] = 0;
                }
            }
        } pend;
        pend.q = act;
        pend.c = c;
        uint64_t Rtot = 0, loctot = 0;
        for (uint32_t a = 0; a < nq; a++) {
            WideQuery &x = *act[a];
            const HostQuery &q = *x.q;
            const uint32_t j = x.j, u = x.order[j];
            WQ &Q = hq[a];
            memset(&Q, 0, sizeof(Q));
            Q.M = x.M;
            Q.R = x.R;
            Q.rbase = Rtot;
            Q.Cu = x.Cu[j];
            Q.j = j;
            Q.k = q.k;
            Q.final_level = j == q.k - 1;
            Q.efirst = (uint32_t)he.size();
            for (uint32_t i = 0; i < j; i++)
                for (auto &p : q.adj[u])
                    if (p.first == x.order[i]) {
                        const uint32_t l = p.second;
                        WEdge ed;
                        ed.gl = g->gl + g->group_base[l] * GROUP_WORDS;
                        ed.ci = g->ci + g->ci_base[l];
                        ed.G = g->G[l];
                        ed.H = g->H[l];
                        ed.col = i;
                        ed.ci_off = (uint32_t)g->ci_base[l];
                        if (x.order[i] == x.e0src[j]) Q.e0 = Q.ne;
                        he.push_back(ed);
                        Q.ne++;
                    }
            Q.locbase = loctot;
            for (uint32_t v = 0; v < q.k; v++) Q.qcol[v] = x.col[v];
            for (uint32_t c = 0; c < j; c++)
                if (q.multi || q.vl[x.order[c]] == q.vl[u]) Q.mmask |= 1u << c;
            x.stats_rows[j] = x.R;
            Rtot += x.R;
            loctot += (2ull * Q.ne + 2) * x.R;
        }
        WQ *d_q = s.get<WQ>(nq, "wide queries");
        WEdge *d_e = s.get<WEdge>(he.size(), "wide edges");
        uint32_t *loc = s.get<uint32_t>(loctot, "wide lookups");
        uint32_t *bound = s.get<uint32_t>(Rtot, "wide bounds");
        uint32_t *rowq = s.get<uint32_t>(Rtot, "wide row queries");
        uint64_t *F = s.get<uint64_t>(Rtot + 1, "wide offsets F");
        uint64_t *scal = s.get<uint64_t>(2, "wide scalars");
        GSI_HIP(hipMemcpyAsync(d_q, hq.data(), sizeof(WQ) * nq, hipMemcpyHostToDevice, c->stream));
        GSI_HIP(hipMemcpyAsync(d_e, he.data(), sizeof(WEdge) * he.size(), hipMemcpyHostToDevice, c->stream));
        double lb = 0;
        for (auto &Q : hq) lb += (double)Q.R * (4.0 * Q.ne + 128.0 * Q.ne + 8.0 * Q.ne + 4.0);
        launch(c, "k_wlocate", lb, k_wlocate, wblocks(Rtot), WT, (const WQ *)d_q, nq, (const WEdge *)d_e, Rtot, loc,
               bound, rowq);
        exclusive_scan(c, bound, Rtot, F, s, scal);
        uint64_t gba;
        read_scalars(c, scal, &gba, 1);  // also orders the uploads above before `hq`/`he` change
        if (gba == 0) {
            pend.commit = true;
            for (auto *x : act) {
                x->stats_gba[x->j] = 0;
                x->levels = x->j;
                x->finish_empty();
            }
            return;
        }
        const uint64_t ntiles = (gba + WT - 1) / WT;
        uint64_t *trow = s.get<uint64_t>(ntiles + 1, "wide tile rows");
        uint64_t *bitmap = s.get<uint64_t>(ntiles * (WT / 64), "wide GBA bitmap");
        uint32_t *tcnt = s.get<uint32_t>(ntiles, "wide tile counts");
        uint64_t *toff = s.get<uint64_t>(ntiles + 1, "wide tile offsets");
        uint64_t *sb = s.get<uint64_t>(4ull * nq, "wide survivor ranges");
        tile_rows(c, F, Rtot, ntiles, trow);
        double jb = 4.0 * gba + gba / 8.0 + 4.0 * ntiles;
        for (auto &Q : hq) jb += (double)Q.R * (8.0 + 8.0 * Q.ne + 4.0 * Q.j);
        {
            const uint32_t grid = (uint32_t)((ntiles + tpw - 1) / tpw);
            auto join = [&](auto kern) {
                launch(c, "k_wjoin", jb, kern, grid, WT, (const WQ *)d_q, (const uint32_t *)rowq, (const WEdge *)d_e,
                       (const uint32_t *)g->ci, (const uint64_t *)F, (const uint64_t *)trow, ntiles, gba,
                       (const uint32_t *)loc, bitmap, tcnt);
            };
            if (tpw == 1) join(k_wjoin<1>);
            else if (tpw == 2) join(k_wjoin<2>);
            else if (tpw == 8) join(k_wjoin<8>);
            else join(k_wjoin<4>);
        }
        exclusive_scan(c, tcnt, ntiles, toff, s, scal + 1);
        launch(c, "k_wsurv", 48.0 * nq, k_wsurv, wblocks(nq), WT, (const WQ *)d_q, nq, (const uint64_t *)F,
               (const uint64_t *)bitmap, (const uint64_t *)toff, gba, sb);
        std::vector<uint64_t> hsb(4ull * nq);
        GSI_HIP(hipMemcpyAsync(hsb.data(), sb, 32ull * nq, hipMemcpyDeviceToHost, c->stream));
        uint64_t Stot;
        read_scalars(c, scal + 1, &Stot, 1);
        // next tables (exact sizes) and result rows
        bool any_final = false;
        std::vector<uint64_t> items;
        std::vector<uint32_t> item_q;
        double kb = gba / 8.0 + 8.0 * ntiles;
        for (uint32_t a = 0; a < nq; a++) {
            WideQuery &x = *act[a];
            WQ &Q = hq[a];
            Q.sbase = hsb[4 * a];
            Q.S = hsb[4 * a + 1] - hsb[4 * a];
            x.stats_gba[x.j] = hsb[4 * a + 3] - hsb[4 * a + 2];
            x.stats_surv[x.j] = Q.S;
            if (Q.S == 0) continue;
            kb += (double)Q.S * (4.0 + 4.0 * Q.j);
            if (Q.final_level) {
                any_final = true;
                if (!count_only) {
                    Q.out = persist<uint32_t>(c, Q.S * Q.k, "result rows");
                    x.rows = Q.out;
                    kb += 4.0 * Q.k * Q.S;
                }
                for (uint64_t t = Q.sbase; t < Q.sbase + Q.S; t += DIGEST_ITEM) {
                    items.push_back(t);
                    items.push_back(std::min(t + DIGEST_ITEM, Q.sbase + Q.S));
                    item_q.push_back(a);
                }
            } else {
                x.next = c->arena.alloc(4ull * (Q.j + 1) * Q.S, false);
                if (!x.next)
                    fail(GSI_E_NOMEM, "arena exhausted allocating %llu bytes for a next table",
                         (unsigned long long)(4ull * (Q.j + 1) * Q.S));
                Q.Mn = static_cast<uint32_t *>(x.next);
                kb += 4.0 * (Q.j + 1) * Q.S;
            }
        }
        uint64_t *hv = any_final ? s.get<uint64_t>(Stot, "wide row hashes") : nullptr;
        GSI_HIP(hipMemcpyAsync(d_q, hq.data(), sizeof(WQ) * nq, hipMemcpyHostToDevice, c->stream));
        {
            const uint32_t grid = (uint32_t)((ntiles + tpw - 1) / tpw);
            auto link = [&](auto kern) {
                launch(c, "k_wlink", kb, kern, grid, WT, (const WQ *)d_q, (const uint32_t *)rowq,
                       (const uint32_t *)g->ci, (const uint64_t *)F, (const uint64_t *)trow, ntiles,
                       (const uint32_t *)loc, (const uint64_t *)bitmap, (const uint64_t *)toff, hv);
            };
            if (tpw == 1) link(k_wlink<1>);
            else if (tpw == 2) link(k_wlink<2>);
            else if (tpw == 8) link(k_wlink<8>);
            else link(k_wlink<4>);
        }
        std::vector<uint64_t> part;
        if (any_final) {
            const uint64_t ni = item_q.size();
            uint64_t *d_items = s.get<uint64_t>(2 * ni, "digest items");
            uint64_t *d_part = s.get<uint64_t>(2 * ni, "digest partials");
            GSI_HIP(hipMemcpyAsync(d_items, items.data(), 16 * ni, hipMemcpyHostToDevice, c->stream));
            launch(c, "k_wdigest", 8.0 * Stot, k_wdigest, (uint32_t)ni, WT, (const uint64_t *)d_items,
                   (const uint64_t *)hv, d_part);
            part.resize(2 * ni);
            GSI_HIP(hipMemcpyAsync(part.data(), d_part, 16 * ni, hipMemcpyDeviceToHost, c->stream));
        }
        sync(c);  // uploads done, partials read
        for (size_t t = 0; t < item_q.size(); t++) {
            WideQuery &x = *act[item_q[t]];
            x.digest[0] += part[2 * t];
            x.digest[1] ^= part[2 * t + 1];
        }
        pend.commit = true;
        for (uint32_t a = 0; a < nq; a++) {
            WideQuery &x = *act[a];
            const WQ &Q = hq[a];
            if (Q.S == 0) {
                x.levels = x.j;
                x.finish_empty();
            } else if (Q.final_level) {
                x.count = Q.S;
                x.levels = x.j;
                x.release_table();
                x.done = true;
            } else {
                x.release_table();
                x.own = x.next;
                x.next = nullptr;
                x.M = Q.Mn;
                x.R = Q.S;
                x.j++;
            }
        }
    }
}

// Estimated scratch bytes of one step for a query (lookups, bounds, F, one
// slot per row for the bitmap and tiles, and a next table of the same rows).
static uint64_t step_bytes(const WideQuery &x) {
    const uint64_t ne = x.j;  // at most j linking edges
    return x.R * (8 * ne + 4 + 8 + 8) + 4096;
}

WideEngine::WideEngine(gsi_graph *g, bool count_only, bool tolerant, uint32_t tiles)
    : g_(g), count_only_(count_only), tolerant_(tolerant),
      tpw_(tiles == 1 || tiles == 2 || tiles == 8 ? tiles : WJ_TILES) {}

void WideEngine::add(WideQuery &&q) { qs_.push_back(std::move(q)); }

bool WideEngine::idle() const {
    for (auto &x : qs_)
        if (!x.done) return false;
    return true;
}

uint32_t WideEngine::step() {
    std::vector<WideQuery *> act;
    for (auto &x : qs_)
        if (!x.done) act.push_back(&x);
    if (act.empty()) return 0;
    // start with the queries whose estimated step scratch fits in half the
    // largest free block; halve on an arena failure
    gsi_ctx *c = g_->ctx;
    const uint64_t room = c->arena.largest_free() / 2;
    size_t n = 0;
    uint64_t est = 0;
    while (n < act.size() && (n == 0 || est + step_bytes(*act[n]) <= room)) est += step_bytes(*act[n++]);
    size_t skipped = 0;  // queries moved behind the others (tolerant engine)
    for (;;) {
        std::vector<WideQuery *> part(act.begin(), act.begin() + n);
        try {
            wide_step(g_, part, count_only_, tpw_);
            steps_++;
            break;
        } catch (const Fail &f) {
            if (f.st != GSI_E_NOMEM || (n == 1 && !tolerant_)) throw;
            clear_error();
            if (n > 1) {
                n = (n + 1) / 2;
                continue;
            }
            WideQuery *x = act.front();
            if (act.size() == 1 || skipped + 1 >= act.size()) {
                // nothing else holds step memory that could be waited for
                x->release_table();
                x->status = GSI_E_NOMEM;
                x->count = 0;
                x->levels = x->j;
                x->done = true;
                break;
            }
            act.erase(act.begin());
            act.push_back(x);
            skipped++;
        }
    }
    uint32_t done = 0;
    for (auto *x : act) done += x->done;
    return done;
}

std::vector<WideQuery> WideEngine::take_done() {
    std::vector<WideQuery> out, keep;
    for (auto &x : qs_) (x.done ? out : keep).push_back(std::move(x));
    qs_ = std::move(keep);
    return out;
}

void wide_run(gsi_graph *g, std::vector<WideQuery> &wq, bool count_only, uint32_t tiles) {
    WideEngine e(g, count_only, false, tiles);
    for (auto &x : wq) e.add(std::move(x));
    while (!e.idle()) e.step();
    wq = e.take_done();
}

}  // namespace gsi
