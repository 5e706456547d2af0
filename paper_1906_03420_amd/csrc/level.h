// Arguments of one join level of the per-level kernels (Algorithms 3-4) and
// device helpers shared by the join variants.
#pragma once

#include "gsi_internal.h"
#include "join_device.h"

namespace gsi {

struct EdgeRef {
    const uint32_t *gl;  // this label's groups
    const uint32_t *ci;  // this label's neighbour lists
    uint32_t G, H;       // groups, home groups
    uint32_t col;        // column of M holding the placed endpoint
    uint32_t ci_off;     // offset of this label's lists in the whole ci array
    // compressed representation (ablation): the label's vertices in
    // ascending order, each one's list offset in the label's ci, and the
    // start of its entries in the (label, source, target) order of all
    // directed edges, whose differences give the lengths
    const uint32_t *cr_vid, *cr_start, *cr_off;
    uint32_t cr_end;     // end of the label's entries in that order
    uint32_t pad;
};

struct LevelArgs {
    const uint32_t *M;
    uint64_t R;
    uint64_t ldm;  // column stride of M (>= R): column c of row i at M[c * ldm + i]
    uint32_t j, ne, e0, k;
    uint32_t pick;  // 1: each row scans its shortest linking list (else e0's)
    uint32_t homo;  // 1: homomorphism (no subtraction of m_i, Sec. VII-A)
    // ablations: lists located by binary search in the compressed
    // representation; survivors counted, then the join repeated to write
    // (two-step output); last-level rows written without LDS staging
    uint32_t abl_cr, abl_two_step, abl_no_stage;
    // 1: every row scans its e0 list already filtered by C(u) (held in
    // ci_all for this level), so the join skips the C(u) test
    uint32_t prefiltered;
    // single-pass last level (k_join_last): per-tile look-back status words,
    // the dynamic tile counter and a failure flag (both zeroed before the
    // launch), and where the last tile writes the total row count
    unsigned long long *tstat;
    uint32_t *tctr;
    uint64_t *total;
    uint64_t out_cap;  // rows the output can hold
    EdgeRef e[GSI_MAX_K];
    const uint32_t *ci_all;  // every label's lists
    const uint64_t *Cu;
    // N(m_i[col_e], l_e) of row i as a (start, length) pair at words
    // 2(e*R + i), 2(e*R + i) + 1 (one 8-byte load reads both); the scanned
    // list of row i starts at ci_all[loc[2ne*R + i]] and is linking edge
    // loc[(2ne+1)*R + i]
    uint32_t *loc;
    uint32_t *bound;
    uint64_t *part;            // per-workgroup partial sums of k_locate
    const uint64_t *F;
    const uint64_t *tile_row;  // row holding the first slot of tile t (entry ntiles = R-1)
    uint64_t gba;
    uint64_t *bitmap;
    uint32_t *tile_cnt;
    // survivor records (when set, instead of the bitmap): the q-th kept slot
    // of tile t, in slot order, has its element at rec_x[t * TS + q] and its
    // row, less the tile's first row, at rec_r[t * TS + q]
    uint32_t *rec_x, *rec_r;
    const uint64_t *tile_off;
    uint32_t *Mn;
    uint64_t S;
    uint32_t *out;
    uint64_t *dig_part;  // per tile (sum, xor) of the tuple hashes (last level)
    uint32_t qcol[GSI_MAX_K];  // query vertex -> column (last level)
    // the columns of m_i that can hold a candidate x: those whose query
    // vertex has u's label (a single-label graph's C(u) holds only vertices
    // with u's label); every column on a multi-labelled graph
    uint32_t nmc;
    uint32_t mcol[GSI_MAX_K];
    // the linking edges in the order the join tests them: rarest label
    // first, so that most candidates fail at the first search
    uint32_t eorder[GSI_MAX_K];
    uint32_t final_level, count_only;
    // k_locate with one workgroup (R <= its threads): it also scans the
    // row bounds into F, writes |GBA| to scan_total and posts seq_value to
    // seq_slot (the mailbox completion word), so the level needs no scan
    // launch; nullptr otherwise
    uint64_t *scan_total;
    uint64_t *seq_slot;
    uint64_t seq_value;
    // 1: R <= 256, the join finds each tile's rows in F itself and writes
    // tile_row for the link (no k_tile_rows launch)
    uint32_t rows_in_join;
};

// The located (start, length) of linking edge e for row i
__device__ __forceinline__ uint2 loc_pair(const LevelArgs &a, uint32_t e, uint64_t i) {
    return reinterpret_cast<const uint2 *>(a.loc)[(uint64_t)e * a.R + i];
}

// N(v, l) by binary search over the label's ascending vertex IDs (the
// compressed representation the paper compares PCSR with, Sec. IV)
__device__ __forceinline__ uint2 cr_find(const EdgeRef &er, uint32_t v) {
    uint32_t lo = 0, hi = er.G;
    while (lo < hi) {
        uint32_t mid = (lo + hi) >> 1;
        if (er.cr_vid[mid] < v) lo = mid + 1;
        else hi = mid;
    }
    if (lo >= er.G || er.cr_vid[lo] != v) return make_uint2(0, 0);
    const uint32_t b = er.cr_start[lo], e = lo + 1 < er.G ? er.cr_start[lo + 1] : er.cr_end;
    return make_uint2(er.cr_off[lo], e - b);
}

// largest i in [lo, hi] with F[i] <= p (F non-decreasing, F[lo] <= p)
__device__ __forceinline__ uint64_t row_of(const uint64_t *F, uint64_t lo, uint64_t hi, uint64_t p) {
    while (lo < hi) {
        uint64_t mid = lo + (hi - lo + 1) / 2;
        if (F[mid] <= p) lo = mid;
        else hi = mid - 1;
    }
    return lo;
}

// The costly tests of U candidates at once: keep[u] (on entry: whether
// candidate u is live) becomes x[u] not in m_i of row i[u] and x[u] in
// every other linking list of that row.  Every step issues the loads of
// all U candidates before using any (the row's values, the scanned edge,
// the lists' bounds, each search round), so a thread waits for one chain of
// dependent loads per step instead of U.
// Search rounds of the per-level join split a range in JOIN_ARITY parts
// (in_sorted_many).  The join is bound by its load instructions, so 4-ary
// rounds (3 probes, one more dependent round per factor 16) beat 8-ary ones
// (7 probes): 6 % less join time on an R-MAT graph of 8.4M vertices and
// 100M edges.
constexpr uint32_t JOIN_ARITY = 4;

// The row values of U rows in N consecutive entries of a column list
// (cols[c0 .. c0 + N), an entry past `nc` re-reading entry nc - 1, a valid
// column): loads issued together, straight-line, one wait.
template <uint32_t U, uint32_t N>
__device__ __forceinline__ void load_cols(const LevelArgs &a, const uint32_t *cols, uint32_t c0, uint32_t nc,
                                          const uint64_t *i, uint32_t (*m)[8]) {
    uint32_t col[N];
#pragma unroll
    for (uint32_t t = 0; t < N; t++) col[t] = __builtin_amdgcn_readfirstlane(cols[c0 + t < nc ? c0 + t : nc - 1]);
#pragma unroll
    for (uint32_t u = 0; u < U; u++)
#pragma unroll
        for (uint32_t t = 0; t < N; t++) m[u][t] = a.M[(uint64_t)col[t] * a.ldm + i[u]];
}

// The costly tests of U candidates at once: keep[u] (on entry: whether
// candidate u is live) becomes x[u] not in m_i of row i[u] and x[u] in
// every other linking list of that row.  Every step issues the loads of
// all U candidates before using any (the row's values, the scanned edge,
// the lists' bounds, each search round), so a thread waits for one chain of
// dependent loads per step instead of U.  The joins are bound by the
// address units, which pay per load instruction, so the row values are
// read in chunks of 1, 2, 4 or 8 columns, the smallest that holds what is
// left (a uniform choice), not always 8.
template <uint32_t U>
__device__ __forceinline__ void keep_many(const LevelArgs &a, const uint32_t *x, const uint64_t *i, bool *keep) {
    if (!a.homo) {
        // x not among the row's values in the columns that can hold it
        for (uint32_t c = 0; c < a.nmc; c += 8) {
            const uint32_t left = a.nmc - c;
            uint32_t m[U][8];
            uint32_t w;
            if (left >= 5) {
                load_cols<U, 8>(a, a.mcol, c, a.nmc, i, m);
                w = 8;
            } else if (left >= 3) {
                load_cols<U, 4>(a, a.mcol, c, a.nmc, i, m);
                w = 4;
            } else if (left == 2) {
                load_cols<U, 2>(a, a.mcol, c, a.nmc, i, m);
                w = 2;
            } else {
                load_cols<U, 1>(a, a.mcol, c, a.nmc, i, m);
                w = 1;
            }
#pragma unroll
            for (uint32_t u = 0; u < U; u++)
#pragma unroll
                for (uint32_t t = 0; t < 8; t++) keep[u] = keep[u] && (t >= w || m[u][t] != x[u]);
        }
    }
    if (a.ne < 2) return;
    uint32_t be[U];
#pragma unroll
    for (uint32_t u = 0; u < U; u++) be[u] = a.loc[(uint64_t)(2 * a.ne + 1) * a.R + i[u]];
    for (uint32_t t = 0; t < a.ne; t++) {
        const uint32_t e2 = __builtin_amdgcn_readfirstlane(a.eorder[t]);
        uint32_t st[U], len[U];
        bool act[U], hit[U], any = false;
#pragma unroll
        for (uint32_t u = 0; u < U; u++) {
            act[u] = keep[u] && e2 != be[u];
            any |= act[u];
        }
        if (!any) continue;
#pragma unroll
        for (uint32_t u = 0; u < U; u++) {
            const uint2 sl = loc_pair(a, e2, i[u]);
            st[u] = sl.x;
            len[u] = sl.y;
        }
#pragma unroll
        for (uint32_t u = 0; u < U; u++)
            if (!act[u]) len[u] = 0;
        in_sorted_many<U, true, JOIN_ARITY>(a.e[e2].ci, st, len, x, hit);
#pragma unroll
        for (uint32_t u = 0; u < U; u++)
            if (act[u]) keep[u] = hit[u];
    }
}

// Copies the j values of row i to column-major dst (column c at
// dst[c * stride + pos]): loads issued together in chunks of 1, 2, 4 or 8
// columns, the smallest that holds what is left (a column past j re-reads
// column j - 1, a valid address, instead of branching around the load,
// which would make each load wait for the one before it).
template <uint32_t N>
__device__ __forceinline__ void copy_cols(const LevelArgs &a, uint64_t i, uint32_t c, uint32_t *dst, uint64_t stride,
                                          uint64_t pos) {
    uint32_t m[N];
#pragma unroll
    for (uint32_t t = 0; t < N; t++) {
        const uint32_t cc = c + t < a.j ? c + t : a.j - 1;
        m[t] = a.M[(uint64_t)cc * a.ldm + i];
    }
#pragma unroll
    for (uint32_t t = 0; t < N; t++)
        if (c + t < a.j) dst[(uint64_t)(c + t) * stride + pos] = m[t];
}
__device__ __forceinline__ void copy_row(const LevelArgs &a, uint64_t i, uint32_t *dst, uint64_t stride,
                                         uint64_t pos) {
    for (uint32_t c = 0; c < a.j; c += 8) {
        const uint32_t left = a.j - c;
        if (left >= 5) copy_cols<8>(a, i, c, dst, stride, pos);
        else if (left >= 3) copy_cols<4>(a, i, c, dst, stride, pos);
        else if (left == 2) copy_cols<2>(a, i, c, dst, stride, pos);
        else copy_cols<1>(a, i, c, dst, stride, pos);
    }
}

// slot x of row i survives: x in C(u), x not in m_i, x in every other
// linking list of the row
__device__ __forceinline__ bool slot_keep(const LevelArgs &a, uint64_t i, uint32_t x) {
    bool keep = (a.Cu[x >> 6] >> (x & 63)) & 1ull;
    for (uint32_t c = 0; keep && !a.homo && c < a.j; c++) keep = a.M[(uint64_t)c * a.ldm + i] != x;
    const uint32_t be = (keep && a.ne > 1) ? a.loc[(uint64_t)(2 * a.ne + 1) * a.R + i] : a.e0;
    for (uint32_t e = 0; keep && e < a.ne; e++) {
        if (e == be) continue;
        const uint2 sl = loc_pair(a, e, i);
        keep = in_sorted(a.e[e].ci + sl.x, sl.y, x);
    }
    return keep;
}

// The paper's ablations of the join step (GSI_ABL_NAIVE_SETOPS,
// GSI_ABL_ROW_PER_WAVE, GSI_ABL_FOUR_LAYER, GSI_ABL_DUP_REMOVAL): fills
// a.bitmap and a.tile_cnt for the level exactly as k_join does.
void run_join_ablation(gsi_ctx *c, const LevelArgs &a, uint32_t flags, uint64_t ntiles, uint32_t ts,
                       double join_bytes, Scratch &s);

}  // namespace gsi
