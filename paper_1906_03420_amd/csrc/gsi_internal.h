// Internal declarations of the gfx950 subgraph-isomorphism library.
#pragma once

#include <hip/hip_ext.h>
#include <hip/hip_runtime.h>

#include <atomic>
#include <cstdint>
#include <map>
#include <set>
#include <string>
#include <vector>

#include "gsi.h"

namespace gsi {

// Elements the lists' array holds past its end (never read as list
// entries): the last round of in_sorted_many reads a 16-byte-aligned window
// that may reach up to 11 elements beyond a list, so the array is allocated
// with this many spare elements.
constexpr uint32_t CI_PAD = 16;


constexpr uint32_t NONE32 = 0xFFFFFFFFu;
constexpr uint32_t KEYS_PER_GROUP = GSI_PCSR_GPN - 1;  // 15 keys + (GID, END)
constexpr uint32_t GROUP_WORDS = 2 * GSI_PCSR_GPN;      // 32 uint32 = 128 bytes
constexpr uint32_t SIG_GROUPS = 240;                     // (512 - 32) / 2

// ------------------------------------------------------------------ errors
void set_error(const char *fmt, ...);
void clear_error();

struct Fail {
    gsi_status st;
};

#define GSI_HIP(call)                                                                      \
    do {                                                                                   \
        hipError_t e_ = (call);                                                            \
        if (e_ != hipSuccess) {                                                            \
            ::gsi::set_error("%s failed: %s (%s:%d)", #call, hipGetErrorString(e_), __FILE__, \
                             __LINE__);                                                    \
            throw ::gsi::Fail{GSI_E_DEVICE};                                               \
        }                                                                                  \
    } while (0)

[[noreturn]] void fail(gsi_status st, const char *fmt, ...);

// ------------------------------------------------------------------- arena
// First-fit allocator over the caller's device buffer.  Long-lived blocks
// (graph structures, result tables) are placed from the high end, per-call
// scratch from the low end, so scratch holes coalesce back between calls.
class Arena {
  public:
    void init(void *base, uint64_t size);
    void *alloc(uint64_t bytes, bool high);  // nullptr when it does not fit
    void release(void *p);
    void shrink(void *p, uint64_t bytes);  // keep the first `bytes`, free the rest
    uint64_t used() const { return used_; }
    uint64_t peak() const { return peak_; }
    uint64_t largest_free() const;

  private:
    uintptr_t base_ = 0;
    uint64_t size_ = 0;
    std::map<uint64_t, uint64_t> free_;  // offset -> size
    std::map<uint64_t, uint64_t> live_;  // offset -> size
    uint64_t used_ = 0, peak_ = 0;
};

struct KernelRec {
    int kid;
    hipEvent_t a, b;
    double bytes;
};

}  // namespace gsi

struct gsi_ctx {
    int device = 0;
    hipStream_t stream = nullptr;
    uint32_t flags = 0;
    gsi::Arena arena;
    uint64_t *pinned = nullptr;  // host-pinned staging: scalars [0,4K), status [4K,8K), plans [8K,64K)
    // Host-coherent mailbox (MAILBOX_WORDS words) that kernels write the
    // scalars the host waits for straight into: after a stream sync the host
    // reads them without a device-to-host copy.  mbox_dev is its device
    // address, mbox_host the host one.
    uint64_t *mbox_host = nullptr, *mbox_dev = nullptr;
    // Completion word: a kernel that writes scalars the host is about to
    // read can also store `seq` into mailbox word MBOX_SEQ (after them, with
    // a system-scope release); while seq_armed (that kernel was the last
    // launch) the host spins on that word instead of synchronising the
    // stream, which answers ~5 us sooner.  Every launch disarms it.
    uint64_t seq = 0;
    bool seq_armed = false;
    std::atomic<int> busy{0};
    std::set<gsi_graph *> graphs;
    std::set<gsi_result *> results;
    // profiling
    std::vector<std::string> knames;
    std::vector<gsi::KernelRec> recs;
    std::vector<hipEvent_t> free_events;
    std::vector<gsi_kernel_stat> acc;
};

struct gsi_graph {
    gsi_ctx *ctx = nullptr;
    uint32_t n = 0;
    uint64_t m = 0;
    uint32_t nlab = 0;      // max edge label + 1
    uint32_t flags = 0;
    uint32_t *sig = nullptr;  // [16 * n] column-first
    uint32_t *gl = nullptr;   // [total_groups * 32]
    // compressed representation, kept with GSI_GRAPH_KEEP_CR: per label
    // (from group_base[l], G[l] entries) its vertices ascending, the offset
    // of each one's list in the label's ci, and where each one's entries
    // start among all directed edges sorted by (label, source, target), whose
    // differences are the list lengths
    uint32_t *cr_vid = nullptr, *cr_start = nullptr, *cr_off = nullptr;
    uint32_t *ci = nullptr;   // [2m]
    // multi-labelled graphs (Sec. VII-B): vertex v's labels, ascending, at
    // vl_lab[vl_off[v] .. vl_off[v+1]); a vertex pair may carry several edge
    // labels (one entry per label in its partitions)
    bool multi = false;
    uint32_t *vl_off = nullptr, *vl_lab = nullptr;
    std::vector<uint64_t> group_base;  // per label: first global group
    std::vector<uint32_t> G;           // per label: |V(D)| groups
    std::vector<uint32_t> H;           // per label: home groups the hash spreads over
    std::vector<uint64_t> ci_base;     // per label: first ci entry
    std::vector<uint64_t> edges;       // per label: |E_l| (undirected)
    uint64_t total_groups = 0;
    uint32_t max_chain = 0;
    uint64_t bytes = 0;
    double build_ms = 0;
    gsi_batch_schedule tuned{0, 0};  // schedule picked by gsi_batch_tune
};

struct gsi_result {
    gsi_ctx *ctx = nullptr;
    uint32_t k = 0;
    uint64_t count = 0;
    uint64_t digest[2] = {0, 0};
    uint32_t *rows = nullptr;  // device, row-major count x k (arena, high end)
    bool count_only = false;
    gsi_stats stats{};
};

namespace gsi {

// Kernel launch on the context stream.  With GSI_CTX_PROFILE the launch goes
// through hipExtLaunchKernelGGL with a start and a stop event that the
// command processor records with the dispatch itself, so the measured span is
// the kernel's own execution; the pair is kept with the kernel's algorithmic
// bytes until gsi_ctx_kernel_stats drains it.
int kernel_id(gsi_ctx *c, const char *name);
hipEvent_t take_event(gsi_ctx *c);

template <typename K, typename... Args>
inline void launch(gsi_ctx *c, const char *name, double alg_bytes, K kernel, dim3 grid, dim3 block,
                   Args... args) {
    c->seq_armed = false;
    if (c->flags & GSI_CTX_PROFILE) {
        int kid = kernel_id(c, name);
        hipEvent_t a = take_event(c), b = take_event(c);
        hipExtLaunchKernelGGL(kernel, grid, block, 0, c->stream, a, b, 0, args...);
        GSI_HIP(hipGetLastError());
        c->recs.push_back(KernelRec{kid, a, b, alg_bytes});
    } else {
        hipLaunchKernelGGL(kernel, grid, block, 0, c->stream, args...);
        GSI_HIP(hipGetLastError());
    }
}

// Scoped scratch allocations, released in reverse order on scope exit.
struct Scratch {
    gsi_ctx *c;
    std::vector<void *> held;
    explicit Scratch(gsi_ctx *cc) : c(cc) {}
    ~Scratch() {
        for (auto it = held.rbegin(); it != held.rend(); ++it) c->arena.release(*it);
    }
    template <typename T>
    T *get(uint64_t count, const char *what) {
        uint64_t bytes = count * sizeof(T);
        if (bytes == 0) bytes = 256;
        void *p = c->arena.alloc(bytes, false);
        if (!p)
            fail(GSI_E_NOMEM, "arena exhausted allocating %llu bytes for %s (largest free block %llu)",
                 (unsigned long long)bytes, what, (unsigned long long)c->arena.largest_free());
        held.push_back(p);
        return static_cast<T *>(p);
    }
    void drop(void *p) {
        for (auto it = held.begin(); it != held.end(); ++it)
            if (*it == p) {
                held.erase(it);
                c->arena.release(p);
                return;
            }
    }
};

template <typename T>
T *persist(gsi_ctx *c, uint64_t count, const char *what) {
    uint64_t bytes = count * sizeof(T);
    if (bytes == 0) bytes = 256;
    void *p = c->arena.alloc(bytes, true);
    if (!p)
        fail(GSI_E_NOMEM, "arena exhausted allocating %llu bytes for %s (largest free block %llu)",
             (unsigned long long)bytes, what, (unsigned long long)c->arena.largest_free());
    return static_cast<T *>(p);
}

// Reads back `n` uint64 values from device memory (synchronises the stream).
constexpr uint64_t MAILBOX_WORDS = 512;
// a candidate bitset is counted in this many consecutive runs of words (one
// per wave of a 1024-thread workgroup)
constexpr uint32_t BITS_RUNS = 16;
// mailbox words of one query: candidate counts (32 x u32), level scalars,
// the fused workgroup's status
constexpr uint64_t MBOX_COUNTS = 0, MBOX_SCALARS = 16, MBOX_STATUS = 32, MBOX_SEQ = MAILBOX_WORDS - 1;
// The completion word for a kernel whose scalar output `dst` may lie in the
// mailbox: its device address and the next sequence value when it does
// (the caller arms the context after the launch), nullptr otherwise.
inline uint64_t *seq_slot(gsi_ctx *c, const void *dst, uint64_t *value) {
    const uint64_t *d = static_cast<const uint64_t *>(dst);
    if (!c->mbox_dev || !d || d < c->mbox_dev || d >= c->mbox_dev + MBOX_SEQ) return nullptr;
    *value = ++c->seq;
    return c->mbox_dev + MBOX_SEQ;
}
// Device side: the scalars this thread wrote before are visible to the host
// once it sees `value` in the completion word.
__device__ __forceinline__ void post_seq(uint64_t *slot, uint64_t value) {
    if (slot) __hip_atomic_store(slot, value, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_SYSTEM);
}
// Reads back `n` uint64 values from device memory, or from the mailbox
// without a copy (synchronises the stream either way).
void read_scalars(gsi_ctx *c, const uint64_t *dev, uint64_t *host, int n);
// Returns once the mailbox holds what every launch so far wrote there (the
// completion word, else a stream sync); device memory is not covered.
void wait_mailbox(gsi_ctx *c);
void sync(gsi_ctx *c);

// ------------------------------------------------------------- primitives
void fill_u32(gsi_ctx *c, uint32_t *p, uint32_t value, uint64_t n);
void fill_u64(gsi_ctx *c, uint64_t *p, uint64_t value, uint64_t n);
// out[i] = sum_{j<i} in[j] for i in [0, n]; out has n+1 entries.  When
// `total` is given the sum is also written there (device memory).
void exclusive_scan(gsi_ctx *c, const uint32_t *in, uint64_t n, uint64_t *out, Scratch &s,
                    uint64_t *total = nullptr);
// Stable LSD radix sort of `n` tuples held in `na` parallel uint32 arrays
// (a[0..na-1]); pass p orders by bits [shift, shift+8) of array key_arr[p].
// tmp holds na arrays of n entries.  Returns true if the result ended in tmp
// (the caller swaps pointers).
struct SortPass {
    int key_arr;
    int shift;
};
bool radix_sort(gsi_ctx *c, uint32_t n, int na, uint32_t *const *a, uint32_t *const *tmp,
                const std::vector<SortPass> &passes, Scratch &s);

// --------------------------------------------------------------- pieces
// d_vlabel: one label per vertex; for a multi-labelled graph (g->multi) it
// is unused and g->vl_off / g->vl_lab hold the label sets already.
void build_graph(gsi_graph *g, const uint32_t *d_vlabel, const uint32_t *d_src, const uint32_t *d_dst,
                 const uint32_t *d_elabel);

struct HostQuery {
    uint32_t k = 0;
    std::vector<uint32_t> vl, src, dst, el;
    std::vector<std::vector<std::pair<uint32_t, uint32_t>>> adj;  // (neighbour, label)
    // multi-label queries (Sec. VII-B): label set of each vertex (ascending);
    // a vertex pair may have several edges, one per label
    bool multi = false;
    std::vector<std::vector<uint32_t>> vls;
};
HostQuery validate_query(uint32_t k, const uint32_t *vl, uint32_t qm, const uint32_t *s, const uint32_t *d,
                         const uint32_t *l);
// label sets lab[off[u] .. off[u+1]); repeated vertex pairs allowed with
// distinct labels
HostQuery validate_query_multi(uint32_t k, const uint32_t *off, const uint32_t *lab, uint32_t qm, const uint32_t *s,
                               const uint32_t *d, const uint32_t *l);
// a single-label query as the multi-label query with singleton sets
void make_multi(HostQuery &q);
// the bit of a vertex label in word 0 of a multi-labelled signature
__host__ __device__ __forceinline__ uint32_t label_bit(uint32_t x) { return 1u << ((x * 0x9E3779B1u) >> 27); }
constexpr uint32_t MULTI_MAX_QUERY_LABELS = 256;  // labels over all vertices of one query
void run_filter(gsi_graph *g, const HostQuery &q, uint64_t *d_bits, uint32_t *d_counts);
// query vertex u of query i has bitset row / count slot qbase[i] + u
void run_filter_many(gsi_graph *g, const std::vector<const HostQuery *> &qs, const std::vector<uint32_t> &qbase,
                     uint64_t *d_bits, uint32_t *d_counts);
void make_plan(const gsi_graph *g, const HostQuery &q, const std::vector<uint32_t> &cand,
               std::vector<uint32_t> &order, std::vector<uint32_t> &e0src);
// tile_row[t] = row r with F[r] <= 256 t < F[r+1]; tile_row[ntiles] = R - 1
void tile_rows(gsi_ctx *c, const uint64_t *F, uint64_t R, uint64_t ntiles, uint64_t *tile_row);
gsi_result *run_query(gsi_graph *g, const HostQuery &q, const gsi_query_options *opt);
// takes the device address of the fixed scratch of gsi_query_run_noalloc on
// `device` (current), once per device
void noalloc_init(int device);

}  // namespace gsi

// ------------------------------------------------------- device helpers
namespace gsi {

__device__ __forceinline__ uint32_t lane_id() { return __lane_id(); }

// number of set bits of m strictly below this lane
__device__ __forceinline__ uint32_t rank_below(uint64_t m) {
    return __builtin_amdgcn_mbcnt_hi((uint32_t)(m >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)m, 0u));
}

template <typename T>
__device__ __forceinline__ T wave_inclusive_sum(T v) {
    const uint32_t lane = lane_id();
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        T t = __shfl_up(v, o, 64);
        if (lane >= (uint32_t)o) v += t;
    }
    return v;
}

template <typename T>
__device__ __forceinline__ T wave_sum(T v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}

__device__ __forceinline__ uint64_t wave_xor(uint64_t v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v ^= __shfl_xor(v, o, 64);
    return v;
}

// PCSR home group (Sec. IV hash f): Knuth multiplicative hash of the vertex
// id, reduced to [0, H) by a multiply-shift.
__device__ __host__ __forceinline__ uint32_t pcsr_home(uint32_t v, uint32_t H) {
    uint32_t x = v * 0x9E3779B1u;
    return (uint32_t)(((uint64_t)x * (uint64_t)H) >> 32);
}

// Signature group of the key (edge label, neighbour label), Sec. III-A.
__device__ __host__ __forceinline__ uint32_t sig_group(uint32_t elabel, uint32_t nlabel) {
    uint64_t key = ((uint64_t)elabel << 32) | nlabel;
    uint64_t hi = (key * 0x9E3779B97F4A7C15ull) >> 32;
    return (uint32_t)((hi * (uint64_t)SIG_GROUPS) >> 32);
}

}  // namespace gsi

namespace gsi {

// Marks the context busy for the length of one ABI call.
struct Busy {
    gsi_ctx *c;
    explicit Busy(gsi_ctx *cc) : c(cc) {
        int z = 0;
        if (!c->busy.compare_exchange_strong(z, 1)) fail(GSI_E_BUSY, "context is already running a call");
    }
    ~Busy() { c->busy.store(0); }
};

}  // namespace gsi

// Body of an ABI function: exceptions become status codes and the message
// of the thread's last error.
#define GSI_TRY(...)                                     \
    try {                                                 \
        gsi::clear_error();                               \
        __VA_ARGS__;                                      \
        return GSI_OK;                                    \
    } catch (const gsi::Fail &f_) {                       \
        return f_.st;                                     \
    } catch (const std::bad_alloc &) {                    \
        gsi::set_error("host allocation failed");         \
        return GSI_E_NOMEM;                               \
    } catch (...) {                                       \
        gsi::set_error("unexpected internal exception");  \
        return GSI_E_INTERNAL;                            \
    }
