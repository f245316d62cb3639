// fm_internal.hpp -- host-side structures shared by the library's translation units.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <string>
#include <vector>

#include "../../include/fm.h"
#include "fm_build.hpp"
#include "fm_device.hpp"

struct fm_index {
    int device = 0;
    uint64_t n = 0;
    uint64_t dollar = 0, rev_dollar = 0;
    uint64_t C[5] = {0, 0, 0, 0, 0}, rev_C[5] = {0, 0, 0, 0, 0};
    bool has_rev = false;
    void *mem = nullptr;   // one device block holding the layouts and SA samples
    bool owns_mem = true;  // false: mem is the caller's dev_buf (never freed here)
    void *lay[7] = {};     // forward layouts for I = 64, 96, 128, 192, 224, 256, 448 (inside mem)
    void *rlay[7] = {};    // layouts of reverse(R)
    uint64_t device_bytes = 0;
    uint32_t *sa_samples = nullptr;   // SA[32 j] for j = 0 .. n / 32 (fm_locate), or nullptr
    uint2 *ptab = nullptr;            // prefix table of R (see prefix_table_levels), or nullptr
    uint32_t table_levels = 0;
    fm_tuning tune[4] = {};
    int cu_count = 0;
    std::string arch;
    // phase timing (diagnostics): events recorded per call, 5 boundaries per call
    mutable uint32_t timing_cap = 0;
    mutable std::vector<hipEvent_t> ev_pool;
    mutable std::vector<int> ev_kind;      // per recorded call: 0 exact, 1 inexact
    mutable uint32_t ev_calls = 0;
};

namespace fm {

constexpr uint32_t kQueueChunk = 64;   // read-strands a wave takes from the work queue at once
constexpr uint32_t kHitSlots = 4;      // hits stored per read-strand without an atomic
constexpr uint32_t kOrderBins = 256;   // weight classes of the DFS claim order
constexpr uint32_t kOrderBlocks = 1024; // workgroups that count and place the claim order

inline uint32_t nstrands_of(uint32_t flags) { return ((flags & FM_FWD) ? 1u : 0u) + ((flags & FM_REVCOMP) ? 1u : 0u); }

constexpr int kLayouts = 7;
constexpr uint32_t kIntervals[kLayouts] = {64, 96, 128, 192, 224, 256, 448};
// slot of a checkpoint interval in the index's layout arrays, -1 when unsupported
inline int ilog(uint32_t I)
{
    for (int i = 0; i < kLayouts; ++i)
        if (kIntervals[i] == I) return i;
    return -1;
}
inline bool compact_layout(uint32_t I) { return I == 96 || I == 224; }
inline uint64_t superblock_buckets(uint32_t I) { return I == 96 ? 682 : 292; }
inline uint64_t num_buckets(uint64_t n, uint32_t I) { return n / I + 1; }
inline uint64_t bucket_bytes(uint32_t I) { return I <= 96 ? 32 : (I <= 224 ? 64 : 128); }
inline uint32_t max_lanes(uint32_t I) { return I <= 96 ? 2 : (I <= 224 ? 4 : 8); }
// buckets, then (compact layouts) one uint4 of counts per superblock
inline uint64_t layout_bytes(uint64_t n, uint32_t I)
{
    const uint64_t nb = num_buckets(n, I);
    return nb * bucket_bytes(I) + (compact_layout(I) ? ((nb + superblock_buckets(I) - 1) / superblock_buckets(I)) * 16 : 0);
}

DevLayout dev_layout(const fm_index *idx, uint32_t I, bool rev);

// Prefix table of R: for t = 1..T, the interval that Listing 1 gives the string
// s_0 .. s_{t-1} from (0, n) (empty ones as Listing 1 leaves them, k > l), at entry
// table_level_base(t) + sum_j s_j 4^j, so that the four children b.S of a string S of
// length t - 1 are four consecutive entries (32 bytes) at 4 * code(S). T grows with n up
// to one level short of log4(n), where a string still occurs a few times on average, and
// stops at 14 (2.86 GB): a node shallower than T reads one table entry instead of the one
// or two buckets of an Occ8, and every level added moved the genome-scale DFS closer to
// one read per node.
inline uint32_t prefix_table_levels(uint64_t n)
{
    int t = 0;
    while (t < 16 && ((n + 1) >> (2 * (t + 1))) > 0) ++t;    // t = floor(log4(n + 1))
    t -= 1;
    return t < 1 ? 0u : (t > 14 ? 14u : (uint32_t)t);
}
__host__ __device__ inline uint64_t table_level_base(uint32_t t) { return ((1ull << (2 * t)) - 4) / 3; }
inline uint64_t prefix_table_entries(uint32_t T) { return T ? table_level_base(T + 1) : 0; }
hipError_t build_prefix_table(const fm_index *idx, uint32_t I, hipStream_t s);

// Workspace header (byte offsets); the rest of the workspace follows at kWsHeader.
enum : size_t {
    kWsQueue = 0,        // uint32 work-queue counter (exact / D walk)
    kWsRequired = 8,     // uint64 hits every read would need
    kWsPool = 16,        // uint64 hits appended to the staging pool
    kWsQueue2 = 24,      // uint32 work-queue counter (DFS)
    kWsCut = 32,         // uint64 hit offset where the listed reads end
    kWsStatOcc = 64,     // uint64 Occ8 queries
    kWsStatBuckets = 72, // uint64 distinct buckets fetched
    kWsStatWalk = 80,    // uint64 walk steps that fetched
    kWsStatWalkBk = 88,  // uint64 buckets those steps fetched
    kWsStatSteal = 96,   // uint64 subtrees idle DFS lanes took over (dfs_steal)
    kWsStatTable = 104,  // uint64 DFS nodes whose children came from the prefix table
    kWsHeader = 256
};

struct InexactWs {       // sub-buffers of the inexact workspace
    size_t bp, rs_count, rs_status, rs_nodes, tf_count, tf_status, tf_nodes, cursor, rd_status, cnt, offs, part, slots,
        opool, bin, ohist, rec, total;
};
InexactWs inexact_ws_layout(uint64_t nreads, uint32_t nstr, uint32_t zmax, uint64_t hit_cap);

// ------------------------------------------------------------------ launchers

hipError_t build_layout(const uint32_t *packed_dev, uint64_t n, uint32_t I, void *out,
                        void *scratch, hipStream_t s);
size_t build_layout_scratch(uint64_t n, uint32_t I);

// Device suffix sorting (sa_build.hip). device_bwt writes the 2-bit BWT words of text$
// (or reverse(text)$) and its '$' row, and (samples != nullptr) the SA values of rows
// 0, 32, 64, ...; text_dev holds n codes 0..3. It allocates
// device_bwt_bytes(n) of working memory for the call. device_symbol_counts counts codes
// 0..3 into out[0..3] and codes above 3 into out[4].
hipError_t device_bwt(const uint8_t *text_dev, uint64_t n, bool rev, uint32_t *words, uint64_t *dollar_row,
                      uint32_t *samples, int cu_count, hipStream_t s);
size_t device_bwt_bytes(uint64_t n);
hipError_t device_symbol_counts(const uint8_t *text_dev, uint64_t n, uint64_t out[5], int cu_count, hipStream_t s);

hipError_t launch_fill(void *p, uint32_t value, size_t words, hipStream_t s);

// fm_locate: prefix sums of the interval sizes into offs, then the SA value of every row
// of the intervals (the first cap of them) into pos (search.hip).
size_t locate_ws_bytes(uint64_t niv);
hipError_t launch_locate(const fm_index *idx, const fm_tuning &t, const uint32_t *kl, uint64_t niv, uint32_t stride,
                         uint64_t *offs, uint32_t *pos, uint64_t cap, void *ws, bool stats, hipStream_t s);

hipError_t launch_occ8(const fm_index *idx, const fm_tuning &t, const fm_interval *q, uint64_t nq,
                       uint32_t *out, hipStream_t s);

struct WalkCall {
    const uint8_t *codes;
    const uint64_t *offs;
    const uint8_t *z;
    uint64_t nreads;
    uint32_t flags;
    uint32_t zmax;
    void *out;
    void *ws;
};
enum { WALK_EXACT = 0, WALK_DBP = 1, WALK_DFULL = 2 };
hipError_t launch_walk(const fm_index *idx, const fm_tuning &t, int mode, bool plain,
                       const WalkCall &c, hipStream_t s);
hipError_t launch_darray_full(const fm_index *idx, const fm_tuning &t, const WalkCall &c, uint64_t total_len,
                              hipStream_t s);

struct DfsCall {
    const uint8_t *codes;
    const uint64_t *offs;
    const uint8_t *z;
    uint64_t nreads;
    uint32_t flags;
    uint32_t zmax;
    fm_hit *hits;
    uint64_t hit_cap;
    uint64_t *hit_offs;
    uint32_t *status;
    void *ws;
    fm_interval *ex_out = nullptr;   // non-null: exact intervals of the ex_flags strands, taken from the DFS
    uint32_t ex_flags = 0;
};
// Phase boundaries of one call: HIP events recorded there (nullptr entries: not recorded),
// or, while a plan is captured, a cut of the capture into a new graph segment.
struct PhaseEvents {
    hipEvent_t ev[5] = {nullptr, nullptr, nullptr, nullptr, nullptr};
    void (*cut)(void *ctx, int i, hipStream_t s) = nullptr;
    void *ctx = nullptr;
    void mark(int i, hipStream_t s) const
    {
        if (cut) cut(ctx, i, s);
        else if (ev[i]) (void)hipEventRecord(ev[i], s);
    }
};
hipError_t launch_inexact(const fm_index *idx, const fm_tuning &t, const fm_tuning &tw, bool plain,
                          const DfsCall &c, hipStream_t s, const PhaseEvents *pe);

// Phase boundaries of the plan being captured on this thread (see fm_plan_create), or
// nullptr: search calls then record the index's own phase events, if any.
extern thread_local const PhaseEvents *g_plan_events;

int max_blocks_per_cu(const void *kernel, int block, size_t lds);

}  // namespace fm
