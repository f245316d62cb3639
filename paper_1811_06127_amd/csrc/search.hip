// search.hip -- backward searches on the interleaved layout.
//
//  walk kernels  : one left-to-right or right-to-left pass per read-strand with two Occ
//                  values per step. Mode EXACT is the backward exact match (Listing 1);
//                  modes DBP / DFULL compute BWA's D lower bound over the index of
//                  reverse(R) (breakpoint records for the DFS, or the full array).
//  dfs kernels   : inexact match with substitutions (Listing 2), one Occ8 per expanded
//                  node giving all four children at once.
//  compaction    : per-read status and counts -> CSR offsets -> hits grouped by read
//                  and sorted by (strand, k).
//
// Each search has a plain form (one thread per read-strand) and a batched form: a
// persistent grid whose lane groups (L lanes share one read-strand and split each
// bucket fetch between them) pull read-strands from a work queue in chunks, keep P
// read-strands in flight (walks) and keep DFS stacks in LDS.
#include "fm_internal.hpp"

namespace fm {

constexpr uint32_t kEmpty = 0xFFFFFFFFu;

// ------------------------------------------------------------------ work queue

// Per-wave view of the global work queue: the current chunk [qb, qe) of read-strands and,
// in lane 0, the start of the next chunk, claimed one chunk ahead so that taking work
// never waits for the atomic. The first chunk of every wave is its own without an atomic
// (wave w of the grid takes chunk w); the chunks after those are claimed from the queue
// counter, and not at all when the first chunks already cover the work, so a small
// launch makes no atomic on the shared counter. Dealt (the DFS with subtree transfers
// and a claim order): the first chunks are dealt round-robin instead, wave w taking
// items w, w + W, w + 2W, ... of the W waves' share, so that the heaviest read-strands,
// which the claim order puts first, land in different waves, where each has lanes of its
// own to help with it.
struct WaveQueue {
    uint32_t qb, qe;
    uint32_t nxt;          // lane 0: start of the next claimed chunk
    uint32_t fixed;        // items handed out as the waves' first chunks
    uint32_t chunk;        // items per chunk
    uint32_t wave, waves;  // this wave's index in the grid, and the grid's wave count
    uint32_t first;        // dealt: items in this wave's first chunk (0 once taken)
    bool dealt, strided;   // first chunks dealt; the current chunk is the dealt one
    bool exhausted;

    __device__ void start(uint32_t items_per_chunk, uint32_t total, bool deal)
    {
        const uint32_t wpb = blockDim.x / 64;
        qb = qe = 0;
        exhausted = false;
        chunk = items_per_chunk;
        waves = gridDim.x * wpb;
        wave = blockIdx.x * wpb + threadIdx.x / 64;
        fixed = waves * chunk;
        nxt = wave * chunk;
        dealt = deal;
        strided = false;
        const uint32_t share = fixed < total ? fixed : total;
        first = wave < share ? (share - wave + waves - 1) / waves : 0u;
    }

    // The chunk after the current one (lane 0): from the queue counter while work is left.
    __device__ uint32_t claim(uint32_t *queue, uint32_t total) const
    {
        return fixed >= total ? total : fixed + atomicAdd(queue, chunk);
    }
};

// Gives one item to every group of this wave whose `need` is set (need is uniform within
// a group); returns the group's item or kEmpty. Must be called by the whole wave.
template <int L>
__device__ uint32_t wave_take(WaveQueue &wq, bool need, uint32_t *queue, uint32_t total)
{
    const uint32_t lane = __lane_id(), lead = lane & ~(uint32_t)(L - 1);
    uint32_t got = kEmpty;
    uint64_t mask = __ballot(need && (lane & (L - 1)) == 0);
    while (mask) {
        if (wq.qb >= wq.qe) {
            if (wq.exhausted) break;
            if (wq.dealt) {
                // the dealt first chunk: positions 0 .. first - 1 stand for items wave + j * waves
                wq.dealt = false;
                wq.strided = true;
                wq.qb = 0;
                wq.qe = wq.first;
                if (lane == 0) wq.nxt = wq.claim(queue, total);
                continue;
            }
            const uint32_t base = (uint32_t)__builtin_amdgcn_readfirstlane((int)wq.nxt);
            if (base >= total) {
                wq.exhausted = true;
                break;
            }
            wq.strided = false;
            wq.qb = base;
            wq.qe = base + wq.chunk < total ? base + wq.chunk : total;
            if (lane == 0) wq.nxt = wq.claim(queue, total);
        }
        const uint32_t avail = wq.qe - wq.qb;
        const uint32_t r = lanes_below(mask) - ((lane != lead && ((mask >> lead) & 1ull)) ? 1u : 0u);
        const bool mine = need && ((mask >> lead) & 1ull) && r < avail;
        if (mine) got = wq.strided ? wq.wave + (wq.qb + r) * wq.waves : wq.qb + r;
        const uint32_t cnt = (uint32_t)__popcll(mask);
        wq.qb += cnt < avail ? cnt : avail;
        need = need && !mine;
        mask = __ballot(need && (lane & (L - 1)) == 0);
    }
    return got;
}

// Lanes of a wave that lead a group of L lanes.
template <int L>
__device__ constexpr uint64_t group_leads()
{
    return L == 1 ? ~0ull : (L == 2 ? 0x5555555555555555ull : (L == 4 ? 0x1111111111111111ull : 0x0101010101010101ull));
}

// Idle groups are refilled together once an eighth of the wave's groups is idle (or all
// are): the take and the header loads then run for many groups at once instead of in
// nearly every round, at the price of a few groups idling for a few rounds.
template <int L>
__device__ __forceinline__ bool refill_now(bool idle_lead)
{
    constexpr uint32_t th = (64 / L) / 8 ? (64 / L) / 8 : 1;
    const uint64_t idle = __ballot(idle_lead);
    return (uint32_t)__popcll(idle) >= th || idle == group_leads<L>();
}

__device__ __forceinline__ void wave_add(unsigned long long *dst, uint64_t v)
{
    if (!dst) return;
    for (int d = 32; d >= 1; d >>= 1) v += __shfl_xor(v, d);
    if (__lane_id() == 0 && v) atomicAdd(dst, (unsigned long long)v);
}

// ------------------------------------------------------------------ walks

struct WalkArgs {
    DevLayout lay;
    const uint8_t *codes;
    const uint64_t *offs;
    const uint8_t *z;
    uint32_t total;        // read-strands
    uint32_t nstr;         // strands per read (1 or 2)
    uint32_t strand0;      // strand searched when nstr == 1
    uint32_t zmax;
    void *out;
    uint64_t dstride;      // DFULL: bytes per strand block
    uint32_t *queue;
    unsigned long long *stat_steps, *stat_bk;
    uint32_t full_rank;    // EXACT: no early exit, report (k, l) as Listing 1 leaves it
};

template <int MODE>
struct Walker {
    uint32_t rs;           // read-strand, kEmpty when idle
    uint64_t addr;         // byte of `codes` holding the next pattern symbol
    uint32_t rem;          // symbols left
    int32_t dir;
    uint32_t comp;         // 1: complement symbols (strand 1)
    uint32_t k, l;
    uint32_t i;            // D modes: position in the strand pattern
    uint32_t cnt;          // D modes: failed segments so far
    uint32_t zr;           // DBP: the read's budget
    uint64_t outp;         // DFULL: output byte of position 0
    uint64_t bp03;         // DBP: positions of failures 1..4 (16 bits each, 0xFFFF: none)
    uint32_t bp4;          // DBP: position of failure 5
    bool fin;              // finished; the result is stored by retire()
    uint64_t wtag;         // 16-byte block of `codes` held in win, as its address / 16 (~0: none)
    uint4 win;

    // Loads the aligned 16-byte block that holds the next pattern symbol, unless win
    // already holds it (a block serves up to 16 steps). The block lies in the same page
    // as that symbol, so reading all of it cannot fault where it extends past the reads.
    __device__ void fetch_code(const WalkArgs &a)
    {
        const uint8_t *p = a.codes + addr;
        const uint64_t t = (uint64_t)(uintptr_t)p >> 4;
        if (t != wtag) {
            win = *(const uint4 *)(p - ((uintptr_t)p & 15u));
            wtag = t;
        }
    }

    __device__ uint32_t code(const WalkArgs &a) const
    {
        const uint32_t o = (uint32_t)((uintptr_t)(a.codes + addr) & 15u);
        return (sel4(o >> 2, win.x, win.y, win.z, win.w) >> (8 * (o & 3))) & 0xFFu;
    }

    __device__ void retire(const WalkArgs &a, bool lead_lane)
    {
        if (lead_lane) {
            if (MODE == WALK_EXACT) {
                ((uint2 *)a.out)[rs] = (k <= l || a.full_rank) ? make_uint2(k, l) : make_uint2(1u, 0u);
            } else if (MODE == WALK_DBP) {
                const uint32_t lo = (uint32_t)bp03, hi = (uint32_t)(bp03 >> 32);
                ((uint4 *)a.out)[rs] = make_uint4(cnt | (lo << 16), (lo >> 16) | (hi << 16), (hi >> 16) | (bp4 << 16), 0u);
            }
        }
        rs = kEmpty;
        fin = false;
    }

    // Header of a new read-strand: its offsets (and budget) are loaded here and used by
    // begin() one iteration later, so fetching them never delays the other lanes' steps.
    uint64_t h0, h1;
    uint32_t hz;

    __device__ void request(const WalkArgs &a, uint32_t item)
    {
        rs = item;
        const uint32_t read = a.nstr == 2 ? item >> 1 : item;
        h0 = a.offs[read];
        h1 = a.offs[read + 1];
        hz = MODE == WALK_DBP ? a.z[read] : 0u;
    }

    __device__ void init(const WalkArgs &a, uint32_t item, bool lead_lane)
    {
        request(a, item);
        begin(a, lead_lane);
    }

    __device__ void begin(const WalkArgs &a, bool lead_lane)
    {
        const uint32_t item = rs;
        const uint32_t strand = a.nstr == 2 ? (item & 1u) : a.strand0;
        const uint64_t b0 = h0;
        const uint32_t m = (uint32_t)(h1 - b0);
        // Listing 1 consumes the pattern right to left; the D walk left to right. The
        // strand-1 pattern is the reverse complement, so its direction flips.
        const bool asc = (MODE == WALK_EXACT) ? strand == 1 : strand == 0;
        addr = asc ? b0 : b0 + m - 1;
        dir = asc ? 1 : -1;
        comp = strand;
        rem = m;
        k = 0;
        l = a.lay.n;
        i = 0;
        cnt = 0;
        bp03 = ~0ull;
        bp4 = 0xFFFFu;
        wtag = ~0ull;
        if (MODE == WALK_DBP) zr = hz < a.zmax ? hz : a.zmax;
        if (MODE == WALK_DFULL) outp = (a.nstr == 2 ? strand : 0u) * a.dstride + b0;
        fin = m == 0;
    }

    // One step with pattern symbol c (already complemented for strand 1); ok/ol are
    // Occ(b, k-1), Occ(b, l), unused while the interval is still (0, n).
    __device__ void step(const WalkArgs &a, uint32_t b, uint32_t ok, uint32_t ol, bool lead_lane)
    {
        // From the root (0, n), Occ(b, -1) is zero and Occ(b, n) is read from the layout
        // like any other value (ol was computed at l = n), which gives C[b+1].
        const uint32_t cb = c_of(a.lay, b & 3);
        uint32_t nk = cb + (k ? ok : 0u) + 1;
        uint32_t nl = cb + ol;
        if (b > 3) {                                     // a non-base occurs nowhere
            // ranked above T (C = n, no occurrences) when the rank is reported
            nk = (MODE == WALK_EXACT && a.full_rank) ? a.lay.n + 1 : 1u;
            nl = (MODE == WALK_EXACT && a.full_rank) ? a.lay.n : 0u;
        }
        addr += dir;
        rem -= 1;
        if (MODE == WALK_EXACT) {
            k = nk;
            l = nl;
            fin = (nk > nl && !a.full_rank) || rem == 0;
            return;
        }
        const bool fail = nk > nl;                       // a difference is certain in this segment
        const uint32_t sh = 16u * (cnt & 3u);            // field of this failure (the cnt-th, 0-based)
        const uint64_t fm = (fail && cnt < 4) ? (0xFFFFull << sh) : 0ull;
        bp03 = (bp03 & ~fm) | (((uint64_t)(i & 0xFFFFu) << sh) & fm);
        bp4 = (fail && cnt == 4) ? (i & 0xFFFFu) : bp4;
        cnt += fail ? 1u : 0u;
        k = fail ? 0u : nk;
        l = fail ? a.lay.n : nl;
        if (MODE == WALK_DFULL && lead_lane) ((uint8_t *)a.out)[outp + i] = (uint8_t)(cnt < 255 ? cnt : 255);
        i += 1;
        fin = rem == 0 || (MODE == WALK_DBP && cnt > zr);
    }
};

__device__ __forceinline__ uint32_t strand_sym(uint32_t c, uint32_t comp) { return (comp && c < 4) ? 3u - c : c; }

// One walk from start to end on the calling lane (one thread per read-strand).
template <int I, int MODE>
__device__ void walk_one(const WalkArgs &a, uint32_t item, uint64_t &steps, uint64_t &bks)
{
    Walker<MODE> w;
    w.init(a, item, true);
    if (w.fin) w.retire(a, true);
    while (w.rs != kEmpty) {
        w.fetch_code(a);
        const uint32_t c = w.code(a);
        Pair<I, 1> pr;
        pr.load(a.lay, 0, w.k ? w.k : 1u, w.l);          // at the root only the bucket of l = n is used
        const uint32_t b = strand_sym(c, w.comp);
        uint32_t ok, ol;
        occ2<I, 1>(a.lay, pr, 0, b & 3, w.k ? w.k : 1u, w.l, ok, ol);
        if (a.stat_steps && w.k && b < 4) {
            ++steps;
            bks += pr.same ? 1 : 2;
        }
        w.step(a, b, ok, ol, true);
        if (w.fin) w.retire(a, true);
    }
}

template <int I, int MODE>
__global__ void __launch_bounds__(256) walk_plain(WalkArgs a)
{
    const uint32_t item = blockIdx.x * blockDim.x + threadIdx.x;
    if (item >= a.total) return;
    uint64_t steps = 0, bks = 0;
    walk_one<I, MODE>(a, item, steps, bks);
    if (a.stat_steps && steps) {
        atomicAdd(a.stat_steps, (unsigned long long)steps);
        atomicAdd(a.stat_bk, (unsigned long long)bks);
    }
}

// Exact intervals the DFS left undecided: read-strands of the DFS (dfs_total of them,
// dfs_nstr strands per read) whose search stopped before its end (FM_EINVAL, FM_ERANGE,
// FM_EBUDGET) get Listing 1's walk here, for the strands the exact output holds (a:
// the exact search's arguments). Grid-stride; nearly every read-strand only has its
// status read.
template <int I>
__global__ void __launch_bounds__(256) exact_rest(WalkArgs a, const uint32_t *rs_status, uint32_t dfs_total,
                                                  uint32_t dfs_nstr, uint32_t dfs_strand0)
{
    uint64_t steps = 0, bks = 0;
    for (uint32_t rs = blockIdx.x * blockDim.x + threadIdx.x; rs < dfs_total; rs += gridDim.x * blockDim.x) {
        const uint32_t st = rs_status[rs];
        if (st == FM_OK || st == FM_EOVERFLOW) continue;
        const uint32_t read = dfs_nstr == 2 ? rs >> 1 : rs;
        const uint32_t strand = dfs_nstr == 2 ? (rs & 1u) : dfs_strand0;
        if (a.nstr == 1 && strand != a.strand0) continue;
        walk_one<I, WALK_EXACT>(a, a.nstr == 2 ? 2 * read + strand : read, steps, bks);
    }
}

template <int I, int L, int P, int MODE>
__global__ void __launch_bounds__(256) walk_batched(WalkArgs a)
{
    const uint32_t q = L == 1 ? 0u : (__lane_id() & (L - 1));
    const bool lead = q == 0;
    Walker<MODE> w[P];
    bool pending[P];
#pragma unroll
    for (int p = 0; p < P; ++p) {
        w[p].rs = kEmpty;
        w[p].fin = false;
        pending[p] = false;
    }
    WaveQueue wq;
    wq.start(kQueueChunk, a.total, false);
    uint64_t steps = 0, bks = 0;
    for (;;) {
        // 1. the loads of every running slot
        Pair<I, L> pr[P];
#pragma unroll
        for (int p = 0; p < P; ++p) {
            const bool act = w[p].rs != kEmpty && !w[p].fin;
            if (act) w[p].fetch_code(a);
            pr[p].load(a.lay, q, act && w[p].k ? w[p].k : 1u, act ? w[p].l : 0u);
        }
        // 2. results of the read-strands that finished last round: stored after this
        //    round's loads, so waiting for those loads never waits for these stores, and
        //    the stores are complete before their registers are written again
#pragma unroll
        for (int p = 0; p < P; ++p)
            if (w[p].fin) w[p].retire(a, lead);
        // 3. idle slots take a read-strand and request its header, which arrives with the
        //    round's bucket loads; it begins in step 4 and steps from the next round
#pragma unroll
        for (int p = 0; p < P; ++p) {
            pending[p] = false;
            if (refill_now<L>(lead && w[p].rs == kEmpty)) {
                const uint32_t it = wave_take<L>(wq, w[p].rs == kEmpty, a.queue, a.total);
                pending[p] = it != kEmpty;
                if (pending[p]) w[p].request(a, it);
            }
        }
        bool any = false;
#pragma unroll
        for (int p = 0; p < P; ++p) any |= w[p].rs != kEmpty;
        const bool quit = !__any(any);     // tested at the end of the round, after every load is read
        // 4. steps of the running slots; pending ones begin
#pragma unroll
        for (int p = 0; p < P; ++p) {
            if (pending[p]) {
                w[p].begin(a, lead);
                continue;
            }
            if (w[p].rs == kEmpty) continue;
            const uint32_t b = strand_sym(w[p].code(a), w[p].comp);
            uint32_t ok, ol;
            occ2<I, L>(a.lay, pr[p], q, b & 3, w[p].k ? w[p].k : 1u, w[p].l, ok, ol);
            if (a.stat_steps && lead && w[p].k && b < 4) {
                ++steps;
                bks += pr[p].same ? 1 : 2;
            }
            w[p].step(a, b, ok, ol, lead);
        }
        // The round's loads are issued and read under different conditions; reading
        // their registers here on every path lets the compiler retire them now rather
        // than wait on every memory operation where the registers are next written.
#pragma unroll
        for (int p = 0; p < P; ++p) {
            asm volatile("" ::"v"(w[p].h0), "v"(w[p].h1), "v"(w[p].hz), "v"(w[p].win.x), "v"(w[p].win.y),
                         "v"(w[p].win.z), "v"(w[p].win.w));
#pragma unroll
            for (int t = 0; t < Bucket<I, L>::NPL; ++t)
                asm volatile("" ::"v"(pr[p].a.v[t].x), "v"(pr[p].a.v[t].y), "v"(pr[p].a.v[t].z), "v"(pr[p].a.v[t].w),
                             "v"(pr[p].b.v[t].x), "v"(pr[p].b.v[t].y), "v"(pr[p].b.v[t].z), "v"(pr[p].b.v[t].w));
        }
        if (quit) break;
    }
    wave_add(a.stat_steps, steps);
    wave_add(a.stat_bk, bks);
}

template <int I, int L, int P, int MODE>
static hipError_t walk_launch_batched(const fm_index *idx, const fm_tuning &t, const WalkArgs &a, hipStream_t s)
{
    const int block = (int)t.block;
    int per = max_blocks_per_cu((const void *)walk_batched<I, L, P, MODE>, block, 0);
    if (t.waves_per_cu) {
        int want = (int)(t.waves_per_cu * 64 / block);
        if (want >= 1 && want < per) per = want;
    }
    uint64_t grid = (uint64_t)idx->cu_count * per;
    const uint64_t need = ((uint64_t)a.total * L + block - 1) / block;
    if (need < grid) grid = need ? need : 1;
    hipLaunchKernelGGL((walk_batched<I, L, P, MODE>), dim3((uint32_t)grid), dim3(block), 0, s, a);
    return hipGetLastError();
}

template <int I, int L, int MODE>
static hipError_t walk_by_depth(const fm_index *idx, const fm_tuning &t, const WalkArgs &a, hipStream_t s)
{
    switch (t.depth) {
    case 1: return walk_launch_batched<I, L, 1, MODE>(idx, t, a, s);
    case 2: return walk_launch_batched<I, L, 2, MODE>(idx, t, a, s);
    default: return hipErrorInvalidValue;
    }
}

template <int I, int MODE>
static hipError_t walk_by_lanes(const fm_index *idx, const fm_tuning &t, const WalkArgs &a, hipStream_t s)
{
    switch (t.lanes) {
    case 1: return walk_by_depth<I, 1, MODE>(idx, t, a, s);
    case 2: return walk_by_depth<I, 2, MODE>(idx, t, a, s);
    case 4: if constexpr (Geo<I>::USED > 2) return walk_by_depth<I, 4, MODE>(idx, t, a, s); break;
    case 8: if constexpr (Geo<I>::USED > 4) return walk_by_depth<I, 8, MODE>(idx, t, a, s); break;
    default: break;
    }
    return hipErrorInvalidValue;
}

template <int MODE>
static hipError_t walk_dispatch(const fm_index *idx, const fm_tuning &t, bool plain, const WalkArgs &a, hipStream_t s)
{
    if (plain) {
        const uint32_t grid = (a.total + 255) / 256;
        switch (t.occ_interval) {
        case 64: hipLaunchKernelGGL((walk_plain<64, MODE>), dim3(grid), dim3(256), 0, s, a); break;
        case 96: hipLaunchKernelGGL((walk_plain<96, MODE>), dim3(grid), dim3(256), 0, s, a); break;
        case 128: hipLaunchKernelGGL((walk_plain<128, MODE>), dim3(grid), dim3(256), 0, s, a); break;
        case 192: hipLaunchKernelGGL((walk_plain<192, MODE>), dim3(grid), dim3(256), 0, s, a); break;
        case 224: hipLaunchKernelGGL((walk_plain<224, MODE>), dim3(grid), dim3(256), 0, s, a); break;
        case 256: hipLaunchKernelGGL((walk_plain<256, MODE>), dim3(grid), dim3(256), 0, s, a); break;
        case 448: hipLaunchKernelGGL((walk_plain<448, MODE>), dim3(grid), dim3(256), 0, s, a); break;
        default: return hipErrorInvalidValue;
        }
        return hipGetLastError();
    }
    switch (t.occ_interval) {
    case 64: return walk_by_lanes<64, MODE>(idx, t, a, s);
    case 96: return walk_by_lanes<96, MODE>(idx, t, a, s);
    case 128: return walk_by_lanes<128, MODE>(idx, t, a, s);
    case 192: return walk_by_lanes<192, MODE>(idx, t, a, s);
    case 224: return walk_by_lanes<224, MODE>(idx, t, a, s);
    case 256: return walk_by_lanes<256, MODE>(idx, t, a, s);
    case 448: return walk_by_lanes<448, MODE>(idx, t, a, s);
    default: return hipErrorInvalidValue;
    }
}

static uint32_t strand_count(uint32_t flags) { return ((flags & FM_FWD) ? 1u : 0u) + ((flags & FM_REVCOMP) ? 1u : 0u); }

hipError_t launch_walk(const fm_index *idx, const fm_tuning &t, int mode, bool plain, const WalkCall &c, hipStream_t s)
{
    WalkArgs a;
    const bool rev = mode != WALK_EXACT;
    a.lay = dev_layout(idx, t.occ_interval, rev);
    a.codes = c.codes;
    a.offs = c.offs;
    a.z = c.z;
    a.nstr = strand_count(c.flags);
    a.strand0 = (c.flags & FM_FWD) ? 0u : 1u;
    a.total = (uint32_t)(c.nreads * a.nstr);
    a.zmax = c.zmax;
    a.out = c.out;
    a.dstride = 0;
    a.queue = (uint32_t *)((char *)c.ws + kWsQueue);
    a.full_rank = (mode == WALK_EXACT && (c.flags & FM_FULL_RANK)) ? 1u : 0u;
    a.stat_steps = nullptr;
    a.stat_bk = nullptr;
    if ((c.flags & FM_STATS) && c.ws) {
        a.stat_steps = (unsigned long long *)((char *)c.ws + kWsStatWalk);
        a.stat_bk = (unsigned long long *)((char *)c.ws + kWsStatWalkBk);
    }
    if (a.total == 0) return hipSuccess;
    switch (mode) {
    case WALK_EXACT: return walk_dispatch<WALK_EXACT>(idx, t, plain, a, s);
    case WALK_DBP: return walk_dispatch<WALK_DBP>(idx, t, plain, a, s);
    default: return hipErrorInvalidValue;   // the full D array has its own entry (plain walk)
    }
}

hipError_t launch_darray_full(const fm_index *idx, const fm_tuning &t, const WalkCall &c, uint64_t total_len,
                              hipStream_t s)
{
    WalkArgs a;
    a.lay = dev_layout(idx, t.occ_interval, true);
    a.codes = c.codes;
    a.offs = c.offs;
    a.z = nullptr;
    a.nstr = strand_count(c.flags);
    a.strand0 = (c.flags & FM_FWD) ? 0u : 1u;
    a.total = (uint32_t)(c.nreads * a.nstr);
    a.zmax = 0;
    a.out = c.out;
    a.dstride = total_len;
    a.queue = nullptr;
    a.full_rank = 0;
    a.stat_steps = nullptr;
    a.stat_bk = nullptr;
    if (a.total == 0) return hipSuccess;
    return walk_dispatch<WALK_DFULL>(idx, t, true, a, s);
}

// ------------------------------------------------------------------ inexact DFS

struct DfsArgs {
    DevLayout lay;
    const uint8_t *codes;
    const uint64_t *offs;
    const uint8_t *z;
    const uint4 *bp;       // D breakpoint records per read-strand, or nullptr
    // claim order (nullptr: read-strand order): item j of the queue is the read-strand
    // whose header is rec[2j], rec[2j+1] (see order_place)
    const uint4 *rec;
    uint32_t total, nstr, strand0, zmax;
    uint32_t fcap;         // stack frames per read-strand: zmax (one more where lanes take
                           // subtrees from one another), plus one spare
    uint32_t budget;       // expanded nodes per read-strand
    uint32_t chunk;        // read-strands a wave takes from the work queue at once
    fm_hit *slots;         // kHitSlots hits per read-strand
    fm_hit *opool;         // hits beyond the slots
    uint64_t ocap;
    unsigned long long *ocount;
    // per read-strand: hits, status and expanded nodes of the lane that took it (its
    // owner), and the same summed over the subtrees other lanes took from it (see
    // dfs_steal; zeroed before the launch, nullptr when no launch lane steals)
    uint32_t *rs_count, *rs_status, *rs_nodes;
    uint32_t *tf_count, *tf_status, *tf_nodes;
    uint32_t *queue;
    unsigned long long *stat_occ, *stat_bk, *stat_steal;
    // exact intervals taken from the DFS (see dfs_emit), or ex_out == nullptr: ex_nstr
    // slots per read, for the strands in ex_strands (bit s: strand s)
    uint2 *ex_out;
    uint32_t ex_nstr, ex_strands;
    // prefix table (see table_level_base): substitution nodes whose matched suffix is
    // shorter than tdepth read their children from it (tdepth = 0: never)
    const uint4 *tab;
    uint32_t tdepth;
    unsigned long long *stat_tbl;
};

// Stack frame (48 bytes in LDS): the intervals of a node's four children and, in
// meta.x, the node's pattern position less one (bits 0-15), its remaining budget (16-19),
// its pattern symbol (20-23) and the children still to visit (24-27); in meta.y the code
// of the node's matched suffix (see Dfs::code).
struct Frame {
    uint4 k, l;
    uint4 meta;
};

struct Dfs {
    uint32_t rs;                    // kEmpty when idle
    uint32_t read, strand, m, z0;
    uint64_t base;
    uint64_t bp03;                  // D breakpoints 0..3, 16 bits each (0xFFFF: none)
    uint32_t bp4;                   // D breakpoint 4
    uint32_t i, zr, k, l;           // current node: pattern symbol i (>= 0) still to match
    // substitution search: code of the node's matched suffix S = W'[i+1 .. m-1], sum_j
    // S[j] 4^j (exact while S is shorter than the prefix table's depth, unused after)
    uint32_t code;
    uint32_t sp;                    // frames on the stack
    uint32_t hits, status, nodes;
    bool done;
    bool thief;                     // searching a subtree taken from another lane's stack
    // hits produced by the last expansion (children of a node with i == 0): bits 0-3 the
    // steps by b, bit 4 (gapped search) the deletion of the last symbol
    uint32_t pend, pk[5], pl[5], pd;
    // exact interval of the strand pattern: its hit with no substitution, (1, 0) while
    // there is none
    uint32_t ek, el;

    // First pattern position at which the D bound exceeds zc (0xFFFF: none).
    __device__ uint32_t bp_at(uint32_t zc) const
    {
        const uint32_t f = (uint32_t)(bp03 >> (16u * (zc & 3u))) & 0xFFFFu;
        return zc >= 4 ? bp4 : f;
    }

    // D(pos) > zc, i.e. a node that may still spend zc substitutions on pattern[0..pos]
    // cannot lead to a hit (pos = -1: nothing is left to match, never pruned).
    __device__ bool dprune(uint32_t zc, int pos) const { return (int)bp_at(zc) <= pos; }

    // 16-byte block of `codes` holding the pattern symbol in use (see Walker::fetch_code)
    uint64_t wtag;
    uint4 win;

    __device__ const uint8_t *code_ptr(const DfsArgs &a) const { return a.codes + base + (strand ? m - 1 - i : i); }

    __device__ void fetch_code(const DfsArgs &a)
    {
        const uint8_t *p = code_ptr(a);
        const uint64_t t = (uint64_t)(uintptr_t)p >> 4;
        if (t != wtag) {
            win = *(const uint4 *)(p - ((uintptr_t)p & 15u));
            wtag = t;
        }
    }

    // Pattern symbol i of the strand (complemented on strand 1). Every code above 3 is
    // returned as 4: such a symbol matches no base, and the frames keep it in 4 bits.
    __device__ uint32_t sym(const DfsArgs &a) const
    {
        const uint32_t o = (uint32_t)((uintptr_t)code_ptr(a) & 15u);
        const uint32_t c = (sel4(o >> 2, win.x, win.y, win.z, win.w) >> (8 * (o & 3))) & 0xFFu;
        return strand_sym(c < 4u ? c : 4u, strand);
    }

    // Header of a new read-strand (offsets, budget, D record): loaded into registers of
    // its own by request() and used by begin() after the round's loads have arrived.
    // With a claim order the header is one record: h0 = its start, h1 = its length, hrs
    // = the read-strand; the loads go straight into these registers, nothing waits.
    uint64_t h0, h1;
    uint32_t hz, hrs;
    uint4 hbp;

    __device__ void request(const DfsArgs &a, uint32_t item)
    {
        rs = item;                                   // busy from now on; begin() sets rs
        if (a.rec) {
            const uint4 r0 = a.rec[2 * (size_t)item], r1 = a.rec[2 * (size_t)item + 1];
            hrs = r0.x;
            h0 = u64_of(r0.y, r0.z);
            h1 = r0.w;
            hz = r1.x;
            hbp = make_uint4(r1.y, r1.z, r1.w, 0u);
            return;
        }
        hrs = item;
        const uint32_t rd = a.nstr == 2 ? item >> 1 : item;
        h0 = a.offs[rd];
        h1 = a.offs[rd + 1];
        hz = a.z[rd];
        hbp = a.bp ? a.bp[item] : make_uint4(0, 0, 0, 0);
    }

    __device__ void begin(const DfsArgs &a)
    {
        rs = hrs;
        read = a.nstr == 2 ? rs >> 1 : rs;
        strand = a.nstr == 2 ? (rs & 1u) : a.strand0;
        base = h0;
        m = a.rec ? (uint32_t)h1 : (uint32_t)(h1 - h0);
        z0 = hz;
        sp = 0;
        hits = 0;
        nodes = 0;
        thief = false;
        pd = 0;
        k = 0;
        l = a.lay.n;
        i = m - 1;
        zr = z0;
        code = 0;
        wtag = ~0ull;
        uint32_t nbp = 0;
        bp03 = ~0ull;
        bp4 = 0xFFFFu;
        if (a.bp) {
            const uint4 r = hbp;
            nbp = r.x & 0xFFFFu;
            bp03 = u64_of((r.x >> 16) | (r.y << 16), (r.y >> 16) | (r.z << 16));
            bp4 = r.z >> 16;
        }
        const bool bad_z = z0 > a.zmax, bad_m = m > 65535u;
        status = bad_z ? FM_EINVAL : (bad_m ? FM_ERANGE : FM_OK);
        // decided at once: invalid budget or length, root pruned (D(m-1) > z), or the
        // empty pattern, which matches every row with no substitution
        const bool ok = !bad_z && !bad_m && nbp <= z0;
        done = !ok || m == 0;
        pend = (ok && m == 0) ? 1u : 0u;
        pk[0] = 0;
        pl[0] = a.lay.n;
        ek = 1;
        el = 0;
    }
};

// Loads of one expansion, issued before anything waits on them: the symbol, the buckets
// (or, for a node whose matched suffix is shorter than the prefix table's depth, its
// children's 32 bytes of the table instead) and the frame on top of the stack, which is
// the one a pop takes (a node pops only when it pushes nothing).
template <int I, int L>
struct NodeLoads {
    Pair<I, L> pr;
    uint4 t0, t1;          // table: (k, l) of children 0, 1 and of children 2, 3
    bool tbl;
    uint4 tk, tl;
    uint2 tmeta;
};

// TB: the launch uses the prefix table (one lane per read-strand, substitution search);
// without it the kernel keeps no suffix codes at all.
template <int I, int L, bool TB>
__device__ __forceinline__ void dfs_load(const DfsArgs &a, Dfs &d, uint32_t q, const Frame *fr, NodeLoads<I, L> &nl)
{
    d.fetch_code(a);
    nl.tbl = false;
    if constexpr (TB) {
        const uint32_t depth = d.m - 1 - d.i;        // length of the matched suffix
        nl.tbl = d.k != 0 && depth < a.tdepth;
        if (nl.tbl) {
            const uint4 *t = a.tab + (table_level_base(depth + 1) / 2 + 2 * (uint64_t)d.code);
            nl.t0 = t[0];
            nl.t1 = t[1];
            nl.pr.same = true;
        } else {
            nl.pr.load(a.lay, q, d.k ? d.k : 1u, d.l);
        }
    } else {
        nl.pr.load(a.lay, q, d.k ? d.k : 1u, d.l);
    }
    const Frame *ft = fr + (d.sp ? d.sp - 1 : a.fcap - 1);
    nl.tk = ft->k;
    nl.tl = ft->l;
    nl.tmeta = make_uint2(ft->meta.x, TB ? ft->meta.y : 0u);
}

// Expands the current node: one Occ8 at (k-1, l) gives the intervals of all four
// one-symbol extensions (Listing 2's loop over b, each computed from the parent's
// interval and kept only when k_b <= l_b). Children needing more substitutions than
// remain, or than the D bound allows, are dropped. At i == 0 the survivors are hits.
// Otherwise a mismatch child, if any, is continued and the node's other survivors are
// pushed as one frame; frames hand out their mismatch children first and the match
// child last, so the current node descends from a mismatch child of every node with a
// frame on the stack, and at most z frames are stacked that way. In the tail of a
// launch (sf: lanes are taking subtrees from one another, see dfs_steal) a node whose
// stack is empty instead continues with its match child and leaves all its mismatch
// children in the one frame, where idle lanes take them: the path that matches every
// symbol, which no other lane can take, is then walked without waiting for those
// subtrees. That frame is the bottom one, so the stack holds at most z + 1 frames. A
// bottom frame whose children other lanes took is dropped. Frame `fcap - 1` is a spare
// that absorbs the writes and reads of lanes that neither push nor pop, which keeps the
// update free of branches.
template <int I, int L, bool TB>
__device__ __forceinline__ void dfs_expand(const DfsArgs &a, Dfs &d, const NodeLoads<I, L> &nl, uint32_t q,
                                           Frame *fr, bool lead, bool sf, uint64_t &n_occ, uint64_t &n_bk,
                                           uint64_t &n_tb)
{
    const uint32_t kk = d.k ? d.k : 1u;
    const uint32_t wi = d.sym(a);
    const bool root = d.k == 0;
    const uint32_t C0 = a.lay.C[0], C1 = a.lay.C[1], C2 = a.lay.C[2], C3 = a.lay.C[3];
    uint32_t kb[4], lb[4];
    if (TB && nl.tbl) {
        // the children's intervals as the table holds them (Listing 1 from (0, n))
        kb[0] = nl.t0.x;
        lb[0] = nl.t0.y;
        kb[1] = nl.t0.z;
        lb[1] = nl.t0.w;
        kb[2] = nl.t1.x;
        lb[2] = nl.t1.y;
        kb[3] = nl.t1.z;
        lb[3] = nl.t1.w;
    } else {
        Occ4 o1, o2;
        occ8<I, L>(a.lay, nl.pr, q, kk, d.l, o1, o2);
        // children; at the root (0, n) Occ(., -1) is zero and Occ(., n) is every symbol's total
        kb[0] = C0 + 1 + (root ? 0u : o1.a);
        kb[1] = C1 + 1 + (root ? 0u : o1.c);
        kb[2] = C2 + 1 + (root ? 0u : o1.g);
        kb[3] = C3 + 1 + (root ? 0u : o1.t);
        lb[0] = C0 + o2.a;
        lb[1] = C1 + o2.c;
        lb[2] = C2 + o2.g;
        lb[3] = C3 + o2.t;
    }
    if (a.stat_occ && lead) {
        n_occ += 1;
        n_bk += (root || nl.tbl) ? 0 : (nl.pr.same ? 1 : 2);
        n_tb += nl.tbl ? 1 : 0;
    }
    // surviving children
    const int cpos = (int)d.i - 1;
    const bool keep_match = !d.dprune(d.zr, cpos);
    const bool keep_mism = d.zr >= 1 && !d.dprune(d.zr - 1, cpos);
    const uint32_t mbit = wi < 4 ? 1u << wi : 0u;
    uint32_t le = 0;
#pragma unroll
    for (int b = 0; b < 4; ++b) le |= kb[b] <= lb[b] ? (1u << b) : 0u;
    const uint32_t valid = le & ((keep_match ? mbit : 0u) | (keep_mism ? (0xFu & ~mbit) : 0u));
    const bool leaf = d.i == 0;
    // hits
    d.pend = leaf ? valid : 0u;
#pragma unroll
    for (int b = 0; b < 4; ++b) {
        d.pk[b] = kb[b];
        d.pl[b] = lb[b];
    }
    d.pd = (d.z0 - d.zr) | (wi << 8);
    // a bottom frame emptied by other lanes is dropped (it is the top one only when alone)
    const uint32_t sp = (d.sp == 1 && ((nl.tmeta.x >> 24) & 0xFu) == 0) ? 0u : d.sp;
    // continue with a mismatch child if there is one, else with the match child; the
    // other survivors of a node that continues with a mismatch go into a frame (in the
    // tail, a node with an empty stack continues with the match child instead)
    const uint32_t go = leaf ? 0u : valid;
    const uint32_t mism = go & ~mbit;
    const bool advance = go != 0;
    const bool spine = sf && sp == 0 && mism != 0 && (go & mbit) != 0;
    const uint32_t cont = (mism && !spine) ? (uint32_t)__builtin_ctz(mism) : (wi & 3u);
    const uint32_t rest = spine ? mism : (mism ? (go & ~(1u << cont)) : 0u);
    const uint32_t ci = d.i - 1;
    const uint32_t spare = a.fcap - 1;
    Frame *fw = fr + (rest ? sp : spare);
    if (lead) {
        fw->k = make_uint4(kb[0], kb[1], kb[2], kb[3]);
        fw->l = make_uint4(lb[0], lb[1], lb[2], lb[3]);
        fw->meta.x = (ci & 0xFFFFu) | (d.zr << 16) | (wi << 20) | (rest << 24);
        if constexpr (TB) fw->meta.y = d.code;
    }
    const uint32_t nsp = sp + (rest ? 1u : 0u);
    // otherwise the next node comes from the top frame: a mismatch child while there is
    // one, then the match child, which retires the frame
    const bool pop = !advance && nsp > 0;
    Frame *ft = fr + (pop ? nsp - 1 : spare);
    const uint4 tk = nl.tk, tl = nl.tl;
    const uint32_t meta = nl.tmeta.x;
    const uint32_t trest = (meta >> 24) & 0xFu, twi = (meta >> 20) & 0xFu;
    const uint32_t tmm = trest & ~(twi < 4 ? 1u << twi : 0u);
    const uint32_t bt = (uint32_t)__builtin_ctz((tmm ? tmm : trest) | 0x10u) & 3u;
    const uint32_t left = trest & ~(1u << bt);
    if (lead) ft->meta.x = (meta & 0x00FFFFFFu) | (left << 24);
    d.k = advance ? sel4(cont, kb[0], kb[1], kb[2], kb[3]) : sel4(bt, tk.x, tk.y, tk.z, tk.w);
    d.l = advance ? sel4(cont, lb[0], lb[1], lb[2], lb[3]) : sel4(bt, tl.x, tl.y, tl.z, tl.w);
    d.i = advance ? ci : (meta & 0xFFFFu);
    if constexpr (TB) d.code = advance ? (d.code << 2) | cont : (nl.tmeta.y << 2) | bt;
    d.zr = advance ? d.zr - (cont != wi ? 1u : 0u) : ((meta >> 16) & 0xFu) - (bt != twi ? 1u : 0u);
    d.sp = pop && !left ? nsp - 1 : nsp;
    d.done = !advance && !pop;
    d.nodes += 1;
    if (!d.done && d.nodes >= a.budget) {
        d.status = FM_EBUDGET;
        d.done = true;
    }
}

// DFS kinds: substitutions (Listing 2's substitution branches), the same with the exact
// intervals taken from it (see dfs_emit), and Listing 2 with all its branches.
enum { kDfsSub = 0, kDfsSubExact = 1, kDfsGap = 2 };

// Loads of one gapped expansion: as dfs_load, with the whole top frame (the gapped frame
// also holds its node's interval and the children still to visit).
template <int I, int L>
struct GapLoads {
    Pair<I, L> pr;
    uint4 tk, tl, tmeta;
};

template <int I, int L>
__device__ __forceinline__ void gap_load(const DfsArgs &a, Dfs &d, uint32_t q, const Frame *fr, GapLoads<I, L> &nl)
{
    d.fetch_code(a);
    nl.pr.load(a.lay, q, d.k ? d.k : 1u, d.l);
    const Frame *ft = fr + (d.sp ? d.sp - 1 : a.fcap - 1);
    nl.tk = ft->k;
    nl.tl = ft->l;
    nl.tmeta = ft->meta;
}

// Child `c` of a gapped node (i, zr, interval (k, l), pattern symbol wi, child intervals
// kb, lb): c = 0-3 the step by symbol c (to i - 1, a substitution unless c = wi), 4-7
// the insertion of symbol c - 4 (stays at i), 8 the deletion of pattern symbol i (to
// i - 1, same interval). Every one but a matching step costs 1.
__device__ __forceinline__ void gap_child(uint32_t c, uint32_t i, uint32_t zr, uint32_t wi, uint32_t k, uint32_t l,
                                          const uint4 &kb, const uint4 &lb, uint32_t &ni, uint32_t &nz, uint32_t &nk,
                                          uint32_t &nl)
{
    const uint32_t b = c & 3u;
    const bool del = c >= 8;
    ni = (c >= 4 && c < 8) ? i : i - 1;
    nz = zr - ((c < 4 && c == wi) ? 0u : 1u);
    nk = del ? k : sel4(b, kb.x, kb.y, kb.z, kb.w);
    nl = del ? l : sel4(b, lb.x, lb.y, lb.z, lb.w);
}

// Expands a node of Listing 2 with all its branches. One Occ8 at (k-1, l) gives the
// intervals of the four one-symbol extensions, which serve both the steps over pattern
// symbol i and the insertions before it; the deletion keeps the node's interval. A child
// is dropped when its interval is empty or when its remaining budget is below the D
// bound of the pattern left to match (positions i - 1 for steps and the deletion, i for
// insertions). At i == 0 the steps and the deletion are hits and only insertions go on.
// The node continues with a costly child if there is one and pushes the rest as one
// frame (children: bits 0-3 steps, 4-7 insertions, 8 deletion, with the node's i, budget,
// symbol and interval); frames hand out costly children first and the matching step
// last, so every frame on the stack lies on a costly edge of the current path and at
// most z frames are stacked, as in the substitution search.
template <int I, int L>
__device__ __forceinline__ void gap_expand(const DfsArgs &a, Dfs &d, const GapLoads<I, L> &nl, uint32_t q,
                                           Frame *fr, bool lead, uint64_t &n_occ, uint64_t &n_bk)
{
    const uint32_t kk = d.k ? d.k : 1u;
    const uint32_t wi = d.sym(a);
    Occ4 o1, o2;
    occ8<I, L>(a.lay, nl.pr, q, kk, d.l, o1, o2);
    const bool root = d.k == 0;
    const uint32_t C0 = a.lay.C[0], C1 = a.lay.C[1], C2 = a.lay.C[2], C3 = a.lay.C[3];
    const uint4 kb = make_uint4(C0 + 1 + (root ? 0u : o1.a), C1 + 1 + (root ? 0u : o1.c),
                                C2 + 1 + (root ? 0u : o1.g), C3 + 1 + (root ? 0u : o1.t));
    const uint4 lb = make_uint4(C0 + o2.a, C1 + o2.c, C2 + o2.g, C3 + o2.t);
    if (a.stat_occ && lead) {
        n_occ += 1;
        n_bk += root ? 0 : (nl.pr.same ? 1 : 2);
    }
    const int ipos = (int)d.i, cpos = ipos - 1;
    const bool keep_match = !d.dprune(d.zr, cpos);
    const bool keep_costly = d.zr >= 1 && !d.dprune(d.zr - 1, cpos);   // substitutions, the deletion
    const bool keep_ins = d.zr >= 1 && !d.dprune(d.zr - 1, ipos);
    const uint32_t mbit = wi < 4 ? 1u << wi : 0u;
    const uint32_t le = (kb.x <= lb.x ? 1u : 0u) | (kb.y <= lb.y ? 2u : 0u) | (kb.z <= lb.z ? 4u : 0u) |
                        (kb.w <= lb.w ? 8u : 0u);
    const uint32_t step = le & ((keep_match ? mbit : 0u) | (keep_costly ? (0xFu & ~mbit) : 0u));
    const uint32_t ins = keep_ins ? le : 0u;
    const uint32_t del = keep_costly ? 1u : 0u;
    const bool leaf = d.i == 0;
    d.pend = leaf ? (step | (del << 4)) : 0u;
    d.pk[0] = kb.x, d.pk[1] = kb.y, d.pk[2] = kb.z, d.pk[3] = kb.w, d.pk[4] = d.k;
    d.pl[0] = lb.x, d.pl[1] = lb.y, d.pl[2] = lb.z, d.pl[3] = lb.w, d.pl[4] = d.l;
    d.pd = (d.z0 - d.zr) | (wi << 8);
    const uint32_t go = (leaf ? 0u : (step | (del << 8))) | (ins << 4);
    const uint32_t costly = go & ~mbit;
    const bool advance = go != 0;
    const uint32_t cont = (uint32_t)__builtin_ctz((costly ? costly : go) | 0x200u);
    const uint32_t rest = costly ? (go & ~(1u << cont)) : 0u;
    const uint32_t spare = a.fcap - 1;
    // a bottom frame emptied by other lanes (dfs_steal) is dropped
    const uint32_t sp = (d.sp == 1 && (nl.tmeta.w & 0x1FFu) == 0) ? 0u : d.sp;
    Frame *fw = fr + (rest ? sp : spare);
    if (lead) {
        fw->k = kb;
        fw->l = lb;
        fw->meta = make_uint4((d.i & 0xFFFFu) | (d.zr << 16) | (wi << 20), d.k, d.l, rest);
    }
    const uint32_t nsp = sp + (rest ? 1u : 0u);
    // otherwise the next node comes from the top frame: a costly child while there is one,
    // then the matching step, which retires the frame
    const bool pop = !advance && nsp > 0;
    Frame *ft = fr + (pop ? nsp - 1 : spare);
    const uint4 tm = nl.tmeta;
    const uint32_t trest = tm.w & 0x1FFu, twi = (tm.x >> 20) & 0xFu;
    const uint32_t tcostly = trest & ~(twi < 4 ? 1u << twi : 0u);
    const uint32_t bt = (uint32_t)__builtin_ctz((tcostly ? tcostly : trest) | 0x200u);
    const uint32_t left = trest & ~(1u << bt);
    if (lead) ft->meta.w = left;
    uint32_t ai, az, ak, al, pi, pz, pk, pl;
    gap_child(cont, d.i, d.zr, wi, d.k, d.l, kb, lb, ai, az, ak, al);
    gap_child(bt, tm.x & 0xFFFFu, (tm.x >> 16) & 0xFu, twi, tm.y, tm.z, nl.tk, nl.tl, pi, pz, pk, pl);
    d.i = advance ? ai : pi;
    d.zr = advance ? az : pz;
    d.k = advance ? ak : pk;
    d.l = advance ? al : pl;
    d.sp = pop && !left ? nsp - 1 : nsp;
    d.done = !advance && !pop;
    d.nodes += 1;
    if (!d.done && d.nodes >= a.budget) {
        d.status = FM_EBUDGET;
        d.done = true;
    }
}

// Stores the hits of the last expansion: the first kHitSlots hits of a read-strand go
// to its own slots with plain stores; later ones are appended to the overflow pool
// (one atomic per wave, rarely needed). Then retires finished read-strands. Must be
// called by the whole wave.
//
// With XD the exact intervals come out of the same DFS. The path that matches every
// symbol is Listing 1's search: its node intervals are computed by the same update,
// and the D bound never prunes it when the pattern occurs (D is then zero). So a
// read-strand whose DFS runs to the end (FM_OK, or FM_EOVERFLOW, which still explores
// everything) has as exact interval its hit with no substitution, or none; a root
// pruned by D (D(m-1) > z >= 0) has none either. A DFS that stops early leaves its
// interval to exact_rest.
template <int L, int K, bool S>
__device__ void dfs_emit(const DfsArgs &a, Dfs &d, bool active, bool lead)
{
    constexpr bool XD = K == kDfsSubExact;
    constexpr int NB = K == kDfsGap ? 5 : 4;   // hit kinds: steps by b, and the deletion (gapped)
    const uint32_t pend = active ? d.pend : 0u;
    const uint32_t wi = d.pd >> 8;
    uint32_t over = 0;                        // children whose hit goes to the overflow pool
    if (pend) {
        if (XD && (d.pd & 0xFFu) == 0 && wi < 4 && ((pend >> wi) & 1u)) {
            d.ek = sel4(wi, d.pk[0], d.pk[1], d.pk[2], d.pk[3]);
            d.el = sel4(wi, d.pl[0], d.pl[1], d.pl[2], d.pl[3]);
        }
        uint32_t h = d.hits;
#pragma unroll
        for (int b = 0; b < NB; ++b) {
            if ((pend >> b) & 1u) {
                const uint32_t nmm = (d.pd & 0xFFu) + ((b == 4 || (uint32_t)b != wi) ? 1u : 0u);
                if (h < kHitSlots && !(S && d.thief)) {
                    if (lead)
                        ((uint4 *)a.slots)[(size_t)d.rs * kHitSlots + h] =
                            make_uint4(d.read, d.pk[b], d.pl[b], d.strand | (nmm << 8));
                } else {
                    over |= 1u << b;
                }
                ++h;
            }
        }
    }
    if (__ballot(over != 0)) {
        const uint32_t lane = __lane_id(), leadlane = lane & ~(uint32_t)(L - 1);
        uint64_t mb[NB];
        uint32_t tot = 0;
#pragma unroll
        for (int b = 0; b < NB; ++b) {
            mb[b] = __ballot(lead && ((over >> b) & 1u));
            tot += (uint32_t)__popcll(mb[b]);
        }
        unsigned long long base = 0;
        if (lane == 0) base = atomicAdd(a.ocount, (unsigned long long)tot);
        base = __shfl(base, 0);
        uint64_t off = base;
#pragma unroll
        for (int b = 0; b < NB; ++b) {
            if ((over >> b) & 1u) {
                const uint64_t pos = off + rank_below(mb[b], leadlane);
                const uint32_t nmm = (d.pd & 0xFFu) + ((b == 4 || (uint32_t)b != wi) ? 1u : 0u);
                if (pos < a.ocap) {
                    if (lead) ((uint4 *)a.opool)[pos] = make_uint4(d.read, d.pk[b], d.pl[b], d.strand | (nmm << 8));
                } else {
                    d.status = d.status > FM_EOVERFLOW ? d.status : FM_EOVERFLOW;   // a spent budget wins
                }
            }
            off += (uint64_t)__popcll(mb[b]);
        }
    }
    if (active) {
        d.hits += (uint32_t)__popc(pend);
        d.pend = 0;
        if (d.done) {
            if (S && lead && d.thief) {
                // a stolen subtree adds its part
                atomicAdd(&a.tf_count[d.rs], d.hits);
                atomicMax(&a.tf_status[d.rs], d.status);
                atomicAdd(&a.tf_nodes[d.rs], d.nodes);
            } else if (lead) {
                // the owner, whose first kHitSlots hits are in the slots and who followed the
                // path that matches every symbol (the exact interval)
                a.rs_count[d.rs] = d.hits;
                a.rs_status[d.rs] = d.status;
                if (S) a.rs_nodes[d.rs] = d.nodes;
                const uint32_t ran_to_end = (1u << FM_OK) | (1u << FM_EOVERFLOW);
                if (XD && ((a.ex_strands >> d.strand) & 1u) && ((ran_to_end >> d.status) & 1u))
                    a.ex_out[(size_t)d.read * a.ex_nstr + (a.ex_nstr == 2 ? d.strand : 0u)] = make_uint2(d.ek, d.el);
            }
            d.rs = kEmpty;
        }
    }
}

template <int I, int K, bool TB>
__global__ void __launch_bounds__(256) dfs_plain(DfsArgs a)
{
    extern __shared__ Frame lds_frames[];
    const uint32_t item = blockIdx.x * blockDim.x + threadIdx.x;
    Frame *fr = lds_frames + (size_t)threadIdx.x * a.fcap;
    Dfs d;
    d.rs = kEmpty;
    d.done = false;
    if (item < a.total) {
        d.request(a, item);
        d.begin(a);
    }
    uint64_t n_occ = 0, n_bk = 0, n_tb = 0;
    for (;;) {
        const bool active = d.rs != kEmpty;
        if (!__any(active)) break;
        if (active && !d.done) {
            if constexpr (K == kDfsGap) {
                GapLoads<I, 1> nl;
                gap_load<I, 1>(a, d, 0, fr, nl);
                gap_expand<I, 1>(a, d, nl, 0, fr, true, n_occ, n_bk);
            } else {
                NodeLoads<I, 1> nl;
                dfs_load<I, 1, TB>(a, d, 0, fr, nl);
                dfs_expand<I, 1, TB>(a, d, nl, 0, fr, true, false, n_occ, n_bk, n_tb);
            }
        }
        dfs_emit<1, K, false>(a, d, active, true);
    }
    wave_add(a.stat_occ, n_occ);
    wave_add(a.stat_bk, n_bk);
    wave_add(a.stat_tbl, n_tb);
}

// Each round: idle groups (refilled in batches) take read-strands and issue their
// header loads; running groups issue their node loads and expand their nodes, by which
// time the older header loads have arrived too; new read-strands begin; hits are stored
// and finished read-strands retired. K: the kind of search (kDfsSubExact: exact intervals
// as well, see dfs_emit; kDfsGap: Listing 2 with all its branches).
// The tail of a launch: once the work queue is exhausted, lanes fall idle while the
// last trees are still being searched. Idle lanes then take pending costly children (a
// substitution, or in the gapped search also an insertion or the deletion) from the
// lowest (shallowest, so largest) frames that have them in busy lanes of their wave and
// search those subtrees of the same read-strands. Every idle lane can take one child per
// round: the children on offer are numbered in lane order, the r-th idle lane takes
// child r, and each donor clears the children it gave from its own frame (the gapped
// search gives only children left with a budget of one or more). The child that matches
// is never taken, so the path that matches every symbol (and with it the exact interval)
// stays with the owner; a bottom frame left with no child is dropped by its owner
// (dfs_expand, gap_expand), and a frame above it always keeps one. Hits of a stolen subtree go to the overflow
// pool; its hit count, status and node count are summed per read-strand apart from the
// owner's (tf_*), and the compaction adds the two. One lane per read-strand only (frames
// are per lane).
template <int K>
__device__ __forceinline__ void dfs_steal(const DfsArgs &a, Dfs &d, Frame *frames, Frame *fr, uint64_t &n_steal)
{
    constexpr bool G = K == kDfsGap;
    const uint32_t lane = __lane_id();
    const bool busy = d.rs != kEmpty;
    const uint64_t idle = __ballot(!busy);
    if (!idle) return;
    // The lowest frame of this lane with children to give (its node's budget and symbol, and
    // the children still to visit): a costly child can leave the bottom frame whatever else
    // stays (an emptied bottom frame is dropped by its owner), a frame above it only while
    // another child stays, so those frames never empty. The gapped search gives away only
    // children left with a budget of one or more (its zero-budget subtrees are short and
    // many: measured no faster to share).
    uint4 m = make_uint4(0u, 0u, 0u, 0u);
    uint32_t fsel = 0, pend = 0, costly = 0, cnt = 0;
    if (busy) {
        for (uint32_t f = 0; f < d.sp && cnt == 0; ++f) {
            const uint4 mf = fr[f].meta;
            const uint32_t pf = G ? (mf.w & 0x1FFu) : ((mf.x >> 24) & 0xFu);
            const uint32_t wf = (mf.x >> 20) & 0xFu;
            const bool ok = !G || ((mf.x >> 16) & 0xFu) >= 2;
            const uint32_t cf = ok ? pf & ~(wf < 4 ? 1u << wf : 0u) : 0u;
            const uint32_t nc = (uint32_t)__popc(cf), np = (uint32_t)__popc(pf);
            const uint32_t can = (f == 0 || nc < np) ? nc : np - 1;
            if (can) {
                fsel = f;
                m = mf;
                pend = pf;
                costly = cf;
                cnt = can;
            }
        }
    }
    const uint32_t wi = (m.x >> 20) & 0xFu;
    // numbering: this lane's costly children start at pre; the wave has tot of them
    uint32_t pre = 0, tot = 0;
#pragma unroll
    for (int bit = 0; bit < 4; ++bit) {
        const uint64_t bb = __ballot((cnt >> bit) & 1u);
        pre += lanes_below(bb) << bit;
        tot += (uint32_t)__popcll(bb) << bit;
    }
    if (tot == 0) return;
    const uint32_t nidle = (uint32_t)__popcll(idle);
    // a donor gives its children numbered below the idle count, lowest first
    const uint32_t given = pre >= nidle ? 0u : (cnt < nidle - pre ? cnt : nidle - pre);
    if (given) {
        uint32_t rem = costly, gone = 0;
        for (uint32_t g = 0; g < given; ++g) {
            const uint32_t lo = rem & (0u - rem);
            gone |= lo;
            rem ^= lo;
        }
        const uint32_t left = pend & ~gone;
        if constexpr (G)
            fr[fsel].meta.w = left;
        else
            fr[fsel].meta.x = (m.x & 0x00FFFFFFu) | (left << 24);
    }
    // an idle lane of rank r takes child r: its donor is the first lane whose numbering
    // ends above r
    const uint32_t r = lanes_below(idle);
    const bool take = !busy && r < tot;
    const uint32_t end = pre + cnt;
    uint32_t v = 0;
#pragma unroll
    for (uint32_t step = 32; step >= 1; step >>= 1) {
        const uint32_t e = __shfl(end, (int)(v + step - 1));
        v += e <= r ? step : 0u;
    }
    const uint32_t vpre = __shfl(pre, (int)v), vcost = __shfl(costly, (int)v), vf = __shfl(fsel, (int)v);
    const uint32_t vmx = __shfl(m.x, (int)v), vmy = __shfl(m.y, (int)v), vmz = __shfl(m.z, (int)v);
    const uint32_t vrs = __shfl(d.rs, (int)v), vread = __shfl(d.read, (int)v);
    const uint32_t vstrand = __shfl(d.strand, (int)v), vm = __shfl(d.m, (int)v), vz0 = __shfl(d.z0, (int)v);
    const uint32_t vb0 = __shfl((uint32_t)d.base, (int)v), vb1 = __shfl((uint32_t)(d.base >> 32), (int)v);
    const uint32_t vp0 = __shfl((uint32_t)d.bp03, (int)v), vp1 = __shfl((uint32_t)(d.bp03 >> 32), (int)v);
    const uint32_t vbp4 = __shfl(d.bp4, (int)v);
    if (!take) return;
    if (a.stat_steal) n_steal += 1;
    // the (r - vpre)-th costly child of the donor's frame, counting from the lowest
    uint32_t x = vcost;
    for (uint32_t g = r - vpre; g > 0; --g) x &= x - 1;
    const uint32_t c = (uint32_t)__builtin_ctz(x);
    const Frame *df = frames + (size_t)(threadIdx.x - lane + v) * a.fcap + vf;
    const uint32_t vwi = (vmx >> 20) & 0xFu, vzr = (vmx >> 16) & 0xFu;
    const uint4 kk = df->k, ll = df->l;
    if constexpr (G) {
        gap_child(c, vmx & 0xFFFFu, vzr, vwi, vmy, vmz, kk, ll, d.i, d.zr, d.k, d.l);
    } else {
        d.k = sel4(c, kk.x, kk.y, kk.z, kk.w);
        d.l = sel4(c, ll.x, ll.y, ll.z, ll.w);
        d.i = vmx & 0xFFFFu;
        d.code = (vmy << 2) | c;
        d.zr = vzr - 1u;
    }
    d.rs = vrs;
    d.read = vread;
    d.strand = vstrand;
    d.m = vm;
    d.z0 = vz0;
    d.base = u64_of(vb0, vb1);
    d.bp03 = u64_of(vp0, vp1);
    d.bp4 = vbp4;
    d.sp = 0;
    d.hits = 0;
    d.nodes = 0;
    d.status = FM_OK;
    d.done = false;
    d.thief = true;
    d.pend = 0;
    d.pd = 0;
    d.wtag = ~0ull;
    d.ek = 1;
    d.el = 0;
}

// S: lanes take subtrees from one another at the end of the launch (dfs_steal). TB: the
// prefix table serves shallow nodes (dfs_load).
template <int I, int L, int K, bool S, bool TB>
__global__ void __launch_bounds__(256) dfs_batched(DfsArgs a)
{
    extern __shared__ Frame lds_frames[];
    const uint32_t q = L == 1 ? 0u : (__lane_id() & (L - 1));
    const bool lead = q == 0;
    Frame *fr = lds_frames + (size_t)(threadIdx.x / L) * a.fcap;
    Dfs d;
    d.rs = kEmpty;
    d.done = false;
    WaveQueue wq;
    wq.start(a.chunk, a.total, S && a.rec != nullptr);
    uint64_t n_occ = 0, n_bk = 0, n_tb = 0, n_steal = 0;
    for (;;) {
        if constexpr (S) {
            if (wq.exhausted) dfs_steal<K>(a, d, lds_frames, fr, n_steal);
        }
        const bool running = d.rs != kEmpty;
        bool fresh = false;
        if (refill_now<L>(lead && !running)) {
            const uint32_t it = wave_take<L>(wq, !running, a.queue, a.total);
            if (it != kEmpty) {
                fresh = true;
                d.request(a, it);
            }
        }
        if (running) {
            if constexpr (K == kDfsGap) {
                GapLoads<I, L> nl;
                gap_load<I, L>(a, d, q, fr, nl);
                gap_expand<I, L>(a, d, nl, q, fr, lead, n_occ, n_bk);
            } else {
                NodeLoads<I, L> nl;
                dfs_load<I, L, TB>(a, d, q, fr, nl);
                dfs_expand<I, L, TB>(a, d, nl, q, fr, lead, S && wq.exhausted, n_occ, n_bk, n_tb);
            }
        }
        if (fresh) d.begin(a);
        // The header registers are loaded and read under two separate conditions; reading
        // them here on every path lets the compiler retire those loads now instead of
        // waiting on all memory operations where the registers are next written.
        asm volatile("" ::"v"(d.h0), "v"(d.h1), "v"(d.hz), "v"(d.hrs), "v"(d.hbp.x), "v"(d.hbp.y), "v"(d.hbp.z),
                     "v"(d.hbp.w));
        dfs_emit<L, K, S>(a, d, running || fresh, lead);
        if (!__any(d.rs != kEmpty) && wq.exhausted) break;
    }
    wave_add(a.stat_occ, n_occ);
    wave_add(a.stat_bk, n_bk);
    wave_add(a.stat_tbl, n_tb);
    wave_add(a.stat_steal, n_steal);
}

// A batch with fewer read-strands than the launch has lanes is spread over every wave
// that fits (with subtree transfers, S): each wave then starts with fewer read-strands
// than lanes, and its idle lanes share its trees from the first round. Otherwise waves
// take kQueueChunk read-strands at a time.
template <int I, int L, int K, bool S, bool TB = false>
static hipError_t dfs_launch_batched(const fm_index *idx, const fm_tuning &t, const DfsArgs &a0, hipStream_t s)
{
    const int block = (int)t.block;
    const size_t lds = (size_t)(block / L) * a0.fcap * sizeof(Frame);
    int per = max_blocks_per_cu((const void *)dfs_batched<I, L, K, S, TB>, block, lds);
    if (t.waves_per_cu) {
        int want = (int)(t.waves_per_cu * 64 / block);
        if (want >= 1 && want < per) per = want;
    }
    const uint64_t wpb = (uint64_t)block / 64, cap = (uint64_t)idx->cu_count * per, waves = cap * wpb;
    DfsArgs a = a0;
    a.chunk = kQueueChunk;
    uint64_t need;                        // workgroups the batch fills
    if (S && (uint64_t)a.total < waves * kQueueChunk) {
        const uint64_t c = ((uint64_t)a.total + waves - 1) / waves;
        a.chunk = (uint32_t)(c ? c : 1);
        need = (((uint64_t)a.total + a.chunk - 1) / a.chunk + wpb - 1) / wpb;
    } else {
        need = ((uint64_t)a.total * L + block - 1) / block;
    }
    const uint64_t grid = need < cap ? (need ? need : 1) : cap;
    hipLaunchKernelGGL((dfs_batched<I, L, K, S, TB>), dim3((uint32_t)grid), dim3(block), lds, s, a);
    return hipGetLastError();
}

template <int I, int K>
static hipError_t dfs_by_lanes(const fm_index *idx, const fm_tuning &t, const DfsArgs &a, hipStream_t s)
{
    switch (t.lanes) {
    case 1:
        if constexpr (K != kDfsGap) {
            if (a.tdepth)
                return a.tf_count ? dfs_launch_batched<I, 1, K, true, true>(idx, t, a, s)
                                  : dfs_launch_batched<I, 1, K, false, true>(idx, t, a, s);
        }
        return a.tf_count ? dfs_launch_batched<I, 1, K, true>(idx, t, a, s)
                          : dfs_launch_batched<I, 1, K, false>(idx, t, a, s);
    case 2: return dfs_launch_batched<I, 2, K, false>(idx, t, a, s);
    case 4: if constexpr (Geo<I>::USED > 2) return dfs_launch_batched<I, 4, K, false>(idx, t, a, s); break;
    case 8: if constexpr (Geo<I>::USED > 4) return dfs_launch_batched<I, 8, K, false>(idx, t, a, s); break;
    default: break;
    }
    return hipErrorInvalidValue;
}

// ------------------------------------------------------------------ claim order

// The persistent DFS claims read-strands heaviest first (longest processing time first).
// Its node count is largest where the D bound leaves the most room for substitutions:
// the weight is sum_i max(0, z - D(i)), i.e. the sum over c < z of the first position at
// which D exceeds c (the breakpoints of the D walk). A launch in read order ends with the
// last few heavy trees running on a mostly idle chip; heaviest first leaves the light and
// root-pruned read-strands for the end, where they fill lanes as they free up. The order
// only decides which lane searches which read-strand and when: results are unchanged.
// Weights are bucketed into kOrderBins classes (exact below 64, then 16 per octave);
// read-strands of one class are claimed in no particular order. The gapped search keeps
// read order: there the heaviest class (patterns that occur, D zero throughout) holds
// most of the work in trees of 2.5-fold different sizes, which the weight cannot rank.

struct OrderArgs {
    const uint64_t *offs;
    const uint8_t *z;
    const uint4 *bp;
    uint32_t total, nstr, zmax;
    uint32_t chunk;        // read-strands per workgroup of the counting and placing passes
    uint8_t *bin;          // per read-strand: kOrderBins - 1 - its weight class
    uint32_t *hist;        // per workgroup and bin: count, then the bin's first slot
    uint32_t *tot;         // per bin: read-strands in it
    uint4 *rec;            // two uint4 per slot of the claim order (see Dfs::request)
};

static_assert(kOrderBins == 256, "the claim-order passes keep one bin per thread of a 256-thread workgroup");

// Workgroups of the counting and placing passes: one per kOrderChunk read-strands, at
// most kOrderBlocks (one thread of the scan pass per workgroup).
constexpr uint32_t kOrderChunk = 2048;

static uint32_t order_blocks(uint64_t nrs)
{
    const uint64_t b = (nrs + kOrderChunk - 1) / kOrderChunk;
    return (uint32_t)(b < 1 ? 1 : (b < kOrderBlocks ? b : kOrderBlocks));
}

__device__ __forceinline__ uint32_t order_class(uint32_t w)
{
    if (w < 64) return w;
    const uint32_t e = 31u - __clz(w);               // 6 ... 31
    const uint32_t v = 64u + (e - 6u) * 16u + ((w >> (e - 4u)) & 15u);
    return v < kOrderBins - 1 ? v : kOrderBins - 1;
}

// Weight of a read-strand from its D record (first 16 bits: breakpoints found, then
// breakpoint c at bits 16 (c + 1) ..., 0xFFFF when D never exceeds c); zero when the
// search decides the read-strand at once (budget above zmax, read over 65535, root pruned).
__device__ __forceinline__ uint32_t order_weight(const OrderArgs &o, uint64_t b0, uint64_t b1, uint32_t z, uint4 r)
{
    const uint64_t len = b1 - b0;
    const uint32_t nbp = r.x & 0xFFFFu;
    if (z > o.zmax || len > 65535u || nbp > z) return 0u;
    const uint32_t m = (uint32_t)len;
    const uint32_t f[4] = {r.x >> 16, r.y & 0xFFFFu, r.y >> 16, r.z & 0xFFFFu};
    uint32_t w = 0;
    for (uint32_t c = 0; c < 4; ++c)
        if (c < z) w += f[c] < m ? f[c] : m;
    return w;
}

// Inclusive sum over the block's N threads (one value each), in s[N].
template <uint32_t N>
__device__ __forceinline__ uint32_t block_inclusive(uint32_t *s, uint32_t v)
{
    const uint32_t t = threadIdx.x;
    s[t] = v;
    __syncthreads();
    for (uint32_t d = 1; d < N; d <<= 1) {
        const uint32_t u = t >= d ? s[t - d] : 0u;
        __syncthreads();
        s[t] += u;
        __syncthreads();
    }
    return s[t];
}

// Pass 1: each workgroup classifies its chunk and counts the bins.
__global__ void __launch_bounds__(256) order_count(OrderArgs o)
{
    __shared__ uint32_t h[kOrderBins];
    h[threadIdx.x] = 0;
    __syncthreads();
    const uint64_t lo = (uint64_t)blockIdx.x * o.chunk;
    const uint64_t hi = lo + o.chunk < o.total ? lo + o.chunk : o.total;
    for (uint64_t j = lo + threadIdx.x; j < hi; j += 256) {
        const uint32_t rs = (uint32_t)j, rd = o.nstr == 2 ? rs >> 1 : rs;
        const uint32_t w = order_weight(o, o.offs[rd], o.offs[rd + 1], o.z[rd], o.bp[rs]);
        const uint32_t b = kOrderBins - 1 - order_class(w);
        o.bin[rs] = (uint8_t)b;
        atomicAdd(&h[b], 1u);
    }
    __syncthreads();
    o.hist[blockIdx.x * kOrderBins + threadIdx.x] = h[threadIdx.x];
}

// Pass 2, a workgroup per bin and a thread per counting workgroup: each workgroup's first
// slot within the bin, and the bin's total.
__global__ void __launch_bounds__(kOrderBlocks) order_scan(uint32_t *hist, uint32_t *tot, uint32_t nblk)
{
    __shared__ uint32_t s[kOrderBlocks];
    const uint32_t b = blockIdx.x, g = threadIdx.x;
    const uint32_t v = g < nblk ? hist[g * kOrderBins + b] : 0u;
    const uint32_t inc = block_inclusive<kOrderBlocks>(s, v);
    if (g < nblk) hist[g * kOrderBins + b] = inc - v;
    if (g == kOrderBlocks - 1) tot[b] = inc;
}

// Pass 3: each workgroup finds the bins' first slots (bins in order, heaviest first) and
// writes the header records of its chunk into its slots.
__global__ void __launch_bounds__(256) order_place(OrderArgs o)
{
    __shared__ uint32_t s[256];
    __shared__ uint32_t cur[kOrderBins];
    const uint32_t t = o.tot[threadIdx.x];
    const uint32_t first = block_inclusive<kOrderBins>(s, t) - t + o.hist[blockIdx.x * kOrderBins + threadIdx.x];
    cur[threadIdx.x] = first;
    __syncthreads();
    const uint64_t lo = (uint64_t)blockIdx.x * o.chunk;
    const uint64_t hi = lo + o.chunk < o.total ? lo + o.chunk : o.total;
    for (uint64_t j = lo + threadIdx.x; j < hi; j += 256) {
        const uint32_t rs = (uint32_t)j, rd = o.nstr == 2 ? rs >> 1 : rs;
        const uint64_t b0 = o.offs[rd], b1 = o.offs[rd + 1];
        const uint4 r = o.bp[rs];
        const uint32_t slot = atomicAdd(&cur[o.bin[rs]], 1u);
        o.rec[2 * (size_t)slot] = make_uint4(rs, (uint32_t)b0, (uint32_t)(b0 >> 32), (uint32_t)(b1 - b0));
        o.rec[2 * (size_t)slot + 1] = make_uint4(o.z[rd], r.x, r.y, r.z);
    }
}

static hipError_t launch_order(const DfsCall &c, const InexactWs &W, uint32_t nstr, uint32_t total, hipStream_t s)
{
    char *ws = (char *)c.ws;
    OrderArgs o;
    o.offs = c.offs;
    o.z = c.z;
    o.bp = (const uint4 *)(ws + W.bp);
    o.total = total;
    o.nstr = nstr;
    o.zmax = c.zmax;
    const uint32_t nblk = order_blocks(total);
    o.chunk = (uint32_t)(((uint64_t)total + nblk - 1) / nblk);
    o.bin = (uint8_t *)(ws + W.bin);
    o.hist = (uint32_t *)(ws + W.ohist);
    o.tot = o.hist + (size_t)nblk * kOrderBins;
    o.rec = (uint4 *)(ws + W.rec);
    hipLaunchKernelGGL(order_count, dim3(nblk), dim3(256), 0, s, o);
    hipLaunchKernelGGL(order_scan, dim3(kOrderBins), dim3(kOrderBlocks), 0, s, o.hist, o.tot, nblk);
    hipLaunchKernelGGL(order_place, dim3(nblk), dim3(256), 0, s, o);
    return hipGetLastError();
}

// ------------------------------------------------------------------ compaction

// Per read: the worst strand status, the number of hits to list (0 unless FM_OK), and
// the number every read would need (FM_OK and FM_EOVERFLOW reads). Clears the
// overflow cursors.
// Grid-stride over reads; the required total is summed per block and added with one
// atomic per block (one per wave contends on the single counter).
__global__ void __launch_bounds__(256) finalize_reads(uint32_t nreads, uint32_t nstr, const uint32_t *rs_count,
                                                      const uint32_t *rs_status, const uint32_t *rs_nodes,
                                                      const uint32_t *tf_count, const uint32_t *tf_status,
                                                      const uint32_t *tf_nodes, uint32_t budget, uint32_t *rd_status,
                                                      uint32_t *cnt, uint32_t *cursor, unsigned long long *required)
{
    __shared__ uint64_t part[4];
    uint64_t need = 0;
    for (uint32_t r = blockIdx.x * blockDim.x + threadIdx.x; r < nreads; r += gridDim.x * blockDim.x) {
        uint32_t st = 0, c = 0;
        for (uint32_t s = 0; s < nstr; ++s) {
            const uint32_t rs = r * nstr + s;
            uint32_t v = rs_status[rs];
            c += rs_count[rs];
            if (tf_count) {
                // parts taken by other lanes: their hits and statuses, and the node budget,
                // which a tree searched in parts can exceed with no part doing so
                const uint32_t u = tf_status[rs];
                v = u > v ? u : v;
                c += tf_count[rs];
                if ((uint64_t)rs_nodes[rs] + tf_nodes[rs] > budget && v < FM_EBUDGET) v = FM_EBUDGET;
            }
            st = v > st ? v : st;
            cursor[rs] = 0;
        }
        rd_status[r] = st;
        cnt[r] = st == FM_OK ? c : 0u;
        need += (st == FM_OK || st == FM_EOVERFLOW) ? c : 0u;
    }
    for (int d = 32; d >= 1; d >>= 1) need += __shfl_xor(need, d);
    if (__lane_id() == 0) part[threadIdx.x >> 6] = need;
    __syncthreads();
    if (threadIdx.x == 0) {
        const uint64_t t = part[0] + part[1] + part[2] + part[3];
        if (t) atomicAdd(required, (unsigned long long)t);
    }
}

constexpr int kTile = 8;
constexpr int kScanBlock = 256;

__global__ void scan_reduce_u64(const uint32_t *cnt, uint64_t n, uint64_t *part)
{
    __shared__ uint64_t lds[32];
    const uint64_t base = (blockIdx.x * (uint64_t)blockDim.x + threadIdx.x) * kTile;
    uint64_t acc = 0;
    for (int t = 0; t < kTile; ++t)
        if (base + t < n) acc += cnt[base + t];
    uint64_t tot;
    block_scan_u64(acc, lds, &tot);
    if (threadIdx.x == 0) part[blockIdx.x] = tot;
}

__global__ void scan_partials_u64(uint64_t *part, uint64_t np)
{
    __shared__ uint64_t lds[32];
    const uint64_t per = (np + blockDim.x - 1) / blockDim.x;
    const uint64_t b0 = threadIdx.x * per;
    uint64_t acc = 0;
    for (uint64_t i = b0; i < b0 + per && i < np; ++i) acc += part[i];
    uint64_t tot;
    uint64_t off = block_scan_u64(acc, lds, &tot);
    for (uint64_t i = b0; i < b0 + per && i < np; ++i) {
        const uint64_t v = part[i];
        part[i] = off;
        off += v;
    }
}

__global__ void scan_write_u64(const uint32_t *cnt, uint64_t n, const uint64_t *part, uint64_t *out)
{
    __shared__ uint64_t lds[32];
    const uint64_t base = (blockIdx.x * (uint64_t)blockDim.x + threadIdx.x) * kTile;
    uint64_t loc[kTile];
    uint64_t acc = 0;
    for (int t = 0; t < kTile; ++t) {
        loc[t] = acc;
        if (base + t < n) acc += cnt[base + t];
    }
    uint64_t tot;
    const uint64_t off = part[blockIdx.x] + block_scan_u64(acc, lds, &tot);
    for (int t = 0; t < kTile; ++t) {
        const uint64_t j = base + t;
        if (j < n) out[j] = off + loc[t];
        if (j + 1 == n) out[n] = off + loc[t] + cnt[j];
    }
}

// The listed prefix of reads: reads are listed in order while their hits fit in cap.
// cut = the largest offset <= cap; exactly one r in [0, n] satisfies the test.
__global__ void find_cut(const uint64_t *offs, uint64_t n, uint64_t cap, uint64_t *cut)
{
    const uint64_t r = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x;
    if (r > n) return;
    if (offs[r] <= cap && (r == n || offs[r + 1] > cap)) *cut = offs[r];
}

// Final offsets and statuses, and the slot hits of every listed read (strand 0's hits,
// then strand 1's; within a strand the slot hits precede its overflow-pool hits).
__global__ void gather_hits(uint32_t nreads, uint32_t nstr, const uint32_t *rs_count, const uint32_t *tf_count,
                            const uint32_t *rd_status, const uint64_t *offs, const uint64_t *cut, const fm_hit *slots,
                            uint64_t *hit_offs, uint32_t *status, fm_hit *hits)
{
    const uint32_t r = blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= nreads) return;
    const uint64_t c = *cut;
    const uint64_t o0 = offs[r], o1 = offs[r + 1];
    hit_offs[r] = o0 < c ? o0 : c;
    if (r + 1 == nreads) hit_offs[nreads] = o1 < c ? o1 : c;
    uint32_t st = rd_status[r];
    if (st == FM_OK && o1 > c) st = FM_EOVERFLOW;    // beyond hit_cap: not listed
    status[r] = st;
    if (st != FM_OK) return;
    uint64_t dst = o0;
    for (uint32_t s = 0; s < nstr; ++s) {
        const uint32_t rs = r * nstr + s;
        const uint32_t own = rs_count[rs], ns = own < kHitSlots ? own : kHitSlots;
        const uint32_t n = own + (tf_count ? tf_count[rs] : 0u);
        for (uint32_t h = 0; h < ns; ++h) ((uint4 *)hits)[dst + h] = ((const uint4 *)slots)[(size_t)rs * kHitSlots + h];
        dst += n;
    }
}

// Overflow-pool hits of listed reads, after their read-strand's slot hits.
__global__ void scatter_overflow(const fm_hit *opool, const unsigned long long *ocount, uint64_t ocap, uint32_t nstr,
                                 const uint32_t *rs_count, const uint32_t *tf_count, const uint32_t *status,
                                 const uint64_t *hit_offs, uint32_t *cursor, fm_hit *hits)
{
    const uint64_t total = *ocount < ocap ? *ocount : ocap;
    for (uint64_t e = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; e < total; e += (uint64_t)gridDim.x * blockDim.x) {
        const uint4 h = ((const uint4 *)opool)[e];
        const uint32_t r = h.x, s = nstr == 2 ? (h.w & 0xFFu) : 0u;
        if (status[r] != FM_OK) continue;
        // after the strand's slot hits (the first kHitSlots of its owner), and after all
        // hits of strand 0
        const uint32_t own = rs_count[r * nstr + s];
        const uint64_t before = s ? (uint64_t)rs_count[r * nstr] + (tf_count ? tf_count[r * nstr] : 0u) : 0u;
        const uint64_t start = hit_offs[r] + before + (own < kHitSlots ? own : kHitSlots);
        ((uint4 *)hits)[start + atomicAdd(&cursor[r * nstr + s], 1u)] = h;
    }
}

// Hits of one read sorted by (strand, k): in substitution mode every (strand, k) is
// distinct, so the order is unique whatever order the hits were found in.
// Order of a read's hits: strand, then k, then l, then the number of differences.
__device__ __forceinline__ bool hit_before(const uint4 &u, const uint4 &v)
{
    if ((u.w & 0xFFu) != (v.w & 0xFFu)) return (u.w & 0xFFu) < (v.w & 0xFFu);
    if (u.y != v.y) return u.y < v.y;
    if (u.z != v.z) return u.z < v.z;
    return ((u.w >> 8) & 0xFFu) < ((v.w >> 8) & 0xFFu);
}

__global__ void sort_read_hits(uint64_t nreads, const uint64_t *hit_offs, fm_hit *hits)
{
    const uint64_t r = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x;
    if (r >= nreads) return;
    const uint64_t b = hit_offs[r], e = hit_offs[r + 1];
    uint4 *h = (uint4 *)hits;
    for (uint64_t x = b + 1; x < e; ++x) {
        const uint4 v = h[x];
        uint64_t y = x;
        while (y > b) {
            const uint4 u = h[y - 1];
            if (!hit_before(v, u)) break;
            h[y] = u;
            --y;
        }
        h[y] = v;
    }
}

// Gapped search: one hit per (strand, k, l), the one with the fewest differences (the
// first of its run in the sorted order), moved to the front of the read's hits; cnt[r]
// gets how many remain.
__global__ void dedupe_read_hits(uint64_t nreads, const uint64_t *hit_offs, fm_hit *hits, uint32_t *cnt)
{
    const uint64_t r = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x;
    if (r >= nreads) return;
    const uint64_t b = hit_offs[r], e = hit_offs[r + 1];
    uint4 *h = (uint4 *)hits;
    uint64_t u = 0;
    for (uint64_t x = b; x < e; ++x) {
        const uint4 v = h[x];
        if (u > 0) {
            const uint4 p = h[b + u - 1];
            if ((p.w & 0xFFu) == (v.w & 0xFFu) && p.y == v.y && p.z == v.z) continue;
        }
        h[b + u++] = v;
    }
    cnt[r] = (uint32_t)u;
}

// Moves each read's remaining hits to their new offsets in tmp.
__global__ void move_read_hits(uint64_t nreads, const uint64_t *hit_offs, const uint64_t *new_offs, const fm_hit *hits,
                               fm_hit *tmp)
{
    const uint64_t r = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x;
    if (r >= nreads) return;
    const uint64_t b = hit_offs[r], d = new_offs[r], u = new_offs[r + 1] - new_offs[r];
    for (uint64_t x = 0; x < u; ++x) ((uint4 *)tmp)[d + x] = ((const uint4 *)hits)[b + x];
}

// The new offsets, and the hits back from tmp.
__global__ void place_read_hits(uint64_t nreads, const uint64_t *new_offs, const fm_hit *tmp, uint64_t *hit_offs,
                                fm_hit *hits)
{
    const uint64_t total = new_offs[nreads];
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    for (uint64_t j = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; j <= nreads; j += stride)
        hit_offs[j] = new_offs[j];
    for (uint64_t j = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; j < total; j += stride)
        ((uint4 *)hits)[j] = ((const uint4 *)tmp)[j];
}

InexactWs inexact_ws_layout(uint64_t nreads, uint32_t nstr, uint32_t zmax, uint64_t hit_cap)
{
    (void)zmax;
    auto al = [](size_t x) { return (x + 255) & ~(size_t)255; };
    InexactWs w;
    size_t off = kWsHeader;
    const uint64_t nrs = nreads * nstr;
    w.bp = off;        off = al(off + nrs * 16);
    w.rs_count = off;  off = al(off + nrs * 4);
    w.rs_status = off; off = al(off + nrs * 4);
    w.rs_nodes = off;  off = al(off + nrs * 4);
    w.tf_count = off;  off = al(off + nrs * 4);
    w.tf_status = off; off = al(off + nrs * 4);
    w.tf_nodes = off;  off = al(off + nrs * 4);
    w.cursor = off;    off = al(off + nrs * 4);
    w.rd_status = off; off = al(off + nreads * 4);
    w.cnt = off;       off = al(off + nreads * 4);
    w.offs = off;      off = al(off + (nreads + 1) * 8);
    const uint64_t nblk = (nreads + kScanBlock * kTile - 1) / (kScanBlock * kTile);
    w.part = off;      off = al(off + (nblk + 1) * 8);
    w.slots = off;     off = al(off + nrs * kHitSlots * 16);
    w.opool = off;     off = al(off + hit_cap * 16);
    w.bin = off;       off = al(off + nrs);
    w.ohist = off;     off = al(off + ((size_t)order_blocks(nrs) + 1) * kOrderBins * 4);
    w.rec = off;       off = al(off + nrs * 32);
    w.total = off;
    return w;
}

template <int K, bool TB>
static hipError_t dfs_plain_launch(const fm_tuning &t, const DfsArgs &a, hipStream_t s)
{
    const uint32_t grid = (a.total + 255) / 256;
    const size_t lds = (size_t)256 * a.fcap * sizeof(Frame);
    switch (t.occ_interval) {
    case 64: hipLaunchKernelGGL((dfs_plain<64, K, TB>), dim3(grid), dim3(256), lds, s, a); break;
    case 96: hipLaunchKernelGGL((dfs_plain<96, K, TB>), dim3(grid), dim3(256), lds, s, a); break;
    case 128: hipLaunchKernelGGL((dfs_plain<128, K, TB>), dim3(grid), dim3(256), lds, s, a); break;
    case 192: hipLaunchKernelGGL((dfs_plain<192, K, TB>), dim3(grid), dim3(256), lds, s, a); break;
    case 224: hipLaunchKernelGGL((dfs_plain<224, K, TB>), dim3(grid), dim3(256), lds, s, a); break;
    case 256: hipLaunchKernelGGL((dfs_plain<256, K, TB>), dim3(grid), dim3(256), lds, s, a); break;
    case 448: hipLaunchKernelGGL((dfs_plain<448, K, TB>), dim3(grid), dim3(256), lds, s, a); break;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

template <int K>
static hipError_t dfs_batched_launch(const fm_index *idx, const fm_tuning &t, const DfsArgs &a, hipStream_t s)
{
    switch (t.occ_interval) {
    case 64: return dfs_by_lanes<64, K>(idx, t, a, s);
    case 96: return dfs_by_lanes<96, K>(idx, t, a, s);
    case 128: return dfs_by_lanes<128, K>(idx, t, a, s);
    case 192: return dfs_by_lanes<192, K>(idx, t, a, s);
    case 224: return dfs_by_lanes<224, K>(idx, t, a, s);
    case 256: return dfs_by_lanes<256, K>(idx, t, a, s);
    case 448: return dfs_by_lanes<448, K>(idx, t, a, s);
    default: return hipErrorInvalidValue;
    }
}

hipError_t launch_inexact(const fm_index *idx, const fm_tuning &t, const fm_tuning &tw, bool plain, const DfsCall &c,
                          hipStream_t s, const PhaseEvents *pe)
{
    const PhaseEvents none;
    if (!pe) pe = &none;
    // exact intervals from the DFS: batched kernels only, and strands the DFS searches
    if (c.ex_out && (plain || (c.ex_flags & ~c.flags & FM_BOTH))) return hipErrorInvalidValue;
    char *ws = (char *)c.ws;
    const uint32_t nstr = strand_count(c.flags);
    const InexactWs W = inexact_ws_layout(c.nreads, nstr, c.zmax, c.hit_cap);
    hipError_t e = launch_fill(ws, 0, kWsHeader / 4, s);
    if (e != hipSuccess) return e;
    if (c.nreads == 0) return launch_fill(c.hit_offs, 0, 2, s);
    const bool use_d = (c.flags & FM_DARRAY) != 0;
    pe->mark(1, s);
    if (use_d) {
        WalkCall wc{c.codes, c.offs, c.z, c.nreads, c.flags, c.zmax, ws + W.bp, ws};
        e = launch_walk(idx, tw, WALK_DBP, plain, wc, s);
        if (e != hipSuccess) return e;
    }
    DfsArgs a;
    a.lay = dev_layout(idx, t.occ_interval, false);
    a.codes = c.codes;
    a.offs = c.offs;
    a.z = c.z;
    a.bp = use_d ? (const uint4 *)(ws + W.bp) : nullptr;
    a.rec = nullptr;
    a.nstr = nstr;
    a.strand0 = (c.flags & FM_FWD) ? 0u : 1u;
    a.total = (uint32_t)(c.nreads * nstr);
    a.zmax = c.zmax;
    a.fcap = c.zmax + 1;
    a.chunk = kQueueChunk;
    a.budget = t.node_budget ? t.node_budget : 0xFFFFFFFFu;
    a.slots = (fm_hit *)(ws + W.slots);
    a.opool = (fm_hit *)(ws + W.opool);
    a.ocap = c.hit_cap;
    a.ocount = (unsigned long long *)(ws + kWsPool);
    a.rs_count = (uint32_t *)(ws + W.rs_count);
    a.rs_status = (uint32_t *)(ws + W.rs_status);
    a.rs_nodes = (uint32_t *)(ws + W.rs_nodes);
    a.tf_count = a.tf_status = a.tf_nodes = nullptr;
    a.queue = (uint32_t *)(ws + kWsQueue2);
    a.stat_occ = (c.flags & FM_STATS) ? (unsigned long long *)(ws + kWsStatOcc) : nullptr;
    a.stat_bk = (c.flags & FM_STATS) ? (unsigned long long *)(ws + kWsStatBuckets) : nullptr;
    a.stat_steal = (c.flags & FM_STATS) ? (unsigned long long *)(ws + kWsStatSteal) : nullptr;
    a.stat_tbl = (c.flags & FM_STATS) ? (unsigned long long *)(ws + kWsStatTable) : nullptr;
    // the prefix table serves substitution nodes (the gapped search consumes pattern and
    // string at different rates, so a node's depth is not m - 1 - i there)
    a.tab = (const uint4 *)idx->ptab;
    a.tdepth = (c.flags & FM_GAPS) || !idx->ptab ? 0u : (t.table_depth < idx->table_levels ? t.table_depth
                                                                                            : idx->table_levels);
    const bool ex = c.ex_out != nullptr;
    a.ex_out = (uint2 *)c.ex_out;
    a.ex_nstr = strand_count(c.ex_flags);
    a.ex_strands = c.ex_flags & FM_BOTH;
    const bool gap = (c.flags & FM_GAPS) != 0;
    if (use_d && !plain && t.order && !gap) {
        // claim order for the persistent DFS, from the D records just written
        e = launch_order(c, W, nstr, a.total, s);
        if (e != hipSuccess) return e;
        a.rec = (const uint4 *)(ws + W.rec);
    }
    // Lanes of the batched DFS take subtrees from one another at the end of the launch,
    // with room for the frame a node leaves there when it walks its match child first. At
    // z = 1 only in batches with fewer read-strands than an 8-wave-per-CU launch has lanes:
    // in larger ones the trees are small next to the launch, and stolen hits, which go
    // through the overflow pool, cost more than the shorter tail gains.
    const bool small_batch = (uint64_t)a.total < (uint64_t)idx->cu_count * 8 * 64;
    if (!plain && t.lanes == 1 && (c.zmax >= 2 || (c.zmax == 1 && small_batch))) {
        a.fcap = c.zmax + 2;
        a.tf_count = (uint32_t *)(ws + W.tf_count);
        a.tf_status = (uint32_t *)(ws + W.tf_status);
        a.tf_nodes = (uint32_t *)(ws + W.tf_nodes);
        e = launch_fill(a.tf_count, 0, (W.tf_nodes + (size_t)a.total * 4 - W.tf_count) / 4, s);
        if (e != hipSuccess) return e;
    }
    pe->mark(2, s);
    if (plain)
        e = gap ? dfs_plain_launch<kDfsGap, false>(t, a, s)
                : (a.tdepth ? dfs_plain_launch<kDfsSub, true>(t, a, s) : dfs_plain_launch<kDfsSub, false>(t, a, s));
    else if (gap)
        e = dfs_batched_launch<kDfsGap>(idx, t, a, s);
    else
        e = ex ? dfs_batched_launch<kDfsSubExact>(idx, t, a, s) : dfs_batched_launch<kDfsSub>(idx, t, a, s);
    if (e != hipSuccess) return e;
    if (ex) {
        WalkArgs w;
        w.lay = a.lay;
        w.codes = c.codes;
        w.offs = c.offs;
        w.z = nullptr;
        w.nstr = a.ex_nstr;
        w.strand0 = (c.ex_flags & FM_FWD) ? 0u : 1u;
        w.total = (uint32_t)(c.nreads * w.nstr);
        w.zmax = 0;
        w.out = c.ex_out;
        w.dstride = 0;
        w.queue = nullptr;
        w.full_rank = 0;
        w.stat_steps = nullptr;
        w.stat_bk = nullptr;
        const uint32_t blocks = (a.total + 255) / 256, cap = (uint32_t)idx->cu_count * 4;
        const dim3 grid(blocks < cap ? blocks : cap);
        switch (t.occ_interval) {
        case 64: hipLaunchKernelGGL(exact_rest<64>, grid, dim3(256), 0, s, w, a.rs_status, a.total, a.nstr, a.strand0); break;
        case 96: hipLaunchKernelGGL(exact_rest<96>, grid, dim3(256), 0, s, w, a.rs_status, a.total, a.nstr, a.strand0); break;
        case 128: hipLaunchKernelGGL(exact_rest<128>, grid, dim3(256), 0, s, w, a.rs_status, a.total, a.nstr, a.strand0); break;
        case 192: hipLaunchKernelGGL(exact_rest<192>, grid, dim3(256), 0, s, w, a.rs_status, a.total, a.nstr, a.strand0); break;
        case 224: hipLaunchKernelGGL(exact_rest<224>, grid, dim3(256), 0, s, w, a.rs_status, a.total, a.nstr, a.strand0); break;
        case 256: hipLaunchKernelGGL(exact_rest<256>, grid, dim3(256), 0, s, w, a.rs_status, a.total, a.nstr, a.strand0); break;
        case 448: hipLaunchKernelGGL(exact_rest<448>, grid, dim3(256), 0, s, w, a.rs_status, a.total, a.nstr, a.strand0); break;
        default: return hipErrorInvalidValue;
        }
        e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    pe->mark(3, s);
    // compaction
    uint32_t *cnt = (uint32_t *)(ws + W.cnt), *cursor = (uint32_t *)(ws + W.cursor);
    uint32_t *rd_status = (uint32_t *)(ws + W.rd_status);
    uint64_t *offs_tmp = (uint64_t *)(ws + W.offs);
    uint64_t *cut = (uint64_t *)(ws + kWsCut);
    const uint32_t nr = (uint32_t)c.nreads;
    uint32_t fgrid = (nr + 255) / 256;
    if (fgrid > (uint32_t)idx->cu_count * 4) fgrid = (uint32_t)idx->cu_count * 4;
    hipLaunchKernelGGL(finalize_reads, dim3(fgrid ? fgrid : 1), dim3(256), 0, s, nr, nstr, a.rs_count, a.rs_status,
                       a.rs_nodes, a.tf_count, a.tf_status, a.tf_nodes, a.budget, rd_status, cnt, cursor,
                       (unsigned long long *)(ws + kWsRequired));
    const uint64_t nblk = (c.nreads + kScanBlock * kTile - 1) / (kScanBlock * kTile);
    uint64_t *part = (uint64_t *)(ws + W.part);
    hipLaunchKernelGGL(scan_reduce_u64, dim3((uint32_t)nblk), dim3(kScanBlock), 0, s, cnt, c.nreads, part);
    hipLaunchKernelGGL(scan_partials_u64, dim3(1), dim3(1024), 0, s, part, nblk);
    hipLaunchKernelGGL(scan_write_u64, dim3((uint32_t)nblk), dim3(kScanBlock), 0, s, cnt, c.nreads, part, offs_tmp);
    hipLaunchKernelGGL(find_cut, dim3((nr + 1 + 255) / 256), dim3(256), 0, s, offs_tmp, c.nreads, c.hit_cap, cut);
    hipLaunchKernelGGL(gather_hits, dim3((nr + 255) / 256), dim3(256), 0, s, nr, nstr, a.rs_count, a.tf_count, rd_status,
                       offs_tmp, cut, a.slots, c.hit_offs, c.status, c.hits);
    uint64_t sgrid = (c.hit_cap + 255) / 256;
    if (sgrid > (uint64_t)idx->cu_count * 4) sgrid = (uint64_t)idx->cu_count * 4;
    if (sgrid == 0) sgrid = 1;
    hipLaunchKernelGGL(scatter_overflow, dim3((uint32_t)sgrid), dim3(256), 0, s, a.opool, a.ocount, a.ocap, nstr,
                       a.rs_count, a.tf_count, c.status, c.hit_offs, cursor, c.hits);
    hipLaunchKernelGGL(sort_read_hits, dim3((nr + 255) / 256), dim3(256), 0, s, c.nreads, c.hit_offs, c.hits);
    if (gap) {
        // one hit per interval: dedupe in place, then re-pack through the (spent) overflow pool
        hipLaunchKernelGGL(dedupe_read_hits, dim3((nr + 255) / 256), dim3(256), 0, s, c.nreads, c.hit_offs, c.hits, cnt);
        hipLaunchKernelGGL(scan_reduce_u64, dim3((uint32_t)nblk), dim3(kScanBlock), 0, s, cnt, c.nreads, part);
        hipLaunchKernelGGL(scan_partials_u64, dim3(1), dim3(1024), 0, s, part, nblk);
        hipLaunchKernelGGL(scan_write_u64, dim3((uint32_t)nblk), dim3(kScanBlock), 0, s, cnt, c.nreads, part, offs_tmp);
        hipLaunchKernelGGL(move_read_hits, dim3((nr + 255) / 256), dim3(256), 0, s, c.nreads, c.hit_offs, offs_tmp,
                           c.hits, a.opool);
        hipLaunchKernelGGL(place_read_hits, dim3((uint32_t)sgrid), dim3(256), 0, s, c.nreads, offs_tmp, a.opool,
                           c.hit_offs, c.hits);
    }
    pe->mark(4, s);
    return hipGetLastError();
}

// ------------------------------------------------------------------ locate (Eq. 4-5)

struct LocateArgs {
    DevLayout lay;               // forward index
    const uint32_t *kl;          // interval j: k = kl[j * stride], l = kl[j * stride + 1]
    uint64_t niv;
    uint32_t stride;
    const uint64_t *offs;        // niv + 1: exclusive prefix sums of the interval sizes
    const uint32_t *samples;     // SA at every kSaSample-th row
    uint32_t *pos;
    uint64_t cap;                // rows located: the first min(cap, offs[niv])
    uint32_t *queue;
    unsigned long long *stat_steps;
};

// Sizes of the intervals: l - k + 1 for k <= l <= n, else 0 (misses such as (1, 0), and
// rows past the index, which are never located).
__global__ void __launch_bounds__(256) interval_sizes(const uint32_t *kl, uint64_t niv, uint32_t stride, uint32_t n,
                                                      uint32_t *cnt)
{
    for (uint64_t j = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; j < niv; j += (uint64_t)gridDim.x * blockDim.x) {
        const uint32_t k = kl[j * stride], l = kl[j * stride + 1];
        cnt[j] = (k <= l && l <= n) ? l - k + 1 : 0u;
    }
}

// The interval holding item r of the concatenated rows: the last j with offs[j] <= r.
// A lane's items only increase (work is claimed in increasing chunks), so the search
// gallops forward from the lane's previous interval.
__device__ __forceinline__ uint64_t locate_interval(const LocateArgs &a, uint64_t r, uint64_t from)
{
    uint64_t lo = from, step = 1, hi = from + 1;
    while (hi < a.niv && a.offs[hi] <= r) {
        lo = hi;
        step *= 2;
        hi = lo + step;
    }
    if (hi > a.niv) hi = a.niv;
    while (hi - lo > 1) {
        const uint64_t mid = (lo + hi) / 2;
        if (a.offs[mid] <= r) lo = mid;
        else hi = mid;
    }
    return lo;
}

// Eq. 4-5: from row k, apply Psi^-1(i) = C[BWT[i]] + Occ(BWT[i], i) until the row is a
// multiple of kSaSample (its SA value is stored) or is the '$' row (SA = 0); SA[k] is
// that value plus the number of steps. One bucket fetch per step gives both BWT[i] and
// Occ(BWT[i], i); only the stepped symbol's occurrences are counted. Each lane keeps P
// rows in flight (independent chains, each step waiting only for its own bucket), so a
// lane has P bucket loads outstanding per round. Persistent, with the work queue and
// round order of walk_batched.
template <int I, int P>
__global__ void __launch_bounds__(256) locate_batched(LocateArgs a)
{
    const uint64_t all = a.offs[a.niv];
    const uint32_t total = (uint32_t)(all < a.cap ? all : a.cap);
    uint32_t item[P], row[P], steps[P], sv[P];
    bool fin[P];
#pragma unroll
    for (int p = 0; p < P; ++p) {
        item[p] = kEmpty;
        row[p] = steps[p] = sv[p] = 0;
        fin[p] = false;
    }
    uint64_t jprev = 0, nsteps = 0;
    WaveQueue wq;
    wq.start(kQueueChunk, total, false);
    for (;;) {
        // 1. the bucket of every running row
        bool act[P];
        Bucket<I, 1> bk[P];
        uint4 sbc[P];
#pragma unroll
        for (int p = 0; p < P; ++p) {
            act[p] = item[p] != kEmpty && !fin[p];
            const uint32_t j = (act[p] ? row[p] : 0u) / I;
            fetch<I, 1>(a.lay, j, 0, bk[p]);
            sbc[p] = make_uint4(0, 0, 0, 0);
            if constexpr (Geo<I>::COMPACT) sbc[p] = a.lay.sb[j / Geo<I>::SB];
        }
        // 2. positions of the rows that finished last round (their sample loads are in)
#pragma unroll
        for (int p = 0; p < P; ++p) {
            if (fin[p]) {
                a.pos[item[p]] = sv[p] + steps[p];
                item[p] = kEmpty;
                fin[p] = false;
            }
        }
        // 3. idle slots take an item (items a lane takes only increase, across slots too)
        bool fresh[P];
#pragma unroll
        for (int p = 0; p < P; ++p) {
            fresh[p] = false;
            if (refill_now<1>(item[p] == kEmpty)) {
                const uint32_t it = wave_take<1>(wq, item[p] == kEmpty, a.queue, total);
                if (it != kEmpty) {
                    item[p] = it;
                    fresh[p] = true;
                }
            }
        }
        bool any = false;
#pragma unroll
        for (int p = 0; p < P; ++p) any |= item[p] != kEmpty;
        const bool quit = !__any(any);
        // 4. one step of the running rows; new rows begin
#pragma unroll
        for (int p = 0; p < P; ++p) {
            if (fresh[p]) {
                jprev = locate_interval(a, item[p], jprev);
                row[p] = a.kl[jprev * a.stride] + (uint32_t)(item[p] - a.offs[jprev]);
                steps[p] = 0;
            } else if (act[p]) {
                const uint32_t r = row[p] % I;
                const uint32_t c = symbol_at<I>(bk[p], r);
                // '$' is stored as A: rows past it hold one A too many (row is never the '$' row here)
                const uint32_t occ = part1<I>(bk[p], r, c, sbc[p]) - ((c == 0 && row[p] > a.lay.dollar) ? 1u : 0u);
                row[p] = c_of(a.lay, c) + occ;
                steps[p] += 1;
                nsteps += 1;
            }
            if (fresh[p] || act[p]) {
                fin[p] = row[p] % kSaSample == 0 || row[p] == a.lay.dollar;
                if (fin[p]) sv[p] = row[p] == a.lay.dollar ? 0u : a.samples[row[p] / kSaSample];
            }
        }
#pragma unroll
        for (int p = 0; p < P; ++p) {
#pragma unroll
            for (int t = 0; t < Bucket<I, 1>::NPL; ++t)
                asm volatile("" ::"v"(bk[p].v[t].x), "v"(bk[p].v[t].y), "v"(bk[p].v[t].z), "v"(bk[p].v[t].w));
            asm volatile("" ::"v"(sbc[p].x), "v"(sbc[p].y), "v"(sbc[p].z), "v"(sbc[p].w));
        }
        if (quit) break;
    }
    wave_add(a.stat_steps, nsteps);
}

template <int I, int P>
static hipError_t locate_launch(const fm_index *idx, const fm_tuning &t, const LocateArgs &a, hipStream_t s)
{
    const int block = 256;
    int per = max_blocks_per_cu((const void *)locate_batched<I, P>, block, 0);
    if (t.waves_per_cu) {
        const int want = (int)(t.waves_per_cu * 64 / block);
        if (want >= 1 && want < per) per = want;
    }
    uint64_t grid = (uint64_t)idx->cu_count * per;
    const uint64_t need = (a.cap + (uint64_t)block * P - 1) / ((uint64_t)block * P);
    if (need < grid) grid = need;
    if (grid == 0) grid = 1;
    hipLaunchKernelGGL((locate_batched<I, P>), dim3((uint32_t)grid), dim3(block), 0, s, a);
    return hipGetLastError();
}

template <int I>
static hipError_t locate_by_depth(const fm_index *idx, const fm_tuning &t, const LocateArgs &a, hipStream_t s)
{
    switch (t.depth) {
    case 1: return locate_launch<I, 1>(idx, t, a, s);
    case 2: return locate_launch<I, 2>(idx, t, a, s);
    case 4: return locate_launch<I, 4>(idx, t, a, s);
    default: return hipErrorInvalidValue;
    }
}

size_t locate_ws_bytes(uint64_t niv)
{
    const uint64_t nblk = (niv + kScanBlock * kTile - 1) / (kScanBlock * kTile);
    return kWsHeader + ((niv * 4 + 255) & ~(uint64_t)255) + nblk * 8 + 256;
}

hipError_t launch_locate(const fm_index *idx, const fm_tuning &t, const uint32_t *kl, uint64_t niv, uint32_t stride,
                         uint64_t *offs, uint32_t *pos, uint64_t cap, void *ws, bool stats, hipStream_t s)
{
    char *w = (char *)ws;
    hipError_t e = launch_fill(w, 0, kWsHeader / 4, s);
    if (e != hipSuccess) return e;
    uint32_t *cnt = (uint32_t *)(w + kWsHeader);
    uint64_t *part = (uint64_t *)(w + kWsHeader + ((niv * 4 + 255) & ~(uint64_t)255));
    const uint64_t nblk = (niv + kScanBlock * kTile - 1) / (kScanBlock * kTile);
    if (niv == 0) return launch_fill(offs, 0, 2, s);
    uint64_t g = (niv + 255) / 256;
    if (g > (uint64_t)idx->cu_count * 8) g = (uint64_t)idx->cu_count * 8;
    hipLaunchKernelGGL(interval_sizes, dim3((uint32_t)g), dim3(256), 0, s, kl, niv, stride, (uint32_t)idx->n, cnt);
    hipLaunchKernelGGL(scan_reduce_u64, dim3((uint32_t)nblk), dim3(kScanBlock), 0, s, cnt, niv, part);
    hipLaunchKernelGGL(scan_partials_u64, dim3(1), dim3(1024), 0, s, part, nblk);
    hipLaunchKernelGGL(scan_write_u64, dim3((uint32_t)nblk), dim3(kScanBlock), 0, s, cnt, niv, part, offs);
    e = hipGetLastError();
    if (e != hipSuccess || cap == 0) return e;
    LocateArgs a;
    a.lay = dev_layout(idx, t.occ_interval, false);
    a.kl = kl;
    a.niv = niv;
    a.stride = stride;
    a.offs = offs;
    a.samples = idx->sa_samples;
    a.pos = pos;
    a.cap = cap;
    a.queue = (uint32_t *)(w + kWsQueue);
    a.stat_steps = stats ? (unsigned long long *)(w + kWsStatWalk) : nullptr;
    switch (t.occ_interval) {
    case 64: return locate_by_depth<64>(idx, t, a, s);
    case 96: return locate_by_depth<96>(idx, t, a, s);
    case 128: return locate_by_depth<128>(idx, t, a, s);
    case 192: return locate_by_depth<192>(idx, t, a, s);
    case 224: return locate_by_depth<224>(idx, t, a, s);
    case 256: return locate_by_depth<256>(idx, t, a, s);
    case 448: return locate_by_depth<448>(idx, t, a, s);
    default: return hipErrorInvalidValue;
    }
}

}  // namespace fm
