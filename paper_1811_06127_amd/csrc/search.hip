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

struct WaveQueue {
    uint32_t qb, qe;
    bool exhausted;
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
            uint32_t base = 0;
            if (lane == 0) base = atomicAdd(queue, kQueueChunk);
            base = __shfl(base, 0);
            if (base >= total) {
                wq.exhausted = true;
                break;
            }
            wq.qb = base;
            wq.qe = base + kQueueChunk < total ? base + kQueueChunk : total;
        }
        const uint32_t avail = wq.qe - wq.qb;
        const uint32_t r = rank_below(mask, lead);
        const bool mine = need && ((mask >> lead) & 1ull) && r < avail;
        if (mine) got = wq.qb + r;
        const uint32_t cnt = (uint32_t)__popcll(mask);
        wq.qb += cnt < avail ? cnt : avail;
        need = need && !mine;
        mask = __ballot(need && (lane & (L - 1)) == 0);
    }
    return got;
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
    unsigned long long *stat_steps;
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
    uint32_t bp01, bp23;   // DBP: breakpoints 0..3 (16 bits each)
    uint32_t bp4;

    __device__ void finish(const WalkArgs &a, bool lead_lane)
    {
        if (lead_lane) {
            if (MODE == WALK_EXACT) {
                ((uint2 *)a.out)[rs] = (k <= l) ? make_uint2(k, l) : make_uint2(1u, 0u);
            } else if (MODE == WALK_DBP) {
                ((uint4 *)a.out)[rs] = make_uint4(cnt | (bp01 << 16), (bp01 >> 16) | (bp23 << 16), (bp23 >> 16) | (bp4 << 16), 0u);
            }
        }
        rs = kEmpty;
    }

    __device__ void init(const WalkArgs &a, uint32_t item, bool lead_lane)
    {
        rs = item;
        const uint32_t read = a.nstr == 2 ? item >> 1 : item;
        const uint32_t strand = a.nstr == 2 ? (item & 1u) : a.strand0;
        const uint64_t b0 = a.offs[read];
        const uint32_t m = (uint32_t)(a.offs[read + 1] - b0);
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
        bp01 = bp23 = bp4 = 0;
        if (MODE == WALK_DBP) zr = a.z[read] < a.zmax ? a.z[read] : a.zmax;
        if (MODE == WALK_DFULL) outp = (a.nstr == 2 ? strand : 0u) * a.dstride + b0;
        if (m == 0) finish(a, lead_lane);
    }

    // One step with pattern symbol c; ok/ol are Occ(b, k-1), Occ(b, l) (unused when k == 0).
    __device__ void step(const WalkArgs &a, uint32_t c, uint32_t ok, uint32_t ol, bool lead_lane)
    {
        const uint32_t b = (comp && c < 4) ? 3u - c : c;
        uint32_t nk = 1, nl = 0;
        if (b < 4) {
            if (k == 0) {                 // from the empty-pattern interval (0, n)
                nk = a.lay.C[b] + 1;
                nl = a.lay.C[b + 1];
            } else {
                nk = a.lay.C[b] + ok + 1;
                nl = a.lay.C[b] + ol;
            }
        }
        addr += dir;
        rem -= 1;
        if (MODE == WALK_EXACT) {
            k = nk;
            l = nl;
            if (nk > nl || rem == 0) finish(a, lead_lane);
            return;
        }
        if (nk > nl) {                    // a difference is certain in this segment
            cnt += 1;
            const uint32_t pos = i & 0xFFFFu;
            if (cnt == 1) bp01 |= pos;
            else if (cnt == 2) bp01 |= pos << 16;
            else if (cnt == 3) bp23 |= pos;
            else if (cnt == 4) bp23 |= pos << 16;
            else if (cnt == 5) bp4 |= pos;
            k = 0;
            l = a.lay.n;
        } else {
            k = nk;
            l = nl;
        }
        if (MODE == WALK_DFULL && lead_lane) ((uint8_t *)a.out)[outp + i] = (uint8_t)(cnt < 255 ? cnt : 255);
        i += 1;
        if (rem == 0 || (MODE == WALK_DBP && cnt > zr)) finish(a, lead_lane);
    }
};

template <int I, int MODE>
__global__ void __launch_bounds__(256) walk_plain(WalkArgs a)
{
    const uint32_t item = blockIdx.x * blockDim.x + threadIdx.x;
    if (item >= a.total) return;
    Walker<MODE> w;
    w.init(a, item, true);
    uint64_t steps = 0;
    while (w.rs != kEmpty) {
        const uint32_t c = a.codes[w.addr];
        const uint32_t b = (w.comp && c < 4) ? 3u - c : c;
        uint32_t ok = 0, ol = 0;
        if (b < 4 && w.k != 0) {
            occ2<I, 1>(a.lay, 0, b, w.k, w.l, ok, ol);
            ++steps;
        }
        w.step(a, c, ok, ol, true);
    }
    if (a.stat_steps && steps) atomicAdd(a.stat_steps, (unsigned long long)steps);
}

template <int I, int L, int P, int MODE>
__global__ void __launch_bounds__(256) walk_batched(WalkArgs a)
{
    constexpr int LOG = Geo<I>::LOG;
    const uint32_t q = L == 1 ? 0u : (__lane_id() & (L - 1));
    const bool lead = q == 0;
    Walker<MODE> w[P];
#pragma unroll
    for (int p = 0; p < P; ++p) w[p].rs = kEmpty;
    WaveQueue wq = {0, 0, false};
    uint64_t steps = 0;
    for (;;) {
#pragma unroll
        for (int p = 0; p < P; ++p) {
            const uint32_t it = wave_take<L>(wq, w[p].rs == kEmpty, a.queue, a.total);
            if (it != kEmpty) w[p].init(a, it, lead);
        }
        bool any = false;
#pragma unroll
        for (int p = 0; p < P; ++p) any |= w[p].rs != kEmpty;
        if (!__any(any)) break;

        // issue every load of every slot before using any of them
        uint32_t c[P], j1[P], j2[P];
        Bucket<I, L> b1[P], b2[P];
#pragma unroll
        for (int p = 0; p < P; ++p) {
            if (w[p].rs != kEmpty) {
                c[p] = a.codes[w[p].addr];
                if (w[p].k != 0) {
                    j2[p] = w[p].l >> LOG;
                    j1[p] = (w[p].k - 1) >> LOG;
                    fetch<I, L>(a.lay, j1[p], q, b1[p]);
                    if (j1[p] != j2[p]) fetch<I, L>(a.lay, j2[p], q, b2[p]);
                }
            }
        }
#pragma unroll
        for (int p = 0; p < P; ++p) {
            if (w[p].rs != kEmpty) {
                const uint32_t cc = c[p];
                const uint32_t b = (w[p].comp && cc < 4) ? 3u - cc : cc;
                uint32_t ok = 0, ol = 0;
                if (b < 4 && w[p].k != 0) {
                    const bool same = j1[p] == j2[p];
                    uint32_t c1 = part1<I, L>(b1[p], q, (w[p].k - 1) & (I - 1), b);
                    uint32_t c2 = same ? part1<I, L>(b1[p], q, w[p].l & (I - 1), b)
                                       : part1<I, L>(b2[p], q, w[p].l & (I - 1), b);
                    c1 = group_sum<L>(c1);
                    c2 = group_sum<L>(c2);
                    if (b == 0) {
                        c1 -= (w[p].k - 1 >= a.lay.dollar) ? 1u : 0u;
                        c2 -= (w[p].l >= a.lay.dollar) ? 1u : 0u;
                    }
                    ok = c1;
                    ol = c2;
                    steps += lead ? 1 : 0;
                }
                w[p].step(a, cc, ok, ol, lead);
            }
        }
    }
    wave_add(a.stat_steps, steps);
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
    case 4: return walk_by_depth<I, 4, MODE>(idx, t, a, s);
    case 8: return walk_by_depth<I, 8, MODE>(idx, t, a, s);
    default: return hipErrorInvalidValue;
    }
}

template <int MODE>
static hipError_t walk_dispatch(const fm_index *idx, const fm_tuning &t, bool plain, const WalkArgs &a, hipStream_t s)
{
    if (plain) {
        const uint32_t grid = (a.total + 255) / 256;
        switch (t.occ_interval) {
        case 64: hipLaunchKernelGGL((walk_plain<64, MODE>), dim3(grid), dim3(256), 0, s, a); break;
        case 128: hipLaunchKernelGGL((walk_plain<128, MODE>), dim3(grid), dim3(256), 0, s, a); break;
        case 256: hipLaunchKernelGGL((walk_plain<256, MODE>), dim3(grid), dim3(256), 0, s, a); break;
        default: return hipErrorInvalidValue;
        }
        return hipGetLastError();
    }
    switch (t.occ_interval) {
    case 64: return walk_by_lanes<64, MODE>(idx, t, a, s);
    case 128: return walk_by_lanes<128, MODE>(idx, t, a, s);
    case 256: return walk_by_lanes<256, MODE>(idx, t, a, s);
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
    a.stat_steps = nullptr;
    if (c.flags & FM_STATS) a.stat_steps = (unsigned long long *)((char *)c.ws + kWsStatWalk);
    if (a.total == 0) return hipSuccess;
    switch (mode) {
    case WALK_EXACT: return walk_dispatch<WALK_EXACT>(idx, t, plain, a, s);
    case WALK_DBP: return walk_dispatch<WALK_DBP>(idx, t, plain, a, s);
    case WALK_DFULL: {
        // the full D array is a test and diagnostics output: plain kernel only
        a.dstride = 0;
        return hipErrorInvalidValue;
    }
    default: return hipErrorInvalidValue;
    }
}

// D array entry: needs the total length for the strand blocks.
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
    a.stat_steps = nullptr;
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
    uint32_t total, nstr, strand0, zmax;
    uint32_t scap;         // stack entries per read-strand (3 * zmax)
    uint32_t budget;       // expanded nodes per read-strand
    fm_hit *pool;
    uint64_t cap;
    unsigned long long *pool_count;
    uint32_t *rs_count, *rs_status;
    uint32_t *queue;
    uint32_t *gstack;      // plain kernel: scap * 3 words per read-strand
    unsigned long long *stat_occ, *stat_bk;
};

struct Dfs {
    uint32_t rs;                    // kEmpty when idle
    uint32_t read, strand, m, z0;
    uint64_t base;
    uint32_t nbp, bpw0, bpw1, bpw2; // D breakpoints: nbp, then 16-bit positions
    uint32_t i, zr, k, l;           // current node: pattern symbol i (>= 0) still to match
    uint32_t sp;
    uint32_t hits, status, nodes;
    bool done;
    // hits produced by the last expansion (children of a node with i == 0)
    uint32_t pend, pk[4], pl[4], pd;

    __device__ uint32_t bp_at(uint32_t j) const
    {
        const uint32_t w = j == 0 ? (bpw0 >> 16) : (j == 1 ? bpw1 : (j == 2 ? (bpw1 >> 16) : (j == 3 ? bpw2 : (bpw2 >> 16))));
        return w & 0xFFFFu;
    }

    // D(pos) > zc, i.e. a node needing zc more substitutions for pattern[0..pos] is pruned.
    __device__ bool dprune(uint32_t zc, int pos, bool use_d) const
    {
        if (!use_d || pos < 0) return false;
        return zc < nbp && bp_at(zc) <= (uint32_t)pos;
    }

    __device__ uint32_t sym(const DfsArgs &a, uint32_t pos) const
    {
        if (strand == 0) return a.codes[base + pos];
        const uint32_t c = a.codes[base + m - 1 - pos];
        return c < 4 ? 3u - c : c;
    }

    __device__ void init(const DfsArgs &a, uint32_t item)
    {
        rs = item;
        read = a.nstr == 2 ? item >> 1 : item;
        strand = a.nstr == 2 ? (item & 1u) : a.strand0;
        base = a.offs[read];
        m = (uint32_t)(a.offs[read + 1] - base);
        z0 = a.z[read];
        sp = 0;
        hits = 0;
        status = FM_OK;
        nodes = 0;
        done = false;
        pend = 0;
        pd = 0;
        nbp = 0;
        bpw0 = bpw1 = bpw2 = 0;
        if (z0 > a.zmax) {
            status = FM_EINVAL;
            done = true;
            return;
        }
        if (m > 65535u) {
            status = FM_ERANGE;
            done = true;
            return;
        }
        if (a.bp) {
            const uint4 r = a.bp[item];
            nbp = r.x & 0xFFFFu;
            bpw0 = r.x;
            bpw1 = r.y;
            bpw2 = r.z;
            if (nbp > z0) {               // root pruned: D(m-1) > z
                done = true;
                return;
            }
        }
        if (m == 0) {                     // the empty pattern matches every row
            pend = 1;
            pk[0] = 0;
            pl[0] = a.lay.n;
            pd = 0;
            done = true;
            return;
        }
        i = m - 1;
        zr = z0;
        k = 0;
        l = a.lay.n;
    }
};

// Stack of one read-strand: entries (k, l, i | zr << 16); LDS for the batched kernel,
// global memory for the plain one.
struct StackRef {
    uint32_t *p;
    __device__ void push(uint32_t sp, uint32_t k, uint32_t l, uint32_t iz, bool w) const
    {
        if (w) {
            p[3 * sp] = k;
            p[3 * sp + 1] = l;
            p[3 * sp + 2] = iz;
        }
    }
};

// Expands the current node: one Occ8 at (k-1, l) yields the intervals of all four
// one-symbol extensions (Listing 2's loop over b, each computed from the parent's
// interval and guarded by k_b <= l_b). Children needing more substitutions than left
// (or than the D bound allows) are dropped. At i == 0 the surviving children are hits.
// Otherwise one mismatch child (if any) is continued and the match child and the other
// mismatch children are pushed, the match child deepest -- so the stack never holds
// more than 3 entries per unit of budget spent on the current path (3 * zmax in all).
template <int I, int L>
__device__ void dfs_expand(const DfsArgs &a, Dfs &d, uint32_t q, const Occ4 &ok, const Occ4 &ol,
                           uint32_t wi, const StackRef &st, bool lead)
{
    uint32_t kb[4], lb[4];
    if (d.k == 0) {
#pragma unroll
        for (int b = 0; b < 4; ++b) {
            kb[b] = a.lay.C[b] + 1;
            lb[b] = a.lay.C[b + 1];
        }
    } else {
        const uint32_t o1[4] = {ok.a, ok.c, ok.g, ok.t}, o2[4] = {ol.a, ol.c, ol.g, ol.t};
#pragma unroll
        for (int b = 0; b < 4; ++b) {
            kb[b] = a.lay.C[b] + o1[b] + 1;
            lb[b] = a.lay.C[b] + o2[b];
        }
    }
    const bool use_d = a.bp != nullptr;
    const int child_pos = (int)d.i - 1;
    uint32_t valid = 0;
#pragma unroll
    for (int b = 0; b < 4; ++b) {
        const uint32_t cost = (uint32_t)b != wi ? 1u : 0u;
        if (kb[b] <= lb[b] && d.zr >= cost && !d.dprune(d.zr - cost, child_pos, use_d)) valid |= 1u << b;
    }
    if (d.i == 0) {
        d.pend = valid;
#pragma unroll
        for (int b = 0; b < 4; ++b) {
            d.pk[b] = kb[b];
            d.pl[b] = lb[b];
        }
        d.pd = (d.z0 - d.zr) | (wi << 8);
    } else {
        const uint32_t match = wi < 4 ? (valid & (1u << wi)) : 0u;
        uint32_t mism = valid & ~match;
        if (mism) {
            const uint32_t cont = (uint32_t)__builtin_ctz(mism);
            mism &= ~(1u << cont);
            const uint32_t ci = d.i - 1;
            if (match) {
                st.push(d.sp, kb[wi], lb[wi], ci | (d.zr << 16), lead);
                d.sp += 1;
            }
#pragma unroll
            for (int b = 0; b < 4; ++b) {
                if (mism & (1u << b)) {
                    st.push(d.sp, kb[b], lb[b], ci | ((d.zr - 1) << 16), lead);
                    d.sp += 1;
                }
            }
            d.i = ci;
            d.zr -= 1;
            d.k = kb[cont];
            d.l = lb[cont];
            return;
        }
        if (match) {
            d.i -= 1;
            d.k = kb[wi];
            d.l = lb[wi];
            return;
        }
    }
    // no child to continue: take the next pending node
    if (d.sp == 0) {
        d.done = true;
        return;
    }
    d.sp -= 1;
    const uint32_t *e = st.p + 3 * d.sp;
    d.k = e[0];
    d.l = e[1];
    d.i = e[2] & 0xFFFFu;
    d.zr = e[2] >> 16;
}

// Appends pending hits to the staging pool (one atomic per wave) and retires finished
// read-strands. Must be called by the whole wave.
template <int L>
__device__ void dfs_emit(const DfsArgs &a, Dfs &d, bool active, bool lead)
{
    const uint32_t lane = __lane_id(), leadlane = lane & ~(uint32_t)(L - 1);
    const uint32_t pend = active ? d.pend : 0u;
    uint64_t mb[4];
    uint32_t tot = 0;
#pragma unroll
    for (int b = 0; b < 4; ++b) {
        mb[b] = __ballot(lead && ((pend >> b) & 1u));
        tot += (uint32_t)__popcll(mb[b]);
    }
    if (tot) {
        unsigned long long base = 0;
        if (lane == 0) base = atomicAdd(a.pool_count, (unsigned long long)tot);
        base = __shfl(base, 0);
        uint64_t off = base;
#pragma unroll
        for (int b = 0; b < 4; ++b) {
            if ((pend >> b) & 1u) {
                const uint64_t pos = off + rank_below(mb[b], leadlane);
                const uint32_t wi = d.pd >> 8;
                const uint32_t nmm = (d.pd & 0xFFu) + ((uint32_t)b != wi ? 1u : 0u);
                if (pos < a.cap) {
                    if (lead) ((uint4 *)a.pool)[pos] = make_uint4(d.read, d.pk[b], d.pl[b], d.strand | (nmm << 8));
                } else {
                    d.status = FM_EOVERFLOW;
                }
            }
            off += (uint64_t)__popcll(mb[b]);
        }
    }
    if (active) {
        d.hits += (uint32_t)__popc(pend);
        d.pend = 0;
        if (d.done) {
            if (lead) {
                a.rs_count[d.rs] = d.hits;
                a.rs_status[d.rs] = d.status;
            }
            d.rs = kEmpty;
        }
    }
}

template <int I, int L>
__device__ __forceinline__ void dfs_fetch_expand(const DfsArgs &a, Dfs &d, uint32_t q, const StackRef &st, bool lead,
                                                 uint64_t &n_occ, uint64_t &n_bk)
{
    constexpr int LOG = Geo<I>::LOG;
    const uint32_t wi = d.sym(a, d.i);
    Occ4 o1 = {0, 0, 0, 0}, o2 = {0, 0, 0, 0};
    if (d.k != 0) {
        const uint32_t j2 = d.l >> LOG, j1 = (d.k - 1) >> LOG;
        Bucket<I, L> b1, b2;
        fetch<I, L>(a.lay, j1, q, b1);
        if (j1 != j2) fetch<I, L>(a.lay, j2, q, b2);
        o1 = group_sum4<L>(part4<I, L>(b1, q, (d.k - 1) & (I - 1)));
        o2 = group_sum4<L>(j1 != j2 ? part4<I, L>(b2, q, d.l & (I - 1)) : part4<I, L>(b1, q, d.l & (I - 1)));
        o1.a -= (d.k - 1 >= a.lay.dollar) ? 1u : 0u;
        o2.a -= (d.l >= a.lay.dollar) ? 1u : 0u;
        n_bk += lead ? (j1 != j2 ? 2 : 1) : 0;
    }
    n_occ += lead ? 1 : 0;
    dfs_expand<I, L>(a, d, q, o1, o2, wi, st, lead);
    d.nodes += 1;
    if (!d.done && d.nodes >= a.budget) {
        d.status = FM_EBUDGET;
        d.done = true;
    }
}

template <int I>
__global__ void __launch_bounds__(256) dfs_plain(DfsArgs a)
{
    const uint32_t item = blockIdx.x * blockDim.x + threadIdx.x;
    const bool live = item < a.total;
    Dfs d;
    d.rs = kEmpty;
    if (live) d.init(a, item);
    StackRef st{a.gstack + (size_t)(live ? item : 0) * a.scap * 3};
    uint64_t n_occ = 0, n_bk = 0;
    for (;;) {
        const bool active = d.rs != kEmpty;
        if (!__any(active)) break;
        if (active && !d.done) dfs_fetch_expand<I, 1>(a, d, 0, st, true, n_occ, n_bk);
        dfs_emit<1>(a, d, active, true);
    }
    wave_add(a.stat_occ, n_occ);
    wave_add(a.stat_bk, n_bk);
}

template <int I, int L>
__global__ void __launch_bounds__(256) dfs_batched(DfsArgs a)
{
    extern __shared__ uint32_t lds_stack[];
    const uint32_t q = L == 1 ? 0u : (__lane_id() & (L - 1));
    const bool lead = q == 0;
    const uint32_t group = threadIdx.x / L;
    StackRef st{lds_stack + (size_t)group * a.scap * 3};
    Dfs d;
    d.rs = kEmpty;
    WaveQueue wq = {0, 0, false};
    uint64_t n_occ = 0, n_bk = 0;
    for (;;) {
        const uint32_t it = wave_take<L>(wq, d.rs == kEmpty, a.queue, a.total);
        if (it != kEmpty) d.init(a, it);
        const bool active = d.rs != kEmpty;
        if (!__any(active)) break;
        if (active && !d.done) dfs_fetch_expand<I, L>(a, d, q, st, lead, n_occ, n_bk);
        dfs_emit<L>(a, d, active, lead);
    }
    wave_add(a.stat_occ, n_occ);
    wave_add(a.stat_bk, n_bk);
}

template <int I, int L>
static hipError_t dfs_launch_batched(const fm_index *idx, const fm_tuning &t, const DfsArgs &a, hipStream_t s)
{
    const int block = (int)t.block;
    const size_t lds = (size_t)(block / L) * a.scap * 3 * sizeof(uint32_t);
    int per = max_blocks_per_cu((const void *)dfs_batched<I, L>, block, lds);
    if (t.waves_per_cu) {
        int want = (int)(t.waves_per_cu * 64 / block);
        if (want >= 1 && want < per) per = want;
    }
    uint64_t grid = (uint64_t)idx->cu_count * per;
    const uint64_t need = ((uint64_t)a.total * L + block - 1) / block;
    if (need < grid) grid = need ? need : 1;
    hipLaunchKernelGGL((dfs_batched<I, L>), dim3((uint32_t)grid), dim3(block), lds, s, a);
    return hipGetLastError();
}

template <int I>
static hipError_t dfs_by_lanes(const fm_index *idx, const fm_tuning &t, const DfsArgs &a, hipStream_t s)
{
    switch (t.lanes) {
    case 1: return dfs_launch_batched<I, 1>(idx, t, a, s);
    case 2: return dfs_launch_batched<I, 2>(idx, t, a, s);
    case 4: return dfs_launch_batched<I, 4>(idx, t, a, s);
    case 8: return dfs_launch_batched<I, 8>(idx, t, a, s);
    default: return hipErrorInvalidValue;
    }
}

// ------------------------------------------------------------------ compaction

// Per read: the worst strand status, the hit count to list (0 unless FM_OK), the
// cursor reset, and the count every read would need (for FM_OK and FM_EOVERFLOW reads).
__global__ void finalize_reads(uint32_t nreads, uint32_t nstr, const uint32_t *rs_count, const uint32_t *rs_status,
                               uint32_t *status, uint32_t *cnt, uint32_t *cursor, unsigned long long *required)
{
    const uint32_t r = blockIdx.x * blockDim.x + threadIdx.x;
    uint64_t need = 0;
    if (r < nreads) {
        uint32_t st = 0, c = 0;
        for (uint32_t s = 0; s < nstr; ++s) {
            const uint32_t v = rs_status[r * nstr + s];
            st = v > st ? v : st;
            c += rs_count[r * nstr + s];
        }
        status[r] = st;
        cnt[r] = st == FM_OK ? c : 0u;
        cursor[r] = 0;
        need = (st == FM_OK || st == FM_EOVERFLOW) ? c : 0u;
    }
    wave_add(required, need);
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

__global__ void scatter_hits(const fm_hit *pool, const unsigned long long *pool_count, uint64_t cap,
                             const uint32_t *status, const uint64_t *hit_offs, uint32_t *cursor, fm_hit *hits)
{
    const uint64_t total = *pool_count < cap ? *pool_count : cap;
    for (uint64_t e = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; e < total; e += (uint64_t)gridDim.x * blockDim.x) {
        const uint4 h = ((const uint4 *)pool)[e];
        if (status[h.x] != FM_OK) continue;
        const uint64_t pos = hit_offs[h.x] + atomicAdd(&cursor[h.x], 1u);
        ((uint4 *)hits)[pos] = h;
    }
}

// Hits of one read sorted by (strand, k): in substitution mode every (strand, k) is
// distinct, so the order is unique whatever order the pool received them in.
__global__ void sort_read_hits(uint64_t nreads, const uint64_t *hit_offs, fm_hit *hits)
{
    const uint64_t r = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x;
    if (r >= nreads) return;
    const uint64_t b = hit_offs[r], e = hit_offs[r + 1];
    uint4 *h = (uint4 *)hits;
    for (uint64_t x = b + 1; x < e; ++x) {
        const uint4 v = h[x];
        const uint64_t key = ((uint64_t)(v.w & 0xFFu) << 32) | v.y;
        uint64_t y = x;
        while (y > b) {
            const uint4 u = h[y - 1];
            const uint64_t ku = ((uint64_t)(u.w & 0xFFu) << 32) | u.y;
            if (ku <= key) break;
            h[y] = u;
            --y;
        }
        h[y] = v;
    }
}

InexactWs inexact_ws_layout(uint64_t nreads, uint32_t nstr, uint32_t zmax, uint64_t hit_cap, bool plain)
{
    auto al = [](size_t x) { return (x + 255) & ~(size_t)255; };
    InexactWs w;
    size_t off = kWsHeader;
    const uint64_t nrs = nreads * nstr;
    w.bp = off;        off = al(off + nrs * 16);
    w.rs_count = off;  off = al(off + nrs * 4);
    w.rs_status = off; off = al(off + nrs * 4);
    w.cursor = off;    off = al(off + nreads * 4);
    w.cnt = off;       off = al(off + nreads * 4);
    const uint64_t nblk = (nreads + kScanBlock * kTile - 1) / (kScanBlock * kTile);
    w.part = off;      off = al(off + (nblk + 1) * 8);
    w.pool = off;      off = al(off + hit_cap * 16);
    w.stack = off;
    if (plain) off = al(off + nrs * (3ull * (zmax ? zmax : 1)) * 12);
    w.total = off;
    return w;
}

hipError_t launch_inexact(const fm_index *idx, const fm_tuning &t, const fm_tuning &tw, bool plain, const DfsCall &c,
                          hipStream_t s)
{
    char *ws = (char *)c.ws;
    const uint32_t nstr = strand_count(c.flags);
    const InexactWs W = inexact_ws_layout(c.nreads, nstr, c.zmax, c.hit_cap, plain);
    hipError_t e = launch_fill(ws, 0, kWsHeader / 4, s);
    if (e != hipSuccess) return e;
    if (c.nreads == 0) return launch_fill(c.hit_offs, 0, 2, s);
    const bool use_d = (c.flags & FM_DARRAY) != 0;
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
    a.nstr = nstr;
    a.strand0 = (c.flags & FM_FWD) ? 0u : 1u;
    a.total = (uint32_t)(c.nreads * nstr);
    a.zmax = c.zmax;
    a.scap = 3 * (c.zmax ? c.zmax : 1);
    a.budget = t.node_budget ? t.node_budget : 0xFFFFFFFFu;
    a.pool = (fm_hit *)(ws + W.pool);
    a.cap = c.hit_cap;
    a.pool_count = (unsigned long long *)(ws + kWsPool);
    a.rs_count = (uint32_t *)(ws + W.rs_count);
    a.rs_status = (uint32_t *)(ws + W.rs_status);
    a.queue = (uint32_t *)(ws + kWsQueue2);
    a.gstack = (uint32_t *)(ws + W.stack);
    a.stat_occ = (c.flags & FM_STATS) ? (unsigned long long *)(ws + kWsStatOcc) : nullptr;
    a.stat_bk = (c.flags & FM_STATS) ? (unsigned long long *)(ws + kWsStatBuckets) : nullptr;
    if (plain) {
        const uint32_t grid = (a.total + 255) / 256;
        switch (t.occ_interval) {
        case 64: hipLaunchKernelGGL(dfs_plain<64>, dim3(grid), dim3(256), 0, s, a); break;
        case 128: hipLaunchKernelGGL(dfs_plain<128>, dim3(grid), dim3(256), 0, s, a); break;
        case 256: hipLaunchKernelGGL(dfs_plain<256>, dim3(grid), dim3(256), 0, s, a); break;
        default: return hipErrorInvalidValue;
        }
        e = hipGetLastError();
    } else {
        switch (t.occ_interval) {
        case 64: e = dfs_by_lanes<64>(idx, t, a, s); break;
        case 128: e = dfs_by_lanes<128>(idx, t, a, s); break;
        case 256: e = dfs_by_lanes<256>(idx, t, a, s); break;
        default: return hipErrorInvalidValue;
        }
    }
    if (e != hipSuccess) return e;
    // compaction
    uint32_t *cnt = (uint32_t *)(ws + W.cnt), *cursor = (uint32_t *)(ws + W.cursor);
    const uint32_t nr = (uint32_t)c.nreads;
    hipLaunchKernelGGL(finalize_reads, dim3((nr + 255) / 256), dim3(256), 0, s, nr, nstr, a.rs_count, a.rs_status,
                       c.status, cnt, cursor, (unsigned long long *)(ws + kWsRequired));
    const uint64_t nblk = (c.nreads + kScanBlock * kTile - 1) / (kScanBlock * kTile);
    uint64_t *part = (uint64_t *)(ws + W.part);
    hipLaunchKernelGGL(scan_reduce_u64, dim3((uint32_t)nblk), dim3(kScanBlock), 0, s, cnt, c.nreads, part);
    hipLaunchKernelGGL(scan_partials_u64, dim3(1), dim3(1024), 0, s, part, nblk);
    hipLaunchKernelGGL(scan_write_u64, dim3((uint32_t)nblk), dim3(kScanBlock), 0, s, cnt, c.nreads, part, c.hit_offs);
    uint64_t sgrid = (c.hit_cap + 255) / 256;
    if (sgrid > (uint64_t)idx->cu_count * 8) sgrid = (uint64_t)idx->cu_count * 8;
    if (sgrid == 0) sgrid = 1;
    hipLaunchKernelGGL(scatter_hits, dim3((uint32_t)sgrid), dim3(256), 0, s, a.pool, a.pool_count, c.hit_cap, c.status,
                       c.hit_offs, cursor, c.hits);
    hipLaunchKernelGGL(sort_read_hits, dim3((nr + 255) / 256), dim3(256), 0, s, c.nreads, c.hit_offs, c.hits);
    return hipGetLastError();
}

}  // namespace fm
