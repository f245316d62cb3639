// fm_device.hpp -- device-side building blocks of the Occ computation on gfx950.
//
// Interleaved layout (one bucket per aligned line). Bucket j of the layout with
// checkpoint interval I holds
//   chunk 0        : uint32 counts of A, C, G, T over BWT rows [0, I*j)  ('$' counted as A)
//   chunks 1..I/64 : the I BWT symbols of rows [I*j, I*(j+1)), 2 bits each, LSB first
//                    (row I*j + 16*w + s at bits 2s, 2s+1 of word w, the order of Fig. 2)
//   remaining      : padding up to the bucket size (32, 64, 64, 128, 128 bytes for
//                    I = 64, 128, 192, 256, 448; the dense 192 and 448 have none).
// This is the checkpoint-plus-block arrangement of the Background section (counters of
// every I-th row followed by I 2-bit symbols), with 32-bit counters because n+1 < 2^32.
//
// Occ(c, p) = counts[p / I][c] + (symbols equal to c in rows I*(p/I) .. p)
//             - [c == A and p >= dollar_row]
// The '$' row stores code 0 (A) since two bits cannot hold a fifth symbol; the last
// term removes it. The in-bucket count masks the symbols after p and takes population
// counts of bit planes (Solution section: zero-masking past position k, then counting;
// the half-byte lookup tables are replaced by the native popcount).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace fm {

struct DevLayout {
    const uint4 *bk;     // buckets, Geo<I>::CH chunks of 16 bytes each
    const uint4 *sb;     // compact layouts: uint32 counts at each superblock start
    uint32_t n;          // text length: rows 0..n
    uint32_t dollar;     // row of '$'
    uint32_t C[5];       // C[4] = n
};

// Bucket geometry: CH 16-byte chunks per bucket, of which USED are fetched (counts and
// symbols; the rest is padding). I = 192 and 448 fill their 64- and 128-byte lines.
//
// The compact layouts (I = 96 in 32 bytes, I = 224 in 64 bytes) keep 16-bit counts: the
// bucket's chunk 0 holds the counts of A, C, G, T from the start of its superblock (SB
// buckets, SB * I < 65536 rows) to the bucket, as 4 x uint16, then the bucket's first 32
// symbols; later chunks hold 64 symbols each. A table of uint32 counts at every
// superblock start completes them. Fewer bytes per row keep more of the index in L2.
template <int I> struct Geo;
template <> struct Geo<64> { static constexpr int CH = 2, USED = 2, SB = 0; static constexpr bool COMPACT = false; };
template <> struct Geo<96> { static constexpr int CH = 2, USED = 2, SB = 682; static constexpr bool COMPACT = true; };
template <> struct Geo<128> { static constexpr int CH = 4, USED = 3, SB = 0; static constexpr bool COMPACT = false; };
template <> struct Geo<192> { static constexpr int CH = 4, USED = 4, SB = 0; static constexpr bool COMPACT = false; };
template <> struct Geo<224> { static constexpr int CH = 4, USED = 4, SB = 292; static constexpr bool COMPACT = true; };
template <> struct Geo<256> { static constexpr int CH = 8, USED = 5, SB = 0; static constexpr bool COMPACT = false; };
template <> struct Geo<448> { static constexpr int CH = 8, USED = 8, SB = 0; static constexpr bool COMPACT = false; };

constexpr uint32_t EVEN = 0x55555555u;

// One of four values by a runtime index 0..3 (selects, no indexed memory access).
template <typename T>
__device__ __forceinline__ T sel4(uint32_t i, T a0, T a1, T a2, T a3)
{
    const T lo = (i & 1) ? a1 : a0;
    const T hi = (i & 1) ? a3 : a2;
    return (i & 2) ? hi : lo;
}

__device__ __forceinline__ uint32_t c_of(const DevLayout &lay, uint32_t b)
{
    return sel4(b, lay.C[0], lay.C[1], lay.C[2], lay.C[3]);
}

// Chunks of one bucket held by one lane of an L-lane group: lane q holds chunks
// q, q+L, q+2L, ... below Geo<I>::USED (padding is never fetched).
template <int I, int L> struct Bucket {
    static constexpr int NPL = (Geo<I>::USED + L - 1) / L;
    uint4 v[NPL];
};

template <int I, int L>
__device__ __forceinline__ void fetch(const DevLayout &lay, uint32_t j, uint32_t q, Bucket<I, L> &b)
{
    const uint4 *p = lay.bk + (size_t)j * Geo<I>::CH;
#pragma unroll
    for (int t = 0; t < Bucket<I, L>::NPL; ++t) {
        const uint32_t c = q + L * t;
        if (c < (uint32_t)Geo<I>::USED) b.v[t] = p[c];
        else b.v[t] = make_uint4(0, 0, 0, 0);
    }
}

// Offset of position r (0 <= r < I) relative to the first symbol of chunk c (chunk 0
// holds counts; chunk c >= 1 holds symbols 64(c-1) .. 64c-1), clamped to [-1, 63]:
// -1 = no symbol of the chunk is at or before r, 63 = all are.
__device__ __forceinline__ int chunk_rel(uint32_t r, int c)
{
    if (c < 1) return -1;
    const int rel = (int)r - 64 * (c - 1);
    return rel < -1 ? -1 : (rel > 63 ? 63 : rel);
}

__device__ __forceinline__ uint64_t u64_of(uint32_t lo, uint32_t hi) { return ((uint64_t)hi << 32) | lo; }

// Symbols 0..rel (rel in [-1, 63]) of a 64-symbol chunk given as two 64-bit halves (32
// symbols each, 2 bits per symbol): the half holding symbol rel shifted left so that
// only symbols up to rel remain (the bits shifted in are zero), and the earlier half
// when it is counted whole (else zero). Shifts are by even amounts, so bit pairs stay
// aligned to symbols.
struct Prefix {
    uint64_t part, full;
};

__device__ __forceinline__ Prefix prefix_of(uint64_t h0, uint64_t h1, int rel)
{
    const bool upper = rel >= 32;
    const uint32_t sh = 62u - 2u * ((uint32_t)rel & 31u);
    Prefix p;
    p.part = rel < 0 ? 0ull : ((upper ? h1 : h0) << sh);
    p.full = upper ? h0 : 0ull;
    return p;
}

// Bit 2s set when symbol s of word w equals the symbol whose code, repeated in every
// pair of bits, is pat.
__device__ __forceinline__ uint32_t eq_bits(uint32_t w, uint32_t pat)
{
    const uint32_t x = w ^ pat;
    return ~(x | (x >> 1)) & EVEN;
}

// Population count of a 64-bit value whose set bits are all at even positions: the
// high word moves onto the odd positions of the low one, so one count covers both.
__device__ __forceinline__ uint32_t popc_even64(uint64_t v)
{
    return __popc((uint32_t)v | ((uint32_t)(v >> 32) << 1));
}

// Symbols equal to the symbol of `pat` among symbols 0..rel of a chunk.
__device__ __forceinline__ uint32_t eq_count_chunk(uint4 v, uint32_t pat, int rel)
{
    const Prefix p = prefix_of(u64_of(eq_bits(v.x, pat), eq_bits(v.y, pat)),
                               u64_of(eq_bits(v.z, pat), eq_bits(v.w, pat)), rel);
    return popc_even64(p.part) + popc_even64(p.full);
}

// Adds the bit-plane counts of 32 symbols (low bits set, high bits set, both set). The
// two 16-symbol words share one count per plane: the second word's plane bits take the
// odd positions.
__device__ __forceinline__ void add_planes(uint64_t v, uint32_t &slo, uint32_t &shi, uint32_t &sboth)
{
    const uint32_t u0 = (uint32_t)v, u1 = (uint32_t)(v >> 32);
    const uint32_t lo = (u0 & EVEN) | ((u1 << 1) & ~EVEN);
    const uint32_t hi = ((u0 >> 1) & EVEN) | (u1 & ~EVEN);
    slo = __popc(lo) + slo;
    shi = __popc(hi) + shi;
    sboth = __popc(lo & hi) + sboth;
}

struct Occ4 {
    uint32_t a, c, g, t;
};

// Counts of A, C, G, T among symbols 0..rel of a chunk, from the two bit planes
// (codes 00 01 10 11: T has both bits, C only the low, G only the high one).
__device__ __forceinline__ Occ4 count4_chunk(uint4 v, int rel)
{
    const Prefix p = prefix_of(u64_of(v.x, v.y), u64_of(v.z, v.w), rel);
    uint32_t slo = 0, shi = 0, sboth = 0;
    add_planes(p.part, slo, shi, sboth);
    add_planes(p.full, slo, shi, sboth);
    const uint32_t npos = (uint32_t)(rel + 1);
    return Occ4{npos - slo - shi + sboth, slo - sboth, shi - sboth, sboth};
}

// Mask of the symbols of global word gw (16 symbols) at or before offset r of a bucket.
__device__ __forceinline__ uint32_t gword_mask(int gw, uint32_t r)
{
    const int wr = (int)(r >> 4);
    const uint32_t pm = 0xFFFFFFFFu >> (30 - 2 * (r & 15));
    return gw < wr ? 0xFFFFFFFFu : (gw == wr ? pm : 0u);
}

// Symbols of global word gw counted at offset r (0..16).
__device__ __forceinline__ uint32_t gword_npos(int gw, uint32_t r)
{
    const int v = (int)r + 1 - 16 * gw;
    return (uint32_t)(v < 0 ? 0 : (v > 16 ? 16 : v));
}

// Compact layouts: the global word index of word i (0..3) of chunk c, or -1 for the
// counts half of chunk 0.
__device__ __forceinline__ int compact_gw(int c, int i) { return c == 0 ? (i < 2 ? -1 : i - 2) : 4 * c - 2 + i; }

__device__ __forceinline__ uint32_t u16_count(uint4 v, uint32_t sym)
{
    return sel4(sym, v.x & 0xFFFFu, v.x >> 16, v.y & 0xFFFFu, v.y >> 16);
}

// This lane's share of Occ(sym, p1) and Occ(sym, p2) for positions at offsets r1 (in
// bucket a) and r2 (in bucket b2). The group sums are the two Occ values before the
// '$' correction.
template <int I, int L>
__device__ __forceinline__ void part2(const Bucket<I, L> &a, const Bucket<I, L> &b2, uint32_t q,
                                      uint32_t r1, uint32_t r2, uint32_t sym, uint4 sb1, uint4 sb2,
                                      uint32_t &o1, uint32_t &o2)
{
    const uint32_t pat = sym * EVEN;
    uint32_t s1 = 0, s2 = 0;
#pragma unroll
    for (int t = 0; t < Bucket<I, L>::NPL; ++t) {
        const int c = (int)q + L * t;
        const uint4 va = a.v[t];
        const uint4 vb = b2.v[t];
        if constexpr (Geo<I>::COMPACT) {
            if (c >= Geo<I>::USED) continue;
            if (c == 0) {
                s1 += u16_count(va, sym) + sel4(sym, sb1.x, sb1.y, sb1.z, sb1.w);
                s2 += u16_count(vb, sym) + sel4(sym, sb2.x, sb2.y, sb2.z, sb2.w);
            }
            const uint32_t wa[4] = {va.x, va.y, va.z, va.w}, wb[4] = {vb.x, vb.y, vb.z, vb.w};
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                const int gw = compact_gw(c, i);
                if (gw < 0) continue;
                const uint32_t xa = wa[i] ^ pat, xb = wb[i] ^ pat;
                const uint32_t ea = ~(xa | (xa >> 1)) & EVEN, eb = ~(xb | (xb >> 1)) & EVEN;
                s1 = __popc(ea & gword_mask(gw, r1)) + s1;
                s2 = __popc(eb & gword_mask(gw, r2)) + s2;
            }
        } else {
            if (c == 0) {
                s1 += sel4(sym, va.x, va.y, va.z, va.w);
                s2 += sel4(sym, vb.x, vb.y, vb.z, vb.w);
            } else if (c < Geo<I>::USED) {
                s1 += eq_count_chunk(va, pat, chunk_rel(r1, c));
                s2 += eq_count_chunk(vb, pat, chunk_rel(r2, c));
            }
        }
    }
    o1 = s1;
    o2 = s2;
}

// Occ(sym, p) before the '$' correction for the position at offset r of a bucket held
// whole by one lane (L = 1): the bucket's count of sym plus the symbols equal to sym at
// offsets 0..r (sbc: the superblock counts of compact layouts).
template <int I>
__device__ __forceinline__ uint32_t part1(const Bucket<I, 1> &bk, uint32_t r, uint32_t sym, uint4 sbc)
{
    const uint32_t pat = sym * EVEN;
    uint32_t s = 0;
#pragma unroll
    for (int c = 0; c < Geo<I>::USED; ++c) {
        const uint4 v = bk.v[c];
        if constexpr (Geo<I>::COMPACT) {
            if (c == 0) s += u16_count(v, sym) + sel4(sym, sbc.x, sbc.y, sbc.z, sbc.w);
            const uint32_t w[4] = {v.x, v.y, v.z, v.w};
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                const int gw = compact_gw(c, i);
                if (gw < 0) continue;
                const uint32_t x = w[i] ^ pat;
                s = __popc(~(x | (x >> 1)) & EVEN & gword_mask(gw, r)) + s;
            }
        } else {
            if (c == 0) s += sel4(sym, v.x, v.y, v.z, v.w);
            else s += eq_count_chunk(v, pat, chunk_rel(r, c));
        }
    }
    return s;
}

// The BWT symbol at offset r of a bucket held whole by one lane (L = 1): 2 bits of the
// symbol word r / 16. Compact layouts keep symbol words 0-1 in chunk 0 (after the
// counts) and four per chunk after it; the others keep four per chunk from chunk 1. The
// word is picked by masks rather than selects: a select between two of the bucket's
// loaded words lets the compiler turn it into one load at a computed offset, which moves
// the bucket to scratch memory.
template <int I>
__device__ __forceinline__ uint32_t symbol_at(const Bucket<I, 1> &bk, uint32_t r)
{
    const int g = (int)(r / 16);
    uint32_t word = 0;
#pragma unroll
    for (int t = 0; t < Bucket<I, 1>::NPL; ++t) {
        const uint32_t w[4] = {bk.v[t].x, bk.v[t].y, bk.v[t].z, bk.v[t].w};
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            const int gw = Geo<I>::COMPACT ? compact_gw(t, i) : (t == 0 ? -1 : 4 * (t - 1) + i);
            if (gw < 0) continue;
            word |= w[i] & (0u - (uint32_t)(g == gw));
        }
    }
    return (word >> (2 * (r % 16))) & 3u;
}

// This lane's share of Occ(., p) for all four symbols at offset r of a bucket (sbc:
// the superblock counts of compact layouts).
template <int I, int L>
__device__ __forceinline__ Occ4 part4(const Bucket<I, L> &bk, uint32_t q, uint32_t r, uint4 sbc)
{
    Occ4 o = {0, 0, 0, 0};
#pragma unroll
    for (int t = 0; t < Bucket<I, L>::NPL; ++t) {
        const int c = (int)q + L * t;
        const uint4 v = bk.v[t];
        if constexpr (Geo<I>::COMPACT) {
            if (c >= Geo<I>::USED) continue;
            if (c == 0) {
                o.a += (v.x & 0xFFFFu) + sbc.x;
                o.c += (v.x >> 16) + sbc.y;
                o.g += (v.y & 0xFFFFu) + sbc.z;
                o.t += (v.y >> 16) + sbc.w;
            }
            const uint32_t w[4] = {v.x, v.y, v.z, v.w};
            uint32_t slo = 0, shi = 0, sboth = 0, npos = 0;
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                const int gw = compact_gw(c, i);
                if (gw < 0) continue;
                const uint32_t m = gword_mask(gw, r);
                const uint32_t lo = w[i] & EVEN & m, hi = (w[i] >> 1) & EVEN & m;
                slo = __popc(lo) + slo;
                shi = __popc(hi) + shi;
                sboth = __popc(lo & hi) + sboth;
                npos += gword_npos(gw, r);
            }
            o.a += npos - slo - shi + sboth;
            o.c += slo - sboth;
            o.g += shi - sboth;
            o.t += sboth;
        } else {
            if (c == 0) {
                o.a += v.x;
                o.c += v.y;
                o.g += v.z;
                o.t += v.w;
            } else if (c < Geo<I>::USED) {
                const Occ4 p = count4_chunk(v, chunk_rel(r, c));
                o.a += p.a;
                o.c += p.c;
                o.g += p.g;
                o.t += p.t;
            }
        }
    }
    return o;
}

// Sum over the L lanes of a group (groups are aligned runs of L lanes).
template <int L>
__device__ __forceinline__ uint32_t group_sum(uint32_t v)
{
    if (L >= 2) v += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0xB1, 0xF, 0xF, false);  // lane ^ 1
    if (L >= 4) v += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x4E, 0xF, 0xF, false);  // lane ^ 2
    if (L >= 8) v += (uint32_t)__builtin_amdgcn_ds_swizzle((int)v, 0x101F);                     // lane ^ 4
    return v;
}

template <int L>
__device__ __forceinline__ Occ4 group_sum4(Occ4 o)
{
    o.a = group_sum<L>(o.a);
    o.c = group_sum<L>(o.c);
    o.g = group_sum<L>(o.g);
    o.t = group_sum<L>(o.t);
    return o;
}

// Buckets of one query (k, l): the bucket of k-1 and the bucket of l, both loads issued
// before either is used. The second is loaded even when both positions share a bucket:
// the line is then already on its way, and a conditional load would let the compiler
// fill the second bucket from the first, which waits for the first load before issuing
// the second. Callers guarantee k >= 1.
template <int I, int L>
struct Pair {
    Bucket<I, L> a, b;
    uint4 sa, sbk;         // compact layouts: superblock counts of the two buckets
    bool same;
    __device__ __forceinline__ void load(const DevLayout &lay, uint32_t q, uint32_t k, uint32_t l)
    {
        const uint32_t j1 = (k - 1) / I, j2 = l / I;
        same = j1 == j2;
        fetch<I, L>(lay, j1, q, a);
        fetch<I, L>(lay, j2, q, b);
        if constexpr (Geo<I>::COMPACT) {
            sa = lay.sb[j1 / Geo<I>::SB];
            sbk = lay.sb[j2 / Geo<I>::SB];
        } else {
            sa = sbk = make_uint4(0, 0, 0, 0);
        }
    }
};

// Occ(sym, k-1) and Occ(sym, l) -- the two values one step of Listing 1 consumes.
template <int I, int L>
__device__ __forceinline__ void occ2(const DevLayout &lay, const Pair<I, L> &pr, uint32_t q, uint32_t sym,
                                     uint32_t k, uint32_t l, uint32_t &ok, uint32_t &ol)
{
    uint32_t c1, c2;
    part2<I, L>(pr.a, pr.b, q, (k - 1) % I, l % I, sym, pr.sa, pr.sbk, c1, c2);
    c1 = group_sum<L>(c1);
    c2 = group_sum<L>(c2);
    const bool a = sym == 0;
    ok = c1 - ((a && k - 1 >= lay.dollar) ? 1u : 0u);
    ol = c2 - ((a && l >= lay.dollar) ? 1u : 0u);
}

// The eight values of one inexact step: Occ(., k-1) and Occ(., l).
template <int I, int L>
__device__ __forceinline__ void occ8(const DevLayout &lay, const Pair<I, L> &pr, uint32_t q, uint32_t k, uint32_t l,
                                     Occ4 &ok, Occ4 &ol)
{
    Occ4 o1 = group_sum4<L>(part4<I, L>(pr.a, q, (k - 1) % I, pr.sa));
    Occ4 o2 = group_sum4<L>(part4<I, L>(pr.b, q, l % I, pr.sbk));
    o1.a -= (k - 1 >= lay.dollar) ? 1u : 0u;
    o2.a -= (l >= lay.dollar) ? 1u : 0u;
    ok = o1;
    ol = o2;
}

// ------------------------------------------------------------------ block scans

// Exclusive scan of one uint32 per thread over a block of blockDim.x (multiple of 64,
// <= 1024) threads. Returns the exclusive prefix; *total gets the block sum.
__device__ __forceinline__ uint32_t block_scan_u32(uint32_t v, uint32_t *lds, uint32_t *total)
{
    const uint32_t lane = __lane_id(), wave = threadIdx.x >> 6, nw = blockDim.x >> 6;
    uint32_t x = v;
#pragma unroll
    for (int d = 1; d < 64; d <<= 1) {
        uint32_t y = __shfl_up(x, d);
        if (lane >= (uint32_t)d) x += y;
    }
    if (lane == 63) lds[wave] = x;
    __syncthreads();
    if (threadIdx.x == 0) {
        uint32_t acc = 0;
        for (uint32_t w = 0; w < nw; ++w) {
            uint32_t t = lds[w];
            lds[w] = acc;
            acc += t;
        }
        lds[16] = acc;
    }
    __syncthreads();
    uint32_t r = lds[wave] + x - v;
    *total = lds[16];
    __syncthreads();
    return r;
}

__device__ __forceinline__ uint64_t block_scan_u64(uint64_t v, uint64_t *lds, uint64_t *total)
{
    const uint32_t lane = __lane_id(), wave = threadIdx.x >> 6, nw = blockDim.x >> 6;
    uint64_t x = v;
#pragma unroll
    for (int d = 1; d < 64; d <<= 1) {
        uint64_t y = __shfl_up(x, d);
        if (lane >= (uint32_t)d) x += y;
    }
    if (lane == 63) lds[wave] = x;
    __syncthreads();
    if (threadIdx.x == 0) {
        uint64_t acc = 0;
        for (uint32_t w = 0; w < nw; ++w) {
            uint64_t t = lds[w];
            lds[w] = acc;
            acc += t;
        }
        lds[16] = acc;
    }
    __syncthreads();
    uint64_t r = lds[wave] + x - v;
    *total = lds[16];
    __syncthreads();
    return r;
}

// ------------------------------------------------------------------ wave helpers

// Bits of `mask` for lanes strictly below the calling lane.
__device__ __forceinline__ uint32_t lanes_below(uint64_t mask)
{
    return __builtin_amdgcn_mbcnt_hi((uint32_t)(mask >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)mask, 0u));
}

// Bits of `mask` for lanes strictly below `lane`.
__device__ __forceinline__ uint32_t rank_below(uint64_t mask, uint32_t lane)
{
    const uint64_t below = lane ? (mask & ((~0ull) >> (64 - lane))) : 0ull;
    return (uint32_t)__popcll(below);
}

}  // namespace fm
