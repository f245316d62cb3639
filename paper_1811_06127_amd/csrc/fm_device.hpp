// fm_device.hpp -- device-side building blocks of the Occ computation on gfx950.
//
// Interleaved layout (one bucket per aligned line). Bucket j of the layout with
// checkpoint interval I holds
//   chunk 0        : uint32 counts of A, C, G, T over BWT rows [0, I*j)  ('$' counted as A)
//   chunks 1..I/64 : the I BWT symbols of rows [I*j, I*(j+1)), 2 bits each, LSB first
//                    (row I*j + 16*w + s at bits 2s, 2s+1 of word w, the order of Fig. 2)
//   remaining      : padding up to the bucket size (32, 64, 128 bytes for I = 64, 128, 256).
// This is the checkpoint-plus-block arrangement of the Background section (counters of
// every I-th row followed by I 2-bit symbols), with 32-bit counters because n+1 < 2^32.
//
// Occ(c, p) = counts[p / I][c] + (symbols equal to c in rows I*(p/I) .. p)
//             - [c == A and p >= dollar_row]
// The '$' row stores code 0 (A) since two bits cannot hold a fifth symbol; the last
// term removes it. The in-bucket count masks the symbols after p and takes population
// counts of the two bit planes (Solution section: zero-masking past position k, then
// counting; the half-byte lookup tables are replaced by the native popcount).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace fm {

struct DevLayout {
    const uint4 *bk;     // buckets, Geo<I>::CH chunks of 16 bytes each
    uint32_t n;          // text length: rows 0..n
    uint32_t dollar;     // row of '$'
    uint32_t C[5];       // C[4] = n
};

template <int I> struct Geo;
template <> struct Geo<64> { static constexpr int CH = 2, USED = 2, LOG = 6; };
template <> struct Geo<128> { static constexpr int CH = 4, USED = 3, LOG = 7; };
template <> struct Geo<256> { static constexpr int CH = 8, USED = 5, LOG = 8; };

constexpr uint32_t EVEN = 0x55555555u;

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

// Mask of the symbols of one 16-symbol word that lie at or before the position:
// rel = position - first row of the word.
__device__ __forceinline__ uint32_t word_mask(int rel)
{
    uint32_t m = 0xFFFFFFFFu >> (30 - 2 * (rel < 0 ? 0 : (rel > 15 ? 15 : rel)));
    return rel < 0 ? 0u : m;
}

// Symbols equal to `b` (pat = b * 0x55555555) among the masked symbols of w.
__device__ __forceinline__ uint32_t count_eq(uint32_t w, uint32_t pat, uint32_t m, uint32_t acc)
{
    const uint32_t x = w ^ pat;
    const uint32_t eq = ~(x | (x >> 1)) & EVEN & m;
    return __popc(eq) + acc;
}

// This lane's share of Occ(b, p) for p at offset r of the bucket: its counts chunk
// (if it holds chunk 0) plus its symbol chunks. The group sum is Occ(b, p), before the
// '$' correction.
template <int I, int L>
__device__ __forceinline__ uint32_t part1(const Bucket<I, L> &bk, uint32_t q, uint32_t r, uint32_t b)
{
    const uint32_t pat = b * EVEN;
    uint32_t acc = 0;
#pragma unroll
    for (int t = 0; t < Bucket<I, L>::NPL; ++t) {
        const int c = (int)q + L * t;
        const uint4 v = bk.v[t];
        const uint32_t sel = b == 0 ? v.x : (b == 1 ? v.y : (b == 2 ? v.z : v.w));
        acc += (c == 0) ? sel : 0u;
        const int rel = (c >= 1 && c < Geo<I>::USED) ? (int)r - (c - 1) * 64 : -1;
        acc = count_eq(v.x, pat, word_mask(rel), acc);
        acc = count_eq(v.y, pat, word_mask(rel - 16), acc);
        acc = count_eq(v.z, pat, word_mask(rel - 32), acc);
        acc = count_eq(v.w, pat, word_mask(rel - 48), acc);
    }
    return acc;
}

struct Occ4 {
    uint32_t a, c, g, t;
};

// This lane's share of Occ(., p) for all four symbols (same conventions as part1).
template <int I, int L>
__device__ __forceinline__ Occ4 part4(const Bucket<I, L> &bk, uint32_t q, uint32_t r)
{
    Occ4 o = {0, 0, 0, 0};
#pragma unroll
    for (int t = 0; t < Bucket<I, L>::NPL; ++t) {
        const int c = (int)q + L * t;
        const uint4 v = bk.v[t];
        const uint32_t keep = (c == 0) ? 0xFFFFFFFFu : 0u;
        o.a += v.x & keep;
        o.c += v.y & keep;
        o.g += v.z & keep;
        o.t += v.w & keep;
        const int rel = (c >= 1 && c < Geo<I>::USED) ? (int)r - (c - 1) * 64 : -1;
        const uint32_t w[4] = {v.x, v.y, v.z, v.w};
        uint32_t slo = 0, shi = 0, sboth = 0;
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            const uint32_t m = word_mask(rel - 16 * i);
            const uint32_t lo = w[i] & EVEN & m;          // low bit of each symbol
            const uint32_t hi = (w[i] >> 1) & EVEN & m;   // high bit of each symbol
            slo += __popc(lo);
            shi += __popc(hi);
            sboth += __popc(lo & hi);
        }
        const int npos = rel < 0 ? 0 : (rel >= 63 ? 64 : rel + 1);
        o.a += (uint32_t)npos - slo - shi + sboth;        // 00
        o.c += slo - sboth;                               // 01
        o.g += shi - sboth;                               // 10
        o.t += sboth;                                     // 11
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

// Occ(b, k-1) and Occ(b, l) -- the two values one step of Listing 1 consumes.
// Fetches one bucket, or two when k-1 and l fall in different buckets.
template <int I, int L>
__device__ __forceinline__ void occ2(const DevLayout &lay, uint32_t q, uint32_t b, uint32_t k,
                                     uint32_t l, uint32_t &ok, uint32_t &ol)
{
    constexpr int LOG = Geo<I>::LOG;
    const uint32_t j2 = l >> LOG;
    const uint32_t j1 = k ? (k - 1) >> LOG : j2;
    Bucket<I, L> b1, b2;
    fetch<I, L>(lay, j1, q, b1);
    if (j1 != j2) fetch<I, L>(lay, j2, q, b2);
    else b2 = b1;
    uint32_t c1 = part1<I, L>(b1, q, (k - 1) & (I - 1), b);
    uint32_t c2 = part1<I, L>(b2, q, l & (I - 1), b);
    c1 = group_sum<L>(c1);
    c2 = group_sum<L>(c2);
    if (b == 0) {
        c1 -= (k - 1 >= lay.dollar) ? 1u : 0u;
        c2 -= (l >= lay.dollar) ? 1u : 0u;
    }
    ok = k ? c1 : 0u;
    ol = c2;
}

// The eight values of one inexact step: Occ(., k-1) and Occ(., l).
template <int I, int L>
__device__ __forceinline__ void occ8(const DevLayout &lay, uint32_t q, uint32_t k, uint32_t l,
                                     Occ4 &ok, Occ4 &ol)
{
    constexpr int LOG = Geo<I>::LOG;
    const uint32_t j2 = l >> LOG;
    const uint32_t j1 = k ? (k - 1) >> LOG : j2;
    Bucket<I, L> b1, b2;
    fetch<I, L>(lay, j1, q, b1);
    if (j1 != j2) fetch<I, L>(lay, j2, q, b2);
    else b2 = b1;
    Occ4 o1 = group_sum4<L>(part4<I, L>(b1, q, (k - 1) & (I - 1)));
    Occ4 o2 = group_sum4<L>(part4<I, L>(b2, q, l & (I - 1)));
    o1.a -= (k - 1 >= lay.dollar) ? 1u : 0u;
    o2.a -= (l >= lay.dollar) ? 1u : 0u;
    if (!k) o1 = Occ4{0, 0, 0, 0};
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

__device__ __forceinline__ uint32_t lane_id() { return __lane_id(); }

__device__ __forceinline__ uint64_t ballot(bool p) { return __ballot(p); }

// Bits of `mask` for lanes strictly below `lane`.
__device__ __forceinline__ uint32_t rank_below(uint64_t mask, uint32_t lane)
{
    const uint64_t below = lane ? (mask & ((~0ull) >> (64 - lane))) : 0ull;
    return (uint32_t)__popcll(below);
}

}  // namespace fm
