// layout.hip -- interleaved checkpoint layout (built once at load time), the fill
// kernel used instead of memsets, and the Occ8 kernel.
#include <mutex>
#include <unordered_map>

#include "fm_internal.hpp"

namespace fm {

// ------------------------------------------------------------------ fill

__global__ void fill_kernel(uint32_t *p, uint32_t value, size_t words)
{
    for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < words; i += (size_t)gridDim.x * blockDim.x)
        p[i] = value;
}

hipError_t launch_fill(void *p, uint32_t value, size_t words, hipStream_t s)
{
    if (!words) return hipSuccess;
    size_t blocks = (words + 255) / 256;
    if (blocks > 65536) blocks = 65536;
    hipLaunchKernelGGL(fill_kernel, dim3((uint32_t)blocks), dim3(256), 0, s, (uint32_t *)p, value, words);
    return hipGetLastError();
}

// ------------------------------------------------------------------ layout build

constexpr int kTile = 8;          // buckets per thread in the scan passes
constexpr int kScanBlock = 256;

// Symbol totals (A, C, G, T; '$' counted as A) of each full bucket j < nb - 1; the last
// bucket's total is never needed (no checkpoint follows it) and is left at zero.
template <int I>
__global__ void bucket_totals(const uint32_t *packed, uint64_t nb, uint4 *tot)
{
    const uint64_t j = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x;
    if (j >= nb) return;
    if (j == nb - 1) {
        tot[j] = make_uint4(0, 0, 0, 0);
        return;
    }
    const uint32_t *w = packed + j * (I / 16);
    uint32_t slo = 0, shi = 0, sb = 0;
#pragma unroll
    for (int i = 0; i < I / 16; ++i) {
        const uint32_t lo = w[i] & EVEN, hi = (w[i] >> 1) & EVEN;
        slo += __popc(lo);
        shi += __popc(hi);
        sb += __popc(lo & hi);
    }
    tot[j] = make_uint4(I - slo - shi + sb, slo - sb, shi - sb, sb);
}

// Pass A: per-block sums of kScanBlock * kTile consecutive totals.
__global__ void scan_reduce4(const uint4 *tot, uint64_t nb, uint4 *part)
{
    __shared__ uint32_t lds[32];
    const uint64_t base = (blockIdx.x * (uint64_t)blockDim.x + threadIdx.x) * kTile;
    uint4 acc = make_uint4(0, 0, 0, 0);
    for (int t = 0; t < kTile; ++t) {
        if (base + t < nb) {
            uint4 v = tot[base + t];
            acc.x += v.x; acc.y += v.y; acc.z += v.z; acc.w += v.w;
        }
    }
    uint32_t sx, sy, sz, sw;
    block_scan_u32(acc.x, lds, &sx);
    block_scan_u32(acc.y, lds, &sy);
    block_scan_u32(acc.z, lds, &sz);
    block_scan_u32(acc.w, lds, &sw);
    if (threadIdx.x == 0) part[blockIdx.x] = make_uint4(sx, sy, sz, sw);
}

// Pass B: exclusive scan of the per-block sums, in place, by one block.
__global__ void scan_partials4(uint4 *part, uint64_t np)
{
    __shared__ uint32_t lds[32];
    const uint64_t per = (np + blockDim.x - 1) / blockDim.x;
    const uint64_t b0 = threadIdx.x * per;
    uint4 acc = make_uint4(0, 0, 0, 0);
    for (uint64_t i = b0; i < b0 + per && i < np; ++i) {
        uint4 v = part[i];
        acc.x += v.x; acc.y += v.y; acc.z += v.z; acc.w += v.w;
    }
    uint32_t t;
    uint4 off;
    off.x = block_scan_u32(acc.x, lds, &t);
    off.y = block_scan_u32(acc.y, lds, &t);
    off.z = block_scan_u32(acc.z, lds, &t);
    off.w = block_scan_u32(acc.w, lds, &t);
    for (uint64_t i = b0; i < b0 + per && i < np; ++i) {
        uint4 v = part[i];
        part[i] = off;
        off.x += v.x; off.y += v.y; off.z += v.z; off.w += v.w;
    }
}

// Pass C: checkpoint of every bucket (exclusive prefix of the totals) and the bucket
// itself: counts chunk, symbol chunks copied from the packed BWT, zero padding.
template <int I>
__global__ void write_buckets(const uint32_t *packed, uint64_t nwords, const uint4 *tot, uint64_t nb,
                              const uint4 *part, uint4 *out)
{
    __shared__ uint32_t lds[32];
    constexpr int CH = Geo<I>::CH, USED = Geo<I>::USED;
    const uint64_t base = (blockIdx.x * (uint64_t)blockDim.x + threadIdx.x) * kTile;
    uint4 loc[kTile];
    uint4 acc = make_uint4(0, 0, 0, 0);
    for (int t = 0; t < kTile; ++t) {
        loc[t] = acc;
        if (base + t < nb) {
            uint4 v = tot[base + t];
            acc.x += v.x; acc.y += v.y; acc.z += v.z; acc.w += v.w;
        }
    }
    uint32_t dummy;
    uint4 off = part[blockIdx.x];
    off.x += block_scan_u32(acc.x, lds, &dummy);
    off.y += block_scan_u32(acc.y, lds, &dummy);
    off.z += block_scan_u32(acc.z, lds, &dummy);
    off.w += block_scan_u32(acc.w, lds, &dummy);
    for (int t = 0; t < kTile; ++t) {
        const uint64_t j = base + t;
        if (j >= nb) break;
        uint4 *b = out + j * CH;
        b[0] = make_uint4(off.x + loc[t].x, off.y + loc[t].y, off.z + loc[t].z, off.w + loc[t].w);
        for (int c = 1; c < CH; ++c) {
            uint4 v = make_uint4(0, 0, 0, 0);
            if (c < USED) {
                const uint64_t w0 = j * (I / 16) + (uint64_t)(c - 1) * 4;
                if (w0 + 0 < nwords) v.x = packed[w0 + 0];
                if (w0 + 1 < nwords) v.y = packed[w0 + 1];
                if (w0 + 2 < nwords) v.z = packed[w0 + 2];
                if (w0 + 3 < nwords) v.w = packed[w0 + 3];
            }
            b[c] = v;
        }
    }
}

// Compact layouts, pass C: the checkpoint of every bucket (exclusive prefix of the
// totals) replaces its total in `tot`, and every superblock start is recorded in sb.
template <int I>
__global__ void compact_checkpoints(uint4 *tot, uint64_t nb, const uint4 *part, uint4 *sb)
{
    __shared__ uint32_t lds[32];
    const uint64_t base = (blockIdx.x * (uint64_t)blockDim.x + threadIdx.x) * kTile;
    uint4 loc[kTile];
    uint4 acc = make_uint4(0, 0, 0, 0);
    for (int t = 0; t < kTile; ++t) {
        loc[t] = acc;
        if (base + t < nb) {
            uint4 v = tot[base + t];
            acc.x += v.x; acc.y += v.y; acc.z += v.z; acc.w += v.w;
        }
    }
    uint32_t dummy;
    uint4 off = part[blockIdx.x];
    off.x += block_scan_u32(acc.x, lds, &dummy);
    off.y += block_scan_u32(acc.y, lds, &dummy);
    off.z += block_scan_u32(acc.z, lds, &dummy);
    off.w += block_scan_u32(acc.w, lds, &dummy);
    for (int t = 0; t < kTile; ++t) {
        const uint64_t j = base + t;
        if (j >= nb) break;
        const uint4 g = make_uint4(off.x + loc[t].x, off.y + loc[t].y, off.z + loc[t].z, off.w + loc[t].w);
        tot[j] = g;
        if (j % Geo<I>::SB == 0) sb[j / Geo<I>::SB] = g;
    }
}

// Compact layouts, pass D: 16-bit counts relative to the bucket's superblock, then the
// bucket's symbols (words 0-1 in chunk 0, then four words per chunk).
template <int I>
__global__ void compact_buckets(const uint32_t *packed, uint64_t nwords, const uint4 *gck, uint64_t nb,
                                const uint4 *sb, uint4 *out)
{
    const uint64_t j = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x;
    if (j >= nb) return;
    constexpr int CH = Geo<I>::CH, NW = I / 16;
    const uint4 g = gck[j], s0 = sb[j / Geo<I>::SB];
    uint32_t w[4 * CH - 2];
    for (int i = 0; i < 4 * CH - 2; ++i) {
        const uint64_t wi = j * NW + i;
        w[i] = (i < NW && wi < nwords) ? packed[wi] : 0u;
    }
    uint4 *b = out + j * CH;
    b[0] = make_uint4((g.x - s0.x) | ((g.y - s0.y) << 16), (g.z - s0.z) | ((g.w - s0.w) << 16), w[0], w[1]);
    for (int c = 1; c < CH; ++c) b[c] = make_uint4(w[4 * c - 2], w[4 * c - 1], w[4 * c], w[4 * c + 1]);
}

size_t build_layout_scratch(uint64_t n, uint32_t I)
{
    const uint64_t nb = num_buckets(n, I);
    const uint64_t nblk = (nb + kScanBlock * kTile - 1) / (kScanBlock * kTile);
    return (size_t)(nb * 16 + nblk * 16 + 256);
}

template <int I>
static hipError_t build_layout_t(const uint32_t *packed, uint64_t n, void *out, void *scratch, hipStream_t s)
{
    const uint64_t nb = num_buckets(n, I);
    const uint64_t nwords = (n + 1 + 15) / 16;
    const uint64_t nblk = (nb + kScanBlock * kTile - 1) / (kScanBlock * kTile);
    uint4 *tot = (uint4 *)scratch;
    uint4 *part = (uint4 *)((char *)scratch + nb * 16);
    hipLaunchKernelGGL(bucket_totals<I>, dim3((uint32_t)((nb + 255) / 256)), dim3(256), 0, s, packed, nb, tot);
    hipLaunchKernelGGL(scan_reduce4, dim3((uint32_t)nblk), dim3(kScanBlock), 0, s, tot, nb, part);
    hipLaunchKernelGGL(scan_partials4, dim3(1), dim3(1024), 0, s, part, nblk);
    if constexpr (Geo<I>::COMPACT) {
        uint4 *sb = (uint4 *)((char *)out + nb * bucket_bytes(I));
        hipLaunchKernelGGL(compact_checkpoints<I>, dim3((uint32_t)nblk), dim3(kScanBlock), 0, s, tot, nb, part, sb);
        hipLaunchKernelGGL(compact_buckets<I>, dim3((uint32_t)((nb + 255) / 256)), dim3(256), 0, s, packed, nwords,
                           tot, nb, sb, (uint4 *)out);
    } else {
        hipLaunchKernelGGL(write_buckets<I>, dim3((uint32_t)nblk), dim3(kScanBlock), 0, s, packed, nwords, tot, nb,
                           part, (uint4 *)out);
    }
    return hipGetLastError();
}

hipError_t build_layout(const uint32_t *packed_dev, uint64_t n, uint32_t I, void *out, void *scratch, hipStream_t s)
{
    switch (I) {
    case 64: return build_layout_t<64>(packed_dev, n, out, scratch, s);
    case 96: return build_layout_t<96>(packed_dev, n, out, scratch, s);
    case 128: return build_layout_t<128>(packed_dev, n, out, scratch, s);
    case 192: return build_layout_t<192>(packed_dev, n, out, scratch, s);
    case 224: return build_layout_t<224>(packed_dev, n, out, scratch, s);
    case 256: return build_layout_t<256>(packed_dev, n, out, scratch, s);
    case 448: return build_layout_t<448>(packed_dev, n, out, scratch, s);
    default: return hipErrorInvalidValue;
    }
}

// ------------------------------------------------------------------ Occ8

// One query per group of L lanes, grid-stride. Out-of-range queries are answered with
// all-ones and fetch bucket 0 instead of their own.
template <int I, int L>
__global__ void __launch_bounds__(256) occ8_kernel(DevLayout lay, const uint2 *q, uint64_t nq, uint32_t *out)
{
    const uint32_t q_lane = L == 1 ? 0 : (__lane_id() & (L - 1));
    const uint64_t groups = (uint64_t)gridDim.x * (blockDim.x / L);
    for (uint64_t g = (blockIdx.x * (uint64_t)blockDim.x + threadIdx.x) / L; g < nq; g += groups) {
        const uint2 kl = q[g];
        const bool ok = kl.x <= lay.n + 1 && kl.y <= lay.n;
        // row k-1 = -1 has no bucket (its values are 0); row 0's stands in for it
        const uint32_t k = ok && kl.x ? kl.x : 1u, l = ok ? kl.y : 0u;
        Pair<I, L> pr;
        pr.load(lay, q_lane, k, l);
        Occ4 a, b;
        occ8<I, L>(lay, pr, q_lane, k, l, a, b);
        if (!kl.x) a = Occ4{0, 0, 0, 0};
        if (!ok) {
            a = Occ4{~0u, ~0u, ~0u, ~0u};
            b = a;
        }
        uint32_t *o = out + g * 8;
        if (L == 1) {
            ((uint4 *)o)[0] = make_uint4(a.a, a.c, a.g, a.t);
            ((uint4 *)o)[1] = make_uint4(b.a, b.c, b.g, b.t);
        } else if (L == 2) {
            ((uint4 *)o)[q_lane] = q_lane ? make_uint4(b.a, b.c, b.g, b.t) : make_uint4(a.a, a.c, a.g, a.t);
        } else if (q_lane < 4) {
            const Occ4 s = q_lane < 2 ? a : b;
            ((uint2 *)o)[q_lane] = (q_lane & 1) ? make_uint2(s.g, s.t) : make_uint2(s.a, s.c);
        }
    }
}

template <int I, int L>
static hipError_t occ8_launch(DevLayout lay, const fm_tuning &t, int cus, const fm_interval *q, uint64_t nq,
                              uint32_t *out, hipStream_t s)
{
    const int block = (int)t.block;
    int per = max_blocks_per_cu((const void *)occ8_kernel<I, L>, block, 0);
    uint64_t want = (nq * L + block - 1) / block;
    uint64_t grid = (uint64_t)cus * (per > 0 ? per : 1);
    if (want < grid) grid = want;
    if (grid == 0) grid = 1;
    hipLaunchKernelGGL((occ8_kernel<I, L>), dim3((uint32_t)grid), dim3(block), 0, s, lay, (const uint2 *)q, nq, out);
    return hipGetLastError();
}

template <int I>
static hipError_t occ8_by_lanes(DevLayout lay, const fm_tuning &t, int cus, const fm_interval *q, uint64_t nq,
                                uint32_t *out, hipStream_t s)
{
    switch (t.lanes) {
    case 1: return occ8_launch<I, 1>(lay, t, cus, q, nq, out, s);
    case 2: return occ8_launch<I, 2>(lay, t, cus, q, nq, out, s);
    case 4: if constexpr (Geo<I>::USED > 2) return occ8_launch<I, 4>(lay, t, cus, q, nq, out, s); break;
    case 8: if constexpr (Geo<I>::USED > 4) return occ8_launch<I, 8>(lay, t, cus, q, nq, out, s); break;
    default: break;
    }
    return hipErrorInvalidValue;
}

hipError_t launch_occ8(const fm_index *idx, const fm_tuning &t, const fm_interval *q, uint64_t nq, uint32_t *out,
                       hipStream_t s)
{
    if (!nq) return hipSuccess;
    DevLayout lay = dev_layout(idx, t.occ_interval, false);
    switch (t.occ_interval) {
    case 64: return occ8_by_lanes<64>(lay, t, idx->cu_count, q, nq, out, s);
    case 96: return occ8_by_lanes<96>(lay, t, idx->cu_count, q, nq, out, s);
    case 128: return occ8_by_lanes<128>(lay, t, idx->cu_count, q, nq, out, s);
    case 192: return occ8_by_lanes<192>(lay, t, idx->cu_count, q, nq, out, s);
    case 224: return occ8_by_lanes<224>(lay, t, idx->cu_count, q, nq, out, s);
    case 256: return occ8_by_lanes<256>(lay, t, idx->cu_count, q, nq, out, s);
    case 448: return occ8_by_lanes<448>(lay, t, idx->cu_count, q, nq, out, s);
    default: return hipErrorInvalidValue;
    }
}

// ------------------------------------------------------------------ prefix table

// Level t of the prefix table from level t - 1: each parent string S (level 0: the empty
// string, interval (0, n)) gives its four children b.S by one Occ8 at (k - 1, l), Listing
// 1's update k_b = C[b] + Occ(b, k - 1) + 1, l_b = C[b] + Occ(b, l), with Occ(b, -1) = 0.
// An empty parent (k > l) gives empty children, as Listing 1 keeps them. Children are
// written as 32 bytes at 4 * (parent entry).
template <int I>
__global__ void __launch_bounds__(256) prefix_level(DevLayout lay, const uint2 *parent, uint64_t np, uint4 *child)
{
    const uint64_t p = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x;
    if (p >= np) return;
    const uint2 kl = parent ? parent[p] : make_uint2(0u, lay.n);
    const uint32_t k = kl.x ? kl.x : 1u, l = kl.y;
    Pair<I, 1> pr;
    pr.load(lay, 0, k, l);
    Occ4 a, b;
    occ8<I, 1>(lay, pr, 0, k, l, a, b);
    if (!kl.x) a = Occ4{0, 0, 0, 0};
    const uint32_t C0 = lay.C[0], C1 = lay.C[1], C2 = lay.C[2], C3 = lay.C[3];
    child[2 * p] = make_uint4(C0 + a.a + 1, C0 + b.a, C1 + a.c + 1, C1 + b.c);
    child[2 * p + 1] = make_uint4(C2 + a.g + 1, C2 + b.g, C3 + a.t + 1, C3 + b.t);
}

template <int I>
static hipError_t prefix_table_t(DevLayout lay, uint2 *tab, uint32_t T, hipStream_t s)
{
    for (uint32_t t = 1; t <= T; ++t) {
        const uint64_t np = 1ull << (2 * (t - 1));
        const uint2 *parent = t == 1 ? nullptr : tab + table_level_base(t - 1);
        uint4 *child = (uint4 *)(tab + table_level_base(t));
        hipLaunchKernelGGL(prefix_level<I>, dim3((uint32_t)((np + 255) / 256)), dim3(256), 0, s, lay, parent, np,
                           child);
        if (hipError_t e = hipGetLastError()) return e;
    }
    return hipSuccess;
}

hipError_t build_prefix_table(const fm_index *idx, uint32_t I, hipStream_t s)
{
    if (!idx->ptab || !idx->table_levels) return hipSuccess;
    const DevLayout lay = dev_layout(idx, I, false);
    switch (I) {
    case 64: return prefix_table_t<64>(lay, idx->ptab, idx->table_levels, s);
    case 96: return prefix_table_t<96>(lay, idx->ptab, idx->table_levels, s);
    case 128: return prefix_table_t<128>(lay, idx->ptab, idx->table_levels, s);
    case 192: return prefix_table_t<192>(lay, idx->ptab, idx->table_levels, s);
    case 224: return prefix_table_t<224>(lay, idx->ptab, idx->table_levels, s);
    case 256: return prefix_table_t<256>(lay, idx->ptab, idx->table_levels, s);
    case 448: return prefix_table_t<448>(lay, idx->ptab, idx->table_levels, s);
    default: return hipErrorInvalidValue;
    }
}

// Resident workgroups per CU for a kernel; the runtime query is slow, so each
// (device, kernel, block, LDS) answer is computed once and kept.
int max_blocks_per_cu(const void *kernel, int block, size_t lds)
{
    struct Key {
        int dev;
        const void *k;
        int block;
        size_t lds;
        bool operator==(const Key &o) const { return dev == o.dev && k == o.k && block == o.block && lds == o.lds; }
    };
    struct Hash {
        size_t operator()(const Key &x) const
        {
            return std::hash<const void *>()(x.k) ^ ((size_t)x.block << 20) ^ (x.lds << 32) ^ (size_t)x.dev;
        }
    };
    static std::mutex mu;
    static std::unordered_map<Key, int, Hash> cache;
    int dev = 0;
    (void)hipGetDevice(&dev);
    const Key key{dev, kernel, block, lds};
    {
        std::lock_guard<std::mutex> g(mu);
        auto it = cache.find(key);
        if (it != cache.end()) return it->second;
    }
    int n = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, kernel, block, lds) != hipSuccess || n < 1) n = 1;
    std::lock_guard<std::mutex> g(mu);
    cache[key] = n;
    return n;
}

}  // namespace fm
