// Suffix sorting and the BWT on the device (Background, Eq. 1-2), for building the index of
// large texts without the host's induced sorting: prefix doubling over radix sorts.
//
// Suffixes of T$ (N = n + 1 of them, '$' smallest) are first sorted by their first 21
// symbols, packed 3 bits each into a 63-bit key ('$' = 0, bases 1..4, nothing after '$'
// matters because '$' occurs once). Suffixes whose key is unique are placed for good. The
// others keep, as rank, the first sorted position of their group; with all suffixes
// ordered by their first L symbols, the pair (rank[i], rank[i + L]) orders them by their
// first 2L symbols, so each round sorts only the open suffixes by that pair, splits their
// groups and doubles L. A suffix still open after sorting by L symbols has no '$' among
// them, so i + L <= n and rank[i + L] exists. Rounds end when every group is a singleton;
// the BWT row j is then T[SA[j] - 1], or '$' where SA[j] = 0 (Eq. 2).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstring>

#include <rocprim/device/device_radix_sort.hpp>
#include <rocprim/device/device_scan.hpp>
#include <rocprim/device/device_select.hpp>
#include <rocprim/functional.hpp>
#include <rocprim/iterator/counting_iterator.hpp>

#include "fm_internal.hpp"

namespace fm {

namespace {

constexpr uint32_t kFirstSymbols = 21;

__device__ __forceinline__ uint64_t gid() { return (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; }
__device__ __forceinline__ uint64_t gstride() { return (uint64_t)gridDim.x * blockDim.x; }

// Symbol p of the text being sorted (text, or its reverse when rev): '$' = 0, A..T = 1..4,
// and 0 past the end.
__device__ __forceinline__ uint64_t sym3(const uint8_t *t, uint64_t n, bool rev, uint64_t p)
{
    return p < n ? 1u + t[rev ? n - 1 - p : p] : 0u;
}

// Symbol counts of the text (cnt[0..3]) and the number of codes above 3 (cnt[4]).
__global__ void __launch_bounds__(256) count_codes(const uint8_t *t, uint64_t n, unsigned long long *cnt)
{
    uint64_t c[5] = {0, 0, 0, 0, 0};
    for (uint64_t i = gid(); i < n; i += gstride()) {
        const uint32_t v = t[i];
        c[v < 4 ? v : 4] += 1;
    }
    for (int b = 0; b < 5; ++b) {
        uint64_t x = c[b];
        for (int d = 32; d >= 1; d >>= 1) x += __shfl_xor(x, d);
        if (__lane_id() == 0 && x) atomicAdd(cnt + b, (unsigned long long)x);
    }
}

__global__ void __launch_bounds__(256) first_keys(const uint8_t *t, uint64_t n, bool rev, uint64_t *keys,
                                                  uint32_t *ids)
{
    const uint64_t N = n + 1;
    for (uint64_t i = gid(); i < N; i += gstride()) {
        uint64_t k = 0;
        for (uint32_t d = 0; d < kFirstSymbols; ++d) k = (k << 3) | sym3(t, n, rev, i + d);
        keys[i] = k;
        ids[i] = (uint32_t)i;
    }
}

// Keys of the open suffixes x[0..U): (rank of the suffix, rank of the suffix L further).
__global__ void __launch_bounds__(256) pair_keys(const uint32_t *x, uint64_t U, const uint32_t *rank, uint64_t L,
                                                 uint64_t *keys, uint32_t *ids)
{
    for (uint64_t e = gid(); e < U; e += gstride()) {
        const uint32_t s = x[e];
        keys[e] = ((uint64_t)rank[s] << 32) | rank[s + L];
        ids[e] = s;
    }
}

// After a sort: the slot of every element that starts a run of equal keys, else 0. The
// slots (sorted positions; slots == nullptr: p itself) increase with p, so an inclusive
// max-scan gives each element the first slot of its group.
__global__ void __launch_bounds__(256) run_starts(const uint64_t *keys, const uint32_t *slots, uint64_t U,
                                                  uint32_t *out)
{
    for (uint64_t p = gid(); p < U; p += gstride()) {
        const uint32_t s = slots ? slots[p] : (uint32_t)p;
        out[p] = (p == 0 || keys[p] != keys[p - 1]) ? s : 0u;
    }
}

// Stores each element at its slot, gives it its group's first slot as rank and flags the
// elements whose group has more than one member.
__global__ void __launch_bounds__(256) settle(const uint32_t *ids, const uint32_t *slots, const uint32_t *head,
                                              uint64_t U, uint32_t *rank, uint32_t *sa, uint8_t *open)
{
    for (uint64_t p = gid(); p < U; p += gstride()) {
        const uint32_t s = slots ? slots[p] : (uint32_t)p;
        const uint32_t x = ids[p];
        const uint32_t h = head[p];
        rank[x] = h;
        sa[s] = x;
        const bool starts = h == s;
        const bool next_starts =
            p + 1 == U || head[p + 1] == (slots ? slots[p + 1] : (uint32_t)(p + 1));
        open[p] = (starts && next_starts) ? 0 : 1;
    }
}

// SA values kept for locating: rows that are multiples of kSaSample.
__global__ void __launch_bounds__(256) take_samples(const uint32_t *sa, uint64_t N, uint32_t *samples)
{
    const uint64_t ns = (N + kSaSample - 1) / kSaSample;
    for (uint64_t j = gid(); j < ns; j += gstride()) samples[j] = sa[j * kSaSample];
}

// 2-bit BWT words (row j at bits 2(j mod 16), '$' stored as 0) and the '$' row.
__global__ void __launch_bounds__(256) pack_bwt(const uint32_t *sa, const uint8_t *t, uint64_t n, bool rev,
                                                uint32_t *words, unsigned long long *dollar)
{
    const uint64_t N = n + 1, nw = (N + 15) / 16;
    for (uint64_t w = gid(); w < nw; w += gstride()) {
        uint32_t v = 0;
        for (uint32_t q = 0; q < 16; ++q) {
            const uint64_t j = w * 16 + q;
            if (j >= N) break;
            const uint64_t s = sa[j];
            uint32_t c = 0;
            if (s == 0)
                *dollar = j;
            else
                c = t[rev ? n - s : s - 1];       // symbol s-1 of the sorted text
            v |= c << (2 * q);
        }
        words[w] = v;
    }
}

struct Buf {
    void *p = nullptr;
    ~Buf()
    {
        if (p) (void)hipFree(p);
    }
    hipError_t alloc(size_t bytes) { return hipMalloc(&p, bytes ? bytes : 16); }
    template <class T> T *as() const { return (T *)p; }
};

#define FM_TRY(x)                                                                                                    \
    do {                                                                                                             \
        const hipError_t e_ = (x);                                                                                   \
        if (e_ != hipSuccess) return e_;                                                                             \
    } while (0)

}  // namespace

hipError_t device_symbol_counts(const uint8_t *text_dev, uint64_t n, uint64_t out[5], int cu_count, hipStream_t s)
{
    Buf cnt;
    FM_TRY(cnt.alloc(5 * sizeof(unsigned long long)));
    FM_TRY(hipMemsetAsync(cnt.p, 0, 5 * sizeof(unsigned long long), s));
    if (n) hipLaunchKernelGGL(count_codes, dim3(cu_count * 8), dim3(256), 0, s, text_dev, n, cnt.as<unsigned long long>());
    FM_TRY(hipGetLastError());
    unsigned long long h[5];
    FM_TRY(hipMemcpyAsync(h, cnt.p, sizeof h, hipMemcpyDeviceToHost, s));
    FM_TRY(hipStreamSynchronize(s));
    for (int b = 0; b < 5; ++b) out[b] = h[b];
    return hipSuccess;
}

size_t device_bwt_bytes(uint64_t n)
{
    const uint64_t N = n + 1;
    return 41 * N;
}

hipError_t device_bwt(const uint8_t *text_dev, uint64_t n, bool rev, uint32_t *words, uint64_t *dollar_row,
                      uint32_t *samples, int cu_count, hipStream_t s)
{
    const uint64_t N = n + 1;
    const dim3 grid(cu_count * 8), block(256);
    Buf K0, K1, I0, I1, SA, R, S0, S1, F, cnt, tmp;
    FM_TRY(K0.alloc(8 * N));
    FM_TRY(K1.alloc(8 * N));
    FM_TRY(I0.alloc(4 * N));
    FM_TRY(I1.alloc(4 * N));
    FM_TRY(SA.alloc(4 * N));
    FM_TRY(R.alloc(4 * N));
    FM_TRY(S0.alloc(4 * N));
    FM_TRY(S1.alloc(4 * N));
    FM_TRY(F.alloc(N));
    FM_TRY(cnt.alloc(16));

    // temporary storage: the largest that the sort, the scan and the selection need at N
    size_t tb = 0, b = 0;
    {
        rocprim::double_buffer<uint64_t> kb(K0.as<uint64_t>(), K1.as<uint64_t>());
        rocprim::double_buffer<uint32_t> ib(I0.as<uint32_t>(), I1.as<uint32_t>());
        FM_TRY(rocprim::radix_sort_pairs(nullptr, b, kb, ib, N, 0, 64, s));
        tb = std::max(tb, b);
        FM_TRY(rocprim::inclusive_scan(nullptr, b, I0.as<uint32_t>(), I1.as<uint32_t>(), N,
                                       rocprim::maximum<uint32_t>(), s));
        tb = std::max(tb, b);
        FM_TRY(rocprim::select(nullptr, b, I0.as<uint32_t>(), F.as<uint8_t>(), I1.as<uint32_t>(),
                               cnt.as<uint64_t>(), N, s));
        tb = std::max(tb, b);
        FM_TRY(rocprim::select(nullptr, b, rocprim::counting_iterator<uint32_t>(0), F.as<uint8_t>(),
                               S0.as<uint32_t>(), cnt.as<uint64_t>(), N, s));
        tb = std::max(tb, b);
    }
    FM_TRY(tmp.alloc(tb));

    uint32_t *rank = R.as<uint32_t>(), *sa = SA.as<uint32_t>();
    uint32_t *slots = S0.as<uint32_t>(), *slots_next = S1.as<uint32_t>();
    uint8_t *open = F.as<uint8_t>();
    uint64_t *ucount = cnt.as<uint64_t>();
    rocprim::double_buffer<uint64_t> kb(K0.as<uint64_t>(), K1.as<uint64_t>());
    rocprim::double_buffer<uint32_t> ib(I0.as<uint32_t>(), I1.as<uint32_t>());

    // first round: every suffix, slots are the sorted positions themselves
    hipLaunchKernelGGL(first_keys, grid, block, 0, s, text_dev, n, rev, kb.current(), ib.current());
    FM_TRY(hipGetLastError());
    size_t bytes = tb;
    FM_TRY(rocprim::radix_sort_pairs(tmp.p, bytes, kb, ib, N, 0, 3 * kFirstSymbols, s));
    uint32_t *starts = (uint32_t *)kb.alternate(), *heads = starts + N;   // the free key buffer holds 8N bytes
    hipLaunchKernelGGL(run_starts, grid, block, 0, s, kb.current(), (const uint32_t *)nullptr, N, starts);
    FM_TRY(hipGetLastError());
    bytes = tb;
    FM_TRY(rocprim::inclusive_scan(tmp.p, bytes, starts, heads, N, rocprim::maximum<uint32_t>(), s));
    hipLaunchKernelGGL(settle, grid, block, 0, s, ib.current(), (const uint32_t *)nullptr, heads, N, rank, sa, open);
    FM_TRY(hipGetLastError());
    bytes = tb;
    FM_TRY(rocprim::select(tmp.p, bytes, rocprim::counting_iterator<uint32_t>(0), open, slots, ucount, N, s));
    bytes = tb;
    FM_TRY(rocprim::select(tmp.p, bytes, ib.current(), open, ib.alternate(), ucount, N, s));
    ib.swap();                                   // current: the open suffixes, in slot order
    uint64_t U = 0;
    FM_TRY(hipMemcpyAsync(&U, ucount, sizeof U, hipMemcpyDeviceToHost, s));
    FM_TRY(hipStreamSynchronize(s));

    for (uint64_t L = kFirstSymbols; U > 0; L *= 2) {
        if (L > N) return hipErrorUnknown;       // cannot happen: a group of L > n equal prefixes
        hipLaunchKernelGGL(pair_keys, grid, block, 0, s, ib.current(), U, rank, L, kb.current(), ib.alternate());
        FM_TRY(hipGetLastError());
        ib.swap();                               // current: ids to sort; alternate: free
        bytes = tb;
        FM_TRY(rocprim::radix_sort_pairs(tmp.p, bytes, kb, ib, U, 0, 64, s));
        starts = (uint32_t *)kb.alternate();
        heads = starts + U;
        hipLaunchKernelGGL(run_starts, grid, block, 0, s, kb.current(), slots, U, starts);
        FM_TRY(hipGetLastError());
        bytes = tb;
        FM_TRY(rocprim::inclusive_scan(tmp.p, bytes, starts, heads, U, rocprim::maximum<uint32_t>(), s));
        hipLaunchKernelGGL(settle, grid, block, 0, s, ib.current(), slots, heads, U, rank, sa, open);
        FM_TRY(hipGetLastError());
        bytes = tb;
        FM_TRY(rocprim::select(tmp.p, bytes, slots, open, slots_next, ucount, U, s));
        bytes = tb;
        FM_TRY(rocprim::select(tmp.p, bytes, ib.current(), open, ib.alternate(), ucount, U, s));
        ib.swap();
        std::swap(slots, slots_next);
        FM_TRY(hipMemcpyAsync(&U, ucount, sizeof U, hipMemcpyDeviceToHost, s));
        FM_TRY(hipStreamSynchronize(s));
    }

    if (samples) {
        hipLaunchKernelGGL(take_samples, grid, block, 0, s, (const uint32_t *)sa, N, samples);
        FM_TRY(hipGetLastError());
    }
    Buf dl;
    FM_TRY(dl.alloc(sizeof(unsigned long long)));
    hipLaunchKernelGGL(pack_bwt, grid, block, 0, s, (const uint32_t *)sa, text_dev, n, rev, words,
                       dl.as<unsigned long long>());
    FM_TRY(hipGetLastError());
    unsigned long long d = 0;
    FM_TRY(hipMemcpyAsync(&d, dl.p, sizeof d, hipMemcpyDeviceToHost, s));
    FM_TRY(hipStreamSynchronize(s));
    *dollar_row = d;
    return hipSuccess;
}

}  // namespace fm
