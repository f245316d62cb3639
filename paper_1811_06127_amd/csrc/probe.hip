// probe.hip -- fm_probe_random_reads: the rate at which the device serves independent
// reads of random 32-byte blocks of a span of memory. Every Occ8 of the searches reads
// one or two random 32-byte buckets of the index (I=64), so this rate, measured over a
// span about the size of the index, is the ceiling those kernels can reach with the
// index they read; the 8 TB/s of streaming HBM reads is not.
#include <hip/hip_runtime.h>

#include "fm_internal.hpp"

namespace {

constexpr uint32_t kProbeWaves = 16;   // waves per CU: the rate saturates from about 8
constexpr uint32_t kProbeDepth = 4;    // reads in flight per lane

// SplitMix64's output function: spreads the block numbers over the whole span.
__device__ __forceinline__ uint64_t probe_mix(uint64_t x)
{
    x ^= x >> 30;
    x *= 0xBF58476D1CE4E5B9ull;
    x ^= x >> 27;
    x *= 0x94D049BB133111EBull;
    return x ^ (x >> 31);
}

// Each lane makes `rounds` rounds of kProbeDepth independent reads, each of one random
// 32-byte block (two 16-byte loads); block b of round r and slot u is a hash of the lane,
// r, u and the seed, masked to the span (a power of two), so every read is in bounds.
// The sum of the loaded words decides whether the one-word sink is written, which keeps
// every load live.
__global__ void __launch_bounds__(256) random_reads(const uint4 *buf, uint64_t block_mask, uint32_t rounds,
                                                    uint64_t seed, uint32_t *sink)
{
    const uint64_t t = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x;
    const uint64_t base = seed ^ (t * 0x9E3779B97F4A7C15ull);
    uint32_t acc = 0;
    for (uint32_t r = 0; r < rounds; ++r) {
        uint4 v[kProbeDepth][2];
#pragma unroll
        for (uint32_t u = 0; u < kProbeDepth; ++u) {
            const uint64_t b = probe_mix(base + ((uint64_t)(r * kProbeDepth + u) << 32)) & block_mask;
            v[u][0] = buf[2 * b];
            v[u][1] = buf[2 * b + 1];
        }
#pragma unroll
        for (uint32_t u = 0; u < kProbeDepth; ++u) acc += v[u][0].x ^ v[u][1].w;
    }
    if (acc == 0x5EEDF00Du) sink[0] = acc;
}

}  // namespace

extern "C" int fm_probe_random_reads(const fm_index *idx, const void *buf, uint64_t span, uint32_t rounds,
                                     uint32_t *sink, uint64_t *reads, void *stream)
{
    if (!idx || !buf || !sink || !reads || rounds == 0 || rounds > 4096) return FM_EINVAL;
    if (span < 4096 || (span & (span - 1)) || ((uintptr_t)buf & 15u)) return FM_EINVAL;
    int prev = -1;
    if (hipGetDevice(&prev) != hipSuccess) return FM_EDEVICE;
    if (prev != idx->device && hipSetDevice(idx->device) != hipSuccess) return FM_EDEVICE;
    const uint64_t threads = (uint64_t)idx->cu_count * kProbeWaves * 64;
    const uint64_t seed = 0x243F6A8885A308D3ull ^ (uint64_t)span ^ ((uint64_t)rounds << 40);
    hipLaunchKernelGGL(random_reads, dim3((uint32_t)(threads / 256)), dim3(256), 0, (hipStream_t)stream,
                       (const uint4 *)buf, span / 32 - 1, rounds, seed, sink);
    const hipError_t e = hipGetLastError();
    if (prev != idx->device) (void)hipSetDevice(prev);
    if (e != hipSuccess) return FM_EDEVICE;
    *reads = threads * rounds * kProbeDepth;
    return FM_OK;
}
