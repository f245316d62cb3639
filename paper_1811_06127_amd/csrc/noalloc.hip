// noalloc.hip -- fm_search_inexact_noalloc: the inexact search with its workspace in a
// static device array instead of caller or library allocations, for callers that cannot
// allocate device memory (code under graph capture, tight serving loops).
#include <hip/hip_runtime.h>

#include <mutex>

#include "fm_internal.hpp"

// The workspace of every fm_search_inexact_noalloc call on a device. Host code never
// names it directly: its device address comes from hipGetSymbolAddress, per device.
static __device__ __align__(256) unsigned char scratch[FM_NOALLOC_WS_BYTES];

namespace {

constexpr int kMaxDevices = 64;
std::mutex g_mu;
void *g_ptr[kMaxDevices] = {};

// Device address of `scratch` on device dev, looked up once per device with dev current.
int scratch_on(int dev, void **out)
{
    if (dev < 0 || dev >= kMaxDevices) return FM_EDEVICE;
    std::lock_guard<std::mutex> lk(g_mu);
    if (!g_ptr[dev]) {
        int prev = -1;
        if (hipGetDevice(&prev) != hipSuccess) return FM_EDEVICE;
        if (prev != dev && hipSetDevice(dev) != hipSuccess) return FM_EDEVICE;
        void *p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (prev != dev) (void)hipSetDevice(prev);
        if (e != hipSuccess || !p) return FM_EDEVICE;
        g_ptr[dev] = p;
    }
    *out = g_ptr[dev];
    return FM_OK;
}

__global__ void copy_required(const unsigned long long *src, unsigned long long *dst)
{
    if (threadIdx.x == 0) *dst = *src;
}

}  // namespace

extern "C" int fm_search_inexact_noalloc(const fm_index *idx, const uint8_t *codes, const uint64_t *offs,
                                         const uint8_t *z, uint64_t nreads, uint32_t flags, uint32_t zmax,
                                         fm_hit *hits, uint64_t hit_cap, uint64_t *hit_offs, uint32_t *status,
                                         uint64_t *required, void *stream)
{
    if (!idx || !fm::nstrands_of(flags) || zmax > FM_ZMAX || (flags & FM_STATS)) return FM_EINVAL;
    if (nreads * fm::nstrands_of(flags) >= 0xFFFFFFFFull) return FM_ERANGE;
    const size_t need = fm::inexact_ws_layout(nreads, fm::nstrands_of(flags), zmax, hit_cap).total;
    if (need > (size_t)FM_NOALLOC_WS_BYTES) return FM_ERANGE;
    void *ws = nullptr;
    if (int st = scratch_on(idx->device, &ws)) return st;
    int st = fm_search_inexact(idx, codes, offs, z, nreads, flags, zmax, hits, hit_cap, hit_offs, status, ws,
                               (size_t)FM_NOALLOC_WS_BYTES, stream);
    if (st || !required) return st;
    int prev = -1;
    if (hipGetDevice(&prev) != hipSuccess) return FM_EDEVICE;
    if (prev != idx->device && hipSetDevice(idx->device) != hipSuccess) return FM_EDEVICE;
    hipLaunchKernelGGL(copy_required, dim3(1), dim3(64), 0, (hipStream_t)stream,
                       (const unsigned long long *)((const char *)ws + fm::kWsRequired), (unsigned long long *)required);
    const hipError_t e = hipGetLastError();
    if (prev != idx->device) (void)hipSetDevice(prev);
    return e == hipSuccess ? FM_OK : FM_EDEVICE;
}
