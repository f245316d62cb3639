// server.cpp -- the request server of the C ABI (fm_server_*): the scheduling of
// server_core.hpp driven by a HIP executor, one non-blocking stream and completion event
// per lane, lane memory in device memory with a pinned host mirror, the symbol ring in
// pinned host memory, and fm_search_inexact as the search.
#include "fm_internal.hpp"
#include "server_core.hpp"

namespace {

int hip_err(hipError_t e) { return e == hipSuccess ? FM_OK : (e == hipErrorOutOfMemory ? FM_ENOMEM : FM_EDEVICE); }

struct DeviceScope {      // makes a device current for a scope, then restores the previous one
    int prev = -1;
    explicit DeviceScope(int dev)
    {
        if (hipGetDevice(&prev) != hipSuccess) prev = -1;
        if (prev != dev) (void)hipSetDevice(dev);
    }
    ~DeviceScope()
    {
        int cur = -1;
        if (prev >= 0 && hipGetDevice(&cur) == hipSuccess && cur != prev) (void)hipSetDevice(prev);
    }
};

// Writes every page of freshly pinned host memory once, on several threads: the first
// write to each page is a fault that runs about ten times slower than the copies that
// follow, and those copies are on the submission path.
void prefault(uint8_t *p, size_t bytes)
{
    const unsigned nt = std::max(1u, std::min(8u, std::thread::hardware_concurrency()));
    const size_t part = (bytes / nt + 4095) & ~(size_t)4095;
    std::vector<std::thread> th;
    for (unsigned t = 0; t < nt; ++t) {
        const size_t a = (size_t)t * part;
        if (a >= bytes) break;
        const size_t len = std::min(part, bytes - a);
        th.emplace_back([p, a, len] { std::memset(p + a, 0, len); });
    }
    for (auto &x : th) x.join();
}

struct HipExec {
    static constexpr size_t kRequiredAt = fm::kWsRequired;

    const fm_index *idx = nullptr;
    uint32_t flags = 0, zmax = 0;

    struct Lane {
        hipStream_t stream = nullptr;
        hipEvent_t ev = nullptr;
        uint8_t *dev = nullptr, *host = nullptr;   // lane memory and its pinned host mirror
        uint8_t *xdev = nullptr, *xhost = nullptr; // larger buffers for a batch whose hits outgrew the lane
        size_t xbytes = 0;
    };

    static size_t ws_bytes(uint64_t n, uint32_t strands, uint32_t zmax, uint64_t hit_cap)
    {
        return fm::inexact_ws_layout(n, strands, zmax, hit_cap).total;
    }

    int open(Lane &L, size_t bytes)
    {
        DeviceScope g(idx->device);
        if (hipStreamCreateWithFlags(&L.stream, hipStreamNonBlocking) != hipSuccess ||
            hipEventCreateWithFlags(&L.ev, hipEventDisableTiming) != hipSuccess)
            return FM_EDEVICE;
        if (hipMalloc((void **)&L.dev, bytes) != hipSuccess ||
            hipHostMalloc((void **)&L.host, bytes, hipHostMallocDefault) != hipSuccess)
            return FM_ENOMEM;
        try {
            prefault(L.host, bytes);
        } catch (...) {
            return FM_ENOMEM;
        }
        return FM_OK;
    }

    int grow(Lane &L, size_t bytes)
    {
        if (L.xbytes >= bytes) return FM_OK;
        DeviceScope g(idx->device);
        if (L.xdev) (void)hipFree(L.xdev);
        if (L.xhost) (void)hipHostFree(L.xhost);
        L.xdev = L.xhost = nullptr;
        L.xbytes = 0;
        if (hipMalloc((void **)&L.xdev, bytes) != hipSuccess) return FM_ENOMEM;
        if (hipHostMalloc((void **)&L.xhost, bytes, hipHostMallocDefault) != hipSuccess) return FM_ENOMEM;
        L.xbytes = bytes;
        return FM_OK;
    }

    void close(Lane &L)
    {
        DeviceScope g(idx->device);
        if (L.stream) (void)hipStreamSynchronize(L.stream);
        if (L.ev) (void)hipEventDestroy(L.ev);
        if (L.stream) (void)hipStreamDestroy(L.stream);
        if (L.dev) (void)hipFree(L.dev);
        if (L.host) (void)hipHostFree(L.host);
        if (L.xdev) (void)hipFree(L.xdev);
        if (L.xhost) (void)hipHostFree(L.xhost);
        L = Lane();
    }

    uint8_t *dev(Lane &L, bool big) { return big ? L.xdev : L.dev; }
    uint8_t *host(Lane &L, bool big) { return big ? L.xhost : L.host; }

    int h2d(Lane &L, void *dst, const void *src, size_t n)
    {
        return hip_err(hipMemcpyAsync(dst, src, n, hipMemcpyHostToDevice, L.stream));
    }
    int d2h(Lane &L, void *dst, const void *src, size_t n)
    {
        return hip_err(hipMemcpyAsync(dst, src, n, hipMemcpyDeviceToHost, L.stream));
    }
    int d2d(Lane &L, void *dst, const void *src, size_t n)
    {
        return hip_err(hipMemcpyAsync(dst, src, n, hipMemcpyDeviceToDevice, L.stream));
    }

    int search(Lane &L, uint8_t *d, const fm::srv::BatchLayout &B, uint64_t n)
    {
        return fm_search_inexact(idx, d + B.codes, (const uint64_t *)(d + B.offs), d + B.z, n, flags, zmax,
                                 (fm_hit *)(d + B.hits), B.hit_cap, (uint64_t *)(d + B.hit_offs),
                                 (uint32_t *)(d + B.status), d + B.ws, B.ws_bytes, L.stream);
    }

    int mark(Lane &L) { return hip_err(hipEventRecord(L.ev, L.stream)); }

    int poll(Lane &L)
    {
        const hipError_t q = hipEventQuery(L.ev);
        if (q == hipErrorNotReady) return FM_EAGAIN;
        return q == hipSuccess ? FM_OK : FM_EDEVICE;
    }

    int alloc_ring(uint8_t **p, size_t bytes)
    {
        DeviceScope g(idx->device);
        if (hipHostMalloc((void **)p, bytes, hipHostMallocDefault) != hipSuccess) {
            *p = nullptr;
            return FM_ENOMEM;
        }
        try {
            prefault(*p, bytes);
        } catch (...) {
            return FM_ENOMEM;
        }
        return FM_OK;
    }

    void free_ring(uint8_t *p)
    {
        DeviceScope g(idx->device);
        (void)hipHostFree(p);
    }

    void bind() { (void)hipSetDevice(idx->device); }
};

using HipServer = fm::srv::Server<HipExec>;

}  // namespace

struct fm_server : HipServer {
    explicit fm_server(HipExec &&x) : HipServer(std::move(x)) {}
};

extern "C" {

int fm_server_bytes(const fm_server_opts *opts, uint64_t nreads, uint64_t total_len, uint64_t *bytes)
{
    if (!fm::srv::valid_opts(opts) || !bytes) return FM_EINVAL;
    *bytes = HipServer::batch_bytes(*opts, nreads, total_len);
    return FM_OK;
}

int fm_server_create(const fm_index *idx, const fm_server_opts *opts, fm_server **out)
{
    if (!out) return FM_EINVAL;
    *out = nullptr;
    if (!idx || !fm::srv::valid_opts(opts)) return FM_EINVAL;
    if ((opts->flags & FM_DARRAY) && !idx->has_rev) return FM_EINVAL;
    HipExec x;
    x.idx = idx;
    x.flags = opts->flags;
    x.zmax = opts->zmax;
    fm_server *s = new (std::nothrow) fm_server(std::move(x));
    if (!s) return FM_ENOMEM;
    const int e = s->start(*opts);
    if (e != FM_OK) {
        delete s;
        return e;
    }
    *out = s;
    return FM_OK;
}

int fm_server_submit(fm_server *s, const uint8_t *codes, const uint64_t *offs, const uint8_t *z, uint64_t nreads,
                     uint64_t *ticket)
{
    if (!s) return FM_EINVAL;
    return s->submit(codes, offs, z, nreads, ticket);
}

int fm_server_wait(fm_server *s, uint64_t ticket, double timeout_s, fm_result *out)
{
    if (!s) return FM_EINVAL;
    return s->wait(ticket, timeout_s, out);
}

int fm_server_release(fm_server *s, uint64_t ticket)
{
    if (!s) return FM_EINVAL;
    return s->release(ticket);
}

double fm_server_clock(const fm_server *s) { return s ? s->now() : 0.0; }

int fm_server_stats(fm_server *s, fm_server_counts *out)
{
    if (!s || !out) return FM_EINVAL;
    s->stats(out);
    return FM_OK;
}

void fm_server_free(fm_server *s) { delete s; }

}  // extern "C"
