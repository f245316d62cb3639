// server.cpp -- a request server over the inexact search with continuous batching.
//
// Requests (reads with per-read budgets) are queued in arrival order; their symbols are
// copied once, at submission, into a ring of pinned host memory. A worker thread keeps
// up to `lanes` batches in flight, each on a stream of its own with a fixed share of a
// device arena: whenever a lane is idle it admits queued requests, oldest first, while
// the batch still fits the lane's memory (and the read cap), uploads their symbols
// straight from the ring and their offsets and budgets from the lane's pinned mirror,
// runs the search and brings back status and hit offsets, then the hits. Requests that arrive while batches run join the next batch of whichever lane
// frees up first, so their work overlaps with the batches already on the device.
// Every read is searched independently of its batch, so a request's result does not
// depend on what it was batched with.
#include "fm_internal.hpp"

#include <algorithm>
#include <chrono>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <memory>
#include <mutex>
#include <new>
#include <thread>
#include <unordered_map>
#include <vector>

namespace {

using Clock = std::chrono::steady_clock;

size_t al256(size_t x) { return (x + 255) & ~(size_t)255; }

uint32_t strands_of(uint32_t flags) { return ((flags & FM_FWD) ? 1u : 0u) + ((flags & FM_REVCOMP) ? 1u : 0u); }

// Byte offsets of one batch's buffers inside a lane's memory. The inputs come first
// (one upload covers [0, status)); status, hit offsets and the workspace header
// follow (one download covers [status, ws + 16)); the hits come last.
struct BatchLayout {
    size_t codes, offs, z, status, hit_offs, ws, hits, end, ws_bytes;
    uint64_t hit_cap;
};

BatchLayout batch_layout(const fm_server_opts &o, uint64_t n, uint64_t total_len, uint64_t hit_cap)
{
    BatchLayout L;
    const size_t ws = fm::inexact_ws_layout(n, strands_of(o.flags), o.zmax, hit_cap).total;
    size_t p = 0;
    L.codes = p;    p = al256(p + total_len);
    L.offs = p;     p = al256(p + 8 * (n + 1));
    L.z = p;        p = al256(p + n);
    L.status = p;   p = al256(p + 4 * n);
    L.hit_offs = p; p = al256(p + 8 * (n + 1));
    L.ws = p;       p = al256(p + ws);
    L.hits = p;     p = al256(p + 16 * hit_cap);
    L.end = p;
    L.ws_bytes = ws;
    L.hit_cap = hit_cap;
    return L;
}

uint64_t reserve_of(const fm_server_opts &o, uint64_t n) { return (uint64_t)o.hit_reserve * n * strands_of(o.flags); }

struct Req {
    uint64_t ticket = 0;
    uint64_t rv = 0, len = 0;       // symbols: ring bytes [rv, rv + len) (positions grow without wrapping)
    bool ring_free = false;         // the symbols have been uploaded; their ring space may be reused
    std::vector<uint64_t> offs;     // request-local, offs[0] = 0
    std::vector<uint8_t> z;
    uint64_t nreads = 0;
    std::vector<fm_hit> hits;
    std::vector<uint64_t> hit_offs;
    std::vector<uint32_t> status;
    int error = FM_OK;
    double t_submit = 0, t_launch = 0, t_done = 0;
    uint64_t batch = 0;
    bool done = false;
};

struct Lane {
    hipStream_t stream = nullptr;
    hipEvent_t ev = nullptr;
    uint8_t *dev = nullptr, *host = nullptr;   // lane memory and its pinned host mirror
    size_t bytes = 0;
    uint8_t *xdev = nullptr, *xhost = nullptr; // larger buffers for a batch whose hits outgrew the lane
    size_t xbytes = 0;
    int stage = 0;                             // 0 idle, 1 search in flight, 2 hit copy in flight
    bool big = false;                          // the batch runs in the x buffers
    std::vector<std::shared_ptr<Req>> reqs;
    uint64_t n = 0, total_len = 0, batch = 0;
    BatchLayout lay{};
    uint8_t *d() const { return big ? xdev : dev; }
    uint8_t *h() const { return big ? xhost : host; }
};

}  // namespace

struct fm_server {
    const fm_index *idx = nullptr;
    fm_server_opts o{};
    std::vector<Lane> lanes;
    std::mutex mu;
    std::condition_variable cv_submit, cv_done, cv_space;
    // pinned ring for the symbols of queued and in-flight requests: [ring_tail, ring_head)
    // of a position space that only grows; a position p lives at ring[p % ring_bytes]
    uint8_t *ring = nullptr;
    uint64_t ring_bytes = 0, ring_head = 0, ring_tail = 0;
    std::deque<std::shared_ptr<Req>> ring_order;   // requests holding ring space, oldest first
    std::deque<std::shared_ptr<Req>> pending;
    std::unordered_map<uint64_t, std::shared_ptr<Req>> table;
    uint64_t next_ticket = 1, batches = 0, retries = 0, reads_done = 0, requests_done = 0;
    bool stop = false;
    int fatal = FM_OK;
    Clock::time_point t0;
    std::thread worker;

    double now() const { return std::chrono::duration<double>(Clock::now() - t0).count(); }
};

namespace {

// Returns the ring space of the batch's requests (caller holds s->mu): space is reused
// oldest first, so the tail moves past every request released so far in order.
void release_ring(fm_server *s, Lane &ln)
{
    for (auto &r : ln.reqs) r->ring_free = true;
    while (!s->ring_order.empty() && s->ring_order.front()->ring_free) s->ring_order.pop_front();
    s->ring_tail = s->ring_order.empty() ? s->ring_head : s->ring_order.front()->rv;
    s->cv_space.notify_all();
}

// Ends every request of the lane's batch with `err` (device failure).
void fail_batch(fm_server *s, Lane &ln, int err)
{
    std::lock_guard<std::mutex> lk(s->mu);
    release_ring(s, ln);
    const double t = s->now();
    for (auto &r : ln.reqs) {
        r->error = err;
        r->done = true;
        r->t_done = t;
        ++s->requests_done;
    }
    if (s->fatal == FM_OK) s->fatal = err;
    ln.reqs.clear();
    ln.stage = 0;
    ln.big = false;
    s->cv_done.notify_all();
}

int hip_err(hipError_t e) { return e == hipSuccess ? FM_OK : (e == hipErrorOutOfMemory ? FM_ENOMEM : FM_EDEVICE); }

// Enqueues the search of the lane's batch (inputs already on the device at lay's
// offsets of d()), the download of status, hit offsets and the workspace header, and
// the completion event.
int enqueue_search(fm_server *s, Lane &ln)
{
    uint8_t *d = ln.d();
    const BatchLayout &L = ln.lay;
    int e = fm_search_inexact(s->idx, d + L.codes, (const uint64_t *)(d + L.offs), d + L.z, ln.n, s->o.flags,
                              s->o.zmax, (fm_hit *)(d + L.hits), L.hit_cap, (uint64_t *)(d + L.hit_offs),
                              (uint32_t *)(d + L.status), d + L.ws, L.ws_bytes, ln.stream);
    if (e != FM_OK) return e;
    if (hipError_t he = hipMemcpyAsync(ln.h() + L.status, d + L.status, L.ws + 16 - L.status, hipMemcpyDeviceToHost,
                                       ln.stream))
        return hip_err(he);
    return hip_err(hipEventRecord(ln.ev, ln.stream));
}

// Admits queued requests into an idle lane and launches the batch. Returns true if a
// batch was launched.
bool admit(fm_server *s, Lane &ln)
{
    std::vector<std::shared_ptr<Req>> take;
    uint64_t n = 0, len = 0;
    {
        std::lock_guard<std::mutex> lk(s->mu);
        while (!s->pending.empty()) {
            const auto &r = s->pending.front();
            const uint64_t n2 = n + r->nreads, len2 = len + r->len;
            if (!take.empty()) {
                if (s->o.max_batch_reads && n2 > s->o.max_batch_reads) break;
                if (batch_layout(s->o, n2, len2, reserve_of(s->o, n2)).end > ln.bytes) break;
            }
            take.push_back(r);
            s->pending.pop_front();
            n = n2;
            len = len2;
        }
        if (take.empty()) return false;
        ln.batch = ++s->batches;
    }
    ln.reqs = std::move(take);
    ln.n = n;
    ln.total_len = len;
    ln.big = false;
    ln.lay = batch_layout(s->o, n, len, reserve_of(s->o, n));
    // offsets and budgets go through the pinned mirror, in the device layout; the symbols
    // are uploaded straight from the ring, one copy per run of adjacent requests
    uint8_t *h = ln.host;
    uint64_t *offs = (uint64_t *)(h + ln.lay.offs);
    uint64_t rbase = 0, cbase = 0;
    offs[0] = 0;
    int e = FM_OK;
    uint64_t run_src = 0, run_dst = 0, run_len = 0;
    auto flush = [&]() {
        if (run_len && e == FM_OK)
            e = hip_err(hipMemcpyAsync(ln.dev + ln.lay.codes + run_dst, s->ring + run_src, run_len,
                                       hipMemcpyHostToDevice, ln.stream));
        run_len = 0;
    };
    for (auto &r : ln.reqs) {
        if (r->nreads) std::memcpy(h + ln.lay.z + rbase, r->z.data(), r->nreads);
        for (uint64_t i = 1; i <= r->nreads; ++i) offs[rbase + i] = cbase + r->offs[i];
        if (r->len) {
            const uint64_t src = r->rv % s->ring_bytes;
            if (run_len && run_src + run_len == src) {
                run_len += r->len;
            } else {
                flush();
                run_src = src;
                run_dst = cbase;
                run_len = r->len;
            }
        }
        rbase += r->nreads;
        cbase += r->len;
    }
    flush();
    const double t = s->now();
    for (auto &r : ln.reqs) {
        r->t_launch = t;
        r->batch = ln.batch;
    }
    if (e == FM_OK)
        e = hip_err(hipMemcpyAsync(ln.dev + ln.lay.offs, h + ln.lay.offs, ln.lay.status - ln.lay.offs,
                                   hipMemcpyHostToDevice, ln.stream));
    if (e == FM_OK) e = enqueue_search(s, ln);
    if (e != FM_OK) {
        fail_batch(s, ln, e);
        return true;
    }
    ln.stage = 1;
    return true;
}

// Grows the lane's retry buffers to `bytes`.
int ensure_x(Lane &ln, size_t bytes)
{
    if (ln.xbytes >= bytes) return FM_OK;
    if (ln.xdev) (void)hipFree(ln.xdev);
    if (ln.xhost) (void)hipHostFree(ln.xhost);
    ln.xdev = ln.xhost = nullptr;
    ln.xbytes = 0;
    if (hipMalloc((void **)&ln.xdev, bytes) != hipSuccess) return FM_ENOMEM;
    if (hipHostMalloc((void **)&ln.xhost, bytes, hipHostMallocDefault) != hipSuccess) return FM_ENOMEM;
    ln.xbytes = bytes;
    return FM_OK;
}

// Hands each request of the finished batch its share of the results.
void distribute(fm_server *s, Lane &ln)
{
    const uint8_t *h = ln.h();
    const fm_hit *H = (const fm_hit *)(h + ln.lay.hits);
    const uint64_t *HO = (const uint64_t *)(h + ln.lay.hit_offs);
    const uint32_t *ST = (const uint32_t *)(h + ln.lay.status);
    uint64_t rb = 0;
    for (auto &r : ln.reqs) {
        const uint64_t lo = HO[rb], hi = HO[rb + r->nreads];
        r->hit_offs.resize(r->nreads + 1);
        for (uint64_t i = 0; i <= r->nreads; ++i) r->hit_offs[i] = HO[rb + i] - lo;
        r->status.assign(ST + rb, ST + rb + r->nreads);
        r->hits.assign(H + lo, H + hi);
        for (auto &x : r->hits) x.read -= (uint32_t)rb;
        rb += r->nreads;
    }
    std::lock_guard<std::mutex> lk(s->mu);
    const double t = s->now();
    for (auto &r : ln.reqs) {
        r->done = true;
        r->t_done = t;
        s->reads_done += r->nreads;
        ++s->requests_done;
    }
    ln.reqs.clear();
    ln.stage = 0;
    ln.big = false;
    s->cv_done.notify_all();
}

// Moves a busy lane forward when its last enqueued event has completed. Returns true
// on progress.
bool advance(fm_server *s, Lane &ln)
{
    if (ln.stage == 0) return false;
    const hipError_t q = hipEventQuery(ln.ev);
    if (q == hipErrorNotReady) return false;
    if (q != hipSuccess) {
        fail_batch(s, ln, FM_EDEVICE);
        return true;
    }
    if (ln.stage == 2) {
        distribute(s, ln);
        return true;
    }
    {
        // the uploads of this batch are complete: its ring space may be reused
        std::lock_guard<std::mutex> lk(s->mu);
        release_ring(s, ln);
    }
    const uint8_t *h = ln.h();
    const uint64_t required = *(const uint64_t *)(h + ln.lay.ws + fm::kWsRequired);
    if (required > ln.lay.hit_cap) {
        // some reads' hits did not fit: search the batch again with room for all
        BatchLayout L2 = batch_layout(s->o, ln.n, ln.total_len, required);
        int e = FM_OK;
        if (L2.end > ln.bytes) {
            e = ensure_x(ln, L2.end);
            if (e == FM_OK && !ln.big)
                e = hip_err(hipMemcpyAsync(ln.xdev, ln.dev, L2.status, hipMemcpyDeviceToDevice, ln.stream));
            if (e == FM_OK) ln.big = true;
        }
        if (e == FM_OK) {
            ln.lay = L2;
            e = enqueue_search(s, ln);
        }
        if (e != FM_OK) {
            fail_batch(s, ln, e);
            return true;
        }
        std::lock_guard<std::mutex> lk(s->mu);
        ++s->retries;
        return true;
    }
    const uint64_t total = ((const uint64_t *)(h + ln.lay.hit_offs))[ln.n];
    if (total == 0) {
        distribute(s, ln);
        return true;
    }
    int e = hip_err(hipMemcpyAsync(ln.h() + ln.lay.hits, ln.d() + ln.lay.hits, 16 * total, hipMemcpyDeviceToHost,
                                   ln.stream));
    if (e == FM_OK) e = hip_err(hipEventRecord(ln.ev, ln.stream));
    if (e != FM_OK) {
        fail_batch(s, ln, e);
        return true;
    }
    ln.stage = 2;
    return true;
}

void run(fm_server *s)
{
    (void)hipSetDevice(s->idx->device);
    for (;;) {
        bool progress = false;
        for (auto &ln : s->lanes) progress |= advance(s, ln);
        for (auto &ln : s->lanes)
            if (ln.stage == 0) progress |= admit(s, ln);
        if (progress) continue;
        bool busy = false;
        for (auto &ln : s->lanes) busy |= ln.stage != 0;
        std::unique_lock<std::mutex> lk(s->mu);
        if (!busy && s->pending.empty()) {
            if (s->stop) break;
            s->cv_submit.wait(lk, [&] { return s->stop || !s->pending.empty(); });
        } else if (busy) {
            // batches on the device: poll their events at a fine grain
            lk.unlock();
            std::this_thread::sleep_for(std::chrono::microseconds(20));
        }
    }
}

void free_lanes(fm_server *s)
{
    for (auto &ln : s->lanes) {
        if (ln.stream) (void)hipStreamSynchronize(ln.stream);
        if (ln.ev) (void)hipEventDestroy(ln.ev);
        if (ln.stream) (void)hipStreamDestroy(ln.stream);
        if (ln.dev) (void)hipFree(ln.dev);
        if (ln.host) (void)hipHostFree(ln.host);
        if (ln.xdev) (void)hipFree(ln.xdev);
        if (ln.xhost) (void)hipHostFree(ln.xhost);
    }
    s->lanes.clear();
    if (s->ring) (void)hipHostFree(s->ring);
    s->ring = nullptr;
}

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

bool valid_opts(const fm_server_opts *o)
{
    return o && o->lanes >= 1 && o->lanes <= 8 && strands_of(o->flags) && o->zmax <= FM_ZMAX &&
           (o->flags & ~(uint32_t)(FM_BOTH | FM_DARRAY)) == 0 && o->arena_bytes >= o->lanes;
}

}  // namespace

extern "C" {

int fm_server_bytes(const fm_server_opts *opts, uint64_t nreads, uint64_t total_len, uint64_t *bytes)
{
    if (!valid_opts(opts) || !bytes) return FM_EINVAL;
    *bytes = batch_layout(*opts, nreads, total_len, reserve_of(*opts, nreads)).end;
    return FM_OK;
}

int fm_server_create(const fm_index *idx, const fm_server_opts *opts, fm_server **out)
{
    if (!out) return FM_EINVAL;
    *out = nullptr;
    if (!idx || !valid_opts(opts)) return FM_EINVAL;
    if ((opts->flags & FM_DARRAY) && !idx->has_rev) return FM_EINVAL;
    fm_server *s = new (std::nothrow) fm_server;
    if (!s) return FM_ENOMEM;
    s->idx = idx;
    s->o = *opts;
    s->t0 = Clock::now();
    int prev = -1;
    (void)hipGetDevice(&prev);
    (void)hipSetDevice(idx->device);
    int e = FM_OK;
    try {
        s->lanes.resize(opts->lanes);
    } catch (const std::bad_alloc &) {
        e = FM_ENOMEM;
    }
    const size_t per = (size_t)(opts->arena_bytes / opts->lanes) & ~(size_t)255;
    s->ring_bytes = opts->ring_bytes ? opts->ring_bytes : opts->arena_bytes;
    if (hipHostMalloc((void **)&s->ring, s->ring_bytes, hipHostMallocDefault) != hipSuccess) e = FM_ENOMEM;
    for (auto &ln : s->lanes) {
        if (e != FM_OK) break;
        ln.bytes = per;
        if (hipStreamCreateWithFlags(&ln.stream, hipStreamNonBlocking) != hipSuccess ||
            hipEventCreateWithFlags(&ln.ev, hipEventDisableTiming) != hipSuccess)
            e = FM_EDEVICE;
        else if (hipMalloc((void **)&ln.dev, per) != hipSuccess ||
                 hipHostMalloc((void **)&ln.host, per, hipHostMallocDefault) != hipSuccess)
            e = FM_ENOMEM;
    }
    if (prev >= 0) (void)hipSetDevice(prev);
    if (e != FM_OK) {
        free_lanes(s);
        delete s;
        return e;
    }
    try {
        prefault(s->ring, s->ring_bytes);
        for (auto &ln : s->lanes) prefault(ln.host, ln.bytes);
        s->worker = std::thread(run, s);
    } catch (...) {
        free_lanes(s);
        delete s;
        return FM_ENOMEM;
    }
    *out = s;
    return FM_OK;
}

int fm_server_submit(fm_server *s, const uint8_t *codes, const uint64_t *offs, const uint8_t *z, uint64_t nreads,
                     uint64_t *ticket)
{
    if (!s || !ticket || !offs || (nreads && !z)) return FM_EINVAL;
    const double t_call = s->now();                // latency counts any wait for ring space
    const uint64_t base = offs[0], len = offs[nreads] - base;
    if (offs[nreads] < base || (len && !codes)) return FM_EINVAL;
    for (uint64_t i = 0; i < nreads; ++i)
        if (offs[i + 1] < offs[i]) return FM_EINVAL;
    if (nreads * strands_of(s->o.flags) >= 0xFFFFFFFFull) return FM_ERANGE;
    if (batch_layout(s->o, nreads, len, reserve_of(s->o, nreads)).end > s->lanes[0].bytes) return FM_ERANGE;
    if (len > s->ring_bytes) return FM_ERANGE;
    auto r = std::make_shared<Req>();
    try {
        r->offs.resize(nreads + 1);
        for (uint64_t i = 0; i <= nreads; ++i) r->offs[i] = offs[i] - base;
        r->z.assign(z, z + nreads);
    } catch (const std::bad_alloc &) {
        return FM_ENOMEM;
    }
    r->nreads = nreads;
    r->len = len;
    std::unique_lock<std::mutex> lk(s->mu);
    // reserve ring space (a request is never split across the end of the ring), waiting
    // for older requests' uploads when the ring is full
    for (;;) {
        if (s->stop) return FM_EINVAL;
        if (s->ring_order.empty()) {                 // empty ring: restart at its beginning
            s->ring_head = s->ring_tail = (s->ring_head + s->ring_bytes - 1) / s->ring_bytes * s->ring_bytes;
        }
        uint64_t start = s->ring_head;
        const uint64_t phys = start % s->ring_bytes;
        if (len && phys + len > s->ring_bytes) start += s->ring_bytes - phys;
        if (start + len - s->ring_tail <= s->ring_bytes) {
            r->rv = start;
            s->ring_head = start + len;
            break;
        }
        s->cv_space.wait(lk);
    }
    s->ring_order.push_back(r);
    lk.unlock();
    if (len) std::memcpy(s->ring + r->rv % s->ring_bytes, codes + base, len);
    lk.lock();
    r->ticket = s->next_ticket++;
    r->t_submit = t_call;
    s->table[r->ticket] = r;
    s->pending.push_back(r);
    *ticket = r->ticket;
    s->cv_submit.notify_one();
    return FM_OK;
}

int fm_server_wait(fm_server *s, uint64_t ticket, double timeout_s, fm_result *out)
{
    if (!s || !out) return FM_EINVAL;
    std::unique_lock<std::mutex> lk(s->mu);
    auto it = s->table.find(ticket);
    if (it == s->table.end()) return FM_EINVAL;
    std::shared_ptr<Req> r = it->second;
    auto ready = [&] { return r->done; };
    if (timeout_s < 0) {
        s->cv_done.wait(lk, ready);
    } else if (!s->cv_done.wait_for(lk, std::chrono::duration<double>(timeout_s), ready)) {
        return FM_EAGAIN;
    }
    out->nreads = r->nreads;
    out->hits = r->hits.empty() ? nullptr : r->hits.data();
    out->nhits = r->hits.size();
    out->hit_offs = r->hit_offs.empty() ? nullptr : r->hit_offs.data();
    out->status = r->status.empty() ? nullptr : r->status.data();
    out->error = r->error;
    out->t_submit = r->t_submit;
    out->t_launch = r->t_launch;
    out->t_done = r->t_done;
    out->batch = r->batch;
    return FM_OK;
}

int fm_server_release(fm_server *s, uint64_t ticket)
{
    if (!s) return FM_EINVAL;
    std::lock_guard<std::mutex> lk(s->mu);
    auto it = s->table.find(ticket);
    if (it == s->table.end() || !it->second->done) return FM_EINVAL;
    s->table.erase(it);
    return FM_OK;
}

double fm_server_clock(const fm_server *s) { return s ? s->now() : 0.0; }

int fm_server_stats(fm_server *s, fm_server_counts *out)
{
    if (!s || !out) return FM_EINVAL;
    std::lock_guard<std::mutex> lk(s->mu);
    out->batches = s->batches;
    out->retries = s->retries;
    out->requests_done = s->requests_done;
    out->reads_done = s->reads_done;
    out->pending = s->pending.size();
    out->error = s->fatal;
    return FM_OK;
}

void fm_server_free(fm_server *s)
{
    if (!s) return;
    {
        std::lock_guard<std::mutex> lk(s->mu);
        s->stop = true;
        s->cv_submit.notify_all();
        s->cv_space.notify_all();
    }
    if (s->worker.joinable()) s->worker.join();
    int prev = -1;
    (void)hipGetDevice(&prev);
    (void)hipSetDevice(s->idx->device);
    free_lanes(s);
    if (prev >= 0) (void)hipSetDevice(prev);
    delete s;
}

}  // extern "C"
