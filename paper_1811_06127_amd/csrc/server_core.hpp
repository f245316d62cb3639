// server_core.hpp -- the request server's scheduling, independent of the device.
//
// Requests (reads with per-read budgets) are queued in arrival order; their symbols are
// copied once, at submission, into a ring of pinned host memory. A worker thread keeps
// up to `lanes` batches in flight, each with a fixed share of the arena: whenever a lane
// is idle it admits queued requests, oldest first, while the batch still fits the lane's
// memory (and the read cap), uploads their symbols straight from the ring and their
// offsets and budgets from the lane's host mirror, runs the search and brings back status
// and hit offsets, then the hits. Requests that arrive while batches run join the next
// batch of whichever lane frees up first, so their work overlaps with the batches already
// running. Every read is searched independently of its batch, so a request's result does
// not depend on what it was batched with.
//
// The device work of a lane goes through an executor type X (the library's runs on HIP
// streams; a host-only one drives the same scheduling in the CPU tests):
//   typename X::Lane                          a lane's stream, completion marker and memory
//   int  X::open(Lane &, size_t bytes)        lane memory of `bytes` and its host mirror
//   int  X::grow(Lane &, size_t bytes)        retry buffers of at least `bytes` (old contents lost)
//   void X::close(Lane &)                     waits for the lane's work and frees everything
//   uint8_t *X::dev(Lane &, bool big)         lane memory (big: the retry buffers), and
//   uint8_t *X::host(Lane &, bool big)        its host mirror
//   int  X::h2d / d2h / d2d(Lane &, void *dst, const void *src, size_t n)
//                                             copies, in order on the lane, asynchronous
//   int  X::search(Lane &, uint8_t *d, const BatchLayout &, uint64_t nreads)
//                                             the inexact search of the batch laid out at d
//   int  X::mark(Lane &)                      a completion marker after the work so far
//   int  X::poll(Lane &)                      FM_OK: marker reached, FM_EAGAIN: not yet,
//                                             another code: the lane's work failed
//   int  X::alloc_ring(uint8_t **p, size_t n), void X::free_ring(uint8_t *p)
//   void X::bind()                            on the worker thread before its first call
//   static size_t X::ws_bytes(uint64_t nreads, uint32_t strands, uint32_t zmax, uint64_t hit_cap)
//   static constexpr size_t kRequiredAt       workspace offset of the uint64 hit total that
//                                             every read of the batch would need
#pragma once

#include <stddef.h>
#include <stdint.h>

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

#include "../../include/fm.h"

namespace fm {
namespace srv {

using Clock = std::chrono::steady_clock;

inline size_t al256(size_t x) { return (x + 255) & ~(size_t)255; }

inline uint32_t strands_of(uint32_t flags) { return ((flags & FM_FWD) ? 1u : 0u) + ((flags & FM_REVCOMP) ? 1u : 0u); }

// Byte offsets of one batch's buffers inside a lane's memory. The inputs come first
// (one upload covers [0, status)); status, hit offsets and the workspace header
// follow (one download covers [status, ws + 16)); the hits come last.
struct BatchLayout {
    size_t codes, offs, z, status, hit_offs, ws, hits, end, ws_bytes;
    uint64_t hit_cap;
};

inline BatchLayout batch_layout(uint64_t n, uint64_t total_len, uint64_t hit_cap, size_t ws)
{
    BatchLayout L;
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

inline uint64_t reserve_of(const fm_server_opts &o, uint64_t n) { return (uint64_t)o.hit_reserve * n * strands_of(o.flags); }

inline bool valid_opts(const fm_server_opts *o)
{
    return o && o->lanes >= 1 && o->lanes <= 8 && strands_of(o->flags) && o->zmax <= FM_ZMAX &&
           (o->flags & ~(uint32_t)(FM_BOTH | FM_DARRAY)) == 0 && o->arena_bytes >= o->lanes;
}

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

template <class X>
struct LaneState {
    typename X::Lane x;
    size_t bytes = 0;
    int stage = 0;                             // 0 idle, 1 search in flight, 2 hit copy in flight
    bool big = false;                          // the batch runs in the retry buffers
    std::vector<std::shared_ptr<Req>> reqs;
    uint64_t n = 0, total_len = 0, batch = 0;
    BatchLayout lay{};
};

template <class X>
class Server {
public:
    explicit Server(X &&x) : x_(std::move(x)) {}
    Server(const Server &) = delete;
    Server &operator=(const Server &) = delete;

    // Device bytes of a batch under o (the admission rule).
    static uint64_t batch_bytes(const fm_server_opts &o, uint64_t n, uint64_t total_len)
    {
        const uint64_t cap = reserve_of(o, n);
        return batch_layout(n, total_len, cap, X::ws_bytes(n, strands_of(o.flags), o.zmax, cap)).end;
    }

    int start(const fm_server_opts &o)
    {
        o_ = o;
        t0_ = Clock::now();
        try {
            lanes_.resize(o.lanes);
        } catch (const std::bad_alloc &) {
            return FM_ENOMEM;
        }
        const size_t per = (size_t)(o.arena_bytes / o.lanes) & ~(size_t)255;
        ring_bytes_ = o.ring_bytes ? o.ring_bytes : o.arena_bytes;
        int e = x_.alloc_ring(&ring_, ring_bytes_);
        for (auto &ln : lanes_) {
            if (e != FM_OK) break;
            ln.bytes = per;
            e = x_.open(ln.x, per);
        }
        if (e != FM_OK) return e;
        try {
            worker_ = std::thread([this] { run(); });
        } catch (...) {
            return FM_ENOMEM;
        }
        return FM_OK;
    }

    // Finishes every queued request, stops the worker and frees the lanes and the ring.
    ~Server()
    {
        {
            std::lock_guard<std::mutex> lk(mu_);
            stop_ = true;
            cv_submit_.notify_all();
            cv_space_.notify_all();
        }
        if (worker_.joinable()) worker_.join();
        for (auto &ln : lanes_) x_.close(ln.x);
        if (ring_) x_.free_ring(ring_);
    }

    X &executor() { return x_; }
    double now() const { return std::chrono::duration<double>(Clock::now() - t0_).count(); }

    int submit(const uint8_t *codes, const uint64_t *offs, const uint8_t *z, uint64_t nreads, uint64_t *ticket)
    {
        if (!ticket || !offs || (nreads && !z)) return FM_EINVAL;
        const double t_call = now();                // latency counts any wait for ring space
        const uint64_t base = offs[0], len = offs[nreads] - base;
        if (offs[nreads] < base || (len && !codes)) return FM_EINVAL;
        for (uint64_t i = 0; i < nreads; ++i)
            if (offs[i + 1] < offs[i]) return FM_EINVAL;
        if (nreads * strands_of(o_.flags) >= 0xFFFFFFFFull) return FM_ERANGE;
        if (batch_bytes(o_, nreads, len) > lanes_[0].bytes) return FM_ERANGE;
        if (len > ring_bytes_) return FM_ERANGE;
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
        std::unique_lock<std::mutex> lk(mu_);
        // reserve ring space (a request is never split across the end of the ring), waiting
        // for older requests' uploads when the ring is full
        for (;;) {
            if (stop_) return FM_EINVAL;
            if (ring_order_.empty())                 // empty ring: restart at its beginning
                ring_head_ = ring_tail_ = (ring_head_ + ring_bytes_ - 1) / ring_bytes_ * ring_bytes_;
            uint64_t start = ring_head_;
            const uint64_t phys = start % ring_bytes_;
            if (len && phys + len > ring_bytes_) start += ring_bytes_ - phys;
            if (start + len - ring_tail_ <= ring_bytes_) {
                r->rv = start;
                ring_head_ = start + len;
                break;
            }
            cv_space_.wait(lk);
        }
        ring_order_.push_back(r);
        lk.unlock();
        if (len) std::memcpy(ring_ + r->rv % ring_bytes_, codes + base, len);
        lk.lock();
        r->ticket = next_ticket_++;
        r->t_submit = t_call;
        table_[r->ticket] = r;
        pending_.push_back(r);
        *ticket = r->ticket;
        cv_submit_.notify_one();
        return FM_OK;
    }

    int wait(uint64_t ticket, double timeout_s, fm_result *out)
    {
        if (!out) return FM_EINVAL;
        std::unique_lock<std::mutex> lk(mu_);
        auto it = table_.find(ticket);
        if (it == table_.end()) return FM_EINVAL;
        std::shared_ptr<Req> r = it->second;
        auto ready = [&] { return r->done; };
        if (timeout_s < 0) {
            cv_done_.wait(lk, ready);
        } else if (!cv_done_.wait_for(lk, std::chrono::duration<double>(timeout_s), ready)) {
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

    int release(uint64_t ticket)
    {
        std::lock_guard<std::mutex> lk(mu_);
        auto it = table_.find(ticket);
        if (it == table_.end() || !it->second->done) return FM_EINVAL;
        table_.erase(it);
        return FM_OK;
    }

    void stats(fm_server_counts *out)
    {
        std::lock_guard<std::mutex> lk(mu_);
        out->batches = batches_;
        out->retries = retries_;
        out->requests_done = requests_done_;
        out->reads_done = reads_done_;
        out->pending = pending_.size();
        out->error = fatal_;
    }

    size_t lane_bytes() const { return lanes_.empty() ? 0 : lanes_[0].bytes; }

private:
    using Lane = LaneState<X>;

    // Returns the ring space of the batch's requests (caller holds mu_): space is reused
    // oldest first, so the tail moves past every request released so far in order.
    void release_ring(Lane &ln)
    {
        for (auto &r : ln.reqs) r->ring_free = true;
        while (!ring_order_.empty() && ring_order_.front()->ring_free) ring_order_.pop_front();
        ring_tail_ = ring_order_.empty() ? ring_head_ : ring_order_.front()->rv;
        cv_space_.notify_all();
    }

    // Ends every request of the lane's batch with `err` (device failure).
    void fail_batch(Lane &ln, int err)
    {
        std::lock_guard<std::mutex> lk(mu_);
        release_ring(ln);
        const double t = now();
        for (auto &r : ln.reqs) {
            r->error = err;
            r->done = true;
            r->t_done = t;
            ++requests_done_;
        }
        if (fatal_ == FM_OK) fatal_ = err;
        ln.reqs.clear();
        ln.stage = 0;
        ln.big = false;
        cv_done_.notify_all();
    }

    BatchLayout layout_of(uint64_t n, uint64_t len, uint64_t cap) const
    {
        return batch_layout(n, len, cap, X::ws_bytes(n, strands_of(o_.flags), o_.zmax, cap));
    }

    // Enqueues the search of the lane's batch (inputs already at lay's offsets of the lane
    // memory), the download of status, hit offsets and the workspace header, and a marker.
    int enqueue_search(Lane &ln)
    {
        uint8_t *d = x_.dev(ln.x, ln.big);
        const BatchLayout &L = ln.lay;
        int e = x_.search(ln.x, d, L, ln.n);
        if (e == FM_OK) e = x_.d2h(ln.x, x_.host(ln.x, ln.big) + L.status, d + L.status, L.ws + 16 - L.status);
        if (e == FM_OK) e = x_.mark(ln.x);
        return e;
    }

    // Admits queued requests into an idle lane and launches the batch. Returns true if a
    // batch was launched.
    bool admit(Lane &ln)
    {
        std::vector<std::shared_ptr<Req>> take;
        uint64_t n = 0, len = 0;
        {
            std::lock_guard<std::mutex> lk(mu_);
            while (!pending_.empty()) {
                const auto &r = pending_.front();
                const uint64_t n2 = n + r->nreads, len2 = len + r->len;
                if (!take.empty()) {
                    if (o_.max_batch_reads && n2 > o_.max_batch_reads) break;
                    if (layout_of(n2, len2, reserve_of(o_, n2)).end > ln.bytes) break;
                }
                take.push_back(r);
                pending_.pop_front();
                n = n2;
                len = len2;
            }
            if (take.empty()) return false;
            ln.batch = ++batches_;
        }
        ln.reqs = std::move(take);
        ln.n = n;
        ln.total_len = len;
        ln.big = false;
        ln.lay = layout_of(n, len, reserve_of(o_, n));
        // offsets and budgets go through the host mirror, in the device layout; the symbols
        // are uploaded straight from the ring, one copy per run of adjacent requests
        uint8_t *h = x_.host(ln.x, false), *d = x_.dev(ln.x, false);
        uint64_t *offs = (uint64_t *)(h + ln.lay.offs);
        uint64_t rbase = 0, cbase = 0;
        offs[0] = 0;
        int e = FM_OK;
        uint64_t run_src = 0, run_dst = 0, run_len = 0;
        auto flush = [&]() {
            if (run_len && e == FM_OK) e = x_.h2d(ln.x, d + ln.lay.codes + run_dst, ring_ + run_src, run_len);
            run_len = 0;
        };
        for (auto &r : ln.reqs) {
            if (r->nreads) std::memcpy(h + ln.lay.z + rbase, r->z.data(), r->nreads);
            for (uint64_t i = 1; i <= r->nreads; ++i) offs[rbase + i] = cbase + r->offs[i];
            if (r->len) {
                const uint64_t src = r->rv % ring_bytes_;
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
        {
            std::lock_guard<std::mutex> lk(mu_);
            const double t = now();
            for (auto &r : ln.reqs) {
                r->t_launch = t;
                r->batch = ln.batch;
            }
        }
        if (e == FM_OK) e = x_.h2d(ln.x, d + ln.lay.offs, h + ln.lay.offs, ln.lay.status - ln.lay.offs);
        if (e == FM_OK) e = enqueue_search(ln);
        if (e != FM_OK) {
            fail_batch(ln, e);
            return true;
        }
        ln.stage = 1;
        return true;
    }

    // Hands each request of the finished batch its share of the results.
    void distribute(Lane &ln)
    {
        const uint8_t *h = x_.host(ln.x, ln.big);
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
        std::lock_guard<std::mutex> lk(mu_);
        const double t = now();
        for (auto &r : ln.reqs) {
            r->done = true;
            r->t_done = t;
            reads_done_ += r->nreads;
            ++requests_done_;
        }
        ln.reqs.clear();
        ln.stage = 0;
        ln.big = false;
        cv_done_.notify_all();
    }

    // Moves a busy lane forward when its last marker has been reached. Returns true on
    // progress.
    bool advance(Lane &ln)
    {
        if (ln.stage == 0) return false;
        const int q = x_.poll(ln.x);
        if (q == FM_EAGAIN) return false;
        if (q != FM_OK) {
            fail_batch(ln, q);
            return true;
        }
        if (ln.stage == 2) {
            distribute(ln);
            return true;
        }
        {
            // the uploads of this batch are complete: its ring space may be reused
            std::lock_guard<std::mutex> lk(mu_);
            release_ring(ln);
        }
        const uint8_t *h = x_.host(ln.x, ln.big);
        uint64_t required;
        std::memcpy(&required, h + ln.lay.ws + X::kRequiredAt, 8);
        if (required > ln.lay.hit_cap) {
            // some reads' hits did not fit: search the batch again with room for all
            const BatchLayout L2 = layout_of(ln.n, ln.total_len, required);
            int e = FM_OK;
            if (L2.end > ln.bytes) {
                // the retry buffers hold the batch from here on (a retry needs no second:
                // the required total is exact)
                e = x_.grow(ln.x, L2.end);
                if (e == FM_OK && !ln.big) e = x_.d2d(ln.x, x_.dev(ln.x, true), x_.dev(ln.x, false), L2.status);
                if (e == FM_OK) ln.big = true;
            }
            if (e == FM_OK) {
                ln.lay = L2;
                e = enqueue_search(ln);
            }
            if (e != FM_OK) {
                fail_batch(ln, e);
                return true;
            }
            std::lock_guard<std::mutex> lk(mu_);
            ++retries_;
            return true;
        }
        uint64_t total;
        std::memcpy(&total, h + ln.lay.hit_offs + 8 * ln.n, 8);
        if (total == 0) {
            distribute(ln);
            return true;
        }
        int e = x_.d2h(ln.x, x_.host(ln.x, ln.big) + ln.lay.hits, x_.dev(ln.x, ln.big) + ln.lay.hits, 16 * total);
        if (e == FM_OK) e = x_.mark(ln.x);
        if (e != FM_OK) {
            fail_batch(ln, e);
            return true;
        }
        ln.stage = 2;
        return true;
    }

    void run()
    {
        x_.bind();
        for (;;) {
            bool progress = false;
            for (auto &ln : lanes_) progress |= advance(ln);
            for (auto &ln : lanes_)
                if (ln.stage == 0) progress |= admit(ln);
            if (progress) continue;
            bool busy = false;
            for (auto &ln : lanes_) busy |= ln.stage != 0;
            std::unique_lock<std::mutex> lk(mu_);
            if (!busy && pending_.empty()) {
                if (stop_) break;
                cv_submit_.wait(lk, [&] { return stop_ || !pending_.empty(); });
            } else if (busy) {
                // batches in flight: poll their markers at a fine grain
                lk.unlock();
                std::this_thread::sleep_for(std::chrono::microseconds(20));
            }
        }
    }

    X x_;
    fm_server_opts o_{};
    std::vector<Lane> lanes_;
    std::mutex mu_;
    std::condition_variable cv_submit_, cv_done_, cv_space_;
    // the ring for the symbols of queued and in-flight requests: [ring_tail_, ring_head_)
    // of a position space that only grows; a position p lives at ring_[p % ring_bytes_]
    uint8_t *ring_ = nullptr;
    uint64_t ring_bytes_ = 0, ring_head_ = 0, ring_tail_ = 0;
    std::deque<std::shared_ptr<Req>> ring_order_;   // requests holding ring space, oldest first
    std::deque<std::shared_ptr<Req>> pending_;
    std::unordered_map<uint64_t, std::shared_ptr<Req>> table_;
    uint64_t next_ticket_ = 1, batches_ = 0, retries_ = 0, reads_done_ = 0, requests_done_ = 0;
    bool stop_ = false;
    int fatal_ = FM_OK;
    Clock::time_point t0_;
    std::thread worker_;
};

}  // namespace srv
}  // namespace fm
