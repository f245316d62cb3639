// fake_server.cpp -- TEST INFRASTRUCTURE: the request server's scheduling
// (paper_1811_06127_amd/csrc/server_core.hpp) driven by a host-only executor, so that
// admission, FIFO order, the symbol ring, retries and failure handling run on the CPU
// (also under ThreadSanitizer). Each lane is a host thread that runs its copies, searches
// and completion markers in order, after random short delays; the search is the CPU
// oracle's Listing 2 (with the D bound) on the batch. Exit status 0 when every check
// holds; each failed check prints a line and makes the status 1.
#include <stdio.h>
#include <stdlib.h>

#include <atomic>
#include <functional>
#include <random>
#include <string>

#include "../../paper_1811_06127_amd/csrc/server_core.hpp"

extern "C" {
typedef struct oracle_index oracle_index;
oracle_index *oracle_index_new(const uint8_t *R, int64_t n);
void oracle_index_free(oracle_index *x);
int64_t oracle_inexact(const oracle_index *x, const oracle_index *rev, const uint8_t *codes, const uint64_t *offs,
                       const uint8_t *z, int64_t nreads, int strands, int method, void *out, int64_t cap,
                       uint64_t *hit_offs, uint64_t *nodes_out);
}

namespace {

int g_failures = 0;
#define CHECK(cond, ...)                                                                                           \
    do {                                                                                                           \
        if (!(cond)) {                                                                                             \
            ++g_failures;                                                                                          \
            printf("CHECK FAILED %s:%d: %s -- ", __FILE__, __LINE__, #cond);                                       \
            printf(__VA_ARGS__);                                                                                   \
            printf("\n");                                                                                          \
        }                                                                                                          \
    } while (0)

// The oracle's hit set of one batch laid out as the library's search leaves it: statuses,
// hit offsets, hits and, at byte 8 of the workspace, the total every read needs.
struct Oracle {
    const oracle_index *x = nullptr, *rev = nullptr;
    uint32_t flags = 0, zmax = 0;

    void search(uint8_t *d, const fm::srv::BatchLayout &B, uint64_t n) const
    {
        const uint64_t *offs = (const uint64_t *)(d + B.offs);
        const uint8_t *codes = d + B.codes, *z = d + B.z;
        std::vector<uint8_t> zz(z, z + n);
        std::vector<uint64_t> ho(n + 1, 0);
        const int method = (flags & FM_DARRAY) ? 2 : 1;
        const int64_t total = n ? oracle_inexact(x, rev, codes, offs, zz.data(), (int64_t)n, (int)(flags & FM_BOTH),
                                                 method, nullptr, 0, ho.data(), nullptr)
                                : 0;
        std::vector<fm_hit> hits((size_t)total + 1);
        if (total) oracle_inexact(x, rev, codes, offs, zz.data(), (int64_t)n, (int)(flags & FM_BOTH), method,
                                  hits.data(), total, ho.data(), nullptr);
        uint32_t *status = (uint32_t *)(d + B.status);
        uint64_t *hit_offs = (uint64_t *)(d + B.hit_offs);
        fm_hit *out = (fm_hit *)(d + B.hits);
        const uint64_t required = (uint64_t)total;
        std::memcpy(d + B.ws + 8, &required, 8);
        uint64_t w = 0;
        hit_offs[0] = 0;
        for (uint64_t r = 0; r < n; ++r) {
            const uint64_t cnt = ho[r + 1] - ho[r];
            if (z[r] > zmax) {
                status[r] = FM_EINVAL;
            } else if (required > B.hit_cap && cnt) {
                status[r] = FM_EOVERFLOW;            // no room: the read lists no hits
            } else {
                status[r] = FM_OK;
                std::memcpy(out + w, hits.data() + ho[r], cnt * sizeof(fm_hit));
                w += cnt;
            }
            hit_offs[r + 1] = w;
        }
    }
};

// Host-only executor: lane memory in host buffers, one thread per lane running its work
// in order after random delays of up to `jitter_us`.
struct FakeExec {
    static constexpr size_t kRequiredAt = 8;
    static size_t ws_bytes(uint64_t n, uint32_t strands, uint32_t, uint64_t hit_cap)
    {
        return 256 + 64 * n * strands + 16 * hit_cap;
    }

    struct Impl {
        std::unique_ptr<uint8_t[]> dev, host, xdev, xhost;
        size_t xbytes = 0;
        std::thread th;
        std::mutex mu;
        std::condition_variable cv;
        std::deque<std::function<int()>> q;
        bool stop = false;
        std::atomic<uint64_t> issued{0}, reached{0};
        std::atomic<int> err{FM_OK};
        std::mt19937 rng;
    };
    struct Lane {
        std::unique_ptr<Impl> p;
    };

    Oracle oracle;
    unsigned jitter_us = 50;
    std::shared_ptr<std::atomic<int>> searches = std::make_shared<std::atomic<int>>(0);
    int fail_search = -1;                            // the search (counted from 0) that fails

    void enqueue(Lane &L, std::function<int()> f)
    {
        std::lock_guard<std::mutex> lk(L.p->mu);
        L.p->q.push_back(std::move(f));
        L.p->cv.notify_one();
    }

    int open(Lane &L, size_t bytes)
    {
        L.p.reset(new Impl);
        Impl *m = L.p.get();
        m->dev.reset(new uint8_t[bytes]());
        m->host.reset(new uint8_t[bytes]());
        m->rng.seed((unsigned)(uintptr_t)m);
        const unsigned jit = jitter_us;
        m->th = std::thread([m, jit] {
            for (;;) {
                std::function<int()> f;
                {
                    std::unique_lock<std::mutex> lk(m->mu);
                    m->cv.wait(lk, [&] { return m->stop || !m->q.empty(); });
                    if (m->q.empty()) return;
                    f = std::move(m->q.front());
                    m->q.pop_front();
                }
                if (jit) std::this_thread::sleep_for(std::chrono::microseconds(m->rng() % jit));
                const int e = f();
                if (e != FM_OK && m->err.load() == FM_OK) m->err = e;
            }
        });
        return FM_OK;
    }

    int grow(Lane &L, size_t bytes)
    {
        if (L.p->xbytes >= bytes) return FM_OK;
        // wait for queued work that may still use the old buffers
        while (L.p->reached.load() < L.p->issued.load()) std::this_thread::yield();
        L.p->xdev.reset(new uint8_t[bytes]());
        L.p->xhost.reset(new uint8_t[bytes]());
        L.p->xbytes = bytes;
        return FM_OK;
    }

    void close(Lane &L)
    {
        if (!L.p) return;
        {
            std::lock_guard<std::mutex> lk(L.p->mu);
            L.p->stop = true;
            L.p->cv.notify_all();
        }
        if (L.p->th.joinable()) L.p->th.join();
        L.p.reset();
    }

    uint8_t *dev(Lane &L, bool big) { return big ? L.p->xdev.get() : L.p->dev.get(); }
    uint8_t *host(Lane &L, bool big) { return big ? L.p->xhost.get() : L.p->host.get(); }

    int copy(Lane &L, void *dst, const void *src, size_t n)
    {
        enqueue(L, [dst, src, n] {
            std::memcpy(dst, src, n);
            return FM_OK;
        });
        return FM_OK;
    }
    int h2d(Lane &L, void *d, const void *s, size_t n) { return copy(L, d, s, n); }
    int d2h(Lane &L, void *d, const void *s, size_t n) { return copy(L, d, s, n); }
    int d2d(Lane &L, void *d, const void *s, size_t n) { return copy(L, d, s, n); }

    int search(Lane &L, uint8_t *d, const fm::srv::BatchLayout &B, uint64_t n)
    {
        const Oracle o = oracle;
        const int k = (*searches)++;
        const bool fail = k == fail_search;
        enqueue(L, [o, d, B, n, fail] {
            if (fail) return FM_EDEVICE;
            o.search(d, B, n);
            return FM_OK;
        });
        return FM_OK;
    }

    int mark(Lane &L)
    {
        L.p->issued++;
        Impl *m = L.p.get();
        enqueue(L, [m] {
            m->reached++;
            return FM_OK;
        });
        return FM_OK;
    }

    int poll(Lane &L)
    {
        if (L.p->err.load() != FM_OK) {
            const int e = L.p->err.load();
            // the failure ends this batch; let the lane finish what is queued and go on
            while (L.p->reached.load() < L.p->issued.load()) std::this_thread::yield();
            L.p->err = FM_OK;
            return e;
        }
        return L.p->reached.load() >= L.p->issued.load() ? FM_OK : FM_EAGAIN;
    }

    int alloc_ring(uint8_t **p, size_t bytes)
    {
        *p = new uint8_t[bytes]();
        return FM_OK;
    }
    void free_ring(uint8_t *p) { delete[] p; }
    void bind() {}
};

using FakeServer = fm::srv::Server<FakeExec>;

struct Request {
    std::vector<uint8_t> codes;
    std::vector<uint64_t> offs;
    std::vector<uint8_t> z;
};

// Reads drawn from the text (either strand, a few substitutions) and a few random ones.
std::vector<Request> make_requests(const std::vector<uint8_t> &R, int count, int max_reads, unsigned seed)
{
    std::mt19937_64 g(seed);
    std::vector<Request> out(count);
    for (auto &q : out) {
        const int nr = 1 + (int)(g() % max_reads);
        q.offs.push_back(0);
        for (int r = 0; r < nr; ++r) {
            const int m = 30 + (int)(g() % 70);
            const uint64_t p = g() % (R.size() - m);
            const bool rnd = g() % 10 == 0, minus = g() % 2;
            for (int i = 0; i < m; ++i) {
                uint8_t c = rnd ? (uint8_t)(g() % 4) : R[p + i];
                if (g() % 50 == 0) c = (uint8_t)((c + 1 + g() % 3) % 4);
                q.codes.push_back(c);
            }
            if (minus) {
                std::reverse(q.codes.end() - m, q.codes.end());
                for (auto it = q.codes.end() - m; it != q.codes.end(); ++it) *it = (uint8_t)(3 - *it);
            }
            q.offs.push_back(q.codes.size());
            q.z.push_back((uint8_t)(g() % 3));
        }
    }
    return out;
}

struct Served {
    fm_result r;
    std::vector<fm_hit> hits;
    std::vector<uint64_t> hit_offs;
    std::vector<uint32_t> status;
};

Served copy_result(const fm_result &r)
{
    Served s;
    s.r = r;
    if (r.nhits) s.hits.assign(r.hits, r.hits + r.nhits);
    if (r.hit_offs) s.hit_offs.assign(r.hit_offs, r.hit_offs + r.nreads + 1);
    if (r.status) s.status.assign(r.status, r.status + r.nreads);
    return s;
}

bool same_hits(const std::vector<fm_hit> &a, const std::vector<fm_hit> &b)
{
    return a.size() == b.size() && (a.empty() || std::memcmp(a.data(), b.data(), a.size() * sizeof(fm_hit)) == 0);
}

// The oracle's answer for one request alone, as the server reports it.
Served alone(const Oracle &o, const Request &q)
{
    const uint64_t n = q.z.size();
    const uint64_t cap = 1 << 20;
    const fm::srv::BatchLayout B =
        fm::srv::batch_layout(n, q.codes.size(), cap, FakeExec::ws_bytes(n, fm::srv::strands_of(o.flags), o.zmax, cap));
    std::vector<uint8_t> d(B.end);
    std::memcpy(d.data() + B.codes, q.codes.data(), q.codes.size());
    std::memcpy(d.data() + B.offs, q.offs.data(), 8 * (n + 1));
    std::memcpy(d.data() + B.z, q.z.data(), n);
    o.search(d.data(), B, n);
    Served s;
    const uint64_t *ho = (const uint64_t *)(d.data() + B.hit_offs);
    s.hit_offs.assign(ho, ho + n + 1);
    const uint32_t *st = (const uint32_t *)(d.data() + B.status);
    s.status.assign(st, st + n);
    const fm_hit *h = (const fm_hit *)(d.data() + B.hits);
    s.hits.assign(h, h + ho[n]);
    return s;
}

// Submits every request from a producer thread (with short random pauses) while the
// calling thread waits for them in order; returns the results.
std::vector<Served> serve(FakeServer &srv, const std::vector<Request> &reqs, unsigned seed, bool check_order = true)
{
    std::vector<uint64_t> tickets(reqs.size(), 0);
    std::atomic<size_t> submitted{0};
    std::thread producer([&] {
        std::mt19937 g(seed);
        for (size_t i = 0; i < reqs.size(); ++i) {
            const Request &q = reqs[i];
            const int e = srv.submit(q.codes.data(), q.offs.data(), q.z.data(), q.z.size(), &tickets[i]);
            CHECK(e == FM_OK, "submit %zu: %d", i, e);
            submitted.store(i + 1);
            if (g() % 3 == 0) std::this_thread::sleep_for(std::chrono::microseconds(g() % 300));
        }
    });
    std::vector<Served> out;
    for (size_t i = 0; i < reqs.size(); ++i) {
        while (submitted.load() <= i) std::this_thread::yield();
        fm_result r;
        const int e = srv.wait(tickets[i], 30.0, &r);
        CHECK(e == FM_OK, "wait %zu: %d", i, e);
        out.push_back(copy_result(r));
        CHECK(srv.release(tickets[i]) == FM_OK, "release %zu", i);
    }
    producer.join();
    if (check_order) {
        for (size_t i = 1; i < reqs.size(); ++i)
            CHECK(tickets[i] > tickets[i - 1], "tickets in submission order");
    }
    return out;
}

void check_equal_to_alone(const Oracle &o, const std::vector<Request> &reqs, const std::vector<Served> &got,
                          const char *tag)
{
    for (size_t i = 0; i < reqs.size(); ++i) {
        const Served w = alone(o, reqs[i]);
        CHECK(got[i].r.error == FM_OK, "%s %zu: error %d", tag, i, got[i].r.error);
        CHECK(got[i].hit_offs == w.hit_offs, "%s %zu: hit offsets", tag, i);
        CHECK(got[i].status == w.status, "%s %zu: statuses", tag, i);
        CHECK(same_hits(got[i].hits, w.hits), "%s %zu: hits", tag, i);
        CHECK(got[i].r.t_submit <= got[i].r.t_launch && got[i].r.t_launch <= got[i].r.t_done, "%s %zu: times", tag, i);
    }
}

// FIFO admission by bytes: the requests of a batch are consecutive in submission order,
// batch numbers never decrease along it, and every batch fits a lane.
void check_batches(const fm_server_opts &o, size_t lane_bytes, const std::vector<Request> &reqs,
                   const std::vector<Served> &got, const char *tag)
{
    size_t i = 0;
    int multi = 0;
    uint64_t prev = 0;
    while (i < reqs.size()) {
        const uint64_t b = got[i].r.batch;
        CHECK(b > prev, "%s: batch %llu after %llu", tag, (unsigned long long)b, (unsigned long long)prev);
        uint64_t n = 0, len = 0;
        size_t j = i;
        while (j < reqs.size() && got[j].r.batch == b) {
            n += reqs[j].z.size();
            len += reqs[j].codes.size();
            ++j;
        }
        for (size_t k = j; k < reqs.size(); ++k) CHECK(got[k].r.batch != b, "%s: batch %llu not contiguous", tag,
                                                       (unsigned long long)b);
        CHECK(FakeServer::batch_bytes(o, n, len) <= lane_bytes || j == i + 1, "%s: batch %llu over the lane", tag,
              (unsigned long long)b);
        if (o.max_batch_reads) CHECK(n <= o.max_batch_reads || j == i + 1, "%s: batch over the read cap", tag);
        multi += j > i + 1;
        prev = b;
        i = j;
    }
    CHECK(multi > 0, "%s: no batch held two requests", tag);
}

}  // namespace

int main()
{
    std::mt19937_64 g(1234);
    std::vector<uint8_t> R(20000);
    for (auto &c : R) c = (uint8_t)(g() % 4);
    for (int k = 0; k < 20; ++k) {                     // repeats, so that reads have several hits
        const size_t a = g() % (R.size() - 400), b = g() % (R.size() - 400);
        std::memcpy(&R[b], &R[a], 300);
    }
    std::vector<uint8_t> Rrev(R.rbegin(), R.rend());
    oracle_index *x = oracle_index_new(R.data(), (int64_t)R.size());
    oracle_index *xr = oracle_index_new(Rrev.data(), (int64_t)Rrev.size());
    Oracle o;
    o.x = x;
    o.rev = xr;
    o.flags = FM_BOTH | FM_DARRAY;
    o.zmax = 2;
    const std::vector<Request> reqs = make_requests(R, 60, 120, 99);

    auto opts = [&](uint32_t lanes, uint64_t arena, uint32_t reserve, uint64_t ring, uint64_t cap) {
        fm_server_opts so{};
        so.lanes = lanes;
        so.flags = o.flags;
        so.zmax = o.zmax;
        so.hit_reserve = reserve;
        so.arena_bytes = arena;
        so.max_batch_reads = cap;
        so.ring_bytes = ring;
        return so;
    };
    auto make = [&](const fm_server_opts &so, int fail_search = -1) {
        FakeExec fx;
        fx.oracle = o;
        fx.fail_search = fail_search;
        auto s = std::unique_ptr<FakeServer>(new FakeServer(std::move(fx)));
        CHECK(s->start(so) == FM_OK, "start");
        return s;
    };

    // 1. three lanes, an arena that holds a few requests per batch: FIFO, by bytes, alone == mixed
    {
        const fm_server_opts so = opts(3, 3 * 160000, 4, 0, 0);
        auto s = make(so);
        const auto got = serve(*s, reqs, 1);
        check_equal_to_alone(o, reqs, got, "mixed");
        check_batches(so, s->lane_bytes(), reqs, got, "mixed");
        fm_server_counts c;
        s->stats(&c);
        CHECK(c.requests_done == reqs.size() && c.error == FM_OK && c.pending == 0, "counts");
        printf("mixed: %llu batches for %zu requests, %llu retries\n", (unsigned long long)c.batches, reqs.size(),
               (unsigned long long)c.retries);
    }
    // 2. a read cap per batch
    {
        const fm_server_opts so = opts(2, 2 << 20, 4, 0, 150);
        auto s = make(so);
        const auto got = serve(*s, reqs, 2);
        check_equal_to_alone(o, reqs, got, "read cap");
        check_batches(so, s->lane_bytes(), reqs, got, "read cap");
    }
    // 3. no hit reserve: batches with hits are searched again, some in larger buffers
    {
        const fm_server_opts so = opts(2, 2 * 200000, 0, 0, 0);
        auto s = make(so);
        const auto got = serve(*s, reqs, 3);
        check_equal_to_alone(o, reqs, got, "retry");
        fm_server_counts c;
        s->stats(&c);
        CHECK(c.retries > 0, "no retries");
        printf("retry: %llu retries in %llu batches\n", (unsigned long long)c.retries, (unsigned long long)c.batches);
    }
    // 4. a ring of about two requests' symbols: submissions wait for uploads
    {
        size_t biggest = 0;
        for (auto &q : reqs) biggest = std::max(biggest, q.codes.size());
        const fm_server_opts so = opts(2, 2 << 20, 4, 2 * biggest + 64, 0);
        auto s = make(so);
        const auto got = serve(*s, reqs, 4);
        check_equal_to_alone(o, reqs, got, "small ring");
    }
    // 5. a failing search: its batch's requests report the failure, the rest are served
    {
        const fm_server_opts so = opts(2, 2 * 160000, 4, 0, 0);
        auto s = make(so, 3);
        std::vector<uint64_t> tickets(reqs.size());
        for (size_t i = 0; i < reqs.size(); ++i)
            CHECK(s->submit(reqs[i].codes.data(), reqs[i].offs.data(), reqs[i].z.data(), reqs[i].z.size(),
                            &tickets[i]) == FM_OK, "submit");
        int failed = 0, ok = 0;
        for (size_t i = 0; i < reqs.size(); ++i) {
            fm_result r;
            CHECK(s->wait(tickets[i], 30.0, &r) == FM_OK, "wait");
            if (r.error == FM_EDEVICE) ++failed;
            else if (r.error == FM_OK) {
                ++ok;
                const Served w = alone(o, reqs[i]);
                const Served g2 = copy_result(r);
                CHECK(g2.hit_offs == w.hit_offs && same_hits(g2.hits, w.hits), "served after a failure %zu", i);
            }
            s->release(tickets[i]);
        }
        fm_server_counts c;
        s->stats(&c);
        CHECK(failed > 0 && ok > 0 && failed + ok == (int)reqs.size(), "failed %d ok %d", failed, ok);
        CHECK(c.error == FM_EDEVICE, "first error %d", c.error);
        printf("failure: %d requests failed, %d served\n", failed, ok);
    }
    // 6. limits: a request larger than a lane or the ring is refused; an empty request is served
    {
        const fm_server_opts so = opts(2, 2 * 4096, 4, 4096, 0);
        auto s = make(so);
        uint64_t t = 0;
        const Request &big = reqs[0].z.size() > 50 ? reqs[0] : reqs[1];
        CHECK(s->submit(big.codes.data(), big.offs.data(), big.z.data(), big.z.size(), &t) == FM_ERANGE, "big");
        const uint64_t zero = 0;
        CHECK(s->submit(nullptr, &zero, nullptr, 0, &t) == FM_OK, "empty submit");
        fm_result r;
        CHECK(s->wait(t, 30.0, &r) == FM_OK && r.nhits == 0 && r.nreads == 0 && r.error == FM_OK, "empty result");
        CHECK(s->release(t) == FM_OK, "empty release");
        CHECK(s->release(t) == FM_EINVAL && s->wait(t, 0.0, &r) == FM_EINVAL, "unknown ticket");
    }
    oracle_index_free(x);
    oracle_index_free(xr);
    printf("%s: %d failed checks\n", g_failures ? "FAILED" : "ok", g_failures);
    return g_failures ? 1 : 0;
}
