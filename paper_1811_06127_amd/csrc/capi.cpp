// capi.cpp -- the C ABI (include/fm.h): argument checks on the host, index creation and
// device memory, and dispatch to the kernels.
#include <hip/hip_runtime.h>
#include <stdio.h>
#include <string.h>

#include <new>
#include <vector>

#include "fm_build.hpp"
#include "fm_internal.hpp"

using namespace fm;

namespace fm {

thread_local const PhaseEvents *g_plan_events = nullptr;

DevLayout dev_layout(const fm_index *idx, uint32_t I, bool rev)
{
    DevLayout d;
    const int li = ilog(I);
    d.bk = (const uint4 *)(rev ? idx->rlay[li] : idx->lay[li]);
    d.sb = compact_layout(I) ? (const uint4 *)((const char *)d.bk + num_buckets(idx->n, I) * bucket_bytes(I)) : nullptr;
    d.n = (uint32_t)idx->n;
    d.dollar = (uint32_t)(rev ? idx->rev_dollar : idx->dollar);
    const uint64_t *C = rev ? idx->rev_C : idx->C;
    for (int c = 0; c < 5; ++c) d.C[c] = (uint32_t)C[c];
    return d;
}

}  // namespace fm

namespace {

struct DeviceGuard {      // makes the index's device current for the duration of a call
    int prev = -1;
    explicit DeviceGuard(int dev)
    {
        if (hipGetDevice(&prev) != hipSuccess) prev = -1;
        if (prev != dev) (void)hipSetDevice(dev);
    }
    ~DeviceGuard()
    {
        int cur = -1;
        if (prev >= 0 && hipGetDevice(&cur) == hipSuccess && cur != prev) hipSetDevice(prev);
    }
};

int hip_status(hipError_t e) { return e == hipSuccess ? FM_OK : (e == hipErrorOutOfMemory ? FM_ENOMEM : FM_EDEVICE); }

// Events for one call's phase boundaries, or none when timing is off or full.
PhaseEvents take_events(const fm_index *idx, int kind)
{
    PhaseEvents pe;
    if (!idx->timing_cap || idx->ev_calls >= idx->timing_cap) return pe;
    const uint32_t j = idx->ev_calls++;
    for (int i = 0; i < 5; ++i) pe.ev[i] = idx->ev_pool[5 * j + i];
    idx->ev_kind[j] = kind;
    return pe;
}

void release_events(const fm_index *idx)
{
    for (hipEvent_t e : idx->ev_pool) (void)hipEventDestroy(e);
    idx->ev_pool.clear();
    idx->ev_kind.clear();
    idx->timing_cap = 0;
    idx->ev_calls = 0;
}

uint32_t nstrands(uint32_t flags) { return ((flags & FM_FWD) ? 1u : 0u) + ((flags & FM_REVCOMP) ? 1u : 0u); }

bool valid_tuning(const fm_index *idx, int op, const fm_tuning &t)
{
    const int li = ilog(t.occ_interval);
    if (li < 0 || !idx->lay[li]) return false;
    if (t.lanes != 1 && t.lanes != 2 && t.lanes != 4 && t.lanes != 8) return false;
    if (t.lanes > max_lanes(t.occ_interval)) return false;
    if (t.depth != 1 && t.depth != 2 && !(op == FM_OP_LOCATE && t.depth == 4)) return false;
    if (t.block < 64 || t.block > 256 || t.block % 64) return false;
    if (t.order > 1) return false;
    if (t.table_depth > idx->table_levels) return false;
    return true;
}

// One lane per read-strand, one read-strand in flight per lane and 8 waves per CU: the
// best setting measured on MI355X for all three searches; fm_autotune refines it.
// Locating runs 16 waves per CU (measured 1.16G against 0.91G rows/s at 8 on the
// 2^24 workload's hits).
void default_tunings(fm_index *idx, uint32_t I)
{
    fm_tuning ex = {I, 1, 1, 256, 8, 0, 0, 0};
    fm_tuning dw = {I, 1, 1, 256, 8, 0, 0, 0};
    fm_tuning in = {I, 1, 1, 256, 8, 1u << 22, 1, idx->table_levels};
    // Psi^-1 walks share no buckets and each step waits for the last: more waves pay
    fm_tuning lo = {I, 1, 1, 256, 16, 0, 0, 0};
    idx->tune[FM_OP_EXACT] = ex;
    idx->tune[FM_OP_DARRAY] = dw;
    idx->tune[FM_OP_INEXACT] = in;
    idx->tune[FM_OP_LOCATE] = lo;
}

// Where an index's pieces go: byte offsets of the forward and reverse layouts (~0: not
// built) and of the SA samples, each 256-byte aligned, and the total.
struct IndexPlan {
    uint64_t lay[kLayouts], rlay[kLayouts], table, samples, total;
    uint32_t table_levels;
};

uint64_t align256(uint64_t x) { return (x + 255) & ~(uint64_t)255; }

int plan_index(uint64_t n, const fm_load_opts *opts, bool rev, bool samples, IndexPlan &p)
{
    if (n + 1 >= (1ull << 32)) return FM_ERANGE;
    const uint32_t I = opts && opts->occ_interval ? opts->occ_interval : 128;
    if (ilog(I) < 0) return FM_EINVAL;
    const bool all = opts && (opts->flags & FM_LOAD_ALL_LAYOUTS);
    uint64_t at = 0;
    for (int side = 0; side < 2; ++side)
        for (int li = 0; li < kLayouts; ++li) {
            uint64_t &slot = side ? p.rlay[li] : p.lay[li];
            slot = ~0ull;
            if ((side && !rev) || (!all && kIntervals[li] != I)) continue;
            slot = at;
            at = align256(at + layout_bytes(n, kIntervals[li]));
        }
    p.table_levels = prefix_table_levels(n);
    p.table = ~0ull;
    if (p.table_levels) {
        p.table = at;
        at = align256(at + prefix_table_entries(p.table_levels) * 8);
    }
    p.samples = ~0ull;
    if (samples) {
        p.samples = at;
        at = align256(at + ((n + 1 + kSaSample - 1) / kSaSample) * 4);
    }
    p.total = at;
    return FM_OK;
}

// Moves packed BWTs to the device (unless they are there already) and builds the
// requested layouts, in one allocation of the index's own or in the caller's dev_buf.
int create_index(const fm_load_opts *opts, uint64_t n, const HostSide &fwd, const HostSide *rev, fm_index **out)
{
    *out = nullptr;
    const int dev = opts ? opts->device : 0;
    uint32_t I = opts && opts->occ_interval ? opts->occ_interval : 128;
    const bool want_samples = !fwd.samples.empty() || fwd.dev_samples;
    IndexPlan plan;
    if (int st = plan_index(n, opts, rev != nullptr, want_samples, plan)) return st;
    int ndev = 0;
    if (hipGetDeviceCount(&ndev) != hipSuccess || dev < 0 || dev >= ndev) return FM_EDEVICE;
    DeviceGuard g(dev);
    void *caller = opts ? opts->dev_buf : nullptr;
    if (caller) {
        hipPointerAttribute_t attr;
        if ((uintptr_t)caller % 256 || opts->dev_buf_bytes < plan.total ||
            hipPointerGetAttributes(&attr, caller) != hipSuccess || attr.type != hipMemoryTypeDevice ||
            attr.device != dev)
            return FM_EINVAL;
    }
    fm_index *idx = new (std::nothrow) fm_index();
    if (!idx) return FM_ENOMEM;
    idx->device = dev;
    idx->n = n;
    idx->dollar = fwd.dollar;
    memcpy(idx->C, fwd.C, sizeof idx->C);
    if (rev) {
        idx->has_rev = true;
        idx->rev_dollar = rev->dollar;
        memcpy(idx->rev_C, rev->C, sizeof idx->rev_C);
    }
    hipDeviceProp_t prop;
    if (hipGetDeviceProperties(&prop, dev) != hipSuccess) {
        delete idx;
        return FM_EDEVICE;
    }
    idx->cu_count = prop.multiProcessorCount;
    idx->arch = prop.gcnArchName;
    if (caller) {
        idx->mem = caller;
        idx->owns_mem = false;
    } else if (hipMalloc(&idx->mem, plan.total ? plan.total : 256) != hipSuccess) {
        idx->mem = nullptr;
        fm_index_free(idx);
        return FM_ENOMEM;
    }
    idx->device_bytes = plan.total;
    char *base = (char *)idx->mem;

    const size_t pbytes = fwd.words.size() * 4;
    size_t sbytes = 0;
    for (uint32_t J : kIntervals) sbytes = std::max(sbytes, build_layout_scratch(n, J));
    void *packed = nullptr, *scratch = nullptr;
    int st = FM_OK;
    if ((!fwd.dev_words && hipMalloc(&packed, pbytes ? pbytes : 16) != hipSuccess) ||
        hipMalloc(&scratch, sbytes) != hipSuccess)
        st = FM_ENOMEM;
    for (int side = 0; side < (rev ? 2 : 1) && !st; ++side) {
        const HostSide &h = side ? *rev : fwd;
        const uint32_t *src = h.dev_words;
        if (!src) {
            if (hipMemcpy(packed, h.words.data(), pbytes, hipMemcpyHostToDevice) != hipSuccess) {
                st = FM_EDEVICE;
                break;
            }
            src = (const uint32_t *)packed;
        }
        for (int li = 0; li < kLayouts; ++li) {
            const uint64_t off = side ? plan.rlay[li] : plan.lay[li];
            if (off == ~0ull) continue;
            void *buf = base + off;
            (side ? idx->rlay : idx->lay)[li] = buf;
            if (hipError_t e = build_layout(src, n, kIntervals[li], buf, scratch, nullptr)) {
                st = hip_status(e);
                break;
            }
        }
        if (!st && hipDeviceSynchronize() != hipSuccess) st = FM_EDEVICE;
    }
    if (packed) (void)hipFree(packed);
    if (scratch) (void)hipFree(scratch);
    // prefix table of R, computed with the index's own Occ8
    if (!st && plan.table_levels) {
        idx->ptab = (uint2 *)(base + plan.table);
        idx->table_levels = plan.table_levels;
        if (hipError_t e = build_prefix_table(idx, I, nullptr)) st = hip_status(e);
        else if (hipDeviceSynchronize() != hipSuccess) st = FM_EDEVICE;
    }
    // SA samples for fm_locate
    const uint64_t ns = (n + 1 + kSaSample - 1) / kSaSample;
    if (!st && want_samples) {
        if (!fwd.dev_samples && fwd.samples.size() != ns) st = FM_EINVAL;
        else {
            idx->sa_samples = (uint32_t *)(base + plan.samples);
            const hipError_t e = fwd.dev_samples
                                     ? hipMemcpy(idx->sa_samples, fwd.dev_samples, ns * 4, hipMemcpyDeviceToDevice)
                                     : hipMemcpy(idx->sa_samples, fwd.samples.data(), ns * 4, hipMemcpyHostToDevice);
            if (e != hipSuccess) st = FM_EDEVICE;
        }
    }
    if (st) {
        fm_index_free(idx);
        return st;
    }
    default_tunings(idx, I);
    *out = idx;
    return FM_OK;
}

}  // namespace

extern "C" {

const char *fm_strerror(int s)
{
    switch (s) {
    case FM_OK: return "ok";
    case FM_EINVAL: return "invalid argument";
    case FM_EIO: return "i/o error";
    case FM_EFORMAT: return "malformed index or BWT";
    case FM_ENOMEM: return "out of memory";
    case FM_EDEVICE: return "HIP device error";
    case FM_EOVERFLOW: return "hit capacity exceeded";
    case FM_EBUDGET: return "node budget exhausted";
    case FM_ERANGE: return "size out of range";
    case FM_EAGAIN: return "not finished yet";
    default: return "unknown status";
    }
}

int fm_version(void) { return 2; }

// The BWTs of text$ and (want_rev) reverse(text)$ sorted on the device, as device words.
static int device_sides(const uint8_t *text, uint64_t n, int dev, bool want_rev, bool want_samples, HostSide &fwd,
                        HostSide &rev, void **words_out)
{
    if (n + 1 >= (1ull << 32)) return FM_ERANGE;
    int ndev = 0;
    if (hipGetDeviceCount(&ndev) != hipSuccess || dev < 0 || dev >= ndev) return FM_EDEVICE;
    DeviceGuard g(dev);
    hipDeviceProp_t prop;
    if (hipGetDeviceProperties(&prop, dev) != hipSuccess) return FM_EDEVICE;
    const uint64_t nw = (n + 1 + 15) / 16, ns = (n + 1 + kSaSample - 1) / kSaSample;
    void *t = nullptr, *w = nullptr;
    if (hipMalloc(&t, n ? n : 16) != hipSuccess) return FM_ENOMEM;
    // packed words of each side, then the forward side's SA samples
    if (hipMalloc(&w, nw * 4 * (want_rev ? 2 : 1) + (want_samples ? ns * 4 : 0)) != hipSuccess) {
        (void)hipFree(t);
        return FM_ENOMEM;
    }
    int st = FM_OK;
    uint64_t cnt[5];
    if (n && hipMemcpy(t, text, n, hipMemcpyHostToDevice) != hipSuccess) st = FM_EDEVICE;
    if (!st) st = hip_status(device_symbol_counts((const uint8_t *)t, n, cnt, prop.multiProcessorCount, nullptr));
    if (!st && cnt[4]) st = FM_EINVAL;
    for (int side = 0; side < (want_rev ? 2 : 1) && !st; ++side) {
        HostSide &h = side ? rev : fwd;
        h.dev_words = (const uint32_t *)w + side * nw;
        uint32_t *samples = (want_samples && side == 0) ? (uint32_t *)w + (want_rev ? 2 : 1) * nw : nullptr;
        h.dev_samples = samples;
        hipError_t e = device_bwt((const uint8_t *)t, n, side == 1, (uint32_t *)h.dev_words, &h.dollar, samples,
                                  prop.multiProcessorCount, nullptr);
        if (e == hipErrorOutOfMemory) st = FM_ENOMEM;
        else if (e != hipSuccess) st = FM_EDEVICE;
        h.C[0] = 0;
        for (int c = 1; c < 5; ++c) h.C[c] = h.C[c - 1] + cnt[c - 1];
    }
    (void)hipFree(t);
    if (st) {
        (void)hipFree(w);
        return st;
    }
    *words_out = w;
    return FM_OK;
}

int fm_bwt_host(const uint8_t *text, uint64_t n, uint8_t *bwt, uint64_t *dollar_row)
{
    if ((!text && n) || !bwt || !dollar_row) return FM_EINVAL;
    return build_bwt(text, n, bwt, dollar_row);
}

int fm_bwt_device(const uint8_t *text, uint64_t n, uint8_t *bwt, uint64_t *dollar_row, int device)
{
    if ((!text && n) || !bwt || !dollar_row) return FM_EINVAL;
    HostSide fwd, rev;
    void *words = nullptr;
    int st = device_sides(text, n, device, false, false, fwd, rev, &words);
    if (st) return st;
    std::vector<uint32_t> w;
    try {
        w.resize((n + 1 + 15) / 16);
    } catch (const std::bad_alloc &) {
        st = FM_ENOMEM;
    }
    DeviceGuard g(device);
    if (!st && hipMemcpy(w.data(), words, w.size() * 4, hipMemcpyDeviceToHost) != hipSuccess) st = FM_EDEVICE;
    (void)hipFree(words);
    if (st) return st;
    for (uint64_t j = 0; j <= n; ++j) bwt[j] = (uint8_t)((w[j / 16] >> (2 * (j % 16))) & 3u);
    bwt[fwd.dollar] = 4;
    *dollar_row = fwd.dollar;
    return FM_OK;
}

int fm_pack_host(const uint8_t *codes, uint64_t count, uint32_t *words)
{
    if ((!codes && count) || (!words && count)) return FM_EINVAL;
    return pack_codes(codes, count, words, ~0ull);
}

int fm_index_build_file(const uint8_t *text, uint64_t n, const char *path, uint32_t flags)
{
    if ((!text && n) || !path) return FM_EINVAL;
    HostSide fwd, rev;
    int st = build_side(text, n, false, fwd);
    if (!st && (flags & FM_LOAD_REVERSE)) st = build_side(text, n, true, rev);
    if (st) return st;
    return write_index_file(path, n, fwd, (flags & FM_LOAD_REVERSE) ? &rev : nullptr);
}

int fm_index_from_text(const uint8_t *text, uint64_t n, const fm_load_opts *opts, fm_index **out)
{
    if ((!text && n) || !out) return FM_EINVAL;
    HostSide fwd, rev;
    const bool want_rev = opts && (opts->flags & FM_LOAD_REVERSE);
    const bool want_samples = opts && (opts->flags & FM_LOAD_LOCATE);
    if (opts && (opts->flags & FM_LOAD_DEVICE_SORT)) {
        void *words = nullptr;
        int st = device_sides(text, n, opts->device, want_rev, want_samples, fwd, rev, &words);
        if (st) return st;
        st = create_index(opts, n, fwd, want_rev ? &rev : nullptr, out);
        DeviceGuard g(opts->device);
        (void)hipFree(words);
        return st;
    }
    int st = build_side(text, n, false, fwd, want_samples);
    if (!st && want_rev) st = build_side(text, n, true, rev);
    if (st) return st;
    return create_index(opts, n, fwd, want_rev ? &rev : nullptr, out);
}

int fm_index_from_codes(const uint8_t *bwt, uint64_t rows, const uint8_t *rev_bwt, const fm_load_opts *opts,
                        fm_index **out)
{
    if (!bwt || !out || rows == 0) return FM_EINVAL;
    if (rows >= (1ull << 32)) return FM_ERANGE;
    HostSide fwd, rev;
    try {
        fwd.words.assign((rows + 15) / 16, 0u);
        if (rev_bwt) rev.words.assign((rows + 15) / 16, 0u);
    } catch (const std::bad_alloc &) {
        return FM_ENOMEM;
    }
    int st = bwt_stats(bwt, rows, &fwd.dollar, fwd.C);
    if (!st) st = pack_codes(bwt, rows, fwd.words.data(), fwd.dollar);
    if (!st && rev_bwt) {
        st = bwt_stats(rev_bwt, rows, &rev.dollar, rev.C);
        if (!st) st = pack_codes(rev_bwt, rows, rev.words.data(), rev.dollar);
        if (!st)
            for (int c = 0; c < 5; ++c)
                if (rev.C[c] != fwd.C[c]) st = FM_EFORMAT;   // reverse(R) has the same symbol counts
    }
    if (st) return st == FM_EINVAL ? FM_EFORMAT : st;
    return create_index(opts, rows - 1, fwd, rev_bwt ? &rev : nullptr, out);
}

int fm_index_load(const char *path, const fm_load_opts *opts, fm_index **out)
{
    if (!path || !out) return FM_EINVAL;
    HostSide fwd, rev;
    uint64_t n = 0;
    bool has_rev = false;
    const bool want_rev = opts && (opts->flags & FM_LOAD_REVERSE);
    int st = read_index_file(path, want_rev, &n, fwd, rev, &has_rev);
    if (st) return st;
    return create_index(opts, n, fwd, (want_rev && has_rev) ? &rev : nullptr, out);
}

int fm_index_bytes(uint64_t n, const fm_load_opts *opts, size_t *bytes)
{
    if (!bytes) return FM_EINVAL;
    IndexPlan p;
    const bool rev = opts && (opts->flags & FM_LOAD_REVERSE), samples = opts && (opts->flags & FM_LOAD_LOCATE);
    if (int st = plan_index(n, opts, rev, samples, p)) return st;
    *bytes = p.total;
    return FM_OK;
}

int fm_index_required_bytes(const char *path, const fm_load_opts *opts, size_t *bytes)
{
    if (!path || !bytes) return FM_EINVAL;
    uint64_t n = 0;
    bool has_rev = false;
    if (int st = read_index_header(path, &n, &has_rev)) return st;
    const bool want_rev = opts && (opts->flags & FM_LOAD_REVERSE);
    if (want_rev && !has_rev) return FM_EINVAL;
    IndexPlan p;
    if (int st = plan_index(n, opts, want_rev, false, p)) return st;
    *bytes = p.total;
    return FM_OK;
}

int fm_index_info(const fm_index *idx, fm_info *out)
{
    if (!idx || !out) return FM_EINVAL;
    memset(out, 0, sizeof *out);
    out->n = idx->n;
    out->dollar_row = idx->dollar;
    memcpy(out->C, idx->C, sizeof out->C);
    out->rev_dollar_row = idx->rev_dollar;
    memcpy(out->rev_C, idx->rev_C, sizeof out->rev_C);
    out->occ_interval = idx->tune[FM_OP_INEXACT].occ_interval;
    for (int i = 0; i < kLayouts; ++i)
        if (idx->lay[i]) out->layouts |= 1u << i;
    out->has_reverse = idx->has_rev ? 1u : 0u;
    out->sa_sample = idx->sa_samples ? kSaSample : 0u;
    out->device_bytes = idx->device_bytes;
    out->caller_memory = idx->owns_mem ? 0u : 1u;
    out->table_depth = idx->table_levels;
    return FM_OK;
}

void fm_index_free(fm_index *idx)
{
    if (!idx) return;
    DeviceGuard g(idx->device);
    release_events(idx);
    if (idx->mem && idx->owns_mem) (void)hipFree(idx->mem);
    delete idx;
}

int fm_get_tuning(const fm_index *idx, int op, fm_tuning *out)
{
    if (!idx || !out || op < 0 || op > FM_OP_LOCATE) return FM_EINVAL;
    *out = idx->tune[op];
    return FM_OK;
}

int fm_set_tuning(fm_index *idx, int op, const fm_tuning *t)
{
    if (!idx || !t || op < 0 || op > FM_OP_LOCATE || !valid_tuning(idx, op, *t)) return FM_EINVAL;
    if (op == FM_OP_DARRAY && (!idx->has_rev || !idx->rlay[ilog(t->occ_interval)])) return FM_EINVAL;
    idx->tune[op] = *t;
    return FM_OK;
}

int fm_occ8(const fm_index *idx, const fm_interval *q, uint64_t nq, uint32_t *out, void *stream)
{
    if (!idx || (nq && (!q || !out))) return FM_EINVAL;
    DeviceGuard g(idx->device);
    fm_tuning t = idx->tune[FM_OP_EXACT];
    return hip_status(launch_occ8(idx, t, q, nq, out, (hipStream_t)stream));
}

int fm_search_exact_workspace(const fm_index *idx, uint64_t nreads, uint32_t flags, size_t *bytes)
{
    (void)nreads;
    if (!idx || !bytes) return FM_EINVAL;
    *bytes = kWsHeader;
    return FM_OK;
}

int fm_search_exact(const fm_index *idx, const uint8_t *codes, const uint64_t *offs, uint64_t nreads, uint32_t flags,
                    fm_interval *out, void *ws, size_t ws_bytes, void *stream)
{
    if (!idx || !nstrands(flags)) return FM_EINVAL;
    if (nreads && (!codes || !offs || !out)) return FM_EINVAL;
    if (nreads * nstrands(flags) >= 0xFFFFFFFFull) return FM_ERANGE;
    const bool plain = (flags & FM_PLAIN) != 0;
    if (!plain && (!ws || ws_bytes < kWsHeader)) return FM_EINVAL;
    if (!nreads) return FM_OK;
    DeviceGuard g(idx->device);
    hipStream_t s = (hipStream_t)stream;
    if ((flags & FM_STATS) && (!ws || ws_bytes < kWsHeader)) return FM_EINVAL;
    // The persistent walk gives every wave a first chunk of its own and goes to the queue
    // counter only for the chunks after those. A launch of at most one workgroup per
    // compute unit (its grid is then exactly the workgroups the read-strands need) covers
    // every read-strand with first chunks, so the counter is never read and a small batch
    // costs one launch, as the plain kernel does.
    const fm_tuning &te = idx->tune[FM_OP_EXACT];
    const bool queue_read = nreads * nstrands(flags) * te.lanes > (uint64_t)idx->cu_count * te.block;
    if ((flags & FM_STATS) || (!plain && queue_read)) {
        if (hipError_t e = launch_fill(ws, 0, kWsHeader / 4, s)) return hip_status(e);
    }
    WalkCall c{codes, offs, nullptr, nreads, flags, 0, out, ws};
    const PhaseEvents pe = g_plan_events ? *g_plan_events : take_events(idx, 0);
    pe.mark(0, s);
    const hipError_t e = launch_walk(idx, idx->tune[FM_OP_EXACT], WALK_EXACT, plain, c, s);
    pe.mark(1, s);
    return hip_status(e);
}

int fm_darray(const fm_index *idx, const uint8_t *codes, const uint64_t *offs, uint64_t nreads, uint64_t total_len,
              uint32_t flags, uint8_t *D, void *stream)
{
    if (!idx || !nstrands(flags) || !idx->has_rev) return FM_EINVAL;
    if (nreads && (!codes || !offs || !D)) return FM_EINVAL;
    if (nreads * nstrands(flags) >= 0xFFFFFFFFull) return FM_ERANGE;
    if (!nreads) return FM_OK;
    DeviceGuard g(idx->device);
    WalkCall c{codes, offs, nullptr, nreads, flags, 0, D, nullptr};
    return hip_status(launch_darray_full(idx, idx->tune[FM_OP_DARRAY], c, total_len, (hipStream_t)stream));
}

int fm_search_inexact_workspace(const fm_index *idx, uint64_t nreads, uint64_t total_len, uint32_t flags, uint32_t zmax,
                                uint64_t hit_cap, size_t *bytes)
{
    (void)total_len;
    if (!idx || !bytes || !nstrands(flags) || zmax > FM_ZMAX) return FM_EINVAL;
    *bytes = inexact_ws_layout(nreads, nstrands(flags), zmax, hit_cap).total;
    return FM_OK;
}

int fm_search_inexact(const fm_index *idx, const uint8_t *codes, const uint64_t *offs, const uint8_t *z,
                      uint64_t nreads, uint32_t flags, uint32_t zmax, fm_hit *hits, uint64_t hit_cap,
                      uint64_t *hit_offs, uint32_t *status, void *ws, size_t ws_bytes, void *stream)
{
    if (!idx || !nstrands(flags) || zmax > FM_ZMAX || !hit_offs || !ws) return FM_EINVAL;
    if (nreads && (!codes || !offs || !z || !status || (hit_cap && !hits))) return FM_EINVAL;
    if (nreads * nstrands(flags) >= 0xFFFFFFFFull) return FM_ERANGE;
    if ((flags & FM_DARRAY) && (!idx->has_rev || !idx->rlay[ilog(idx->tune[FM_OP_DARRAY].occ_interval)]))
        return FM_EINVAL;
    const bool plain = (flags & FM_PLAIN) != 0;
    if (ws_bytes < inexact_ws_layout(nreads, nstrands(flags), zmax, hit_cap).total) return FM_EINVAL;
    DeviceGuard g(idx->device);
    DfsCall c{codes, offs, z, nreads, flags, zmax, hits, hit_cap, hit_offs, status, ws};
    const PhaseEvents pe = g_plan_events ? *g_plan_events : take_events(idx, 1);
    return hip_status(launch_inexact(idx, idx->tune[FM_OP_INEXACT], idx->tune[FM_OP_DARRAY], plain, c,
                                     (hipStream_t)stream, &pe));
}

int fm_search_both(const fm_index *idx, const uint8_t *codes, const uint64_t *offs, const uint8_t *z, uint64_t nreads,
                   uint32_t exact_flags, uint32_t flags, uint32_t zmax, fm_interval *intervals, fm_hit *hits,
                   uint64_t hit_cap, uint64_t *hit_offs, uint32_t *status, void *ws, size_t ws_bytes, void *stream)
{
    if (!idx || !nstrands(exact_flags) || (exact_flags & ~(uint32_t)(FM_BOTH | FM_PLAIN | FM_STATS | FM_FULL_RANK)))
        return FM_EINVAL;
    if (nreads && !intervals) return FM_EINVAL;
    if (nreads * nstrands(exact_flags) >= 0xFFFFFFFFull) return FM_ERANGE;
    if ((flags & (FM_PLAIN | FM_GAPS)) || (exact_flags & ~flags & FM_BOTH) || (exact_flags & FM_FULL_RANK)) {
        // the two searches one after the other: the plain kernels, the gapped search, an
        // exact search of a strand the inexact one does not search, or full ranks (the
        // DFS stops at misses)
        const uint32_t ef = (exact_flags & (FM_BOTH | FM_FULL_RANK)) | (flags & FM_PLAIN);
        const int e = fm_search_exact(idx, codes, offs, nreads, ef, intervals, ws, ws_bytes, stream);
        if (e != FM_OK) return e;
        return fm_search_inexact(idx, codes, offs, z, nreads, flags, zmax, hits, hit_cap, hit_offs, status, ws,
                                 ws_bytes, stream);
    }
    if (!nstrands(flags) || zmax > FM_ZMAX || !hit_offs || !ws) return FM_EINVAL;
    if (nreads && (!codes || !offs || !z || !status || (hit_cap && !hits))) return FM_EINVAL;
    if (nreads * nstrands(flags) + nreads * nstrands(exact_flags) >= 0xFFFFFFFFull) return FM_ERANGE;
    if ((flags & FM_DARRAY) && (!idx->has_rev || !idx->rlay[ilog(idx->tune[FM_OP_DARRAY].occ_interval)]))
        return FM_EINVAL;
    if (ws_bytes < inexact_ws_layout(nreads, nstrands(flags), zmax, hit_cap).total) return FM_EINVAL;
    DeviceGuard g(idx->device);
    DfsCall c{codes, offs, z, nreads, flags, zmax, hits, hit_cap, hit_offs, status, ws};
    c.ex_out = intervals;
    c.ex_flags = exact_flags & FM_BOTH;
    const PhaseEvents pe = g_plan_events ? *g_plan_events : take_events(idx, 1);
    return hip_status(launch_inexact(idx, idx->tune[FM_OP_INEXACT], idx->tune[FM_OP_DARRAY], false, c,
                                     (hipStream_t)stream, &pe));
}

int fm_locate_workspace(const fm_index *idx, uint64_t niv, size_t *bytes)
{
    if (!idx || !bytes) return FM_EINVAL;
    *bytes = locate_ws_bytes(niv);
    return FM_OK;
}

int fm_locate(const fm_index *idx, const uint32_t *kl, uint64_t niv, uint32_t stride, uint64_t *offs, uint32_t *pos,
              uint64_t pos_cap, uint32_t flags, void *ws, size_t ws_bytes, void *stream)
{
    if (!idx || !offs || !ws || stride < 2 || (flags & ~(uint32_t)FM_STATS)) return FM_EINVAL;
    if (niv && !kl) return FM_EINVAL;
    if (pos_cap && !pos) return FM_EINVAL;
    if (!idx->sa_samples) return FM_EINVAL;                 // built without FM_LOAD_LOCATE
    if (pos_cap > (1ull << 31) || niv >= (1ull << 40)) return FM_ERANGE;
    if (ws_bytes < locate_ws_bytes(niv)) return FM_EINVAL;
    DeviceGuard g(idx->device);
    return hip_status(launch_locate(idx, idx->tune[FM_OP_LOCATE], kl, niv, stride, offs, pos, pos_cap, ws,
                                    (flags & FM_STATS) != 0, (hipStream_t)stream));
}

int fm_phase_timing(fm_index *idx, uint32_t capacity)
{
    if (!idx) return FM_EINVAL;
    DeviceGuard g(idx->device);
    release_events(idx);
    if (!capacity) return FM_OK;
    try {
        idx->ev_pool.resize((size_t)capacity * 5, nullptr);
        idx->ev_kind.assign(capacity, 0);
    } catch (const std::bad_alloc &) {
        return FM_ENOMEM;
    }
    for (auto &e : idx->ev_pool) {
        if (hipEventCreate(&e) != hipSuccess) {
            e = nullptr;
            release_events(idx);
            return FM_EDEVICE;
        }
    }
    idx->timing_cap = capacity;
    return FM_OK;
}

int fm_phase_times(fm_index *idx, float ms[4], uint32_t *calls)
{
    if (!idx || !ms) return FM_EINVAL;
    DeviceGuard g(idx->device);
    for (int i = 0; i < 4; ++i) ms[i] = 0.f;
    auto span = [&](hipEvent_t a, hipEvent_t b) {
        float m = 0.f;
        if (hipEventSynchronize(b) != hipSuccess || hipEventElapsedTime(&m, a, b) != hipSuccess) return 0.f;
        return m;
    };
    for (uint32_t j = 0; j < idx->ev_calls; ++j) {
        hipEvent_t *e = &idx->ev_pool[5 * j];
        if (idx->ev_kind[j] == 0) {
            ms[0] += span(e[0], e[1]);
        } else {
            ms[1] += span(e[1], e[2]);
            ms[2] += span(e[2], e[3]);
            ms[3] += span(e[3], e[4]);
        }
    }
    if (calls) *calls = idx->ev_calls;
    idx->ev_calls = 0;
    return FM_OK;
}

}  // extern "C"
