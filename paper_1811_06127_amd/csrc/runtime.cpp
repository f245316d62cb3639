// runtime.cpp -- launch graphs per batch shape and the launch-configuration autotuner.
#include <hip/hip_runtime.h>
#include <stdio.h>
#include <string.h>

#include <string>
#include <vector>

#include "fm_internal.hpp"

using namespace fm;

// A plan is one captured graph, or, when created under phase timing, one graph per phase
// (segment) with HIP events recorded on the replay stream between them.
struct PlanSegment {
    int mark = -1;                 // phase boundary the segment starts at (-1: the call's start)
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr; // nullptr when nothing was captured in the segment
};

struct fm_plan {
    std::vector<PlanSegment> seg;
    int device = 0;
    int kind = 1;                  // 0: exact search, 1: inexact or both
    hipEvent_t ev[5] = {nullptr, nullptr, nullptr, nullptr, nullptr};   // timed plans: one per boundary
    hipError_t cut_error = hipSuccess;
};

namespace {

int hs(hipError_t e) { return e == hipSuccess ? FM_OK : (e == hipErrorOutOfMemory ? FM_ENOMEM : FM_EDEVICE); }

// One call of op with the given buffers (the same entry points the user calls).
int run_op(const fm_index *idx, int op, const uint8_t *codes, const uint64_t *offs, const uint8_t *z, uint64_t nreads,
           uint32_t flags, uint32_t zmax, void *out_buf, uint64_t hit_cap, uint64_t *hit_offs, uint32_t *status,
           void *ws, size_t ws_bytes, hipStream_t s)
{
    if (op == FM_OP_EXACT)
        return fm_search_exact(idx, codes, offs, nreads, flags, (fm_interval *)out_buf, ws, ws_bytes, s);
    return fm_search_inexact(idx, codes, offs, z, nreads, flags, zmax, (fm_hit *)out_buf, hit_cap, hit_offs, status, ws,
                             ws_bytes, s);
}

// Host copy of everything a call produces, for bit-exact comparison.
int snapshot(int op, uint64_t nreads, uint32_t flags, void *out_buf, uint64_t *hit_offs, uint32_t *status,
             hipStream_t s, std::vector<uint8_t> &img)
{
    if (hipStreamSynchronize(s) != hipSuccess) return FM_EDEVICE;
    const uint32_t ns = ((flags & FM_FWD) ? 1u : 0u) + ((flags & FM_REVCOMP) ? 1u : 0u);
    if (op == FM_OP_EXACT) {
        img.resize(nreads * ns * 8);
        return hs(hipMemcpy(img.data(), out_buf, img.size(), hipMemcpyDeviceToHost));
    }
    std::vector<uint64_t> ho(nreads + 1);
    if (hipMemcpy(ho.data(), hit_offs, ho.size() * 8, hipMemcpyDeviceToHost) != hipSuccess) return FM_EDEVICE;
    const uint64_t nh = ho[nreads];
    img.resize(ho.size() * 8 + nreads * 4 + nh * 16);
    memcpy(img.data(), ho.data(), ho.size() * 8);
    if (hipMemcpy(img.data() + ho.size() * 8, status, nreads * 4, hipMemcpyDeviceToHost) != hipSuccess) return FM_EDEVICE;
    if (nh && hipMemcpy(img.data() + ho.size() * 8 + nreads * 4, out_buf, nh * 16, hipMemcpyDeviceToHost) != hipSuccess)
        return FM_EDEVICE;
    return FM_OK;
}

std::string cache_key(const fm_index *idx, int op, uint64_t nreads, uint64_t total_len, uint32_t zmax, uint32_t flags)
{
    char buf[256];
    snprintf(buf, sizeof buf, "%s|op%d|n%llu|r%llu|t%llu|z%u|f%u", idx->arch.c_str(), op, (unsigned long long)idx->n,
             (unsigned long long)nreads, (unsigned long long)total_len, zmax, flags & ~(uint32_t)(FM_PLAIN | FM_STATS));
    return buf;
}

bool cache_lookup(const char *path, const std::string &key, fm_tuning *t, float *ms)
{
    FILE *f = fopen(path, "r");
    if (!f) return false;
    char line[512];
    bool found = false;
    while (fgets(line, sizeof line, f)) {
        char k[300];
        fm_tuning v = {};
        float m = 0;
        if (sscanf(line, "%299s %u %u %u %u %u %u %u %u %f", k, &v.occ_interval, &v.lanes, &v.depth, &v.block,
                   &v.waves_per_cu, &v.node_budget, &v.order, &v.table_depth, &m) == 10 && key == k) {
            *t = v;
            *ms = m;
            found = true;   // last entry wins
        }
    }
    fclose(f);
    return found;
}

void cache_store(const char *path, const std::string &key, const fm_tuning &t, float ms)
{
    FILE *f = fopen(path, "a");
    if (!f) return;
    fprintf(f, "%s %u %u %u %u %u %u %u %u %.6f\n", key.c_str(), t.occ_interval, t.lanes, t.depth, t.block,
            t.waves_per_cu, t.node_budget, t.order, t.table_depth, ms);
    fclose(f);
}

// Ends the capture of the current segment at phase boundary i and starts the next one.
void plan_cut(void *ctx, int i, hipStream_t s)
{
    fm_plan *p = (fm_plan *)ctx;
    PlanSegment &cur = p->seg.back();
    hipError_t e = hipStreamEndCapture(s, &cur.graph);
    PlanSegment next;
    next.mark = i;
    p->seg.push_back(next);
    if (e == hipSuccess) e = hipStreamBeginCapture(s, hipStreamCaptureModeRelaxed);
    if (e != hipSuccess && p->cut_error == hipSuccess) p->cut_error = e;
}

// Captures one call (run) on stream s into the plan: a single graph, or, when the index's
// phase timing is on, one graph per phase and an event per boundary.
template <typename F>
int capture(const fm_index *idx, fm_plan *p, hipStream_t s, F run)
{
    const bool timed = idx->timing_cap > 0;
    if (timed)
        for (int i = 0; i < 5; ++i)
            if (hipEventCreate(&p->ev[i]) != hipSuccess) {
                p->ev[i] = nullptr;
                return FM_EDEVICE;
            }
    p->seg.assign(1, PlanSegment());
    int st = hs(hipStreamBeginCapture(s, hipStreamCaptureModeRelaxed));
    if (st) return st;
    PhaseEvents pe;                    // no index events inside a graph; cuts when timed
    if (timed) {
        pe.cut = plan_cut;
        pe.ctx = p;
    }
    g_plan_events = &pe;
    const int cs = run();
    g_plan_events = nullptr;
    const int es = hs(hipStreamEndCapture(s, &p->seg.back().graph));
    st = cs ? cs : (p->cut_error != hipSuccess ? hs(p->cut_error) : es);
    for (PlanSegment &g : p->seg) {
        if (st || !g.graph) continue;
        size_t nodes = 0;
        if (hipGraphGetNodes(g.graph, nullptr, &nodes) != hipSuccess) st = FM_EDEVICE;
        else if (nodes) st = hs(hipGraphInstantiate(&g.exec, g.graph, nullptr, nullptr, 0));
    }
    return st;
}

}  // namespace

extern "C" {

int fm_plan_create(const fm_index *idx, int op, const uint8_t *codes, const uint64_t *offs, const uint8_t *z,
                   uint64_t nreads, uint32_t flags, uint32_t zmax, void *out_buf, uint64_t hit_cap, uint64_t *hit_offs,
                   uint32_t *status, void *ws, size_t ws_bytes, fm_plan **out)
{
    if (!idx || !out || (op != FM_OP_EXACT && op != FM_OP_INEXACT)) return FM_EINVAL;
    *out = nullptr;
    int prev = 0;
    (void)hipGetDevice(&prev);
    (void)hipSetDevice(idx->device);
    fm_plan *p = new fm_plan();
    p->device = idx->device;
    hipStream_t s = nullptr;
    int st = hs(hipStreamCreateWithFlags(&s, hipStreamNonBlocking));
    p->kind = op == FM_OP_EXACT ? 0 : 1;
    if (!st)
        st = capture(idx, p, s, [&] {
            return run_op(idx, op, codes, offs, z, nreads, flags, zmax, out_buf, hit_cap, hit_offs, status, ws,
                          ws_bytes, s);
        });
    if (s) (void)hipStreamDestroy(s);
    (void)hipSetDevice(prev);
    if (st) {
        fm_plan_free(p);
        return st;
    }
    *out = p;
    return FM_OK;
}

int fm_plan_create_both(const fm_index *idx, const uint8_t *codes, const uint64_t *offs, const uint8_t *z,
                        uint64_t nreads, uint32_t exact_flags, uint32_t flags, uint32_t zmax, fm_interval *intervals,
                        fm_hit *hits, uint64_t hit_cap, uint64_t *hit_offs, uint32_t *status, void *ws, size_t ws_bytes,
                        fm_plan **out)
{
    if (!idx || !out) return FM_EINVAL;
    *out = nullptr;
    int prev = 0;
    (void)hipGetDevice(&prev);
    (void)hipSetDevice(idx->device);
    fm_plan *p = new fm_plan();
    p->device = idx->device;
    hipStream_t s = nullptr;
    int st = hs(hipStreamCreateWithFlags(&s, hipStreamNonBlocking));
    if (!st)
        st = capture(idx, p, s, [&] {
            return fm_search_both(idx, codes, offs, z, nreads, exact_flags, flags, zmax, intervals, hits, hit_cap,
                                  hit_offs, status, ws, ws_bytes, s);
        });
    if (s) (void)hipStreamDestroy(s);
    (void)hipSetDevice(prev);
    if (st) {
        fm_plan_free(p);
        return st;
    }
    *out = p;
    return FM_OK;
}

int fm_plan_launch(fm_plan *plan, void *stream)
{
    if (!plan || plan->seg.empty()) return FM_EINVAL;
    hipStream_t s = (hipStream_t)stream;
    for (const PlanSegment &g : plan->seg) {
        if (g.mark >= 0 && plan->ev[g.mark] && hipEventRecord(plan->ev[g.mark], s) != hipSuccess) return FM_EDEVICE;
        if (g.exec && hipGraphLaunch(g.exec, s) != hipSuccess) return FM_EDEVICE;
    }
    return FM_OK;
}

int fm_plan_phase_times(fm_plan *plan, float ms[4])
{
    if (!plan || !ms || !plan->ev[0]) return FM_EINVAL;
    int prev = 0;
    (void)hipGetDevice(&prev);
    (void)hipSetDevice(plan->device);
    int st = FM_OK;
    auto span = [&](hipEvent_t a, hipEvent_t b) {
        float m = 0.f;
        if (hipEventSynchronize(b) != hipSuccess || hipEventElapsedTime(&m, a, b) != hipSuccess) st = FM_EDEVICE;
        return m;
    };
    for (int i = 0; i < 4; ++i) ms[i] = 0.f;
    const hipEvent_t *e = plan->ev;
    if (plan->kind == 0) {
        ms[0] = span(e[0], e[1]);
    } else {
        ms[1] = span(e[1], e[2]);
        ms[2] = span(e[2], e[3]);
        ms[3] = span(e[3], e[4]);
    }
    if (st) (void)hipGetLastError();     // leave no error behind for later calls to pick up
    (void)hipSetDevice(prev);
    return st;
}

void fm_plan_free(fm_plan *plan)
{
    if (!plan) return;
    for (PlanSegment &g : plan->seg) {
        if (g.exec) (void)hipGraphExecDestroy(g.exec);
        if (g.graph) (void)hipGraphDestroy(g.graph);
    }
    for (hipEvent_t e : plan->ev)
        if (e) (void)hipEventDestroy(e);
    delete plan;
}

int fm_autotune(fm_index *idx, int op, const uint8_t *codes, const uint64_t *offs, const uint8_t *z, uint64_t nreads,
                uint32_t flags, uint32_t zmax, void *out_buf, uint64_t hit_cap, uint64_t *hit_offs, uint32_t *status,
                void *ws, size_t ws_bytes, const char *cache_path, void *stream, fm_tuning *best, float *ms)
{
    if (!idx || op < 0 || op > 2 || nreads == 0) return FM_EINVAL;
    if (op == FM_OP_DARRAY && (!idx->has_rev || !(flags & FM_DARRAY))) return FM_EINVAL;
    hipStream_t s = (hipStream_t)stream;
    const int call_op = op == FM_OP_EXACT ? FM_OP_EXACT : FM_OP_INEXACT;
    uint64_t total_len = 0;
    if (hipMemcpy(&total_len, offs + nreads, 8, hipMemcpyDeviceToHost) != hipSuccess) return FM_EDEVICE;
    std::string key = cache_key(idx, op, nreads, total_len, zmax, flags);
    if (flags & FM_TUNE_KEEP_LAYOUT)   // the choice then depends on the layout and lanes kept
        key += "|I" + std::to_string(idx->tune[op].occ_interval) + "|L" + std::to_string(idx->tune[op].lanes);
    if (cache_path) {
        fm_tuning t;
        float m;
        if (cache_lookup(cache_path, key, &t, &m) && fm_set_tuning(idx, op, &t) == FM_OK) {
            if (best) *best = t;
            if (ms) *ms = m;
            return FM_OK;
        }
    }
    // reference output: the plain kernels
    const bool keep_layout = (flags & FM_TUNE_KEEP_LAYOUT) != 0;
    flags &= ~(uint32_t)FM_TUNE_KEEP_LAYOUT;
    const uint32_t plain_flags = (flags | FM_PLAIN) & ~(uint32_t)FM_STATS;
    size_t need = 0;
    if (call_op == FM_OP_INEXACT) fm_search_inexact_workspace(idx, nreads, total_len, plain_flags, zmax, hit_cap, &need);
    void *pws = ws;
    bool own_ws = false;
    if (call_op == FM_OP_INEXACT && need > ws_bytes) {
        if (hipMalloc(&pws, need) != hipSuccess) return FM_ENOMEM;
        own_ws = true;
    }
    std::vector<uint8_t> ref, got;
    int st = run_op(idx, call_op, codes, offs, z, nreads, plain_flags, zmax, out_buf, hit_cap, hit_offs, status, pws,
                    own_ws ? need : ws_bytes, s);
    if (!st) st = snapshot(call_op, nreads, flags, out_buf, hit_offs, status, s, ref);
    if (own_ws) (void)hipFree(pws);
    if (st) return st;

    const fm_tuning base = idx->tune[op];
    fm_tuning win = base;
    float win_ms = 1e30f;
    hipEvent_t e0, e1;
    (void)hipEventCreate(&e0);
    (void)hipEventCreate(&e1);
    const uint32_t run_flags = flags & ~(uint32_t)(FM_PLAIN | FM_STATS);
    for (uint32_t I : kIntervals) {
        if (!idx->lay[ilog(I)]) continue;
        if (op == FM_OP_DARRAY && !idx->rlay[ilog(I)]) continue;
        if (keep_layout && I != base.occ_interval) continue;
        for (uint32_t lanes = 1; lanes <= max_lanes(I); lanes *= 2) {
            if (keep_layout && lanes != base.lanes) continue;
            for (uint32_t depth = 1; depth <= (op == FM_OP_INEXACT ? 1u : 2u); ++depth) {
                // the claim order matters only to the substitution DFS with the D bound, and
                // the prefix table only to the substitution DFS with one lane per read-strand
                const bool orders = op == FM_OP_INEXACT && (flags & FM_DARRAY) && !(flags & FM_GAPS);
                const bool tables = op == FM_OP_INEXACT && !(flags & FM_GAPS) && lanes == 1 && idx->table_levels;
                const uint32_t ncand = (orders ? 10u : 5u) * (tables ? 2u : 1u);
                for (uint32_t cand = 0; cand < ncand; ++cand) {
                    static const uint32_t kWaves[5] = {0u, 4u, 8u, 12u, 16u};
                    fm_tuning t = base;
                    t.occ_interval = I;
                    t.lanes = lanes;
                    t.depth = depth;
                    t.waves_per_cu = kWaves[cand % 5];
                    if (orders) t.order = (cand / 5) % 2 == 0 ? 1u : 0u;
                    if (tables) t.table_depth = cand < ncand / 2 ? idx->table_levels : 0u;
                    if (fm_set_tuning(idx, op, &t) != FM_OK) continue;
                    st = run_op(idx, call_op, codes, offs, z, nreads, run_flags, zmax, out_buf, hit_cap, hit_offs,
                                status, ws, ws_bytes, s);
                    if (!st) st = snapshot(call_op, nreads, flags, out_buf, hit_offs, status, s, got);
                    if (st) break;
                    if (got != ref) continue;   // never pick a configuration that changes the output
                    float best_t = 1e30f;
                    for (int rep = 0; rep < 3; ++rep) {
                        (void)hipEventRecord(e0, s);
                        run_op(idx, call_op, codes, offs, z, nreads, run_flags, zmax, out_buf, hit_cap, hit_offs,
                               status, ws, ws_bytes, s);
                        (void)hipEventRecord(e1, s);
                        (void)hipEventSynchronize(e1);
                        float m = 0;
                        (void)hipEventElapsedTime(&m, e0, e1);
                        if (m < best_t) best_t = m;
                    }
                    // a later candidate must be 1% faster: settings within timing noise of
                    // each other keep the earlier one, so repeated tunings agree
                    if (best_t < win_ms * 0.99f) {
                        win_ms = best_t;
                        win = t;
                    }
                }
                if (st) break;
            }
            if (st) break;
        }
        if (st) break;
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (st) {
        fm_set_tuning(idx, op, &base);
        return st;
    }
    if (win_ms >= 1e29f) {   // nothing reproduced the reference: keep the old setting
        fm_set_tuning(idx, op, &base);
        return FM_EDEVICE;
    }
    fm_set_tuning(idx, op, &win);
    if (cache_path) cache_store(cache_path, key, win, win_ms);
    if (best) *best = win;
    if (ms) *ms = win_ms;
    return FM_OK;
}

}  // extern "C"
