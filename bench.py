#!/usr/bin/env python3
"""Throughput of the FM-index hot path on one MI355X.

Headline workload: batching at genome scale. A 3.1e9-base reference (55% i.i.d. bases,
45% copies of 500 repeat families with 5-15% divergence) and 16M reads of 150 bp from
either strand with 1% substitutions, all resident in device memory; every read gets the
exact backward search (Listing 1) and the z=2 substitution search (Listing 2) on both
strands, pruned by the D lower bound, in one pass, in batches of 4M reads, each replayed
from a launch graph captured for it. A step is one batch. The index is built once,
untimed (suffixes sorted on the device).

Prints one JSON line: reads/s of the batched persistent kernels (value), the plain
one-thread-per-read-strand kernels on the same batch, the roofline of the dominant kernel
(the DFS) with its duration measured by the graphs' own events on every timed replay,
and the oracle's rate on a sample of the same reads. Further keys hold the other
workloads: the 2^24 step, the small exact workload, the mixed-budget batch and serving
on the 2^28 index, Occ8 micro-benchmarks, locate, the gapped and full-rank searches.
"""
from __future__ import annotations

import argparse
import ctypes
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
METRIC = "reads/s & Occ8 queries/s, batched vs plain kernel, bit-exact; p99 latency"

# Bytes per launch of the dominant kernel measured with rocprofv3 (read requests and WRITE_SIZE per dispatch, checked
# against the same counters on a plain 1 GiB copy kernel; profiles/genome_dfs_3e9_counters.md). They hold only for
# the kernel sources, launch settings and workload they were measured with: the key is a hash of the kernel sources,
# the kernel, its tuning and the workload (index size / reads per launch); any other combination reports traffic
# as null.
MEASURED_TRAFFIC = {
    # read = TCC_EA0_RDREQ x 128 B (each EA read request moves a 128 B line on gfx950), write = WRITE_SIZE
    ("1ad2b605713d0b55", "dfs_batched<64, 1, 1, true, true>", (64, 1, 1, 256, 8, 1, 14), "3.1e9/4000000"):
        (1_047_402_509_952, 969_603_605),
}
TRAFFIC_KEY_FIELDS = ("occ_interval", "lanes", "depth", "block", "waves_per_cu", "order", "table_depth")
KERNEL_SOURCES = ("search.hip", "fm_device.hpp", "fm_internal.hpp")


def kernel_source_hash() -> str:
    import hashlib
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        with open(os.path.join(ROOT, "paper_1811_06127_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def search_trace(fm, torch, idx, rd, count: int, dev):
    """(k, l) of every node that Listing 2's substitution search (both strands, D bound)
    expands for the first `count` reads of the step, level by level: the queries of the
    search, to be replayed as independent Occ8 queries. Each level's children come from
    fm_occ8 (k_b = C[b] + Occ(b, k-1) + 1, l_b = C[b] + Occ(b, l), kept when non-empty and
    within the budget and the D bound from fm_darray), so the trace holds the queries as the
    kernels issue them (at k = 0 the k-1 side reads row 0). Returns the (n, 2) uint32
    queries and the same reads on the device, for checking the count against the DFS's."""
    sub = rd.subset(np.arange(count))
    m = int(sub.offs[1] - sub.offs[0])
    assert (np.diff(sub.offs.astype(np.int64)) == m).all()
    codes, offs, z = fm.reads_to_device(sub.codes, sub.offs, sub.z, dev)
    D = fm.fm_darray(idx, codes, offs, m * count, fm.FM_BOTH).cpu().numpy()
    W = sub.codes.reshape(count, m)
    comp = np.where(W < 4, 3 - W, W)[:, ::-1]             # the strand-1 pattern
    P = np.stack([W, comp], 1).reshape(2 * count, m)       # read-strand 2r + s
    DD = np.stack([D[0].reshape(count, m), D[1].reshape(count, m)], 1).reshape(2 * count, m).astype(np.int16)
    info = idx.info()
    C = np.array(info["C"][:4], np.int64)
    zz = np.repeat(sub.z.astype(np.int16), 2)
    rs = np.nonzero(zz >= DD[:, m - 1])[0]                 # the root is pruned when z < D(m-1)
    zr, k, l = zz[rs], np.zeros(rs.size, np.int64), np.full(rs.size, info["n"], np.int64)
    out = []
    for i in range(m - 1, -1, -1):
        if rs.size == 0:
            break
        q = np.stack([np.maximum(k, 1), l], 1).astype(np.uint32)
        out.append(q)
        if i == 0:
            break
        o = fm.fm_occ8(idx, torch.from_numpy(q.view(np.int32)).to(dev)).cpu().numpy().view(np.uint32).astype(np.int64)
        nxt = []
        for b in range(4):
            kb = C[b] + np.where(k == 0, 0, o[:, b]) + 1
            lb = C[b] + o[:, 4 + b]
            z2 = zr - (P[rs, i] != b)
            ok = (kb <= lb) & (z2 >= 0) & (z2 >= DD[rs, i - 1])
            nxt.append((kb[ok], lb[ok], rs[ok], z2[ok]))
        k, l, rs, zr = (np.concatenate([x[j] for x in nxt]) for j in range(4))
    return np.concatenate(out), (codes, offs, z, int(sub.offs[-1]))


def dfs_kernel_name(tcfg: dict, zmax: int) -> str:
    """The compiled DFS of fm_search_both: kind 1 takes the exact intervals from the DFS; the
    fourth argument says whether its lanes split trees at the end of the launch (one lane
    per read-strand and zmax >= 2; at zmax 1 only batches below 512 read-strands per CU,
    smaller than any the bench times), the fifth whether the prefix table serves shallow
    nodes (one lane per read-strand and a table depth above zero)."""
    steal = tcfg["lanes"] == 1 and zmax >= 2
    table = tcfg["lanes"] == 1 and tcfg.get("table_depth", 0) > 0
    return "dfs_batched<%d, %d, 1, %s, %s>" % (tcfg["occ_interval"], tcfg["lanes"], "true" if steal else "false",
                                                "true" if table else "false")


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def locate_rate(fm, torch, idx, hits, nh: int, reps: int = 3) -> dict:
    """fm_locate over the rows of the first nh hit records (Eq. 4-5): rows located per
    second and Psi^-1 steps per row, event-timed on the current stream, at 1, 2 and 4 rows
    in flight per lane and 8 or 16 waves per CU; the fastest is kept as the index's locate
    setting, and every setting must give the same positions."""
    offs, ref, steps = fm.fm_locate(idx, hits[:nh], stats=True)
    rows = int(offs[-1].item())
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(2)]
    base = idx.get_tuning(fm.FM_OP_LOCATE)
    sweep, best, same = {}, None, True
    for depth in (1, 2, 4):
        for waves in (8, 16):
            idx.set_tuning(fm.FM_OP_LOCATE, depth=depth, waves_per_cu=waves)
            _, pos = fm.fm_locate(idx, hits[:nh], cap=rows)
            same &= bool(torch.equal(pos, ref))
            ev[0].record()
            for _ in range(reps):
                fm.fm_locate(idx, hits[:nh], cap=rows)
            ev[1].record()
            torch.cuda.synchronize()
            ms = ev[0].elapsed_time(ev[1]) / reps
            sweep["depth%d_waves%d" % (depth, waves)] = round(rows / (ms / 1e3), 1)
            if best is None or ms < best[0]:
                best = (ms, depth, waves)
    idx.set_tuning(fm.FM_OP_LOCATE, **{**base, "depth": best[1], "waves_per_cu": best[2]})
    ms = best[0]
    # algorithmic bytes: a 32 B bucket per Psi^-1 step (I=64), a sample and a position per row,
    # an interval and an offset per hit
    alg = steps * 32 + rows * 8 + nh * 16
    return {"hits": nh, "rows": rows, "ms": round(ms, 4), "rows_per_s": round(rows / (ms / 1e3), 1),
            "steps_per_row": round(steps / max(rows, 1), 2), "steps_per_s": round(steps / (ms / 1e3), 1),
            "algorithmic_gb_per_s": round(alg / (ms / 1e3) / 1e9, 1),
            "rows_in_flight_per_lane": best[1], "waves_per_cu": best[2], "rows_per_s_by_setting": sweep,
            "same_positions_every_setting": same}


def parse():
    ap = argparse.ArgumentParser(description=__doc__)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=16,
                    help="timed steps of the headline; a step is one batch of the genome-scale run, cycling through "
                         "the batches")
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--headline-only", action="store_true",
                    help="run the genome-scale headline alone (no 2^24 step, small workload or serving legs)")
    ap.add_argument("--legs", default="headline,small,step,serving",
                    help="comma-separated legs to run (a profiling run may take one); the JSON line's headline "
                         "fields are null without the headline leg")
    ap.add_argument("--genome-cpu-sample", type=int, default=2000,
                    help="reads of the genome-scale workload the oracle's text-only checkers search")
    ap.add_argument("--genome-trace-reads", type=int, default=10_000,
                    help="reads whose search trace is replayed as independent Occ8 queries at genome scale")
    ap.add_argument("--batch-reads", type=int, default=4_000_000,
                    help="reads of the mixed-budget batch on the 2^28-base index")
    ap.add_argument("--tune-sample", type=int, default=250_000,
                    help="reads of the mixed-budget batch the autotuner times")
    ap.add_argument("--reads", type=int, default=1_000_000)
    ap.add_argument("--plain-steps", type=int, default=2)
    ap.add_argument("--occ8-queries", type=int, default=1 << 26)
    ap.add_argument("--cpu-sample", type=int, default=300_000,
                    help="reads the CPU oracle searches for the baseline (0 skips it)")
    ap.add_argument("--cpu-threads", type=int, default=min(16, os.cpu_count() or 1),
                    help="host threads of the CPU baseline (the GPU box's share is 16 cores)")
    ap.add_argument("--no-tune", action="store_true")
    ap.add_argument("--tune-cache", default=None)
    ap.add_argument("--serve-requests", type=int, default=2000,
                    help="requests in the serving run on the 2^28-base index (0 skips it)")
    ap.add_argument("--serve-load", type=float, default=0.8, help="arrival rate as a fraction of capacity")
    ap.add_argument("--serve-lanes", type=int, default=3)
    ap.add_argument("--serve-pool", type=int, default=2_000_000, help="reads the requests are drawn from")
    ap.add_argument("--genome-batches", type=int, default=4,
                    help="batches in the genome-scale run on the 3.1e9-base index")
    ap.add_argument("--genome-batch-reads", type=int, default=4_000_000,
                    help="reads per batch (one launch graph each) in the genome-scale run: each DFS launch "
                         "ends with a tail of about 8 ms in which its last trees keep part of the chip busy, "
                         "so larger batches spend less of their time there")
    ap.add_argument("--skip-two-stream", action="store_true",
                    help="skip the genome-scale replays on two streams")
    ap.add_argument("--pcie-two-streams", action="store_true",
                    help="also time the step end to end on two streams, copies overlapping the other batch's search")
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="MIB",
                    help="also run one plain device-to-device copy of this many MiB (a kernel of known "
                         "traffic for scaling hardware byte counters)")
    return ap.parse_args()


def step_2e24(args):
    """The 2^24 step: a 2^24-base reference (95% i.i.d. bases plus 500-5,000 bp copies with 2%
    substitutions), 1,000,000 reads of 100 bp sampled from either strand with 1%
    substitutions; the exact backward search of every read on both strands and the z=1
    substitution search on both strands pruned by the D lower bound, in one pass
    (fm_search_both). Its 8.4 MB index lives in the caches, not HBM."""
    import torch

    import synth
    from paper_1811_06127_amd import fm

    dev = torch.device("cuda", 0)
    t0 = time.time()
    R = synth.repeats_2e24_reference()
    rd = synth.reads_2e24(R, args.reads)
    log("inputs generated in %.1fs: n=%d reads=%d" % (time.time() - t0, R.size, rd.count))
    t0 = time.time()
    idx = fm.Index.from_text(R, occ_interval=64,
                             flags=fm.FM_LOAD_REVERSE | fm.FM_LOAD_ALL_LAYOUTS | fm.FM_LOAD_LOCATE)
    log("index built in %.1fs" % (time.time() - t0))

    nreads = rd.count
    total_len = int(rd.offs[-1])
    codes, offs, z = fm.reads_to_device(rd.codes, rd.offs, rd.z, dev)
    EXACT = fm.FM_BOTH
    INEXACT = fm.FM_BOTH | fm.FM_DARRAY
    ZMAX = 1
    hit_cap = 4 * nreads
    ex_out = torch.empty((2 * nreads, 2), dtype=torch.int32, device=dev)
    ex_ws = torch.zeros(fm.fm_search_exact_workspace(idx, nreads, EXACT), dtype=torch.uint8, device=dev)
    # workspace sized for the plain kernels too (they keep their DFS stacks in it)
    bufs = fm.InexactBuffers(idx, nreads, total_len, INEXACT | fm.FM_PLAIN, ZMAX, hit_cap, dev)

    tuning = {}
    if not args.no_tune:
        t0 = time.time()
        tuning["exact"] = fm.fm_autotune(idx, fm.FM_OP_EXACT, codes, offs, None, EXACT, out=ex_out, ws=ex_ws,
                                         cache_path=args.tune_cache)
        tuning["inexact"] = fm.fm_autotune(idx, fm.FM_OP_INEXACT, codes, offs, z, INEXACT, ZMAX, bufs=bufs,
                                           cache_path=args.tune_cache)
        tuning["d_walk"] = fm.fm_autotune(idx, fm.FM_OP_DARRAY, codes, offs, z, INEXACT, ZMAX, bufs=bufs,
                                          cache_path=args.tune_cache)
        log("autotuned in %.1fs: %s" % (time.time() - t0, tuning))
    for name, op in (("exact", fm.FM_OP_EXACT), ("d_walk", fm.FM_OP_DARRAY), ("inexact", fm.FM_OP_INEXACT)):
        tuning.setdefault(name, (idx.get_tuning(op), None))
        tuning[name] = {"config": idx.get_tuning(op), "ms": tuning[name][1]}

    def step(extra=0):
        # both searches in one pass: the exact intervals come out of the DFS
        fm.fm_search_both(idx, codes, offs, z, EXACT, INEXACT | extra, ZMAX, hit_cap, out=ex_out, bufs=bufs)

    def separate(extra=0):
        fm.fm_search_exact(idx, codes, offs, EXACT | extra, out=ex_out, ws=ex_ws)
        fm.fm_search_inexact(idx, codes, offs, z, INEXACT | extra, ZMAX, hit_cap, bufs=bufs)

    def timed(f, steps, calls_per_step):
        idx.phase_timing(calls_per_step * steps)
        t0, t1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        torch.cuda.synchronize()
        t0.record()
        for _ in range(steps):
            f()
        t1.record()
        torch.cuda.synchronize()
        ph, calls = idx.phase_times()
        idx.phase_timing(0)
        assert calls == calls_per_step * steps, calls
        return t0.elapsed_time(t1) / steps, {k: v / steps for k, v in ph.items()}

    # work counters of one step (untimed)
    separate(fm.FM_STATS)
    torch.cuda.synchronize()
    ex_stats = fm.exact_stats(ex_ws)
    in_stats = bufs.stats()
    step(fm.FM_STATS)
    torch.cuda.synchronize()
    both_stats = bufs.stats()
    log("stats: exact", ex_stats, "inexact", in_stats, "one pass", both_stats)

    for _ in range(args.warmup):
        separate()
    sep_ms, sep_phase = timed(separate, args.steps, 2)
    log("separate calls: %.3f ms/step, phases %s" % (sep_ms, sep_phase))
    ex_separate = ex_out.clone()
    in_separate = fm.hits_to_numpy(bufs, nreads)
    for _ in range(args.warmup):
        step()
    ms_step, both_phase = timed(step, args.steps, 1)
    phase_ms = {"d_walk": both_phase["d_walk"], "dfs": both_phase["dfs"], "compaction": both_phase["compaction"]}
    log("batched: %.3f ms/step, phases per step %s" % (ms_step, phase_ms))
    ex_batched = ex_out.clone()
    in_batched = fm.hits_to_numpy(bufs, nreads)
    fused_equal = bool(torch.equal(ex_batched, ex_separate)) and all(
        np.array_equal(a, b) for a, b in zip(in_batched, in_separate))
    log("one pass equals separate calls:", fused_equal)
    # text positions of the step's hits (fm_locate)
    loc = locate_rate(fm, torch, idx, bufs.hits, int(in_batched[1][-1]))
    log("locate:", loc)
    # Listing 2 with all its branches (z=1 edits) on the same reads
    gap = gapped_rate(fm, torch, idx, codes, offs, z, nreads, total_len, args)
    log("gapped:", gap)
    gap["z2"] = gapped_z2_rate(fm, torch, idx, rd, args)
    log("gapped z=2:", gap["z2"])
    frank = full_rank_rate(fm, torch, idx, codes, offs, nreads, ex_ws, args)
    log("full rank:", frank)
    layouts = layout_rates(fm, torch, idx, step, ex_out, bufs, nreads, (ex_batched, in_batched))
    log("layouts:", layouts)

    # the same step replayed from a launch graph captured for this batch shape
    plans = [fm.Plan.both(idx, codes, offs, z, EXACT, INEXACT, ZMAX, ex_out, bufs)]
    for p in plans:
        p.launch()
    torch.cuda.synchronize()
    g0, g1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    g0.record()
    for _ in range(args.steps):
        for p in plans:
            p.launch()
    g1.record()
    torch.cuda.synchronize()
    graph_ms = g0.elapsed_time(g1) / args.steps
    graph_equal = bool(torch.equal(ex_out, ex_batched)) and all(
        np.array_equal(a, b) for a, b in zip(fm.hits_to_numpy(bufs, nreads), in_batched))
    for p in plans:
        p.free()
    log("graph replay: %.3f ms/step, identical: %s" % (graph_ms, graph_equal))

    # the step end to end over PCIe: reads uploaded from pinned host memory, then the exact
    # intervals, hit offsets, statuses and the listed hits read back (their count is the
    # same on every step of this batch, so no extra round trip reads it first)
    n_listed = int(in_batched[1][-1])
    h_in = [torch.from_numpy(np.ascontiguousarray(a)).pin_memory()
            for a in (rd.codes, rd.offs.view(np.int64), rd.z)]
    h_out = [torch.empty(t.shape, dtype=t.dtype).pin_memory()
             for t in (ex_out, bufs.hit_offs, bufs.status, bufs.hits[:n_listed])]

    def end_to_end():
        for d, h in zip((codes, offs, z), h_in):
            d.copy_(h, non_blocking=True)
        step()
        for h, d in zip(h_out, (ex_out, bufs.hit_offs, bufs.status, bufs.hits[:n_listed])):
            h.copy_(d, non_blocking=True)

    end_to_end()
    torch.cuda.synchronize()
    x0, x1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    x0.record()
    for _ in range(args.steps):
        end_to_end()
    x1.record()
    torch.cuda.synchronize()
    e2e_ms = x0.elapsed_time(x1) / args.steps
    e2e_equal = bool(torch.equal(h_out[0], ex_batched.cpu())) and bool(
        np.array_equal(h_out[3].numpy().view(np.uint32).reshape(-1), in_batched[0].view(np.uint32).reshape(-1)))
    e2e_bytes = sum(t.numel() * t.element_size() for t in h_in + h_out)
    log("end to end over PCIe: %.3f ms/step (%.1f MB moved), identical: %s" % (e2e_ms, e2e_bytes / 1e6, e2e_equal))
    del h_out

    def two_stream_e2e():
        # the same with two buffer sets on two streams (default priority), so that one batch's
        # copies overlap the other's search, as the server's lanes do. Off by default: streams
        # made here share the GPU's few hardware queues with the serving leg's and were seen to
        # slow both (the serving leg measures overlapped copies under load anyway).
        streams = [torch.cuda.Stream(), torch.cuda.Stream()]
        sets = []
        for st_ in streams:
            with torch.cuda.stream(st_):
                c2, o2, z2, e2 = (torch.empty_like(t) for t in (codes, offs, z, ex_out))
                b2 = fm.InexactBuffers(idx, nreads, total_len, INEXACT, ZMAX, hit_cap, dev)
                ho = [torch.empty(t.shape, dtype=t.dtype).pin_memory()
                      for t in (e2, b2.hit_offs, b2.status, b2.hits[:n_listed])]
            sets.append((st_, c2, o2, z2, e2, b2, ho))

        def overlapped(i):
            st_, c2, o2, z2, e2, b2, ho = sets[i % 2]
            with torch.cuda.stream(st_):
                for d, h in zip((c2, o2, z2), h_in):
                    d.copy_(h, non_blocking=True)
                fm.fm_search_both(idx, c2, o2, z2, EXACT, INEXACT, ZMAX, hit_cap, out=e2, bufs=b2, stream=st_)
                for h, d in zip(ho, (e2, b2.hit_offs, b2.status, b2.hits[:n_listed])):
                    h.copy_(d, non_blocking=True)

        for i in range(2):
            overlapped(i)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for i in range(args.steps):
            overlapped(i)
        torch.cuda.synchronize()
        ovl_ms = (time.perf_counter() - t0) * 1e3 / args.steps
        ovl_equal = all(bool(torch.equal(ho[0], ex_batched.cpu())) and bool(np.array_equal(
            ho[3].numpy().view(np.uint32).reshape(-1), in_batched[0].view(np.uint32).reshape(-1)))
            for (_, _, _, _, _, _, ho) in sets)
        log("end to end over PCIe, two streams: %.3f ms/step, identical: %s" % (ovl_ms, ovl_equal))
        del sets
        return ovl_ms, ovl_equal

    # the plain kernels on the same step, and their agreement with the batched ones
    plain_ms = None
    plain_equal = None
    if args.plain_steps > 0:
        step(fm.FM_PLAIN)
        torch.cuda.synchronize()
        p0, p1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        p0.record()
        for _ in range(args.plain_steps):
            step(fm.FM_PLAIN)       # the plain exact kernel, then the plain inexact kernels
        p1.record()
        torch.cuda.synchronize()
        plain_ms = p0.elapsed_time(p1) / args.plain_steps
        in_plain = fm.hits_to_numpy(bufs, nreads)
        plain_equal = bool(torch.equal(ex_out, ex_batched)) and all(
            np.array_equal(a, b) for a, b in zip(in_plain, in_batched))
        log("plain: %.3f ms/step, identical to batched: %s" % (plain_ms, plain_equal))

    # Occ8 micro-benchmark: independent uniform (k, l) pairs (two buckets each), narrow ones,
    # l uniform and k = l + 1 - w with w in [0, 8] (mostly one bucket), and the queries the
    # inexact search itself makes (its trace on the step's first reads, replayed independently)
    occ8_rate, occ8_lanes = {}, {}
    trace_info = None
    if args.occ8_queries:
        t0 = time.time()
        count = min(nreads, max(1000, args.occ8_queries // 160))
        trace, (tc, to, tz, tlen) = search_trace(fm, torch, idx, rd, count, dev)
        tb = fm.InexactBuffers(idx, count, tlen, INEXACT, ZMAX, 4 * count, dev)
        fm.fm_search_inexact(idx, tc, to, tz, INEXACT | fm.FM_STATS, ZMAX, 4 * count, bufs=tb)
        torch.cuda.synchronize()
        trace_info = {"reads": count, "queries": int(trace.shape[0]),
                      "equals_dfs_node_count": int(trace.shape[0]) == tb.stats()["occ8"]}
        log("search trace of %d reads: %d queries in %.1fs, DFS node count equal: %s" % (
            count, trace.shape[0], time.time() - t0, trace_info["equals_dfs_node_count"]))
        del tb, tc, to, tz
        for kind in ("uniform", "narrow", "search_trace"):
            if kind == "search_trace":
                qh = trace
            else:
                qh = synth.occ8_queries(R.size, args.occ8_queries, 4242, kind)
            q = torch.from_numpy(qh.view(np.int32)).to(dev)
            nq = qh.shape[0]
            qo = torch.empty((nq, 8), dtype=torch.int32, device=dev)
            # fm_occ8 runs with the exact search's layout and lanes per query; the best of
            # one and two lanes per query is reported for each query set
            ex_cfg = idx.get_tuning(fm.FM_OP_EXACT)
            for lanes in (1, 2):
                idx.set_tuning(fm.FM_OP_EXACT, lanes=lanes)
                fm.fm_occ8(idx, q, out=qo)
                torch.cuda.synchronize()
                q0, q1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
                q0.record()
                for _ in range(3):
                    fm.fm_occ8(idx, q, out=qo)
                q1.record()
                torch.cuda.synchronize()
                rate = nq / (q0.elapsed_time(q1) / 3 / 1e3)
                if rate > occ8_rate.get(kind, 0.0):
                    occ8_rate[kind], occ8_lanes[kind] = rate, lanes
            idx.set_tuning(fm.FM_OP_EXACT, **ex_cfg)
            del q, qo

    # roofline of the dominant kernel: algorithmic bytes per launch / its event-timed duration
    I = tuning["inexact"]["config"]["occ_interval"]
    Iw = tuning["d_walk"]["config"]["occ_interval"]
    nrs = 2 * nreads
    n_hits = int(in_batched[1][-1])
    # per read-strand: the D walk reads the pattern and writes a 16-byte D record; the DFS
    # reads the pattern and the record and writes a hit count, a status and the exact
    # interval (8 bytes), plus 16 bytes per hit
    alg = {
        "d_walk": both_stats["walk_buckets"] * (16 + Iw // 4) + 2 * total_len + 16 * nrs,
        "dfs": both_stats["buckets"] * (16 + I // 4) + 32 * both_stats["table"] + 2 * total_len + 32 * nrs
        + 16 * n_hits,
    }
    dom = max(("d_walk", "dfs"), key=lambda k: phase_ms[k])
    achieved = alg[dom] / (phase_ms[dom] / 1e3) / 1e9
    tcfg = tuning[{"d_walk": "d_walk", "dfs": "inexact"}[dom]]["config"]
    # the kernel as compiled: DFS kind 1 takes the exact intervals from the DFS; walk mode 1 is the D walk
    kname = (dfs_kernel_name(tcfg, ZMAX) if dom == "dfs" else
             "walk_batched<%d, %d, %d, 1>" % (tcfg["occ_interval"], tcfg["lanes"], tcfg["depth"]))
    key = (kernel_source_hash(), kname, tuple(tcfg[f] for f in TRAFFIC_KEY_FIELDS), "2^24")
    traffic = MEASURED_TRAFFIC.get(key)
    roofline = {"bound": residency_bound(idx.info()["device_bytes"]), "kernel": kname,
                "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": round(achieved / HBM_PEAK_GBS, 4),
                "traffic": int(sum(traffic)) if traffic else None,
                "traffic_gb_per_s": round(sum(traffic) / (phase_ms[dom] / 1e3) / 1e9, 1) if traffic else None,
                "bytes_per_launch": int(alg[dom]), "avg_launch_ms": round(phase_ms[dom], 4),
                "kernel_source_hash": key[0]}

    cpu = None
    parity = None
    if args.cpu_sample > 0:
        cpu, parity = cpu_baseline(R, rd, min(args.cpu_sample, nreads), ex_batched, in_batched, args.cpu_threads)

    ovl = two_stream_e2e() if args.pcie_two_streams else None
    del h_in
    index_bytes = idx.info()["device_bytes"]
    del codes, offs, z, ex_out, ex_ws, bufs
    idx.free()
    torch.cuda.empty_cache()
    reads_s = nreads / (ms_step / 1e3)
    out = {
        "workload": "2^24-base reference with 5% copies (2% divergence); 1M reads x 100 bp, 1% substitutions, "
                    "either strand; exact + z=1 substitution search, both strands, D-array pruning",
        "n": int(R.size), "reads": nreads, "read_len": 100, "z": ZMAX, "strands": 2, "hit_cap": hit_cap,
        "index_bytes_all_layouts": int(index_bytes),
        "reads_per_s": round(reads_s, 1),
        "ms_per_step": round(ms_step, 4),
        "plain_reads_per_s": round(nreads / (plain_ms / 1e3), 1) if plain_ms else None,
        "batched_vs_plain": round(plain_ms / ms_step, 3) if plain_ms else None,
        "batched_equals_plain": plain_equal,
        "graph_ms_per_step": round(graph_ms, 4),
        "pcie_inclusive": {"ms_per_step": round(e2e_ms, 4), "reads_per_s": round(nreads / (e2e_ms / 1e3), 1),
                           "bytes_moved": int(e2e_bytes), "equals_device_resident": e2e_equal,
                           "two_streams": None if ovl is None else {
                               "ms_per_step": round(ovl[0], 4), "reads_per_s": round(nreads / (ovl[0] / 1e3), 1),
                               "equals_device_resident": ovl[1]}},
        "graph_equals_eager": graph_equal,
        "occ8_queries_per_s": {**{"fm_occ8_" + k: round(v, 1) for k, v in occ8_rate.items()},
                               "dfs_in_separate_call": round(in_stats["occ8"] / (sep_phase["dfs"] / 1e3), 1)},
        "full_rank_exact": frank,
        "step_by_layout": layouts,
        "occ8_search_trace": trace_info,
        "occ8_lanes_per_query": occ8_lanes,
        "phase_ms": {k: round(v, 4) for k, v in phase_ms.items()},
        "separate_calls": {"ms_per_step": round(sep_ms, 4), "phase_ms": {k: round(v, 4) for k, v in sep_phase.items()},
                           "equal_to_one_pass": fused_equal},
        "work_per_step": {"exact_steps": ex_stats["steps"], "exact_buckets": ex_stats["buckets"],
                          "d_walk_steps": in_stats["walk_steps"], "d_walk_buckets": in_stats["walk_buckets"],
                          "dfs_nodes": both_stats["occ8"], "dfs_buckets": both_stats["buckets"],
                          "dfs_table_nodes": both_stats["table"], "hits": n_hits},
        "tuning": tuning,
        "roofline": roofline,
        "cpu_baseline": cpu,
        "parity_sample": parity,
        "locate": loc,
        "gapped": gap,
    }
    log("2^24 step:", {k: out[k] for k in ("reads_per_s", "ms_per_step", "batched_vs_plain", "roofline")})
    return out


def main():
    args = parse()
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print("bench.py measures one GPU: the search shards by replicating the index and splitting the "
              "reads, and this build runs and reports the single-GPU share only (--gpus 1).", file=sys.stderr)
        sys.exit(2)

    import torch

    torch.cuda.set_device(0)
    dev = torch.device("cuda", 0)
    if args.copy_calibration:
        n = args.copy_calibration << 20
        src = torch.ones(n, dtype=torch.uint8, device=dev)
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        torch.add(src, 1, out=dst)           # one elementwise kernel: n bytes in, n bytes out
        torch.cuda.synchronize()
        log("copy calibration: %d bytes read, %d bytes written" % (n, n))
        del src, dst

    legs = set(args.legs.split(","))
    if args.headline_only:
        legs = {"headline"}
    head = {"value": None, "ms_per_step": None, "config": None, "roofline": None, "cpu_baseline": None,
            "parity_sample": None, "extra": {}}
    if "headline" in legs:
        head = genome_headline(args)
    extra = dict(head["extra"])
    extra["parity_sample"] = head["parity_sample"]
    if "small" in legs:
        extra["small_exact"] = small_exact(args)
    if "step" in legs:
        extra["step_2e24"] = step_2e24(args)
        torch.cuda.empty_cache()
    if "serving" in legs and args.serve_requests > 0:
        extra["serving"] = serve_bench(args)
        extra["p99_latency_ms"] = extra["serving"]["p99_ms"]
        torch.cuda.empty_cache()
    out = {
        "metric": METRIC,
        "value": head["value"],
        "unit": "reads/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": head["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "u32",
        "data": "synthetic (seeded SplitMix64 reference and reads)",
        "config": head["config"],
        "roofline": head["roofline"],
        "cpu_baseline": head["cpu_baseline"],
        **extra,
    }
    print(json.dumps(out), flush=True)


def random_read_ceiling(fm, torch, idx, spans=(1 << 30, 2 << 30, 4 << 30), rounds=64):
    """Independent reads of random 32-byte blocks over each span of device memory
    (fm_probe_random_reads, the median of 3 timed launches after one untimed): the rate at
    which the device serves the searches' bucket fetches over an index of that size."""
    buf = torch.zeros(max(spans), dtype=torch.uint8, device="cuda")
    sink = torch.zeros(1, dtype=torch.int32, device="cuda")
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(2)]
    rates = {}
    for span in spans:
        fm.probe_random_reads(idx, buf, span, rounds, sink)
        ms = []
        for _ in range(3):
            ev[0].record()
            n = fm.probe_random_reads(idx, buf, span, rounds, sink)
            ev[1].record()
            torch.cuda.synchronize()
            ms.append(ev[0].elapsed_time(ev[1]))
        rates["%d GiB" % (span >> 30)] = round(n / (sorted(ms)[1] / 1e3), 1)
    del buf, sink
    return rates


def genome_headline(args):
    """The headline: batching at genome scale. A 3.1e9-base text (55% i.i.d., 45% copies
    of 500 repeat families with 5-15% divergence) and 16M reads of 150 bp with 1%
    substitutions, all resident in device memory; z=2 with the D bound on both strands,
    in batches of `--genome-batch-reads` (4M), each replayed from a launch graph captured for
    it (one per batch, outputs per batch). A step is one batch; steps cycle through the batches.
    The graphs record phase events of their own, so the DFS kernel's duration is measured
    on every replay of the timed region."""
    import torch

    import synth
    from paper_1811_06127_amd import fm

    B, LEN, Z = args.genome_batch_reads, 150, 2
    NB = args.genome_batches
    flags = fm.FM_BOTH | fm.FM_DARRAY
    cap = 16 * B
    t0 = time.time()
    R = synth.genome_like_reference()
    t1 = time.time()
    idx = fm.Index.from_text(R, occ_interval=64,
                             flags=fm.FM_LOAD_REVERSE | fm.FM_LOAD_DEVICE_SORT | fm.FM_LOAD_LOCATE)
    build_s = time.time() - t1
    rd = synth.genome_reads(R, NB * B)
    assert (np.diff(rd.offs) == LEN).all()
    log("genome-scale inputs in %.1fs (index %.1fs, suffixes sorted on the device): %s" % (
        time.time() - t0, build_s, idx.info()))
    codes_all = torch.from_numpy(rd.codes).cuda()
    z_all = torch.from_numpy(rd.z).cuda()
    offs = torch.from_numpy(rd.offs[:B + 1].view(np.int64)).cuda()      # every batch has the same offsets
    batches = []
    for b in range(NB):
        codes = codes_all[b * B * LEN:(b + 1) * B * LEN]
        z = z_all[b * B:(b + 1) * B]
        ex = torch.empty((2 * B, 2), dtype=torch.int32, device="cuda")
        bufs = fm.InexactBuffers(idx, B, B * LEN, flags, Z, cap, "cuda")
        batches.append((codes, z, ex, bufs))
    # the index's default launch settings: at this scale the tuner's choice varies between runs
    # within timing noise, and fixed settings keep runs and their profiles comparable
    tuning = {"inexact": idx.get_tuning(fm.FM_OP_INEXACT), "d_walk": idx.get_tuning(fm.FM_OP_DARRAY)}

    # eager calls with work counters: nodes, buckets and hits per batch, and each batch's outputs
    work = {"occ8": 0, "buckets": 0, "walk_steps": 0, "walk_buckets": 0, "subtrees": 0, "table": 0}
    hits_per_batch, eager = [], []
    for codes, z, ex, bufs in batches:
        fm.fm_search_both(idx, codes, offs, z, fm.FM_BOTH, flags | fm.FM_STATS, Z, cap, out=ex, bufs=bufs)
        torch.cuda.synchronize()
        st = bufs.stats()
        for k in work:
            work[k] += st[k]
        n = int(bufs.hit_offs[-1].item())
        hits_per_batch.append(n)
        eager.append((ex.clone(), bufs.hit_offs.clone(), bufs.status[:B].clone(), bufs.hits[:n].clone()))
    all_ok = all(bool((e[2] == fm.FM_OK).all()) for e in eager)
    # the plain one-thread-per-read-strand kernels on the first batch
    codes, z, ex, bufs = batches[0]
    pex = torch.empty_like(ex)
    pbufs = fm.InexactBuffers(idx, B, B * LEN, flags | fm.FM_PLAIN, Z, cap, "cuda")
    torch.cuda.synchronize()
    t = time.time()
    fm.fm_search_both(idx, codes, offs, z, fm.FM_BOTH, flags | fm.FM_PLAIN, Z, cap, out=pex, bufs=pbufs)
    torch.cuda.synchronize()
    plain_s = time.time() - t
    n0 = hits_per_batch[0]
    plain_equal = bool(torch.equal(pex, eager[0][0]) and torch.equal(pbufs.hit_offs, eager[0][1])
                       and torch.equal(pbufs.status[:B], eager[0][2]) and torch.equal(pbufs.hits[:n0], eager[0][3]))
    del pex, pbufs
    log("genome scale: eager pass with counters done; plain kernels %.1f ms, identical: %s" % (
        plain_s * 1e3, plain_equal))

    # one graph per batch, captured while phase timing is on so that every replay records
    # the boundaries of its D walk, DFS and compaction on the replay stream
    idx.phase_timing(1)
    try:
        plans = [fm.Plan.both(idx, codes, offs, z, fm.FM_BOTH, flags, Z, ex, bufs) for codes, z, ex, bufs in batches]
        timed_events = True
    except fm.FmError as e:
        log("graphs with phase events could not be captured (%s); capturing them without" % e)
        idx.phase_timing(0)
        plans = [fm.Plan.both(idx, codes, offs, z, fm.FM_BOTH, flags, Z, ex, bufs) for codes, z, ex, bufs in batches]
        timed_events = False
    idx.phase_timing(0)
    phase_sum = {"d_walk": 0.0, "dfs": 0.0, "compaction": 0.0}
    phase_n = 0

    def collect(b):
        nonlocal phase_n, timed_events
        if not timed_events:
            return
        try:
            ph = plans[b].phase_times()
        except fm.FmError as e:
            log("phase events of the replays could not be read (%s)" % e)
            timed_events = False
            return
        for k in phase_sum:
            phase_sum[k] += ph[k]
        phase_n += 1

    for s in range(args.warmup):
        plans[s % NB].launch()
    torch.cuda.synchronize()
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(2)]
    K = args.steps
    ev[0].record()
    for s in range(K):
        b = s % NB
        if s >= NB:
            collect(b)           # the replay NB steps back has been queued long before: no idle gap
        plans[b].launch()
    ev[1].record()
    torch.cuda.synchronize()
    total_ms = ev[0].elapsed_time(ev[1])
    for s in range(max(0, K - NB), K):
        collect(s % NB)
    phase_source = "the graphs' own phase events on every timed replay"
    if not timed_events or phase_n != K:
        # the DFS duration from eager calls of the same batches with the index's phase events
        phase_source = "eager calls of the same batches after the timed region (index phase events)"
        idx.phase_timing(NB)
        for codes, z, ex, bufs in batches:
            fm.fm_search_both(idx, codes, offs, z, fm.FM_BOTH, flags, Z, cap, out=ex, bufs=bufs)
        torch.cuda.synchronize()
        ph, _ = idx.phase_times()
        idx.phase_timing(0)
        phase_sum = {k: ph[k] / NB * K for k in phase_sum}
    # The same replays on two streams, batch b on stream b % 2 (a plan's replays stay in order
    # on one stream; consecutive batches share no buffer): one batch's search then runs in
    # the capacity the other's tail leaves idle. Reported beside the headline, which keeps one
    # stream so that each DFS launch's duration (the roofline's) is its own. The two streams
    # come from the HIP runtime and are destroyed afterwards: a process has few hardware
    # queues (4 by default), streams that torch creates hold theirs until the process ends,
    # and streams created later (the serving leg's) then share queues and lose their overlap.
    two_stream = None
    if NB % 2 == 0 and not args.skip_two_stream:
        main = torch.cuda.current_stream()
        hip = ctypes.CDLL("libamdhip64.so.7")
        raw = [ctypes.c_void_p() for _ in range(2)]
        for r in raw:
            if hip.hipStreamCreateWithFlags(ctypes.byref(r), ctypes.c_uint(1)) != 0:   # hipStreamNonBlocking
                raise RuntimeError("hipStreamCreateWithFlags failed")
        pair = [torch.cuda.ExternalStream(r.value) for r in raw]
        ev[0].record()
        for st in pair:
            st.wait_stream(main)
        for s in range(K):
            plans[s % NB].launch(stream=pair[(s % NB) % 2])
        for st in pair:
            main.wait_stream(st)
        ev[1].record()
        torch.cuda.synchronize()
        t2 = ev[0].elapsed_time(ev[1])
        del pair
        for r in raw:
            if hip.hipStreamDestroy(r) != 0:
                raise RuntimeError("hipStreamDestroy failed")
        two_stream = {"ms_per_step": round(t2 / K, 4), "reads_per_s": round(K * B / (t2 / 1e3), 1)}
        log("genome scale on two streams: %d steps in %.1f ms (%.3f ms/step)" % (K, t2, t2 / K))
    replay_equal = all(bool(torch.equal(ex, e[0]) and torch.equal(bufs.hit_offs, e[1])
                            and torch.equal(bufs.status[:B], e[2]) and torch.equal(bufs.hits[:e[3].shape[0]], e[3]))
                       for (codes, z, ex, bufs), e in zip(batches, eager))
    ms_step = total_ms / K
    phase = {k: v / K for k, v in phase_sum.items()}
    ceiling = random_read_ceiling(fm, torch, idx)
    log("random 32-byte reads: %s per second" % ceiling)
    log("genome scale: %d steps of %d reads in %.1f ms (%.3f ms/step), phases %s, replays identical: %s" % (
        K, B, total_ms, ms_step, phase, replay_equal))
    for p in plans:
        p.free()

    # roofline of the DFS: algorithmic bytes per launch (its bucket fetches at 32 B, its
    # prefix-table reads at 32 B, the patterns read twice, 32 B per read-strand of records,
    # 16 B per hit), averaged over the batches, over its average duration in the timed region
    nrs = 2 * B
    alg = ((work["buckets"] + work["table"]) * 32 + NB * (2 * B * LEN + 32 * nrs) + 16 * sum(hits_per_batch)) / NB
    achieved = alg / (phase["dfs"] / 1e3) / 1e9
    tcfg = tuning["inexact"]
    key = (kernel_source_hash(), dfs_kernel_name(tcfg, Z), tuple(tcfg[f] for f in TRAFFIC_KEY_FIELDS), "3.1e9/%d" % B)
    traffic = MEASURED_TRAFFIC.get(key)
    index_bytes = idx.info()["device_bytes"]
    roofline = {"bound": residency_bound(index_bytes), "kernel": key[1], "achieved": round(achieved, 1),
                "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4),
                "traffic": int(sum(traffic)) if traffic else None,
                "traffic_gb_per_s": round(sum(traffic) / (phase["dfs"] / 1e3) / 1e9, 1) if traffic else None,
                "bytes_per_launch": int(alg), "avg_launch_ms": round(phase["dfs"], 3),
                "kernel_source_hash": key[0], "index_bytes": int(index_bytes), "duration_from": phase_source}
    # The DFS's fetches against the rate the device serves independent random 32-byte reads
    # over a span like the one it reads (the 1.55 GB forward layout and the prefix table)
    fetch_rate = (work["buckets"] + work["table"]) / NB / (phase["dfs"] / 1e3)
    roofline["random_read_ceiling"] = {
        "reads_per_s_by_span": ceiling,
        "dfs_fetches_per_s": round(fetch_rate, 1),
        "dfs_line_requests_per_s": round(traffic[0] / 128 / (phase["dfs"] / 1e3), 1) if traffic else None,
        "dfs_fetches_vs_2_GiB": round(fetch_rate / ceiling["2 GiB"], 3),
        "probe": "fm_probe_random_reads: 16 waves per CU, 4 reads of one random 32-byte block in flight per lane",
    }

    # text positions of the first batch's hits (Eq. 4-5)
    codes, z, ex, bufs = batches[0]
    gloc = locate_rate(fm, torch, idx, bufs.hits, hits_per_batch[0])
    # the same index under independent random Occ8 queries, and the search's own queries
    occ8 = {}
    nq = 1 << 26
    ex_cfg = idx.get_tuning(fm.FM_OP_EXACT)
    qsets = {"uniform": synth.occ8_queries(R.size, nq, 4343, "uniform"),
             "narrow": synth.occ8_queries(R.size, nq, 4343, "narrow")}
    trace_info = None
    if args.occ8_queries:
        tcount = min(B, max(1000, args.genome_trace_reads))
        trace, (tc, to, tz, tlen) = search_trace(fm, torch, idx, rd, tcount, "cuda")
        tb = fm.InexactBuffers(idx, tcount, tlen, flags, Z, 16 * tcount, "cuda")
        fm.fm_search_inexact(idx, tc, to, tz, flags | fm.FM_STATS, Z, 16 * tcount, bufs=tb)
        torch.cuda.synchronize()
        trace_info = {"reads": tcount, "queries": int(trace.shape[0]),
                      "equals_dfs_node_count": int(trace.shape[0]) == tb.stats()["occ8"]}
        qsets["search_trace"] = trace
        del tb, tc, to, tz
    for kind, qh in qsets.items():
        q = torch.from_numpy(qh.view(np.int32)).cuda()
        qo = torch.empty((qh.shape[0], 8), dtype=torch.int32, device="cuda")
        for lanes in (1, 2):                       # the best of one and two lanes per query
            idx.set_tuning(fm.FM_OP_EXACT, lanes=lanes)
            fm.fm_occ8(idx, q, out=qo)
            torch.cuda.synchronize()
            ev[0].record()
            for _ in range(3):
                fm.fm_occ8(idx, q, out=qo)
            ev[1].record()
            torch.cuda.synchronize()
            occ8[kind] = max(occ8.get(kind, 0.0), qh.shape[0] / (ev[0].elapsed_time(ev[1]) / 3 / 1e3))
        del q, qo
    idx.set_tuning(fm.FM_OP_EXACT, **ex_cfg)
    del qsets

    # the oracle's text-only checkers on a sample (the first 1,000 reads and 1,000 spread
    # over the set), timed on the host, and the GPU's results for those reads checked
    cpu = parity = None
    if args.cpu_sample > 0:
        sample = np.unique(np.concatenate([np.arange(args.genome_cpu_sample // 2),
                                           np.linspace(args.genome_cpu_sample // 2, NB * B - 1,
                                                       args.genome_cpu_sample // 2).astype(np.int64)]))
        got_ex = np.zeros((sample.size * 2, 2), np.uint32)
        got = []
        host = [None] * NB
        for j, r in enumerate(sample):
            b, i = divmod(int(r), B)
            if host[b] is None:
                e = eager[b]
                h = e[3].cpu().numpy().view(np.uint32).reshape(-1, 4).copy().view(fm.HIT_DTYPE).reshape(-1)
                host[b] = (e[0].cpu().numpy().view(np.uint32), e[1].cpu().numpy().view(np.uint64), h)
            exb, ob, hb = host[b]
            got_ex[2 * j:2 * j + 2] = exb[2 * i:2 * i + 2]
            got.append(hb[int(ob[i]):int(ob[i + 1])])
        cpu, parity = genome_cpu_baseline(R, rd.subset(sample), got_ex, got, args.cpu_threads)
    del eager, batches, codes_all, z_all, offs
    idx.free()
    torch.cuda.empty_cache()
    reads_s = B / (ms_step / 1e3)
    return {
        "value": round(reads_s, 1),
        "ms_per_step": round(ms_step, 4),
        "config": {"workload": "3.1e9-base reference (55%% i.i.d., 45%% copies of 500 repeat families, 5-15%% "
                               "divergence); %d batches of %d reads x 150 bp, 1%% substitutions, either strand, "
                               "all resident in HBM; exact + z=2 substitution search, both strands, D-array "
                               "pruning; one launch graph per batch, replayed; a step is one batch" % (NB, B),
                   "n": int(R.size), "reads": NB * B, "batch_reads": B, "read_len": LEN, "z": Z, "strands": 2,
                   "d_bound": True, "hit_cap_per_batch": cap, "graph_replay": True},
        "roofline": roofline,
        "cpu_baseline": cpu,
        "parity_sample": parity,
        "extra": {
            "plain_reads_per_s": round(B / plain_s, 1),
            "batched_vs_plain": round(plain_s * 1e3 / ms_step, 3),
            "batched_equals_plain": plain_equal,
            "replay_equals_eager": replay_equal,
            "all_status_ok": all_ok,
            "hits": int(sum(hits_per_batch)),
            "index_build_s": round(build_s, 2),
            "phase_ms_per_step": {k: round(v, 3) for k, v in phase.items()},
            "work_per_batch": {"dfs_nodes": work["occ8"] // NB, "dfs_buckets": work["buckets"] // NB,
                               "dfs_table_nodes": work["table"] // NB,
                               "d_walk_steps": work["walk_steps"] // NB, "d_walk_buckets": work["walk_buckets"] // NB,
                               "dfs_subtrees_taken_over": work["subtrees"] // NB},
            "dfs_occ8_per_s": round(work["occ8"] / NB / (phase["dfs"] / 1e3), 1),
            "dfs_buckets_per_s": round(work["buckets"] / NB / (phase["dfs"] / 1e3), 1),
            "occ8_queries_per_s": {"fm_occ8_" + k: round(v, 1) for k, v in occ8.items()},
            "occ8_search_trace": trace_info,
            "two_stream_replay": two_stream,
            "locate_first_batch": gloc,
            "tuning": tuning,
        },
    }


def genome_cpu_baseline(R, srd, got_ex, got_hits, threads):
    """The oracle at genome scale: its text-only checkers (exact intervals
    by a batched rank scan over the text, z-substitution hit sets by a pigeonhole seed pass
    and the rank scan), which need no suffix array, on `threads` host threads; also checks
    the GPU's results for the sampled reads bit for bit."""
    import oracle
    t0 = time.time()
    want_ex = oracle.exact_by_rank_scan_batch(R, srd.codes, srd.offs, oracle.BOTH, threads=threads)
    t1 = time.time()
    wh, wo = oracle.pigeonhole_hits_batch(R, srd.codes, srd.offs, srd.z, oracle.BOTH, threads=threads)
    t2 = time.time()
    ok_ex = bool(np.array_equal(got_ex, want_ex))
    ok_in = True
    for j in range(srd.count):
        a = got_hits[j]
        w = wh[int(wo[j]):int(wo[j + 1])]
        ok_in &= bool(np.array_equal(a["k"], w["k"]) and np.array_equal(a["l"], w["l"]) and
                      np.array_equal(a["strand"], w["strand"]) and np.array_equal(a["nmm"], w["d"]))
    dt = t2 - t0
    log("oracle text-only checkers: %d reads in %.1fs (rank scan %.1fs, pigeonhole %.1fs) on %d threads; "
        "exact equal %s, hits equal %s" % (srd.count, dt, t1 - t0, t2 - t1, threads, ok_ex, ok_in))
    # the same checkers on one thread (each pass is about one sweep of the text)
    one = None
    if threads > 1:
        u0 = time.time()
        one_ex = oracle.exact_by_rank_scan_batch(R, srd.codes, srd.offs, oracle.BOTH, threads=1)
        u1 = time.time()
        one_h, one_o = oracle.pigeonhole_hits_batch(R, srd.codes, srd.offs, srd.z, oracle.BOTH, threads=1)
        u2 = time.time()
        one = {"reads_per_s": round(srd.count / (u2 - u0), 1),
               "seconds": {"rank_scan": round(u1 - u0, 2), "pigeonhole": round(u2 - u1, 2)},
               "same_results": bool(np.array_equal(one_ex, want_ex) and np.array_equal(one_h, wh)
                                    and np.array_equal(one_o, wo))}
        log("oracle text-only checkers on one thread: %.1fs (rank scan %.1fs, pigeonhole %.1fs)" % (
            u2 - u0, u1 - u0, u2 - u1))
    cpu = {"value": round(srd.count / dt, 1), "unit": "reads/s", "cores": threads, "kind": "oracle",
           "sample": "%d reads of the 16M (the first %d and %d spread over the set); the oracle's text-only "
                     "checkers, which need no index: exact intervals of both strands by a batched rank scan "
                     "over the 3.1e9-base text, z=2 hit sets by a pigeonhole seed pass plus rank scans; both "
                     "passes cost about one sweep of the text whatever the sample, so this rate grows with "
                     "the sample" % (srd.count, srd.count // 2, srd.count - srd.count // 2),
           "seconds": {"rank_scan": round(t1 - t0, 2), "pigeonhole": round(t2 - t1, 2)},
           "single_thread": one, "host": host_info()}
    parity = {"reads": srd.count, "exact_bit_exact": ok_ex, "inexact_bit_exact": ok_in,
              "exact_hits": int((want_ex[:, 0] <= want_ex[:, 1]).sum()), "hits": int(wh.size)}
    return cpu, parity


def host_info() -> dict:
    model = ""
    try:
        with open("/proc/cpuinfo") as f:
            model = next((l.split(":", 1)[1].strip() for l in f if l.startswith("model name")), "")
    except OSError:
        pass
    return {"cpu_model": model, "nproc": os.cpu_count()}


def residency_bound(index_bytes: int) -> str:
    """'hbm' when the index (both directions) is far larger than the last-level caches
    (8 x 4 MB of L2 and 256 MB of MALL), so that random bucket fetches are served from HBM;
    'cache' when it fits in them and the HBM fraction measures cache-served bytes."""
    return "hbm" if index_bytes > 4 * (256 << 20) else "cache"


def layout_rates(fm, torch, idx, step, ex_out, bufs, nreads, ref) -> dict:
    """The step at every bucket layout of the index (one lane per read-strand, D walk at the
    same layout): ms and reads/s, and agreement with the tuned run's output."""
    ops = (fm.FM_OP_INEXACT, fm.FM_OP_DARRAY)
    saved = [idx.get_tuning(op) for op in ops]
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(2)]
    out = {}
    try:
        for I in (64, 96, 128, 192, 224, 256, 448):
            for op in ops:
                idx.set_tuning(op, occ_interval=I, lanes=1)
            step()
            torch.cuda.synchronize()
            ev[0].record()
            for _ in range(3):
                step()
            ev[1].record()
            torch.cuda.synchronize()
            ms = ev[0].elapsed_time(ev[1]) / 3
            same = bool(torch.equal(ex_out, ref[0])) and all(
                np.array_equal(a, b) for a, b in zip(fm.hits_to_numpy(bufs, nreads), ref[1]))
            out[str(I)] = {"ms": round(ms, 4), "reads_per_s": round(nreads / (ms / 1e3), 1), "identical": same}
    finally:
        for op, t in zip(ops, saved):
            idx.set_tuning(op, **t)
    return out


def full_rank_rate(fm, torch, idx, codes, offs, nreads, ws, args) -> dict:
    """Full-rank exact search (FM_FULL_RANK: Listing 1 takes every step and a miss reports
    its rank) of the step's reads on both strands: batched and plain, bit-identical."""
    flags = fm.FM_BOTH | fm.FM_FULL_RANK
    out = torch.empty((2 * nreads, 2), dtype=torch.int32, device=codes.device)
    fm.fm_search_exact(idx, codes, offs, flags | fm.FM_STATS, out=out, ws=ws)
    torch.cuda.synchronize()
    steps = fm.exact_stats(ws)["steps"]
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(2)]
    res = {}
    for name, extra, reps in (("batched", 0, args.steps), ("plain", fm.FM_PLAIN, max(args.plain_steps, 1))):
        fm.fm_search_exact(idx, codes, offs, flags | extra, out=out, ws=ws)
        torch.cuda.synchronize()
        ev[0].record()
        for _ in range(reps):
            fm.fm_search_exact(idx, codes, offs, flags | extra, out=out, ws=ws)
        ev[1].record()
        torch.cuda.synchronize()
        res[name] = (ev[0].elapsed_time(ev[1]) / reps, out.clone())
    ms, pms = res["batched"][0], res["plain"][0]
    return {"workload": "the step's 1M reads x 100 bp, both strands; every step taken, misses report their rank",
            "ms": round(ms, 4), "reads_per_s": round(nreads / (ms / 1e3), 1),
            "plain_reads_per_s": round(nreads / (pms / 1e3), 1), "batched_vs_plain": round(pms / ms, 3),
            "batched_equals_plain": bool(torch.equal(res["batched"][1], res["plain"][1])),
            "steps": steps, "steps_per_s": round(steps / (ms / 1e3), 1)}


def gapped_z2_rate(fm, torch, idx, rd, args, count: int = 200_000) -> dict:
    """Listing 2 with all its branches at z=2 edits on the step's first 200K reads, both
    strands, D bound: the hit capacity is sized from the first call's required count (a
    call whose hits overflow reports the total every read needs), then batched and plain
    are timed and compared."""
    flags = fm.FM_BOTH | fm.FM_DARRAY | fm.FM_GAPS
    sub = rd.subset(np.arange(min(count, rd.count)))
    n = sub.count
    codes, offs, _ = fm.reads_to_device(sub.codes, sub.offs, sub.z)
    z = torch.full((n,), 2, dtype=torch.uint8, device="cuda")
    cap = 16 * n
    gb = fm.InexactBuffers(idx, n, int(sub.offs[-1]), flags, 2, cap, "cuda")
    fm.fm_search_inexact(idx, codes, offs, z, flags, 2, cap, bufs=gb)
    torch.cuda.synchronize()
    first_cap, need = cap, gb.required()
    if need > cap:
        cap = need
    gb = fm.InexactBuffers(idx, n, int(sub.offs[-1]), flags | fm.FM_PLAIN, 2, cap, "cuda")
    fm.fm_search_inexact(idx, codes, offs, z, flags | fm.FM_STATS, 2, cap, bufs=gb)
    torch.cuda.synchronize()
    st = gb.stats()
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(2)]
    res = {}
    for name, extra, reps in (("batched", 0, 3), ("plain", fm.FM_PLAIN, 1)):
        fm.fm_search_inexact(idx, codes, offs, z, flags | extra, 2, cap, bufs=gb)
        torch.cuda.synchronize()
        ev[0].record()
        for _ in range(reps):
            fm.fm_search_inexact(idx, codes, offs, z, flags | extra, 2, cap, bufs=gb)
        ev[1].record()
        torch.cuda.synchronize()
        res[name] = (ev[0].elapsed_time(ev[1]) / reps, fm.hits_to_numpy(gb, n))
    hits, _, status = res["batched"][1]
    out = {"workload": "the step's first %d reads x 100 bp; z=2 edits, both strands, D bound; one hit per interval"
                       % n,
           "reads": n, "ms": round(res["batched"][0], 3), "reads_per_s": round(n / res["batched"][0] * 1e3, 1),
           "plain_reads_per_s": round(n / res["plain"][0] * 1e3, 1),
           "batched_vs_plain": round(res["plain"][0] / res["batched"][0], 3),
           "batched_equals_plain": all(np.array_equal(a, b) for a, b in zip(res["batched"][1], res["plain"][1])),
           "hits": int(hits.size), "all_ok": bool((status == fm.FM_OK).all()),
           "hit_capacity": {"first_call": first_cap, "required_before_merging": int(need), "used": cap,
                            "required_per_read": round(need / n, 2)},
           "dfs_nodes": st["occ8"], "dfs_buckets": st["buckets"]}
    del gb, codes, offs, z
    torch.cuda.empty_cache()
    return out


def gapped_rate(fm, torch, idx, codes, offs, z, nreads, total_len, args) -> dict:
    """Listing 2 with its deletion and insertion branches (FM_GAPS), z=1 edits, both
    strands, D bound, on the step's reads: batched and plain, bit-identical."""
    flags = fm.FM_BOTH | fm.FM_DARRAY | fm.FM_GAPS
    cap = 16 * nreads
    gb = fm.InexactBuffers(idx, nreads, total_len, flags | fm.FM_PLAIN, 1, cap, codes.device)

    def call(extra=0):
        fm.fm_search_inexact(idx, codes, offs, z, flags | extra, 1, cap, bufs=gb)

    call(fm.FM_STATS)
    torch.cuda.synchronize()
    st = gb.stats()
    idx.phase_timing(3)
    for _ in range(3):
        call()
    torch.cuda.synchronize()
    ph, _ = idx.phase_times()
    idx.phase_timing(0)
    dfs_ms = ph["dfs"] / 3
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(2)]
    out = {}
    for name, extra, reps in (("batched", 0, args.steps), ("plain", fm.FM_PLAIN, max(args.plain_steps, 1))):
        call(extra)
        torch.cuda.synchronize()
        ev[0].record()
        for _ in range(reps):
            call(extra)
        ev[1].record()
        torch.cuda.synchronize()
        out[name] = (ev[0].elapsed_time(ev[1]) / reps, fm.hits_to_numpy(gb, nreads))
    equal = all(np.array_equal(a, b) for a, b in zip(out["batched"][1], out["plain"][1]))
    hits, _, status = out["batched"][1]
    res = {"workload": "the step's 1M reads x 100 bp; z=1 edit (substitution, deletion or insertion), both strands, "
                       "D bound; one hit per interval",
           "ms": round(out["batched"][0], 4), "reads_per_s": round(nreads / (out["batched"][0] / 1e3), 1),
           "plain_reads_per_s": round(nreads / (out["plain"][0] / 1e3), 1),
           "batched_vs_plain": round(out["plain"][0] / out["batched"][0], 3), "batched_equals_plain": equal,
           "hits": int(hits.size), "all_ok": bool((status == fm.FM_OK).all()),
           "dfs_nodes": st["occ8"], "dfs_buckets": st["buckets"],
           "phase_ms": {"d_walk": round(ph["d_walk"] / 3, 4), "dfs": round(dfs_ms, 4),
                        "compaction": round(ph["compaction"] / 3, 4)},
           # the DFS kernel: 32 B buckets, read codes, D records, counts and statuses, hits
           "dfs_algorithmic_gb_per_s": round((st["buckets"] * 32 + 2 * total_len + 24 * 2 * nreads +
                                              16 * int(hits.size)) / (dfs_ms / 1e3) / 1e9, 1)}
    del gb
    return res


def serve_bench(args):
    """Serving on the 2^28-base index (95% i.i.d., 5% diverged copies, 1% tandem repeats):
    requests of U{1..20,000} reads with lengths U[50, 250], 0.5-3% substitutions and
    budgets z in {0, 1, 2}, both strands with the D bound, arriving as a Poisson stream
    at `serve_load` times the capacity measured with every request queued at once.
    Latency runs from submission to results in host memory (server clock)."""
    import threading

    import synth
    from paper_1811_06127_amd import fm

    t0 = time.time()
    R = synth.repeats_2e28_reference()
    idx = fm.Index.from_text(R, occ_interval=64,
                             flags=fm.FM_LOAD_REVERSE | fm.FM_LOAD_DEVICE_SORT | fm.FM_LOAD_ALL_LAYOUTS)
    log("serving index (n=%d) built in %.1fs (suffixes sorted on the device)" % (R.size, time.time() - t0))
    t0 = time.time()
    pool = synth.mixed_reads_2e28(R, args.serve_pool, seed=3005)
    rng = synth.Rng(3105)
    nreq = args.serve_requests
    sizes = rng.integers(1, 20_000, nreq)
    starts = np.minimum((rng.uniform(nreq) * (pool.count - sizes + 1)).astype(np.int64), pool.count - sizes)
    gaps = rng.exponential(1.0, nreq)                     # unit-rate gaps, scaled below
    reqs = []
    for s0, n in zip(starts, sizes):
        lo, hi = int(pool.offs[s0]), int(pool.offs[s0 + n])
        reqs.append((pool.codes[lo:hi], pool.offs[s0:s0 + n + 1] - np.uint64(lo), pool.z[s0:s0 + n]))
    log("serving requests drawn in %.1fs: %d requests, %d reads" % (time.time() - t0, nreq, int(sizes.sum())))
    mixed = batch_2e28(idx, R, args)
    opts = dict(lanes=args.serve_lanes, flags=fm.FM_BOTH | fm.FM_DARRAY, zmax=2, hit_reserve=4,
                arena_bytes=4 << 30, ring_bytes=1 << 30)
    mean_size = float(sizes.mean())

    srv = fm.Server(idx, **opts)
    # capacity: the first requests all queued at once
    warm = [srv.submit(*r) for r in reqs[:20]]
    for t in warm:
        srv.wait(t)
        srv.release(t)
    m = min(200, nreq)

    def drain_rate():
        c0 = srv.clock()
        tick = [srv.submit(*r) for r in reqs[:m]]
        last = 0.0
        for t in tick:
            last = max(last, srv.wait(t).t_done)
            srv.release(t)
        return float(sizes[:m].sum()) / (last - c0)

    # the median of three drains: a single one varied by up to 7% between runs, and the
    # 0.95 load sits close enough to saturation for that to decide its tail
    rates = sorted(drain_rate() for _ in range(3))
    capacity = rates[1]
    log("serving capacity %.3g reads/s (drains %s); arrival rate %.1f requests/s" % (
        capacity, ["%.3g" % r for r in rates], args.serve_load * capacity / mean_size))

    def run_load(load, count=nreq):
        """The first `count` requests once each, Poisson arrivals at `load` times the
        capacity; returns the results in submission order."""
        arrivals = np.cumsum(gaps / (load * capacity / mean_size))
        results = [None] * count
        tickets = [None] * count
        ready = threading.Semaphore(0)

        def producer():
            base = time.perf_counter()
            for i, r in enumerate(reqs[:count]):
                d = base + arrivals[i] - time.perf_counter()
                if d > 0:
                    time.sleep(d)
                tickets[i] = srv.submit(*r)
                ready.release()

        th = threading.Thread(target=producer)
        th.start()
        for i in range(count):
            ready.acquire()
            results[i] = srv.wait(tickets[i])
            srv.release(tickets[i])
        th.join()
        return results

    def summary(results):
        lat = np.array([r.latency for r in results]) * 1e3
        span = max(r.t_done for r in results) - min(r.t_submit for r in results)
        return {"reads_per_s": round(int(sizes.sum()) / span, 1), "p50_ms": round(float(np.percentile(lat, 50)), 3),
                "p99_ms": round(float(np.percentile(lat, 99)), 3), "mean_ms": round(float(lat.mean()), 3),
                "requests_per_batch": round(nreq / max(1, len({r.batch for r in results})), 2),
                "all_ok": all(r.error == fm.FM_OK for r in results)}

    # an unmeasured warm-up under load: the first loaded run was seen to be slower
    run_load(args.serve_load, min(nreq, 500))
    other = {}
    for load in (0.5, 0.95):
        if abs(load - args.serve_load) > 1e-9:
            other["%.2f" % load] = summary(run_load(load))
    results = run_load(args.serve_load)
    st = srv.stats()
    # a few requests again, alone: their results must not depend on the batch
    same = True
    for i in range(0, nreq, max(1, nreq // 8)):
        t = srv.submit(*reqs[i])
        a = srv.wait(t)
        srv.release(t)
        b = results[i]
        same &= bool(np.array_equal(a.status, b.status) and np.array_equal(a.hit_offs, b.hit_offs)
                     and a.hits.tobytes() == b.hits.tobytes())
    srv.close()
    idx.free()
    out = {"workload": "2^28-base reference (5%% copies, 1%% tandem repeats); Poisson arrivals at %.2f of "
                       "capacity; requests of U{1..20000} reads, length U[50,250], 0.5-3%% substitutions, z in "
                       "{0,1,2}; both strands, D bound" % args.serve_load,
           "requests": nreq, "reads": int(sizes.sum()), "lanes": args.serve_lanes,
           "capacity_reads_per_s": round(capacity, 1), "capacity_drains": [round(r, 1) for r in rates],
           **summary(results),
           "retries": st["retries"], "alone_equals_mixed": same, "other_loads": other, "mixed_batch": mixed}
    log("serving:", out)
    return out


def batch_2e28(idx, R, args):
    """The mixed-budget batch: 4M reads of the 2^28-base reference (lengths U[50, 250],
    0.5-3% substitutions, z in {0, 1, 2}) in one persistent launch of the inexact search,
    both strands with the D bound, with the layout and lanes chosen by the autotuner on a
    sample of the same reads, then the occupancy, claim order and prefix table on the whole
    batch; against the plain kernels. Also Occ8 rates on this index."""
    import torch

    import synth
    from paper_1811_06127_amd import fm

    t0 = time.time()
    pool = synth.mixed_reads_2e28(R, args.batch_reads)
    n = pool.count
    log("mixed-budget reads drawn in %.1fs: %d reads, %d bases" % (time.time() - t0, n, int(pool.offs[-1])))
    flags = fm.FM_BOTH | fm.FM_DARRAY
    cap = 6 * n
    saved = {op: idx.get_tuning(op) for op in (fm.FM_OP_INEXACT, fm.FM_OP_DARRAY)}
    tuning = {}
    if not args.no_tune:
        t0 = time.time()
        ts = pool.subset(np.arange(min(n, args.tune_sample)))
        tc, to, tz = fm.reads_to_device(ts.codes, ts.offs, ts.z)
        tb = fm.InexactBuffers(idx, ts.count, int(ts.offs[-1]), flags | fm.FM_PLAIN, 2, 6 * ts.count, "cuda")
        for name, op in (("inexact", fm.FM_OP_INEXACT), ("d_walk", fm.FM_OP_DARRAY)):
            cfg, ms = fm.fm_autotune(idx, op, tc, to, tz, flags, 2, bufs=tb, cache_path=args.tune_cache)
            tuning[name] = {"config": cfg, "ms_on_sample": ms}
        tuning["sample_reads"] = ts.count
        tuning["seconds"] = round(time.time() - t0, 1)
        log("mixed-budget batch autotuned on %d reads in %.1fs: %s" % (ts.count, time.time() - t0, tuning))
        del tb, tc, to, tz
    codes, offs, z = fm.reads_to_device(pool.codes, pool.offs, pool.z)
    bufs = fm.InexactBuffers(idx, n, int(pool.offs[-1]), flags | fm.FM_PLAIN, 2, cap, "cuda")
    if not args.no_tune:
        # the sample fixes the layout and lanes; occupancy, claim order and the prefix table
        # are then timed on the whole batch, whose launch tail weighs less than the sample's
        t0 = time.time()
        for name, op in (("inexact", fm.FM_OP_INEXACT), ("d_walk", fm.FM_OP_DARRAY)):
            cfg, ms = fm.fm_autotune(idx, op, codes, offs, z, flags | fm.FM_TUNE_KEEP_LAYOUT, 2, bufs=bufs,
                                     cache_path=args.tune_cache)
            tuning[name]["refined_on_batch"] = {"config": cfg, "ms": ms}
        tuning["refine_seconds"] = round(time.time() - t0, 1)
        log("refined on the whole batch in %.1fs: %s" % (time.time() - t0, tuning))

    def timed(extra, reps):
        fm.fm_search_inexact(idx, codes, offs, z, flags | extra, 2, cap, bufs=bufs)
        torch.cuda.synchronize()
        t0, t1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        t0.record()
        for _ in range(reps):
            fm.fm_search_inexact(idx, codes, offs, z, flags | extra, 2, cap, bufs=bufs)
        t1.record()
        torch.cuda.synchronize()
        return t0.elapsed_time(t1) / reps, fm.hits_to_numpy(bufs, n)

    fm.fm_search_inexact(idx, codes, offs, z, flags | fm.FM_STATS, 2, cap, bufs=bufs)
    torch.cuda.synchronize()
    st = bufs.stats()
    ms, hb = timed(0, 3)
    pms, hp = timed(fm.FM_PLAIN, 1)
    occ8 = {}
    nq = 1 << 26
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(2)]
    for kind in ("uniform", "narrow"):
        q = torch.from_numpy(synth.occ8_queries(R.size, nq, 4444, kind).view(np.int32)).cuda()
        qo = torch.empty((nq, 8), dtype=torch.int32, device="cuda")
        fm.fm_occ8(idx, q, out=qo)
        torch.cuda.synchronize()
        ev[0].record()
        for _ in range(3):
            fm.fm_occ8(idx, q, out=qo)
        ev[1].record()
        torch.cuda.synchronize()
        occ8["fm_occ8_" + kind] = round(nq / (ev[0].elapsed_time(ev[1]) / 3 / 1e3), 1)
        del q, qo
    out = {"workload": "2^28-base reference (5%% copies, 1%% tandem repeats); %d reads, length U[50,250], "
                       "0.5-3%% substitutions, z in {0,1,2} mixed in one persistent launch; both strands, D bound"
                       % n,
           "reads": n, "total_bases": int(pool.offs[-1]), "ms": round(ms, 3), "reads_per_s": round(n / ms * 1e3, 1),
           "plain_reads_per_s": round(n / pms * 1e3, 1), "batched_vs_plain": round(pms / ms, 3),
           "batched_equals_plain": all(np.array_equal(a, b) for a, b in zip(hb, hp)), "hits": int(hb[1][-1]),
           "all_ok": bool((hb[2] == fm.FM_OK).all()), "dfs_nodes": st["occ8"], "dfs_buckets": st["buckets"],
           "tuning": tuning or {"inexact": {"config": idx.get_tuning(fm.FM_OP_INEXACT)}},
           "occ8_queries_per_s": occ8}
    log("mixed-budget batch on the 2^28 index:", out)
    for op, t in saved.items():
        idx.set_tuning(op, **t)
    del bufs, codes, offs, z
    torch.cuda.empty_cache()
    return out


def small_exact(args):
    """The small workload: a 65,536-base i.i.d. reference and 10,000 exact queries of 32
    symbols (half copied from the reference, half random), forward strand, I=128: batched
    and plain rates, and the intervals against the oracle's (binary search over its suffix
    array)."""
    import torch

    import oracle
    import synth
    from paper_1811_06127_amd import fm

    w = synth.small_exact_workload()
    # the workload fixes the checkpoint interval, so only the I=128 layout is built and the
    # autotuner chooses lanes, depth and occupancy
    idx = fm.Index.from_text(w.ref, occ_interval=128)
    cd, od, _ = fm.reads_to_device(w.reads.codes, w.reads.offs)
    n = w.reads.count
    ws = torch.zeros(fm.fm_search_exact_workspace(idx, n, fm.FM_FWD), dtype=torch.uint8, device="cuda")
    out = torch.empty((n, 2), dtype=torch.int32, device="cuda")
    tuned = None if args.no_tune else fm.fm_autotune(idx, fm.FM_OP_EXACT, cd, od, None, fm.FM_FWD, out=out, ws=ws)
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(2)]
    res = {}
    reps = 200
    for name, extra in (("batched", 0), ("plain", fm.FM_PLAIN)):
        for _ in range(3):
            fm.fm_search_exact(idx, cd, od, fm.FM_FWD | extra, out=out, ws=ws)
        torch.cuda.synchronize()
        ev[0].record()
        for _ in range(reps):
            fm.fm_search_exact(idx, cd, od, fm.FM_FWD | extra, out=out, ws=ws)
        ev[1].record()
        torch.cuda.synchronize()
        res[name] = (ev[0].elapsed_time(ev[1]) / reps, out.cpu().numpy().view(np.uint32).copy())
    want = oracle.OracleIndex(w.ref).exact(w.reads.codes, w.reads.offs, oracle.FWD, "definition")
    idx.free()
    out = {"workload": "65,536-base i.i.d. reference; 10,000 exact queries of 32 (half copied, half random), "
                       "forward strand, I=128; the queries are too few to fill the chip, so this rate is launch-bound",
           "reads": n, "ms": round(res["batched"][0], 4), "reads_per_s": round(n / res["batched"][0] * 1e3, 1),
           "plain_reads_per_s": round(n / res["plain"][0] * 1e3, 1),
           "batched_vs_plain": round(res["plain"][0] / res["batched"][0], 3),
           "equals_oracle": bool(np.array_equal(res["batched"][1], want) and np.array_equal(res["plain"][1], want)),
           "hits": int((want[:, 0] <= want[:, 1]).sum()), "tuning": tuned[0] if tuned else None}
    log("small exact workload:", out)
    return out


def cpu_baseline(R, rd, sample, ex_batched, in_batched, threads):
    """The CPU oracle (Listing 1 exact + Listing 2 with the D bound) on the first `sample`
    reads of the same batch, split into equal parts searched by `threads` host threads
    (the oracle's searches release the interpreter lock); also checks the GPU's outputs
    for those reads."""
    import concurrent.futures as cf

    import oracle
    t0 = time.time()
    x = oracle.OracleIndex(R)
    xr = oracle.OracleIndex(oracle.reverse_text(R))
    log("oracle indexes built in %.1fs" % (time.time() - t0))
    s = rd.subset(np.arange(sample))
    bounds = np.linspace(0, sample, threads + 1).astype(np.int64)

    def part(i):
        p = s.subset(np.arange(bounds[i], bounds[i + 1]))
        ex = x.exact(p.codes, p.offs, oracle.BOTH, "listing1")
        h, o = x.inexact(p.codes, p.offs, p.z, oracle.BOTH, "listing2_darray", rev=xr)
        h["read"] += np.uint32(bounds[i])
        return ex, h, o

    t0 = time.time()
    with cf.ThreadPoolExecutor(max_workers=threads) as pool:
        parts = list(pool.map(part, range(threads)))
    dt = time.time() - t0
    log("oracle: %d reads in %.1fs on %d threads" % (sample, dt, threads))
    ex = np.concatenate([p[0] for p in parts])
    hits = np.concatenate([p[1] for p in parts])
    hoffs = np.zeros(sample + 1, dtype=np.uint64)
    for i, p in enumerate(parts):
        hoffs[bounds[i] + 1:bounds[i + 1] + 1] = p[2][1:] + hoffs[bounds[i]]
    gex = ex_batched[:2 * sample].cpu().numpy().view(np.uint32)
    gh, go, gs = in_batched
    n = int(go[sample])
    g = gh[:n]
    ok_ex = bool(np.array_equal(gex, ex))
    ok_in = bool(np.array_equal(go[:sample + 1], hoffs) and (gs[:sample] == 0).all()
                 and all(np.array_equal(g[f], hits[f]) for f in ("read", "k", "l", "strand"))
                 and np.array_equal(g["nmm"], hits["d"]))
    # one host thread on the first reads of the sample, for the per-core rate
    one = min(sample, 20_000)
    t0 = time.time()
    p1 = s.subset(np.arange(one))
    x.exact(p1.codes, p1.offs, oracle.BOTH, "listing1")
    x.inexact(p1.codes, p1.offs, p1.z, oracle.BOTH, "listing2_darray", rev=xr)
    dt1 = time.time() - t0
    model = ""
    try:
        with open("/proc/cpuinfo") as f:
            model = next((l.split(":", 1)[1].strip() for l in f if l.startswith("model name")), "")
    except OSError:
        pass
    cpu = {"value": round(sample / dt, 1), "unit": "reads/s", "cores": threads, "kind": "oracle",
           "sample": "first %d of the step's reads; exact (Listing 1) + z=1 inexact (Listing 2, D bound), "
                     "both strands, %d host threads, index prebuilt" % (sample, threads),
           "single_thread": {"reads_per_s": round(one / dt1, 1), "sample": "first %d reads" % one},
           "host": {"cpu_model": model, "nproc": os.cpu_count()}}
    parity = {"reads": sample, "exact_bit_exact": ok_ex, "inexact_bit_exact": ok_in}
    return cpu, parity


if __name__ == "__main__":
    main()
