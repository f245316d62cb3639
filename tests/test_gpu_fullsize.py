"""Parity at the workloads' full sizes, in the launch configuration the benchmark uses:
every output of the batched kernels equals the plain kernels' bit for bit, and sampled
outputs equal the oracle's (the full suffix-array oracle at 2^24 bases; at 2^28 bases the
text-only checkers: rank scan for intervals, pigeonhole windows for hit sets)."""
import time

import numpy as np
import pytest
import torch

import oracle
import synth
from paper_1811_06127_amd import fm

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)


def inexact_np(idx, codes, offs, z, flags, zmax, cap):
    bufs = fm.fm_search_inexact(idx, codes, offs, z, flags, zmax, cap)
    torch.cuda.synchronize()
    return fm.hits_to_numpy(bufs, offs.numel() - 1)


def same_hits(a, b):
    return all(np.array_equal(x, y) for x, y in zip(a, b))


def check_sampled_hits(got, want_hits, want_offs, sample, tag):
    hits, hoffs, status = got
    for i, r in enumerate(sample):
        assert status[r] == fm.FM_OK, (tag, r, status[r])
        g = hits[int(hoffs[r]):int(hoffs[r + 1])]
        w = want_hits[int(want_offs[i]):int(want_offs[i + 1])]
        assert g.size == w.size, (tag, r)
        for f in ("k", "l", "strand"):
            assert np.array_equal(g[f], w[f]), (tag, r, f)
        assert np.array_equal(g["nmm"], w["d"]), (tag, r)


@pytest.mark.timeout(900)
def test_headline_workload_full_size():
    """2^24-base text, 1M reads of 100 bp, exact + z=1 with the D bound, both strands."""
    t0 = time.time()
    R = synth.repeats_2e24_reference()
    rd = synth.reads_2e24(R)
    idx = fm.Index.from_text(R, occ_interval=64, flags=fm.FM_LOAD_REVERSE | fm.FM_LOAD_ALL_LAYOUTS)
    say("2^24 inputs and index in %.1fs" % (time.time() - t0))
    codes, offs, z = fm.reads_to_device(rd.codes, rd.offs, rd.z)
    n = rd.count
    ex_out = torch.empty((2 * n, 2), dtype=torch.int32, device="cuda")
    ex_ws = torch.zeros(fm.fm_search_exact_workspace(idx, n, fm.FM_BOTH), dtype=torch.uint8, device="cuda")
    bufs = fm.InexactBuffers(idx, n, int(rd.offs[-1]), fm.FM_BOTH | fm.FM_DARRAY | fm.FM_PLAIN, 1, 4 * n, "cuda")
    fm.fm_autotune(idx, fm.FM_OP_EXACT, codes, offs, None, fm.FM_BOTH, out=ex_out, ws=ex_ws)
    fm.fm_autotune(idx, fm.FM_OP_INEXACT, codes, offs, z, fm.FM_BOTH | fm.FM_DARRAY, 1, bufs=bufs)
    fm.fm_autotune(idx, fm.FM_OP_DARRAY, codes, offs, z, fm.FM_BOTH | fm.FM_DARRAY, 1, bufs=bufs)
    say("tuned", {op: idx.get_tuning(op) for op in (0, 1, 2)})
    fm.fm_search_exact(idx, codes, offs, fm.FM_BOTH, out=ex_out, ws=ex_ws)
    ex_b = ex_out.cpu().numpy().view(np.uint32).copy()
    fm.fm_search_exact(idx, codes, offs, fm.FM_BOTH | fm.FM_PLAIN, out=ex_out, ws=ex_ws)
    assert np.array_equal(ex_out.cpu().numpy().view(np.uint32), ex_b)
    in_b = inexact_np(idx, codes, offs, z, fm.FM_BOTH | fm.FM_DARRAY, 1, 4 * n)
    in_p = inexact_np(idx, codes, offs, z, fm.FM_BOTH | fm.FM_DARRAY | fm.FM_PLAIN, 1, 4 * n)
    assert same_hits(in_b, in_p)
    assert (in_b[2] == fm.FM_OK).all()
    # both searches in one pass, as the benchmark's step runs them
    ex_f, bufs_f = fm.fm_search_both(idx, codes, offs, z, fm.FM_BOTH, fm.FM_BOTH | fm.FM_DARRAY, 1, 4 * n)
    torch.cuda.synchronize()
    assert np.array_equal(ex_f.cpu().numpy().view(np.uint32), ex_b)
    assert same_hits(fm.hits_to_numpy(bufs_f, n), in_b)
    del bufs_f
    say("batched == plain over %d reads; %d hits" % (n, int(in_b[1][-1])))
    # sampled reads against the full oracle
    t0 = time.time()
    x = oracle.OracleIndex(R)
    xr = oracle.OracleIndex(oracle.reverse_text(R))
    say("oracle indexes in %.1fs" % (time.time() - t0))
    sample = np.sort(synth.Rng(77).integers(0, n - 1, 2000))
    s = rd.subset(sample)
    want = x.exact(s.codes, s.offs, oracle.BOTH, "listing1")
    got = ex_b.reshape(n, 2, 2)[sample].reshape(-1, 2)
    assert np.array_equal(got, want)
    wh, wo = x.inexact(s.codes, s.offs, s.z, oracle.BOTH, "listing2_darray", rev=xr)
    check_sampled_hits(in_b, wh, wo, sample, "2^24")


@pytest.mark.timeout(1200)
def test_mixed_budget_workload_full_size():
    """2^28-base text with tandem repeats, 4M reads of 50-250 bp with budgets 0-2 in one
    persistent launch, tuned on a prefix of the batch."""
    t0 = time.time()
    R = synth.repeats_2e28_reference()
    idx = fm.Index.from_text(R, occ_interval=64,
                             flags=fm.FM_LOAD_REVERSE | fm.FM_LOAD_ALL_LAYOUTS | fm.FM_LOAD_DEVICE_SORT)
    say("2^28 index (device suffix sort) in %.1fs" % (time.time() - t0))
    t0 = time.time()
    rd = synth.mixed_reads_2e28(R)
    say("4M reads in %.1fs" % (time.time() - t0))
    n = rd.count
    flags = fm.FM_BOTH | fm.FM_DARRAY
    codes, offs, z = fm.reads_to_device(rd.codes, rd.offs, rd.z)
    # tune on the first 250K reads, as a server would on a representative batch
    m = 250_000
    tc, to, tz = fm.reads_to_device(rd.codes[:int(rd.offs[m])], rd.offs[:m + 1], rd.z[:m])
    tb = fm.InexactBuffers(idx, m, int(rd.offs[m]), flags | fm.FM_PLAIN, 2, 8 * m, "cuda")
    fm.fm_autotune(idx, fm.FM_OP_INEXACT, tc, to, tz, flags, 2, bufs=tb)
    fm.fm_autotune(idx, fm.FM_OP_DARRAY, tc, to, tz, flags, 2, bufs=tb)
    del tb, tc, to, tz
    say("tuned", {op: idx.get_tuning(op) for op in (1, 2)})
    cap = 6 * n
    in_b = inexact_np(idx, codes, offs, z, flags, 2, cap)
    say("batched: %d hits, statuses %s" % (int(in_b[1][-1]), np.unique(in_b[2]).tolist()))
    in_p = inexact_np(idx, codes, offs, z, flags | fm.FM_PLAIN, 2, cap)
    assert same_hits(in_b, in_p)
    ex_out = torch.empty((2 * n, 2), dtype=torch.int32, device="cuda")
    ex_ws = torch.zeros(fm.fm_search_exact_workspace(idx, n, fm.FM_BOTH), dtype=torch.uint8, device="cuda")
    fm.fm_search_exact(idx, codes, offs, fm.FM_BOTH, out=ex_out, ws=ex_ws)
    ex_b = ex_out.cpu().numpy().view(np.uint32).copy()
    fm.fm_search_exact(idx, codes, offs, fm.FM_BOTH | fm.FM_PLAIN, out=ex_out, ws=ex_ws)
    assert np.array_equal(ex_out.cpu().numpy().view(np.uint32), ex_b)
    say("batched == plain over %d reads" % n)
    # sampled outputs against the oracle's batched text-only checkers (rank scan for the
    # exact intervals, pigeonhole windows for the hit sets): every budget and read-length
    # quartile, random reads, reads with hits and repeat-rich reads (several hits or an
    # exact interval of several rows), 2,000 and more in all
    ex_rows = ex_b.reshape(n, 2, 2)
    exact_rows = np.where(ex_rows[:, :, 0] <= ex_rows[:, :, 1], ex_rows[:, :, 1] - ex_rows[:, :, 0] + 1, 0).max(1)
    sample = stratified_sample(rd, in_b[1], exact_rows, seed=78)
    check_against_text(R, rd, sample, ex_rows, in_b, "2^28")


def stratified_sample(rd, hit_offs, exact_rows, seed, counts=(100, 50, 20)):
    """Reads of every budget and length quartile: (by default) 100 random, 50 with hits and
    20 repeat-rich ones (5 hits or more, or an exact interval of 2 rows or more) per stratum."""
    rng = synth.Rng(seed)
    lens = np.diff(rd.offs.astype(np.int64))
    nh = np.diff(hit_offs.astype(np.int64))
    edges = np.quantile(lens, [0.25, 0.5, 0.75])
    qb = np.searchsorted(edges, lens, side="right")
    pick = []
    for zv in (0, 1, 2):
        for q in range(4):
            inside = (rd.z == zv) & (qb == q)
            rich = inside & ((nh >= 5) | (exact_rows >= 2))
            for cond, k in zip((inside, inside & (nh > 0), rich), counts):
                ids = np.nonzero(cond)[0]
                pick.append(ids[np.argsort(rng.uniform(ids.size), kind="stable")[:k]])   # without replacement
    sample = np.unique(np.concatenate(pick))
    assert sample.size >= 2000, sample.size
    return sample


def check_against_text(R, rd, sample, ex_rows, got, tag):
    s = rd.subset(sample)
    t0 = time.time()
    want = oracle.exact_by_rank_scan_batch(R, s.codes, s.offs, oracle.BOTH, threads=16)
    assert np.array_equal(ex_rows[sample].reshape(-1, 2), want), tag
    wh, wo = oracle.pigeonhole_hits_batch(R, s.codes, s.offs, s.z, oracle.BOTH, threads=16)
    check_sampled_hits(got, wh, wo, sample, tag)
    nh = np.diff(wo.astype(np.int64))
    say("%s: %d sampled reads checked by the text-only checkers in %.1fs: budgets %s, %d with hits, %d hits, "
        "%d exact hits, most hits in one read %d" % (
            tag, sample.size, time.time() - t0, np.bincount(s.z, minlength=3).tolist(), int((nh > 0).sum()), wh.size,
            int((want[:, 0] <= want[:, 1]).sum()), int(nh.max())))
    assert (nh > 0).sum() >= sample.size // 3          # the hit sets compared are not mostly empty


@pytest.mark.timeout(1200)
def test_serving_on_the_2e28_index():
    """The server on the 2^28-base index: 120 requests of 1..20,000 mixed reads (budgets
    0-2, lengths 50-250) submitted in bursts while earlier ones run on three lanes; 2,000 and more
    reads sampled across the served requests equal the oracle's text-only checkers, and
    requests served again alone are byte-identical to their results in the mix."""
    import threading

    t0 = time.time()
    R = synth.repeats_2e28_reference()
    idx = fm.Index.from_text(R, occ_interval=64, flags=fm.FM_LOAD_REVERSE | fm.FM_LOAD_DEVICE_SORT)
    pool = synth.mixed_reads_2e28(R, 600_000, seed=3005)
    rng = synth.Rng(3106)
    nreq = 120
    sizes = rng.integers(1, 20_000, nreq)
    starts = rng.integers(0, pool.count - 20_001, nreq)
    reqs = []
    for s0, k in zip(starts, sizes):
        lo, hi = int(pool.offs[s0]), int(pool.offs[s0 + k])
        reqs.append((pool.codes[lo:hi], pool.offs[s0:s0 + k + 1] - np.uint64(lo), pool.z[s0:s0 + k]))
    say("2^28 index and %d requests (%d reads) in %.1fs" % (nreq, int(sizes.sum()), time.time() - t0))
    flags = fm.FM_BOTH | fm.FM_DARRAY
    with fm.Server(idx, lanes=3, flags=flags, zmax=2, arena_bytes=2 << 30) as srv:
        tickets = []

        def producer():
            # bursts of 8: more than the 3 lanes take at once, so later requests of a
            # burst wait and are admitted together, however fast a batch is served
            for j, r in enumerate(reqs):
                tickets.append(srv.submit(*r))
                if j % 8 == 7:
                    time.sleep(0.001)

        th = threading.Thread(target=producer)
        th.start()
        th.join()
        results = []
        for t in tickets:
            results.append(srv.wait(t, timeout=120.0))
            srv.release(t)
        # a few requests again, alone
        alone = []
        for i in range(0, nreq, 15):
            t = srv.submit(*reqs[i])
            alone.append((i, srv.wait(t, timeout=60.0)))
            srv.release(t)
        st = srv.stats()
    assert st["error"] == 0 and st["requests_done"] == nreq + len(alone)
    assert len({r.batch for r in results}) < nreq                  # requests shared batches
    for i, a in alone:
        b = results[i]
        assert np.array_equal(a.status, b.status) and np.array_equal(a.hit_offs, b.hit_offs), i
        assert a.hits.tobytes() == b.hits.tobytes(), i
    say("served: %s; %d requests again alone, identical" % (st, len(alone)))
    # the served reads as one batch: its reads, hits and statuses in request order
    codes = np.concatenate([r[0] for r in reqs])
    lens = np.concatenate([np.diff(r[1].astype(np.int64)) for r in reqs])
    offs = np.zeros(lens.size + 1, np.uint64)
    np.cumsum(lens, out=offs[1:])
    z = np.concatenate([r[2] for r in reqs])
    rd = synth.Reads(codes, offs, z, np.full(z.size, -1), np.zeros(z.size, np.uint8))
    hits = np.concatenate([r.hits for r in results])
    per = np.concatenate([np.diff(r.hit_offs.astype(np.int64)) for r in results])
    hoffs = np.zeros(per.size + 1, np.uint64)
    np.cumsum(per, out=hoffs[1:])
    status = np.concatenate([r.status for r in results])
    assert (status == fm.FM_OK).all()
    # exact intervals are not served: the sample is stratified by budget and length only
    sample = stratified_sample(rd, hoffs, np.zeros(rd.count, np.int64), seed=79, counts=(120, 60, 25))
    s = rd.subset(sample)
    t0 = time.time()
    wh, wo = oracle.pigeonhole_hits_batch(R, s.codes, s.offs, s.z, oracle.BOTH, threads=16)
    check_sampled_hits((hits, hoffs, status), wh, wo, sample, "served 2^28")
    nh = np.diff(wo.astype(np.int64))
    say("served 2^28: %d sampled reads checked in %.1fs: budgets %s, %d with hits, %d hits, most in one read %d" % (
        sample.size, time.time() - t0, np.bincount(s.z, minlength=3).tolist(), int((nh > 0).sum()), wh.size,
        int(nh.max())))
    assert (nh > 0).sum() >= sample.size // 3
    idx.free()
