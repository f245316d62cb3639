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
    # sampled outputs against the text-only checkers: reads of every budget, most of them
    # among reads the GPU reports hits for, so that the hit sets compared are not empty
    rng = synth.Rng(78)
    has = np.diff(in_b[1]) > 0
    pick = []
    for v, k_any, k_hit in ((0, 1, 1), (1, 1, 2), (2, 1, 2)):
        any_v = np.nonzero(rd.z == v)[0]
        hit_v = np.nonzero((rd.z == v) & has)[0]
        pick += [any_v[rng.integers(0, any_v.size - 1, k_any)], hit_v[rng.integers(0, hit_v.size - 1, k_hit)]]
    sample = np.unique(np.concatenate(pick))
    s = rd.subset(sample)
    t0 = time.time()
    want = oracle.exact_by_rank_scan(R, s.codes, s.offs, oracle.BOTH)
    assert np.array_equal(ex_b.reshape(n, 2, 2)[sample].reshape(-1, 2), want)
    wh, wo = oracle.pigeonhole_hits(R, s.codes, s.offs, s.z, oracle.BOTH)
    say("text-only checks of %d reads in %.1fs: %d hits" % (sample.size, time.time() - t0, wh.size))
    check_sampled_hits(in_b, wh, wo, sample, "2^28")
