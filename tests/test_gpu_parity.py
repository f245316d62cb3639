"""Parity of the HIP kernels (through the C ABI) with the CPU oracle, element by element,
on seeded inputs that span many buckets and end in ragged tails."""
import itertools

import numpy as np
import pytest
import torch

import oracle
import synth
from paper_1811_06127_amd import fm

pytestmark = pytest.mark.gpu

LAYOUTS = (64, 96, 128, 192, 224, 256, 448)
LANES = {64: (1, 2), 96: (1, 2), 128: (1, 2, 4), 192: (1, 2, 4), 224: (1, 2, 4), 256: (1, 2, 4, 8),
         448: (1, 2, 4, 8)}


def say(*a):
    print(*a, flush=True)


@pytest.fixture(scope="module")
def small():
    """A 70,001-base text with repeats (ragged last bucket for every I), its oracle index
    and the reverse-text oracle index, and a GPU index with every layout."""
    R = synth.reference_with_repeats(70_001, 4242, copy_frac=0.08, copy_len=(300, 2000), copy_sub=0.02,
                                     tandem_frac=0.02, tandem_unit=(2, 12), tandem_len=(100, 400))
    x = oracle.OracleIndex(R)
    xr = oracle.OracleIndex(oracle.reverse_text(R))
    idx = fm.Index.from_text(R, occ_interval=128, flags=fm.FM_LOAD_REVERSE | fm.FM_LOAD_ALL_LAYOUTS)
    say("small index built", idx.info())
    return R, x, xr, idx


def to_u32(t):
    return t.cpu().numpy().view(np.uint32)


def test_index_constants(small):
    R, x, xr, idx = small
    info = idx.info()
    assert info["n"] == R.size and info["dollar_row"] == x.dollar_row
    assert info["C"] == x.C.tolist()
    assert info["rev_dollar_row"] == xr.dollar_row and info["rev_C"] == xr.C.tolist()
    assert info["layouts"] == 127 and info["has_reverse"]


def occ8_queries(n, dollar):
    q = [synth.occ8_queries(n, 20_000, 7, "uniform"), synth.occ8_queries(n, 20_000, 8, "narrow")]
    edge = []
    for I in LAYOUTS:
        for b in range(0, n + 2, I * 37):
            for d in (-2, -1, 0, 1, 2):
                p = b + d
                if 0 <= p <= n:
                    edge += [(p, p), (p + 1, p), (0, p), (p, n), (max(p - 5, 0), p)]
    for p in (dollar - 1, dollar, dollar + 1):
        if 0 <= p <= n:
            edge += [(p, p), (p + 1, p), (0, p), (p + 1, n)]
    edge += [(0, 0), (0, n), (n + 1, n), (n, n), (1, 0), (n + 1, 0)]
    bad = [(n + 2, 0), (0, n + 1), (0xFFFFFFFF, 5), (3, 0xFFFFFFFF)]
    return np.concatenate(q + [np.array(edge + bad, np.uint32)])


@pytest.mark.parametrize("I", LAYOUTS)
def test_occ8_all_lanes(small, I):
    R, x, xr, idx = small
    q = occ8_queries(R.size, x.dollar_row)
    want = x.occ8(q)
    qd = torch.from_numpy(q.view(np.int32)).cuda()
    for L in LANES[I]:
        idx.set_tuning(fm.FM_OP_EXACT, occ_interval=I, lanes=L)
        got = to_u32(fm.fm_occ8(idx, qd))
        torch.cuda.synchronize()
        bad = np.nonzero((got != want).any(axis=1))[0]
        assert bad.size == 0, (I, L, q[bad[:5]], got[bad[:5]], want[bad[:5]])
    idx.set_tuning(fm.FM_OP_EXACT, occ_interval=128, lanes=1)


def test_occ8_fig2_block():
    """The 32 symbols of Fig. 2 at the start of a BWT: Occ at row 31 counts them (G = 6,
    the figure's final value), and every prefix count matches a direct count."""
    s = "ccacttgcgaaatttacaaggtttattaggtt"
    code = {"a": 0, "c": 1, "g": 2, "t": 3}
    head = np.array([code[c] for c in s], np.uint8)
    tail = synth.iid_reference(300, 5)
    bwt = np.concatenate([head, tail, np.array([4], np.uint8)])
    for I in LAYOUTS:
        idx = fm.Index.from_codes(bwt, occ_interval=I)
        q = np.array([[0, p] for p in range(bwt.size)], np.uint32)
        got = to_u32(fm.fm_occ8(idx, torch.from_numpy(q.view(np.int32)).cuda()))[:, 4:]
        assert got[31].tolist() == [9, 5, 6, 12]
        want = np.zeros((bwt.size, 4), np.int64)
        for p in range(bwt.size):
            want[p] = [np.count_nonzero(bwt[:p + 1] == c) for c in range(4)]
        assert np.array_equal(got, want)
        idx.free()


def exact_inputs(R):
    rng = np.random.default_rng(99)
    pats = []
    for j in range(3000):
        m = int(rng.integers(1, 120))
        if j % 3 == 0:
            w = rng.integers(0, 4, m).astype(np.uint8)
        else:
            p = int(rng.integers(0, R.size - m))
            w = R[p:p + m].copy()
            if j % 7 == 0:
                w[int(rng.integers(0, m))] = (w[0] + 1) % 4
        if j % 50 == 0:
            w[int(rng.integers(0, m))] = 4
        pats.append(w)
    pats += [np.zeros(0, np.uint8), np.zeros(0, np.uint8), R[:40].copy(), R[-40:].copy(), np.array([4], np.uint8)]
    offs = np.zeros(len(pats) + 1, np.uint64)
    offs[1:] = np.cumsum([p.size for p in pats])
    return np.concatenate(pats), offs


@pytest.mark.parametrize("flags", [fm.FM_FWD, fm.FM_REVCOMP, fm.FM_BOTH])
def test_exact_plain_and_batched(small, flags):
    R, x, xr, idx = small
    codes, offs = exact_inputs(R)
    want = x.exact(codes, offs, flags, "definition")
    cd, od, _ = fm.reads_to_device(codes, offs)
    got = to_u32(fm.fm_search_exact(idx, cd, od, flags | fm.FM_PLAIN))
    assert np.array_equal(got, want)
    for I in LAYOUTS:
        for L in LANES[I]:
            for P in (1, 2):
                idx.set_tuning(fm.FM_OP_EXACT, occ_interval=I, lanes=L, depth=P)
                got = to_u32(fm.fm_search_exact(idx, cd, od, flags))
                bad = np.nonzero((got != want).any(axis=1))[0]
                assert bad.size == 0, (I, L, P, bad[:5], got[bad[:5]], want[bad[:5]])
    idx.set_tuning(fm.FM_OP_EXACT, occ_interval=128, lanes=1, depth=1)


@pytest.mark.parametrize("flags", [fm.FM_FWD, fm.FM_BOTH])
def test_exact_full_rank(small, flags):
    """FM_FULL_RANK: Listing 1 without the early exit reports (k, k - 1 + occ) with k the
    number of smaller suffixes, for hits and misses alike (reading G5), as the oracle's
    rank scan computes it from the text; patterns with N rank above T."""
    R, x, xr, idx = small
    codes, offs = exact_inputs(R)
    want = oracle.exact_by_rank_scan_batch(R, codes, offs, flags, threads=4, full_rank=True)
    canon = x.exact(codes, offs, flags, "definition")
    hit = canon[:, 0] <= canon[:, 1]
    assert np.array_equal(want[hit], canon[hit]) and (~hit).sum() > 100
    cd, od, _ = fm.reads_to_device(codes, offs)
    got = to_u32(fm.fm_search_exact(idx, cd, od, flags | fm.FM_PLAIN | fm.FM_FULL_RANK))
    assert np.array_equal(got, want)
    for I in LAYOUTS:
        for L in LANES[I]:
            idx.set_tuning(fm.FM_OP_EXACT, occ_interval=I, lanes=L)
            got = to_u32(fm.fm_search_exact(idx, cd, od, flags | fm.FM_FULL_RANK))
            bad = np.nonzero((got != want).any(axis=1))[0]
            assert bad.size == 0, (I, L, bad[:5], got[bad[:5]], want[bad[:5]])
    idx.set_tuning(fm.FM_OP_EXACT, occ_interval=128, lanes=1)


def test_exact_work_queue_with_a_dirty_workspace(small):
    """The exact search clears its work-queue counter only when some wave goes back to it,
    i.e. when the read-strands need more than one workgroup per CU; a smaller batch is
    covered by the waves' own first chunks and never reads the counter. With every
    workspace byte set to garbage first, batches on both sides of that size, at several
    occupancies and lanes, equal the oracle."""
    R, x, xr, idx = small
    cu = torch.cuda.get_device_properties(0).multi_processor_count
    rng = np.random.default_rng(17)
    m = 24
    for nreads in (1000, 40 * cu * 2, 200 * cu):
        pos = rng.integers(0, R.size - m, nreads)
        pats = R[pos[:, None] + np.arange(m)].copy()
        flip = rng.random(nreads) < 0.3
        pats[flip, rng.integers(0, m, int(flip.sum()))] ^= 1
        codes = pats.reshape(-1)
        offs = (np.arange(nreads + 1, dtype=np.uint64) * m)
        want = x.exact(codes, offs, fm.FM_BOTH, "definition")
        cd, od, _ = fm.reads_to_device(codes, offs)
        ws = torch.empty(fm.fm_search_exact_workspace(idx, nreads, fm.FM_BOTH), dtype=torch.uint8, device="cuda")
        for I, L, waves in ((128, 1, 0), (128, 1, 4), (64, 2, 16), (256, 8, 8)):
            idx.set_tuning(fm.FM_OP_EXACT, occ_interval=I, lanes=L, depth=1, waves_per_cu=waves)
            ws.fill_(0xAB)
            queue_read = nreads * 2 * L > cu * 256
            say("dirty workspace:", nreads, "reads", (I, L, waves), "queue read:", queue_read)
            got = to_u32(fm.fm_search_exact(idx, cd, od, fm.FM_BOTH, ws=ws))
            bad = np.nonzero((got != want).any(axis=1))[0]
            assert bad.size == 0, (nreads, I, L, waves, bad[:5])
    idx.set_tuning(fm.FM_OP_EXACT, occ_interval=128, lanes=1, depth=1, waves_per_cu=0)


def test_exact_small_workload():
    w = synth.small_exact_workload()
    x = oracle.OracleIndex(w.ref)
    want = x.exact(w.reads.codes, w.reads.offs, oracle.FWD, "definition")
    idx = fm.Index.from_text(w.ref, occ_interval=128)
    cd, od, _ = fm.reads_to_device(w.reads.codes, w.reads.offs)
    for flags in (fm.FM_FWD | fm.FM_PLAIN, fm.FM_FWD):
        got = to_u32(fm.fm_search_exact(idx, cd, od, flags))
        assert np.array_equal(got, want)
    hits = np.count_nonzero(want[:5000, 0] <= want[:5000, 1])
    assert hits == 5000          # the copied half always occurs
    idx.free()


@pytest.mark.parametrize("flags", [fm.FM_FWD, fm.FM_BOTH])
def test_darray(small, flags):
    R, x, xr, idx = small
    codes, offs = exact_inputs(R)
    want = xr.darray(codes, offs, flags)
    cd, od, _ = fm.reads_to_device(codes, offs)
    for I in LAYOUTS:
        idx.set_tuning(fm.FM_OP_DARRAY, occ_interval=I, lanes=1)
        got = fm.fm_darray(idx, cd, od, int(offs[-1]), flags).cpu().numpy()
        assert np.array_equal(got, want), I
    idx.set_tuning(fm.FM_OP_DARRAY, occ_interval=128)


def inexact_inputs(R, count=1500, seed=3):
    rd = synth.simulate_reads(R, count, seed, length=(20, 90), sub=(0.0, 0.06), z=(0, 2))
    codes = rd.codes.copy()
    codes[::997] = 4                                # sprinkle N
    # an empty read and a read of N only
    codes = np.concatenate([codes, np.array([4, 4, 4], np.uint8)])
    offs = np.concatenate([rd.offs, [rd.offs[-1], rd.offs[-1] + 3]]).astype(np.uint64)
    z = np.concatenate([rd.z, [1, 2]]).astype(np.uint8)
    return codes, offs, z


def run_inexact(idx, codes, offs, z, flags, zmax, cap=1 << 16):
    cd, od, zd = fm.reads_to_device(codes, offs, z)
    bufs = fm.fm_search_inexact(idx, cd, od, zd, flags, zmax, cap)
    return fm.hits_to_numpy(bufs, offs.size - 1), bufs


def assert_same_hits(got, want_hits, want_offs, tag):
    hits, hoffs, status = got
    assert (status == 0).all(), (tag, np.unique(status))
    assert np.array_equal(hoffs, want_offs), tag
    for f in ("read", "k", "l", "strand"):
        assert np.array_equal(hits[f], want_hits[f]), (tag, f)
    assert np.array_equal(hits["nmm"], want_hits["d"]), tag


@pytest.mark.parametrize("use_d", [False, True])
def test_inexact_plain_and_batched(small, use_d):
    R, x, xr, idx = small
    codes, offs, z = inexact_inputs(R)
    method = "listing2_darray" if use_d else "listing2"
    wh, wo = x.inexact(codes, offs, z, oracle.BOTH, method, rev=xr)
    say("oracle hits", wh.size)
    flags = fm.FM_BOTH | (fm.FM_DARRAY if use_d else 0)
    assert_same_hits(run_inexact(idx, codes, offs, z, flags | fm.FM_PLAIN, 2)[0], wh, wo, "plain")
    for I in LAYOUTS:
        for L in LANES[I]:
            idx.set_tuning(fm.FM_OP_INEXACT, occ_interval=I, lanes=L)
            idx.set_tuning(fm.FM_OP_DARRAY, occ_interval=I, lanes=min(L, 4))
            assert_same_hits(run_inexact(idx, codes, offs, z, flags, 2)[0], wh, wo, (I, L))
    idx.set_tuning(fm.FM_OP_INEXACT, occ_interval=128, lanes=1)
    idx.set_tuning(fm.FM_OP_DARRAY, occ_interval=128, lanes=1)


@pytest.mark.parametrize("use_d", [False, True])
def test_search_both_equals_separate_calls(small, use_d):
    """fm_search_both (exact intervals taken from the DFS) gives the exact and the inexact
    results of the separate calls for every layout, lane count and strand set."""
    R, x, xr, idx = small
    codes, offs, z = inexact_inputs(R)
    flags = fm.FM_BOTH | (fm.FM_DARRAY if use_d else 0)
    wh, wo = x.inexact(codes, offs, z, oracle.BOTH, "listing2_darray" if use_d else "listing2", rev=xr)
    cd, od, zd = fm.reads_to_device(codes, offs, z)
    for exf in (fm.FM_FWD, fm.FM_REVCOMP, fm.FM_BOTH):
        want_ex = x.exact(codes, offs, exf, "listing1")
        ex, bufs = fm.fm_search_both(idx, cd, od, zd, exf, flags | fm.FM_PLAIN, 2, 1 << 16)
        assert np.array_equal(to_u32(ex), want_ex), ("plain", exf)
        assert_same_hits(fm.hits_to_numpy(bufs, offs.size - 1), wh, wo, ("plain", exf))
        for I in LAYOUTS:
            for L in LANES[I]:
                idx.set_tuning(fm.FM_OP_INEXACT, occ_interval=I, lanes=L)
                idx.set_tuning(fm.FM_OP_DARRAY, occ_interval=I, lanes=min(L, 4))
                ex, bufs = fm.fm_search_both(idx, cd, od, zd, exf, flags, 2, 1 << 16)
                assert np.array_equal(to_u32(ex), want_ex), (I, L, exf)
                assert_same_hits(fm.hits_to_numpy(bufs, offs.size - 1), wh, wo, (I, L, exf))
    idx.set_tuning(fm.FM_OP_INEXACT, occ_interval=128, lanes=1)
    idx.set_tuning(fm.FM_OP_DARRAY, occ_interval=128, lanes=1)


def test_claim_order_changes_nothing(small):
    """The DFS may claim read-strands heaviest first (tuning field `order`, weights from
    the D records) or in read order: hits, statuses, exact intervals and node counts are
    the same, with every decided-at-once case in the batch (budgets above zmax, a read
    over 65535, reads with N, an empty read, root-pruned strands), for substitutions and
    for the gapped search, one and two strands."""
    R, x, xr, idx = small
    rd = synth.simulate_reads(R, 3000, 37, length=(0, 120), sub=(0.0, 0.05), z=(0, 3))
    long_read = R[2000:2000 + 66_000]
    codes = np.concatenate([rd.codes, long_read, np.array([4, 0, 4, 1], np.uint8)])
    offs = np.concatenate([rd.offs, rd.offs[-1] + np.cumsum([long_read.size, 4])]).astype(np.uint64)
    z = np.concatenate([rd.z, [1, 2]]).astype(np.uint8)
    nr = offs.size - 1
    cd, od, zd = fm.reads_to_device(codes, offs, z)
    want_ex = x.exact(codes, offs, oracle.BOTH, "listing1")
    for flags in (fm.FM_BOTH | fm.FM_DARRAY, fm.FM_FWD | fm.FM_DARRAY, fm.FM_REVCOMP | fm.FM_DARRAY,
                  fm.FM_BOTH | fm.FM_DARRAY | fm.FM_GAPS):
        runs = []
        for order in (0, 1):
            idx.set_tuning(fm.FM_OP_INEXACT, occ_interval=64, lanes=1, order=order)
            try:
                bufs = fm.fm_search_inexact(idx, cd, od, zd, flags | fm.FM_STATS, 2, 1 << 17)
                got = fm.hits_to_numpy(bufs, nr)
                stats = bufs.stats()
                ex = None
                if not flags & fm.FM_GAPS and flags & fm.FM_BOTH == fm.FM_BOTH:
                    ex, b2 = fm.fm_search_both(idx, cd, od, zd, fm.FM_BOTH, flags, 2, 1 << 17)
                    ex = to_u32(ex)
                    for u, v in zip(fm.hits_to_numpy(b2, nr), got):
                        assert np.array_equal(u, v), (flags, order)
            finally:
                idx.set_tuning(fm.FM_OP_INEXACT, occ_interval=128, lanes=1, order=1)
            runs.append((got, stats["occ8"], ex))
        (g0, n0, e0), (g1, n1, e1) = runs
        for u, v in zip(g0, g1):
            assert np.array_equal(u, v), flags
        assert n0 == n1, flags
        st = g1[2]
        assert st[-2] == fm.FM_ERANGE and ((st == fm.FM_EINVAL) == (z > 2)).all()
        if e1 is not None:
            assert np.array_equal(e0, want_ex) and np.array_equal(e1, want_ex)
        plain = fm.hits_to_numpy(fm.fm_search_inexact(idx, cd, od, zd, flags | fm.FM_PLAIN, 2, 1 << 17), nr)
        for u, v in zip(plain, g1):
            assert np.array_equal(u, v), flags
        say(hex(flags), "hits", g1[0].size, "nodes", n1)
    # batches of one and three reads: one counting workgroup, mostly idle lanes
    for count in (1, 3):
        sub = rd.subset(np.arange(count))
        cd, od, zd = fm.reads_to_device(sub.codes, sub.offs, sub.z)
        flags = fm.FM_BOTH | fm.FM_DARRAY
        want = x.inexact(sub.codes, sub.offs, sub.z, oracle.BOTH, "listing2_darray", rev=xr)
        idx.set_tuning(fm.FM_OP_INEXACT, occ_interval=64, lanes=1, order=1)
        try:
            got = fm.hits_to_numpy(fm.fm_search_inexact(idx, cd, od, zd, flags, 2, 1 << 12), count)
        finally:
            idx.set_tuning(fm.FM_OP_INEXACT, occ_interval=128, lanes=1, order=1)
        ok = got[2] == fm.FM_OK
        assert ((got[2] == fm.FM_EINVAL) == (sub.z > 2)).all() and ok.any() == (sub.z <= 2).any()
        for r in np.nonzero(ok)[0]:
            a = got[0][int(got[1][r]):int(got[1][r + 1])]
            w = want[0][int(want[1][r]):int(want[1][r + 1])]
            for f in ("k", "l", "strand"):
                assert np.array_equal(a[f], w[f]), (count, r, f)
            assert np.array_equal(a["nmm"], w["d"]), (count, r)


def test_subtree_transfers(small):
    """With one lane per read-strand, idle lanes of the batched DFS take subtrees over from
    busy lanes at the end of the launch (FM_STATS counts them), and there a node with an
    empty stack walks its match child first and leaves its mismatch children to them.
    Hits, statuses and node counts equal the oracle's, for substitutions with and without
    the D bound and for the gapped search, at z = 1 and 2, in a full batch and in batches
    of a few reads (where the work queue is empty from the start and a few trees are
    spread over the whole wave); two lanes per read-strand take none, nor does the gapped
    search at z = 1 (it gives away only children left with a budget)."""
    R, x, xr, idx = small
    rd = synth.simulate_reads(R, 1500, 41, length=(60, 120), sub=(0.0, 0.03), z=(2, 2))
    r1 = synth.simulate_reads(R, 1500, 42, length=(60, 120), sub=(0.0, 0.03), z=(1, 1))
    tiny2 = rd.subset(np.arange(6))
    tiny1 = r1.subset(np.arange(3))
    cases = ((fm.FM_BOTH | fm.FM_DARRAY, "listing2_darray"), (fm.FM_BOTH, "listing2"),
             (fm.FM_BOTH | fm.FM_DARRAY | fm.FM_GAPS, "listing2_gaps_darray"))
    for flags, method in cases:
        for reads, zmax in ((rd, 2), (r1, 1), (tiny2, 2), (tiny1, 1)):
            cd, od, zd = fm.reads_to_device(reads.codes, reads.offs, reads.z)
            wh, wo, wn = x.inexact(reads.codes, reads.offs, reads.z, oracle.BOTH, method, rev=xr, return_nodes=True)
            for lanes in (1, 2):
                idx.set_tuning(fm.FM_OP_INEXACT, occ_interval=64, lanes=lanes)
                try:
                    bufs = fm.fm_search_inexact(idx, cd, od, zd, flags | fm.FM_STATS, zmax, 1 << 22)
                    got = fm.hits_to_numpy(bufs, reads.count)
                    st = bufs.stats()
                finally:
                    idx.set_tuning(fm.FM_OP_INEXACT, occ_interval=128, lanes=1)
                assert_same_hits(got, wh, wo, (flags, zmax, lanes, reads.count))
                assert st["occ8"] == int(wn.sum()), (flags, zmax, lanes, reads.count)
                # the gapped search gives away only children left with a budget of one or more
                if lanes == 1 and not (flags & fm.FM_GAPS and zmax < 2):
                    assert st["subtrees"] > 0, (flags, zmax, reads.count)
                else:
                    assert st["subtrees"] == 0, (flags, zmax, lanes)
                say(hex(flags), "zmax", zmax, "reads", reads.count, "lanes", lanes, "nodes", st["occ8"],
                    "subtrees", st["subtrees"])


def test_search_both_where_the_dfs_stops_early(small):
    """fm_search_both takes exact intervals from the DFS. Read-strands whose DFS ends
    before reaching the match-only leaf still get theirs: budgets above zmax (FM_EINVAL),
    reads longer than 65535 (FM_ERANGE; one occurs, one does not) and spent node budgets
    (FM_EBUDGET). An exact strand that the inexact search does not cover runs as a
    separate search."""
    R, x, xr, idx = small
    rd = synth.simulate_reads(R, 500, 31, length=(30, 90), sub=(0.0, 0.04), z=(0, 4))
    occurs = R[1000:1000 + 66_000].copy()
    differs = occurs.copy()
    differs[33_000] = (differs[33_000] + 1) % 4
    codes = np.concatenate([rd.codes, occurs, differs, R[5000:5080]])
    ends = rd.offs[-1] + np.cumsum([occurs.size, differs.size, 80])
    offs = np.concatenate([rd.offs, ends]).astype(np.uint64)
    z = np.concatenate([rd.z, [1, 0, 3]]).astype(np.uint8)
    nr = offs.size - 1
    cd, od, zd = fm.reads_to_device(codes, offs, z)
    want_ex = x.exact(codes, offs, oracle.BOTH, "listing1")
    assert (want_ex[-6:, 0] <= want_ex[-6:, 1]).tolist() == [True, False, False, False, True, False]
    flags = fm.FM_BOTH | fm.FM_DARRAY
    for budget in (1 << 22, 30):
        idx.set_tuning(fm.FM_OP_INEXACT, occ_interval=64, lanes=1, node_budget=budget)
        try:
            sep = fm.hits_to_numpy(fm.fm_search_inexact(idx, cd, od, zd, flags, 2, 1 << 16), nr)
            ex, bufs = fm.fm_search_both(idx, cd, od, zd, fm.FM_BOTH, flags, 2, 1 << 16)
            got = fm.hits_to_numpy(bufs, nr)
        finally:
            idx.set_tuning(fm.FM_OP_INEXACT, occ_interval=128, lanes=1, node_budget=1 << 22)
        st = got[2]
        say("budget", budget, "statuses", np.unique(st, return_counts=True))
        assert st[-3] == fm.FM_ERANGE and st[-2] == fm.FM_ERANGE and st[-1] == fm.FM_EINVAL
        assert ((st == fm.FM_EINVAL) == (z > 2)).all()
        if budget == 30:
            assert (st == fm.FM_EBUDGET).any()
        assert np.array_equal(to_u32(ex), want_ex), budget
        for u, v in zip(got, sep):
            assert np.array_equal(u, v), budget
    # exact on both strands, inexact on the forward strand only
    for extra in (0, fm.FM_PLAIN):
        ex, bufs = fm.fm_search_both(idx, cd, od, zd, fm.FM_BOTH, fm.FM_FWD | fm.FM_DARRAY | extra, 2, 1 << 16)
        sep = fm.hits_to_numpy(fm.fm_search_inexact(idx, cd, od, zd, fm.FM_FWD | fm.FM_DARRAY | extra, 2, 1 << 16), nr)
        assert np.array_equal(to_u32(ex), want_ex), extra
        for u, v in zip(fm.hits_to_numpy(bufs, nr), sep):
            assert np.array_equal(u, v), extra


def test_inexact_definition_and_node_count(small):
    """Hits equal the Hamming-ball definition; expanded nodes equal the oracle's."""
    R, x, xr, idx = small
    codes, offs, z = inexact_inputs(R, count=300, seed=11)
    z = np.minimum(z, 1)
    wh, wo = x.inexact(codes, offs, z, oracle.BOTH, "definition")
    lh, lo, nodes = x.inexact(codes, offs, z, oracle.BOTH, "listing2_darray", rev=xr, return_nodes=True)
    assert np.array_equal(wh, lh) and np.array_equal(wo, lo)
    for extra in (fm.FM_PLAIN, 0):
        got, bufs = run_inexact(idx, codes, offs, z, fm.FM_BOTH | fm.FM_DARRAY | fm.FM_STATS | extra, 1)
        assert_same_hits(got, wh, wo, "def")
        assert bufs.stats()["occ8"] == int(nodes.sum())


def test_inexact_zmax4_and_limits(small):
    R, x, xr, idx = small
    rd = synth.simulate_reads(R, 60, 21, length=(12, 18), sub=(0.0, 0.1), z=(0, 4))
    wh, wo = x.inexact(rd.codes, rd.offs, rd.z, oracle.BOTH, "listing2_darray", rev=xr)
    for extra in (fm.FM_PLAIN, 0):
        got, _ = run_inexact(idx, rd.codes, rd.offs, rd.z, fm.FM_BOTH | fm.FM_DARRAY | extra, 4, cap=1 << 20)
        assert_same_hits(got, wh, wo, "z4")
    # budgets above zmax are rejected per read, others unaffected
    got, _ = run_inexact(idx, rd.codes, rd.offs, rd.z, fm.FM_BOTH | fm.FM_DARRAY, 2, cap=1 << 20)
    hits, hoffs, status = got
    assert ((status == fm.FM_EINVAL) == (rd.z > 2)).all()
    ok = np.nonzero(rd.z <= 2)[0]
    for r in ok[:20]:
        a = hits[int(hoffs[r]):int(hoffs[r + 1])]
        b = wh[int(wo[r]):int(wo[r + 1])]
        assert np.array_equal(a["k"], b["k"]) and np.array_equal(a["nmm"], b["d"])


def test_inexact_overflow_and_retry(small):
    R, x, xr, idx = small
    codes, offs, z = inexact_inputs(R, count=400, seed=5)
    wh, wo = x.inexact(codes, offs, z, oracle.BOTH, "listing2")
    total = int(wo[-1])
    cap = total // 3
    (hits, hoffs, status), bufs = run_inexact(idx, codes, offs, z, fm.FM_BOTH, 2, cap=cap)
    assert bufs.required() == total
    assert (status == fm.FM_EOVERFLOW).any()
    okr = np.nonzero(status == 0)[0]
    for r in okr:
        a = hits[int(hoffs[r]):int(hoffs[r + 1])]
        b = wh[int(wo[r]):int(wo[r + 1])]
        assert np.array_equal(a["k"], b["k"]) and np.array_equal(a["l"], b["l"])
    for r in np.nonzero(status == fm.FM_EOVERFLOW)[0]:
        assert hoffs[r] == hoffs[r + 1]
    got, _ = run_inexact(idx, codes, offs, z, fm.FM_BOTH, 2, cap=bufs.required())
    assert_same_hits(got, wh, wo, "retry")


def test_inexact_node_budget(small):
    """A read-strand whose tree needs more nodes than the budget ends FM_EBUDGET. The
    batched DFS (whose lanes split trees between them at the end of a launch, z >= 2)
    agrees with the plain kernel at budgets around the trees' sizes."""
    R, x, xr, idx = small
    codes, offs, z = inexact_inputs(R, count=200, seed=6)
    for flags in (fm.FM_BOTH, fm.FM_BOTH | fm.FM_DARRAY):
        for budget in (30, 90, 250):
            idx.set_tuning(fm.FM_OP_INEXACT, node_budget=budget)
            try:
                a = run_inexact(idx, codes, offs, z, flags | fm.FM_PLAIN, 2)[0]
                b = run_inexact(idx, codes, offs, z, flags, 2)[0]
            finally:
                idx.set_tuning(fm.FM_OP_INEXACT, node_budget=1 << 22)
            if budget == 30:
                assert (a[2] == fm.FM_EBUDGET).any()
            assert np.array_equal(a[2], b[2]) and np.array_equal(a[1], b[1]), (flags, budget)
            assert np.array_equal(a[0], b[0]), (flags, budget)


def test_determinism_and_batch_independence(small):
    R, x, xr, idx = small
    codes, offs, z = inexact_inputs(R, count=800, seed=8)
    flags = fm.FM_BOTH | fm.FM_DARRAY
    a = run_inexact(idx, codes, offs, z, flags, 2)[0]
    b = run_inexact(idx, codes, offs, z, flags, 2)[0]
    for u, v in zip(a, b):
        assert np.array_equal(u, v)
    # a permuted batch gives each read the same hits
    rng = np.random.default_rng(1)
    perm = rng.permutation(offs.size - 1)
    rd = synth.Reads(codes, offs, z, np.zeros(z.size, np.int64), np.zeros(z.size, np.uint8)).subset(perm)
    c = run_inexact(idx, rd.codes, rd.offs, rd.z, flags, 2)[0]
    for j, r in enumerate(perm):
        ha = a[0][int(a[1][r]):int(a[1][r + 1])]
        hc = c[0][int(c[1][j]):int(c[1][j + 1])]
        assert np.array_equal(ha[["k", "l", "strand", "nmm"]], hc[["k", "l", "strand", "nmm"]])


def test_non_base_codes_above_4(small):
    """Any read code above 3 matches no base (fm.h): reads holding codes 5, 16, 78 and 255
    give the oracle's hits (which treats every such code alike) and the same results as
    with code 4 in their place, for substitutions and the gapped search, plain and batched,
    with subtree transfers on (one lane per read-strand, z = 2)."""
    R, x, xr, idx = small
    rd = synth.simulate_reads(R, 800, 57, length=(40, 100), sub=(0.0, 0.03), z=(0, 2))
    odd = rd.codes.copy()
    pos = np.arange(5, odd.size, 61)
    odd[pos] = np.resize(np.array([5, 16, 78, 255], np.uint8), pos.size)
    n4 = odd.copy()
    n4[pos] = 4
    cases = ((fm.FM_BOTH | fm.FM_DARRAY, "listing2_darray"), (fm.FM_BOTH, "listing2"),
             (fm.FM_BOTH | fm.FM_DARRAY | fm.FM_GAPS, "listing2_gaps_darray"))
    for flags, method in cases:
        wh, wo = x.inexact(odd, rd.offs, rd.z, oracle.BOTH, method, rev=xr)
        w4 = x.inexact(n4, rd.offs, rd.z, oracle.BOTH, method, rev=xr)
        assert np.array_equal(wo, w4[1]) and np.array_equal(wh, w4[0])
        assert_same_hits(run_inexact(idx, odd, rd.offs, rd.z, flags | fm.FM_PLAIN, 2)[0], wh, wo, ("plain", flags))
        for lanes in (1, 2):
            idx.set_tuning(fm.FM_OP_INEXACT, occ_interval=64, lanes=lanes)
            try:
                got = run_inexact(idx, odd, rd.offs, rd.z, flags, 2)[0]
            finally:
                idx.set_tuning(fm.FM_OP_INEXACT, occ_interval=128, lanes=1)
            assert_same_hits(got, wh, wo, (flags, lanes))
    want_ex = x.exact(n4, rd.offs, oracle.BOTH, "listing1")
    cd, od, zd = fm.reads_to_device(odd, rd.offs, rd.z)
    assert np.array_equal(to_u32(fm.fm_search_exact(idx, cd, od, fm.FM_BOTH)), want_ex)
    ex, bufs = fm.fm_search_both(idx, cd, od, zd, fm.FM_BOTH, fm.FM_BOTH | fm.FM_DARRAY, 2, 1 << 16)
    assert np.array_equal(to_u32(ex), want_ex)
    wh, wo = x.inexact(odd, rd.offs, rd.z, oracle.BOTH, "listing2_darray", rev=xr)
    assert_same_hits(fm.hits_to_numpy(bufs, rd.count), wh, wo, "both")


def test_prefix_table_depths():
    """The prefix table (children of nodes whose matched suffix is shorter than
    table_depth come from the table, not from an Occ8) changes nothing: at every depth
    0..T, hits and node counts equal the oracle's (Listing 2 with and without the D bound,
    z up to 2 with subtree transfers), exact intervals from fm_search_both equal Listing
    1's, for the plain and batched kernels and several layouts; FM_STATS counts the table
    nodes (none at depth 0, none with two lanes per read-strand, and they fetch no
    bucket; the root takes its children from C at any depth)."""
    R = synth.reference_with_repeats(1 << 20, 4343, copy_frac=0.08, copy_len=(300, 3000), copy_sub=0.02,
                                     tandem_frac=0.01, tandem_unit=(2, 30), tandem_len=(100, 600))
    x = oracle.OracleIndex(R)
    xr = oracle.OracleIndex(oracle.reverse_text(R))
    idx = fm.Index.from_text(R, occ_interval=64, flags=fm.FM_LOAD_REVERSE | fm.FM_LOAD_ALL_LAYOUTS)
    T = idx.info()["table_depth"]
    assert T == 9 and idx.get_tuning(fm.FM_OP_INEXACT)["table_depth"] == T
    with pytest.raises(fm.FmError):
        idx.set_tuning(fm.FM_OP_INEXACT, table_depth=T + 1)
    rd = synth.simulate_reads(R, 1200, 77, length=(40, 120), sub=(0.0, 0.03), z=(0, 2))
    cd, od, zd = fm.reads_to_device(rd.codes, rd.offs, rd.z)
    want_ex = x.exact(rd.codes, rd.offs, oracle.BOTH, "listing1")
    for flags, method in ((fm.FM_BOTH | fm.FM_DARRAY, "listing2_darray"), (fm.FM_BOTH, "listing2")):
        wh, wo, wn = x.inexact(rd.codes, rd.offs, rd.z, oracle.BOTH, method, rev=xr, return_nodes=True)
        for depth in (0, 1, 3, 5, T):
            for I, lanes, extra in ((64, 1, 0), (64, 1, fm.FM_PLAIN), (128, 1, 0), (448, 1, 0), (64, 2, 0)):
                idx.set_tuning(fm.FM_OP_INEXACT, occ_interval=I, lanes=lanes, table_depth=depth)
                try:
                    bufs = fm.fm_search_inexact(idx, cd, od, zd, flags | fm.FM_STATS | extra, 2, 1 << 16)
                    got = fm.hits_to_numpy(bufs, rd.count)
                    st = bufs.stats()
                    ex, b2 = fm.fm_search_both(idx, cd, od, zd, fm.FM_BOTH, flags | extra, 2, 1 << 16)
                    got2 = fm.hits_to_numpy(b2, rd.count)
                finally:
                    idx.set_tuning(fm.FM_OP_INEXACT, occ_interval=64, lanes=1, table_depth=T)
                tag = (hex(flags), depth, I, lanes, extra)
                assert_same_hits(got, wh, wo, tag)
                assert_same_hits(got2, wh, wo, tag)
                assert np.array_equal(to_u32(ex), want_ex), tag
                assert st["occ8"] == int(wn.sum()), tag
                if depth <= 1 or lanes > 1:             # depth 1 would serve the root alone, which reads C
                    assert st["table"] == 0, tag
                else:
                    assert st["table"] > 0, tag
                say(tag, "nodes", st["occ8"], "table nodes", st["table"], "buckets", st["buckets"])
    idx.free()
