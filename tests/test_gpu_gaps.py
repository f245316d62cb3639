"""Listing 2 with all its branches (FM_GAPS): substitutions, deletions and insertions,
one hit per interval at the smallest edit count, against the oracle's gapped recursion."""
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
def text():
    R = synth.reference_with_repeats(70_001, 4244, copy_frac=0.08, copy_len=(300, 2000), copy_sub=0.02,
                                     tandem_frac=0.02, tandem_unit=(2, 12), tandem_len=(100, 400))
    x = oracle.OracleIndex(R)
    xr = oracle.OracleIndex(oracle.reverse_text(R))
    idx = fm.Index.from_text(R, occ_interval=128, flags=fm.FM_LOAD_REVERSE | fm.FM_LOAD_ALL_LAYOUTS)
    return R, x, xr, idx


def indel_reads(R, count, seed, length=(20, 60), z=(0, 2)):
    """Reads sampled from R (either strand) with up to two edits each (substitution,
    deletion or insertion), some N, an empty read and a read of N only."""
    rd = synth.simulate_reads(R, count, seed, length=length, sub=(0.0, 0.0), z=z)
    rng = np.random.default_rng(seed)
    reads = []
    for r in range(rd.count):
        w = rd.read(r).copy()
        for _ in range(int(rng.integers(0, 3))):
            j = int(rng.integers(0, w.size))
            kind = int(rng.integers(0, 3))
            if kind == 0:
                w[j] = (w[j] + 1 + int(rng.integers(0, 3))) % 4
            elif kind == 1 and w.size > 1:
                w = np.delete(w, j)
            else:
                w = np.insert(w, j, int(rng.integers(0, 4))).astype(np.uint8)
        if r % 97 == 0:
            w[int(rng.integers(0, w.size))] = 4
        reads.append(w)
    reads += [np.zeros(0, np.uint8), np.array([4, 4, 4], np.uint8)]
    z = np.concatenate([rd.z, [2, 1]]).astype(np.uint8)
    offs = np.zeros(len(reads) + 1, np.uint64)
    offs[1:] = np.cumsum([w.size for w in reads])
    return np.concatenate(reads), offs, z


def run(idx, codes, offs, z, flags, zmax, cap=1 << 18):
    cd, od, zd = fm.reads_to_device(codes, offs, z)
    bufs = fm.fm_search_inexact(idx, cd, od, zd, flags, zmax, cap)
    return fm.hits_to_numpy(bufs, offs.size - 1), bufs


def assert_same(got, wh, wo, tag):
    hits, hoffs, status = got
    assert (status == 0).all(), (tag, np.unique(status))
    assert np.array_equal(hoffs, wo), tag
    for f in ("read", "k", "l", "strand"):
        assert np.array_equal(hits[f], wh[f]), (tag, f)
    assert np.array_equal(hits["nmm"], wh["d"]), tag


@pytest.mark.parametrize("use_d", [True, False])
def test_gapped_all_layouts_and_lanes(text, use_d):
    R, x, xr, idx = text
    codes, offs, z = indel_reads(R, 600, 5)
    method = "listing2_gaps_darray" if use_d else "listing2_gaps"
    wh, wo = x.inexact(codes, offs, z, oracle.BOTH, method, rev=xr)
    subs, _ = x.inexact(codes, offs, z, oracle.BOTH, "listing2_darray", rev=xr)
    say("oracle gapped hits", wh.size, "substitution hits", subs.size)
    assert wh.size > subs.size
    flags = fm.FM_BOTH | fm.FM_GAPS | (fm.FM_DARRAY if use_d else 0)
    assert_same(run(idx, codes, offs, z, flags | fm.FM_PLAIN, 2)[0], wh, wo, "plain")
    for I in LAYOUTS:
        for L in LANES[I]:
            idx.set_tuning(fm.FM_OP_INEXACT, occ_interval=I, lanes=L)
            idx.set_tuning(fm.FM_OP_DARRAY, occ_interval=I, lanes=min(L, 4))
            assert_same(run(idx, codes, offs, z, flags, 2)[0], wh, wo, (I, L))
    idx.set_tuning(fm.FM_OP_INEXACT, occ_interval=128, lanes=1)
    idx.set_tuning(fm.FM_OP_DARRAY, occ_interval=128, lanes=1)


def test_gapped_node_count_and_exact_case(text):
    """Expanded nodes equal the oracle recursion's; with z = 0 the gapped search is the
    exact search."""
    R, x, xr, idx = text
    codes, offs, z = indel_reads(R, 300, 6, z=(0, 2))
    wh, wo, nodes = x.inexact(codes, offs, z, oracle.BOTH, "listing2_gaps_darray", rev=xr, return_nodes=True)
    for extra in (fm.FM_PLAIN, 0):
        got, bufs = run(idx, codes, offs, z, fm.FM_BOTH | fm.FM_GAPS | fm.FM_DARRAY | fm.FM_STATS | extra, 2)
        assert_same(got, wh, wo, ("stats", extra))
        assert bufs.stats()["occ8"] == int(nodes.sum())
    z0 = np.zeros_like(z)
    hits, hoffs, _ = run(idx, codes, offs, z0, fm.FM_BOTH | fm.FM_GAPS | fm.FM_DARRAY, 2)[0]
    ex = x.exact(codes, offs, oracle.BOTH, "definition")
    want = [(r, s, int(ex[2 * r + s, 0]), int(ex[2 * r + s, 1])) for r in range(offs.size - 1) for s in (0, 1)
            if ex[2 * r + s, 0] <= ex[2 * r + s, 1]]
    got = [(int(h["read"]), int(h["strand"]), int(h["k"]), int(h["l"])) for h in hits]
    assert got == want and (hits["nmm"] == 0).all()


def test_gapped_overflow_budget_and_both(text):
    """Hit overflow with a retry at the required size, the node budget (plain and batched
    agree), and fm_search_both with gaps, which runs the two searches separately."""
    R, x, xr, idx = text
    codes, offs, z = indel_reads(R, 400, 7)
    flags = fm.FM_BOTH | fm.FM_GAPS | fm.FM_DARRAY
    wh, wo = x.inexact(codes, offs, z, oracle.BOTH, "listing2_gaps_darray", rev=xr)
    got, bufs = run(idx, codes, offs, z, flags, 2, cap=wh.size // 3)
    hits, hoffs, status = got
    assert (status == fm.FM_EOVERFLOW).any()
    assert bufs.required() >= wh.size
    for r in np.nonzero(status == fm.FM_OK)[0]:
        a = hits[int(hoffs[r]):int(hoffs[r + 1])]
        b = wh[int(wo[r]):int(wo[r + 1])]
        assert np.array_equal(a["k"], b["k"]) and np.array_equal(a["l"], b["l"]) and np.array_equal(a["nmm"], b["d"])
    assert_same(run(idx, codes, offs, z, flags, 2, cap=bufs.required())[0], wh, wo, "retry")
    idx.set_tuning(fm.FM_OP_INEXACT, node_budget=40)
    try:
        a = run(idx, codes, offs, z, flags | fm.FM_PLAIN, 2)[0]
        b = run(idx, codes, offs, z, flags, 2)[0]
    finally:
        idx.set_tuning(fm.FM_OP_INEXACT, node_budget=1 << 22)
    assert (a[2] == fm.FM_EBUDGET).any()
    for u, v in zip(a, b):
        assert np.array_equal(u, v)
    cd, od, zd = fm.reads_to_device(codes, offs, z)
    ex, bb = fm.fm_search_both(idx, cd, od, zd, fm.FM_BOTH, flags, 2, 1 << 18)
    assert np.array_equal(ex.cpu().numpy().view(np.uint32), x.exact(codes, offs, oracle.BOTH, "definition"))
    assert_same(fm.hits_to_numpy(bb, offs.size - 1), wh, wo, "both")
