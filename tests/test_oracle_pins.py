"""Pins of the CPU oracle against the paper's printed values, closed forms, invariants
and brute force on tiny inputs (no GPU)."""
import itertools
import os
import random

import numpy as np
import pytest

import oracle
from oracle import OracleIndex, reverse_text
from tests import bruteforce as bf

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")
CODE = {"A": 0, "C": 1, "G": 2, "T": 3, "$": 4}


def enc(s):
    return np.array([CODE[c] for c in s.upper()], dtype=np.uint8)


def read_golden(name):
    out = {}
    for line in open(os.path.join(GOLDEN, name)):
        line = line.strip()
        if not line or line.startswith("#"):
            continue
        key, *vals = line.split()
        out.setdefault(key, []).append(vals)
    return out


def csr(patterns):
    codes = np.concatenate([np.asarray(p, np.uint8) for p in patterns]) if patterns else np.zeros(0, np.uint8)
    offs = np.zeros(len(patterns) + 1, np.uint64)
    offs[1:] = np.cumsum([len(p) for p in patterns])
    return codes, offs


# ------------------------------------------------------------------ Fig. 1

def test_fig1_sa_bwt_occ_c():
    g = read_golden("fig1_acag.txt")
    x = OracleIndex(enc(g["R"][0][0]))
    assert x.sa.tolist() == [int(v) for v in g["SA"][0]]
    assert x.bwt.tolist() == [CODE[c] for c in g["BWT"][0]]
    assert x.dollar_row == 1
    assert x.occ.tolist() == [[int(v) for v in row] for row in g["OCC"]]
    assert x.C.tolist() == [int(v) for v in g["C"][0]]


def test_fig1_exact_search_cases():
    """Intervals read off Fig. 1's sorted rotations; T, GA, TT do not occur."""
    x = OracleIndex(enc("ACAG"))
    cases = {"A": (1, 2), "C": (3, 3), "G": (4, 4), "AG": (2, 2), "CA": (3, 3),
             "ACAG": (1, 1), "T": (1, 0), "GA": (1, 0), "TT": (1, 0), "": (0, 4)}
    pats = list(cases)
    codes, offs = csr([enc(p) for p in pats])
    for method in ("definition", "listing1"):
        got = x.exact(codes, offs, oracle.FWD, method)
        assert [tuple(r) for r in got.tolist()] == [cases[p] for p in pats], method


def test_fig1_occ8():
    x = OracleIndex(enc("ACAG"))
    q = np.array([[0, 4], [1, 2], [3, 3], [5, 4], [6, 0], [0, 5]], np.uint32)
    got = x.occ8(q)
    assert got[0].tolist() == [0, 0, 0, 0, 2, 1, 1, 0]       # k-1 = -1 gives zeros
    assert got[1].tolist() == [0, 0, 1, 0, 0, 1, 1, 0]       # Occ(.,0) and Occ(.,2)
    assert got[2].tolist() == [0, 1, 1, 0, 1, 1, 1, 0]
    assert got[3].tolist() == [2, 1, 1, 0, 2, 1, 1, 0]       # k = n+1 is legal
    assert got[4].tolist() == [0xFFFFFFFF] * 8               # k > n+1
    assert got[5].tolist() == [0xFFFFFFFF] * 8               # l > n


# ------------------------------------------------------------------ invariants

def random_text(n, seed):
    rng = np.random.default_rng(seed)
    return rng.integers(0, 4, n).astype(np.uint8)


@pytest.mark.parametrize("n,seed", [(1, 0), (2, 1), (7, 2), (64, 3), (333, 4), (2000, 5)])
def test_sa_bwt_against_rotation_sort(n, seed):
    R = random_text(n, seed)
    x = OracleIndex(R)
    assert x.sa.tolist() == bf.suffix_array(R)
    ref = [c if c >= 0 else 4 for c in bf.bwt(R)]
    assert x.bwt.tolist() == ref


@pytest.mark.parametrize("n,seed", [(1, 10), (5, 11), (100, 12), (4096, 13)])
def test_occ_c_invariants(n, seed):
    R = random_text(n, seed)
    x = OracleIndex(R)
    occ = x.occ.astype(np.int64)
    counts = np.bincount(R, minlength=4)
    assert occ[n].tolist() == counts.tolist()                      # Occ(c, n) = count of c
    rows = np.arange(n + 1)
    assert (occ.sum(axis=1) == rows + 1 - (rows >= x.dollar_row)).all()
    C = x.C.astype(np.int64)
    assert C[4] == n and C.tolist() == [0, *np.cumsum(counts).tolist()]
    bwt = x.bwt
    # Occ increases exactly at the rows holding that character
    step = np.diff(np.vstack([np.zeros((1, 4), np.int64), occ]), axis=0)
    for c in range(4):
        assert (step[:, c] == (bwt == c)).all()


@pytest.mark.parametrize("n,seed", [(6, 20), (200, 21), (5000, 22)])
def test_lf_mapping_eq4_eq5(n, seed):
    """SA[C[b] + Occ(b, i)] = SA[i] - 1 for every row i other than the '$' row (Eq. 4, 5)."""
    R = random_text(n, seed)
    x = OracleIndex(R)
    sa, bwt, occ, C = x.sa.astype(np.int64), x.bwt, x.occ.astype(np.int64), x.C.astype(np.int64)
    for i in range(n + 1):
        if i == x.dollar_row:
            assert sa[i] == 0
            continue
        b = bwt[i]
        assert sa[C[b] + occ[i, b]] == sa[i] - 1


# ------------------------------------------------------------------ exact search vs brute force

def test_exact_exhaustive_tiny():
    """Every text over ACGT up to length 5 against every pattern up to length 3."""
    pats = [p for m in range(0, 4) for p in itertools.product(range(4), repeat=m)]
    codes, offs = csr([np.array(p, np.uint8) for p in pats])
    for n in range(1, 6):
        for R in itertools.product(range(4), repeat=n):
            R = np.array(R, np.uint8)
            x = OracleIndex(R)
            want = [bf.interval(R, p) if len(p) else (0, n) for p in pats]
            for method in ("definition", "listing1"):
                got = [tuple(v) for v in x.exact(codes, offs, oracle.FWD, method).tolist()]
                assert got == want, (R, method)


@pytest.mark.parametrize("seed", range(4))
def test_exact_random_both_strands(seed):
    rng = random.Random(seed)
    R = random_text(300 + 50 * seed, 100 + seed)
    x = OracleIndex(R)
    pats = []
    for _ in range(120):
        m = rng.randint(1, 12)
        if rng.random() < 0.6:
            p = rng.randint(0, len(R) - m)
            w = R[p:p + m].copy()
        else:
            w = np.array([rng.randint(0, 3) for _ in range(m)], np.uint8)
        if rng.random() < 0.1:
            w[rng.randrange(m)] = 4
        pats.append(w)
    codes, offs = csr(pats)
    want = []
    for w in pats:
        want.append(bf.interval(R, w))
        want.append(bf.interval(R, bf.revcomp(w)))
    for method in ("definition", "listing1"):
        got = [tuple(v) for v in x.exact(codes, offs, oracle.BOTH, method).tolist()]
        assert got == want, method


# ------------------------------------------------------------------ inexact search vs brute force

def hits_by_read(hits, offs, r):
    seg = hits[int(offs[r]):int(offs[r + 1])]
    return [(int(h["strand"]), int(h["k"]), int(h["l"]), int(h["d"])) for h in seg]


@pytest.mark.parametrize("seed", range(6))
def test_inexact_vs_enumeration(seed):
    rng = random.Random(1000 + seed)
    n = rng.randint(1, 14)
    R = random_text(n, 200 + seed)
    x = OracleIndex(R)
    xr = OracleIndex(reverse_text(R))
    pats, zs = [], []
    for _ in range(25):
        m = rng.randint(0, 4)
        w = [rng.randint(0, 3) for _ in range(m)]
        if m and rng.random() < 0.15:
            w[rng.randrange(m)] = 4
        pats.append(np.array(w, np.uint8))
        zs.append(rng.randint(0, 2))
    codes, offs = csr(pats)
    z = np.array(zs, np.uint8)
    results = {m: x.inexact(codes, offs, z, oracle.BOTH, m, rev=xr)
               for m in ("definition", "listing2", "listing2_darray")}
    for r, (w, zz) in enumerate(zip(pats, zs)):
        want = []
        for s, pat in enumerate((list(w), bf.revcomp(w))):
            for (k, l, d) in sorted(bf.hamming_hits(R, pat, zz)):
                want.append((s, k, l, d))
        want.sort()
        for m, (hits, hoffs) in results.items():
            assert hits_by_read(hits, hoffs, r) == want, (m, R.tolist(), w.tolist(), zz)


@pytest.mark.parametrize("seed", range(3))
def test_inexact_properties_medium(seed):
    """z=0 equals the exact search; hits(z) within hits(z+1) with the same d; the D
    bound changes nothing; strand 1 of W equals strand 0 of revcomp(W); definition
    equals Listing 2."""
    rng = np.random.default_rng(300 + seed)
    R = rng.integers(0, 4, 3000).astype(np.uint8)
    x = OracleIndex(R)
    xr = OracleIndex(reverse_text(R))
    pats = []
    for _ in range(60):
        m = int(rng.integers(8, 20))
        p = int(rng.integers(0, R.size - m))
        w = R[p:p + m].copy()
        flips = rng.random(m) < 0.1
        w[flips] = (w[flips] + rng.integers(1, 4, flips.sum())) % 4
        pats.append(w.astype(np.uint8))
    codes, offs = csr(pats)
    per_z = {}
    for z in (0, 1, 2):
        a = x.inexact(codes, offs, z, oracle.BOTH, "listing2")
        b = x.inexact(codes, offs, z, oracle.BOTH, "listing2_darray", rev=xr)
        assert np.array_equal(a[0], b[0]) and np.array_equal(a[1], b[1])
        if z <= 1:
            c = x.inexact(codes, offs, z, oracle.BOTH, "definition")
            assert np.array_equal(a[0], c[0]) and np.array_equal(a[1], c[1])
        per_z[z] = a
    ex = x.exact(codes, offs, oracle.BOTH)
    hits0, offs0 = per_z[0]
    for r in range(len(pats)):
        got = hits_by_read(hits0, offs0, r)
        want = [(s, int(ex[2 * r + s, 0]), int(ex[2 * r + s, 1]), 0)
                for s in (0, 1) if ex[2 * r + s, 0] <= ex[2 * r + s, 1]]
        assert got == want
    for z in (0, 1):
        lo, hi = per_z[z], per_z[z + 1]
        for r in range(len(pats)):
            assert set(hits_by_read(*lo, r)) <= set(hits_by_read(*hi, r))
    # strand symmetry
    rc = [np.array(bf.revcomp(w), np.uint8) for w in pats]
    c2, o2 = csr(rc)
    h1 = x.inexact(codes, offs, 1, oracle.REVCOMP, "listing2")
    h2 = x.inexact(c2, o2, 1, oracle.FWD, "listing2")
    a = [(int(h["read"]), int(h["k"]), int(h["l"]), int(h["d"])) for h in h1[0]]
    b = [(int(h["read"]), int(h["k"]), int(h["l"]), int(h["d"])) for h in h2[0]]
    assert a == b


def test_inexact_empty_read_and_all_n():
    R = enc("ACGTACGTTG")
    x = OracleIndex(R)
    codes, offs = csr([np.zeros(0, np.uint8), np.array([4, 4], np.uint8), np.array([4], np.uint8)])
    hits, hoffs = x.inexact(codes, offs, np.array([0, 1, 1], np.uint8), oracle.FWD, "listing2")
    assert hits_by_read(hits, hoffs, 0) == [(0, 0, 10, 0)]          # empty read: whole range
    assert hits_by_read(hits, hoffs, 1) == []                       # two N need z >= 2
    want = sorted((0, *bf.interval(R, [b]), 1) for b in range(4))
    assert hits_by_read(hits, hoffs, 2) == want                      # one N, z = 1: every base


# ------------------------------------------------------------------ D-array

@pytest.mark.parametrize("seed", range(5))
def test_darray_is_lower_bound(seed):
    rng = random.Random(500 + seed)
    n = rng.randint(3, 40)
    R = random_text(n, 600 + seed)
    xr = OracleIndex(reverse_text(R))
    pats = []
    for _ in range(30):
        m = rng.randint(1, 10)
        w = [rng.randint(0, 3) for _ in range(m)]
        if rng.random() < 0.2:
            w[rng.randrange(m)] = 4
        pats.append(np.array(w, np.uint8))
    codes, offs = csr(pats)
    D = xr.darray(codes, offs, oracle.FWD)[0]
    for r, w in enumerate(pats):
        d = D[int(offs[r]):int(offs[r + 1])].astype(int)
        assert all(d[i] <= d[i + 1] <= d[i] + 1 for i in range(len(d) - 1))
        for i in range(len(w)):
            assert d[i] <= bf.min_prefix_mismatch(R, w, i)
        # D counts completed segments that do not occur: recompute from substrings
        z, start = 0, 0
        for i in range(len(w)):
            seg = w[start:i + 1]
            if any(c > 3 for c in seg) or bf.occurrences(R, seg) == 0:
                z += 1
                start = i + 1
            assert d[i] == z


def test_darray_zero_for_substrings_and_both_strands_layout():
    R = random_text(500, 77)
    xr = OracleIndex(reverse_text(R))
    w = R[100:160].copy()
    codes, offs = csr([w, w[:10]])
    D = xr.darray(codes, offs, oracle.BOTH)
    assert D.shape == (2, 70)
    assert (D[0] == 0).all()
    rc = np.array(bf.revcomp(w), np.uint8)
    c2, o2 = csr([rc, np.array(bf.revcomp(w[:10]), np.uint8)])
    assert np.array_equal(D[1], xr.darray(c2, o2, oracle.FWD)[0])


# ------------------------------------------------------------------ text-only checkers

def _text_with_repeats(seed, n):
    rng = random.Random(seed)
    base = [rng.randrange(4) for _ in range(n)]
    for _ in range(n // 40):               # copies and short tandem runs, so intervals are wide
        a = rng.randrange(n - 20)
        b = rng.randrange(n - 20)
        base[b:b + 12] = base[a:a + 12]
    return np.array(base[:n], dtype=np.uint8)


@pytest.mark.parametrize("seed", [1, 2, 3])
def test_rank_scan_equals_sa_definition(seed):
    """The text scan and the suffix-array binary search agree on every kind of pattern:
    occurring, missing, with N, running past the text end, and empty."""
    R = _text_with_repeats(seed, 3000)
    x = OracleIndex(R)
    rng = random.Random(seed)
    pats = [np.zeros(0, np.uint8)]
    for _ in range(150):
        m = rng.randrange(1, 14)
        p = rng.randrange(R.size - m)
        pats.append(R[p:p + m].copy())                                  # occurs
        pats.append(np.array([rng.randrange(4) for _ in range(m)], np.uint8))
    pats.append(R[-5:].copy())                                          # a suffix of R
    pats.append(np.concatenate([R[-5:], [0]]).astype(np.uint8))         # runs past the end
    pats.append(np.array([0, 4, 1], np.uint8))                          # holds N
    codes, offs = csr(pats)
    want = x.exact(codes, offs, oracle.BOTH, "definition")
    got = oracle.exact_by_rank_scan(R, codes, offs, oracle.BOTH)
    assert np.array_equal(got, want)


@pytest.mark.parametrize("seed,z", [(4, 0), (5, 1), (6, 2), (7, 2)])
def test_pigeonhole_equals_hamming_ball(seed, z):
    """Hits from the pigeonhole windows and rank scans equal the Hamming-ball enumeration
    over the suffix-array index (including reads with N and strand 1)."""
    R = _text_with_repeats(seed, 2500)
    x = OracleIndex(R)
    rng = random.Random(seed)
    reads = []
    for i in range(40):
        m = rng.randrange(6, 13)
        p = rng.randrange(R.size - m)
        w = R[p:p + m].copy()
        for _ in range(rng.randrange(0, 3)):
            w[rng.randrange(m)] = rng.randrange(4)
        if i % 7 == 0:
            w[rng.randrange(m)] = 4
        if i % 3 == 0:
            w = oracle.strand_pattern(w, 1)
        reads.append(w)
    codes, offs = csr(reads)
    zz = np.full(len(reads), z, np.uint8)
    wh, wo = x.inexact(codes, offs, zz, oracle.BOTH, "definition")
    gh, go = oracle.pigeonhole_hits(R, codes, offs, zz, oracle.BOTH)
    assert np.array_equal(go, wo)
    for f in ("read", "k", "l", "strand", "d"):
        assert np.array_equal(gh[f], wh[f]), f
    assert wh.size > (len(reads) if z else len(reads) // 4)   # the check is not vacuous


@pytest.mark.parametrize("seed", [8, 9])
def test_rank_scan_batch_equals_sa_definition(seed):
    """The batched rank scan (key histogram plus full comparisons) agrees with the
    suffix-array definition on short and long patterns, patterns with N, patterns that
    reach the end of the text, and the empty pattern."""
    R = _text_with_repeats(seed, 6000)
    x = OracleIndex(R)
    rng = random.Random(seed)
    pats = [np.zeros(0, np.uint8)]
    for _ in range(200):
        m = rng.choice([1, 2, 5, 9, 10, 11, 17, 30, 45])
        p = rng.randrange(R.size - m)
        w = R[p:p + m].copy()
        if rng.random() < 0.3:
            w[rng.randrange(m)] = rng.randrange(4)
        if rng.random() < 0.1:
            w[rng.randrange(m)] = 4
        pats.append(w)
    for t in (3, 9, 10, 11, 25):
        pats.append(R[-t:].copy())                                      # suffixes of R
        pats.append(np.concatenate([R[-t:], [1, 2]]).astype(np.uint8))  # run past the end
    codes, offs = csr(pats)
    want = x.exact(codes, offs, oracle.BOTH, "definition")
    for threads in (1, 3):
        got = oracle.exact_by_rank_scan_batch(R, codes, offs, oracle.BOTH, threads=threads)
        assert np.array_equal(got, want), threads


@pytest.mark.parametrize("seed,z", [(10, 0), (11, 1), (12, 2)])
def test_pigeonhole_batch_equals_hamming_ball(seed, z):
    """The batched pigeonhole checker (seeds of at least 12 symbols found in one pass)
    equals the Hamming-ball enumeration, with reads long enough for the seed path, reads
    with N, and short reads that take the per-pattern path."""
    R = _text_with_repeats(seed, 8000)
    x = OracleIndex(R)
    rng = random.Random(seed)
    reads = []
    for i in range(36):
        m = rng.randrange(12 * (z + 1), 12 * (z + 1) + 14) if i % 6 else rng.randrange(5, 12)
        p = rng.randrange(R.size - m)
        w = R[p:p + m].copy()
        for _ in range(rng.randrange(0, z + 2)):
            w[rng.randrange(m)] = rng.randrange(4)
        if i % 7 == 0:
            w[rng.randrange(m)] = 4
        if i % 3 == 0:
            w = oracle.strand_pattern(w, 1)
        reads.append(w)
    codes, offs = csr(reads)
    zz = np.full(len(reads), z, np.uint8)
    wh, wo = x.inexact(codes, offs, zz, oracle.BOTH, "definition")
    for threads in (1, 4):
        gh, go = oracle.pigeonhole_hits_batch(R, codes, offs, zz, oracle.BOTH, threads=threads)
        assert np.array_equal(go, wo), threads
        for f in ("read", "k", "l", "strand", "d"):
            assert np.array_equal(gh[f], wh[f]), (threads, f)
    assert wh.size > len(reads) // 2                                    # the check is not vacuous


def test_full_rank_scan_equals_per_pattern_scan():
    """Full ranks from the batched scan are the per-pattern scan's (smaller suffixes,
    occurrences), misses and patterns with N included."""
    R = _text_with_repeats(13, 4000)
    rng = random.Random(13)
    pats = [np.zeros(0, np.uint8), np.array([4], np.uint8), np.array([3, 3, 3, 3, 3, 3, 3, 3, 3, 3, 3, 3], np.uint8)]
    for _ in range(120):
        m = rng.choice([1, 4, 10, 13, 30])
        w = np.array([rng.randrange(4) for _ in range(m)], np.uint8)
        if rng.random() < 0.4:
            p = rng.randrange(R.size - m)
            w = R[p:p + m].copy()
        if rng.random() < 0.15:
            w[rng.randrange(m)] = 4
        pats.append(w)
    codes, offs = csr(pats)
    got = oracle.exact_by_rank_scan_batch(R, codes, offs, oracle.FWD, threads=2, full_rank=True)
    lib = oracle.load()
    import ctypes as C
    for q, P in enumerate(pats):
        k, occ = C.c_int64(), C.c_int64()
        Pc = np.ascontiguousarray(P)
        lib.oracle_rank_scan(R.ctypes.data, R.size, Pc.ctypes.data if P.size else None, P.size, C.byref(k), C.byref(occ))
        assert got[q].tolist() == [k.value, (k.value + occ.value - 1) & 0xFFFFFFFF], q


# ------------------------------------------------------------------ Listing 2 with gaps

@pytest.mark.parametrize("seed", [21, 22, 23])
def test_gapped_listing2_equals_bruteforce(seed):
    """Listing 2 with its deletion and insertion branches, deduplicated per interval at the
    smallest cost, equals the brute force over edit scripts (text scans, no suffix array)
    and the oracle's own definition."""
    rng = random.Random(seed)
    n = rng.randrange(25, 60)
    R = np.array([rng.randrange(4) for _ in range(n)], np.uint8)
    for _ in range(4):                               # repeats, so intervals are wide
        a, b = rng.randrange(n - 6), rng.randrange(n - 6)
        R[b:b + 6] = R[a:a + 6]
    x = OracleIndex(R)
    xr = OracleIndex(reverse_text(R))
    reads, zs = [np.zeros(0, np.uint8)], [1]
    for i in range(14):
        m = rng.randrange(1, 5)
        p = rng.randrange(n - m)
        w = R[p:p + m].copy()
        if i % 3 == 0:
            w[rng.randrange(m)] = rng.randrange(4)
        if i % 5 == 0:
            w[rng.randrange(m)] = 4
        reads.append(w)
        zs.append(rng.randrange(0, 3))
    codes, offs = csr(reads)
    zz = np.array(zs, np.uint8)
    lh, lo = x.inexact(codes, offs, zz, oracle.FWD, "listing2_gaps")
    dh, do = x.inexact(codes, offs, zz, oracle.FWD, "definition_gaps")
    gh, go = x.inexact(codes, offs, zz, oracle.FWD, "listing2_gaps_darray", rev=xr)
    assert np.array_equal(lo, do) and np.array_equal(lo, go)
    for f in ("k", "l", "d"):
        assert np.array_equal(lh[f], dh[f]) and np.array_equal(lh[f], gh[f]), f
    total = 0
    for r, w in enumerate(reads):
        got = {(int(h["k"]), int(h["l"]), int(h["d"])) for h in lh[int(lo[r]):int(lo[r + 1])]}
        assert got == bf.gapped_hits(R, w, zs[r]), (r, w, zs[r])
        total += len(got)
    assert total > len(reads)                        # not vacuous


@pytest.mark.parametrize("seed", [24, 25])
def test_gapped_properties_medium(seed):
    """On reads of 20-40 bases: the D bound leaves the gapped hits unchanged; z = 0 gives
    the exact search; every substitution hit is a gapped hit at no higher cost; both
    strands behave alike."""
    R = _text_with_repeats(seed, 3000)
    x = OracleIndex(R)
    xr = OracleIndex(reverse_text(R))
    rng = random.Random(seed)
    reads = []
    for _ in range(40):
        m = rng.randrange(20, 41)
        p = rng.randrange(R.size - m)
        w = R[p:p + m].copy()
        for _ in range(rng.randrange(0, 3)):
            j = rng.randrange(len(w))
            if rng.random() < 0.5:
                w = np.delete(w, j)
            else:
                w = np.insert(w, j, rng.randrange(4)).astype(np.uint8)
        reads.append(w)
    codes, offs = csr(reads)
    for z in (0, 1, 2):
        zz = np.full(len(reads), z, np.uint8)
        gh, go = x.inexact(codes, offs, zz, oracle.BOTH, "listing2_gaps")
        dh, do = x.inexact(codes, offs, zz, oracle.BOTH, "listing2_gaps_darray", rev=xr)
        assert np.array_equal(go, do) and all(np.array_equal(gh[f], dh[f]) for f in ("k", "l", "strand", "d"))
        sh, so = x.inexact(codes, offs, zz, oracle.BOTH, "listing2")
        for r in range(len(reads)):
            g = {(int(h["strand"]), int(h["k"]), int(h["l"])): int(h["d"]) for h in gh[int(go[r]):int(go[r + 1])]}
            for h in sh[int(so[r]):int(so[r + 1])]:
                key = (int(h["strand"]), int(h["k"]), int(h["l"]))
                assert key in g and g[key] <= int(h["d"]), (z, r, key)
        if z == 0:
            ex = x.exact(codes, offs, oracle.BOTH, "definition")
            want = [(r, s, int(ex[2 * r + s, 0]), int(ex[2 * r + s, 1])) for r in range(len(reads)) for s in (0, 1)
                    if ex[2 * r + s, 0] <= ex[2 * r + s, 1]]
            got = [(int(h["read"]), int(h["strand"]), int(h["k"]), int(h["l"])) for h in gh]
            assert got == want and (gh["d"] == 0).all()
        else:
            assert gh.size > sh.size                 # gaps add hits
