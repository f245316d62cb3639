"""Plants plausible mistakes in copies of the oracle source (on the CPU) and checks that
the pins catch every one of them: a dropped term, a wrong sign or index, a swapped
operand. The real oracle is never modified."""
import os
import random

import numpy as np
import pytest

import oracle
from oracle import OracleIndex, reverse_text
from tests import bruteforce as bf

SRC = os.path.join(os.path.dirname(oracle.__file__), "fm_oracle.c")

MUTANTS = {
    "dollar_sorts_high": ("return (la < lb) ? -1 : (la > lb);", "return (la > lb) ? -1 : (la < lb);"),
    "bwt_no_shift": ("BWT[i] = R[SA[i] - 1];", "BWT[i] = R[SA[i]];"),
    "occ_exclusive": ("if (BWT[k] < 4) run[BWT[k]]++;\n        memcpy(occ + 4 * k, run, sizeof run);",
                      "memcpy(occ + 4 * k, run, sizeof run);\n        if (BWT[k] < 4) run[BWT[k]]++;"),
    "occ_minus1_nonzero": ("if (k < 0) return 0;", "if (k < 0) return 1;"),
    "c_inclusive": ("C[c] = acc;\n        acc += occ_at(x, c, x->n);", "acc += occ_at(x, c, x->n);\n        C[c] = acc;"),
    "listing1_k_index": ("k = (int64_t)x->C[b] + occ_at(x, b, k - 1) + 1;\n        l = (int64_t)x->C[b] + occ_at(x, b, l);\n    }",
                         "k = (int64_t)x->C[b] + occ_at(x, b, k) + 1;\n        l = (int64_t)x->C[b] + occ_at(x, b, l);\n    }"),
    "listing1_drop_plus1": ("k = (int64_t)x->C[b] + occ_at(x, b, k - 1) + 1;\n        l = (int64_t)x->C[b] + occ_at(x, b, l);\n    }",
                            "k = (int64_t)x->C[b] + occ_at(x, b, k - 1);\n        l = (int64_t)x->C[b] + occ_at(x, b, l);\n    }"),
    "listing2_swap_cost": ("b == c->W[i] ? z : z - 1, kb, lb}", "b == c->W[i] ? z - 1 : z, kb, lb}"),
    "listing2_strict_guard": ("if (kb > lb) continue;", "if (kb >= lb) continue;"),
    "listing2_k_index": ("const int64_t kb = (int64_t)c->x->C[b] + occ_at(c->x, b, k - 1) + 1;",
                         "const int64_t kb = (int64_t)c->x->C[b] + occ_at(c->x, b, k) + 1;"),
    "dbound_too_strong": ("const int need = (c->D && i >= 0) ? c->D[i] : 0;",
                          "const int need = (c->D && i >= 0) ? c->D[i] + 1 : 0;"),
    "darray_no_restart": ("k = 0;\n            l = rev->n;", "k = 0;\n            l = 0;"),
    "revcomp_no_complement": ("P[i] = c < 4 ? (uint8_t)(3 - c) : c;", "P[i] = c;"),
    "definition_dollar_high": ("if (s + j >= x->n) return -1;", "if (s + j >= x->n) return 1;"),
    "ball_budget_plus1": ("if (used == budget) return;", "if (used == budget + 1) return;"),
    "occ8_k_index": ("o[c] = occ_at(x, c, k - 1);", "o[c] = occ_at(x, c, k);"),
    "rank_scan_prefix_not_smaller": ("if (r < 0 || (r == 0 && avail < m)) less++;", "if (r < 0) less++;"),
    "pigeonhole_strict_budget": ("if (hamming(R + s, P, m) > z) continue;", "if (hamming(R + s, P, m) >= z) continue;"),
    "pigeonhole_piece_offset": ("const int64_t s = p - a[i];", "const int64_t s = p;"),
    "gap_insert_consumes": ("(inex_child){i, z - 1, kb, lb}", "(inex_child){i - 1, z - 1, kb, lb}"),
    "gap_delete_free": ("(inex_child){i - 1, z - 1, k, l}", "(inex_child){i - 1, z, k, l}"),
    "gap_leading_insert_allowed": ("if (i == 0) v = j == 0 ? 0 : inf;", "if (i == 0) v = (int)j;"),
    "gap_keeps_largest_cost": ("return (a->d > b->d) - (a->d < b->d);", "return (a->d < b->d) - (a->d > b->d);"),
}


def csr(patterns):
    codes = np.concatenate([np.asarray(p, np.uint8) for p in patterns]) if patterns else np.zeros(0, np.uint8)
    offs = np.zeros(len(patterns) + 1, np.uint64)
    offs[1:] = np.cumsum([len(p) for p in patterns])
    return codes, offs


def battery(lib):
    """Runs the pins against the library at `lib`; raises AssertionError on the first miss."""
    # Fig. 1
    x = OracleIndex(np.array([0, 1, 0, 2], np.uint8), lib)
    assert x.sa.tolist() == [4, 0, 2, 1, 3]
    assert x.bwt.tolist() == [2, 4, 1, 0, 0]
    assert x.occ.tolist() == [[0, 0, 1, 0], [0, 0, 1, 0], [0, 1, 1, 0], [1, 1, 1, 0], [2, 1, 1, 0]]
    assert x.C.tolist() == [0, 2, 3, 4, 4]
    assert x.occ8(np.array([[1, 2], [3, 3], [0, 4]], np.uint32)).tolist() == [
        [0, 0, 1, 0, 0, 1, 1, 0], [0, 1, 1, 0, 1, 1, 1, 0], [0, 0, 0, 0, 2, 1, 1, 0]]
    rng = random.Random(7)
    for trial in range(3):
        R = np.array([rng.randint(0, 3) for _ in range(rng.randint(4, 12))], np.uint8)
        x = OracleIndex(R, lib)
        xr = OracleIndex(reverse_text(R), lib)
        pats = [np.array([rng.randint(0, 3) for _ in range(rng.randint(1, 4))], np.uint8) for _ in range(12)]
        codes, offs = csr(pats)
        want = []
        for w in pats:
            want += [bf.interval(R, w), bf.interval(R, bf.revcomp(w))]
        for method in ("definition", "listing1"):
            got = [tuple(v) for v in x.exact(codes, offs, oracle.BOTH, method).tolist()]
            assert got == want
        # the text-only checkers, on a pattern set that includes one running past the end
        tail = [R[-2:].copy(), np.concatenate([R[-2:], [0]]).astype(np.uint8)]
        c2, o2 = csr(pats + tail)
        want2 = want + sum(([bf.interval(R, w), bf.interval(R, bf.revcomp(w))] for w in tail), [])
        assert [tuple(v) for v in oracle.exact_by_rank_scan(R, c2, o2, oracle.BOTH, lib).tolist()] == want2
        z = np.array([rng.randint(0, 2) for _ in pats], np.uint8)
        for method in ("definition", "listing2", "listing2_darray", "pigeonhole"):
            if method == "pigeonhole":
                hits, hoffs = oracle.pigeonhole_hits(R, codes, offs, z, oracle.BOTH, lib)
            else:
                hits, hoffs = x.inexact(codes, offs, z, oracle.BOTH, method, rev=xr)
            for r, w in enumerate(pats):
                seg = hits[int(hoffs[r]):int(hoffs[r + 1])]
                got = sorted((int(h["strand"]), int(h["k"]), int(h["l"]), int(h["d"])) for h in seg)
                exp = sorted([(0, *t) for t in bf.hamming_hits(R, w, int(z[r]))] +
                             [(1, *t) for t in bf.hamming_hits(R, bf.revcomp(w), int(z[r]))])
                assert got == exp
        # Listing 2 with gaps, its D-bounded form and its definition, against edit scripts
        gp = [p[:3] for p in pats[:6]] + [np.zeros(0, np.uint8)]
        gc, go = csr(gp)
        gz = np.array([rng.randint(0, 1) for _ in gp], np.uint8)
        for method in ("listing2_gaps", "listing2_gaps_darray", "definition_gaps"):
            hits, hoffs = x.inexact(gc, go, gz, oracle.FWD, method, rev=xr)
            for r, w in enumerate(gp):
                seg = hits[int(hoffs[r]):int(hoffs[r + 1])]
                assert sorted((int(h["k"]), int(h["l"]), int(h["d"])) for h in seg) == sorted(
                    bf.gapped_hits(R, w, int(gz[r]))), method
        D = xr.darray(codes, offs, oracle.FWD)[0]
        for r, w in enumerate(pats):
            d = D[int(offs[r]):int(offs[r + 1])]
            zc, start = 0, 0
            for i in range(len(w)):
                if bf.occurrences(R, w[start:i + 1]) == 0:
                    zc += 1
                    start = i + 1
                assert d[i] == zc


def test_battery_passes_on_real_oracle():
    battery(oracle._LIB if os.path.exists(oracle._LIB) else oracle.build())


@pytest.mark.parametrize("name", sorted(MUTANTS))
def test_mutant_is_caught(name, tmp_path):
    old, new = MUTANTS[name]
    src = open(SRC).read()
    assert src.count(old) == 1, "mutation site drifted: " + name
    path = tmp_path / "mutant.c"
    path.write_text(src.replace(old, new))
    lib = oracle.build(str(path), str(tmp_path / ("lib_%s.so" % name)))
    with pytest.raises(AssertionError):
        battery(lib)
