"""Brute-force checkers that pin the oracle to something other than itself.

Pure Python over the raw text: no suffix array, no BWT, no Occ, no C. Each routine
follows a plain definition and is only usable on tiny inputs.
"""
from __future__ import annotations

import itertools

DOLLAR = -1   # '$' compares below every base


def suffix_key(R, j):
    return tuple(int(c) for c in R[j:]) + (DOLLAR,)


def suffix_array(R):
    """Rows of the sorted suffixes of R$ (Eq. 1), by Python's tuple order."""
    return sorted(range(len(R) + 1), key=lambda j: suffix_key(R, j))


def bwt(R):
    """Eq. 2 by forming the rotations of R$ and sorting them."""
    T = [int(c) for c in R] + [DOLLAR]
    rots = sorted(T[i:] + T[:i] for i in range(len(T)))
    return [r[-1] for r in rots]


def occurrences(R, P):
    m = len(P)
    P = tuple(int(c) for c in P)
    return sum(1 for j in range(len(R) - m + 1) if tuple(int(c) for c in R[j:j + m]) == P)


def rank(R, P):
    """Number of suffixes of R$ that sort strictly below the pattern P."""
    P = tuple(int(c) for c in P)
    return sum(1 for j in range(len(R) + 1) if suffix_key(R, j) < P)


def interval(R, P):
    """(k, l) with rows k..l starting with P; (1, 0) when P does not occur."""
    occ = occurrences(R, P) if all(0 <= int(c) <= 3 for c in P) else 0
    if occ == 0:
        return (1, 0)
    k = rank(R, P)
    return (k, k + occ - 1)


def revcomp(W):
    return [3 - int(c) if int(c) < 4 else int(c) for c in reversed(list(W))]


def hamming_hits(R, W, z):
    """{(k, l, d)} over every W' in ACGT^|W| with d = d_H(W, W') <= z and W' in R."""
    out = set()
    m = len(W)
    for Wp in itertools.product(range(4), repeat=m):
        d = sum(1 for a, b in zip(W, Wp) if int(a) != b)
        if d > z:
            continue
        if occurrences(R, Wp):
            k, l = interval(R, Wp)
            out.add((k, l, d))
    return out


def min_prefix_mismatch(R, W, i):
    """min over placements of W[0..i] inside R of the Hamming distance (inf if |R| < i+1)."""
    L = i + 1
    best = None
    for j in range(len(R) - L + 1):
        d = sum(1 for a, b in zip(W[:L], R[j:j + L]) if int(a) != int(b))
        best = d if best is None else min(best, d)
    return best if best is not None else 10 ** 9


def constrained_edit(W, Wp):
    """Edit cost of aligning W with Wp the way Listing 2 builds alignments: substitutions,
    deletions of W symbols and insertions of Wp symbols cost 1, a non-ACGT W symbol never
    matches, and nothing may be inserted before W[0]."""
    inf = 10 ** 9
    prev = [0] + [inf] * len(Wp)                 # no W symbol consumed: only the empty Wp
    for i in range(1, len(W) + 1):
        cur = [i] + [0] * len(Wp)
        for j in range(1, len(Wp) + 1):
            cur[j] = min(prev[j] + 1, cur[j - 1] + 1, prev[j - 1] + (int(W[i - 1]) != Wp[j - 1]))
        prev = cur
    return prev[len(Wp)]


def gapped_hits(R, W, z):
    """{(k, l, d)}: every Wp over ACGT within constrained edit cost d <= z of W that occurs
    in R (the empty Wp occurs everywhere: rows 0..n), once per interval at its smallest d."""
    best = {}
    m = len(W)
    for L in range(max(0, m - z), m + z + 1):
        for Wp in itertools.product(range(4), repeat=L):
            d = constrained_edit(W, Wp)
            if d > z:
                continue
            if L == 0:
                kl = (0, len(R))
            elif occurrences(R, Wp):
                kl = interval(R, Wp)
            else:
                continue
            if kl not in best or d < best[kl]:
                best[kl] = d
    return {(k, l, d) for (k, l), d in best.items()}
