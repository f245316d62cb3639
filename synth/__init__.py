"""Seeded synthetic inputs for the FM-index workloads.

This module only draws random numbers and assembles texts, reads, Occ queries and
request streams. It holds none of the FM-index arithmetic (no suffix order, no BWT,
no Occ, no search) so that both the CPU oracle and the GPU library can consume the
same inputs without sharing any of the method's code.

Random numbers come from one counter-based generator, SplitMix64 (Steele, Lea and
Flood, "Fast splittable pseudorandom number generators", OOPSLA 2014): output i of a
stream with seed s is the SplitMix64 finaliser applied to s + (i + 1) * 0x9E3779B97F4A7C15.

Symbol codes: A=0, C=1, G=2, T=3; 4 marks any non-ACGT read symbol (N).
"""
from __future__ import annotations

import dataclasses
import os
from concurrent.futures import ThreadPoolExecutor

import numpy as np

_GAMMA = np.uint64(0x9E3779B97F4A7C15)
_M1 = np.uint64(0xBF58476D1CE4E5B9)
_M2 = np.uint64(0x94D049BB133111EB)


def splitmix64(seed: int, counters: np.ndarray) -> np.ndarray:
    """SplitMix64 outputs for the given counters of the stream `seed` (uint64 array)."""
    with np.errstate(over="ignore"):
        z = counters.astype(np.uint64)          # a fresh array, updated in place below
        t = np.empty_like(z)
        z += np.uint64(1)
        z *= _GAMMA
        z += np.uint64(seed & 0xFFFFFFFFFFFFFFFF)
        for sh, mul in ((30, _M1), (27, _M2)):
            np.right_shift(z, np.uint64(sh), out=t)
            z ^= t
            z *= mul
        np.right_shift(z, np.uint64(31), out=t)
        z ^= t
        return z


def _in_blocks(n: int, block: int, fn) -> None:
    """fn(a, b) over [0, n) in blocks, on host threads when there are several blocks
    (numpy releases the GIL inside its array operations)."""
    spans = [(a, min(n, a + block)) for a in range(0, n, block)]
    if len(spans) <= 1:
        for a, b in spans:
            fn(a, b)
        return
    with ThreadPoolExecutor(max_workers=min(16, os.cpu_count() or 1, len(spans))) as ex:
        for f in [ex.submit(fn, a, b) for a, b in spans]:
            f.result()


class Rng:
    """A SplitMix64 stream that hands out consecutive blocks of outputs."""

    def __init__(self, seed: int):
        self.seed = int(seed)
        self.ctr = 0

    def u64(self, n: int) -> np.ndarray:
        out = splitmix64(self.seed, np.arange(self.ctr, self.ctr + n, dtype=np.uint64))
        self.ctr += n
        return out

    def uniform(self, n: int) -> np.ndarray:
        """Floats in [0, 1) from the top 53 bits."""
        return (self.u64(n) >> np.uint64(11)).astype(np.float64) * (1.0 / 9007199254740992.0)

    def integers(self, lo: int, hi: int, n: int) -> np.ndarray:
        """Integers uniform in [lo, hi] (both ends included), int64."""
        span = hi - lo + 1
        return lo + np.minimum((self.uniform(n) * span).astype(np.int64), span - 1)

    def bases(self, n: int) -> np.ndarray:
        """n i.i.d. uniform codes 0..3 (32 codes per 64-bit output, lowest bits first)."""
        nw = (n + 31) // 32
        out = np.empty(nw * 32, np.uint8)
        ctr0 = self.ctr
        self.ctr += nw

        def fill(a, b):
            words = splitmix64(self.seed, np.arange(ctr0 + a, ctr0 + b, dtype=np.uint64))
            shifts = np.arange(0, 64, 2, dtype=np.uint64)
            out[32 * a:32 * b] = ((words[:, None] >> shifts[None, :]) & np.uint64(3)).astype(np.uint8).reshape(-1)
        _in_blocks(nw, 1 << 20, fill)
        return out[:n] if n == out.size else out[:n].copy()

    def fork(self, n: int) -> "Rng":
        """A view of the next n outputs of this stream, which is advanced past them."""
        r = Rng(self.seed)
        r.ctr = self.ctr
        self.ctr += n
        return r

    def exponential(self, rate: float, n: int) -> np.ndarray:
        return -np.log1p(-self.uniform(n)) / rate


def substitute(codes: np.ndarray, rate, rng: Rng) -> np.ndarray:
    """I.i.d. substitutions: each position mutates with probability `rate` (scalar or
    per-position array) to one of the three other bases, chosen uniformly.

    One 64-bit draw per position: its high 32 bits decide the substitution (below
    rate * 2^32), its low 32 bits pick the replacement (floor(3 * low / 2^32) + 1 added
    to the code, mod 4). Positions holding code 4 (N) are left alone."""
    out = codes.copy()
    rate = np.broadcast_to(np.asarray(rate, dtype=np.float64), codes.shape)
    draws = rng.fork(codes.size)

    def block(a, b):
        u = splitmix64(draws.seed, np.arange(draws.ctr + a, draws.ctr + b, dtype=np.uint64))
        thr = (rate[a:b] * 4294967296.0).astype(np.uint64)
        hit = (u >> np.uint64(32)) < thr
        shift = (((u & np.uint64(0xFFFFFFFF)) * np.uint64(3)) >> np.uint64(32)).astype(np.uint8) + np.uint8(1)
        seg = out[a:b]
        m = hit & (seg < 4)
        seg[m] = (seg[m] + shift[m]) & 3
    _in_blocks(codes.size, 1 << 24, block)
    return out


def _complement_reverse(codes: np.ndarray) -> np.ndarray:
    """Minus-strand copy of a simulated fragment (used to simulate reads only)."""
    r = codes[::-1].copy()
    m = r < 4
    r[m] = 3 - r[m]
    return r


# --------------------------------------------------------------------------- texts

def iid_reference(n: int, seed: int) -> np.ndarray:
    return Rng(seed).bases(n)


def reference_with_repeats(n: int, seed: int, copy_frac: float = 0.05, copy_len=(500, 5000),
                           copy_sub: float = 0.02, tandem_frac: float = 0.0,
                           tandem_unit=(2, 50), tandem_len=(100, 1000)) -> np.ndarray:
    """A text of exactly n codes: (1 - copy_frac - tandem_frac) * n i.i.d. bases, then
    diverged copies of base-text segments and exact tandem repeats inserted at uniform
    positions until the length is n (the last insert is truncated).

    Copies: length ~ U[copy_len], source ~ U over the i.i.d. base text, i.i.d.
    substitutions at rate copy_sub. Tandem repeats: a unit of length ~ U[tandem_unit]
    of i.i.d. bases repeated to a region length ~ U[tandem_len], without divergence.
    """
    rng = Rng(seed)
    base_len = int(round(n * (1.0 - copy_frac - tandem_frac)))
    base = rng.bases(base_len)
    inserts = []
    total = base_len
    copy_goal = min(n, base_len + int(round(n * copy_frac)))
    while total < copy_goal:
        L = int(rng.integers(copy_len[0], copy_len[1], 1)[0])
        L = min(L, copy_goal - total, base_len)
        src = int(rng.integers(0, base_len - L, 1)[0])
        inserts.append(substitute(base[src:src + L], copy_sub, rng))
        total += L
    while total < n:
        u = int(rng.integers(tandem_unit[0], tandem_unit[1], 1)[0])
        L = int(rng.integers(tandem_len[0], tandem_len[1], 1)[0])
        L = min(L, n - total)
        unit = rng.bases(u)
        inserts.append(np.resize(unit, L))
        total += L
    if not inserts:
        return base
    pos = rng.integers(0, base_len, len(inserts))
    order = np.argsort(pos, kind="stable")
    pieces = []
    prev = 0
    for j in order:
        p = int(pos[j])
        pieces.append(base[prev:p])
        pieces.append(inserts[j])
        prev = p
    pieces.append(base[prev:])
    out = np.concatenate(pieces)
    assert out.size == n
    return out


def reference_families(n: int, seed: int, iid_frac: float = 0.55, families: int = 500,
                       fam_len=(100, 6000), div=(0.05, 0.15)) -> np.ndarray:
    """Genome-like text: iid_frac of n i.i.d. bases with interspersed copies of
    `families` consensus sequences (length log-uniform in fam_len). Each copy is a
    random 5'-truncation of its consensus with i.i.d. substitutions at a per-copy rate
    ~ U[div]. Copies are inserted at uniform positions until the length is n.

    Draw order: the i.i.d. bases; the family lengths and consensus bases; then, in
    blocks of 2^16 copies, the family, start and divergence of each (the last copy is
    truncated to fill n exactly); the substitution draws of the copies in order; the
    insertion positions. Copies inserted at the same position keep their draw order."""
    rng = Rng(seed)
    base_len = int(round(n * iid_frac))
    base = rng.bases(base_len)
    lens = np.exp(np.log(fam_len[0]) + rng.uniform(families) * (np.log(fam_len[1]) - np.log(fam_len[0])))
    cons = [rng.bases(int(x)) for x in lens]
    clen = np.array([c.size for c in cons], np.int64)
    coff = np.zeros(families + 1, np.int64)
    np.cumsum(clen, out=coff[1:])
    allc = np.concatenate(cons)
    need = n - base_len
    fams, starts, rates, plens = [], [], [], []
    got = 0
    while got < need:
        k = 1 << 16
        f = rng.integers(0, families - 1, k)
        st = np.minimum((rng.uniform(k) * clen[f]).astype(np.int64), clen[f] - 1)
        rt = div[0] + rng.uniform(k) * (div[1] - div[0])
        pl = clen[f] - st
        take = min(k, int(np.searchsorted(np.cumsum(pl), need - got, side="left")) + 1)
        pl = pl[:take].copy()
        over = got + int(pl.sum()) - need
        if over > 0:
            pl[-1] -= over
        fams.append(f[:take])
        starts.append(st[:take])
        rates.append(rt[:take])
        plens.append(pl)
        got += int(pl.sum())
    f = np.concatenate(fams) if fams else np.zeros(0, np.int64)
    st = np.concatenate(starts) if starts else np.zeros(0, np.int64)
    rt = np.concatenate(rates) if rates else np.zeros(0)
    pl = np.concatenate(plens) if plens else np.zeros(0, np.int64)
    poff = np.zeros(pl.size + 1, np.int64)
    np.cumsum(pl, out=poff[1:])
    copies = np.empty(need, np.uint8)
    sub = rng.fork(need)             # one substitution draw per copied position, in order

    def make(a, b):
        lo, hi = int(poff[a]), int(poff[b])
        src = np.repeat(coff[f[a:b]] + st[a:b] - (poff[a:b] - lo), pl[a:b]) + np.arange(hi - lo, dtype=np.int64)
        r = Rng(seed)
        r.ctr = sub.ctr + lo
        copies[lo:hi] = substitute(allc[src], np.repeat(rt[a:b], pl[a:b]), r)
    _in_blocks(pl.size, 1 << 13, make)
    pos = rng.integers(0, base_len, pl.size)
    order = np.argsort(pos, kind="stable")
    out = np.empty(n, np.uint8)
    o = prev = 0
    for j in order.tolist():
        p = int(pos[j])
        if p > prev:
            out[o:o + p - prev] = base[prev:p]
            o += p - prev
            prev = p
        c0, c1 = int(poff[j]), int(poff[j + 1])
        out[o:o + c1 - c0] = copies[c0:c1]
        o += c1 - c0
    out[o:] = base[prev:]
    assert o + base_len - prev == n
    return out


# --------------------------------------------------------------------------- reads

@dataclasses.dataclass
class Reads:
    codes: np.ndarray        # uint8, concatenated reads
    offs: np.ndarray         # uint64, count + 1 offsets
    z: np.ndarray            # uint8, mismatch budget per read
    pos: np.ndarray          # int64, sampled start (-1 for random reads)
    strand: np.ndarray       # uint8, 1 when sampled from the minus strand

    @property
    def count(self) -> int:
        return int(self.offs.size - 1)

    def read(self, r: int) -> np.ndarray:
        return self.codes[int(self.offs[r]):int(self.offs[r + 1])]

    def subset(self, idx) -> "Reads":
        idx = np.asarray(idx, dtype=np.int64)
        lens = (self.offs[idx + 1] - self.offs[idx]).astype(np.int64)
        offs = np.zeros(idx.size + 1, dtype=np.uint64)
        np.cumsum(lens, out=offs[1:])
        parts = [self.read(int(r)) for r in idx]
        codes = np.concatenate(parts) if parts else np.zeros(0, np.uint8)
        return Reads(codes.astype(np.uint8), offs, self.z[idx].copy(), self.pos[idx].copy(),
                     self.strand[idx].copy())


def _gather(ref: np.ndarray, starts: np.ndarray, lens: np.ndarray, minus: np.ndarray) -> np.ndarray:
    """Concatenated fragments ref[start, start + len), reverse-complemented where minus
    is set; built in chunks of reads to bound the temporaries."""
    offs = np.zeros(lens.size + 1, dtype=np.int64)
    np.cumsum(lens, out=offs[1:])
    out = np.empty(int(offs[-1]), dtype=np.uint8)

    def block(a, b):
        ln = lens[a:b].astype(np.int64)
        base = offs[a:b] - offs[a]
        rid = np.repeat(np.arange(b - a, dtype=np.int32), ln)
        j = np.arange(int(offs[b] - offs[a]), dtype=np.int64) - base[rid]
        mrow = minus[a:b].astype(bool)[rid]
        first = starts[a:b].astype(np.int64)[rid]
        idx = np.where(mrow, first + (ln[rid] - 1 - j), first + j)
        seg = ref[idx]
        seg[mrow] = 3 - seg[mrow]
        out[offs[a]:offs[b]] = seg
    _in_blocks(lens.size, 1 << 18, block)
    return out


def simulate_reads(ref: np.ndarray, count: int, seed: int, length=(100, 100), sub=(0.01, 0.01),
                   z=(1, 1), both_strands: bool = True) -> Reads:
    """Reads sampled from uniform positions of the text (and of its reverse complement
    with probability 1/2), with i.i.d. substitutions at a per-read rate ~ U[sub]."""
    rng = Rng(seed)
    lens = rng.integers(length[0], length[1], count)
    n = ref.size
    starts = np.minimum((rng.uniform(count) * (n - lens + 1)).astype(np.int64), n - lens)
    minus = (rng.uniform(count) < 0.5) if both_strands else np.zeros(count, dtype=bool)
    rate = sub[0] + rng.uniform(count) * (sub[1] - sub[0])
    codes = _gather(ref, starts, lens, minus)
    per_char = np.repeat(rate, lens)
    codes = substitute(codes, per_char, rng)
    zz = rng.integers(z[0], z[1], count).astype(np.uint8)
    offs = np.zeros(count + 1, dtype=np.uint64)
    np.cumsum(lens, out=offs[1:])
    return Reads(codes, offs, zz, starts, minus.astype(np.uint8))


def random_reads(count: int, length: int, seed: int, z: int = 0) -> Reads:
    rng = Rng(seed)
    codes = rng.bases(count * length)
    offs = (np.arange(count + 1, dtype=np.uint64) * np.uint64(length))
    return Reads(codes, offs, np.full(count, z, np.uint8), np.full(count, -1, np.int64),
                 np.zeros(count, np.uint8))


def concat_reads(a: Reads, b: Reads) -> Reads:
    offs = np.concatenate([a.offs[:-1], b.offs + a.offs[-1]]).astype(np.uint64)
    return Reads(np.concatenate([a.codes, b.codes]), offs, np.concatenate([a.z, b.z]),
                 np.concatenate([a.pos, b.pos]), np.concatenate([a.strand, b.strand]))


def occ8_queries(n: int, count: int, seed: int, kind: str = "uniform") -> np.ndarray:
    """(k, l) pairs as a (count, 2) uint32 array. 'uniform': k in [0, n+1] and l in
    [0, n] independent; 'narrow': l uniform, k = l + 1 - w with w ~ U[0, 8], k >= 0."""
    rng = Rng(seed)
    if kind == "uniform":
        k = rng.integers(0, n + 1, count)
        l = rng.integers(0, n, count)
    elif kind == "narrow":
        l = rng.integers(0, n, count)
        w = rng.integers(0, 8, count)
        k = np.maximum(l + 1 - w, 0)
    else:
        raise ValueError(kind)
    return np.stack([k, l], axis=1).astype(np.uint32)


# --------------------------------------------------------------------------- workloads

@dataclasses.dataclass
class Workload:
    name: str
    ref: np.ndarray
    reads: Reads
    flags: str           # "fwd" or "both"
    z_mode: str          # "exact", "fixed", "mixed"


def small_exact_workload() -> Workload:
    """65,536 i.i.d. bases; 10,000 length-32 queries, half copied from uniform text
    positions, half uniform random; exact search on the forward strand."""
    ref = iid_reference(65536, 1001)
    rng = Rng(2001)
    half = 5000
    starts = rng.integers(0, ref.size - 32, half)
    copied = _gather(ref, starts, np.full(half, 32, np.int64), np.zeros(half, bool))
    rand = rng.bases(half * 32)
    codes = np.concatenate([copied, rand])
    offs = np.arange(2 * half + 1, dtype=np.uint64) * np.uint64(32)
    reads = Reads(codes, offs, np.zeros(2 * half, np.uint8),
                  np.concatenate([starts, np.full(half, -1)]), np.zeros(2 * half, np.uint8))
    return Workload("small-exact", ref, reads, "fwd", "exact")


def repeats_2e24_reference(n: int = 1 << 24) -> np.ndarray:
    return reference_with_repeats(n, 1002, copy_frac=0.05, copy_len=(500, 5000), copy_sub=0.02)


def reads_2e24(ref: np.ndarray, count: int = 1_000_000) -> Reads:
    return simulate_reads(ref, count, 2002, length=(100, 100), sub=(0.01, 0.01), z=(1, 1))


def repeats_2e28_reference(n: int = 1 << 28) -> np.ndarray:
    return reference_with_repeats(n, 1003, copy_frac=0.05, copy_len=(500, 5000), copy_sub=0.02,
                                  tandem_frac=0.01, tandem_unit=(2, 50), tandem_len=(100, 1000))


def mixed_reads_2e28(ref: np.ndarray, count: int = 4_000_000, seed: int = 2003) -> Reads:
    return simulate_reads(ref, count, seed, length=(50, 250), sub=(0.005, 0.03), z=(0, 2))


def genome_like_reference(n: int = 3_100_000_000) -> np.ndarray:
    return reference_families(n, 1004)


def genome_reads(ref: np.ndarray, count: int = 16_000_000, seed: int = 2004) -> Reads:
    return simulate_reads(ref, count, seed, length=(150, 150), sub=(0.01, 0.01), z=(2, 2))


@dataclasses.dataclass
class Request:
    rid: int
    arrival: float       # seconds from stream start
    reads: Reads


def request_stream(ref: np.ndarray, count: int, rate: float, seed: int = 3005,
                   size=(1, 20000), length=(50, 250), sub=(0.005, 0.03), z=(0, 2)) -> list:
    """Poisson arrivals at `rate` requests/s; each request holds U{size} reads with
    lengths ~ U[length], substitution rate ~ U[sub] and budgets z ~ U{z}."""
    rng = Rng(seed)
    gaps = rng.exponential(rate, count)
    arrivals = np.cumsum(gaps)
    sizes = rng.integers(size[0], size[1], count)
    out = []
    for i in range(count):
        rd = simulate_reads(ref, int(sizes[i]), seed * 1_000_003 + i, length=length, sub=sub, z=z)
        out.append(Request(i, float(arrivals[i]), rd))
    return out
