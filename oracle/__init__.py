"""CPU oracle for the FM-index hot path -- TEST INFRASTRUCTURE ONLY.

Plain, slow, obviously correct reference computations written from "Vectorized
Character Counting for Faster Pattern Matching" (Snytsar); the arithmetic lives in
fm_oracle.c (compiled with gcc, loaded with ctypes). Only the test suite, the smoke
check and the benchmark's CPU-baseline leg may import this package. It shares no code
with the GPU library and the GPU library never imports it.

What each function follows:
  OracleIndex          suffix array by direct comparison (Background, Eq. 1), BWT from
                       the SA (Eq. 2), Occ by linear scan and C (Background, Fig. 1)
  occ8                 Occ(c, k-1) and Occ(c, l) for all four bases (the eight values of
                       one inexact step, Background)
  exact                SA interval by its definition (method="definition") or by the
                       backward exact match (Listing 1, method="listing1")
  darray               BWA's D lower bound over the index of reverse(R)
  inexact              hit set by Hamming-ball enumeration (method="definition") or by the
                       inexact match restricted to substitutions (Listing 2,
                       method="listing2", optionally with the D bound)
  rank_interval,       text-only checkers for large texts (no SA, BWT, Occ or C): the SA
  exact_by_rank_scan   interval of a pattern from the number of smaller suffixes and of
                       occurrences, counted by one scan of the text
  pigeonhole_hits      the substitution hit set from the windows of R that agree exactly
                       with one of z+1 pieces of the pattern (pigeonhole principle)
Every function is pinned by tests/test_oracle_*.py (Fig. 1 values, invariants,
brute force on tiny inputs); none is "parity unpinned".
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "fm_oracle.c")
_LIB = os.path.join(_HERE, "_build", "liboracle.so")

FWD, REVCOMP, BOTH = 1, 2, 3

HIT_DTYPE = np.dtype([("read", "<u4"), ("k", "<u4"), ("l", "<u4"), ("strand", "u1"),
                      ("d", "u1"), ("pad", "<u2")])


def build(src: str = _SRC, out: str = _LIB, extra: tuple = ()) -> str:
    """Compile the oracle with gcc into a shared object."""
    os.makedirs(os.path.dirname(out), exist_ok=True)
    tmp = out + ".tmp%d" % os.getpid()
    subprocess.check_call(["gcc", "-O2", "-std=c99", "-shared", "-fPIC", "-pthread", *extra, "-o", tmp, src])
    os.replace(tmp, out)
    return out


_lib_cache: dict = {}


def load(path: str = _LIB) -> C.CDLL:
    if path in _lib_cache:
        return _lib_cache[path]
    if not os.path.exists(path):
        if path != _LIB:
            raise FileNotFoundError(path)
        build()
    lib = C.CDLL(path)
    p, i64, u8p, u32p, u64p = C.c_void_p, C.c_int64, C.c_void_p, C.c_void_p, C.c_void_p
    lib.oracle_index_new.restype = p
    lib.oracle_index_new.argtypes = [u8p, i64]
    lib.oracle_index_free.argtypes = [p]
    lib.oracle_index_n.restype = i64
    lib.oracle_index_n.argtypes = [p]
    lib.oracle_index_dollar_row.restype = i64
    lib.oracle_index_dollar_row.argtypes = [p]
    lib.oracle_index_sa.restype = p
    lib.oracle_index_sa.argtypes = [p]
    lib.oracle_index_bwt.restype = p
    lib.oracle_index_bwt.argtypes = [p]
    lib.oracle_index_occ.restype = p
    lib.oracle_index_occ.argtypes = [p]
    lib.oracle_index_c.argtypes = [p, u64p]
    lib.oracle_occ8.argtypes = [p, u32p, i64, u32p]
    lib.oracle_exact.argtypes = [p, u8p, u64p, i64, C.c_int, C.c_int, u32p]
    lib.oracle_darray.argtypes = [p, u8p, u64p, i64, C.c_int, u8p]
    lib.oracle_inexact.restype = i64
    lib.oracle_inexact.argtypes = [p, p, u8p, u64p, u8p, i64, C.c_int, C.c_int, p, i64, u64p, u64p]
    lib.oracle_rank_scan.argtypes = [u8p, i64, u8p, i64, C.POINTER(C.c_int64), C.POINTER(C.c_int64)]
    lib.oracle_rank_scan.restype = None
    lib.oracle_hits_pigeonhole.argtypes = [u8p, i64, u8p, i64, C.c_int, u32p, i64]
    lib.oracle_hits_pigeonhole.restype = i64
    lib.oracle_rank_scan_batch.argtypes = [u8p, i64, u8p, u64p, i64, C.c_int, p, p]
    lib.oracle_rank_scan_batch.restype = C.c_int
    lib.oracle_hits_pigeonhole_batch.argtypes = [u8p, i64, u8p, u64p, p, i64, C.c_int, u32p, i64, p]
    lib.oracle_hits_pigeonhole_batch.restype = i64
    _lib_cache[path] = lib
    return lib


def _ptr(a: np.ndarray) -> int:
    return a.ctypes.data


class OracleIndex:
    """SA, BWT, Occ table and C of the text R (codes 0..3), built on the host."""

    def __init__(self, R: np.ndarray, lib_path: str = _LIB):
        self._lib = load(lib_path)
        R = np.ascontiguousarray(R, dtype=np.uint8)
        if R.size and R.max() > 3:
            raise ValueError("text codes must be 0..3")
        self._R = R
        self.n = int(R.size)
        h = self._lib.oracle_index_new(_ptr(R) if R.size else None, self.n)
        if not h:
            raise MemoryError("oracle index")
        self._h = h

    def __del__(self):
        h = getattr(self, "_h", None)
        if h:
            self._lib.oracle_index_free(h)
            self._h = None

    def _view(self, addr, dtype, count) -> np.ndarray:
        buf = (C.c_char * (np.dtype(dtype).itemsize * count)).from_address(addr)
        return np.frombuffer(buf, dtype=dtype, count=count).copy()

    @property
    def sa(self) -> np.ndarray:
        return self._view(self._lib.oracle_index_sa(self._h), np.uint32, self.n + 1)

    @property
    def bwt(self) -> np.ndarray:
        """n+1 codes: 0..3, and 4 at the '$' row."""
        return self._view(self._lib.oracle_index_bwt(self._h), np.uint8, self.n + 1)

    @property
    def occ(self) -> np.ndarray:
        """(n+1, 4) table: occ[k, c] = Occ(c, k)."""
        return self._view(self._lib.oracle_index_occ(self._h), np.uint32, 4 * (self.n + 1)).reshape(-1, 4)

    @property
    def dollar_row(self) -> int:
        return int(self._lib.oracle_index_dollar_row(self._h))

    @property
    def C(self) -> np.ndarray:
        out = np.zeros(5, dtype=np.uint64)
        self._lib.oracle_index_c(self._h, _ptr(out))
        return out

    def occ8(self, q: np.ndarray) -> np.ndarray:
        q = np.ascontiguousarray(q, dtype=np.uint32).reshape(-1, 2)
        out = np.zeros((q.shape[0], 8), dtype=np.uint32)
        self._lib.oracle_occ8(self._h, _ptr(q), q.shape[0], _ptr(out))
        return out

    def exact(self, codes, offs, strands: int = FWD, method: str = "definition") -> np.ndarray:
        codes = np.ascontiguousarray(codes, dtype=np.uint8)
        offs = np.ascontiguousarray(offs, dtype=np.uint64)
        nreads = offs.size - 1
        ns = bin(strands & 3).count("1")
        out = np.zeros((nreads * ns, 2), dtype=np.uint32)
        m = {"definition": 0, "listing1": 1}[method]
        self._lib.oracle_exact(self._h, _ptr(codes) if codes.size else None, _ptr(offs), nreads,
                               strands, m, _ptr(out))
        return out

    def darray(self, codes, offs, strands: int = FWD) -> np.ndarray:
        """D for each requested strand: an array (strands, total_len) of uint8."""
        codes = np.ascontiguousarray(codes, dtype=np.uint8)
        offs = np.ascontiguousarray(offs, dtype=np.uint64)
        ns = bin(strands & 3).count("1")
        out = np.zeros((ns, codes.size), dtype=np.uint8)
        self._lib.oracle_darray(self._h, _ptr(codes) if codes.size else None, _ptr(offs),
                                offs.size - 1, strands, _ptr(out) if out.size else None)
        return out

    def inexact(self, codes, offs, z, strands: int = BOTH, method: str = "listing2",
                rev: "OracleIndex | None" = None, return_nodes: bool = False):
        """Hits sorted by (read, strand, k) as a HIT_DTYPE array plus CSR offsets.
        Methods: "definition", "listing2", "listing2_darray" (substitutions only), and with
        the deletion and insertion branches of Listing 2 too: "listing2_gaps",
        "listing2_gaps_darray" and "definition_gaps" (edit costs, small inputs only),
        whose hits are sorted by l as well and kept once per interval at the smallest cost."""
        codes = np.ascontiguousarray(codes, dtype=np.uint8)
        offs = np.ascontiguousarray(offs, dtype=np.uint64)
        nreads = offs.size - 1
        z = np.ascontiguousarray(np.broadcast_to(np.asarray(z, dtype=np.uint8), (nreads,)))
        m = {"definition": 0, "listing2": 1, "listing2_darray": 2, "listing2_gaps": 3, "listing2_gaps_darray": 4,
             "definition_gaps": 5}[method]
        if m in (2, 4) and rev is None:
            raise ValueError("the D bound needs the index of reverse(R)")
        hit_offs = np.zeros(nreads + 1, dtype=np.uint64)
        nodes = np.zeros(max(nreads, 1), dtype=np.uint64)
        cap = max(16, 4 * nreads)
        while True:
            out = np.zeros(cap, dtype=HIT_DTYPE)
            total = self._lib.oracle_inexact(self._h, rev._h if rev is not None else None,
                                             _ptr(codes) if codes.size else None, _ptr(offs),
                                             _ptr(z) if z.size else None, nreads, strands, m,
                                             _ptr(out), cap, _ptr(hit_offs), _ptr(nodes))
            if total <= cap:
                break
            cap = int(total)
        hits = out[:total].copy()
        if return_nodes:
            return hits, hit_offs, nodes[:nreads].copy()
        return hits, hit_offs


def reverse_text(R: np.ndarray) -> np.ndarray:
    """reverse(R): the text whose index gives the D-array bound (BWA)."""
    return np.ascontiguousarray(np.asarray(R, dtype=np.uint8)[::-1])


# ---------------------------------------------------------------- text-only checkers

def strand_pattern(W: np.ndarray, strand: int) -> np.ndarray:
    """Strand 0: W itself; strand 1: W reversed with c -> 3 - c for the bases (4 stays 4)."""
    W = np.asarray(W, dtype=np.uint8)
    if strand == 0:
        return np.ascontiguousarray(W)
    r = W[::-1].copy()
    b = r < 4
    r[b] = 3 - r[b]
    return r


def rank_interval(R: np.ndarray, P: np.ndarray, lib_path: str = _LIB) -> tuple:
    """(k, l) of P from one scan of R$ (k = smaller suffixes, l = k + occurrences - 1);
    the canonical miss (1, 0) when P does not occur."""
    lib = load(lib_path)
    R = np.ascontiguousarray(R, dtype=np.uint8)
    P = np.ascontiguousarray(P, dtype=np.uint8)
    k, occ = C.c_int64(), C.c_int64()
    lib.oracle_rank_scan(_ptr(R), R.size, _ptr(P) if P.size else None, P.size, C.byref(k), C.byref(occ))
    return (int(k.value), int(k.value + occ.value - 1)) if occ.value else (1, 0)


def exact_by_rank_scan(R: np.ndarray, codes, offs, strands: int = FWD, lib_path: str = _LIB) -> np.ndarray:
    """Exact intervals like OracleIndex.exact, computed by rank scans of the text."""
    offs = np.asarray(offs, dtype=np.uint64)
    out = []
    for r in range(offs.size - 1):
        W = np.asarray(codes[int(offs[r]):int(offs[r + 1])], dtype=np.uint8)
        for s in (0, 1):
            if strands & (1 << s):
                out.append(rank_interval(R, strand_pattern(W, s), lib_path))
    return np.array(out, dtype=np.uint32).reshape(-1, 2)


def pigeonhole_hits(R: np.ndarray, codes, offs, z, strands: int = BOTH, lib_path: str = _LIB):
    """Substitution hit sets like OracleIndex.inexact (HIT_DTYPE sorted by (read, strand,
    k), plus CSR offsets), computed from the text alone by the pigeonhole principle."""
    lib = load(lib_path)
    R = np.ascontiguousarray(R, dtype=np.uint8)
    offs = np.asarray(offs, dtype=np.uint64)
    nreads = offs.size - 1
    z = np.broadcast_to(np.asarray(z, dtype=np.uint8), (nreads,))
    rows = []
    hit_offs = np.zeros(nreads + 1, dtype=np.uint64)
    for r in range(nreads):
        W = np.asarray(codes[int(offs[r]):int(offs[r + 1])], dtype=np.uint8)
        for s in (0, 1):
            if not strands & (1 << s):
                continue
            P = strand_pattern(W, s)
            cap = 64
            while True:
                buf = np.zeros(3 * cap, dtype=np.uint32)
                nh = int(lib.oracle_hits_pigeonhole(_ptr(R), R.size, _ptr(P) if P.size else None, P.size,
                                                    int(z[r]), _ptr(buf), cap))
                if nh <= cap:
                    break
                cap = nh
            for h in buf[:3 * nh].reshape(-1, 3):
                rows.append((r, int(h[0]), int(h[1]), s, int(h[2]), 0))
        hit_offs[r + 1] = len(rows)
    return np.array(rows, dtype=HIT_DTYPE), hit_offs


# ---------------------------------------------------------------- batched text-only checkers

def _strand_patterns(codes, offs, strands: int):
    """The strand patterns of every read (strand order within a read) as codes + offsets,
    with their read and strand."""
    offs = np.asarray(offs, dtype=np.uint64)
    pats, rid, sid = [], [], []
    for r in range(offs.size - 1):
        W = np.asarray(codes[int(offs[r]):int(offs[r + 1])], dtype=np.uint8)
        for s in (0, 1):
            if strands & (1 << s):
                pats.append(strand_pattern(W, s))
                rid.append(r)
                sid.append(s)
    po = np.zeros(len(pats) + 1, dtype=np.uint64)
    np.cumsum([x.size for x in pats], out=po[1:])
    pc = np.concatenate(pats) if pats and po[-1] else np.zeros(1, np.uint8)
    return pc, po, np.array(rid, dtype=np.int64), np.array(sid, dtype=np.int64)


def exact_by_rank_scan_batch(R: np.ndarray, codes, offs, strands: int = FWD, threads: int = 1,
                             full_rank: bool = False, lib_path: str = _LIB) -> np.ndarray:
    """exact_by_rank_scan for a whole batch: two passes over the text on `threads`
    host threads. With full_rank every pattern gets (k, k + occ - 1) as the definition
    gives it (k = suffixes smaller than the pattern), misses included."""
    lib = load(lib_path)
    R = np.ascontiguousarray(R, dtype=np.uint8)
    pc, po, _, _ = _strand_patterns(codes, offs, strands)
    npat = po.size - 1
    k = np.zeros(npat, np.int64)
    occ = np.zeros(npat, np.int64)
    if lib.oracle_rank_scan_batch(_ptr(R), R.size, _ptr(pc), _ptr(po), npat, threads, _ptr(k), _ptr(occ)):
        raise MemoryError("oracle_rank_scan_batch")
    out = np.zeros((npat, 2), np.uint32)
    if full_rank:
        out[:, 0] = k
        out[:, 1] = (k + occ - 1).astype(np.int64).astype(np.uint32)
        return out
    hit = occ > 0
    out[hit, 0] = k[hit]
    out[hit, 1] = k[hit] + occ[hit] - 1
    out[~hit] = (1, 0)
    return out


def pigeonhole_hits_batch(R: np.ndarray, codes, offs, z, strands: int = BOTH, threads: int = 1,
                          lib_path: str = _LIB):
    """pigeonhole_hits for a whole batch: one pass over the text for the seeds and two for
    the intervals of the distinct windows, on `threads` host threads."""
    lib = load(lib_path)
    R = np.ascontiguousarray(R, dtype=np.uint8)
    nreads = np.asarray(offs).size - 1
    zr = np.broadcast_to(np.asarray(z, dtype=np.uint8), (nreads,))
    pc, po, rid, sid = _strand_patterns(codes, offs, strands)
    npat = po.size - 1
    zq = zr[rid].astype(np.int32) if npat else np.zeros(0, np.int32)
    cap = max(1024, 4 * npat)
    while True:
        buf = np.zeros(3 * cap, np.uint32)
        hoff = np.zeros(npat + 1, np.int64)
        tot = int(lib.oracle_hits_pigeonhole_batch(_ptr(R), R.size, _ptr(pc), _ptr(po), _ptr(zq), npat, threads,
                                                    _ptr(buf), cap, _ptr(hoff)))
        if tot < 0:
            raise MemoryError("oracle_hits_pigeonhole_batch")
        if tot <= cap:
            break
        cap = tot
    trip = buf[:3 * tot].reshape(-1, 3)
    hits = np.zeros(tot, dtype=HIT_DTYPE)
    per = np.diff(hoff)
    hits["read"] = np.repeat(rid, per)
    hits["strand"] = np.repeat(sid, per)
    hits["k"] = trip[:, 0]
    hits["l"] = trip[:, 1]
    hits["d"] = trip[:, 2]
    hit_offs = np.zeros(nreads + 1, dtype=np.uint64)
    np.cumsum(np.bincount(hits["read"].astype(np.int64), minlength=nreads), out=hit_offs[1:])
    return hits, hit_offs
