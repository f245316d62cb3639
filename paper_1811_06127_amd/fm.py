"""ctypes binding of libfmocc (include/fm.h), with torch tensors for device memory and
torch.cuda streams (HIP streams under ROCm).

Argument marshalling only: every step of every search runs in the library's HIP
kernels. There is no fallback: if the library is not built, every call raises.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np
import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libfmocc.so")

FM_OK, FM_EINVAL, FM_EIO, FM_EFORMAT, FM_ENOMEM, FM_EDEVICE, FM_EOVERFLOW, FM_EBUDGET, FM_ERANGE, FM_EAGAIN = range(10)
FM_FWD, FM_REVCOMP, FM_BOTH, FM_DARRAY, FM_PLAIN, FM_STATS, FM_FULL_RANK, FM_GAPS = 1, 2, 3, 4, 16, 32, 64, 128
FM_TUNE_KEEP_LAYOUT = 256
FM_LOAD_REVERSE, FM_LOAD_ALL_LAYOUTS, FM_LOAD_DEVICE_SORT, FM_LOAD_LOCATE = 1, 2, 4, 8
FM_OP_EXACT, FM_OP_DARRAY, FM_OP_INEXACT, FM_OP_LOCATE = 0, 1, 2, 3
FM_ZMAX = 4

# byte offsets inside the inexact workspace (see fm_search_inexact in fm.h)
WS_REQUIRED, WS_STAT_OCC, WS_STAT_BUCKETS, WS_STAT_WALK, WS_STAT_WALK_BK, WS_STAT_STEAL, WS_STAT_TABLE = \
    8, 64, 72, 80, 88, 96, 104


class FmError(RuntimeError):
    def __init__(self, status: int, what: str):
        super().__init__("%s: %s (status %d)" % (what, strerror(status), status))
        self.status = status


class Interval(C.Structure):
    _fields_ = [("k", C.c_uint32), ("l", C.c_uint32)]


class LoadOpts(C.Structure):
    _fields_ = [("device", C.c_int), ("occ_interval", C.c_uint32), ("flags", C.c_uint32),
                ("dev_buf", C.c_void_p), ("dev_buf_bytes", C.c_size_t)]


class Info(C.Structure):
    _fields_ = [("n", C.c_uint64), ("dollar_row", C.c_uint64), ("C", C.c_uint64 * 5),
                ("rev_dollar_row", C.c_uint64), ("rev_C", C.c_uint64 * 5), ("occ_interval", C.c_uint32),
                ("layouts", C.c_uint32), ("has_reverse", C.c_uint32), ("sa_sample", C.c_uint32),
                ("device_bytes", C.c_uint64), ("caller_memory", C.c_uint32), ("table_depth", C.c_uint32)]


class Tuning(C.Structure):
    _fields_ = [("occ_interval", C.c_uint32), ("lanes", C.c_uint32), ("depth", C.c_uint32),
                ("block", C.c_uint32), ("waves_per_cu", C.c_uint32), ("node_budget", C.c_uint32),
                ("order", C.c_uint32), ("table_depth", C.c_uint32)]

    def as_dict(self) -> dict:
        return {f: int(getattr(self, f)) for f, _ in self._fields_}


class ServerOpts(C.Structure):
    _fields_ = [("lanes", C.c_uint32), ("flags", C.c_uint32), ("zmax", C.c_uint32), ("hit_reserve", C.c_uint32),
                ("arena_bytes", C.c_uint64), ("max_batch_reads", C.c_uint64), ("ring_bytes", C.c_uint64)]


class ServerResult(C.Structure):
    _fields_ = [("nreads", C.c_uint64), ("hits", C.c_void_p), ("nhits", C.c_uint64), ("hit_offs", C.c_void_p),
                ("status", C.c_void_p), ("error", C.c_int), ("t_submit", C.c_double), ("t_launch", C.c_double),
                ("t_done", C.c_double), ("batch", C.c_uint64)]


class ServerCounts(C.Structure):
    _fields_ = [("batches", C.c_uint64), ("retries", C.c_uint64), ("requests_done", C.c_uint64),
                ("reads_done", C.c_uint64), ("pending", C.c_uint64), ("error", C.c_int)]


HIT_DTYPE = np.dtype([("read", "<u4"), ("k", "<u4"), ("l", "<u4"), ("strand", "u1"), ("nmm", "u1"),
                      ("pad", "<u2")])

_lib = None


def lib() -> C.CDLL:
    """The loaded library; raises if it has not been built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError("libfmocc.so is not built (run __graft_entry__.build()); "
                           "the FM-index searches have no other implementation")
    L = C.CDLL(LIB_PATH)
    vp, u32, u64, i32 = C.c_void_p, C.c_uint32, C.c_uint64, C.c_int
    sig = {
        "fm_strerror": (C.c_char_p, [i32]),
        "fm_version": (i32, []),
        "fm_bwt_host": (i32, [vp, u64, vp, C.POINTER(C.c_uint64)]),
        "fm_bwt_device": (i32, [vp, u64, vp, C.POINTER(C.c_uint64), C.c_int]),
        "fm_pack_host": (i32, [vp, u64, vp]),
        "fm_index_build_file": (i32, [vp, u64, C.c_char_p, u32]),
        "fm_index_from_text": (i32, [vp, u64, C.POINTER(LoadOpts), C.POINTER(vp)]),
        "fm_index_from_codes": (i32, [vp, u64, vp, C.POINTER(LoadOpts), C.POINTER(vp)]),
        "fm_index_load": (i32, [C.c_char_p, C.POINTER(LoadOpts), C.POINTER(vp)]),
        "fm_index_bytes": (i32, [u64, C.POINTER(LoadOpts), C.POINTER(C.c_size_t)]),
        "fm_index_required_bytes": (i32, [C.c_char_p, C.POINTER(LoadOpts), C.POINTER(C.c_size_t)]),
        "fm_index_info": (i32, [vp, C.POINTER(Info)]),
        "fm_index_free": (None, [vp]),
        "fm_get_tuning": (i32, [vp, i32, C.POINTER(Tuning)]),
        "fm_set_tuning": (i32, [vp, i32, C.POINTER(Tuning)]),
        "fm_autotune": (i32, [vp, i32, vp, vp, vp, u64, u32, u32, vp, u64, vp, vp, vp, C.c_size_t, C.c_char_p,
                              vp, C.POINTER(Tuning), C.POINTER(C.c_float)]),
        "fm_occ8": (i32, [vp, vp, u64, vp, vp]),
        "fm_probe_random_reads": (i32, [vp, vp, u64, u32, vp, C.POINTER(C.c_uint64), vp]),
        "fm_search_exact_workspace": (i32, [vp, u64, u32, C.POINTER(C.c_size_t)]),
        "fm_search_exact": (i32, [vp, vp, vp, u64, u32, vp, vp, C.c_size_t, vp]),
        "fm_darray": (i32, [vp, vp, vp, u64, u64, u32, vp, vp]),
        "fm_search_inexact_workspace": (i32, [vp, u64, u64, u32, u32, u64, C.POINTER(C.c_size_t)]),
        "fm_search_inexact": (i32, [vp, vp, vp, vp, u64, u32, u32, vp, u64, vp, vp, vp, C.c_size_t, vp]),
        "fm_plan_create": (i32, [vp, i32, vp, vp, vp, u64, u32, u32, vp, u64, vp, vp, vp, C.c_size_t,
                                 C.POINTER(vp)]),
        "fm_plan_launch": (i32, [vp, vp]),
        "fm_plan_phase_times": (i32, [vp, C.POINTER(C.c_float)]),
        "fm_phase_timing": (i32, [vp, u32]),
        "fm_phase_times": (i32, [vp, C.POINTER(C.c_float), C.POINTER(C.c_uint32)]),
        "fm_plan_free": (None, [vp]),
        "fm_search_inexact_noalloc": (i32, [vp, vp, vp, vp, u64, u32, u32, vp, u64, vp, vp, vp, vp]),
        "fm_search_both": (i32, [vp, vp, vp, vp, u64, u32, u32, u32, vp, vp, u64, vp, vp, vp, C.c_size_t, vp]),
        "fm_locate_workspace": (i32, [vp, u64, C.POINTER(C.c_size_t)]),
        "fm_locate": (i32, [vp, vp, u64, u32, vp, vp, u64, u32, vp, C.c_size_t, vp]),
        "fm_plan_create_both": (i32, [vp, vp, vp, vp, u64, u32, u32, u32, vp, vp, u64, vp, vp, vp, C.c_size_t,
                                      C.POINTER(vp)]),
        "fm_server_bytes": (i32, [C.POINTER(ServerOpts), u64, u64, C.POINTER(C.c_uint64)]),
        "fm_server_create": (i32, [vp, C.POINTER(ServerOpts), C.POINTER(vp)]),
        "fm_server_submit": (i32, [vp, vp, vp, vp, u64, C.POINTER(C.c_uint64)]),
        "fm_server_wait": (i32, [vp, u64, C.c_double, C.POINTER(ServerResult)]),
        "fm_server_release": (i32, [vp, u64]),
        "fm_server_clock": (C.c_double, [vp]),
        "fm_server_stats": (i32, [vp, C.POINTER(ServerCounts)]),
        "fm_server_free": (None, [vp]),
    }
    for name, (res, args) in sig.items():
        f = getattr(L, name)
        f.restype = res
        f.argtypes = args
    _lib = L
    return L


def strerror(status: int) -> str:
    return lib().fm_strerror(status).decode()


def _check(status: int, what: str):
    if status != FM_OK:
        raise FmError(status, what)


def _ptr(t) -> int | None:
    if t is None:
        return None
    if isinstance(t, torch.Tensor):
        return t.data_ptr() if t.numel() else None
    if isinstance(t, np.ndarray):
        return t.ctypes.data if t.size else None
    raise TypeError(type(t))


def _stream(stream) -> int | None:
    if stream is None:
        return torch.cuda.current_stream().cuda_stream
    return stream.cuda_stream if hasattr(stream, "cuda_stream") else stream


def _dev(t: torch.Tensor, dtype, what: str):
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise TypeError("%s must be a device tensor" % what)
    if t.dtype != dtype or not t.is_contiguous():
        raise TypeError("%s must be a contiguous %s tensor" % (what, dtype))


def nstrands(flags: int) -> int:
    return (1 if flags & FM_FWD else 0) + (1 if flags & FM_REVCOMP else 0)


# ---------------------------------------------------------------- host helpers

def fm_bwt_host(text: np.ndarray):
    text = np.ascontiguousarray(text, dtype=np.uint8)
    bwt = np.zeros(text.size + 1, np.uint8)
    dr = C.c_uint64(0)
    _check(lib().fm_bwt_host(_ptr(text), text.size, _ptr(bwt), C.byref(dr)), "fm_bwt_host")
    return bwt, int(dr.value)


def fm_bwt_device(text: np.ndarray, device: int = 0):
    """fm_bwt_host's result, computed by the device suffix sort."""
    text = np.ascontiguousarray(text, dtype=np.uint8)
    bwt = np.zeros(text.size + 1, np.uint8)
    dr = C.c_uint64(0)
    _check(lib().fm_bwt_device(_ptr(text), text.size, _ptr(bwt), C.byref(dr), device), "fm_bwt_device")
    return bwt, int(dr.value)


def fm_pack_host(codes: np.ndarray) -> np.ndarray:
    codes = np.ascontiguousarray(codes, dtype=np.uint8)
    words = np.zeros((codes.size + 15) // 16, np.uint32)
    _check(lib().fm_pack_host(_ptr(codes), codes.size, _ptr(words)), "fm_pack_host")
    return words


def fm_index_build_file(text: np.ndarray, path: str, flags: int = 0):
    text = np.ascontiguousarray(text, dtype=np.uint8)
    _check(lib().fm_index_build_file(_ptr(text), text.size, path.encode(), flags), "fm_index_build_file")


# ---------------------------------------------------------------- index

def fm_index_bytes(n: int, occ_interval: int = 128, flags: int = 0) -> int:
    """Device bytes an index over n symbols keeps when built with these options."""
    b = C.c_size_t(0)
    o = LoadOpts(0, occ_interval, flags, None, 0)
    _check(lib().fm_index_bytes(n, C.byref(o), C.byref(b)), "fm_index_bytes")
    return int(b.value)


def fm_index_required_bytes(path: str, occ_interval: int = 128, flags: int = 0) -> int:
    """Device bytes Index.load(path, ...) keeps, from the file's header alone."""
    b = C.c_size_t(0)
    o = LoadOpts(0, occ_interval, flags, None, 0)
    _check(lib().fm_index_required_bytes(path.encode(), C.byref(o), C.byref(b)), "fm_index_required_bytes")
    return int(b.value)


class Index:
    """An FM-index resident in device memory (owner of an fm_index handle). With dev_buf
    (a contiguous uint8 device tensor of at least fm_index_bytes / fm_index_required_bytes bytes) the
    index keeps its layouts in that tensor, which this object holds on to until free()."""

    def __init__(self, handle: int, dev_buf: torch.Tensor | None = None):
        self._h = C.c_void_p(handle)
        self._buf = dev_buf

    @staticmethod
    def _opts(device, occ_interval, flags, dev_buf=None):
        if dev_buf is None:
            return LoadOpts(device, occ_interval, flags, None, 0)
        _dev(dev_buf, torch.uint8, "dev_buf")
        return LoadOpts(device, occ_interval, flags, _ptr(dev_buf), dev_buf.numel())

    @classmethod
    def from_text(cls, text: np.ndarray, device: int = 0, occ_interval: int = 128, flags: int = 0,
                  dev_buf: torch.Tensor | None = None) -> "Index":
        text = np.ascontiguousarray(text, dtype=np.uint8)
        h = C.c_void_p()
        o = cls._opts(device, occ_interval, flags, dev_buf)
        _check(lib().fm_index_from_text(_ptr(text), text.size, C.byref(o), C.byref(h)), "fm_index_from_text")
        return cls(h.value, dev_buf)

    @classmethod
    def from_codes(cls, bwt: np.ndarray, rev_bwt: np.ndarray | None = None, device: int = 0,
                   occ_interval: int = 128, flags: int = 0, dev_buf: torch.Tensor | None = None) -> "Index":
        bwt = np.ascontiguousarray(bwt, dtype=np.uint8)
        rb = None if rev_bwt is None else np.ascontiguousarray(rev_bwt, dtype=np.uint8)
        h = C.c_void_p()
        o = cls._opts(device, occ_interval, flags, dev_buf)
        _check(lib().fm_index_from_codes(_ptr(bwt), bwt.size, _ptr(rb), C.byref(o), C.byref(h)),
               "fm_index_from_codes")
        return cls(h.value, dev_buf)

    @classmethod
    def load(cls, path: str, device: int = 0, occ_interval: int = 128, flags: int = 0,
             dev_buf: torch.Tensor | None = None) -> "Index":
        h = C.c_void_p()
        o = cls._opts(device, occ_interval, flags, dev_buf)
        _check(lib().fm_index_load(path.encode(), C.byref(o), C.byref(h)), "fm_index_load")
        return cls(h.value, dev_buf)

    @property
    def handle(self) -> C.c_void_p:
        if not self._h:
            raise RuntimeError("index was freed")
        return self._h

    def info(self) -> dict:
        i = Info()
        _check(lib().fm_index_info(self.handle, C.byref(i)), "fm_index_info")
        return {"n": i.n, "dollar_row": i.dollar_row, "C": list(i.C), "rev_dollar_row": i.rev_dollar_row,
                "rev_C": list(i.rev_C), "occ_interval": i.occ_interval, "layouts": i.layouts,
                "has_reverse": bool(i.has_reverse), "sa_sample": i.sa_sample, "device_bytes": i.device_bytes,
                "caller_memory": bool(i.caller_memory), "table_depth": i.table_depth}

    def get_tuning(self, op: int) -> dict:
        t = Tuning()
        _check(lib().fm_get_tuning(self.handle, op, C.byref(t)), "fm_get_tuning")
        return t.as_dict()

    def set_tuning(self, op: int, **kw):
        cur = self.get_tuning(op)
        cur.update(kw)
        t = Tuning(**cur)
        _check(lib().fm_set_tuning(self.handle, op, C.byref(t)), "fm_set_tuning")

    def phase_timing(self, capacity: int):
        _check(lib().fm_phase_timing(self.handle, capacity), "fm_phase_timing")

    def phase_times(self) -> tuple:
        ms = (C.c_float * 4)()
        calls = C.c_uint32(0)
        _check(lib().fm_phase_times(self.handle, ms, C.byref(calls)), "fm_phase_times")
        return {"exact_walk": ms[0], "d_walk": ms[1], "dfs": ms[2], "compaction": ms[3]}, int(calls.value)

    def free(self):
        if self._h:
            lib().fm_index_free(self._h)
            self._h = C.c_void_p()
        self._buf = None

    def __del__(self):
        try:
            self.free()
        except Exception:
            pass


# ---------------------------------------------------------------- searches

def fm_occ8(idx: Index, q: torch.Tensor, out: torch.Tensor | None = None, stream=None) -> torch.Tensor:
    """q: (nq, 2) int32 device tensor of (k, l); returns (nq, 8) int32 (bit pattern of uint32)."""
    _dev(q, torch.int32, "q")
    nq = q.numel() // 2
    if out is None:
        out = torch.empty((nq, 8), dtype=torch.int32, device=q.device)
    _dev(out, torch.int32, "out")
    _check(lib().fm_occ8(idx.handle, _ptr(q), nq, _ptr(out), _stream(stream)), "fm_occ8")
    return out


def probe_random_reads(idx: Index, buf: torch.Tensor, span: int, rounds: int, sink: torch.Tensor,
                       stream=None) -> int:
    """One launch of random 32-byte reads over buf[:span] (device tensor of at least span
    bytes) on idx's device; sink: one-word int32 device tensor. Returns the reads made."""
    if not buf.is_cuda or buf.numel() * buf.element_size() < span:
        raise ValueError("buf must be a device tensor of at least span bytes")
    _dev(sink, torch.int32, "sink")
    n = C.c_uint64(0)
    _check(lib().fm_probe_random_reads(idx.handle, _ptr(buf), span, rounds, _ptr(sink), C.byref(n),
                                       _stream(stream)), "fm_probe_random_reads")
    return int(n.value)


def fm_search_exact_workspace(idx: Index, nreads: int, flags: int) -> int:
    b = C.c_size_t(0)
    _check(lib().fm_search_exact_workspace(idx.handle, nreads, flags, C.byref(b)), "fm_search_exact_workspace")
    return int(b.value)


def exact_stats(ws: torch.Tensor) -> dict:
    v = ws[WS_STAT_WALK:WS_STAT_WALK + 16].cpu().numpy().view(np.uint64)
    return {"steps": int(v[0]), "buckets": int(v[1])}


def fm_search_exact(idx: Index, codes: torch.Tensor, offs: torch.Tensor, flags: int = FM_FWD,
                    out: torch.Tensor | None = None, ws: torch.Tensor | None = None, stream=None) -> torch.Tensor:
    """codes: uint8 device tensor; offs: int64 device tensor (nreads+1). Returns
    (nreads * strands, 2) int32 intervals (k, l), strand-major within a read."""
    _dev(codes, torch.uint8, "codes")
    _dev(offs, torch.int64, "offs")
    nreads = offs.numel() - 1
    if out is None:
        out = torch.empty((nreads * nstrands(flags), 2), dtype=torch.int32, device=codes.device)
    if ws is None and not (flags & FM_PLAIN and not flags & FM_STATS):
        ws = torch.empty(fm_search_exact_workspace(idx, nreads, flags), dtype=torch.uint8, device=codes.device)
    wsb = ws.numel() if ws is not None else 0
    _check(lib().fm_search_exact(idx.handle, _ptr(codes), _ptr(offs), nreads, flags, _ptr(out), _ptr(ws), wsb,
                                 _stream(stream)), "fm_search_exact")
    return out


def fm_darray(idx: Index, codes: torch.Tensor, offs: torch.Tensor, total_len: int, flags: int = FM_FWD,
              out: torch.Tensor | None = None, stream=None) -> torch.Tensor:
    """D for each requested strand: (strands, total_len) uint8."""
    _dev(codes, torch.uint8, "codes")
    _dev(offs, torch.int64, "offs")
    nreads = offs.numel() - 1
    if out is None:
        out = torch.zeros((nstrands(flags), total_len), dtype=torch.uint8, device=codes.device)
    _check(lib().fm_darray(idx.handle, _ptr(codes), _ptr(offs), nreads, total_len, flags, _ptr(out),
                           _stream(stream)), "fm_darray")
    return out


def fm_search_inexact_workspace(idx: Index, nreads: int, total_len: int, flags: int, zmax: int, hit_cap: int) -> int:
    b = C.c_size_t(0)
    _check(lib().fm_search_inexact_workspace(idx.handle, nreads, total_len, flags, zmax, hit_cap, C.byref(b)),
           "fm_search_inexact_workspace")
    return int(b.value)


class InexactBuffers:
    """Device buffers of one inexact call shape."""

    def __init__(self, idx: Index, nreads: int, total_len: int, flags: int, zmax: int, hit_cap: int, device):
        self.hits = torch.empty((max(hit_cap, 1), 4), dtype=torch.int32, device=device)
        self.hit_offs = torch.empty(nreads + 1, dtype=torch.int64, device=device)
        self.status = torch.empty(max(nreads, 1), dtype=torch.int32, device=device)
        n = fm_search_inexact_workspace(idx, nreads, total_len, flags, zmax, hit_cap)
        self.ws = torch.empty(n, dtype=torch.uint8, device=device)
        self.hit_cap = hit_cap

    def required(self) -> int:
        return int(self.ws[WS_REQUIRED:WS_REQUIRED + 8].cpu().numpy().view(np.uint64)[0])

    def stats(self) -> dict:
        v = self.ws[WS_STAT_OCC:WS_STAT_OCC + 48].cpu().numpy().view(np.uint64)
        return {"occ8": int(v[0]), "buckets": int(v[1]), "walk_steps": int(v[2]), "walk_buckets": int(v[3]),
                "subtrees": int(v[4]), "table": int(v[5])}


def fm_search_inexact(idx: Index, codes: torch.Tensor, offs: torch.Tensor, z: torch.Tensor, flags: int,
                      zmax: int, hit_cap: int, bufs: InexactBuffers | None = None, stream=None) -> InexactBuffers:
    _dev(codes, torch.uint8, "codes")
    _dev(offs, torch.int64, "offs")
    _dev(z, torch.uint8, "z")
    nreads = offs.numel() - 1
    if bufs is None:
        total_len = codes.numel()
        bufs = InexactBuffers(idx, nreads, total_len, flags, zmax, hit_cap, codes.device)
    _check(lib().fm_search_inexact(idx.handle, _ptr(codes), _ptr(offs), _ptr(z), nreads, flags, zmax,
                                   _ptr(bufs.hits), bufs.hit_cap, _ptr(bufs.hit_offs), _ptr(bufs.status),
                                   _ptr(bufs.ws), bufs.ws.numel(), _stream(stream)), "fm_search_inexact")
    return bufs


FM_NOALLOC_WS_BYTES = 64 << 20


def fm_search_inexact_noalloc(idx: Index, codes: torch.Tensor, offs: torch.Tensor, z: torch.Tensor, flags: int,
                              zmax: int, hits: torch.Tensor, hit_offs: torch.Tensor, status: torch.Tensor,
                              required: torch.Tensor | None = None, stream=None):
    """fm_search_inexact_noalloc: the inexact search with the library's static per-device
    workspace. The caller passes the outputs: hits (hit_cap, 4) int32, hit_offs (nreads+1)
    int64, status (>= nreads) int32, and optionally required (1) int64."""
    _dev(codes, torch.uint8, "codes")
    _dev(offs, torch.int64, "offs")
    _dev(z, torch.uint8, "z")
    _dev(hits, torch.int32, "hits")
    _dev(hit_offs, torch.int64, "hit_offs")
    _dev(status, torch.int32, "status")
    if required is not None:
        _dev(required, torch.int64, "required")
    nreads = offs.numel() - 1
    _check(lib().fm_search_inexact_noalloc(idx.handle, _ptr(codes), _ptr(offs), _ptr(z), nreads, flags, zmax,
                                           _ptr(hits), hits.shape[0], _ptr(hit_offs), _ptr(status), _ptr(required),
                                           _stream(stream)), "fm_search_inexact_noalloc")


def fm_search_both(idx: Index, codes: torch.Tensor, offs: torch.Tensor, z: torch.Tensor, exact_flags: int,
                   flags: int, zmax: int, hit_cap: int, out: torch.Tensor | None = None,
                   bufs: InexactBuffers | None = None, stream=None):
    """Exact and inexact search of one batch (fm_search_both; the exact intervals are taken
    from the inexact search's DFS). Returns (intervals, bufs) as fm_search_exact and
    fm_search_inexact would."""
    _dev(codes, torch.uint8, "codes")
    _dev(offs, torch.int64, "offs")
    _dev(z, torch.uint8, "z")
    nreads = offs.numel() - 1
    if out is None:
        out = torch.empty((nreads * nstrands(exact_flags), 2), dtype=torch.int32, device=codes.device)
    if bufs is None:
        total_len = int(offs[-1].item()) if nreads else 0
        bufs = InexactBuffers(idx, nreads, total_len, flags, zmax, hit_cap, codes.device)
    _check(lib().fm_search_both(idx.handle, _ptr(codes), _ptr(offs), _ptr(z), nreads, exact_flags, flags, zmax,
                                _ptr(out), _ptr(bufs.hits), bufs.hit_cap, _ptr(bufs.hit_offs), _ptr(bufs.status),
                                _ptr(bufs.ws), bufs.ws.numel(), _stream(stream)), "fm_search_both")
    return out, bufs


def fm_locate(idx: Index, kl: torch.Tensor, cap: int | None = None, stats: bool = False, stream=None):
    """Text positions of the rows of SA intervals (fm_locate). kl: device int32 tensor of
    (k, l) pairs, shape (niv, 2), or of fm_hit records, shape (nhits, 4) (k, l are then
    columns 1 and 2). Returns (offs, pos[, steps]): offs (niv+1 int64) and pos (int32,
    the located rows in interval order). With cap None, the total is read back first and
    every row is located."""
    if kl.dtype not in (torch.int32, torch.uint32) or kl.device.type != "cuda" or kl.dim() != 2 or \
            kl.shape[1] not in (2, 4) or not kl.is_contiguous():
        raise ValueError("kl: contiguous device int32 tensor of shape (n, 2) or (n, 4)")
    niv = kl.shape[0]
    stride = kl.shape[1]
    base = _ptr(kl) + (4 if stride == 4 else 0)
    nb = C.c_size_t(0)
    _check(lib().fm_locate_workspace(idx.handle, niv, C.byref(nb)), "fm_locate_workspace")
    ws = torch.empty(max(nb.value, 1), dtype=torch.uint8, device=kl.device)
    offs = torch.empty(niv + 1, dtype=torch.int64, device=kl.device)
    flags = FM_STATS if stats else 0
    if cap is None:
        _check(lib().fm_locate(idx.handle, base, niv, stride, _ptr(offs), None, 0, 0, _ptr(ws), ws.numel(),
                               _stream(stream)), "fm_locate")
        cap = int(offs[-1].item())
    pos = torch.empty(max(cap, 1), dtype=torch.int32, device=kl.device)
    _check(lib().fm_locate(idx.handle, base, niv, stride, _ptr(offs), _ptr(pos), cap, flags, _ptr(ws), ws.numel(),
                           _stream(stream)), "fm_locate")
    if stats:
        torch.cuda.synchronize(kl.device)
        steps = int(ws[80:88].cpu().numpy().view(np.uint64)[0])
        return offs, pos[:cap], steps
    return offs, pos[:cap]


def hits_to_numpy(bufs: InexactBuffers, nreads: int):
    """(hits as HIT_DTYPE array, hit_offs uint64, status uint32) copied to the host."""
    offs = bufs.hit_offs[:nreads + 1].cpu().numpy().view(np.uint64).copy()
    total = int(offs[-1]) if nreads >= 0 else 0
    raw = bufs.hits[:total].cpu().numpy()
    hits = raw.view(np.uint32).reshape(-1, 4).copy().view(HIT_DTYPE).reshape(-1)
    status = bufs.status[:nreads].cpu().numpy().view(np.uint32).copy()
    return hits, offs, status


def fm_autotune(idx: Index, op: int, codes, offs, z, flags: int, zmax: int = 0, out=None,
                bufs: InexactBuffers | None = None, ws=None, cache_path: str | None = None, stream=None):
    nreads = offs.numel() - 1
    best = Tuning()
    ms = C.c_float(0)
    if op == FM_OP_EXACT:
        if out is None:
            out = torch.empty((nreads * nstrands(flags), 2), dtype=torch.int32, device=codes.device)
        if ws is None:
            ws = torch.empty(max(fm_search_exact_workspace(idx, nreads, flags), 1), dtype=torch.uint8,
                             device=codes.device)
        st = lib().fm_autotune(idx.handle, op, _ptr(codes), _ptr(offs), None, nreads, flags, 0, _ptr(out), 0,
                               None, None, _ptr(ws), ws.numel(), cache_path.encode() if cache_path else None,
                               _stream(stream), C.byref(best), C.byref(ms))
    else:
        st = lib().fm_autotune(idx.handle, op, _ptr(codes), _ptr(offs), _ptr(z), nreads, flags, zmax,
                               _ptr(bufs.hits), bufs.hit_cap, _ptr(bufs.hit_offs), _ptr(bufs.status), _ptr(bufs.ws),
                               bufs.ws.numel(), cache_path.encode() if cache_path else None, _stream(stream),
                               C.byref(best), C.byref(ms))
    _check(st, "fm_autotune")
    return best.as_dict(), float(ms.value)


class Plan:
    """A captured launch graph for one batch shape (fm_plan_*)."""

    def __init__(self, idx: Index, op: int, codes, offs, z, flags: int, zmax: int = 0, out=None,
                 bufs: InexactBuffers | None = None, ws=None):
        nreads = offs.numel() - 1
        h = C.c_void_p()
        self._keep = (idx, codes, offs, z, out, bufs, ws)
        if op == FM_OP_EXACT:
            st = lib().fm_plan_create(idx.handle, op, _ptr(codes), _ptr(offs), None, nreads, flags, 0, _ptr(out), 0,
                                      None, None, _ptr(ws), ws.numel() if ws is not None else 0, C.byref(h))
        else:
            st = lib().fm_plan_create(idx.handle, op, _ptr(codes), _ptr(offs), _ptr(z), nreads, flags, zmax,
                                      _ptr(bufs.hits), bufs.hit_cap, _ptr(bufs.hit_offs), _ptr(bufs.status),
                                      _ptr(bufs.ws), bufs.ws.numel(), C.byref(h))
        _check(st, "fm_plan_create")
        self._h = h

    @classmethod
    def both(cls, idx: Index, codes, offs, z, exact_flags: int, flags: int, zmax: int, out, bufs: InexactBuffers):
        """A plan of one fm_search_both call."""
        self = cls.__new__(cls)
        nreads = offs.numel() - 1
        h = C.c_void_p()
        self._keep = (idx, codes, offs, z, out, bufs)
        _check(lib().fm_plan_create_both(idx.handle, _ptr(codes), _ptr(offs), _ptr(z), nreads, exact_flags, flags, zmax,
                                         _ptr(out), _ptr(bufs.hits), bufs.hit_cap, _ptr(bufs.hit_offs),
                                         _ptr(bufs.status), _ptr(bufs.ws), bufs.ws.numel(), C.byref(h)),
               "fm_plan_create_both")
        self._h = h
        return self

    def launch(self, stream=None):
        _check(lib().fm_plan_launch(self._h, _stream(stream)), "fm_plan_launch")

    def phase_times(self) -> dict:
        """Milliseconds per phase of the last replay (fm_plan_phase_times); the plan must have
        been created while the index's phase timing was on."""
        ms = (C.c_float * 4)()
        _check(lib().fm_plan_phase_times(self._h, ms), "fm_plan_phase_times")
        return {"exact_walk": ms[0], "d_walk": ms[1], "dfs": ms[2], "compaction": ms[3]}

    def free(self):
        if self._h:
            lib().fm_plan_free(self._h)
            self._h = C.c_void_p()

    def __del__(self):
        try:
            self.free()
        except Exception:
            pass


def reads_to_device(codes: np.ndarray, offs: np.ndarray, z: np.ndarray | None = None, device="cuda"):
    c = torch.from_numpy(np.ascontiguousarray(codes, dtype=np.uint8)).to(device)
    o = torch.from_numpy(np.ascontiguousarray(offs, dtype=np.uint64).view(np.int64)).to(device)
    zz = None if z is None else torch.from_numpy(np.ascontiguousarray(z, dtype=np.uint8)).to(device)
    return c, o, zz


# ---------------------------------------------------------------- serving

def server_opts(lanes: int = 2, flags: int = FM_BOTH | FM_DARRAY, zmax: int = 2, hit_reserve: int = 4,
                arena_bytes: int = 1 << 30, max_batch_reads: int = 0, ring_bytes: int = 0) -> ServerOpts:
    return ServerOpts(lanes, flags, zmax, hit_reserve, arena_bytes, max_batch_reads, ring_bytes)


def fm_server_bytes(opts: ServerOpts, nreads: int, total_len: int) -> int:
    """Device bytes a batch of this shape takes under opts (the admission rule)."""
    out = C.c_uint64()
    _check(lib().fm_server_bytes(C.byref(opts), nreads, total_len, C.byref(out)), "fm_server_bytes")
    return int(out.value)


class Served:
    """One finished request: hits (HIT_DTYPE, read numbers local to the request),
    hit_offs, status and the server-clock times."""

    def __init__(self, r: ServerResult):
        n = int(r.nreads)
        self.error = int(r.error)
        self.hits = np.empty(int(r.nhits), dtype=HIT_DTYPE)
        if r.nhits:
            C.memmove(self.hits.ctypes.data, r.hits, 16 * int(r.nhits))
        self.hit_offs = np.zeros(n + 1, dtype=np.uint64)
        if r.hit_offs:
            C.memmove(self.hit_offs.ctypes.data, r.hit_offs, 8 * (n + 1))
        self.status = np.zeros(n, dtype=np.uint32)
        if n and r.status:
            C.memmove(self.status.ctypes.data, r.status, 4 * n)
        self.t_submit, self.t_launch, self.t_done = float(r.t_submit), float(r.t_launch), float(r.t_done)
        self.batch = int(r.batch)

    @property
    def latency(self) -> float:
        return self.t_done - self.t_submit


class Server:
    """fm_server_*: continuous batching of inexact-search requests on one index."""

    def __init__(self, index: "Index", **kw):
        self.index = index                    # kept alive while the server runs
        self.opts = server_opts(**kw)
        h = C.c_void_p()
        _check(lib().fm_server_create(index.handle, C.byref(self.opts), C.byref(h)), "fm_server_create")
        self.handle = h

    def submit(self, codes: np.ndarray, offs: np.ndarray, z: np.ndarray) -> int:
        codes = np.ascontiguousarray(codes, dtype=np.uint8)
        offs = np.ascontiguousarray(offs, dtype=np.uint64)
        z = np.ascontiguousarray(z, dtype=np.uint8)
        t = C.c_uint64()
        _check(lib().fm_server_submit(self.handle, _ptr(codes), _ptr(offs), _ptr(z), offs.size - 1, C.byref(t)),
               "fm_server_submit")
        return int(t.value)

    def wait(self, ticket: int, timeout: float | None = None) -> Served | None:
        """The finished request, or None if it is still running after `timeout` s."""
        r = ServerResult()
        st = lib().fm_server_wait(self.handle, ticket, -1.0 if timeout is None else float(timeout), C.byref(r))
        if st == FM_EAGAIN:
            return None
        _check(st, "fm_server_wait")
        return Served(r)

    def release(self, ticket: int):
        _check(lib().fm_server_release(self.handle, ticket), "fm_server_release")

    def clock(self) -> float:
        return float(lib().fm_server_clock(self.handle))

    def stats(self) -> dict:
        c = ServerCounts()
        _check(lib().fm_server_stats(self.handle, C.byref(c)), "fm_server_stats")
        return {f: int(getattr(c, f)) for f, _ in c._fields_}

    def close(self):
        if self.handle:
            lib().fm_server_free(self.handle)
            self.handle = None

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
