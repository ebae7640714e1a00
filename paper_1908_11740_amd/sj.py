"""Thin ctypes binding to libsj.so (include/sj.h).

Argument marshalling only: every step of the join runs in the HIP library.
Tensors are used for device memory and streams; the library sees raw device
pointers and the current HIP stream.  If libsj.so is missing the first call
raises; there is no fallback.
"""
import ctypes
import os

import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libsj.so")

SJ_OK = 0
SJ_ERR_ARG = -1
SJ_ERR_RECT = -2
SJ_ERR_CAPACITY = -3
SJ_ERR_GRID_MISMATCH = -4
SJ_ERR_OOM = -5
SJ_ERR_DEVICE = -6
SJ_ERR_TOO_LARGE = -7

SJ_K_MAX = 8192
SJ_PLAIN = 0x1
SJ_RULE_ONLY = 0x2
SJ_TWO_PASS = 0x4
INT32_MAX = 2**31 - 1


class SjError(RuntimeError):
    def __init__(self, status, where):
        self.status = status
        detail = lib().sj_last_error().decode()
        super().__init__(f"{where}: {status_string(status)} ({status}) {detail}")


class Grid(ctypes.Structure):
    _fields_ = [("k", ctypes.c_int32), ("split_tau", ctypes.c_int32),
                ("domain", ctypes.c_float * 4), ("flags", ctypes.c_uint32)]


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is not built; run paper_1908_11740_amd.build")
        L = ctypes.CDLL(LIB_PATH)
        vp, i64, i64p = ctypes.c_void_p, ctypes.c_int64, ctypes.POINTER(ctypes.c_int64)
        L.sj_partition.argtypes = [vp, i64, ctypes.POINTER(Grid), ctypes.POINTER(vp), vp]
        L.sj_join.argtypes = [vp, vp, vp, i64, i64p, vp]
        L.sj_join_count.argtypes = [vp, vp, i64p, vp]
        L.sj_part_info.argtypes = [vp, i64p, i64p, ctypes.POINTER(Grid)]
        L.sj_part_download.argtypes = [vp, i64p, ctypes.POINTER(ctypes.c_int32), vp]
        L.sj_part_free.argtypes = [vp]
        L.sj_part_free.restype = None
        L.sj_status_string.argtypes = [ctypes.c_int]
        L.sj_status_string.restype = ctypes.c_char_p
        L.sj_version.restype = ctypes.c_char_p
        L.sj_last_error.restype = ctypes.c_char_p
        L.sj_prof_enable.argtypes = [ctypes.c_int]
        L.sj_prof_enable.restype = None
        L.sj_prof_collect.restype = ctypes.c_int
        L.sj_prof_name.argtypes = [ctypes.c_int]
        L.sj_prof_name.restype = ctypes.c_char_p
        L.sj_prof_total_ms.argtypes = [ctypes.c_int]
        L.sj_prof_total_ms.restype = ctypes.c_double
        L.sj_prof_calls.argtypes = [ctypes.c_int]
        L.sj_prof_calls.restype = ctypes.c_int64
        for f in ("sj_partition", "sj_join", "sj_join_count", "sj_part_info", "sj_part_download"):
            getattr(L, f).restype = ctypes.c_int
        _lib = L
    return _lib


def status_string(s):
    return lib().sj_status_string(int(s)).decode()


def _check(s, where):
    if s != SJ_OK:
        raise SjError(s, where)


def _stream(stream):
    if stream is None:
        stream = torch.cuda.current_stream()
    return ctypes.c_void_p(stream.cuda_stream)


def make_grid(k, split_tau=0, domain=None, flags=0):
    g = Grid()
    g.k = int(k)
    g.split_tau = int(split_tau)
    dom = (0.0, 0.0, 0.0, 0.0) if domain is None else domain
    for i in range(4):
        g.domain[i] = float(dom[i])
    g.flags = int(flags)
    return g


def _rects(t):
    if not (isinstance(t, torch.Tensor) and t.is_cuda and t.dtype == torch.float32 and t.dim() == 2
            and t.shape[1] == 4 and t.is_contiguous()):
        raise ValueError("rectangles must be a contiguous (n, 4) float32 CUDA tensor")
    return t


class Part:
    """A partitioned input (owns an sj_part handle)."""

    def __init__(self, handle, src):
        self._h = handle
        self._src_len = src

    @property
    def handle(self):
        return self._h

    def info(self):
        n, m, g = ctypes.c_int64(), ctypes.c_int64(), Grid()
        _check(lib().sj_part_info(self._h, ctypes.byref(n), ctypes.byref(m), ctypes.byref(g)),
               "sj_part_info")
        return n.value, m.value, g

    def download(self, stream=None):
        n, m, g = self.info()
        C = g.k * g.k
        off = (ctypes.c_int64 * (C + 1))()
        ids = (ctypes.c_int32 * max(m, 1))()
        _check(lib().sj_part_download(self._h, off, ids, _stream(stream)), "sj_part_download")
        import numpy as np
        return (np.ctypeslib.as_array(off).copy(), np.ctypeslib.as_array(ids)[:m].copy())

    def free(self):
        if self._h:
            lib().sj_part_free(self._h)
            self._h = None

    def __del__(self):
        try:
            self.free()
        except Exception:
            pass


def partition(rects, k, split_tau=0, domain=None, flags=0, reuse=None, stream=None):
    """Partitioning phase: sj_partition on an (n, 4) float32 device tensor."""
    rects = _rects(rects)
    g = make_grid(k, split_tau, domain, flags)
    h = ctypes.c_void_p(reuse.handle if reuse is not None else None)
    s = lib().sj_partition(ctypes.c_void_p(rects.data_ptr()), rects.shape[0], ctypes.byref(g),
                           ctypes.byref(h), _stream(stream))
    _check(s, "sj_partition")
    if reuse is not None:
        return reuse
    return Part(h.value, rects.shape[0])


def join_count(R, S, stream=None):
    n = ctypes.c_int64()
    _check(lib().sj_join_count(R.handle, S.handle, ctypes.byref(n), _stream(stream)),
           "sj_join_count")
    return n.value


def join_into(R, S, out, stream=None):
    """Join into a preallocated (cap, 2) int32 device tensor; returns (status, n_pairs)."""
    n = ctypes.c_int64()
    cap = out.shape[0]
    s = lib().sj_join(R.handle, S.handle, ctypes.c_void_p(out.data_ptr() if cap else None), cap,
                      ctypes.byref(n), _stream(stream))
    if s not in (SJ_OK, SJ_ERR_CAPACITY):
        raise SjError(s, "sj_join")
    return s, n.value


def join(R, S, capacity=None, stream=None):
    """Joining phase: all intersecting (r, s) pairs as an (P, 2) int32 device tensor
    (unspecified order)."""
    dev = torch.device("cuda", torch.cuda.current_device())
    if capacity is None:
        capacity = 1 << 16
    out = torch.empty((capacity, 2), dtype=torch.int32, device=dev)
    s, n = join_into(R, S, out, stream)
    if s == SJ_ERR_CAPACITY:
        out = torch.empty((n, 2), dtype=torch.int32, device=dev)
        s, n = join_into(R, S, out, stream)
        _check(s, "sj_join")
    return out[:n]


def version():
    return lib().sj_version().decode()


def prof_enable(on=True):
    """Per-kernel HIP-event timer of the library (see sj_prof_enable)."""
    lib().sj_prof_enable(1 if on else 0)


def prof_collect():
    """{kernel name: (total ms, calls)} since prof_enable(True)."""
    L = lib()
    n = L.sj_prof_collect()
    return {L.sj_prof_name(i).decode(): (L.sj_prof_total_ms(i), L.sj_prof_calls(i)) for i in range(n)}
