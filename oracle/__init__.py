"""CPU oracle for the MBR filter step of the partition-based spatial join
(arXiv 1908.11740).

TEST INFRASTRUCTURE ONLY.  Only ``tests/``, ``__graft_entry__.smoke()`` and
the CPU-baseline leg of ``bench.py`` may import this package.  It shares no
code with the GPU library and never imports it.

Python wrappers around ``sj_oracle.c`` (brute force = the definition of
Sec. 1; Algorithm 1 over the whole input, Sec. 2.1; PBSM with the parallel
phases of Sec. 3.4 and the duplicate test of Eq. (1); the epsilon-distance
join of point sets of Sec. 1, by its definition and by the filter-and-refine
steps: squares of side eps, PBSM, distance check).  Every wrapper returns
the pair set as an ``(P, 2)`` int32 array sorted lexicographically by
``(r, s)``; the sort is a library primitive applied to the oracle's output.
"""
import ctypes
import os

import numpy as np

from . import build as _build

_lib = None


def _load():
    global _lib
    if _lib is None:
        path = _build.LIB
        if not os.path.exists(path) or os.path.getmtime(path) < os.path.getmtime(_build.SRC):
            _build.build()
        lib = ctypes.CDLL(path)
        f32p = ctypes.POINTER(ctypes.c_float)
        i32pp = ctypes.POINTER(ctypes.POINTER(ctypes.c_int32))
        i64 = ctypes.c_int64
        lib.oracle_bruteforce.argtypes = [f32p, i64, f32p, i64, i32pp]
        lib.oracle_bruteforce.restype = i64
        lib.oracle_sweep.argtypes = [f32p, i64, f32p, i64, i32pp]
        lib.oracle_sweep.restype = i64
        lib.oracle_pbsm.argtypes = [f32p, i64, f32p, i64, ctypes.c_int, f32p, ctypes.c_int,
                                    i32pp, ctypes.POINTER(ctypes.c_double),
                                    ctypes.POINTER(ctypes.c_double)]
        lib.oracle_pbsm.restype = i64
        lib.oracle_partition_ids.argtypes = [f32p, i64, ctypes.c_int, f32p,
                                             ctypes.POINTER(ctypes.c_int64), i32pp]
        lib.oracle_partition_ids.restype = i64
        lib.oracle_distance_brute.argtypes = [f32p, i64, f32p, i64, ctypes.c_float, i32pp]
        lib.oracle_distance_brute.restype = i64
        lib.oracle_distance_refine.argtypes = [f32p, f32p, ctypes.c_float,
                                               ctypes.POINTER(ctypes.c_int32), i64]
        lib.oracle_distance_refine.restype = i64
        lib.oracle_gbda.argtypes = [f32p, i64, f32p, i64, ctypes.c_int, f32p, i32pp]
        lib.oracle_gbda.restype = i64
        lib.oracle_free.argtypes = [ctypes.c_void_p]
        lib.oracle_free.restype = None
        lib.oracle_max_threads.argtypes = []
        lib.oracle_max_threads.restype = ctypes.c_int
        _lib = lib
    return _lib


def _rects(a):
    a = np.ascontiguousarray(a, dtype=np.float32)
    if a.ndim != 2 or a.shape[1] != 4:
        raise ValueError("rectangles must be an (n, 4) float32 array of (x_l, y_l, x_u, y_u)")
    return a


def _fp(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_float))


def _take(n, ptr, sort=True):
    lib = _load()
    if n < 0:
        raise MemoryError("oracle allocation failed")
    if n == 0:
        return np.zeros((0, 2), dtype=np.int32)
    arr = np.ctypeslib.as_array(ptr, shape=(n * 2,)).copy().reshape(n, 2)
    lib.oracle_free(ptr)
    if sort:
        arr = arr[np.lexsort((arr[:, 1], arr[:, 0]))]
    return arr


def bruteforce(R, S):
    """The definition: every (i, j) whose closed rectangles intersect."""
    R, S = _rects(R), _rects(S)
    out = ctypes.POINTER(ctypes.c_int32)()
    n = _load().oracle_bruteforce(_fp(R), len(R), _fp(S), len(S), ctypes.byref(out))
    return _take(n, out)


def sweep(R, S):
    """Algorithm 1 (forward-scan plane sweep) over the whole input."""
    R, S = _rects(R), _rects(S)
    out = ctypes.POINTER(ctypes.c_int32)()
    n = _load().oracle_sweep(_fp(R), len(R), _fp(S), len(S), ctypes.byref(out))
    return _take(n, out)


def pbsm(R, S, K, domain=None, threads=0, timings=False, sort=True):
    """PBSM on a K x K grid: partition (Sec. 3.4 steps 1-4), per-tile sort and
    Algorithm 1 (steps 5-6), duplicate test of Eq. (1).

    threads <= 0 uses every core OpenMP reports.  With ``timings=True``
    returns ``(pairs, t_partition_s, t_join_s)``.
    """
    R, S = _rects(R), _rects(S)
    dom = None
    if domain is not None:
        dom = np.ascontiguousarray(domain, dtype=np.float32)
    out = ctypes.POINTER(ctypes.c_int32)()
    tp, tj = ctypes.c_double(0), ctypes.c_double(0)
    n = _load().oracle_pbsm(_fp(R), len(R), _fp(S), len(S), int(K),
                            _fp(dom) if dom is not None else None, int(threads),
                            ctypes.byref(out), ctypes.byref(tp), ctypes.byref(tj))
    if n == -2:
        raise ValueError("K must be >= 1")
    pairs = _take(n, out, sort=sort)
    if timings:
        return pairs, tp.value, tj.value
    return pairs


def gbda(R, S, K, domain=None):
    """The class-based duplicate avoidance (GBDA) variant of PBSM: per tile,
    the 9 class-class joins that can hold a pair whose reference point is in
    the tile, Algorithm 1 on each, no duplicate test."""
    R, S = _rects(R), _rects(S)
    dom = None if domain is None else np.ascontiguousarray(domain, dtype=np.float32)
    out = ctypes.POINTER(ctypes.c_int32)()
    n = _load().oracle_gbda(_fp(R), len(R), _fp(S), len(S), int(K),
                            _fp(dom) if dom is not None else None, ctypes.byref(out))
    if n == -2:
        raise ValueError("K must be >= 1")
    return _take(n, out, sort=False)


def partition_ids(A, K, domain=None):
    """Per-tile membership under the oracle's grid: (offsets[K*K+1], ids)."""
    A = _rects(A)
    dom = None if domain is None else np.ascontiguousarray(domain, dtype=np.float32)
    off = np.zeros(K * K + 1, dtype=np.int64)
    ids = ctypes.POINTER(ctypes.c_int32)()
    n = _load().oracle_partition_ids(_fp(A), len(A), int(K),
                                     _fp(dom) if dom is not None else None,
                                     off.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)),
                                     ctypes.byref(ids))
    if n < 0:
        raise MemoryError("oracle allocation failed")
    if n == 0:
        return off, np.zeros(0, dtype=np.int32)
    arr = np.ctypeslib.as_array(ids, shape=(n,)).copy()
    _load().oracle_free(ids)
    return off, arr


def max_threads():
    return int(_load().oracle_max_threads())


# ----------------------------------------------------------------------------
# Epsilon-distance join of point sets (Sec. 1)
# ----------------------------------------------------------------------------
def _points(a):
    a = np.ascontiguousarray(a, dtype=np.float32)
    if a.ndim != 2 or a.shape[1] != 2:
        raise ValueError("points must be an (n, 2) float32 array of (x, y)")
    return a


def distance_brute(P, Q, eps):
    """The definition: every (i, j) with dx*dx + dy*dy <= eps*eps, in float64
    from the float32 coordinates, each operation rounded once."""
    P, Q = _points(P), _points(Q)
    out = ctypes.POINTER(ctypes.c_int32)()
    n = _load().oracle_distance_brute(_fp(P), len(P), _fp(Q), len(Q), float(np.float32(eps)),
                                      ctypes.byref(out))
    return _take(n, out)


def squares(P, eps, rel=2.0 ** -40):
    """Filter rectangles of Sec. 1: the square of side eps centred on each
    point, as the smallest float32 box containing the square widened by
    rel * (|c| + eps/2) per coordinate c (so that no pair the distance test
    accepts is lost to rounding).  Returns (n, 4) float32."""
    P = _points(P).astype(np.float64)
    h = 0.5 * float(np.float32(eps))
    m = (np.abs(P) + h) * rel
    lo, hi = P - h - m, P + h + m
    lo32, hi32 = lo.astype(np.float32), hi.astype(np.float32)
    lo32 = np.where(lo32.astype(np.float64) > lo, np.nextafter(lo32, np.float32(-np.inf)), lo32)
    hi32 = np.where(hi32.astype(np.float64) < hi, np.nextafter(hi32, np.float32(np.inf)), hi32)
    return np.ascontiguousarray(np.stack([lo32[:, 0], lo32[:, 1], hi32[:, 0], hi32[:, 1]], 1),
                                dtype=np.float32)


def refine(P, Q, eps, pairs):
    """The refinement step: the candidate pairs that pass the distance test."""
    P, Q = _points(P), _points(Q)
    c = np.ascontiguousarray(pairs, dtype=np.int32).reshape(-1, 2).copy()
    if len(c) and (c[:, 0].max() >= len(P) or c[:, 1].max() >= len(Q) or c.min() < 0):
        raise IndexError("candidate index out of range")
    k = _load().oracle_distance_refine(_fp(P), _fp(Q), float(np.float32(eps)),
                                       c.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)), len(c))
    return c[:k]


def distance_filter_refine(P, Q, eps, K, domain=None, threads=0):
    """The paper's steps (Sec. 1): squares of side eps around both point
    sets, their intersection join by PBSM on a K x K grid, then the distance
    test on every candidate.  Returns the sorted pair set."""
    cand = pbsm(squares(P, eps), squares(Q, eps), K, domain=domain, threads=threads, sort=False)
    out = refine(P, Q, eps, cand)
    return out[np.lexsort((out[:, 1], out[:, 0]))] if len(out) else out
