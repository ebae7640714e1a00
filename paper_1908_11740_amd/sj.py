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
SJ_STRIPES = 0x8
SJ_SWEEP_X = 0x10
SJ_GBDA = 0x20
SJ_SORTED_OUTPUT = 0x40
INT32_MAX = 2**31 - 1


class SjError(RuntimeError):
    def __init__(self, status, where):
        self.status = status
        detail = lib().sj_last_error().decode()
        super().__init__(f"{where}: {status_string(status)} ({status}) {detail}")


class Grid(ctypes.Structure):
    _fields_ = [("k", ctypes.c_int32), ("split_tau", ctypes.c_int32),
                ("domain", ctypes.c_float * 4), ("flags", ctypes.c_uint32)]


class Choice(ctypes.Structure):
    _fields_ = [("mean_extent", ctypes.c_double), ("k_rule", ctypes.c_int32),
                ("k_learned", ctypes.c_int32), ("tau_learned", ctypes.c_int32),
                ("used_learned", ctypes.c_int32), ("mean_x_extent", ctypes.c_double),
                ("k_cap", ctypes.c_int32)]


class Tuning(ctypes.Structure):
    _fields_ = [("block", ctypes.c_int32), ("small_cap", ctypes.c_int32),
                ("med_cap", ctypes.c_int32), ("split_tau", ctypes.c_int32),
                ("ms", ctypes.c_double)]


class JoinStats(ctypes.Structure):
    _fields_ = [(f, ctypes.c_int64) for f in (
        "n_pairs", "small_tiles", "small_units", "medium_tiles", "dense_tiles", "dense_units",
        "small_entries", "medium_entries", "dense_entries", "pairs_small", "pairs_medium",
        "pairs_dense")] + [("single_pass", ctypes.c_int32), ("small_cap", ctypes.c_int32),
                           ("med_cap", ctypes.c_int32), ("axis_tiles", ctypes.c_int64),
                           ("axis_y", ctypes.c_int64)]


FEAT_SIDE = 1029
FEAT_DIM = 2 * FEAT_SIDE

_lib = None


class DistanceInfo(ctypes.Structure):
    _fields_ = [("candidates", ctypes.c_int64), ("entries_p", ctypes.c_int64),
                ("entries_q", ctypes.c_int64), ("level1_entries_p", ctypes.c_int64),
                ("level1_entries_q", ctypes.c_int64)]


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
        L.sj_join_rects.argtypes = [vp, i64, vp, i64, ctypes.POINTER(Grid), ctypes.POINTER(vp),
                                    ctypes.POINTER(vp), vp, i64, i64p, vp]
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
        f32 = ctypes.c_float
        L.sj_part_stats.argtypes = [vp, i64p, i64p]
        L.sj_part_stats.restype = ctypes.c_int
        L.sj_last_join_stats.argtypes = [ctypes.POINTER(JoinStats)]
        L.sj_last_join_stats.restype = ctypes.c_int
        L.sj_tune.argtypes = [vp, vp, vp, i64, ctypes.c_int32, ctypes.POINTER(Tuning), vp]
        L.sj_tune.restype = ctypes.c_int
        L.sj_tune_set.argtypes = [vp, vp, ctypes.c_int32, ctypes.POINTER(Tuning)]
        L.sj_tune_set.restype = ctypes.c_int
        L.sj_tune_clear.argtypes = []
        L.sj_tune_clear.restype = None
        L.sj_tune_lookup.argtypes = [vp, vp, ctypes.c_int32, ctypes.POINTER(Tuning)]
        L.sj_tune_lookup.restype = ctypes.c_int
        L.sj_tune_save.argtypes = [ctypes.c_char_p]
        L.sj_tune_save.restype = ctypes.c_int
        L.sj_tune_load.argtypes = [ctypes.c_char_p, ctypes.POINTER(ctypes.c_int32)]
        L.sj_tune_load.restype = ctypes.c_int
        L.sj_batch_create.argtypes = [ctypes.c_int32, vp, vp, vp, vp, vp, vp, vp,
                                      ctypes.POINTER(vp), vp]
        L.sj_batch_run.argtypes = [vp, vp, vp]
        L.sj_batch_run_eager.argtypes = [vp, vp, vp]
        L.sj_batch_stats.argtypes = [vp, vp]
        L.sj_batch_entries.argtypes = [vp, vp, vp]
        L.sj_batch_info.argtypes = [vp, vp, vp]
        L.sj_batch_free.argtypes = [vp]
        L.sj_batch_free.restype = None
        L.sj_batch_join.argtypes = [ctypes.c_int32, vp, vp, vp, vp, vp, vp, vp, vp, vp]
        for f in ("sj_batch_create", "sj_batch_run", "sj_batch_run_eager", "sj_batch_stats",
                  "sj_batch_entries", "sj_batch_info", "sj_batch_join"):
            getattr(L, f).restype = ctypes.c_int
        L.sj_generate.argtypes = [vp, i64, vp, vp, vp, ctypes.c_int32, f32, ctypes.c_int32, f32,
                                  f32, ctypes.c_uint64, ctypes.c_uint32, vp]
        L.sj_generate.restype = ctypes.c_int
        L.sj_rule_k.argtypes = [ctypes.c_double]
        L.sj_rule_k.restype = ctypes.c_int32
        L.sj_features.argtypes = [vp, i64, vp, i64, ctypes.POINTER(Grid), vp,
                                  ctypes.POINTER(ctypes.c_double), vp]
        L.sj_choose_grid.argtypes = [vp, i64, vp, i64, ctypes.POINTER(Grid),
                                     ctypes.POINTER(Choice), vp]
        L.sj_picker_load.argtypes = [vp, i64]
        L.sj_picker_unload.argtypes = []
        L.sj_picker_unload.restype = None
        L.sj_picker_loaded.restype = ctypes.c_int32
        L.sj_mlp_param_count.argtypes = [ctypes.c_int32]
        L.sj_mlp_param_count.restype = i64
        L.sj_mlp_forward.argtypes = [vp, ctypes.c_int32, vp, vp, vp, ctypes.c_int32, vp, vp, vp]
        L.sj_mlp_loss.argtypes = [vp, vp, ctypes.c_int32, vp, vp, vp]
        L.sj_mlp_backward.argtypes = [vp, ctypes.c_int32, vp, vp, vp, ctypes.c_int32, vp, vp, vp,
                                      vp, vp]
        L.sj_mlp_adam.argtypes = [vp, vp, vp, vp, i64, f32, f32, f32, f32, ctypes.c_int32, vp]
        L.sj_sweep_axis.argtypes = [vp, vp, vp, i64, vp, vp]
        L.sj_sort_pairs.argtypes = [vp, i64, i64, i64, vp]
        L.sj_sort_pairs_noalloc.argtypes = [vp, i64, i64, i64, vp]
        L.sj_distance_join.argtypes = [vp, i64, vp, i64, f32, ctypes.POINTER(Grid), vp, i64,
                                       i64p, vp]
        L.sj_distance_last_info.argtypes = [ctypes.POINTER(DistanceInfo)]
        L.sj_distance_tune.argtypes = [vp, i64, vp, i64, f32, ctypes.POINTER(Grid), ctypes.c_int32,
                                       ctypes.POINTER(Tuning), vp]
        for f in ("sj_partition", "sj_join", "sj_join_count", "sj_part_info", "sj_part_download",
                  "sj_features", "sj_choose_grid", "sj_picker_load", "sj_mlp_forward",
                  "sj_mlp_loss", "sj_mlp_backward", "sj_mlp_adam", "sj_distance_join", "sj_sweep_axis",
                  "sj_distance_last_info", "sj_distance_tune", "sj_sort_pairs",
                  "sj_sort_pairs_noalloc"):
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

    def stats(self):
        """(level-1 entries, level-2 chunks) of the last partition."""
        m1, nc = ctypes.c_int64(), ctypes.c_int64()
        _check(lib().sj_part_stats(self._h, ctypes.byref(m1), ctypes.byref(nc)), "sj_part_stats")
        return m1.value, nc.value

    def download(self, stream=None):
        n, m, g = self.info()
        C = g.k if g.flags & SJ_STRIPES else g.k * g.k
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


def join_rects(R, S, k, split_tau=0, domain=None, flags=0, out=None, parts=None, stream=None):
    """Partition both inputs and join them with one status readback
    (sj_join_rects).  out: (cap, 2) int32 device tensor, None = count only.
    parts: (PR, PS) Part handles to reuse (None: created).  Returns
    (status, n_pairs, (PR, PS)); status SJ_OK or SJ_ERR_CAPACITY."""
    R, S = _rects(R), _rects(S)
    g = make_grid(k, split_tau, domain, flags)
    hr = ctypes.c_void_p(parts[0].handle if parts is not None else None)
    hs = ctypes.c_void_p(parts[1].handle if parts is not None else None)
    n = ctypes.c_int64()
    cap = 0 if out is None else out.shape[0]
    s = lib().sj_join_rects(ctypes.c_void_p(R.data_ptr() if R.numel() else None), R.shape[0],
                            ctypes.c_void_p(S.data_ptr() if S.numel() else None), S.shape[0],
                            ctypes.byref(g), ctypes.byref(hr), ctypes.byref(hs),
                            ctypes.c_void_p(out.data_ptr() if cap else None), cap,
                            ctypes.byref(n), _stream(stream))
    if s not in (SJ_OK, SJ_ERR_CAPACITY):
        raise SjError(s, "sj_join_rects")
    if parts is None:
        parts = (Part(hr.value, R.shape[0]), Part(hs.value, S.shape[0]))
    return s, n.value, parts


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


def _ptr(t):
    return ctypes.c_void_p(t.data_ptr() if t is not None and t.numel() else None)


def tune(R, S, out=None, reps=2, stream=None):
    """sj_tune: time every candidate schedule for (R, S), cache and return the
    fastest as a dict.  out: (cap, 2) int32 device tensor, or None (count-only)."""
    t = Tuning()
    cap = 0 if out is None else out.shape[0]
    _check(lib().sj_tune(R.handle, S.handle, _ptr(out), cap, int(reps), ctypes.byref(t),
                         _stream(stream)), "sj_tune")
    return {f: getattr(t, f) for f, _ in Tuning._fields_}


def tune_set(R, S, block, small_cap, med_cap, split_tau=0, count_only=False):
    t = Tuning(block, small_cap, med_cap, split_tau, 0.0)
    _check(lib().sj_tune_set(R.handle, S.handle, 1 if count_only else 0, ctypes.byref(t)),
           "sj_tune_set")


def tune_lookup(R, S, count_only=False):
    """The cached schedule for the class of (R, S) (dict), or None."""
    t = Tuning()
    if lib().sj_tune_lookup(R.handle, S.handle, 1 if count_only else 0, ctypes.byref(t)) != SJ_OK:
        return None
    return {"block": t.block, "small_cap": t.small_cap, "med_cap": t.med_cap,
            "split_tau": t.split_tau, "ms": t.ms}


def tune_save(path):
    """sj_tune_save: write the autotuner cache to a text file."""
    _check(lib().sj_tune_save(os.fsencode(path)), "sj_tune_save")


def tune_load(path):
    """sj_tune_load: add the entries of a cache file for this device's
    architecture; returns how many were loaded."""
    n = ctypes.c_int32(0)
    _check(lib().sj_tune_load(os.fsencode(path), ctypes.byref(n)), "sj_tune_load")
    return int(n.value)


def tune_clear():
    lib().sj_tune_clear()


def last_join_stats():
    """Work statistics of the last join on the current device (dict)."""
    st = JoinStats()
    _check(lib().sj_last_join_stats(ctypes.byref(st)), "sj_last_join_stats")
    return {f: getattr(st, f) for f, _ in JoinStats._fields_}


def _points(t):
    if not (isinstance(t, torch.Tensor) and t.is_cuda and t.dtype == torch.float32 and t.dim() == 2
            and t.shape[1] == 2 and t.is_contiguous()):
        raise ValueError("points must be a contiguous (n, 2) float32 CUDA tensor")
    return t


def distance_join_into(P, Q, eps, out, grid, stream=None):
    """sj_distance_join into `out` ((cap, 2) int32 device tensor or None for a
    count).  grid: a Grid, updated in place when its k is 0.  Returns
    (status, n_pairs); SJ_ERR_CAPACITY is returned, not raised."""
    _points(P)
    _points(Q)
    n = ctypes.c_int64(0)
    cap = 0 if out is None else out.shape[0]
    s = lib().sj_distance_join(_ptr(P), P.shape[0], _ptr(Q), Q.shape[0], float(eps),
                               ctypes.byref(grid), _ptr(out), cap, ctypes.byref(n),
                               _stream(stream))
    if s not in (SJ_OK, SJ_ERR_CAPACITY):
        _check(s, "sj_distance_join")
    return s, n.value


def distance_join(P, Q, eps, k=0, split_tau=0, domain=None, flags=0, capacity=None,
                  stream=None):
    """Epsilon-distance join of two (n, 2) float32 point sets: every (i, j)
    with |P[i] - Q[j]| <= eps, as an (M, 2) int32 device tensor (unspecified
    order), and the grid used (dict)."""
    dev = torch.device("cuda", torch.cuda.current_device())
    g = make_grid(k, split_tau, domain, flags)
    cap = (1 << 16) if capacity is None else int(capacity)
    out = torch.empty((cap, 2), dtype=torch.int32, device=dev)
    s, n = distance_join_into(P, Q, eps, out, g, stream)
    if s == SJ_ERR_CAPACITY:
        out = torch.empty((n, 2), dtype=torch.int32, device=dev)
        s, n = distance_join_into(P, Q, eps, out, g, stream)
        _check(s, "sj_distance_join")
    return out[:n], {"k": g.k, "split_tau": g.split_tau}


def distance_tune(P, Q, eps, grid, reps=2, stream=None):
    """sj_distance_tune: time every join schedule on the distance join's
    partitions and cache the fastest; grid (a Grid) is updated when its k is
    0.  Returns the winning schedule as a dict."""
    _points(P)
    _points(Q)
    t = Tuning()
    _check(lib().sj_distance_tune(_ptr(P), P.shape[0], _ptr(Q), Q.shape[0], float(eps),
                                  ctypes.byref(grid), int(reps), ctypes.byref(t), _stream(stream)),
           "sj_distance_tune")
    return {f: getattr(t, f) for f, _ in Tuning._fields_}


def distance_last_info():
    """Work of the last distance join on the current device (dict): candidate
    pairs and the tile entries of the two partitions of squares."""
    d = DistanceInfo()
    _check(lib().sj_distance_last_info(ctypes.byref(d)), "sj_distance_last_info")
    return {f: getattr(d, f) for f, _ in DistanceInfo._fields_}


def sort_pairs(pairs, n_r, n_s, stream=None):
    """sj_sort_pairs: sort an (n, 2) int32 device tensor of (r, s) pairs in
    place, lexicographically; r < n_r and s < n_s."""
    if not (isinstance(pairs, torch.Tensor) and pairs.is_cuda and pairs.dtype == torch.int32 and
            pairs.dim() == 2 and pairs.shape[1] == 2 and pairs.is_contiguous()):
        raise ValueError("pairs must be a contiguous (n, 2) int32 CUDA tensor")
    _check(lib().sj_sort_pairs(_ptr(pairs), pairs.shape[0], int(n_r), int(n_s), _stream(stream)),
           "sj_sort_pairs")
    return pairs


SJ_SORT_NOALLOC_MAX = 4194304


def sort_pairs_noalloc(pairs, n_r, n_s, stream=None):
    """sj_sort_pairs_noalloc: the same sort with the library's fixed per-GPU
    work buffer (no device allocation); at most SJ_SORT_NOALLOC_MAX pairs."""
    if not (isinstance(pairs, torch.Tensor) and pairs.is_cuda and pairs.dtype == torch.int32 and
            pairs.dim() == 2 and pairs.shape[1] == 2 and pairs.is_contiguous()):
        raise ValueError("pairs must be a contiguous (n, 2) int32 CUDA tensor")
    _check(lib().sj_sort_pairs_noalloc(_ptr(pairs), pairs.shape[0], int(n_r), int(n_s),
                                       _stream(stream)), "sj_sort_pairs_noalloc")
    return pairs


def sweep_axis(R, S, tiles, stream=None):
    """The sweeping-axis model (Sec. 3.3, Eq. (2)) for tiles (n, 2) int (tx, ty):
    an (n, 4) int64 array of (k, I^x, I^y, axis), axis 1 = y."""
    import numpy as np
    t = np.ascontiguousarray(tiles, dtype=np.int32).reshape(-1, 2)
    out = np.zeros((len(t), 4), dtype=np.int64)
    _check(lib().sj_sweep_axis(R.handle, S.handle, t.ctypes.data_as(ctypes.c_void_p), len(t),
                               out.ctypes.data_as(ctypes.c_void_p), _stream(stream)),
           "sj_sweep_axis")
    return out


def generate(n, mu=None, sigma=None, weights=None, background=1.0, extent="lognormal",
             ext_a=5e-5, ext_b=1.0, seed=0, side=0, stream=None):
    """(n, 4) float32 device tensor of synthetic rectangles (sj_generate).
    mu (k, 2), sigma (k,), weights (k,): the cluster mixture (host arrays)."""
    import numpy as np
    dev = torch.device("cuda", torch.cuda.current_device())
    out = torch.empty((int(n), 4), dtype=torch.float32, device=dev)
    k = 0 if mu is None else len(mu)
    if k:
        cw = np.cumsum(np.asarray(weights, np.float64))
        cw = (cw / cw[-1]).astype(np.float32)
        cw[-1] = 1.0
        mu_d = torch.from_numpy(np.ascontiguousarray(mu, np.float32)).to(dev)
        sg_d = torch.from_numpy(np.ascontiguousarray(sigma, np.float32)).to(dev)
        cw_d = torch.from_numpy(cw).to(dev)
    else:
        mu_d = sg_d = cw_d = None
    mode = 0 if extent == "lognormal" else 1
    _check(lib().sj_generate(_ptr(out), int(n), _ptr(mu_d), _ptr(sg_d), _ptr(cw_d), k,
                             float(background), mode, float(ext_a), float(ext_b),
                             int(seed) & (2**64 - 1), int(side), _stream(stream)), "sj_generate")
    return out


class Batch:
    """Many joins recorded into one hipGraph (sj_batch_create / sj_batch_run).

    pairs: list of (R, S) device tensors.  grids: optional list of (k, split_tau)
    (0 entries are chosen).  capacities: per-join output slices (None:
    count-only batch)."""

    def __init__(self, pairs, grids=None, capacities=None, flags=0, stream=None):
        import numpy as np
        n = len(pairs)
        self.n = n
        self._keep = [(_rects(r), _rects(s)) for r, s in pairs]
        P = ctypes.c_void_p * max(n, 1)
        self._R = P(*[r.data_ptr() if r.numel() else None for r, _ in self._keep])
        self._S = P(*[s.data_ptr() if s.numel() else None for _, s in self._keep])
        self._nR = np.array([r.shape[0] for r, _ in self._keep] or [0], np.int64)
        self._nS = np.array([s.shape[0] for _, s in self._keep] or [0], np.int64)
        g = (Grid * max(n, 1))()
        for j in range(n):
            k, tau = grids[j] if grids is not None else (0, 0)
            g[j] = make_grid(k, tau, flags=flags)
        self._g = g
        dev = torch.device("cuda", torch.cuda.current_device())
        if capacities is None:
            self.out = None
            self.offsets = None
            out_p, off_p = None, None
        else:
            self.offsets = np.concatenate([[0], np.cumsum(capacities)]).astype(np.int64)
            self.out = torch.empty((int(self.offsets[-1]) + 1, 2), dtype=torch.int32, device=dev)
            out_p = ctypes.c_void_p(self.out.data_ptr())
            off_p = self.offsets.ctypes.data_as(ctypes.c_void_p)
        h = ctypes.c_void_p()
        _check(lib().sj_batch_create(n, self._R, self._nR.ctypes.data_as(ctypes.c_void_p),
                                     self._S, self._nS.ctypes.data_as(ctypes.c_void_p), g,
                                     out_p, off_p, ctypes.byref(h), _stream(stream)),
               "sj_batch_create")
        self._h = h.value

    def run(self, stream=None, eager=False):
        """Replay (eager: the same kernels launched one by one, without the
        recorded graph); returns (status, n_pairs array)."""
        import numpy as np
        n = np.zeros(max(self.n, 1), np.int64)
        f = lib().sj_batch_run_eager if eager else lib().sj_batch_run
        s = f(self._h, n.ctypes.data_as(ctypes.c_void_p), _stream(stream))
        if s not in (SJ_OK, SJ_ERR_CAPACITY):
            raise SjError(s, "sj_batch_run")
        return s, n[:self.n]

    def entries(self):
        """(m1, m): coarse-cell and tile entries of every partition of the
        last run, arrays of 2n (R sides, then S sides)."""
        import numpy as np
        m1 = np.zeros(max(2 * self.n, 1), np.int64)
        m = np.zeros(max(2 * self.n, 1), np.int64)
        _check(lib().sj_batch_entries(self._h, m1.ctypes.data_as(ctypes.c_void_p),
                                      m.ctypes.data_as(ctypes.c_void_p)), "sj_batch_entries")
        return m1[:2 * self.n], m[:2 * self.n]

    def stats(self):
        """Work statistics of the last run, summed over the joins (dict)."""
        st = JoinStats()
        _check(lib().sj_batch_stats(self._h, ctypes.byref(st)), "sj_batch_stats")
        return {f: getattr(st, f) for f, _ in JoinStats._fields_}

    def grids(self):
        import numpy as np
        k = np.zeros(max(self.n, 1), np.int32)
        t = np.zeros(max(self.n, 1), np.int32)
        _check(lib().sj_batch_info(self._h, k.ctypes.data_as(ctypes.c_void_p),
                                   t.ctypes.data_as(ctypes.c_void_p)), "sj_batch_info")
        return k[:self.n], t[:self.n]

    def pairs(self, j, n):
        o = int(self.offsets[j])
        return self.out[o:o + int(n)]

    def free(self):
        if getattr(self, "_h", None):
            lib().sj_batch_free(self._h)
            self._h = None

    def __del__(self):
        try:
            self.free()
        except Exception:
            pass


def rule_k(mean_extent):
    return int(lib().sj_rule_k(float(mean_extent)))


def features(R, S, domain=None, stream=None):
    """(SJ_FEAT_DIM,) float32 device tensor of instance features and the rule's
    mean extent e."""
    R, S = _rects(R), _rects(S)
    out = torch.empty(FEAT_DIM, dtype=torch.float32, device=R.device)
    e = ctypes.c_double()
    g = make_grid(1, 0, domain)
    _check(lib().sj_features(_ptr(R), R.shape[0], _ptr(S), S.shape[0], ctypes.byref(g),
                             _ptr(out), ctypes.byref(e), _stream(stream)), "sj_features")
    return out, e.value


def choose_grid(R, S, k=0, split_tau=0, domain=None, flags=0, stream=None):
    """sj_choose_grid: returns (k, split_tau, info dict)."""
    R, S = _rects(R), _rects(S)
    g = make_grid(k, split_tau, domain, flags)
    c = Choice()
    _check(lib().sj_choose_grid(_ptr(R), R.shape[0], _ptr(S), S.shape[0], ctypes.byref(g),
                                ctypes.byref(c), _stream(stream)), "sj_choose_grid")
    info = {f: getattr(c, f) for f, _ in Choice._fields_}
    return g.k, g.split_tau, info


def picker_load(blob):
    """Load a picker blob (host float32 array: mu | sd | ystat | params)."""
    import numpy as np
    b = np.ascontiguousarray(blob, dtype=np.float32)
    _check(lib().sj_picker_load(b.ctypes.data_as(ctypes.c_void_p), b.size), "sj_picker_load")


def picker_unload():
    lib().sj_picker_unload()


def picker_loaded():
    return bool(lib().sj_picker_loaded())


def mlp_param_count(d_in):
    return int(lib().sj_mlp_param_count(int(d_in)))


def mlp_forward(params, X, mu=None, sd=None, act=None, stream=None):
    B, d = X.shape
    Y = torch.empty((B, 2), dtype=torch.float32, device=X.device)
    _check(lib().sj_mlp_forward(_ptr(params), d, _ptr(mu), _ptr(sd), _ptr(X), B, _ptr(Y),
                                _ptr(act), _stream(stream)), "sj_mlp_forward")
    return Y


def mlp_loss(Y, T, stream=None):
    dY = torch.empty_like(Y)
    loss = torch.empty(1, dtype=torch.float32, device=Y.device)
    _check(lib().sj_mlp_loss(_ptr(Y), _ptr(T), Y.shape[0], _ptr(dY), _ptr(loss), _stream(stream)),
           "sj_mlp_loss")
    return loss, dY


def mlp_backward(params, X, act, dY, mu=None, sd=None, grad=None, dact=None, stream=None):
    B, d = X.shape
    if grad is None:
        grad = torch.empty_like(params)
    if dact is None:
        dact = torch.empty((B, 128), dtype=torch.float32, device=X.device)
    _check(lib().sj_mlp_backward(_ptr(params), d, _ptr(mu), _ptr(sd), _ptr(X), B, _ptr(act),
                                 _ptr(dY), _ptr(dact), _ptr(grad), _stream(stream)),
           "sj_mlp_backward")
    return grad


def mlp_adam(params, m, v, grad, step, lr=1e-3, beta1=0.9, beta2=0.999, eps=1e-8, stream=None):
    _check(lib().sj_mlp_adam(_ptr(params), _ptr(m), _ptr(v), _ptr(grad), params.numel(), lr,
                             beta1, beta2, eps, int(step), _stream(stream)), "sj_mlp_adam")


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
