"""The zero-allocation sort (sj_sort_pairs_noalloc) through the C ABI: its
output equals sj_sort_pairs' on the same input, on two calls in a row (the
second smaller, so stale contents of the fixed work buffer would show), at
the size limit, and it rejects a larger input without touching it."""
import ctypes
import sys

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

from paper_1908_11740_amd import sj  # noqa: E402


def say(*a):
    print(*a, file=sys.stderr, flush=True)


def _pairs(n, nr, ns, seed):
    rng = np.random.default_rng(seed)
    p = np.stack([rng.integers(0, nr, n), rng.integers(0, ns, n)], 1).astype(np.int32)
    if n > 10:
        p[: n // 10] = p[n // 10: 2 * (n // 10)]  # duplicates
    return p


def _both(p, nr, ns):
    a = torch.from_numpy(p.copy()).cuda()
    b = torch.from_numpy(p.copy()).cuda()
    sj.sort_pairs(a, nr, ns)
    L = sj.lib()
    st = L.sj_sort_pairs_noalloc(ctypes.c_void_p(b.data_ptr()), b.shape[0], nr, ns,
                                 ctypes.c_void_p(torch.cuda.current_stream().cuda_stream))
    assert st == sj.SJ_OK, sj.status_string(st)
    torch.cuda.synchronize()
    return a.cpu().numpy(), b.cpu().numpy()


def test_noalloc_sort_equals_sort_two_calls_second_smaller():
    for n, nr, ns, seed in ((3_000_001, 10_000_000, 10_000_000, 1), (70_001, 300, 1 << 24, 2)):
        say("noalloc sort", n, nr, ns)
        p = _pairs(n, nr, ns, seed)
        a, b = _both(p, nr, ns)
        assert np.array_equal(a, b)
        assert np.array_equal(b, p[np.lexsort((p[:, 1], p[:, 0]))])


def test_noalloc_sort_at_the_limit_and_tiny():
    n = sj.SJ_SORT_NOALLOC_MAX
    say("noalloc sort at the limit", n)
    p = _pairs(n, 1 << 31, 1 << 31, 3)
    a, b = _both(p, 1 << 31, 1 << 31)
    assert np.array_equal(a, b)
    for n in (0, 1, 2, 4097):
        p = _pairs(n, 50, 60, 4 + n)
        a, b = _both(p, 50, 60)
        assert np.array_equal(a, b)


def test_noalloc_sort_rejects_more_than_the_limit():
    n = sj.SJ_SORT_NOALLOC_MAX + 1
    p = _pairs(n, 1000, 1000, 5)
    d = torch.from_numpy(p.copy()).cuda()
    st = sj.lib().sj_sort_pairs_noalloc(ctypes.c_void_p(d.data_ptr()), n, 1000, 1000,
                                        ctypes.c_void_p(torch.cuda.current_stream().cuda_stream))
    assert st == sj.SJ_ERR_TOO_LARGE
    assert b"SJ_SORT_NOALLOC_MAX" in sj.lib().sj_last_error()
    torch.cuda.synchronize()
    assert np.array_equal(d.cpu().numpy(), p)
