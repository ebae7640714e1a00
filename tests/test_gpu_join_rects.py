"""GPU parity of sj_join_rects (both partitions and the join, one status
readback): the oracle's pair set element by element, reused handles, the
regrowth of partitions that outgrow their first buffers, and the error
contract."""
import sys

import numpy as np
import pytest

import oracle
from paper_1908_11740_amd import datagen

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

from paper_1908_11740_amd import sj  # noqa: E402
from gpu_util import sort_pairs, to_dev  # noqa: E402


def say(*a):
    print(*a, file=sys.stderr, flush=True)


def fused(R, S, K, cap=None, parts=None, **kw):
    Rd, Sd = (R, S) if isinstance(R, torch.Tensor) else (to_dev(R), to_dev(S))
    out = None if cap == 0 else torch.empty((cap or (1 << 18), 2), dtype=torch.int32,
                                            device="cuda")
    st, n, parts = sj.join_rects(Rd, Sd, K, out=out, parts=parts, **kw)
    got = None
    if out is not None and st == sj.SJ_OK:
        torch.cuda.synchronize()
        got = sort_pairs(out[:n].cpu().numpy())
    return st, n, got, parts


@pytest.mark.parametrize("K", [1, 7, 64, 1000])
def test_small_case_matches_the_oracle(K):
    R, S, _ = datagen.small_case()
    ref = oracle.bruteforce(R, S)
    say("join_rects small case K", K)
    st, n, got, parts = fused(R, S, K)
    assert st == sj.SJ_OK and n == len(ref)
    assert np.array_equal(got, ref)
    assert sj.last_join_stats()["n_pairs"] == len(ref)
    st, n, _, _ = fused(R, S, K, cap=0, parts=parts)  # count only, same handles
    assert st == sj.SJ_OK and n == len(ref)
    for P in parts:
        P.free()


def test_partitions_outgrow_their_first_buffers():
    """Extents of 0.05 at K = 200 put each rectangle in about 100 tiles, far
    beyond the first sizing (2n + 4096 entries): the call must grow the
    partitions and run the sequence again, with the oracle's pairs."""
    R = datagen.uniform(3000, 0.05, 31)
    S = datagen.uniform(2500, 0.05, 32)
    ref = oracle.pbsm(R, S, 200)
    say("join_rects regrowth")
    st, n, got, parts = fused(R, S, 200, cap=len(ref) + 10)
    assert st == sj.SJ_OK and n == len(ref)
    assert np.array_equal(got, ref)
    assert parts[0].info()[1] > 2 * 3000 + 4096
    for P in parts:
        P.free()


def test_reused_handles_across_sizes_and_grids():
    Rd0 = to_dev(datagen.uniform(20000, 0.004, 41))
    Sd0 = to_dev(datagen.uniform(15000, 0.004, 42))
    parts = None
    for n_r, n_s, K in ((20000, 15000, 300), (5000, 15000, 64), (20000, 200, 1500),
                        (20000, 15000, 300)):
        R, S = Rd0[:n_r].contiguous(), Sd0[:n_s].contiguous()
        ref = oracle.pbsm(R.cpu().numpy(), S.cpu().numpy(), K)
        say("join_rects reuse", n_r, n_s, K)
        st, n, got, parts = fused(R, S, K, parts=parts)
        assert st == sj.SJ_OK and np.array_equal(got, ref), (n_r, n_s, K)
    for P in parts:
        P.free()


def test_uniform_1m_element_by_element():
    R, S = datagen.uniform_1m()
    K = 1024
    ref = oracle.pbsm(R, S, K)
    say("join_rects uniform 1M K", K)
    st, n, got, parts = fused(R, S, K, cap=len(ref) + 1)
    assert st == sj.SJ_OK and n == len(ref)
    assert np.array_equal(got, ref)
    for P in parts:
        P.free()


def test_capacity_and_errors():
    R, S, K = datagen.small_case()
    ref = oracle.bruteforce(R, S)
    for cap in (1, len(ref) - 1):
        st, n, _, parts = fused(R, S, K, cap=cap)
        assert st == sj.SJ_ERR_CAPACITY and n == len(ref)
        for P in parts:
            P.free()
    bad = R.copy()
    bad[11] = [0.5, 0.1, 0.4, 0.2]
    with pytest.raises(sj.SjError) as ei:
        fused(bad, S, K)
    assert ei.value.status == sj.SJ_ERR_RECT
    with pytest.raises(sj.SjError) as ei:
        fused(R, S, K, flags=sj.SJ_PLAIN)
    assert ei.value.status == sj.SJ_ERR_ARG
    # the library is consistent afterwards
    st, n, got, parts = fused(R, S, K)
    assert st == sj.SJ_OK and np.array_equal(got, ref)
    for P in parts:
        P.free()


def test_empty_inputs():
    R, S, K = datagen.small_case()
    E = np.zeros((0, 4), np.float32)
    for A, B in ((E, S), (R, E), (E, E)):
        st, n, got, parts = fused(A, B, K)
        assert st == sj.SJ_OK and n == 0
        for P in parts:
            P.free()


@pytest.fixture(scope="module")
def mid():
    R = datagen.uniform(20000, 0.01, 51)
    S = datagen.uniform(15000, 0.01, 52)
    return R, S, oracle.bruteforce(R, S)


@pytest.mark.parametrize("name", ["stripes", "gbda", "sorted", "twopass", "sweepx", "tau1"])
def test_schedule_flags_match_the_oracle(mid, name):
    """Every schedule flag through the one-readback path, on a grid of one
    tile (a single dense tile), a coarse grid and a fine one."""
    R, S, ref = mid
    kw = {"stripes": dict(flags=sj.SJ_STRIPES), "gbda": dict(flags=sj.SJ_GBDA),
          "sorted": dict(flags=sj.SJ_SORTED_OUTPUT), "twopass": dict(flags=sj.SJ_TWO_PASS),
          "sweepx": dict(flags=sj.SJ_SWEEP_X), "tau1": dict(split_tau=1)}[name]
    Rd, Sd = to_dev(R), to_dev(S)
    parts = None
    for K in (1, 16, 200):
        say("join_rects", name, "K", K)
        out = torch.empty((len(ref) + 10, 2), dtype=torch.int32, device="cuda")
        st, n, parts = sj.join_rects(Rd, Sd, K, out=out, parts=parts, **kw)
        assert st == sj.SJ_OK and n == len(ref), (name, K)
        raw = out[:n].cpu().numpy()
        if name == "sorted":  # the library's own order: no sort here
            assert np.array_equal(raw, ref), K
        else:
            assert np.array_equal(sort_pairs(raw), ref), (name, K)
    for P in parts:
        P.free()
