"""GPU parity of the epsilon-distance join (Sec. 1: squares of side eps
around the points, the intersection join, a distance check): the pair set
equals the oracle's bit for bit on every grid and schedule, on lattices with
known counts, on pairs within a few ulps of the boundary, and -- at the
benchmark's 10M x 10M size -- on sampled points computed one by one."""
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

SCHED = {"tuned": dict(), "plain": dict(flags=sj.SJ_PLAIN), "twopass": dict(flags=sj.SJ_TWO_PASS),
         "tau1": dict(split_tau=1), "stripes": dict(flags=sj.SJ_STRIPES),
         "gbda": dict(split_tau=1, flags=sj.SJ_GBDA), "sweepx": dict(flags=sj.SJ_SWEEP_X)}


def say(*a):
    print(*a, file=sys.stderr, flush=True)


def gpu_distance(P, Q, eps, k=0, **kw):
    pairs, grid = sj.distance_join(to_dev(P), to_dev(Q), eps, k=k, **kw)
    torch.cuda.synchronize()
    return sort_pairs(pairs.cpu().numpy()), grid


@pytest.fixture(scope="module")
def small():
    mix = datagen.mixture_spec(20, 9)
    P = datagen.points_mixture(3000, mix, 0.2, 21)
    Q = datagen.points_mixture(2500, mix, 0.2, 22)
    eps = 0.01
    return P, Q, eps, oracle.distance_brute(P, Q, eps)


@pytest.mark.parametrize("k", [0, 1, 2, 7, 64, 300])
@pytest.mark.parametrize("sched", sorted(SCHED))
def test_small_vs_definition(small, k, sched):
    P, Q, eps, ref = small
    say("distance small k", k, sched)
    got, grid = gpu_distance(P, Q, eps, k=k, **SCHED[sched])
    assert np.array_equal(got, ref) and len(ref) > 1000
    assert grid["k"] >= 1 and (k == 0 or grid["k"] == k)


@pytest.mark.parametrize("eps,expect", [(0.5, 100), (1.0, 460), (1.5, 784), (2.0, 1104)])
@pytest.mark.parametrize("k", [0, 1, 4, 11])
def test_lattice_counts(eps, expect, k):
    say("distance lattice", eps, k)
    L = datagen.lattice(10, 10)
    got, _ = gpu_distance(L, L, eps, k=k, domain=(-1.0, -1.0, 10.0, 10.0))
    assert len(got) == expect
    assert np.array_equal(got, oracle.distance_brute(L, L, eps))


@pytest.mark.parametrize("eps", [1e-3, 0.0371])
@pytest.mark.parametrize("k", [0, 50])
def test_near_boundary(eps, k):
    say("distance near ring", eps, k)
    P, Q = datagen.near_ring(20_000, eps, 51)
    ref = oracle.distance_brute(P, Q, eps)
    got, _ = gpu_distance(P, Q, eps, k=k)
    assert np.array_equal(got, ref)
    own = int((ref[:, 0] == ref[:, 1]).sum())
    assert 0 < own < len(P)
    # the filter's candidates contain the result
    info = sj.distance_last_info()
    assert info["candidates"] >= len(ref)
    assert info["entries_p"] >= len(P) and info["entries_q"] >= len(Q)


def test_medium_vs_filter_and_refine():
    say("distance medium")
    mix = datagen.mixture_spec(50, 77)
    P = datagen.points_mixture(200_000, mix, 0.2, 61)
    Q = datagen.points_mixture(150_000, mix, 0.2, 62)
    eps = 2e-3
    ref = oracle.distance_filter_refine(P, Q, eps, 200)
    for k, sched in ((0, "tuned"), (123, "tau1"), (0, "stripes")):
        got, _ = gpu_distance(P, Q, eps, k=k, **SCHED[sched])
        assert np.array_equal(got, ref), (k, sched)
    assert len(ref) > 1_000_000


@pytest.mark.parametrize("k", [0, 5, 97])
def test_sorted_output_is_the_oracle_list(small, k):
    """With SJ_SORTED_OUTPUT the pairs come out in the oracle's (i, j) order,
    byte for byte, on any grid."""
    P, Q, eps, ref = small
    pairs, _ = sj.distance_join(to_dev(P), to_dev(Q), eps, k=k, flags=sj.SJ_SORTED_OUTPUT)
    torch.cuda.synchronize()
    got = pairs.cpu().numpy()
    assert got.shape == ref.shape and np.array_equal(got, ref)


def test_filter_pairs_counted_in_every_mode(small):
    """The filter's pair count does not depend on the schedule: single pass,
    two passes (counted once, in the counting pass) and count only agree."""
    P, Q, eps, ref = small
    Pd, Qd = to_dev(P), to_dev(Q)
    counts = []
    for flags in (0, sj.SJ_TWO_PASS):
        gpu_distance(P, Q, eps, k=33, flags=flags)
        counts.append(sj.distance_last_info()["candidates"])
    s, n = sj.distance_join_into(Pd, Qd, eps, None, sj.make_grid(33))
    assert s == sj.SJ_OK and n == len(ref)
    counts.append(sj.distance_last_info()["candidates"])
    assert counts[0] == counts[1] == counts[2] >= len(ref)


def test_zero_eps_and_duplicates():
    P = datagen.points_uniform(5000, 71)
    rng = np.random.default_rng(72)
    Q = np.concatenate([datagen.points_uniform(3000, 73), P[rng.choice(5000, 700)]])
    for k in (0, 16):
        got, _ = gpu_distance(P, Q, 0.0, k=k)
        assert np.array_equal(got, oracle.distance_brute(P, Q, 0.0))


def test_offset_domain_and_points_outside_it():
    L = datagen.lattice(40, 30, 0.25, (1000.0, -7.0))
    ref = oracle.distance_brute(L, L, 0.375)
    got, _ = gpu_distance(L, L, 0.375, k=9, domain=(1000.0, -7.0, 1010.0, 0.5))
    assert np.array_equal(got, ref)
    # a domain covering only part of the points: border tiles take the rest
    got, _ = gpu_distance(L, L, 0.375, k=5, domain=(1002.0, -5.0, 1004.0, -3.0))
    assert np.array_equal(got, ref)


def test_empty_and_single():
    E = np.zeros((0, 2), np.float32)
    P = datagen.points_uniform(100, 81)
    for a, b in ((E, P), (P, E), (E, E)):
        got, _ = gpu_distance(a, b, 0.1, k=4)
        assert len(got) == 0
    one = P[:1]
    got, _ = gpu_distance(one, P, 0.2, k=0)
    assert np.array_equal(got, oracle.distance_brute(one, P, 0.2))


def test_capacity_and_count_only():
    P, Q, eps = datagen.points_uniform(4000, 91), datagen.points_uniform(4000, 92), 0.02
    ref = oracle.distance_brute(P, Q, eps)
    Pd, Qd = to_dev(P), to_dev(Q)
    g = sj.make_grid(32)
    s, n = sj.distance_join_into(Pd, Qd, eps, None, g)
    assert s == sj.SJ_OK and n == len(ref)
    small = torch.empty((len(ref) // 3, 2), dtype=torch.int32, device="cuda")
    s, n = sj.distance_join_into(Pd, Qd, eps, small, g)
    assert s == sj.SJ_ERR_CAPACITY and n == len(ref)
    full = torch.empty((len(ref), 2), dtype=torch.int32, device="cuda")
    s, n = sj.distance_join_into(Pd, Qd, eps, full, g)
    assert s == sj.SJ_OK and np.array_equal(sort_pairs(full.cpu().numpy()), ref)


def test_invalid_arguments():
    P = datagen.points_uniform(10, 1)
    bad = P.copy()
    bad[3, 1] = np.nan
    with pytest.raises(sj.SjError) as e:
        gpu_distance(bad, P, 0.1, k=4)
    assert e.value.status == sj.SJ_ERR_RECT
    for eps in (-1.0, float("inf"), float("nan")):
        with pytest.raises(sj.SjError) as e:
            gpu_distance(P, P, eps, k=4)
        assert e.value.status == sj.SJ_ERR_ARG


def test_full_size_element_by_element():
    """Skewed 10M x 10M points, eps = 1e-4, in the benchmark's configuration
    (grid chosen by the library): the whole pair list equals the oracle's
    filter-and-refine steps (Sec. 1) on the same grid, element by element
    after sorting, and the pair count does not depend on the grid or
    schedule."""
    P, Q, eps = datagen.skewed_points_10m()
    Pd, Qd = to_dev(P), to_dev(Q)
    say("distance full size")
    pairs, grid = sj.distance_join(Pd, Qd, eps)
    n = pairs.shape[0]
    got = sort_pairs(pairs.cpu().numpy())
    del pairs
    say("distance full size: oracle on the grid K =", grid["k"])
    ref = oracle.distance_filter_refine(P, Q, eps, grid["k"])
    assert len(ref) > 0 and got.shape == ref.shape
    assert np.array_equal(got, ref)
    del got, ref
    g2 = sj.make_grid(max(1, grid["k"] // 3), flags=sj.SJ_TWO_PASS)
    s, n2 = sj.distance_join_into(Pd, Qd, eps, None, g2)
    assert s == sj.SJ_OK and n2 == n


def test_tuned_schedule_keeps_the_result():
    mix = datagen.mixture_spec(30, 41)
    P = datagen.points_mixture(120_000, mix, 0.2, 42)
    Q = datagen.points_mixture(100_000, mix, 0.2, 43)
    eps = 1.5e-3
    ref = oracle.distance_filter_refine(P, Q, eps, 128)
    Pd, Qd = to_dev(P), to_dev(Q)
    g = sj.make_grid(0)
    best = sj.distance_tune(Pd, Qd, eps, g, reps=1)
    assert g.k >= 1 and best["block"] in (64, 128, 256, 512)
    got, _ = sj.distance_join(Pd, Qd, eps)
    assert np.array_equal(sort_pairs(got.cpu().numpy()), ref)
    sj.tune_clear()
