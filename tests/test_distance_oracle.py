"""Pins of the epsilon-distance join oracle (Sec. 1: distance join of point
sets through squares of side eps and a distance check).

The definition (``oracle.distance_brute``) is pinned by hand cases, closed
lattice counts, a library k-d tree and invariants; the paper's
filter-and-refine steps (``oracle.distance_filter_refine``) are pinned to
the definition, including on pairs placed within a few ulps of the
boundary."""
import numpy as np
import pytest
from scipy.spatial import cKDTree

import oracle
from paper_1908_11740_amd import datagen


def _set(pairs):
    return {(int(a), int(b)) for a, b in pairs}


def test_three_four_five_boundary():
    P = np.array([[0, 0]], np.float32)
    Q = np.array([[3, 4]], np.float32)
    assert _set(oracle.distance_brute(P, Q, 5.0)) == {(0, 0)}
    assert len(oracle.distance_brute(P, Q, np.nextafter(np.float32(5), np.float32(0)))) == 0
    # the pair order is (P index, Q index)
    P2 = np.array([[9, 9], [0, 0]], np.float32)
    assert _set(oracle.distance_brute(P2, Q, 5.0)) == {(1, 0)}
    assert _set(oracle.distance_brute(Q, P2, 5.0)) == {(0, 1)}


@pytest.mark.parametrize("eps,expect", [
    (0.5, 100),    # only each point with itself
    (1.0, 460),    # + 180 axis neighbours, both orders
    (1.5, 784),    # + 162 diagonal neighbours (sqrt 2)
    (2.0, 1104),   # + 160 at distance 2 (sqrt 5 > 2)
])
def test_lattice_closed_form_counts(eps, expect):
    L = datagen.lattice(10, 10)
    assert len(oracle.distance_brute(L, L, eps)) == expect


def test_lattice_scaled_and_offset():
    # spacing 0.25 (exact in binary) away from the origin: the same counts
    L = datagen.lattice(10, 10, 0.25, (100.0, -3.0))
    assert len(oracle.distance_brute(L, L, 0.25)) == 460
    assert len(oracle.distance_brute(L, L, 0.375)) == 784


def test_matches_a_kd_tree():
    P = datagen.points_uniform(3000, 11)
    Q = datagen.points_uniform(2500, 12)
    eps = 0.02
    got = _set(oracle.distance_brute(P, Q, eps))
    tree = cKDTree(Q.astype(np.float64))
    want = set()
    for i, js in enumerate(tree.query_ball_point(P.astype(np.float64), eps)):
        want.update((i, j) for j in js)
    assert got == want and len(got) > 1000


def test_symmetry_and_zero_eps():
    rng = np.random.default_rng(5)
    P = datagen.points_uniform(500, 13)
    Q = np.concatenate([datagen.points_uniform(400, 14), P[rng.choice(500, 50)]])
    a = oracle.distance_brute(P, Q, 0.03)
    b = oracle.distance_brute(Q, P, 0.03)
    assert _set(a) == {(j, i) for i, j in _set(b)}
    # eps = 0: exactly the equal points
    eq = {(i, j) for i in range(len(P)) for j in range(len(Q)) if (P[i] == Q[j]).all()}
    assert _set(oracle.distance_brute(P, Q, 0.0)) == eq and len(eq) >= 50


def test_squares_contain_the_disc_and_are_float32_tight():
    P = np.array([[0.5, 0.25], [0.0, 0.0], [1e6, -3.5]], np.float32)
    eps = np.float32(0.1)
    B = oracle.squares(P, eps)
    c = P.astype(np.float64)
    h = 0.5 * float(eps)
    assert (B[:, :2].astype(np.float64) <= c - h).all()
    assert (B[:, 2:].astype(np.float64) >= c + h).all()
    # within a few float32 ulps of the exact square
    up = np.nextafter(B[:, :2], np.float32(np.inf)).astype(np.float64)
    assert (up - (c - h) <= 4 * np.spacing(np.abs(c - h).astype(np.float32)) + 1e-30).all()


@pytest.mark.parametrize("K", [1, 3, 16, 61])
def test_filter_refine_equals_definition(K):
    mix = datagen.mixture_spec(20, 9)
    P = datagen.points_mixture(4000, mix, 0.2, 21)
    Q = datagen.points_mixture(3500, mix, 0.2, 22)
    eps = 0.01
    want = oracle.distance_brute(P, Q, eps)
    got = oracle.distance_filter_refine(P, Q, eps, K)
    assert np.array_equal(got, want) and len(want) > 1000


@pytest.mark.parametrize("eps", [1e-3, 0.0371, 0.25])
def test_filter_refine_on_the_boundary(eps):
    P, Q = datagen.near_ring(3000, eps, 31)
    want = oracle.distance_brute(P, Q, eps)
    got = oracle.distance_filter_refine(P, Q, eps, 8)
    assert np.array_equal(got, want)
    # the ring straddles the boundary: some own partners in, some out
    own = {i for i, j in _set(want) if i == j}
    assert 0 < len(own) < len(P)


def test_filter_is_a_superset():
    P, Q = datagen.near_ring(2000, 0.01, 41)
    cand = _set(oracle.pbsm(oracle.squares(P, 0.01), oracle.squares(Q, 0.01), 32))
    assert _set(oracle.distance_brute(P, Q, 0.01)) <= cand


def test_refine_drops_the_corners():
    # a square of side eps reaches sqrt(2) eps / 2 along the diagonal; the
    # squares of two points eps apart on a diagonal still touch, the points
    # are farther than eps
    P = np.array([[0, 0]], np.float32)
    Q = np.array([[0.75, 0.75]], np.float32)
    eps = 1.0
    assert len(oracle.pbsm(oracle.squares(P, eps), oracle.squares(Q, eps), 1)) == 1
    assert len(oracle.distance_brute(P, Q, eps)) == 0
    assert len(oracle.distance_filter_refine(P, Q, eps, 1)) == 0


def test_empty_inputs():
    E = np.zeros((0, 2), np.float32)
    P = datagen.points_uniform(10, 1)
    assert len(oracle.distance_brute(E, P, 0.5)) == 0
    assert len(oracle.distance_filter_refine(P, E, 0.5, 4)) == 0
