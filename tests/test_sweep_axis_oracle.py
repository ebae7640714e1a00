"""Pins of the sweeping-axis model oracle (Sec. 3.3, Eq. (2)) by the
pairwise form of the histogram product, hand layouts, the transpose
symmetry, the sampling and division rules, and by the true candidate counts
of a plane sweep along each axis."""
import numpy as np
import pytest

from oracle import sweep_axis as sa
from paper_1908_11740_amd import datagen


def _pairwise(Rb, Sb):
    """sum over (r, s) of the number of divisions both ranges contain."""
    tot = 0
    for a, b in zip(*Rb):
        for c, d in zip(*Sb):
            tot += max(0, min(b, d) - max(a, c) + 1)
    return tot


@pytest.mark.parametrize("seed", range(5))
def test_histogram_product_equals_pairwise_overlaps(seed):
    rng = np.random.default_rng(seed)
    k = int(rng.integers(1, 60))
    def ranges(n):
        a = rng.integers(0, k, n)
        b = np.minimum(a + rng.integers(0, k, n), k - 1)
        return a, b
    Rb, Sb = ranges(int(rng.integers(1, 30))), ranges(int(rng.integers(1, 30)))
    HR, HS = sa.histogram(*Rb, k), sa.histogram(*Sb, k)
    assert int((HR * HS).sum()) == _pairwise(Rb, Sb)


def _rect(x0, y0, x1, y1):
    return [x0, y0, x1, y1]


def test_hand_layout_horizontal_strips_choose_y():
    # K = 1, unit domain.  Three R and two S strips spanning x, thin in y.
    R = np.array([_rect(0.0, 0.1 * i, 0.5, 0.1 * i + 0.05) for i in range(3)], np.float32)
    S = np.array([_rect(0.25, 0.5 + 0.2 * i, 0.75, 0.55 + 0.2 * i) for i in range(2)], np.float32)
    k, Ix, Iy, axis = sa.tile_model(R, S, 0, 0, 1)
    # mean extent (w + h) / 2 = (3 * 0.275 + 2 * 0.275) / 5 = 0.275 -> k = 3
    assert k == 3
    # x: R covers divisions 0..1, S covers 0..2 -> 2 shared each, 3 x 2 pairs
    assert Ix == 3 * 2 * 2
    # y: R in division 0 (y < 1/3); S at y 0.5-0.55 (div 1), 0.7-0.75 (div 2)
    assert Iy == 0
    assert axis == 1


def test_transpose_swaps_the_estimates():
    mix = datagen.mixture_spec(5, 3)
    R = datagen.anisotropic(3000, mix, 0.2, 2e-2, 16.0, 0.5, 4)
    S = datagen.anisotropic(2500, mix, 0.2, 2e-2, 16.0, 0.5, 5)
    T = lambda A: np.ascontiguousarray(A[:, [1, 0, 3, 2]])
    a = sa.all_tiles(R, S, 4)
    b = sa.all_tiles(T(R), T(S), 4)
    assert a.keys() == {(y, x) for x, y in b.keys()}
    nonzero = 0
    for (tx, ty), (k, Ix, Iy, ax, nr, ns) in a.items():
        k2, Ix2, Iy2, ax2, nr2, ns2 = b[(ty, tx)]
        assert (k, Ix, Iy, nr, ns) == (k2, Iy2, Ix2, nr2, ns2)
        if Ix != Iy:
            assert ax != ax2
            nonzero += 1
    assert nonzero >= 4


def test_sampling_and_empty_samples():
    ids = np.arange(1, 450)
    assert sa.tile_samples(ids).tolist() == [100, 200, 300, 400]
    R = np.array([_rect(0, 0, 1, 0.1)], np.float32)
    assert sa.tile_model(R, R[:0], 0, 0, 1) == (0, 0, 0, 0)


def test_division_count_rule():
    # extents 0.1 of a tile (K = 10 on the unit square: w = h = 0.01) -> k = 10
    R = np.array([_rect(0.0, 0.0, 0.01, 0.01)] * 3, np.float32)
    k, *_ = sa.tile_model(R, R, 0, 0, 10)
    assert k == 10
    # points -> k = 1000; rectangles larger than the tile -> k = 1
    P = np.array([_rect(0.5, 0.5, 0.5, 0.5)], np.float32)
    assert sa.tile_model(P, P, 0, 0, 1)[0] == 1000
    B = np.array([_rect(0, 0, 1, 1)], np.float32)
    assert sa.tile_model(B, B, 0, 0, 1)[0] == 1
    # a tie sweeps along x
    assert sa.tile_model(B, B, 0, 0, 1)[3] == 0


def test_division_count_uses_the_plain_mean_extent():
    """k = floor(tile extent / mean (w + h) / 2) over the sample, with no
    clipping of large extents: ten rectangles of 1/64 and one of 4 tiles
    (K = 1) have mean extent 4.15625 / 11, so k = floor(11 / 4.15625) = 2
    (clipping the large one at 2 tiles would give 5).  One extent beyond any
    fixed-point range still gives k = 1."""
    small = [_rect(0.1 * i, 0.1 * i, 0.1 * i + 1 / 64, 0.1 * i + 1 / 64) for i in range(10)]
    big = [_rect(0.0, 0.0, 4.0, 4.0)]
    A = np.array(small + big, np.float32)
    assert sa.tile_model(A[:5], A[5:], 0, 0, 1)[0] == 2
    H = np.array([_rect(-1e30, 0.0, 1e30, 0.5), _rect(0.2, 0.2, 0.2, 0.2)], np.float32)
    assert sa.tile_model(H[:1], H[1:], 0, 0, 1)[0] == 1


def test_divisions_are_relative_to_the_tile():
    # tile column 3 of K = 4 on [0, 8): cell units u = v / 2, divisions of u - 3
    lo, hi = sa.buckets(np.float32([6.0, 7.0]), np.float32([6.9, 7.99]),
                        *sa.grid_scales(4, (0, 0, 8, 8))[::2], 3, 10)
    assert lo.tolist() == [0, 5] and hi.tolist() == [4, 9]


def _true_overlaps(A, B, lo, hi):
    """pairs of A x B whose [lo, hi] projections meet (closed)."""
    return int(((A[:, None, lo] <= B[None, :, hi]) & (B[None, :, lo] <= A[:, None, hi])).sum())


def test_model_picks_the_axis_with_fewer_candidates():
    # Sec. 4.2: the model chose the better axis for every query; here: for
    # tiles with a real sample, its choice has fewer true candidates (pairs
    # overlapping along the sweep axis) in at least 90% of the tiles
    mix = datagen.mixture_spec(8, 13)
    R = datagen.anisotropic(200_000, mix, 0.1, 5e-3, 25.0, 0.5, 14)
    S = datagen.anisotropic(200_000, mix, 0.1, 5e-3, 25.0, 0.5, 15)
    import oracle
    K = 16
    offR, idsR = oracle.partition_ids(R, K)
    offS, idsS = oracle.partition_ids(S, K)
    model = sa.all_tiles(R, S, K)
    good = total = 0
    for (tx, ty), (k, Ix, Iy, ax, nr, ns) in model.items():
        if min(Ix, Iy) == 0 or nr < 2000 or ns < 2000:
            continue
        t = ty * K + tx
        A = R[idsR[offR[t]:offR[t + 1]]]
        B = S[idsS[offS[t]:offS[t + 1]]]
        cx, cy = _true_overlaps(A, B, 0, 2), _true_overlaps(A, B, 1, 3)
        total += 1
        good += (cy < cx) == (ax == 1)
    assert total >= 20 and good >= 0.9 * total
