"""Pins for the CPU oracle of the join (CPU only).

The oracle's three modes are checked against facts fixed by the definition
of the spatial intersection join (Sec. 1: r and s share at least one point)
and by elementary geometry, never against themselves:

* hand-derived pair sets on small layouts (touching edges and corners,
  containment, zero-area rectangles, x-only and y-only overlaps);
* closed-form pair counts on exact lattices of squares;
* special cases (identical rectangles, disjoint halves, a whole-domain
  rectangle);
* the expected pair count of uniform inputs, within Poisson bounds;
* invariants: Algorithm 1 and PBSM at any grid size return the brute-force
  set, with no duplicates; swapping R and S swaps the pairs;
* partition membership equals exact rational tile membership.
"""
from fractions import Fraction

import numpy as np
import pytest

import oracle
from paper_1908_11740_amd import datagen

MODES = {
    "bruteforce": oracle.bruteforce,
    "sweep": oracle.sweep,
    "pbsm_k1": lambda R, S: oracle.pbsm(R, S, 1),
    "pbsm_k3": lambda R, S: oracle.pbsm(R, S, 3),
    "pbsm_k8": lambda R, S: oracle.pbsm(R, S, 8),
    "pbsm_k64": lambda R, S: oracle.pbsm(R, S, 64),
}


def rects(rows):
    return np.asarray(rows, dtype=np.float32).reshape(-1, 4)


def as_set(p):
    return {(int(a), int(b)) for a, b in p}


# --------------------------------------------------------------------------
# Hand-derived layouts
# --------------------------------------------------------------------------
# Coordinates are multiples of 1/8, exact in float32.
#   R0 = [0.125,0.375]x[0.125,0.375]
#   R1 = [0.5,0.875]x[0.5,0.625]       (wide, spans several tiles of a 3x3 grid)
#   R2 = [0.25,0.25]x[0.75,0.75]       (a point)
#   R3 = [0.0,1.0]x[0.875,0.875]       (a horizontal segment across the domain)
#   S0 = [0.375,0.5]x[0.375,0.5]       touches R0 at its corner (0.375,0.375)
#                                      and R1 at its corner (0.5,0.5)
#   S1 = [0.625,0.75]x[0.0,0.125]      x inside R1's x-range, y below R1: no pair
#   S2 = [0.25,0.25]x[0.5,1.0]         vertical segment through R2's point and R3
#   S3 = [0.6,0.7]x[0.55,0.6]          strictly inside R1
#   S4 = [0.9,1.0]x[0.5,0.625]         same y-range as R1, x beyond R1.x_u: no pair
# Expected pairs (derived by hand from the closed definition):
#   (0,0) corner touch, (1,0) corner touch, (1,3) containment,
#   (2,2) point on segment, (3,2) segment crossing at (0.25,0.875).
HAND_R = rects([[0.125, 0.125, 0.375, 0.375],
                [0.5, 0.5, 0.875, 0.625],
                [0.25, 0.75, 0.25, 0.75],
                [0.0, 0.875, 1.0, 0.875]])
HAND_S = rects([[0.375, 0.375, 0.5, 0.5],
                [0.625, 0.0, 0.75, 0.125],
                [0.25, 0.5, 0.25, 1.0],
                [0.6, 0.55, 0.7, 0.6],
                [0.9, 0.5, 1.0, 0.625]])
HAND_J = {(0, 0), (1, 0), (1, 3), (2, 2), (3, 2)}


@pytest.mark.parametrize("mode", sorted(MODES))
def test_hand_layout(mode):
    assert as_set(MODES[mode](HAND_R, HAND_S)) == HAND_J


@pytest.mark.parametrize("mode", sorted(MODES))
def test_x_only_and_y_only_overlaps_are_not_pairs(mode):
    # Same x-range, disjoint y-ranges: the y-test must reject.
    R = rects([[0.1, 0.1, 0.9, 0.3]])
    S = rects([[0.1, 0.5, 0.9, 0.7]])
    assert len(MODES[mode](R, S)) == 0
    # Same y-range, disjoint x-ranges (forward scan must stop / x-test reject).
    R = rects([[0.1, 0.1, 0.3, 0.9]])
    S = rects([[0.5, 0.1, 0.7, 0.9]])
    assert len(MODES[mode](R, S)) == 0
    # Separated by one float32 ulp: not touching, so no pair.
    a = np.float32(0.5)
    b = np.nextafter(a, np.float32(1))
    R = rects([[0.1, 0.1, a, 0.9]])
    S = rects([[b, 0.1, 0.9, 0.9]])
    assert len(MODES[mode](R, S)) == 0
    S = rects([[a, 0.1, 0.9, 0.9]])
    assert as_set(MODES[mode](R, S)) == {(0, 0)}


# --------------------------------------------------------------------------
# Closed forms on lattices
# --------------------------------------------------------------------------
def lattice(a, shift=0.0):
    """a x a unit squares scaled by 1/a (a a power of two: exact in float32)."""
    i, j = np.meshgrid(np.arange(a), np.arange(a), indexing="ij")
    x0 = (i.ravel() + shift) / a
    y0 = (j.ravel() + shift) / a
    return rects(np.stack([x0, y0, x0 + 1.0 / a, y0 + 1.0 / a], 1))


@pytest.mark.parametrize("mode", sorted(MODES))
@pytest.mark.parametrize("a", [1, 2, 8, 16])
def test_lattice_touching_counts(mode, a):
    # Each square meets, along x, itself and the squares sharing an edge:
    # 3a - 2 ordered index pairs per axis, hence (3a - 2)^2 pairs in 2-D.
    L = lattice(a)
    got = MODES[mode](L, L)
    assert len(got) == (3 * a - 2) ** 2


@pytest.mark.parametrize("mode", sorted(MODES))
@pytest.mark.parametrize("a", [2, 8, 16])
def test_lattice_half_shift_counts(mode, a):
    # S_i = [(i+1/2)/a, (i+3/2)/a] meets R_k = [k/a, (k+1)/a] iff k in {i, i+1}
    # (and k < a): 2a - 1 pairs per axis.
    R = lattice(a)
    S = lattice(a, shift=0.5)
    assert len(MODES[mode](R, S)) == (2 * a - 1) ** 2


# --------------------------------------------------------------------------
# Special cases
# --------------------------------------------------------------------------
@pytest.mark.parametrize("mode", sorted(MODES))
def test_identical_rectangles(mode):
    R = rects([[0.3, 0.3, 0.31, 0.32]] * 7)
    S = rects([[0.3, 0.3, 0.31, 0.32]] * 5)
    got = MODES[mode](R, S)
    assert len(got) == 35
    assert as_set(got) == {(i, j) for i in range(7) for j in range(5)}


@pytest.mark.parametrize("mode", sorted(MODES))
def test_disjoint_halves(mode):
    rng = np.random.default_rng(5)
    R = datagen.uniform(300, 0.05, 1) * np.float32(0.35)   # inside [0,0.4)^2
    S = datagen.uniform(300, 0.05, 2) * np.float32(0.35) + np.float32(0.6)
    assert len(MODES[mode](R, S)) == 0
    del rng


@pytest.mark.parametrize("mode", sorted(MODES))
def test_whole_domain_rectangle_pairs_with_everything(mode):
    S = datagen.uniform(500, 0.01, 3)
    R = rects([[0.0, 0.0, 1.0, 1.0]])
    assert as_set(MODES[mode](R, S)) == {(0, j) for j in range(500)}


@pytest.mark.parametrize("mode", sorted(MODES))
def test_empty_inputs(mode):
    S = datagen.uniform(10, 0.01, 3)
    E = np.zeros((0, 4), np.float32)
    assert len(MODES[mode](E, S)) == 0
    assert len(MODES[mode](S, E)) == 0
    assert len(MODES[mode](E, E)) == 0


# --------------------------------------------------------------------------
# Expected magnitude on the uniform workloads
# --------------------------------------------------------------------------
def test_small_case_expected_count():
    # x-projections of uniform rectangles overlap with probability
    # E[w_r + w_s] = 0.002 (extents U[0,0.002]); same for y; so
    # E|J| = n m 0.002^2 = 400, Poisson sd 20.
    R, S, K = datagen.small_case()
    n = len(oracle.pbsm(R, S, K))
    assert abs(n - 400) < 4 * 20


def test_uniform_1m_expected_count():
    # E|J| = 1e12 * (2e-4)^2 = 40,000, Poisson sd 200.
    R, S = datagen.uniform_1m()
    n = len(oracle.pbsm(R, S, 1024))
    assert abs(n - 40_000) < 4 * 200


# --------------------------------------------------------------------------
# Invariants: every mode, every grid gives the brute-force set once
# --------------------------------------------------------------------------
def adversarial(n, seed, K):
    """Rectangles snapped to cell boundaries of a K-grid, +-1 ulp, zero extents,
    coordinates outside [0,1), duplicates, and signed zeros: lower corners at
    -0.0 or +0.0 (kind 5) and upper corners at -0.0 or +0.0 (kind 6), which
    compare equal but have different bit patterns (the GPU's sort keys
    canonicalise -0.0 to +0.0)."""
    rng = np.random.default_rng(seed)
    kind = rng.integers(0, 7, n)
    x = rng.random((n, 2)).astype(np.float32)
    grid = (rng.integers(-1, K + 2, (n, 2)) / K).astype(np.float32)
    x = np.where(kind[:, None] == 1, grid, x)
    ulp = np.where(rng.random((n, 2)) < 0.5, np.float32(-1), np.float32(1))
    x = np.where(kind[:, None] == 2, np.nextafter(grid, grid + ulp), x)
    zeros = np.where(rng.random((n, 2)) < 0.5, np.float32(-0.0), np.float32(0.0))
    x = np.where(kind[:, None] == 5, zeros, x)
    ext = (rng.random((n, 2)) * rng.choice([0.0, 1.0 / K, 2.5 / K, 0.3], n)[:, None]).astype(np.float32)
    ext = np.where(kind[:, None] == 3, np.float32(0), ext)
    ext = np.where(kind[:, None] == 4, (rng.integers(0, 3, (n, 2)) / K).astype(np.float32), ext)
    lo = x
    hi = (lo + ext).astype(np.float32)
    # kind 6: the rectangle ends at a signed zero
    lo = np.where(kind[:, None] == 6, (-ext).astype(np.float32), lo)
    hi = np.where(kind[:, None] == 6, zeros, hi)
    out = np.stack([lo[:, 0], lo[:, 1], hi[:, 0], hi[:, 1]], 1).astype(np.float32)
    dup = rng.random(n) < 0.05
    if dup.any() and n > 1:
        out[dup] = out[rng.integers(0, n, dup.sum())]
    return out


def test_adversarial_inputs_hold_signed_zeros():
    A = adversarial(2000, 7, 16)
    z = A == 0
    assert (z & np.signbit(A)).any() and (z & ~np.signbit(A)).any()
    assert (A[:, 0] <= A[:, 2]).all() and (A[:, 1] <= A[:, 3]).all()


@pytest.mark.parametrize("seed", range(40))
def test_modes_agree_with_bruteforce_adversarial(seed):
    rng = np.random.default_rng(1000 + seed)
    K = int(rng.choice([1, 2, 3, 5, 7, 16, 64]))
    nR, nS = int(rng.integers(0, 250)), int(rng.integers(0, 250))
    R = adversarial(nR, 2 * seed, K)
    S = adversarial(nS, 2 * seed + 1, K)
    ref = oracle.bruteforce(R, S)
    assert np.array_equal(oracle.sweep(R, S), ref)
    for k in sorted({K, 1, 2, 3, 7, 13, 64}):
        got = oracle.pbsm(R, S, k)
        assert np.array_equal(got, ref), f"K={k}"


@pytest.mark.parametrize("K", [1, 2, 3, 7, 64, 200])
def test_pbsm_small_case_every_grid(K):
    R, S, _ = datagen.small_case()
    ref = oracle.bruteforce(R, S)
    got = oracle.pbsm(R, S, K)
    assert np.array_equal(got, ref)
    # sorted, strictly increasing: no duplicates
    key = got[:, 0].astype(np.int64) * len(S) + got[:, 1]
    assert np.all(np.diff(key) > 0)


def test_pbsm_threads_and_domain():
    R, S, K = datagen.small_case()
    ref = oracle.bruteforce(R, S)
    for th in (1, 2, 5):
        assert np.array_equal(oracle.pbsm(R, S, K, threads=th), ref)
    # A caller domain that is larger than the data, and one that cuts it.
    for dom in ([-1.0, -1.0, 2.0, 2.0], [0.25, 0.25, 0.75, 0.75]):
        assert np.array_equal(oracle.pbsm(R, S, 37, domain=dom), ref)


def test_swap_symmetry():
    R = datagen.uniform(3000, 0.01, 11)
    S = datagen.uniform(2000, 0.01, 12)
    a = oracle.pbsm(R, S, 16)
    b = oracle.pbsm(S, R, 16)[:, ::-1]
    b = b[np.lexsort((b[:, 1], b[:, 0]))]
    assert np.array_equal(a, b)


def test_mixture_case_every_grid():
    mix = datagen.mixture_spec(5, 9)
    R = datagen.mixture(2000, mix, 0.2, 5e-3, 1.0, 10)
    S = datagen.mixture(2500, mix, 0.2, 5e-3, 1.0, 11)
    ref = oracle.bruteforce(R, S)
    assert len(ref) > 1000
    for k in (1, 4, 33, 128, 1024):
        assert np.array_equal(oracle.pbsm(R, S, k), ref)


# --------------------------------------------------------------------------
# Partition membership (Sec. 2.2: a tile gets every rectangle intersecting it)
# --------------------------------------------------------------------------
@pytest.mark.parametrize("K", [1, 2, 4, 16])
def test_partition_membership_exact(K):
    # With K a power of two, cell(v) = floor(v*K) is exact; tiles are the
    # half-open [t/K, (t+1)/K) with the outer tiles extended to infinity.
    A = adversarial(150, 77 + K, K)
    off, ids = oracle.partition_ids(A, K)
    assert off[-1] == len(ids)

    def covers(lo, hi, t):
        lo, hi = Fraction(float(lo)), Fraction(float(hi))
        left = Fraction(t, K) if t > 0 else None
        right = Fraction(t + 1, K) if t < K - 1 else None
        return (right is None or lo < right) and (left is None or hi >= left)

    for ty in range(K):
        for tx in range(K):
            T = ty * K + tx
            want = sorted(i for i in range(len(A))
                          if covers(A[i, 0], A[i, 2], tx) and covers(A[i, 1], A[i, 3], ty))
            assert sorted(ids[off[T]:off[T + 1]].tolist()) == want


# ----------------------------------------------------------------------------
# Hand-derived golden fixture (tests/golden/two_by_two.txt)
# ----------------------------------------------------------------------------
def test_golden_two_by_two():
    from golden.load import load
    R, S, pairs, tiles = load("two_by_two.txt")
    assert np.array_equal(oracle.bruteforce(R, S), pairs)
    assert np.array_equal(oracle.sweep(R, S), pairs)
    for K in (1, 2, 3, 4, 7, 64):
        assert np.array_equal(oracle.pbsm(R, S, K), pairs), K
    # at K = 2 each pair is reported by exactly the tile listed in the fixture:
    # joining R with only the rectangles of one tile's membership reproduces it
    offR, idR = oracle.partition_ids(R, 2)
    offS, idS = oracle.partition_ids(S, 2)
    for (r, s), (tx, ty) in zip(pairs, tiles):
        t = ty * 2 + tx
        assert r in idR[offR[t]:offR[t + 1]] and s in idS[offS[t]:offS[t + 1]]
