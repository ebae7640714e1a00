"""Pins of the grid-choice oracle (rule, features, picker network) by closed
forms, hand-computed cases and finite differences -- nothing here re-types
the oracle's formulas."""
import numpy as np
import pytest

from oracle import picker as op
from paper_1908_11740_amd import datagen


# ----------------------------------------------------------------------------
# Rule of thumb (Sec. 4.3.1, 4.3.3): tile extent = 10 x mean rectangle extent
# ----------------------------------------------------------------------------
def test_rule_closed_forms():
    # extents U[0, 2e-4]: mean 1e-4 -> tile 1e-3 -> K = 1000
    assert op.rule_k(1e-4) == 1000
    # log-normal extents, median 5e-5, sigma 1: mean = 5e-5 exp(1/2)
    assert op.rule_k(5e-5 * np.exp(0.5)) == 1213
    # extents U[0, 0.002]: mean 1e-3 -> K = 100
    assert op.rule_k(1e-3) == 100
    assert op.rule_k(0.0) == op.K_MAX
    assert op.rule_k(1.0) == 1  # rectangles as large as the domain
    assert op.rule_k(1e-9) == op.K_MAX  # clamped


def test_rule_on_generated_workloads():
    R, S = datagen.uniform_1m(200_000)
    assert op.rule_k(op.mean_extent(R, S)) == 1000
    R, S, _ = datagen.small_case()
    assert op.rule_k(op.mean_extent(R, S)) == 100
    mix = datagen.mixture_spec(200, 300)
    A = datagen.mixture(400_000, mix, 0.2, 5e-5, 1.0, 301)
    e = op.mean_extent(A, A[:0])
    assert abs(e / (5e-5 * np.exp(0.5)) - 1) < 0.01
    assert abs(op.rule_k(e) - 1213) <= 10


def test_one_dimensional_rule_uses_the_x_extents():
    # stripes ten times the mean x-extent (Sec. 4.3.1): only w counts
    R = np.array([[0, 0, 0.2, 0.9]], np.float32)   # w = 0.2, h = 0.9
    S = np.array([[0.5, 0.5, 0.5, 0.6]], np.float32)  # w = 0, h = 0.1
    assert op.mean_x_extent(R, S) == pytest.approx(0.1)
    assert op.rule_k(op.mean_x_extent(R, S)) == 1
    R, S = datagen.uniform_1m(200_000)
    assert op.rule_k(op.mean_x_extent(R, S)) == 1000


def test_mean_extent_hand_case_and_domain_scaling():
    R = np.array([[0, 0, 0.2, 0.1]], np.float32)
    S = np.array([[0.5, 0.5, 0.5, 0.9], [0.1, 0.1, 0.3, 0.1]], np.float32)
    # (w + h) / 2 per rectangle: 0.15, 0.2, 0.1 -> mean 0.15
    assert abs(op.mean_extent(R, S) - 0.15) < 1e-7
    # the same data on a domain twice as wide and tall: extents halve
    assert abs(op.mean_extent(R, S, (0, 0, 2, 2)) - 0.075) < 1e-7


# ----------------------------------------------------------------------------
# Features
# ----------------------------------------------------------------------------
def test_features_of_a_hand_layout():
    n = 250  # sampled: positions 0, 100, 200
    A = np.tile(np.array([[0.505, 0.255, 0.515, 0.265]], np.float32), (n, 1))
    f = op.side_features(A)
    assert f[0] == pytest.approx(np.log2(251))
    assert f[1] == pytest.approx(np.log2(0.01 + 1e-9), abs=1e-5)
    assert f[3] == pytest.approx(np.log2(1e-9), abs=1e-3)  # zero spread
    h = f[5:].reshape(32, 32)
    # centre (0.51, 0.26): cx = floor(16.32) = 16, cy = floor(8.32) = 8
    assert h[8, 16] == pytest.approx(np.log2(1 + 1024))
    assert np.count_nonzero(h) == 1
    assert op.histogram_counts(A)[8 * 32 + 16] == 3


def test_features_scale_with_domain():
    R = datagen.uniform(5000, 0.01, 7)
    f1 = op.features(R, R[:10])
    g = R.astype(np.float64) * 4 + 1  # same layout on the domain [1, 5)^2
    f2 = op.features(g.astype(np.float32), g[:10].astype(np.float32), (1, 1, 5, 5))
    assert np.allclose(f1[:5], f2[:5], atol=1e-4)
    assert np.array_equal(op.histogram_counts(R), op.histogram_counts(g, (1, 1, 5, 5)))


def test_histogram_sums_to_sample_count_and_clamps():
    A = datagen.uniform(12345, 0.1, 3)
    A[::7] += 3.0  # far outside: clamped into the border cells
    c = op.histogram_counts(A)
    assert c.sum() == len(A[::op.PHI])
    assert c.reshape(32, 32)[31, 31] >= 1


def test_empty_side():
    f = op.side_features(np.zeros((0, 4), np.float32))
    assert f[0] == 0.0 and np.all(f[5:] == 0.0)


# ----------------------------------------------------------------------------
# Network
# ----------------------------------------------------------------------------
def _params(d, seed, scale=0.5):
    rng = np.random.default_rng(seed)
    return rng.normal(0, scale, op.param_count(d))


def test_param_count_matches_the_sizes():
    # 2 x 64 network on the 2 x 1029 features: ~136k parameters
    assert op.param_count(2058) == 64 * 2058 + 64 + 64 * 64 + 64 + 2 * 64 + 2 == 136_066


def test_forward_hand_case():
    d = 2
    W1 = np.zeros((64, 2)); b1 = np.zeros(64)
    W1[0] = [1.0, 2.0]; W1[1] = [-1.0, 0.0]; b1[1] = 0.5
    W2 = np.zeros((64, 64)); b2 = np.zeros(64)
    W2[0, 0] = 3.0; W2[0, 1] = 1.0; W2[1, 1] = -4.0
    W3 = np.zeros((2, 64)); b3 = np.array([0.25, -1.0])
    W3[0, 0] = 2.0; W3[1, 1] = 5.0
    P = op.pack(W1, b1, W2, b2, W3, b3)
    x = np.array([[1.0, 0.5]])
    # h1 = relu([1 + 1, -1 + 0.5]) = [2, 0]; h2 = relu([6 + 0, -0]) = [6, 0]
    y, h1, h2 = op.forward(P, x)
    assert h1[0, :2].tolist() == [2.0, 0.0]
    assert h2[0, :2].tolist() == [6.0, 0.0]
    assert y[0].tolist() == [12.25, -1.0]
    # standardisation: mu, sd applied before the first layer
    y2, _, _ = op.forward(P, np.array([[3.0, 2.0]]), mu=[1.0, 1.0], sd=[2.0, 2.0])
    assert y2[0].tolist() == y[0].tolist()


def test_loss_closed_form():
    Y = np.array([[1.0, 2.0], [3.0, 4.0]])
    T = Y - np.array([[1.0, -1.0], [2.0, 0.0]])
    L, dY = op.loss(Y, T)
    assert L == pytest.approx((1 + 1 + 4 + 0) / 4)
    assert np.allclose(dY, np.array([[1.0, -1.0], [2.0, 0.0]]) / 2)


@pytest.mark.parametrize("seed", range(4))
def test_backward_matches_central_differences(seed):
    d, B = 5, 3
    rng = np.random.default_rng(100 + seed)
    P = _params(d, seed)
    X = rng.normal(size=(B, d))
    mu, sd = rng.normal(size=d), rng.uniform(0.5, 2.0, d)
    dY = rng.normal(size=(B, 2))
    g = op.backward(P, X, dY, mu, sd)

    def f(p):
        return float((op.forward(p, X, mu, sd)[0] * dY).sum())

    h = 1e-6
    idx = rng.choice(len(P), 200, replace=False)
    for i in idx:
        e = np.zeros_like(P)
        e[i] = h
        num = (f(P + e) - f(P - e)) / (2 * h)
        assert num == pytest.approx(g[i], rel=1e-5, abs=1e-7), i


def test_backward_of_the_loss_matches_central_differences():
    d, B = 4, 6
    rng = np.random.default_rng(9)
    P = _params(d, 9)
    X = rng.normal(size=(B, d))
    T = rng.normal(size=(B, 2))
    _, dY = op.loss(op.forward(P, X)[0], T)
    g = op.backward(P, X, dY)
    h = 1e-6
    for i in rng.choice(len(P), 100, replace=False):
        e = np.zeros_like(P)
        e[i] = h
        num = (op.loss(op.forward(P + e, X)[0], T)[0] - op.loss(op.forward(P - e, X)[0], T)[0]) / (2 * h)
        assert num == pytest.approx(g[i], rel=1e-5, abs=1e-8)


def test_adam_constant_gradient_closed_form():
    # bias correction makes m_hat = g and v_hat = g^2 for a constant g, so
    # every step moves each parameter by lr * g / (|g| + eps)
    P = np.array([1.0, -2.0, 0.5, 3.0])
    G = np.array([0.3, -4.0, 0.0, 1e-3])
    M = np.zeros(4); V = np.zeros(4)
    lr, eps = 0.01, 1e-8
    for t in range(1, 6):
        P2, M, V = op.adam(P, M, V, G, t, lr=lr, eps=eps)
        assert np.allclose(P2 - P, -lr * G / (np.abs(G) + eps), rtol=1e-9, atol=1e-15)
        P = P2


def test_adam_moments_after_two_steps():
    g1, g2 = 2.0, -1.0
    P, M, V = op.adam(np.array([0.0]), np.zeros(1), np.zeros(1), np.array([g1]), 1)
    P, M, V = op.adam(P, M, V, np.array([g2]), 2)
    assert M[0] == pytest.approx(0.9 * 0.1 * g1 + 0.1 * g2)
    assert V[0] == pytest.approx(0.999 * 0.001 * g1 * g1 + 0.001 * g2 * g2)
