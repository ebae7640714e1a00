"""Pins of the GBDA oracle (class-based duplicate avoidance: per tile the 9
class-class joins that can hold a pair whose reference point is in the tile,
Algorithm 1 on each, no duplicate test): the pairs equal the definition's,
each reported once, on adversarial layouts, grids and domains."""
import numpy as np
import pytest

import oracle
from paper_1908_11740_amd import datagen
from test_oracle import adversarial


def _check(R, S, K, domain=None):
    g = oracle.gbda(R, S, K, domain)
    ref = oracle.bruteforce(R, S)
    # no pair twice (no duplicate test, so a wrong class rule would show here)
    assert len(np.unique(g, axis=0)) == len(g)
    assert np.array_equal(g[np.lexsort((g[:, 1], g[:, 0]))] if len(g) else g, ref)
    return len(ref)


@pytest.mark.parametrize("seed", range(40))
def test_gbda_equals_definition_adversarial(seed):
    rng = np.random.default_rng(900 + seed)
    K = int(rng.choice([1, 2, 3, 5, 7, 16, 64]))
    A = adversarial(int(rng.integers(1, 500)), 7 * seed, K)
    B = adversarial(int(rng.integers(1, 500)), 7 * seed + 1, K)
    _check(A, B, K)


@pytest.mark.parametrize("K", [1, 4, 37, 128])
def test_gbda_small_case_and_replication(K):
    R, S, _ = datagen.small_case()
    assert _check(R, S, K) > 300
    # large rectangles: many entries of classes B, C and D
    big_R = datagen.uniform(2000, 0.3, 11)
    big_S = datagen.uniform(2000, 0.3, 12)
    _check(big_R, big_S, K)


def test_gbda_domain():
    R, S, _ = datagen.small_case()
    _check(R, S, 9, (0.25, 0.25, 0.75, 0.75))
    _check(R, S, 9, (-1.0, -1.0, 2.0, 2.0))
