"""Host logic of the picker's corpus tooling (no GPU): the candidate grids,
the capped rule the small-input corpus and the evaluations use, and the
instance recipes (deterministic, within their stated ranges, seeds that do
not collide across the corpora's index ranges)."""
import math

import numpy as np
import pytest

from paper_1908_11740_amd import datagen, picker


def test_k_candidates_are_half_octaves_around_the_rule():
    ks = picker.k_candidates(1000)
    expect = sorted({int(round(1000 * 2.0 ** (j / 2))) for j in range(-6, 7)})
    assert ks == expect
    assert ks[0] == 125 and ks[-1] == 8000


@pytest.mark.parametrize("k_rule,lo", [(10, 8), (10, 2), (9000, 8), (3, 2)])
def test_k_candidates_clamp_to_their_range(k_rule, lo):
    ks = picker.k_candidates(k_rule, lo)
    assert all(lo <= k <= 8192 for k in ks)
    assert ks == sorted(set(ks))


def test_capped_rule_matches_the_library_cap():
    # K^2 <= 8 (nR + nS), as sj_choose_grid applies it to a 2-D grid
    assert picker.capped_rule_k(1000, 1000, 1000) == math.floor(math.sqrt(16000))
    assert picker.capped_rule_k(50, 1000, 1000) == 50
    assert picker.capped_rule_k(1000, 0, 0) == 1
    for n in (1, 7, 1000, 123456):
        k = picker.capped_rule_k(10 ** 6, n, n)
        assert k * k <= 8 * 2 * n < (k + 1) * (k + 1)


def test_small_instances_are_deterministic_and_in_range():
    for i in (0, 1, 899, 900, 1099):
        a, b = datagen.small_instance_spec(i), datagen.small_instance_spec(i)
        assert a == b
        assert 1e3 <= a.n_r <= 1e6 and 1e3 <= a.n_s <= 1e6
        assert 1 <= a.clusters <= 500 and 0.0 <= a.background <= 0.5
        assert 1e-5 <= a.median <= 1e-3


def test_corpus_seeds_do_not_collide():
    """Training and held-out ranges of the three recipes draw from disjoint
    seeds (picker 0-1999, small 0-1099, batch-like held-out 2100-2299; the
    benchmark batch 0-255 is not a corpus)."""
    picker_seeds = {datagen.picker_instance_spec(i).seed for i in range(0, 2000, 37)}
    small_seeds = {datagen.small_instance_spec(i).seed for i in range(0, 1100, 13)}
    held_batch = {datagen.batch_instance_spec(j).seed for j in range(2100, 2300, 7)}
    assert not (picker_seeds & small_seeds)
    assert not (held_batch & small_seeds) and not (held_batch & picker_seeds)
    assert min(s.seed for s in map(datagen.small_instance_spec, (0,))) == 6000
    assert datagen.batch_instance_spec(2100).seed == 7100 > datagen.small_instance_spec(1099).seed


def test_summary_of_an_evaluation():
    ev = {"t_learned": np.array([1.0, 2.0]), "t_rule": np.array([2.0, 2.0]),
          "t_plain": np.array([4.0, 8.0])}
    s = picker.summary(ev)
    assert s["instances"] == 2
    assert s["geomean_speedup_vs_rule_tuned"] == pytest.approx(math.sqrt(2.0))
    assert s["geomean_speedup_vs_rule_plain"] == pytest.approx(4.0)
    assert s["win_rate_vs_rule_tuned"] == 0.5 and s["win_rate_vs_rule_plain"] == 1.0
