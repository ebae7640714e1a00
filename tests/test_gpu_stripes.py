"""GPU parity of one-dimensional partitioning (SJ_STRIPES: k vertical
stripes swept along y, Sec. 3.1; duplicate test on the reference point's x,
Sec. 3.2): the pair set equals the oracle's on every workload, stripe count
and schedule; stripe membership equals the oracle's x-cell ranges."""
import sys

import numpy as np
import pytest

import oracle
from oracle import picker as op
from paper_1908_11740_amd import datagen

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

from paper_1908_11740_amd import sj  # noqa: E402
from gpu_util import gpu_join, to_dev  # noqa: E402

STRIPES = {"tuned": dict(flags=sj.SJ_STRIPES), "plain": dict(flags=sj.SJ_STRIPES | sj.SJ_PLAIN),
           "twopass": dict(flags=sj.SJ_STRIPES | sj.SJ_TWO_PASS),
           "tau1": dict(flags=sj.SJ_STRIPES, split_tau=1)}


def say(*a):
    print(*a, file=sys.stderr, flush=True)


@pytest.fixture(scope="module")
def small():
    R, S, _ = datagen.small_case()
    return R, S, oracle.bruteforce(R, S)


@pytest.mark.parametrize("K", [1, 2, 7, 64, 100, 500, 4096])
@pytest.mark.parametrize("sched", sorted(STRIPES))
def test_small_case_stripes(small, K, sched):
    R, S, ref = small
    say("stripes small K", K, sched)
    assert np.array_equal(gpu_join(R, S, K, **STRIPES[sched]), ref)


def test_stripes_count_golden_and_adversarial(small):
    R, S, ref = small
    assert gpu_join(R, S, 100, count=True, flags=sj.SJ_STRIPES) == len(ref)
    from golden.load import load
    Rg, Sg, pairs, _ = load("two_by_two.txt")
    for K in (1, 2, 3):
        assert np.array_equal(gpu_join(Rg, Sg, K, flags=sj.SJ_STRIPES), pairs)
    from test_oracle import adversarial
    for seed in range(6):
        rng = np.random.default_rng(700 + seed)
        K = int(rng.choice([1, 2, 3, 5, 7, 16, 64]))
        A = adversarial(int(rng.integers(1, 400)), 5 * seed, K)
        B = adversarial(int(rng.integers(1, 400)), 5 * seed + 1, K)
        assert np.array_equal(gpu_join(A, B, K, flags=sj.SJ_STRIPES), oracle.bruteforce(A, B))


@pytest.mark.parametrize("K", [1, 16, 300])
def test_stripe_membership_matches_oracle(K):
    A = datagen.uniform(20_000, 0.02, 33)
    P = sj.partition(to_dev(A), K, flags=sj.SJ_STRIPES)
    off, ids = P.download()
    assert len(off) == K + 1
    ro, rids = oracle.partition_ids(A, K)  # the oracle's K x K tiles
    for tx in range(K):
        want = set()
        for ty in range(K):
            t = ty * K + tx
            want.update(rids[ro[t]:ro[t + 1]].tolist())
        got = ids[off[tx]:off[tx + 1]]
        assert len(got) == len(set(got.tolist()))
        assert set(got.tolist()) == want, tx


def test_uniform_1m_and_rule():
    R, S = datagen.uniform_1m()
    ref = oracle.pbsm(R, S, 1024)
    k, tau, info = sj.choose_grid(to_dev(R), to_dev(S), flags=sj.SJ_STRIPES)
    assert k == op.rule_k(op.mean_x_extent(R, S)) == 1000 and info["used_learned"] == 0
    assert info["mean_x_extent"] == pytest.approx(op.mean_x_extent(R, S), rel=1e-12)
    for K in (k, 4096):
        assert np.array_equal(gpu_join(R, S, K, flags=sj.SJ_STRIPES), ref), K


def test_skewed_10m_stripes():
    R, S = datagen.skewed_10m()
    K = op.rule_k(op.mean_x_extent(R, S))
    ref = oracle.pbsm(R, S, 1213)
    say("skewed 10M stripes K", K)
    got = gpu_join(R, S, K, flags=sj.SJ_STRIPES)
    assert np.array_equal(got, ref)


def test_stripes_and_square_grids_do_not_mix():
    A = to_dev(datagen.uniform(100, 0.01, 1))
    P1 = sj.partition(A, 16, flags=sj.SJ_STRIPES)
    P2 = sj.partition(A, 16)
    with pytest.raises(sj.SjError) as ei:
        sj.join_count(P1, P2)
    assert ei.value.status == sj.SJ_ERR_GRID_MISMATCH


def test_batch_with_stripes():
    js = [datagen.batch_instance(j, 0.005)[:2] for j in range(8)]
    refs = [oracle.pbsm(R, S, 64) for R, S in js]
    grids = [(int(50 + 97 * j), 0) for j in range(8)]
    dev = [(to_dev(R), to_dev(S)) for R, S in js]
    b = sj.Batch(dev, grids=grids, capacities=[len(r) + 1 for r in refs], flags=sj.SJ_STRIPES)
    st, n = b.run()
    assert st == sj.SJ_OK
    for j, ref in enumerate(refs):
        from gpu_util import sort_pairs
        assert np.array_equal(sort_pairs(b.pairs(j, n[j]).cpu().numpy()), ref), j
    b.free()
