"""GPU parity of the many-join batch (one recorded graph for all joins): every
join's pair set equals the oracle's, in pair and count-only mode, across
replays, after its inputs change in place, and with too-small slices."""
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


def _joins(n=24, scale=0.01):
    js = [datagen.batch_instance(j, scale)[:2] for j in range(n)]
    # edge cases: an empty side, single rectangles, a dense clump
    u = datagen.uniform(3000, 0.01, 77)
    js.append((u, u[:0]))
    js.append((u[:1], u[:1]))
    clump = (datagen.uniform(4000, 0.001, 78) * 0.01).astype(np.float32)
    js.append((clump, clump[::-1].copy()))
    return js


@pytest.fixture(scope="module")
def joins():
    js = _joins()
    refs = [oracle.pbsm(R, S, 64) for R, S in js]
    return js, refs


def _check_batch(b, js, refs, status, n):
    assert status == sj.SJ_OK
    for j, (ref, nj) in enumerate(zip(refs, n)):
        assert nj == len(ref), j
        got = sort_pairs(b.pairs(j, nj).cpu().numpy())
        assert np.array_equal(got, ref), j


def test_batch_pairs_match_oracle_and_replays(joins):
    js, refs = joins
    say("batch of", len(js))
    dev = [(to_dev(R), to_dev(S)) for R, S in js]
    caps = [len(r) + 5 for r in refs]
    b = sj.Batch(dev, capacities=caps)
    k, tau = b.grids()
    assert np.all(k >= 1)
    # chosen grids keep K^2 <= (nR + nS) / 4
    for (R, S), kj in zip(js, k):
        assert kj <= max(1, int(np.floor(np.sqrt((len(R) + len(S)) / 4)))), (len(R), len(S), kj)
    for rep in range(3):
        st, n = b.run()
        _check_batch(b, js, refs, st, n)
    # the same kernels launched one by one, and the work statistics
    b.out.fill_(-1)
    st, n = b.run(eager=True)
    _check_batch(b, js, refs, st, n)
    stats = b.stats()
    assert stats["n_pairs"] == sum(len(r) for r in refs)
    assert stats["pairs_small"] + stats["pairs_medium"] + stats["pairs_dense"] == stats["n_pairs"]
    assert stats["small_units"] > 0 and stats["small_entries"] > 0
    b.free()


def test_batch_count_only(joins):
    js, refs = joins
    b = sj.Batch([(to_dev(R), to_dev(S)) for R, S in js])
    st, n = b.run()
    assert st == sj.SJ_OK
    assert list(n) == [len(r) for r in refs]
    b.free()


def test_batch_fixed_grids_and_schedules(joins):
    js, refs = joins
    rng = np.random.default_rng(3)
    grids = [(int(rng.choice([1, 7, 64, 300, 2000])), int(rng.choice([0, 1, 64, sj.INT32_MAX])))
             for _ in js]
    b = sj.Batch([(to_dev(R), to_dev(S)) for R, S in js], grids=grids,
                 capacities=[len(r) for r in refs])
    st, n = b.run()
    _check_batch(b, js, refs, st, n)
    assert [int(x) for x in b.grids()[0]] == [g[0] for g in grids]
    b.free()


def test_batch_inputs_changed_in_place_regrow():
    """A replay reads the inputs again: new, much denser data in the same
    buffers overflows the planned capacities; the batch must regrow and still
    return the oracle's pairs."""
    js = _joins(8)
    dev = [(to_dev(R), to_dev(S)) for R, S in js]
    big = 200_000
    caps = [big] * len(js)
    b = sj.Batch(dev, capacities=caps)
    st, n = b.run()
    assert st == sj.SJ_OK
    new = []
    for j, (Rd, Sd) in enumerate(dev):
        # same sizes, every rectangle now covers many more tiles
        R2 = datagen.uniform(Rd.shape[0], 0.01, 900 + j) if Rd.shape[0] else js[j][0]
        S2 = datagen.uniform(Sd.shape[0], 0.01, 950 + j) if Sd.shape[0] else js[j][1]
        Rd.copy_(torch.from_numpy(R2))
        Sd.copy_(torch.from_numpy(S2))
        new.append((R2, S2))
    refs = [oracle.pbsm(R, S, 16) for R, S in new]
    # the replay that outgrows the buffers (regrowth), then replays of the
    # graph recorded after it, which must not use the freed buffers
    for rep in range(3):
        say("regrow replay", rep)
        st, n = b.run()
        assert list(n) == [len(r) for r in refs]
        if st == sj.SJ_OK:
            _check_batch(b, new, refs, st, n)
        else:
            assert st == sj.SJ_ERR_CAPACITY and any(len(r) > big for r in refs)
    b.free()


def test_batch_capacity_reports_exact_counts(joins):
    js, refs = joins
    caps = [max(len(r) // 2, 0) for r in refs]
    b = sj.Batch([(to_dev(R), to_dev(S)) for R, S in js], capacities=caps)
    st, n = b.run()
    assert st == sj.SJ_ERR_CAPACITY
    assert list(n) == [len(r) for r in refs]
    b.free()


def test_empty_batch():
    b = sj.Batch([], capacities=[])
    st, n = b.run()
    assert st == sj.SJ_OK and len(n) == 0
    b.free()


def test_batch_full_size_256_joins_element_by_element():
    """The many-join workload at its real sizes: 256 joins, n per side
    log-uniform in [1e3, 2e6] (1.4e8 rectangles), grids chosen per join.  A
    count-only batch sizes the output slices, then every join's pair list
    equals the oracle's PBSM on the same grid, element by element, and so do
    the counts of a second replay."""
    n = 256
    say("full-size batch: generating", n, "joins")
    host = [datagen.batch_instance(j)[:2] for j in range(n)]
    dev = [(to_dev(R), to_dev(S)) for R, S in host]
    say("count-only batch")
    counting = sj.Batch(dev)
    st, counts = counting.run()
    counting.free()
    assert st == sj.SJ_OK
    b = sj.Batch(dev, capacities=[int(c) for c in counts])
    st, npairs = b.run()
    assert st == sj.SJ_OK and list(npairs) == list(counts)
    ks, _ = b.grids()
    for j, (R, S) in enumerate(host):
        if j % 32 == 0:
            say("full-size batch: oracle join", j, "K", int(ks[j]))
        ref = oracle.pbsm(R, S, int(ks[j]))
        got = sort_pairs(b.pairs(j, npairs[j]).cpu().numpy())
        assert np.array_equal(got, ref), j
    st, again = b.run()
    assert st == sj.SJ_OK and list(again) == list(npairs)
    b.free()


def test_batch_with_a_grid_beyond_the_batched_scans(joins):
    """A join on a 4096 x 4096 grid has more level-2 counters than the
    batched partition scans take: the batch then runs every join's
    partitions and classification on its own stream, with the same pairs."""
    js, refs = joins
    grids = [(64, 0)] * len(js)
    grids[3] = (4096, 0)
    say("batch with a 4096 grid")
    b = sj.Batch([(to_dev(R), to_dev(S)) for R, S in js], grids=grids,
                 capacities=[len(r) for r in refs])
    for rep in range(2):
        st, n = b.run()
        _check_batch(b, js, refs, st, n)
    b.free()
