"""GPU parity of the per-tile sweeping-axis model (Sec. 3.3, Eq. (2)): the
model's divisions, estimates and choice equal the oracle's on every tile;
joins whose medium and dense tiles sweep along the chosen axis return the
oracle's pair set on every schedule; the join's counts of model tiles and
y-swept tiles equal the oracle's decisions for the tiles of those classes."""
import sys

import numpy as np
import pytest

import oracle
from oracle import sweep_axis as sa
from paper_1908_11740_amd import datagen

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

from paper_1908_11740_amd import sj  # noqa: E402
from gpu_util import sort_pairs, to_dev  # noqa: E402


def say(*a):
    print(*a, file=sys.stderr, flush=True)


def aniso(n, seed, median=2e-3):
    mix = datagen.mixture_spec(12, 700 + seed)
    return (datagen.anisotropic(n, mix, 0.1, median, 25.0, 0.5, 2 * seed + 1),
            datagen.anisotropic(n, mix, 0.1, median, 25.0, 0.5, 2 * seed + 2))


@pytest.fixture(scope="module")
def aniso_small():
    R, S = aniso(150_000, 1)
    return R, S, oracle.pbsm(R, S, 32)


def with_large(n, seed):
    """A mixture where every 11th rectangle is enlarged to span 2 to 10 tiles
    of a 16 x 16 grid: the samples' mean extent then depends on the large
    extents (no clipping in the division count rule)."""
    A = datagen.mixture(n, datagen.mixture_spec(8, 900 + seed), 0.2, 1e-3, 1.0, seed).copy()
    rng = np.random.default_rng(seed)
    big = np.arange(0, n, 11)
    ext = rng.uniform(0.125, 0.625, size=(len(big), 2)).astype(np.float32)
    A[big, 2] = A[big, 0] + ext[:, 0]
    A[big, 3] = A[big, 1] + ext[:, 1]
    return A


CASES = [
    ("aniso K16", lambda: aniso(200_000, 2), 16, None),
    ("aniso K64", lambda: aniso(200_000, 3, 5e-4), 64, None),
    ("mixture K8", lambda: (datagen.mixture(100_000, datagen.mixture_spec(20, 5), 0.2, 2e-3, 1.0, 6),
                            datagen.mixture(80_000, datagen.mixture_spec(20, 5), 0.2, 2e-3, 1.0, 7)),
     8, None),
    ("aniso K32 domain", lambda: tuple(2 * A for A in aniso(100_000, 4)), 32, (0.0, 0.0, 2.0, 2.0)),
    ("large extents K16", lambda: (with_large(60_000, 11), with_large(50_000, 12)), 16, None),
]


@pytest.mark.parametrize("name,make,K,domain", CASES, ids=[c[0] for c in CASES])
def test_model_matches_oracle_on_every_tile(name, make, K, domain):
    say("axis model", name)
    R, S = make()
    R, S = np.ascontiguousarray(R, np.float32), np.ascontiguousarray(S, np.float32)
    ref = sa.all_tiles(R, S, K, domain)
    PR = sj.partition(to_dev(R), K, domain=domain)
    PS = sj.partition(to_dev(S), K, domain=domain)
    tiles = np.array([(tx, ty) for ty in range(K) for tx in range(K)], np.int32)
    got = sj.sweep_axis(PR, PS, tiles)
    PR.free()
    PS.free()
    n_model = n_y = 0
    for (tx, ty), row in zip(tiles, got):
        want = ref.get((int(tx), int(ty)))
        want = (0, 0, 0, 0) if want is None else want[:4]
        assert tuple(int(v) for v in row) == want, (tx, ty)
        n_model += want[0] > 0
        n_y += want[3]
    assert n_model > 0
    if name.startswith("aniso"):
        assert 0 < n_y < n_model


_MODELS = {}


def _model(K):
    if K not in _MODELS:
        R, S = aniso(150_000, 1)
        _MODELS[K] = sa.all_tiles(R, S, K)
    return _MODELS[K]


SCHED = {"tuned": {}, "twopass": dict(flags=sj.SJ_TWO_PASS), "tau1": dict(split_tau=1),
         "sweep_x": dict(flags=sj.SJ_SWEEP_X), "tau64": dict(split_tau=64)}


@pytest.mark.parametrize("K", [1, 2, 4, 16, 64])
@pytest.mark.parametrize("sched", sorted(SCHED))
def test_join_with_model_matches_oracle(aniso_small, K, sched):
    R, S, ref = aniso_small
    say("axis join K", K, sched)
    kw = SCHED[sched]
    PR = sj.partition(to_dev(R), K, **kw)
    PS = sj.partition(to_dev(S), K, **kw)
    got = sort_pairs(sj.join(PR, PS).cpu().numpy())
    st = sj.last_join_stats()
    assert np.array_equal(got, ref)
    # the model runs on the medium and dense tiles unless switched off
    if sched == "sweep_x":
        assert st["axis_tiles"] == 0 and st["axis_y"] == 0
    else:
        assert st["axis_tiles"] == st["medium_tiles"] + st["dense_tiles"]
        model = _model(K)
        want_y = sum(1 for v in model.values()
                     if v[4] + v[5] > st["small_cap"] and v[3] == 1)
        assert st["axis_y"] == want_y
        if 2 <= K <= 16:  # K = 1: one tile holding both halves
            assert want_y > 0
    # joined again (the two-pass write-back leaves valid, re-sorted slabs)
    again = sort_pairs(sj.join(PR, PS).cpu().numpy())
    assert np.array_equal(again, ref)
    assert sj.join_count(PR, PS) == len(ref)
    PR.free()
    PS.free()


def test_dense_tiles_swept_along_y():
    # one tile, far more entries than a medium tile: the dense path sorts by
    # y_l when the model says so
    R, S = aniso(80_000, 5)
    # only the horizontal rectangles (wide, flat): the model picks y
    R = np.ascontiguousarray(R[(R[:, 2] - R[:, 0]) > (R[:, 3] - R[:, 1])])
    S = np.ascontiguousarray(S[(S[:, 2] - S[:, 0]) > (S[:, 3] - S[:, 1])])
    ref = oracle.pbsm(R, S, 8)
    for kw in ({}, dict(split_tau=97), dict(flags=sj.SJ_TWO_PASS)):
        PR = sj.partition(to_dev(R), 1, **kw)
        PS = sj.partition(to_dev(S), 1, **kw)
        got = sort_pairs(sj.join(PR, PS).cpu().numpy())
        st = sj.last_join_stats()
        assert np.array_equal(got, ref)
        assert st["dense_tiles"] == 1 and st["axis_y"] == 1
        row = sj.sweep_axis(PR, PS, np.array([[0, 0]], np.int32))[0]
        assert row[3] == 1 and row[2] < row[1]
        PR.free()
        PS.free()


def test_query_arguments():
    R, S = aniso(2000, 6)
    PR = sj.partition(to_dev(R), 4)
    PS = sj.partition(to_dev(S), 4)
    with pytest.raises(sj.SjError) as e:
        sj.sweep_axis(PR, PS, np.array([[4, 0]], np.int32))
    assert e.value.status == sj.SJ_ERR_ARG
    PT = sj.partition(to_dev(S), 8)
    with pytest.raises(sj.SjError) as e:
        sj.sweep_axis(PR, PT, np.array([[0, 0]], np.int32))
    assert e.value.status == sj.SJ_ERR_GRID_MISMATCH
    assert sj.sweep_axis(PR, PS, np.zeros((0, 2), np.int32)).shape == (0, 4)
    for P in (PR, PS, PT):
        P.free()
