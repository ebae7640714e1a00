"""GPU: the autotuner picks and caches a schedule per workload class; every
candidate schedule and the tuned one return exactly the oracle's pairs."""
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


@pytest.mark.parametrize("workload", ["small", "mixture"])
def test_tuned_schedule_keeps_the_pair_set(workload):
    if workload == "small":
        R, S, K = datagen.small_case()
    else:
        mix = datagen.mixture_spec(30, 31)
        R = datagen.mixture(300_000, mix, 0.2, 1e-4, 1.0, 32)
        S = datagen.mixture(250_000, mix, 0.2, 1e-4, 1.0, 33)
        K = 600
    ref = oracle.pbsm(R, S, 64)
    PR, PS = sj.partition(to_dev(R), K), sj.partition(to_dev(S), K)
    out = torch.empty((len(ref) + 10, 2), dtype=torch.int32, device="cuda")
    sj.tune_clear()
    best = sj.tune(PR, PS, out, reps=1)
    say(workload, "tuned", best)
    assert best["block"] in (64, 128, 256, 512) and best["ms"] > 0
    st, n = sj.join_into(PR, PS, out)
    assert st == sj.SJ_OK and n == len(ref)
    assert np.array_equal(sort_pairs(out[:n].cpu().numpy()), ref)
    # count-only tuning is cached separately and counts exactly
    best_c = sj.tune(PR, PS, None, reps=1)
    assert best_c["block"] in (64, 128, 256, 512)
    assert sj.join_count(PR, PS) == len(ref)
    sj.tune_clear()
    st, n = sj.join_into(PR, PS, out)
    assert np.array_equal(sort_pairs(out[:n].cpu().numpy()), ref)


def test_every_candidate_schedule_is_exact():
    """The tuner's whole candidate space, forced one at a time through the
    cache, on a workload with small, medium and dense tiles, pairs and
    count-only."""
    mix = datagen.mixture_spec(5, 41)
    R = datagen.mixture(120_000, mix, 0.1, 3e-4, 1.0, 42)
    S = datagen.mixture(100_000, mix, 0.1, 3e-4, 1.0, 43)
    ref = oracle.pbsm(R, S, 64)
    PR, PS = sj.partition(to_dev(R), 128), sj.partition(to_dev(S), 128)
    out = torch.empty((len(ref) + 10, 2), dtype=torch.int32, device="cuda")
    E = {64: 256, 128: 1024, 256: 1024, 512: 2048}
    for blk in (64, 128, 256, 512):
        for sc in (E[blk] // 4, E[blk] // 2):
            for mc in (1024, 2048):
                for tau in (128, 256, 1024):
                    sj.tune_set(PR, PS, blk, sc, mc, tau)
                    st, n = sj.join_into(PR, PS, out)
                    assert st == sj.SJ_OK and n == len(ref)
                    assert np.array_equal(sort_pairs(out[:n].cpu().numpy()), ref), (blk, sc, mc, tau)
                    sj.tune_set(PR, PS, blk, sc, mc, tau, count_only=True)
                    assert sj.join_count(PR, PS) == len(ref)
    st_ = sj.last_join_stats()
    assert st_["n_pairs"] == len(ref)
    sj.tune_clear()


def test_tune_cache_save_and_load(tmp_path):
    """The cache written by sj_tune_save comes back with sj_tune_load on this
    device's architecture and drives the join (same schedule, exact pairs);
    entries of another architecture and malformed files are handled."""
    R, S, K = datagen.small_case()
    ref = oracle.pbsm(R, S, 64)
    PR, PS = sj.partition(to_dev(R), K), sj.partition(to_dev(S), K)
    out = torch.empty((len(ref) + 10, 2), dtype=torch.int32, device="cuda")
    sj.tune_clear()
    sj.tune_set(PR, PS, 128, 256, 1024, 128)
    path = tmp_path / "tune.txt"
    sj.tune_save(path)
    lines = [l for l in path.read_text().splitlines() if not l.startswith("#")]
    assert len(lines) == 1
    arch, k, lr, ls, mode, blk, sc, mc, tau, ms = lines[0].split()
    assert arch.startswith("gfx") and int(k) == K and int(mode) == 0
    assert (int(blk), int(sc), int(mc), int(tau)) == (128, 256, 1024, 128)
    sj.tune_clear()
    # another architecture's line is skipped, ours is loaded
    path.write_text(path.read_text() + lines[0].replace(arch, "gfx000", 1) + "\n")
    assert sj.tune_lookup(PR, PS) is None
    assert sj.tune_load(path) == 1
    assert sj.tune_lookup(PR, PS)["small_cap"] == 256
    assert sj.tune_lookup(PR, PS, count_only=True) is None
    # stripes on the same K and entry counts are another class
    QR = sj.partition(to_dev(R), K, flags=sj.SJ_STRIPES)
    QS = sj.partition(to_dev(S), K, flags=sj.SJ_STRIPES)
    assert sj.tune_lookup(QR, QS) is None
    QR.free()
    QS.free()
    st, n = sj.join_into(PR, PS, out)
    assert st == sj.SJ_OK and np.array_equal(sort_pairs(out[:n].cpu().numpy()), ref)
    assert sj.last_join_stats()["small_cap"] == 256
    bad = tmp_path / "bad.txt"
    bad.write_text("gfx950 12 x\n")
    with pytest.raises(sj.SjError):
        sj.tune_load(bad)
    with pytest.raises(sj.SjError):
        sj.tune_load(tmp_path / "missing.txt")
    sj.tune_clear()
