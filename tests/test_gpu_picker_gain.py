"""GPU: what the trained picker gains over the method without it.  On
held-out corpus instances (never seen in training; indices 1800+), the join
with the learned (K, tau) is compared with the join at the statistics rule's
K (same schedule) -- wall time of partition + join, medians of 3 -- and both
pair counts must agree."""
import sys

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

from paper_1908_11740_amd import picker, sj  # noqa: E402


def say(*a):
    print(*a, file=sys.stderr, flush=True)


@pytest.mark.skipif(not picker.weights_available(), reason="no trained picker weights")
def test_learned_pick_beats_the_rule_on_held_out_instances():
    picker.load()
    try:
        ratios = []
        for i in range(1800, 1812):
            R, S, _, _ = picker.sized_instance(i, scale=0.5)
            kl, tl, info = sj.choose_grid(R, S)
            kr = info["k_rule"]
            tm = picker.Timer(R, S)
            n_l = tm.run(kl, tl)
            n_r = tm.run(kr, 0)
            assert n_l == n_r  # the grid never changes the result
            t_l = tm.time(kl, tl, reps=3)
            t_r = tm.time(kr, 0, reps=3)
            tm.free()
            ratios.append(t_r / t_l)
            say(f"instance {i}: learned K={kl} tau={tl} {t_l * 1e3:.2f} ms, rule K={kr} "
                f"{t_r * 1e3:.2f} ms")
        gm = float(np.exp(np.mean(np.log(ratios))))
        say("geometric-mean speedup of the learned pick over the rule:", gm)
        assert gm > 1.05
    finally:
        sj.picker_unload()
