"""GPU parity of grid choice: features, the statistics rule, the learned
picker's network kernels (forward, loss, backward, Adam) and its use by
sj_choose_grid, against the float64 CPU oracle."""
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


def say(*a):
    print(*a, file=sys.stderr, flush=True)


def _instances():
    R, S, _ = datagen.small_case()
    yield "small", R, S, None
    R, S = datagen.uniform_1m(300_000)
    yield "uniform", R, S, None
    mix = datagen.mixture_spec(17, 11)
    yield "mixture", datagen.mixture(200_000, mix, 0.1, 2e-4, 1.0, 12), \
        datagen.mixture(150_001, mix, 0.1, 2e-4, 1.0, 13), None
    yield "domain", R * 3 - 1, S[:1000] * 3 - 1, (-1.0, -1.0, 2.0, 2.0)
    yield "one-empty", R[:777], R[:0], None


@pytest.mark.parametrize("case", range(5))
def test_features_match_oracle(case):
    name, R, S, dom = list(_instances())[case]
    say("features", name)
    f, e = sj.features(to_dev(R), to_dev(S), domain=dom)
    f = f.cpu().numpy()
    ref = op.features(R, S, dom)
    assert e == pytest.approx(op.mean_extent(R, S, dom), rel=1e-12)
    for side in range(2):
        b = side * op.SIDE
        assert np.allclose(f[b:b + 5], ref[b:b + 5], rtol=1e-6, atol=1e-5)
        # the histogram bins are integer counts: identical
        assert np.array_equal(f[b + 5:b + op.SIDE], ref[b + 5:b + op.SIDE].astype(np.float32))


def test_rule_matches_closed_form_on_the_workloads():
    R, S, _ = datagen.small_case()
    k, tau, info = sj.choose_grid(to_dev(R), to_dev(S), flags=sj.SJ_RULE_ONLY)
    assert k == info["k_rule"] == 100 and tau == 0
    R, S = datagen.uniform_1m()
    k, _, info = sj.choose_grid(to_dev(R), to_dev(S))
    assert k == 1000 == op.rule_k(op.mean_extent(R, S))
    assert sj.rule_k(info["mean_extent"]) == 1000
    # caller-fixed fields are kept
    k, tau, _ = sj.choose_grid(to_dev(R), to_dev(S), k=77, split_tau=5)
    assert (k, tau) == (77, 5)


def test_rule_on_skewed_10m():
    R, S = datagen.skewed_10m()
    k, _, info = sj.choose_grid(to_dev(R), to_dev(S))
    assert k == op.rule_k(op.mean_extent(R, S))
    assert abs(k - 1213) <= 5
    assert info["used_learned"] == 0


def test_chosen_grid_is_capped_by_the_input_size():
    """A 2-D grid chosen for n rectangles keeps K^2 <= 8 n: 300 + 200 tiny
    rectangles (rule K = SJ_K_MAX) get K = floor(sqrt(4000)) = 63; stripes
    and caller-fixed grids are not capped."""
    R = datagen.uniform(300, 1e-6, 61)
    S = datagen.uniform(200, 1e-6, 62)
    k, _, info = sj.choose_grid(to_dev(R), to_dev(S), flags=sj.SJ_RULE_ONLY)
    assert info["k_rule"] == sj.SJ_K_MAX and info["k_cap"] == 63 and k == 63
    k, _, info = sj.choose_grid(to_dev(R), to_dev(S), flags=sj.SJ_STRIPES)
    assert info["k_cap"] == sj.SJ_K_MAX and k == info["k_rule"]
    k, _, _ = sj.choose_grid(to_dev(R), to_dev(S), k=4000)
    assert k == 4000


def test_invalid_rectangle_rejected_by_choose():
    R = datagen.uniform(1000, 0.01, 5)
    R[10, 2] = np.nan
    with pytest.raises(sj.SjError) as ei:
        sj.choose_grid(to_dev(R), to_dev(R[:5]))
    assert ei.value.status == sj.SJ_ERR_RECT


# ----------------------------------------------------------------------------
# Network kernels against the float64 oracle (FP32 reduction order differs:
# tolerance 1e-4 relative to the largest magnitude)
# ----------------------------------------------------------------------------
def _close(a, b, rel=1e-4):
    a = np.asarray(a, np.float64)
    b = np.asarray(b, np.float64)
    scale = max(np.abs(b).max(), 1e-30)
    return np.abs(a - b).max() <= rel * scale


def _net(d, B, seed):
    rng = np.random.default_rng(seed)
    P = (rng.normal(0, 1, op.param_count(d)) / np.sqrt(np.r_[
        np.full(64 * d + 64, d), np.full(64 * 64 + 64, 64), np.full(2 * 64 + 2, 64)])).astype(np.float32)
    X = rng.normal(0, 1, (B, d)).astype(np.float32)
    mu = rng.normal(0, 0.3, d).astype(np.float32)
    sd = rng.uniform(0.5, 2, d).astype(np.float32)
    T = rng.normal(0, 1, (B, 2)).astype(np.float32)
    return P, X, mu, sd, T


def _dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


@pytest.mark.parametrize("d,B", [(7, 3), (2058, 64), (2058, 1), (100, 257)])
def test_mlp_forward_loss_backward(d, B):
    say("mlp", d, B)
    P, X, mu, sd, T = _net(d, B, d + B)
    Pd, Xd, mud, sdd, Td = map(_dev, (P, X, mu, sd, T))
    act = torch.empty((B, 128), dtype=torch.float32, device="cuda")
    Y = sj.mlp_forward(Pd, Xd, mud, sdd, act=act)
    yr, h1, h2 = op.forward(P, X, mu, sd)
    assert _close(Y.cpu().numpy(), yr)
    assert _close(act.cpu().numpy(), np.concatenate([h1, h2], 1))
    loss, dY = sj.mlp_loss(Y, Td)
    lr, dyr = op.loss(Y.cpu().numpy().astype(np.float64), T)
    assert loss.item() == pytest.approx(lr, rel=1e-5)
    assert _close(dY.cpu().numpy(), dyr, 1e-6)
    g = sj.mlp_backward(Pd, Xd, act, dY, mud, sdd)
    gr = op.backward(P, X, dY.cpu().numpy(), mu, sd)
    # per tensor, since the scales differ
    o = 0
    for n in (64 * d, 64, 64 * 64, 64, 128, 2):
        assert _close(g.cpu().numpy()[o:o + n], gr[o:o + n]), (o, n)
        o += n


def test_mlp_identity_normalisation_when_null():
    P, X, _, _, _ = _net(9, 5, 1)
    Y = sj.mlp_forward(_dev(P), _dev(X))
    assert _close(Y.cpu().numpy(), op.forward(P, X)[0])


def test_adam_steps_match_oracle():
    rng = np.random.default_rng(3)
    n = 10_000
    P = rng.normal(size=n).astype(np.float32)
    M = np.zeros(n, np.float32)
    V = np.zeros(n, np.float32)
    Pd, Md, Vd = _dev(P), _dev(M), _dev(V)
    Pr, Mr, Vr = P.astype(np.float64), M.astype(np.float64), V.astype(np.float64)
    for t in range(1, 6):
        G = rng.normal(size=n).astype(np.float32)
        G[::17] = 0
        sj.mlp_adam(Pd, Md, Vd, _dev(G), t, lr=1e-2)
        Pr, Mr, Vr = op.adam(Pr, Mr, Vr, G, t, lr=1e-2)
    assert np.allclose(Pd.cpu().numpy(), Pr, rtol=1e-5, atol=1e-6)
    assert np.allclose(Md.cpu().numpy(), Mr, rtol=1e-5, atol=1e-7)
    # 1 - beta2 = 1 - 0.999 rounds to 0.00099998713 in float32 (relative
    # error 1.3e-5), which every second moment inherits
    assert np.allclose(Vd.cpu().numpy(), Vr, rtol=3e-5, atol=1e-9)


def test_training_reduces_the_loss():
    """A few hundred Adam steps of the GPU kernels fit a smooth target."""
    rng = np.random.default_rng(5)
    d, B = 16, 128
    X = rng.normal(size=(B, d)).astype(np.float32)
    T = np.stack([np.sin(X[:, 0]) + 0.5 * X[:, 1], X[:, 2] * X[:, 3] * 0.3], 1).astype(np.float32)
    P, _, _, _, _ = _net(d, 1, 77)
    Pd, Xd, Td = _dev(P), _dev(X), _dev(T)
    Md, Vd = torch.zeros_like(Pd), torch.zeros_like(Pd)
    act = torch.empty((B, 128), dtype=torch.float32, device="cuda")
    first = None
    for t in range(1, 401):
        Y = sj.mlp_forward(Pd, Xd, act=act)
        loss, dY = sj.mlp_loss(Y, Td)
        if first is None:
            first = loss.item()
        g = sj.mlp_backward(Pd, Xd, act, dY)
        sj.mlp_adam(Pd, Md, Vd, g, t, lr=3e-3)
    last = sj.mlp_loss(sj.mlp_forward(Pd, Xd), Td)[0].item()
    say("loss", first, "->", last)
    assert last < 0.2 * first


def _blob(seed, ymu=(10.0, 8.0), ysd=(1.0, 1.0)):
    d = sj.FEAT_DIM
    P, _, mu, sd, _ = _net(d, 1, seed)
    return np.concatenate([mu, sd, np.array([ymu[0], ymu[1], ysd[0], ysd[1]], np.float32), P])


def test_choose_grid_with_loaded_picker_follows_the_network():
    R, S = datagen.uniform_1m(200_000)
    blob = _blob(21)
    sj.picker_load(blob)
    try:
        assert sj.picker_loaded()
        k, tau, info = sj.choose_grid(to_dev(R), to_dev(S))
        d = sj.FEAT_DIM
        mu, sd, ys, P = blob[:d], blob[d:2 * d], blob[2 * d:2 * d + 4], blob[2 * d + 4:]
        y = op.forward(P, op.features(R, S), mu, sd)[0][0]
        l2k = np.clip(y[0] * ys[2] + ys[0], 0, 13)
        l2t = np.clip(y[1] * ys[3] + ys[1], 3, 20)
        assert info["used_learned"] == 1
        assert abs(np.log2(info["k_learned"]) - l2k) < 0.01 and abs(np.log2(tau) - l2t) < 0.01
        # the chosen K is the network's, at most k_cap = floor(sqrt(8 N))
        assert info["k_cap"] == int(np.floor(np.sqrt(8.0 * (len(R) + len(S)))))
        assert k == min(info["k_learned"], info["k_cap"])
        # the rule is still reported, and SJ_RULE_ONLY bypasses the picker
        k2, tau2, info2 = sj.choose_grid(to_dev(R), to_dev(S), flags=sj.SJ_RULE_ONLY)
        assert k2 == info["k_rule"] == 1000 and tau2 == 0 and info2["used_learned"] == 0
        # whatever the picker chooses, the pair set is the oracle's
        ref = oracle.pbsm(R[:50_000], S[:50_000], 256)
        k3, tau3, _ = sj.choose_grid(to_dev(R[:50_000]), to_dev(S[:50_000]))
        assert np.array_equal(gpu_join(R[:50_000], S[:50_000], k3, split_tau=tau3), ref)
    finally:
        sj.picker_unload()
    assert not sj.picker_loaded()


def test_picker_blob_length_checked():
    with pytest.raises(sj.SjError) as ei:
        sj.picker_load(np.zeros(10, np.float32))
    assert ei.value.status == sj.SJ_ERR_ARG
