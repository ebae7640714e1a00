"""Learned grid picker: weights file, loading into the library, and the
training pipeline (labels from GPU-measured join times, training with the
library's own MLP kernels).

The paper chooses K with a rule of thumb (tiles about ten times the mean
rectangle extent, Sec. 4.3.1 / 4.3.3).  The picker maps instance features
(sj_features) to (log2 K, log2 tau) -- tau the dense-tile split threshold --
learned from the best measured candidate per training instance.  It never
changes the join result, only its speed; the rule stays the fallback
(SJ_RULE_ONLY, or no weights).
"""
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
WEIGHTS = os.path.join(HERE, "picker_weights.npz")


def weights_available(path=WEIGHTS):
    return os.path.exists(path)


def load_blob(path=WEIGHTS):
    """Blob for sj_picker_load: mu | sd | ystat | params (float32)."""
    with np.load(path, allow_pickle=False) as z:
        return np.concatenate([z["mu"], z["sd"], z["ystat"], z["params"]]).astype(np.float32)


def load(path=WEIGHTS):
    from . import sj
    sj.picker_load(load_blob(path))


# ----------------------------------------------------------------------------
# Corpus: instances generated on the device, candidates timed on the device
# ----------------------------------------------------------------------------
TAUS = (64, 256, 1024, 4096)
DEFAULT_TAU = 256


def spec(i, kind):
    from . import datagen
    return {"picker": datagen.picker_instance_spec, "small": datagen.small_instance_spec,
            "batch": datagen.batch_instance_spec}[kind](i)


def instance(i, scale=1.0, kind="picker"):
    """Device tensors (R, S) and the spec of corpus instance i (same
    distributions as datagen's picker / small / batch instances, drawn on the
    device)."""
    from . import datagen, sj
    sp = spec(i, kind)
    if kind in ("picker", "small"):
        ext = dict(extent="lognormal", ext_a=sp.median, ext_b=1.0)
    else:
        ext = dict(extent="uniform", ext_a=sp.median)
    mix = datagen.mixture_spec(sp.clusters, sp.seed * 7 + 1)
    nr = max(1, int(sp.n_r * scale))
    ns = max(1, int(sp.n_s * scale))
    seed = sp.seed * 1_000_003 + 17
    R = sj.generate(nr, mix.mu, mix.sigma, mix.weight, sp.background, seed=seed, side=0, **ext)
    S = sj.generate(ns, mix.mu, mix.sigma, mix.weight, sp.background, seed=seed, side=1, **ext)
    return R, S, sp


P_UNIFORM_CAP = 1e7  # pre-scale: expected pairs of the same sizes without clustering
P_CAP = 5e7          # measured pairs at the rule's K


def sized_instance(i, scale=1.0, kind="picker"):
    """instance(i) scaled down (both sides by the same factor) where its join
    output would exceed the caps above -- the dense corner of the corpus
    (large n with extents near 1e-3) yields 1e9+ pairs per join, far beyond
    what a training label needs.  Deterministic in i."""
    from . import sj
    sp = spec(i, kind)
    me = sp.median * np.exp(0.5) if kind in ("picker", "small") else sp.median / 2
    pu = sp.n_r * sp.n_s * scale * scale * (2 * me) ** 2
    if pu > P_UNIFORM_CAP:
        scale *= np.sqrt(P_UNIFORM_CAP / pu)
    for it in range(6):
        R, S, sp = instance(i, scale, kind)
        _, e = sj.features(R, S)
        k = sj.rule_k(e)
        PR, PS = sj.partition(R, k), sj.partition(S, k)
        try:
            p = sj.join_count(PR, PS)
        except sj.SjError as err:  # beyond 2^31 pairs
            if err.status != sj.SJ_ERR_TOO_LARGE:
                raise
            p = 2.0 ** 33
        PR.free()
        PS.free()
        if p <= P_CAP or it == 5:
            break
        del R, S
        scale *= np.sqrt(P_CAP / p)
    return R, S, sp, scale


def k_candidates(k_rule, lo=8):
    """Half-octave steps around the rule's K: K_rule * 2^(j/2), j = -6..6,
    clamped to [lo, 8192]."""
    ks = sorted({int(min(8192, max(lo, round(k_rule * 2.0 ** (j / 2))))) for j in range(-6, 7)})
    return ks


def capped_rule_k(k_rule, n_r, n_s):
    """The rule's K as sj_choose_grid applies it to a 2-D grid: at most
    sqrt(8 (nR + nS))."""
    return int(max(1, min(k_rule, np.floor(np.sqrt(8.0 * (n_r + n_s))))))


class Timer:
    """Times partition(R) + partition(S) + join for a (K, tau, flags) on
    resident device inputs, reusing handles and the output buffer."""

    def __init__(self, R, S):
        import torch
        self.R, self.S = R, S
        self.PR = self.PS = None
        self.out = torch.empty((1 << 20, 2), dtype=torch.int32, device=R.device)

    def run(self, K, tau, flags=0):
        import torch
        from . import sj
        self.PR = sj.partition(self.R, K, split_tau=tau, flags=flags, reuse=self.PR)
        self.PS = sj.partition(self.S, K, split_tau=tau, flags=flags, reuse=self.PS)
        st, n = sj.join_into(self.PR, self.PS, self.out)
        if st == sj.SJ_ERR_CAPACITY:
            self.out = torch.empty((int(n * 1.2) + 1024, 2), dtype=torch.int32,
                                   device=self.R.device)
            st, n = sj.join_into(self.PR, self.PS, self.out)
        return n

    def time(self, K, tau, flags=0, reps=1):
        import time
        import torch
        self.run(K, tau, flags)  # warm-up (allocations)
        torch.cuda.synchronize()
        ts = []
        for _ in range(reps):
            t0 = time.perf_counter()
            self.run(K, tau, flags)
            torch.cuda.synchronize()
            ts.append(time.perf_counter() - t0)
        return float(np.median(ts))

    def free(self):
        for p in (self.PR, self.PS):
            if p is not None:
                p.free()


def collect(indices, scale=1.0, log=print, kind="picker"):
    """Features and candidate timings for corpus instances; returns a dict of
    arrays.  Label = (K, tau) of the fastest candidate: K over the rule's
    half-octave neighbourhood at the default tau, then tau at that K.  The
    small-input corpus centres the neighbourhood on the capped rule, lets K
    go down to 2 and takes the median of three timed runs per candidate
    (joins of well under a millisecond)."""
    from . import sj
    small = kind == "small"
    reps, lo = (3, 2) if small else (1, 8)
    feats, krule, kbest, tbest, trule, tbestv, nrs, nss = [], [], [], [], [], [], [], []
    scales = []
    for c, i in enumerate(indices):
        R, S, sp, sc = sized_instance(i, scale, kind)
        scales.append(sc)
        f, e = sj.features(R, S)
        kr = sj.rule_k(e)
        if small:
            kr = capped_rule_k(kr, R.shape[0], S.shape[0])
        tm = Timer(R, S)
        times = {}
        for K in k_candidates(kr, lo):
            times[(K, DEFAULT_TAU)] = tm.time(K, DEFAULT_TAU, reps=reps)
        kb = min(times, key=times.get)[0]
        for tau in TAUS:
            if (kb, tau) not in times:
                times[(kb, tau)] = tm.time(kb, tau, reps=reps)
        best = min(times, key=times.get)
        tm.free()
        feats.append(f.cpu().numpy())
        krule.append(kr)
        kbest.append(best[0])
        tbest.append(best[1])
        trule.append(times.get((kr, DEFAULT_TAU), np.nan))
        tbestv.append(times[best])
        nrs.append(R.shape[0])
        nss.append(S.shape[0])
        if c % 20 == 0:
            log(f"instance {i}: n={R.shape[0]}+{S.shape[0]} K_rule={kr} best={best} "
                f"t_rule={trule[-1] * 1e3:.2f} ms t_best={times[best] * 1e3:.2f} ms")
        del R, S
    return dict(index=np.asarray(indices), feat=np.asarray(feats, np.float32),
                k_rule=np.asarray(krule), k_best=np.asarray(kbest), tau_best=np.asarray(tbest),
                t_rule=np.asarray(trule), t_best=np.asarray(tbestv), n_r=np.asarray(nrs),
                n_s=np.asarray(nss), scale=np.asarray(scales))


# ----------------------------------------------------------------------------
# Training with the library's MLP kernels (forward, loss, backward, Adam)
# ----------------------------------------------------------------------------
def init_params(d, seed=0):
    """He-uniform weights, zero biases."""
    rng = np.random.default_rng(seed)
    parts = []
    for fan_in, fan_out in ((d, 64), (64, 64), (64, 2)):
        lim = np.sqrt(6.0 / fan_in)
        parts.append(rng.uniform(-lim, lim, fan_out * fan_in))
        parts.append(np.zeros(fan_out))
    return np.concatenate(parts).astype(np.float32)


def train(X, T, epochs=400, batch=256, lr=1e-3, seed=0, log=print):
    """Fit the 2 x 64 MLP to targets T (N x 2, log2 K and log2 tau) on the
    GPU.  Returns (mu, sd, ystat, params) as float32 arrays."""
    import torch
    from . import sj
    X = np.asarray(X, np.float64)
    T = np.asarray(T, np.float64)
    mu = X.mean(0)
    sd = np.maximum(X.std(0), 1e-3)
    ymu, ysd = T.mean(0), np.maximum(T.std(0), 1e-3)
    Tn = (T - ymu) / ysd
    dev = torch.device("cuda", torch.cuda.current_device())
    Xd = torch.from_numpy(X.astype(np.float32)).to(dev)
    Td = torch.from_numpy(Tn.astype(np.float32)).to(dev)
    mud = torch.from_numpy(mu.astype(np.float32)).to(dev)
    sdd = torch.from_numpy(sd.astype(np.float32)).to(dev)
    P = torch.from_numpy(init_params(X.shape[1], seed)).to(dev)
    M, V = torch.zeros_like(P), torch.zeros_like(P)
    rng = np.random.default_rng(seed + 1)
    N = X.shape[0]
    step = 0
    for ep in range(epochs):
        perm = torch.from_numpy(rng.permutation(N)).to(dev)
        tot = 0.0
        for b0 in range(0, N, batch):
            idx = perm[b0:b0 + batch]
            xb, tb = Xd[idx].contiguous(), Td[idx].contiguous()
            B = xb.shape[0]
            act = torch.empty((B, 128), dtype=torch.float32, device=dev)
            Y = sj.mlp_forward(P, xb, mud, sdd, act=act)
            loss, dY = sj.mlp_loss(Y, tb)
            g = sj.mlp_backward(P, xb, act, dY, mud, sdd)
            step += 1
            sj.mlp_adam(P, M, V, g, step, lr=lr)
            tot += loss.item() * B
        if ep % 50 == 0 or ep == epochs - 1:
            log(f"epoch {ep}: loss {tot / N:.4f}")
    return (mu.astype(np.float32), sd.astype(np.float32),
            np.array([ymu[0], ymu[1], ysd[0], ysd[1]], np.float32), P.cpu().numpy())


def save(path, mu, sd, ystat, params):
    np.savez(path, mu=mu, sd=sd, ystat=ystat, params=params)


def targets(corpus):
    return np.stack([np.log2(corpus["k_best"]), np.log2(corpus["tau_best"])], 1)


def evaluate(indices, scale=1.0, reps=3, log=print, kind="picker"):
    """Per held-out instance: time of the learned pick (tuned schedule), of
    the rule (tuned schedule) and of the rule with the plain schedule.  The
    rule's K is capped as sj_choose_grid caps it."""
    from . import sj
    rows = []
    for c, i in enumerate(indices):
        R, S, _, _ = sized_instance(i, scale, kind)
        kl, tl, info = sj.choose_grid(R, S)
        kr = min(info["k_rule"], info["k_cap"])
        tm = Timer(R, S)
        t_learned = tm.time(kl, tl, reps=reps)
        t_rule = tm.time(kr, 0, reps=reps)
        t_plain = tm.time(kr, 0, flags=sj.SJ_PLAIN, reps=reps)
        tm.free()
        rows.append((i, kl, tl, kr, t_learned, t_rule, t_plain))
        if c % 20 == 0:
            log(f"eval {i}: learned K={kl} tau={tl} {t_learned * 1e3:.2f} ms, rule K={kr} "
                f"{t_rule * 1e3:.2f} ms, plain {t_plain * 1e3:.2f} ms")
        del R, S
    a = np.asarray(rows, np.float64)
    return dict(index=a[:, 0].astype(np.int64), k_learned=a[:, 1], tau_learned=a[:, 2],
                k_rule=a[:, 3], t_learned=a[:, 4], t_rule=a[:, 5], t_plain=a[:, 6])


def summary(ev):
    g = lambda x: float(np.exp(np.mean(np.log(x))))  # noqa: E731
    return {
        "instances": int(len(ev["t_learned"])),
        "geomean_speedup_vs_rule_tuned": g(ev["t_rule"] / ev["t_learned"]),
        "geomean_speedup_vs_rule_plain": g(ev["t_plain"] / ev["t_learned"]),
        "win_rate_vs_rule_tuned": float(np.mean(ev["t_learned"] < ev["t_rule"])),
        "win_rate_vs_rule_plain": float(np.mean(ev["t_learned"] < ev["t_plain"])),
    }


def main(argv=None):
    import argparse
    import json
    import sys
    import torch

    ap = argparse.ArgumentParser(description="learned grid picker: corpus, training, evaluation")
    sub = ap.add_subparsers(dest="cmd", required=True)
    c = sub.add_parser("collect")
    c.add_argument("--start", type=int, default=0)
    c.add_argument("--count", type=int, default=1800)
    c.add_argument("--scale", type=float, default=1.0)
    c.add_argument("--out", required=True)
    c.add_argument("--kind", default="picker", choices=["picker", "small", "batch"])
    t = sub.add_parser("train")
    t.add_argument("--corpus", nargs="+", required=True)
    t.add_argument("--epochs", type=int, default=400)
    t.add_argument("--out", default=WEIGHTS)
    e = sub.add_parser("evaluate")
    e.add_argument("--weights", default=WEIGHTS)
    e.add_argument("--start", type=int, default=1800)
    e.add_argument("--count", type=int, default=200)
    e.add_argument("--scale", type=float, default=1.0)
    e.add_argument("--out", default=None)
    e.add_argument("--kind", default="picker", choices=["picker", "small", "batch"])
    a = ap.parse_args(argv)

    def log(*x):
        print(*x, file=sys.stderr, flush=True)

    torch.cuda.set_device(0)
    if a.cmd == "collect":
        cor = collect(range(a.start, a.start + a.count), a.scale, log, a.kind)
        np.savez(a.out, **cor)
        log("wrote", a.out)
    elif a.cmd == "train":
        parts = [dict(np.load(p, allow_pickle=False)) for p in a.corpus]
        cor = {k: np.concatenate([p[k] for p in parts]) for k in parts[0]}
        mu, sd, ys, P = train(cor["feat"], targets(cor), epochs=a.epochs, log=log)
        save(a.out, mu, sd, ys, P)
        log("wrote", a.out)
    else:
        load(a.weights)
        ev = evaluate(range(a.start, a.start + a.count), a.scale, log=log, kind=a.kind)
        if a.out:
            np.savez(a.out, **ev)
        print(json.dumps(summary(ev)), flush=True)


if __name__ == "__main__":
    main()
