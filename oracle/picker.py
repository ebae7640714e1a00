"""CPU oracle for grid choice: the statistics rule, the instance features and
the picker network (2 x 64 MLP, loss, backward, Adam), in float64 numpy.

TEST INFRASTRUCTURE ONLY (see the package docstring).  Written from the
definitions, not from the GPU library:

* Rule of thumb (Sec. 4.3.1, 4.3.3): tiles about one order of magnitude
  larger than the rectangles.  With e the mean over R and S of (w + h) / 2 in
  domain units, K = clamp(round(1 / (10 e)), 1, K_max) for a square grid.
* Features: per side, log2(n + 1), log2 of the mean and standard deviation
  of w and h (+1e-9), and log2(1 + 1024 * share) of the rectangle centres
  of every 100th rectangle over a 32 x 32 grid (the paper samples its
  sweep-axis histograms too, Sec. 3.3).
* Network: h1 = relu(W1 xn + b1), h2 = relu(W2 h1 + b2), y = W3 h2 + b3,
  xn = (x - mu) / sd; loss 1/(2B) sum (y - t)^2; gradients by the chain
  rule; Adam with bias correction (Kingma and Ba, 2015).

Parity of these functions is not pinned by the paper (it has no learned
part); the tests pin them by closed forms, hand-computed cases and central
finite differences.
"""
import numpy as np

K_MAX = 8192
HIST = 32
PHI = 100
SIDE = 5 + HIST * HIST
H = 64
OUT = 2


def rule_k(mean_extent):
    """K = clamp(round(1/(10 e)), 1, K_max); e == 0 -> K_max."""
    e = float(mean_extent)
    if e == 0.0:
        return K_MAX
    if not e > 0.0:
        return 1
    return int(min(max(np.floor(1.0 / (10.0 * e) + 0.5), 1.0), K_MAX))


def _domain(domain):
    if domain is None or all(v == 0 for v in domain):
        return 0.0, 0.0, 1.0, 1.0
    return tuple(float(v) for v in domain)


def mean_extent(R, S, domain=None):
    x0, y0, x1, y1 = _domain(domain)
    tot, n = 0.0, 0
    for A in (R, S):
        A = np.asarray(A, dtype=np.float64).reshape(-1, 4)
        w = (A[:, 2] - A[:, 0]) / (x1 - x0)
        h = (A[:, 3] - A[:, 1]) / (y1 - y0)
        tot += w.sum() + h.sum()
        n += len(A)
    return tot / (2.0 * n) if n else 0.0


def mean_x_extent(R, S, domain=None):
    """Mean over R and S of w in domain units: the statistic of the 1-D rule
    (stripes about ten times the mean x-extent, Sec. 4.3.1)."""
    x0, _, x1, _ = _domain(domain)
    tot, n = 0.0, 0
    for A in (R, S):
        A = np.asarray(A, dtype=np.float64).reshape(-1, 4)
        tot += ((A[:, 2] - A[:, 0]) / (x1 - x0)).sum()
        n += len(A)
    return tot / n if n else 0.0


def side_features(A, domain=None):
    x0, y0, x1, y1 = _domain(domain)
    A32 = np.asarray(A, dtype=np.float32).reshape(-1, 4)
    A = A32.astype(np.float64)
    n = len(A)
    f = np.zeros(SIDE)
    f[0] = np.log2(n + 1.0)
    iw, ih = 1.0 / (x1 - x0), 1.0 / (y1 - y0)
    if n:
        w = (A[:, 2] - A[:, 0]) * iw
        h = (A[:, 3] - A[:, 1]) * ih
        mw, mh = w.mean(), h.mean()
        vw = max((w * w).mean() - mw * mw, 0.0)
        vh = max((h * h).mean() - mh * mh, 0.0)
    else:
        mw = mh = vw = vh = 0.0
    f[1] = np.log2(mw + 1e-9)
    f[2] = np.log2(mh + 1e-9)
    f[3] = np.log2(np.sqrt(vw) + 1e-9)
    f[4] = np.log2(np.sqrt(vh) + 1e-9)
    smp = A[::PHI]
    if len(smp):
        cx = (0.5 * (smp[:, 0] + smp[:, 2]) - x0) * iw * HIST
        cy = (0.5 * (smp[:, 1] + smp[:, 3]) - y0) * ih * HIST
        bx = np.clip(np.floor(cx), 0, HIST - 1).astype(np.int64)
        by = np.clip(np.floor(cy), 0, HIST - 1).astype(np.int64)
        cnt = np.bincount(by * HIST + bx, minlength=HIST * HIST).astype(np.float64)
        f[5:] = np.log2(1.0 + cnt * (HIST * HIST) / len(smp))
    return f


def histogram_counts(A, domain=None):
    """Integer counts of the sampled centres per 32 x 32 cell (row-major by cy)."""
    x0, y0, x1, y1 = _domain(domain)
    A = np.asarray(A, dtype=np.float32).reshape(-1, 4).astype(np.float64)[::PHI]
    iw, ih = 1.0 / (x1 - x0), 1.0 / (y1 - y0)
    cx = (0.5 * (A[:, 0] + A[:, 2]) - x0) * iw * HIST
    cy = (0.5 * (A[:, 1] + A[:, 3]) - y0) * ih * HIST
    bx = np.clip(np.floor(cx), 0, HIST - 1).astype(np.int64)
    by = np.clip(np.floor(cy), 0, HIST - 1).astype(np.int64)
    return np.bincount(by * HIST + bx, minlength=HIST * HIST)


def features(R, S, domain=None):
    return np.concatenate([side_features(R, domain), side_features(S, domain)])


# ----------------------------------------------------------------------------
# Network
# ----------------------------------------------------------------------------
def param_count(d):
    return H * d + H + H * H + H + OUT * H + OUT


def unpack(P, d):
    P = np.asarray(P, dtype=np.float64)
    o = 0
    W1 = P[o:o + H * d].reshape(H, d); o += H * d
    b1 = P[o:o + H]; o += H
    W2 = P[o:o + H * H].reshape(H, H); o += H * H
    b2 = P[o:o + H]; o += H
    W3 = P[o:o + OUT * H].reshape(OUT, H); o += OUT * H
    b3 = P[o:o + OUT]; o += OUT
    assert o == len(P)
    return W1, b1, W2, b2, W3, b3


def pack(W1, b1, W2, b2, W3, b3):
    return np.concatenate([W1.ravel(), b1, W2.ravel(), b2, W3.ravel(), b3])


def normalise(X, mu=None, sd=None):
    X = np.asarray(X, dtype=np.float64)
    if mu is not None:
        X = X - np.asarray(mu, dtype=np.float64)
    if sd is not None:
        X = X / np.asarray(sd, dtype=np.float64)
    return X


def forward(P, X, mu=None, sd=None):
    """Returns y (B x 2), h1 and h2 (B x 64, after ReLU)."""
    X = np.atleast_2d(np.asarray(X, dtype=np.float64))
    W1, b1, W2, b2, W3, b3 = unpack(P, X.shape[1])
    xn = normalise(X, mu, sd)
    h1 = np.maximum(xn @ W1.T + b1, 0.0)
    h2 = np.maximum(h1 @ W2.T + b2, 0.0)
    y = h2 @ W3.T + b3
    return y, h1, h2


def loss(Y, T):
    """L = 1/(2B) sum (y - t)^2 and dL/dY."""
    Y = np.asarray(Y, dtype=np.float64)
    T = np.asarray(T, dtype=np.float64)
    B = Y.shape[0]
    E = Y - T
    return float((E * E).sum() / (2.0 * B)), E / B


def backward(P, X, dY, mu=None, sd=None):
    """Gradient of sum(dY * y) w.r.t. the flat parameter vector."""
    X = np.atleast_2d(np.asarray(X, dtype=np.float64))
    d = X.shape[1]
    W1, b1, W2, b2, W3, b3 = unpack(P, d)
    xn = normalise(X, mu, sd)
    _, h1, h2 = forward(P, X, mu, sd)
    dY = np.asarray(dY, dtype=np.float64)
    gW3 = dY.T @ h2
    gb3 = dY.sum(0)
    dh2 = (dY @ W3) * (h2 > 0)
    gW2 = dh2.T @ h1
    gb2 = dh2.sum(0)
    dh1 = (dh2 @ W2) * (h1 > 0)
    gW1 = dh1.T @ xn
    gb1 = dh1.sum(0)
    return pack(gW1, gb1, gW2, gb2, gW3, gb3)


def adam(P, M, V, G, step, lr=1e-3, b1=0.9, b2=0.999, eps=1e-8):
    """One bias-corrected Adam step; returns new (P, M, V)."""
    P, M, V, G = (np.asarray(a, dtype=np.float64) for a in (P, M, V, G))
    M = b1 * M + (1.0 - b1) * G
    V = b2 * V + (1.0 - b2) * G * G
    mh = M / (1.0 - b1 ** step)
    vh = V / (1.0 - b2 ** step)
    return P - lr * mh / (np.sqrt(vh) + eps), M, V
