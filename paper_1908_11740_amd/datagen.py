"""Seeded synthetic join inputs.

The paper evaluates on real Tiger 2015 / OpenStreetMap MBRs normalised to
[0,1]^2 (Sec. 4.1, Table 1).  Those datasets are not available here, so these
generators stand in for them with the same shape: float32 axis-aligned
rectangles in the unit square, relative extents of 1e-6..1e-3, millions of
rectangles, uniform or strongly clustered.

This module holds no part of the join's arithmetic: it only draws numbers.
Both the GPU library's tests and the CPU oracle are fed from it, and neither
imports the other.  Every array is ``(n, 4)`` float32 ``(x_l, y_l, x_u, y_u)``
with ``x_l <= x_u`` and ``y_l <= y_u``, drawn from numpy's PCG64 generator
with the stated seed.

Workload recipes (sizes and seeds are the defaults of the helpers below):

* ``uniform``: lower corner uniform in [0,1)^2, width and height each uniform
  in [0, max_extent]; upper corner = float32(lower + extent).
    - small case: 10,000 per side, max_extent 0.002, seeds 101 / 102, K = 64.
    - 1M case:  1,000,000 per side, max_extent 2e-4, seeds 201 / 202.
* ``mixture``: centres from a shared mixture of isotropic Gaussians
  (mean uniform in [0,1)^2, sigma uniform in [sigma_lo, sigma_hi], weights
  Dirichlet(alpha)) plus a uniform background fraction; a centre outside
  [0,1)^2 is drawn again until it falls inside.  Width and height are
  log-normal (median, sigma_ln) i.i.d.; the rectangle is
  [c - w/2, c + w/2] x [c - h/2, c + h/2] rounded to float32.
    - skewed 10M case: 10,000,000 per side, 200 clusters (seed 300), sigma in
      [0.005, 0.05], Dirichlet(0.5), 20% background, median 5e-5,
      sigma_ln 1.0, seeds 301 / 302.
* ``picker_instance(i)``: the learned-picker corpus; instance i draws, from
  seed 4000 + i, per-side sizes log-uniform in [1e6, 2e7], cluster count
  log-uniform integer in [1, 500], background uniform in [0, 0.5], extent
  median log-uniform in [1e-5, 1e-3], sigma_ln = 1.0.
* ``anisotropic``: mixture centres as above; each rectangle is long and thin,
  long side = median * sqrt(ratio) and short side = median / sqrt(ratio),
  each times an independent log-normal(0, sigma_ln) factor; horizontal
  (w long) when the centre lies left of x = 0.5, vertical right of it -- a
  stand-in for road maps, where the better sweeping axis differs by region.
    - anisotropic 4M case: 4,000,000 per side, 100 clusters (seed 400),
      10% background, median 2e-4, ratio 25, sigma_ln 0.5, seeds 401 / 402.
* points for the epsilon-distance join (Sec. 1 names it as a use of the
  intersection join): ``(n, 2)`` float32 ``(x, y)``.
    - ``points_mixture``: the centres of ``mixture`` rounded to float32.
    - skewed 10M point case: 10,000,000 per side, the skewed 10M mixture
      (200 clusters, seed 300, 20% background), seeds 311 / 312, eps = 1e-4.
    - ``lattice``: integer lattice points times a spacing (exact in float32).
    - ``near_ring``: Q[i] = P[i] + r (cos t, sin t) rounded to float32 with r
      within a few ulps of eps, so that many pairs sit on the boundary.
* ``batch_instance(j)``: join j of the 256-join batch; from seed 5000 + j,
  per-side sizes log-uniform in [1e3, 2e6] (independently), cluster count and
  background as for the picker corpus, extents uniform in [0, 2e-4] around
  mixture centres.
"""
from dataclasses import dataclass

import numpy as np


def uniform(n, max_extent, seed):
    """Uniform lower corners in [0,1)^2, extents uniform in [0, max_extent]."""
    rng = np.random.default_rng(seed)
    n = int(n)
    xl = rng.random(n, dtype=np.float32)
    yl = rng.random(n, dtype=np.float32)
    w = rng.random(n, dtype=np.float32) * np.float32(max_extent)
    h = rng.random(n, dtype=np.float32) * np.float32(max_extent)
    out = np.empty((n, 4), dtype=np.float32)
    out[:, 0] = xl
    out[:, 1] = yl
    out[:, 2] = xl + w
    out[:, 3] = yl + h
    return out


@dataclass
class Mixture:
    mu: np.ndarray      # (k, 2) cluster means
    sigma: np.ndarray   # (k,)   isotropic standard deviations
    weight: np.ndarray  # (k,)   mixture weights, sum 1


def mixture_spec(k, seed, sigma_lo=0.005, sigma_hi=0.05, alpha=0.5):
    rng = np.random.default_rng(seed)
    k = int(k)
    mu = rng.random((k, 2))
    sigma = rng.uniform(sigma_lo, sigma_hi, size=k)
    weight = rng.dirichlet(np.full(k, alpha)) if k > 1 else np.ones(1)
    weight = np.maximum(weight, 0.0)
    weight = weight / weight.sum()
    return Mixture(mu, sigma, weight)


def _centres(rng, n, mix, background):
    """n centres in [0,1)^2: background fraction uniform, the rest from mix."""
    c = np.empty((n, 2))
    is_bg = rng.random(n) < background
    nb = int(is_bg.sum())
    c[is_bg] = rng.random((nb, 2))
    idx = np.flatnonzero(~is_bg)
    comp = rng.choice(len(mix.weight), size=len(idx), p=mix.weight)
    pts = mix.mu[comp] + mix.sigma[comp, None] * rng.standard_normal((len(idx), 2))
    bad = np.flatnonzero((pts < 0.0).any(1) | (pts >= 1.0).any(1))
    while len(bad):
        pts[bad] = mix.mu[comp[bad]] + mix.sigma[comp[bad], None] * rng.standard_normal((len(bad), 2))
        bad = bad[(pts[bad] < 0.0).any(1) | (pts[bad] >= 1.0).any(1)]
    c[idx] = pts
    return c


def _boxes(c, w, h):
    out = np.empty((len(c), 4), dtype=np.float32)
    out[:, 0] = c[:, 0] - 0.5 * w
    out[:, 1] = c[:, 1] - 0.5 * h
    out[:, 2] = c[:, 0] + 0.5 * w
    out[:, 3] = c[:, 1] + 0.5 * h
    return out


def mixture(n, mix, background, median, sigma_ln, seed):
    """Mixture centres, log-normal extents (median, sigma_ln)."""
    rng = np.random.default_rng(seed)
    n = int(n)
    c = _centres(rng, n, mix, background)
    w = rng.lognormal(np.log(median), sigma_ln, size=n)
    h = rng.lognormal(np.log(median), sigma_ln, size=n)
    return _boxes(c, w, h)


def mixture_uniform_extent(n, mix, background, max_extent, seed):
    """Mixture centres, extents uniform in [0, max_extent]."""
    rng = np.random.default_rng(seed)
    n = int(n)
    c = _centres(rng, n, mix, background)
    w = rng.random(n) * max_extent
    h = rng.random(n) * max_extent
    return _boxes(c, w, h)


# ----------------------------------------------------------------------------
# The named workloads
# ----------------------------------------------------------------------------

def small_case():
    """10,000 x 10,000, extents U[0,0.002], K = 64."""
    return uniform(10_000, 0.002, 101), uniform(10_000, 0.002, 102), 64


def uniform_1m(n=1_000_000):
    """1M x 1M uniform, extents U[0,2e-4]; the grid is swept over 256..4096."""
    return uniform(n, 2e-4, 201), uniform(n, 2e-4, 202)


UNIFORM_1M_GRIDS = (256, 512, 1024, 2048, 4096)


def skewed_10m(n=10_000_000):
    """10M x 10M skewed: 200-cluster mixture + 20% background, log-normal extents."""
    mix = mixture_spec(200, 300)
    return (mixture(n, mix, 0.2, 5e-5, 1.0, 301),
            mixture(n, mix, 0.2, 5e-5, 1.0, 302))


def _log_uniform(rng, lo, hi):
    return float(np.exp(rng.uniform(np.log(lo), np.log(hi))))


@dataclass
class InstanceSpec:
    n_r: int
    n_s: int
    clusters: int
    background: float
    median: float
    seed: int


def picker_instance_spec(i):
    rng = np.random.default_rng(4000 + int(i))
    n_r = int(round(_log_uniform(rng, 1e6, 2e7)))
    n_s = int(round(_log_uniform(rng, 1e6, 2e7)))
    k = int(min(500, max(1, np.floor(_log_uniform(rng, 1.0, 501.0)))))
    bg = float(rng.uniform(0.0, 0.5))
    med = _log_uniform(rng, 1e-5, 1e-3)
    return InstanceSpec(n_r, n_s, k, bg, med, 4000 + int(i))


def small_instance_spec(i):
    """Instance i of the picker's small-input corpus: the distributions of
    picker_instance_spec with 1e3 to 1e6 rectangles per side (the sizes of a
    batch's joins, which the main corpus does not reach)."""
    rng = np.random.default_rng(6000 + int(i))
    n_r = int(round(_log_uniform(rng, 1e3, 1e6)))
    n_s = int(round(_log_uniform(rng, 1e3, 1e6)))
    k = int(min(500, max(1, np.floor(_log_uniform(rng, 1.0, 501.0)))))
    bg = float(rng.uniform(0.0, 0.5))
    med = _log_uniform(rng, 1e-5, 1e-3)
    return InstanceSpec(n_r, n_s, k, bg, med, 6000 + int(i))


def picker_instance(i, scale=1.0):
    """Instance i of the learned-picker corpus (sizes optionally scaled down)."""
    sp = picker_instance_spec(i)
    mix = mixture_spec(sp.clusters, sp.seed * 7 + 1)
    nr = max(1, int(sp.n_r * scale))
    ns = max(1, int(sp.n_s * scale))
    return (mixture(nr, mix, sp.background, sp.median, 1.0, sp.seed * 7 + 2),
            mixture(ns, mix, sp.background, sp.median, 1.0, sp.seed * 7 + 3), sp)


def batch_instance_spec(j):
    rng = np.random.default_rng(5000 + int(j))
    n_r = int(round(_log_uniform(rng, 1e3, 2e6)))
    n_s = int(round(_log_uniform(rng, 1e3, 2e6)))
    k = int(min(500, max(1, np.floor(_log_uniform(rng, 1.0, 501.0)))))
    bg = float(rng.uniform(0.0, 0.5))
    return InstanceSpec(n_r, n_s, k, bg, 2e-4, 5000 + int(j))


def batch_instance(j, scale=1.0):
    """Join j of the many-join batch."""
    sp = batch_instance_spec(j)
    mix = mixture_spec(sp.clusters, sp.seed * 7 + 1)
    nr = max(1, int(sp.n_r * scale))
    ns = max(1, int(sp.n_s * scale))
    return (mixture_uniform_extent(nr, mix, sp.background, 2e-4, sp.seed * 7 + 2),
            mixture_uniform_extent(ns, mix, sp.background, 2e-4, sp.seed * 7 + 3), sp)


# ----------------------------------------------------------------------------
# Point sets for the epsilon-distance join
# ----------------------------------------------------------------------------
def points_uniform(n, seed):
    """n points uniform in [0,1)^2."""
    rng = np.random.default_rng(seed)
    return rng.random((int(n), 2)).astype(np.float32)


def points_mixture(n, mix, background, seed):
    """n mixture centres (as in ``mixture``) rounded to float32."""
    rng = np.random.default_rng(seed)
    return _centres(rng, int(n), mix, background).astype(np.float32)


def skewed_points_10m(n=10_000_000):
    """10M x 10M skewed points: the skewed 10M mixture's centres; eps = 1e-4."""
    mix = mixture_spec(200, 300)
    return points_mixture(n, mix, 0.2, 311), points_mixture(n, mix, 0.2, 312), 1e-4


def lattice(nx, ny, spacing=1.0, origin=(0.0, 0.0)):
    """Points origin + spacing * (i, j), 0 <= i < nx, 0 <= j < ny (row-major by j)."""
    j, i = np.mgrid[0:ny, 0:nx]
    pts = np.stack([origin[0] + spacing * i.ravel(), origin[1] + spacing * j.ravel()], 1)
    return pts.astype(np.float32)


def near_ring(n, eps, seed, ulps=4):
    """P uniform in [0.25, 0.75)^2 and Q[i] = P[i] + r (cos t, sin t) rounded to
    float32, r = eps * (1 + u 2^-23) with u a random integer in [-ulps, ulps]."""
    rng = np.random.default_rng(seed)
    n = int(n)
    P = (0.25 + 0.5 * rng.random((n, 2))).astype(np.float32)
    t = rng.random(n) * 2 * np.pi
    r = float(eps) * (1.0 + rng.integers(-ulps, ulps + 1, n) * 2.0 ** -23)
    Q = (P.astype(np.float64) + r[:, None] * np.stack([np.cos(t), np.sin(t)], 1)).astype(np.float32)
    return P, Q


# ----------------------------------------------------------------------------
# Anisotropic rectangles (per-tile sweeping axis)
# ----------------------------------------------------------------------------
def anisotropic(n, mix, background, median, ratio, sigma_ln, seed):
    """Mixture centres; long thin rectangles, horizontal left of x = 0.5 and
    vertical right of it."""
    rng = np.random.default_rng(seed)
    n = int(n)
    c = _centres(rng, n, mix, background)
    r = np.sqrt(float(ratio))
    long_ = median * r * rng.lognormal(0.0, sigma_ln, size=n)
    short = median / r * rng.lognormal(0.0, sigma_ln, size=n)
    horiz = c[:, 0] < 0.5
    return _boxes(c, np.where(horiz, long_, short), np.where(horiz, short, long_))


def anisotropic_4m(n=4_000_000):
    """4M x 4M long thin rectangles, orientation by half of the domain."""
    mix = mixture_spec(100, 400)
    return (anisotropic(n, mix, 0.1, 2e-4, 25.0, 0.5, 401),
            anisotropic(n, mix, 0.1, 2e-4, 25.0, 0.5, 402))
