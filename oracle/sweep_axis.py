"""CPU oracle of the per-tile sweeping-axis model (Sec. 3.3, Eq. (2)).

TEST INFRASTRUCTURE ONLY (see the package docstring).

For a tile T the model estimates how many pairs of R_T x S_T overlap along
each axis -- the candidates a plane sweep along that axis must check -- and
sweeps along the axis with the smaller estimate.  Per axis, the tile's
extent is cut into k equal divisions; H_R^x[i] counts the sampled
rectangles of R_T whose x-projection meets division i (likewise S, y), and

    I^x_T = sum_i H_R^x[i] * H_S^x[i]                              (Eq. (2))

The sweep runs along y when I^y_T < I^x_T, else along x.

Readings where the paper leaves details open (the same in the GPU library):

* Sample: the paper uses one of every phi = 100 rectangles assigned to the
  tile.  Here a rectangle is sampled when its input index is a multiple of
  phi, which picks about one in phi of every tile's rectangles and does not
  depend on the order of a tile's list.  A tile whose R or S sample is empty
  is swept along x.
* k: 1000 for tiles large against the rectangles, else the number of times
  the tile's extent exceeds the mean extent of the rectangles.  Here the
  mean extent (w + h) / 2 is taken over the tile's sampled rectangles (R and
  S), in cell units (a tile is one cell), summed exactly as integers in
  units of 2^-30 of a cell (each w and h truncated to that unit), so the sum
  does not depend on the order of the tile's list;
  k = clamp(floor(2 n 2^30 / sum), 1, 1000), and 1000 when the sum is 0.
  An extent is capped at 2^32 cells before the sum: one such extent makes
  the sum at least 2^62 > 2 n 2^30 for any n < 2^31, so k = 1 with or
  without the cap, and the cap keeps the GPU's fixed-width sums finite.
* Divisions: the division of a coordinate v in tile column t is
  clamp(floor(fl(fl(u - t) * k)), 0, k - 1) with u = fl(fl(v - x0) * sx),
  the float32 cell coordinate of the grid's cell function (sx = float32(K) /
  float32(width)); every fl is one float32 rounding.
"""
import numpy as np

PHI = 100
K_BUCKETS = 1000
FIX = 2 ** 30

f32 = np.float32


def grid_scales(K, domain=None):
    """(x0, y0, sx, sy) as float32, the grid's cell coordinate u = (v - x0) * sx."""
    d = (0.0, 0.0, 1.0, 1.0) if domain is None or all(v == 0 for v in domain) else domain
    x0, y0 = f32(d[0]), f32(d[1])
    w, h = f32(f32(d[2]) - x0), f32(f32(d[3]) - y0)
    return x0, y0, f32(f32(K) / w), f32(f32(K) / h)


CAP = 2.0 ** 32  # cells; does not change k (see above)


def _fixed(ext):
    """Extents (float32, cell units) in units of 2^-30 of a cell, as Python
    integers (exact sums of any size)."""
    e = np.minimum(np.asarray(ext, dtype=np.float64), CAP)
    return [int(v) for v in np.floor(e * FIX)]


def buckets(lo, hi, origin, scale, t, k):
    """Division range [b(lo), b(hi)] of projections [lo, hi] in tile column t."""
    def b(v):
        u = f32(f32(np.asarray(v, dtype=f32) - origin) * scale)
        f = f32(f32(u - f32(t)) * f32(k))
        return np.clip(np.floor(f.astype(np.float64)), 0, k - 1).astype(np.int64)
    return b(lo), b(hi)


def histogram(lo_b, hi_b, k):
    """H[i] = number of ranges [lo_b, hi_b] that contain division i."""
    H = np.zeros(k, dtype=np.int64)
    for a, c in zip(lo_b, hi_b):
        H[a:c + 1] += 1
    return H


def tile_model(Rt, St, tx, ty, K, domain=None):
    """Eq. (2) for one tile.  Rt, St: the (n, 4) float32 rectangles of the
    tile's sample (already filtered).  Returns (k, Ix, Iy, axis), axis 1 = y."""
    Rt = np.asarray(Rt, dtype=f32).reshape(-1, 4)
    St = np.asarray(St, dtype=f32).reshape(-1, 4)
    if len(Rt) == 0 or len(St) == 0:
        return 0, 0, 0, 0
    x0, y0, sx, sy = grid_scales(K, domain)
    A = np.concatenate([Rt, St])
    wc = f32(f32(A[:, 2] - A[:, 0]) * sx)
    hc = f32(f32(A[:, 3] - A[:, 1]) * sy)
    tot = sum(_fixed(wc)) + sum(_fixed(hc))
    n = len(A)
    k = K_BUCKETS if tot == 0 else int(min(max((2 * n * FIX) // tot, 1), K_BUCKETS))
    I = []
    for lo_i, hi_i, org, sc, t in ((0, 2, x0, sx, tx), (1, 3, y0, sy, ty)):
        HR = histogram(*buckets(Rt[:, lo_i], Rt[:, hi_i], org, sc, t, k), k)
        HS = histogram(*buckets(St[:, lo_i], St[:, hi_i], org, sc, t, k), k)
        I.append(int((HR * HS).sum()))
    return k, I[0], I[1], 1 if I[1] < I[0] else 0


def tile_samples(ids):
    """The sampled members of a tile's id list."""
    ids = np.asarray(ids)
    return ids[ids % PHI == 0]


def all_tiles(R, S, K, domain=None):
    """Eq. (2) for every tile of the K x K grid, using the oracle's tile
    membership.  Returns a dict (tx, ty) -> (k, Ix, Iy, axis, nr, ns) for the
    tiles with at least one R and one S rectangle."""
    import oracle
    offR, idsR = oracle.partition_ids(R, K, domain)
    offS, idsS = oracle.partition_ids(S, K, domain)
    out = {}
    for t in range(K * K):
        a, b = offR[t], offR[t + 1]
        c, d = offS[t], offS[t + 1]
        if a == b or c == d:
            continue
        tx, ty = t % K, t // K
        sr, ss = tile_samples(idsR[a:b]), tile_samples(idsS[c:d])
        out[(tx, ty)] = tile_model(R[sr], S[ss], tx, ty, K, domain) + (int(b - a), int(d - c))
    return out
