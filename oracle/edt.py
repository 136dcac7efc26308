"""Oracle: exact squared Euclidean distance transform of a binary edge map.

Test infrastructure only (see the package header).

The paper builds, for every image, a distance transform field in which each
pixel holds the Euclidean distance to the nearest edge pixel, computed with the
exact L2 transform of Felzenszwalb and Huttenlocher (Sec. 3 "Method", first
paragraph; supplementary Sec. A1.2 "Construction kernels").  Pixels sit at
integer coordinates (x = column, y = row), so squared distances are integers
and every implementation here is exact:

  edt_bruteforce  the definition, d2(x, y) = min over edge pixels (x', y') of
                  (x - x')^2 + (y - y')^2
  edt_fh          Felzenszwalb-Huttenlocher: a 1-D lower envelope of parabolas
                  along columns, then along rows, with breakpoints kept as exact
                  rationals (fractions.Fraction)
  edt_separable   the separable decomposition min_x' [(x - x')^2 +
                  min_y' {(y - y')^2 : E(y', x') != 0}] evaluated with NumPy
                  integer arrays (fast enough for full-size views)

A map without any edge pixel has no finite distance; every pixel then holds the
sentinel INF_D2 = 2^30, larger than any real squared distance of an image with
sides up to 16384.

Pins: brute force on every 4x4 binary map and on random maps, closed forms
(single edge pixel, full map, empty map), 1-D envelope vs brute force.
"""
from __future__ import annotations

from fractions import Fraction

import numpy as np

INF_D2 = 1 << 30


def edt_bruteforce(edge: np.ndarray) -> np.ndarray:
    """Squared distance from every pixel to the nearest nonzero pixel."""
    H, W = edge.shape
    ys, xs = np.nonzero(edge)
    if ys.size == 0:
        return np.full((H, W), INF_D2, np.int64)
    gy, gx = np.mgrid[0:H, 0:W]
    gy = gy.reshape(-1, 1).astype(np.int64)
    gx = gx.reshape(-1, 1).astype(np.int64)
    out = np.empty(H * W, np.int64)
    step = max(1, 4_000_000 // max(1, ys.size))
    for a in range(0, H * W, step):
        d = (gx[a:a + step] - xs[None, :]) ** 2 + (gy[a:a + step] - ys[None, :]) ** 2
        out[a:a + step] = d.min(axis=1)
    return out.reshape(H, W)


def lower_envelope_1d(f) -> list:
    """Felzenszwalb-Huttenlocher 1-D transform D(q) = min_p f(p) + (q - p)^2.

    `f` holds non-negative integers or None for +infinity.  Parabolas with
    infinite height are left out; if every entry is infinite the result is all
    None.  Breakpoints are exact Fractions, so the result is exact."""
    n = len(f)
    v = []   # apex positions of the parabolas on the lower envelope
    z = []   # z[k]: left end of the interval where parabola v[k] is lowest (z[0] = -inf)

    def meet(p, q):   # abscissa where the parabolas with apexes p < q intersect
        return Fraction((f[q] + q * q) - (f[p] + p * p), 2 * (q - p))

    for q in range(n):
        if f[q] is None:
            continue
        # drop parabolas that the new one hides completely; the first one has
        # z = -inf and is never dropped
        while len(v) > 1 and meet(v[-1], q) <= z[-1]:
            v.pop()
            z.pop()
        z.append(meet(v[-1], q) if v else None)
        v.append(q)
    if not v:
        return [None] * n
    out = []
    k = 0
    for q in range(n):
        while k + 1 < len(v) and z[k + 1] < q:
            k += 1
        out.append(f[v[k]] + (q - v[k]) ** 2)
    return out


def edt_fh(edge: np.ndarray) -> np.ndarray:
    """Exact EDT by two 1-D Felzenszwalb-Huttenlocher passes (columns, then rows)."""
    H, W = edge.shape
    col = []
    for x in range(W):
        col.append(lower_envelope_1d([0 if edge[y, x] else None for y in range(H)]))
    out = np.empty((H, W), np.int64)
    for y in range(H):
        g = lower_envelope_1d([col[x][y] for x in range(W)])
        out[y, :] = [INF_D2 if val is None else val for val in g]
    return out


def edt_separable(edge: np.ndarray) -> np.ndarray:
    """Exact EDT as min over columns of (column distance^2 + horizontal offset^2)."""
    H, W = edge.shape
    e = edge != 0
    if not e.any():
        return np.full((H, W), INF_D2, np.int64)
    big = np.int64(4 * (H + W) ** 2)
    rows = np.arange(H, dtype=np.int64)[:, None]
    # nearest edge row at or above / at or below, per column
    above = np.where(e, rows, -1)
    above = np.maximum.accumulate(above, axis=0)
    below = np.where(e, rows, H + 4 * (H + W))
    below = np.minimum.accumulate(below[::-1], axis=0)[::-1]
    da = np.where(above >= 0, rows - above, big)
    db = np.where(below < H, below - rows, big)
    g = np.minimum(da, db)
    g = np.where(g >= big, big, g * g)          # column pass: squared, or "infinite"
    xs = np.arange(W, dtype=np.int64)
    off2 = (xs[:, None] - xs[None, :]) ** 2      # (x, x')
    out = np.empty((H, W), np.int64)
    step = max(1, 8_000_000 // (W * W))
    for a in range(0, H, step):
        blk = g[a:a + step]                       # (h, x')
        out[a:a + step] = (blk[:, None, :] + off2[None, :, :]).min(axis=2)
    return out
