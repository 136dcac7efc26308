"""Oracle: viewgraph estimation by cycle-consistent reprojection (paper Sec. 3
"Viewgraph Estimation", Sec. 4 "Implementation Details"; supplementary Sec.
"Fused Triton kernels", construction kernels).

Test infrastructure only (see the package header).

For a candidate image pair (i, j), i < j, every pixel p of a grid over image i
(stride g, starting at pixel 0) that has a depth Z_i(p) > 0 is
  1. projected into j:   p_ij = pi(K_i, K_j, P_i, P_j, Z_i; p)
     (lift X_c = Z ((x - cx)/fx, (y - cy)/fy, Z), to the world
     X_w = R_i^T (X_c - t_i), into j X' = R_j X_w + t_j, project
     u' = fx_j X'_x / X'_z + cx_j; it needs X'_z > z_min),
  2. projected back:     p_iji = pi(K_j, K_i, P_j, P_i, Z_j; p_ij), with Z_j read
     at the pixel nearest to p_ij (which must lie inside image j and have a
     depth > 0), and the back projection's depth in i above z_min;
  3. called consistent when ||p - p_iji||^2 < tau^2.
The pair is valid (an edge of the viewgraph) when at least min_fraction of the
grid points with depth are consistent: consistent >= min_fraction * total.
Defaults: tau = 3 px, min_fraction = 0.125 (Sec. 4), grid stride 4 px.

Every step is float64 with one rounding per operation, in the order written
below, so that a device implementation computing the same IEEE operations in
the same order (no fused multiply-add) takes the same integer decisions.
"""
from __future__ import annotations

import numpy as np

TAU = 3.0
MIN_FRACTION = 0.125
STRIDE = 4
Z_MIN = 1e-4


def _project(x, y, Z, Ks, Kt, Ps, Pt):
    """pi(K_s, K_t, P_s, P_t, Z; (x, y)): returns u', v', z' in the target."""
    fxs, fys, cxs, cys = (float(np.float64(k)) for k in Ks)
    fxt, fyt, cxt, cyt = (float(np.float64(k)) for k in Kt)
    Rs, ts = Ps[:, :3], Ps[:, 3]
    Rt, tt = Pt[:, :3], Pt[:, 3]
    # lift in the source camera
    X0 = (x - cxs) / fxs * Z
    X1 = (y - cys) / fys * Z
    X2 = Z
    d0, d1, d2 = X0 - ts[0], X1 - ts[1], X2 - ts[2]
    # world point R_s^T (X_c - t_s)
    W0 = (Rs[0, 0] * d0 + Rs[1, 0] * d1) + Rs[2, 0] * d2
    W1 = (Rs[0, 1] * d0 + Rs[1, 1] * d1) + Rs[2, 1] * d2
    W2 = (Rs[0, 2] * d0 + Rs[1, 2] * d1) + Rs[2, 2] * d2
    # target camera R_t X_w + t_t
    Y0 = ((Rt[0, 0] * W0 + Rt[0, 1] * W1) + Rt[0, 2] * W2) + tt[0]
    Y1 = ((Rt[1, 0] * W0 + Rt[1, 1] * W1) + Rt[1, 2] * W2) + tt[1]
    Y2 = ((Rt[2, 0] * W0 + Rt[2, 1] * W1) + Rt[2, 2] * W2) + tt[2]
    with np.errstate(divide="ignore", invalid="ignore"):
        u = fxt * (Y0 / Y2) + cxt
        v = fyt * (Y1 / Y2) + cyt
    return u, v, Y2


def pair_counts(depth_i, depth_j, Ki, Kj, Pi, Pj, stride=STRIDE, tau=TAU, z_min=Z_MIN):
    """(consistent, total) of the round trip i -> j -> i over the grid of i."""
    Hi, Wi = depth_i.shape
    Hj, Wj = depth_j.shape
    ys, xs = np.mgrid[0:Hi:stride, 0:Wi:stride]
    xs = xs.ravel().astype(np.float64)
    ys = ys.ravel().astype(np.float64)
    Z = depth_i[ys.astype(np.int64), xs.astype(np.int64)].astype(np.float64)
    has = np.isfinite(Z) & (Z > 0)
    xs, ys, Z = xs[has], ys[has], Z[has]
    total = int(xs.size)
    u, v, z = _project(xs, ys, Z, Ki, Kj, Pi, Pj)
    ok = z > z_min
    with np.errstate(invalid="ignore"):
        ur = np.floor(u + 0.5)
        vr = np.floor(v + 0.5)
    ok &= (ur >= 0) & (ur < Wj) & (vr >= 0) & (vr < Hj)
    ur_i = np.where(ok, ur, 0).astype(np.int64)
    vr_i = np.where(ok, vr, 0).astype(np.int64)
    Zj = depth_j[vr_i, ur_i].astype(np.float64)
    ok &= np.isfinite(Zj) & (Zj > 0)
    Zj = np.where(ok, Zj, 1.0)
    u2, v2, z2 = _project(np.where(ok, u, 0.0), np.where(ok, v, 0.0), Zj, Kj, Ki, Pj, Pi)
    ok &= z2 > z_min
    with np.errstate(invalid="ignore"):
        e0 = u2 - xs
        e1 = v2 - ys
        err2 = e0 * e0 + e1 * e1
    ok &= err2 < tau * tau
    return int(ok.sum()), total


def candidate_pairs(scene_of_view) -> np.ndarray:
    """All (i, j), i < j, within each scene, in row-major order."""
    sov = np.asarray(scene_of_view)
    out = [(i, j) for i in range(sov.size) for j in range(i + 1, sov.size) if sov[i] == sov[j]]
    return np.array(out, np.int64).reshape(-1, 2)


def build(depth_maps, K, poses, scene_of_view, stride=STRIDE, tau=TAU,
          min_fraction=MIN_FRACTION, z_min=Z_MIN):
    """Counts and validity of every candidate pair.  depth_maps: list of
    (H_v, W_v) arrays."""
    cand = candidate_pairs(scene_of_view)
    cons = np.zeros(len(cand), np.int64)
    tot = np.zeros(len(cand), np.int64)
    for k, (i, j) in enumerate(cand):
        cons[k], tot[k] = pair_counts(depth_maps[i], depth_maps[j], K[i], K[j], poses[i],
                                      poses[j], stride, tau, z_min)
    valid = (tot > 0) & (cons >= min_fraction * tot)
    return cand, cons, tot, valid
