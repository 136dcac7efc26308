"""Hand-built tiny inputs with known answers (inputs only, no method arithmetic).

`shifted_pair` is the exact-zero configuration used as a pin: two views with
identical intrinsics fx = fy = 128, cx = 79.5, cy = 59.5 (160 x 120) and poses
that differ by a pure x-translation of b = 0.5.  A point of view 0 at pixel
(u, v) with depth Z appears in view 1 at (u - fx b / Z, v) with the same depth;
with Z in {8, 16, 32, 64} the shift fx b / Z is 8, 4, 2 or 1 pixels, an exact
integer, so every edge pixel of either view lands exactly on an edge pixel of
the other view.
"""
from __future__ import annotations

import numpy as np

from .scenes import Scene, pack


def problem_from_maps(widths, heights, Ks, edge_maps, depth_maps, poses, pairs, poses_gt=None,
                      name="fixture"):
    """Pack explicit per-view maps into a one-scene Problem."""
    V = len(widths)
    idx, zs = [], []
    for v in range(V):
        e = np.asarray(edge_maps[v]).reshape(-1)
        lin = np.flatnonzero(e)
        idx.append(lin.astype(np.int64))
        zs.append(np.asarray(depth_maps[v], np.float32).reshape(-1)[lin])
    poses = np.asarray(poses, np.float64)
    sc = Scene(width=np.asarray(widths, np.int32), height=np.asarray(heights, np.int32),
               K=np.asarray(Ks, np.float32), edge_idx=idx, edge_z=zs,
               poses_gt=poses if poses_gt is None else np.asarray(poses_gt, np.float64),
               poses_init=poses, pairs=np.asarray(pairs, np.int32).reshape(-1, 2),
               meta=dict(config=name))
    return pack([sc], name)


def shifted_pair(seed: int = 0, per_depth: int = 40):
    W, H = 160, 120
    K = [128.0, 128.0, 79.5, 59.5]
    b = 0.5
    rng = np.random.default_rng(seed)
    e0 = np.zeros((H, W), np.uint8)
    e1 = np.zeros((H, W), np.uint8)
    z0 = np.zeros((H, W), np.float32)
    z1 = np.zeros((H, W), np.float32)
    used0, used1 = set(), set()
    for Z in (8.0, 16.0, 32.0, 64.0):
        shift = int(128 * b / Z)
        placed = 0
        while placed < per_depth:
            u = int(rng.integers(10, W - 10))
            v = int(rng.integers(5, H - 5))
            u1 = u - shift
            if (v, u) in used0 or (v, u1) in used1:
                continue
            used0.add((v, u))
            used1.add((v, u1))
            e0[v, u] = 255
            z0[v, u] = Z
            e1[v, u1] = 255
            z1[v, u1] = Z
            placed += 1
    P0 = np.concatenate([np.eye(3), np.zeros((3, 1))], axis=1)
    P1 = np.concatenate([np.eye(3), np.array([[-b], [0.0], [0.0]])], axis=1)
    return problem_from_maps([W, W], [H, H], [K, K], [e0, e1], [z0, z1], [P0, P1],
                             [[0, 1], [1, 0]], name="shifted_pair")


def odd_size_views(seed: int = 0, density: float = 0.15):
    """One scene of six views whose sizes are not multiples of the texture
    blocks (8 x 4 pixels), down to a single 2 x 2 view: random edge pixels
    with depths in [3, 5], cameras a few degrees and centimetres apart looking
    the same way, every ordered pair."""
    from scipy.spatial.transform import Rotation
    rng = np.random.default_rng(seed)
    sizes = [(37, 23), (9, 5), (130, 67), (17, 41), (2, 2), (8, 4)]
    Ws, Hs, Ks, E, Z, P = [], [], [], [], [], []
    for W, H in sizes:
        f = float(max(W, H))
        Ws.append(W)
        Hs.append(H)
        Ks.append([f, f, (W - 1) / 2.0, (H - 1) / 2.0])
        E.append((rng.random((H, W)) < density).astype(np.uint8))
        Z.append(rng.uniform(3.0, 5.0, (H, W)).astype(np.float32))
        R = Rotation.from_rotvec(np.radians(3.0) * rng.normal(size=3) / np.sqrt(3)).as_matrix()
        P.append(np.concatenate([R, 0.05 * rng.normal(size=(3, 1))], axis=1))
    n = len(sizes)
    pairs = [(i, j) for i in range(n) for j in range(n) if i != j]
    return problem_from_maps(Ws, Hs, Ks, E, Z, P, pairs, name="odd_sizes")


def camera_inside(seed: int = 5):
    """Residuals behind the target camera: the two views of the small
    wireframe workload plus a third camera placed inside the wireframe (near
    the centre of the cube, looking along a seeded random direction), which
    sees the third view's maps of the second view.  Pairs 0 -> 2 and 1 -> 2
    put about half of the source points behind camera 2 (z <= 0) and others
    just in front of it; 2 -> 0, 2 -> 1 and 0 -> 1 are ordinary."""
    from .scenes import config_c1, look_at
    p = config_c1()
    rng = np.random.default_rng(seed)
    d = rng.normal(size=3)
    d /= np.linalg.norm(d)
    c = 0.05 * rng.normal(size=3)
    P2 = look_at(c, c + d)
    poses = np.concatenate([p.poses_init, P2[None]], axis=0)
    idx = [0, 1, 1]
    return problem_from_maps(p.width[idx], p.height[idx], p.K[idx],
                             [p.edge_map(v) for v in idx], [p.depth_map(v) for v in idx], poses,
                             [[0, 2], [1, 2], [2, 0], [2, 1], [0, 1]], name="camera_inside")


# target edge grid of `max_side_pair`: pixels (GRID_X0 + GRID_PITCH a, GRID_Y0 + GRID_PITCH b)
GRID_PITCH, GRID_X0, GRID_Y0 = 8, 3, 5


def max_side_pair(seed: int = 3, n_src: int = 30000):
    """Two 16384 x 16384 views, the largest side a plan takes.  View 0 holds
    n_src random edge pixels (a third of them in its last 64 columns or rows,
    some on the very last ones) at depths in [15, 30]; view 1 holds a regular
    grid of edge pixels, pitch GRID_PITCH from (GRID_X0, GRID_Y0), at depth 20.
    Same intrinsics (f = 8000, principal point at the image centre); view 1 is
    rotated by 2e-4 rad about a random axis and translated by
    (0.013, -0.007, 0.004), so source points land a few pixels from where they
    started, at non-integer positions.  Pair 0 -> 1 only."""
    S = 16384
    f = 8000.0
    K = [f, f, (S - 1) / 2.0, (S - 1) / 2.0]
    rng = np.random.default_rng(seed)
    us = rng.integers(0, S, n_src)
    vs = rng.integers(0, S, n_src)
    k = n_src // 6
    us[:k] = rng.integers(S - 64, S, k)
    vs[k:2 * k] = rng.integers(S - 64, S, k)
    us[2 * k:2 * k + 100] = S - 1
    vs[2 * k + 100:2 * k + 200] = S - 1
    lin0 = np.unique(vs.astype(np.int64) * S + us)
    z0 = rng.uniform(15.0, 30.0, lin0.size).astype(np.float32)
    gx = np.arange(GRID_X0, S, GRID_PITCH, dtype=np.int64)
    gy = np.arange(GRID_Y0, S, GRID_PITCH, dtype=np.int64)
    lin1 = (gy[:, None] * S + gx[None, :]).reshape(-1)
    z1 = np.full(lin1.size, 20.0, np.float32)
    axis = rng.normal(size=3)
    axis /= np.linalg.norm(axis)
    a = 2e-4
    Kx = np.array([[0, -axis[2], axis[1]], [axis[2], 0, -axis[0]], [-axis[1], axis[0], 0]])
    R = np.eye(3) + np.sin(a) * Kx + (1 - np.cos(a)) * (Kx @ Kx)
    P0 = np.hstack([np.eye(3), np.zeros((3, 1))])
    P1 = np.hstack([R, np.array([[0.013], [-0.007], [0.004]])])
    poses = np.stack([P0, P1])
    sc = Scene(width=np.array([S, S], np.int32), height=np.array([S, S], np.int32),
               K=np.array([K, K], np.float32), edge_idx=[lin0, lin1], edge_z=[z0, z1],
               poses_gt=poses, poses_init=poses, pairs=np.array([[0, 1]], np.int32),
               meta=dict(config="max_side_pair"))
    return pack([sc], "max_side_pair")
