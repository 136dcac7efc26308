"""Dense depth maps for the synthetic scenes (inputs of the viewgraph
construction, which projects a grid of pixels rather than edge pixels).

The wireframe scenes have depth only at their edge pixels, so every view also
looks at the inside of a room, the box [-h, h]^3 around the scene (the cameras
stand inside it): a pixel off the wireframe gets the z-depth of the wall its
ray meets, an edge pixel keeps its own depth.  Rendering only: a ray-box exit
distance per pixel, no arithmetic of the method.
"""
from __future__ import annotations

import numpy as np


def room_depth_map(P: np.ndarray, K: np.ndarray, W: int, H: int, half: float = 4.0) -> np.ndarray:
    """z-depth of the room walls for camera P = [R | t] (world->camera)."""
    R, t = P[:, :3].astype(np.float64), P[:, 3].astype(np.float64)
    c = -R.T @ t
    fx, fy, cx, cy = (float(x) for x in K)
    ys, xs = np.mgrid[0:H, 0:W].astype(np.float64)
    # ray with camera-frame z = 1, in world coordinates
    d_cam = np.stack([(xs - cx) / fx, (ys - cy) / fy, np.ones_like(xs)], axis=-1)
    d = d_cam @ R                                    # rows: R^T d_cam
    t_exit = np.full((H, W), np.inf)
    for k in range(3):
        dk = d[..., k]
        with np.errstate(divide="ignore", invalid="ignore"):
            tk = np.where(dk > 0, (half - c[k]) / dk, np.where(dk < 0, (-half - c[k]) / dk, np.inf))
        t_exit = np.minimum(t_exit, tk)
    return t_exit.astype(np.float32)                 # z-depth: the ray has unit camera z


def dense_depth(prob, poses=None, half: float = 4.0, sigma: float = 0.0, seed: int = 0):
    """Packed dense depth of every view (same layout as prob.depth_flat):
    room walls rendered with `poses` (default: the ground truth), the
    wireframe's own depth at edge pixels, optional multiplicative Gaussian
    noise Z (1 + sigma N(0, 1)) on the wall pixels."""
    poses = prob.poses_gt if poses is None else poses
    rng = np.random.default_rng(seed)
    out = np.zeros(int(prob.view_offset[-1]), np.float32)
    for v in range(prob.n_views):
        W, H = int(prob.width[v]), int(prob.height[v])
        z = room_depth_map(poses[v], prob.K[v], W, H, half)
        if sigma > 0:
            z = (z * (1.0 + sigma * rng.standard_normal(z.shape))).astype(np.float32)
        e = prob.edge_map(v) != 0
        z[e] = prob.depth_map(v)[e]
        a = int(prob.view_offset[v])
        out[a:a + W * H] = z.ravel()
    return out
