"""Seeded synthetic wireframe scenes: the inputs that both the FP64 oracle and
the HIP path consume.

This module produces inputs only.  It holds none of the edge-alignment method's
arithmetic (no distance transform, no cost, no gradient, no pose update); the
one piece of geometry it needs is a pinhole camera to rasterize 3-D segments
into 1-px edge maps with a z-buffered depth, which is scene synthesis.  Random
rotations are drawn through scipy so that no SE(3) code is shared with either
side.

Scene recipe (stand-in for the paper's 3DFM outputs, Sec. 3 "Method": the
estimate G = {(K_i, P_i, Z_i)} plus edge maps E_i):
  * intrinsics fx = fy = 0.8 W, principal point at the image centre
    cx = (W - 1) / 2, cy = (H - 1) / 2 (integer pixel centres);
  * world->camera poses [R | t] with OpenCV axes (x right, y down, z forward),
    cameras looking at a target point;
  * 3-D line segments rasterized per view as 8-connected 1-px lines from
    n = ceil(max(|du|, |dv|)) + 1 screen-space samples rounded to the nearest
    pixel; depth by perspective-correct interpolation (1/z linear in screen
    space) with a per-pixel z-buffer; depth 0 off the edges (never read);
  * multiplicative Gaussian depth noise Z (1 + sigma N(0,1)), optional uniform
    depth outliers;
  * initial poses = ground truth with a rotation of exactly `rot_deg` about a
    uniform random axis (applied on the left of R) and the camera centre moved
    by `trans_pct` % of its distance to the look-at point in a uniform random
    direction.
"""
from __future__ import annotations

import math
import os
from dataclasses import dataclass, field

import numpy as np
from scipy.spatial.transform import Rotation

GENERATOR_VERSION = 1


# ----------------------------------------------------------------------------
# data containers
# ----------------------------------------------------------------------------
@dataclass
class Scene:
    """One scene: V views, their edge maps / depth maps, poses and pair list."""
    width: np.ndarray          # (V,) int32
    height: np.ndarray         # (V,) int32
    K: np.ndarray              # (V, 4) float32 (fx, fy, cx, cy)
    edge_idx: list             # V arrays int64: sorted linear indices y*W + x of edge pixels
    edge_z: list               # V arrays float32: depth at those pixels (0 elsewhere)
    poses_gt: np.ndarray       # (V, 3, 4) float64 world->camera
    poses_init: np.ndarray     # (V, 3, 4) float64 world->camera
    pairs: np.ndarray          # (D, 2) int32 directed (src, tgt), view ids local to the scene
    meta: dict = field(default_factory=dict)

    @property
    def n_views(self) -> int:
        return int(self.width.shape[0])

    def edge_map(self, v: int) -> np.ndarray:
        e = np.zeros(int(self.width[v]) * int(self.height[v]), np.uint8)
        e[self.edge_idx[v]] = 255
        return e.reshape(self.height[v], self.width[v])

    def depth_map(self, v: int) -> np.ndarray:
        d = np.zeros(int(self.width[v]) * int(self.height[v]), np.float32)
        d[self.edge_idx[v]] = self.edge_z[v]
        return d.reshape(self.height[v], self.width[v])


@dataclass
class Problem:
    """Several scenes concatenated into flat, packed arrays (global view ids)."""
    scenes: list
    width: np.ndarray          # (V,) int32
    height: np.ndarray         # (V,) int32
    K: np.ndarray              # (V, 4) float32
    scene_of_view: np.ndarray  # (V,) int32
    view_offset: np.ndarray    # (V + 1,) int64 pixel offsets into the packed maps
    edge_flat: np.ndarray      # (sum H W,) uint8
    depth_flat: np.ndarray     # (sum H W,) float32
    poses_gt: np.ndarray       # (V, 3, 4) float64
    poses_init: np.ndarray     # (V, 3, 4) float64
    pairs: np.ndarray          # (D, 2) int32 global view ids
    scene_of_pair: np.ndarray  # (D,) int32
    name: str = ""

    @property
    def n_views(self) -> int:
        return int(self.width.shape[0])

    @property
    def n_scenes(self) -> int:
        return len(self.scenes)

    @property
    def n_pairs(self) -> int:
        return int(self.pairs.shape[0])

    def edge_map(self, v: int) -> np.ndarray:
        a, b = self.view_offset[v], self.view_offset[v + 1]
        return self.edge_flat[a:b].reshape(self.height[v], self.width[v])

    def depth_map(self, v: int) -> np.ndarray:
        a, b = self.view_offset[v], self.view_offset[v + 1]
        return self.depth_flat[a:b].reshape(self.height[v], self.width[v])

    def edge_counts(self) -> np.ndarray:
        return np.array([int(np.count_nonzero(self.edge_map(v))) for v in range(self.n_views)],
                        dtype=np.int64)

    def residual_count(self) -> int:
        """Residuals per iteration: every source edge pixel of every directed pair."""
        cnt = self.edge_counts()
        return int(cnt[self.pairs[:, 0]].sum())


def pack(scenes: list, name: str = "") -> Problem:
    sizes = [int(w) * int(h) for sc in scenes for w, h in zip(sc.width, sc.height)]
    offs = np.zeros(len(sizes) + 1, np.int64)
    offs[1:] = np.cumsum(sizes)
    edge_flat = np.zeros(int(offs[-1]), np.uint8)
    depth_flat = np.zeros(int(offs[-1]), np.float32)
    sov, prs, sop = [], [], []
    base = 0
    for s, sc in enumerate(scenes):
        V = sc.n_views
        for v in range(V):
            idx = sc.edge_idx[v] + offs[base + v]
            edge_flat[idx] = 255
            depth_flat[idx] = sc.edge_z[v]
        sov.append(np.full(V, s, np.int32))
        prs.append(sc.pairs.astype(np.int64) + base)
        sop.append(np.full(sc.pairs.shape[0], s, np.int32))
        base += V
    return Problem(
        scenes=scenes,
        width=np.concatenate([sc.width for sc in scenes]).astype(np.int32),
        height=np.concatenate([sc.height for sc in scenes]).astype(np.int32),
        K=np.concatenate([sc.K for sc in scenes]).astype(np.float32),
        scene_of_view=np.concatenate(sov),
        view_offset=offs,
        edge_flat=edge_flat,
        depth_flat=depth_flat,
        poses_gt=np.concatenate([sc.poses_gt for sc in scenes]).astype(np.float64),
        poses_init=np.concatenate([sc.poses_init for sc in scenes]).astype(np.float64),
        pairs=np.concatenate(prs).astype(np.int32),
        scene_of_pair=np.concatenate(sop),
        name=name,
    )


# ----------------------------------------------------------------------------
# cameras
# ----------------------------------------------------------------------------
def intrinsics(W: int, H: int) -> np.ndarray:
    return np.array([0.8 * W, 0.8 * W, (W - 1) / 2.0, (H - 1) / 2.0], np.float32)


def look_at(center: np.ndarray, target: np.ndarray) -> np.ndarray:
    """World->camera [R | t] for a camera at `center` looking at `target`,
    OpenCV axes, world +y pointing up in the image (camera y down)."""
    z = target - center
    z = z / np.linalg.norm(z)
    x = np.cross(z, np.array([0.0, 1.0, 0.0]))
    x = x / np.linalg.norm(x)
    y = np.cross(z, x)
    R = np.stack([x, y, z])
    t = -R @ center
    return np.concatenate([R, t[:, None]], axis=1)


def perturb_pose(P: np.ndarray, target: np.ndarray, rot_deg: float, trans_pct: float,
                 rng: np.random.Generator) -> np.ndarray:
    R, t = P[:, :3], P[:, 3]
    c = -R.T @ t
    axis = rng.normal(size=3)
    axis /= np.linalg.norm(axis)
    Rn = Rotation.from_rotvec(axis * math.radians(rot_deg)).as_matrix()
    R2 = Rn @ R
    d = rng.normal(size=3)
    d /= np.linalg.norm(d)
    c2 = c + (trans_pct / 100.0) * np.linalg.norm(c - target) * d
    return np.concatenate([R2, (-R2 @ c2)[:, None]], axis=1)


def ring_cameras(n: int, radius: float = 3.0):
    centers = []
    for k in range(n):
        th = 2.0 * math.pi * k / n
        centers.append(np.array([radius * math.sin(th), 0.0, radius * math.cos(th)]))
    return centers


# ----------------------------------------------------------------------------
# rasterization (scene synthesis)
# ----------------------------------------------------------------------------
def rasterize(p0: np.ndarray, p1: np.ndarray, P: np.ndarray, K: np.ndarray, W: int, H: int):
    """Rasterize world segments p0->p1 (N, 3) for the camera P (world->camera)
    and K.  Returns the sorted linear indices y*W + x of the edge pixels and the
    z-buffered (nearest) depth at each of them."""
    R, t = P[:, :3], P[:, 3]
    fx, fy, cx, cy = (float(k) for k in K)
    a = p0 @ R.T + t
    b = p1 @ R.T + t
    keep = (a[:, 2] > 0.05) & (b[:, 2] > 0.05)
    a, b = a[keep], b[keep]
    ua, va = fx * a[:, 0] / a[:, 2] + cx, fy * a[:, 1] / a[:, 2] + cy
    ub, vb = fx * b[:, 0] / b[:, 2] + cx, fy * b[:, 1] / b[:, 2] + cy
    span = np.maximum(np.abs(ub - ua), np.abs(vb - va))
    span = np.minimum(span, 4.0 * (W + H))  # guard against grazing segments
    n = np.ceil(span).astype(np.int64) + 1
    n = np.maximum(n, 2)
    seg = np.repeat(np.arange(n.shape[0]), n)
    start = np.cumsum(n) - n
    k = np.arange(seg.shape[0]) - start[seg]
    s = k / (n[seg] - 1).astype(np.float64)
    u = ua[seg] + s * (ub - ua)[seg]
    v = va[seg] + s * (vb - va)[seg]
    inv_z = (1.0 - s) / a[seg, 2] + s / b[seg, 2]
    z = 1.0 / inv_z
    px = np.rint(u).astype(np.int64)
    py = np.rint(v).astype(np.int64)
    inside = (px >= 0) & (px < W) & (py >= 0) & (py < H)
    px, py, z = px[inside], py[inside], z[inside]
    lin = py * W + px
    order = np.lexsort((z, lin))
    lin, z = lin[order], z[order]
    first = np.ones(lin.shape[0], bool)
    first[1:] = lin[1:] != lin[:-1]
    return lin[first], z[first].astype(np.float32)


def add_depth_noise(z: np.ndarray, sigma: float, outlier_frac: float,
                    rng: np.random.Generator) -> np.ndarray:
    vals = z.astype(np.float64) * (1.0 + sigma * rng.normal(size=z.size))
    if outlier_frac > 0 and z.size:
        lo, hi = float(z.min()), float(z.max())
        m = rng.random(z.size) < outlier_frac
        vals[m] = rng.uniform(lo, hi, size=int(m.sum()))
    return vals.astype(np.float32)


def uniform_cube_segments(n: int, rng: np.random.Generator):
    p0 = rng.uniform(-0.5, 0.5, size=(n, 3))
    p1 = rng.uniform(-0.5, 0.5, size=(n, 3))
    return p0, p1


def short_segments(n: int, length: float, rng: np.random.Generator):
    c = rng.uniform(-0.5, 0.5, size=(n, 3))
    d = rng.normal(size=(n, 3))
    d /= np.linalg.norm(d, axis=1, keepdims=True)
    return c - 0.5 * length * d, c + 0.5 * length * d


def all_ordered_pairs(V: int) -> np.ndarray:
    return np.array([(i, j) for i in range(V) for j in range(V) if i != j], np.int32).reshape(-1, 2)


def knn_pairs(poses: np.ndarray, k: int) -> np.ndarray:
    """(i, j) for the k nearest camera centres j of each i (ties by index)."""
    R, t = poses[:, :, :3], poses[:, :, 3]
    c = -np.einsum("vji,vj->vi", R, t)
    V = c.shape[0]
    out = []
    for i in range(V):
        d = np.linalg.norm(c - c[i], axis=1)
        d[i] = np.inf
        order = np.lexsort((np.arange(V), d))
        for j in order[:k]:
            out.append((i, int(j)))
    return np.asarray(out, np.int32)


def build_scene(segs, centers, targets, W, H, rot_deg, trans_pct, depth_sigma, outlier_frac,
                pairs, rng, meta) -> Scene:
    V = len(centers)
    K = intrinsics(W, H)
    gt, init, idxs, zs = [], [], [], []
    for k in range(V):
        P = look_at(centers[k], targets[k])
        gt.append(P)
        lin, z = rasterize(segs[0], segs[1], P, K, W, H)
        idxs.append(lin)
        zs.append(add_depth_noise(z, depth_sigma, outlier_frac, rng))
    for k in range(V):
        init.append(perturb_pose(gt[k], targets[k], rot_deg, trans_pct, rng))
    init = np.stack(init)
    if pairs is None:
        pairs = all_ordered_pairs(V)
    elif isinstance(pairs, tuple) and pairs[0] == "knn":
        pairs = knn_pairs(init, pairs[1])
    meta = dict(meta)
    meta["edge_px_per_view"] = [int(i.size) for i in idxs]
    meta["generator_version"] = GENERATOR_VERSION
    return Scene(
        width=np.full(V, W, np.int32), height=np.full(V, H, np.int32),
        K=np.tile(K, (V, 1)), edge_idx=idxs, edge_z=zs,
        poses_gt=np.stack(gt), poses_init=init, pairs=np.asarray(pairs, np.int32), meta=meta)


def _mean_edges(segs, centers, targets, W, H, probe_views) -> float:
    K = intrinsics(W, H)
    tot = 0
    for k in probe_views:
        lin, _ = rasterize(segs[0], segs[1], look_at(centers[k], targets[k]), K, W, H)
        tot += int(lin.size)
    return tot / len(probe_views)


# ----------------------------------------------------------------------------
# the five workloads
# ----------------------------------------------------------------------------
def config_c1(seed: int = 1) -> Problem:
    """2 views 160x120, 200 cube segments, noise 2 deg / 2 %, depth 1 %."""
    rng = np.random.default_rng(seed)
    segs = uniform_cube_segments(200, rng)
    centers = ring_cameras(2)
    targets = [np.zeros(3)] * 2
    sc = build_scene(segs, centers, targets, 160, 120, 2.0, 2.0, 0.01, 0.0, None, rng,
                     dict(config="c1", seed=seed, n_segments=200))
    return pack([sc], "c1")


def config_c2(seed: int = 2) -> Problem:
    """8 views 518x392, 2000 cube segments, 56 ordered pairs, noise 3 deg / 5 %."""
    rng = np.random.default_rng(seed)
    segs = uniform_cube_segments(2000, rng)
    centers = ring_cameras(8)
    targets = [np.zeros(3)] * 8
    sc = build_scene(segs, centers, targets, 518, 392, 3.0, 5.0, 0.01, 0.0, None, rng,
                     dict(config="c2", seed=seed, n_segments=2000))
    return pack([sc], "c2")


def _calibrated_cube_scene(rng_seg, rng, n_views, W, H, target_px, rot_deg, trans_pct,
                           depth_sigma, step, tol, meta, half=1.0, max_iter=8):
    """Pick the segment count (a multiple of `step`) whose mean edge px/view
    on probe views is within `tol` of `target_px`; segments for count n are the
    first n of one seeded stream, so the search is reproducible."""
    centers = ring_cameras(n_views)
    targets = [np.zeros(3)] * n_views
    pool = uniform_cube_segments(100000, rng_seg)
    pool = (pool[0] * (2.0 * half), pool[1] * (2.0 * half))
    probe = sorted(set([0, n_views // 3, (2 * n_views) // 3]))
    n = max(step, int(round(target_px / (0.17 * W) / step)) * step)
    for _ in range(max_iter):
        m = _mean_edges((pool[0][:n], pool[1][:n]), centers, targets, W, H, probe)
        if abs(m - target_px) <= tol * target_px:
            break
        n_new = max(step, int(round(n * target_px / max(m, 1.0) / step)) * step)
        if n_new == n:
            break
        n = min(n_new, pool[0].shape[0])
    segs = (pool[0][:n], pool[1][:n])
    meta = dict(meta, n_segments=n, cube_half=half)
    return build_scene(segs, centers, targets, W, H, rot_deg, trans_pct, depth_sigma, 0.0,
                       None, rng, meta)


def config_c3(seed: int = 3) -> Problem:
    """32 views 518x518, all 992 ordered pairs, ~30k edge px/view."""
    rng = np.random.default_rng(seed)
    rng_seg = np.random.default_rng([seed, 1])
    sc = _calibrated_cube_scene(rng_seg, rng, 32, 518, 518, 30000, 3.0, 5.0, 0.01, 10, 0.1,
                                dict(config="c3", seed=seed), half=1.0)
    return pack([sc], "c3")


C4_RESOLUTIONS = [(256, 192), (518, 392), (768, 576), (1024, 768)]


def c4_scene_spec(s: int) -> dict:
    rng = np.random.default_rng([4, s])
    n = int(rng.integers(4, 49))
    W, H = C4_RESOLUTIONS[int(rng.integers(0, 4))]
    target = float(rng.uniform(5000, 60000))
    target = min(target, 0.25 * W * H)
    noise = float(rng.uniform(1.0, 5.0))
    return dict(n_views=n, W=W, H=H, target_px=target, rot_deg=noise, trans_pct=noise,
                seed_seq=[4, s])


def _c4_scene(s: int) -> Scene:
    spec = c4_scene_spec(s)
    rng = np.random.default_rng([4, s, 1])
    rng_seg = np.random.default_rng([4, s, 2])
    return _calibrated_cube_scene(rng_seg, rng, spec["n_views"], spec["W"], spec["H"],
                                  spec["target_px"], spec["rot_deg"], spec["trans_pct"], 0.01,
                                  10, 0.1, dict(config="c4", scene=s, **spec), half=1.0)


def config_c4(n_scenes: int = 64, workers: int | None = None) -> Problem:
    """64 independent scenes of uneven size (views U{4..48}, four resolutions,
    edge px/view U(5k, 60k) capped at 25 % of the image, pose noise U(1, 5) deg).
    Every scene has its own seed, so generating them in worker processes gives
    the same arrays as generating them in order."""
    if workers is None:
        workers = min(16, os.cpu_count() or 1)
    if workers > 1 and n_scenes > 1:
        import multiprocessing as mp
        from concurrent.futures import ProcessPoolExecutor
        # spawn: the workers are fresh interpreters, whatever the parent holds
        with ProcessPoolExecutor(max_workers=workers, mp_context=mp.get_context("spawn")) as ex:
            scenes = list(ex.map(_c4_scene, range(n_scenes)))
    else:
        scenes = [_c4_scene(s) for s in range(n_scenes)]
    return pack(scenes, "c4")


def config_c5(seed: int = 5, n_views: int = 200, n_segments: int = 20000,
              seg_length: float | None = None, target_px: float = 80000.0) -> Problem:
    """200 views 1024x768 on a seeded random walk, 20k short segments, 10
    nearest-camera pairs per view, depth noise 2 % + 10 % uniform outliers."""
    rng = np.random.default_rng(seed)
    W, H = 1024, 768
    centers, targets = [], []
    th, r, y = 0.0, 3.0, 0.0
    for k in range(n_views):
        if k > 0:
            th = th + 2.0 * math.pi / n_views + rng.normal(0.0, 0.005)
            r = float(np.clip(r + rng.normal(0.0, 0.02), 2.5, 3.5))
            y = float(np.clip(y + rng.normal(0.0, 0.02), -0.5, 0.5))
        centers.append(np.array([r * math.sin(th), y, r * math.cos(th)]))
        targets.append(rng.normal(0.0, 0.05, size=3))
    seg_rng = np.random.default_rng([seed, 1])
    cen = seg_rng.uniform(-0.5, 0.5, size=(n_segments, 3))
    dirs = seg_rng.normal(size=(n_segments, 3))
    dirs /= np.linalg.norm(dirs, axis=1, keepdims=True)
    probe = [0, n_views // 2]
    if seg_length is None:
        seg_length = 0.05
        for _ in range(5):
            segs = (cen - 0.5 * seg_length * dirs, cen + 0.5 * seg_length * dirs)
            m = _mean_edges(segs, centers, targets, W, H, probe)
            if abs(m - target_px) <= 0.05 * target_px:
                break
            seg_length *= target_px / max(m, 1.0)
    segs = (cen - 0.5 * seg_length * dirs, cen + 0.5 * seg_length * dirs)
    sc = build_scene(segs, centers, targets, W, H, 3.0, 5.0, 0.02, 0.10, ("knn", 10), rng,
                     dict(config="c5", seed=seed, n_segments=n_segments,
                          seg_length=seg_length))
    return pack([sc], "c5")


CONFIGS = {"c1": config_c1, "c2": config_c2, "c3": config_c3, "c4": config_c4, "c5": config_c5}


def make(name: str, cache_dir: str | None = None, **kw) -> Problem:
    """Build a workload; with `cache_dir` (or $EPO_SYNTH_CACHE) the packed
    arrays are stored once as .npz and reloaded (no pickles)."""
    cache_dir = cache_dir or os.environ.get("EPO_SYNTH_CACHE")
    if cache_dir and not kw:
        path = os.path.join(cache_dir, f"{name}_v{GENERATOR_VERSION}.npz")
        if os.path.exists(path):
            return load_problem(path)
        prob = CONFIGS[name]()
        os.makedirs(cache_dir, exist_ok=True)
        save_problem(prob, path)
        return prob
    return CONFIGS[name](**kw)


_PACKED = ("width", "height", "K", "scene_of_view", "view_offset", "edge_flat", "depth_flat",
           "poses_gt", "poses_init", "pairs", "scene_of_pair")


def save_problem(prob: Problem, path: str) -> None:
    tmp = path + ".tmp.npz"
    np.savez(tmp, **{k: getattr(prob, k) for k in _PACKED}, name=np.array(prob.name))
    os.replace(tmp, path)


def load_problem(path: str) -> Problem:
    with np.load(path, allow_pickle=False) as z:
        d = {k: z[k] for k in _PACKED}
        name = str(z["name"])
    return Problem(scenes=[], name=name, **d)


def subset_scenes(prob: Problem, idx) -> Problem:
    return pack([prob.scenes[i] for i in idx], prob.name + "_sub")
