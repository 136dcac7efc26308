"""CPU: the oracle's cycle-consistent viewgraph test against closed forms
(identical cameras, a pure translation over a fronto-parallel plane, a depth
map off by a factor of two, cameras facing away) and on a synthetic scene."""
import numpy as np
import pytest

from oracle import viewgraph as ovg
from synth import make
from synth.dense import dense_depth

K = np.array([128.0, 128.0, 79.5, 59.5], np.float32)
W, H = 160, 120


def cam(t=(0.0, 0.0, 0.0), R=None):
    R = np.eye(3) if R is None else R
    return np.concatenate([R, np.asarray(t, np.float64)[:, None]], axis=1)


def plane(z, holes=False):
    d = np.full((H, W), z, np.float32)
    if holes:
        d[::3, ::5] = 0.0
    return d


def grid_points(depth, stride):
    g = depth[::stride, ::stride]
    return int((np.isfinite(g) & (g > 0)).sum())


@pytest.mark.parametrize("stride", [1, 4, 7])
def test_identical_cameras_are_fully_consistent(stride):
    d = plane(5.0, holes=True)
    P = cam(R=np.array([[0.8, 0.0, 0.6], [0.0, 1.0, 0.0], [-0.6, 0.0, 0.8]]), t=(0.3, -0.2, 1.0))
    c, t = ovg.pair_counts(d, d, K, K, P, P, stride)
    assert t == grid_points(d, stride)
    assert c == t


@pytest.mark.parametrize("b,disp", [(0.5, 8), (0.25, 4), (1.0, 16)])
def test_pure_translation_over_a_plane(b, disp):
    """Camera j shifted by b along x over the plane Z = 8: p_ij = p - f b / Z
    (an exact dyadic disparity), the round trip returns p, so exactly the grid
    columns x >= disparity land in j and are consistent."""
    d = plane(8.0)
    c, t = ovg.pair_counts(d, d, K, K, cam(), cam(t=(-b, 0.0, 0.0)), stride=4)
    cols = np.arange(0, W, 4)
    rows = np.arange(0, H, 4).size
    assert t == cols.size * rows
    assert c == int((cols >= disp).sum()) * rows


@pytest.mark.parametrize("b,consistent", [(0.25, True), (0.5, False)])
def test_depth_off_by_two_moves_the_round_trip_by_half_the_disparity(b, consistent):
    """With Z_j = 2 Z_i the back projection lands at x - f b / (2 Z): 2 px
    (consistent, tau = 3) for b = 0.25, 4 px (not) for b = 0.5."""
    c, t = ovg.pair_counts(plane(8.0), plane(16.0), K, K, cam(), cam(t=(-b, 0.0, 0.0)),
                           stride=4)
    disp = int(128 * b / 8)
    cols = np.arange(0, W, 4)
    inside = int((cols >= disp).sum()) * np.arange(0, H, 4).size
    assert c == (inside if consistent else 0)


def test_cameras_facing_away_share_nothing():
    Rb = np.diag([-1.0, 1.0, -1.0])            # turned half a revolution about y
    c, t = ovg.pair_counts(plane(5.0), plane(5.0), K, K, cam(), cam(R=Rb, t=(0, 0, -1.0)), 4)
    assert t > 0 and c == 0


def test_thresholds_decide_validity():
    d = plane(8.0)
    P = [cam(), cam(t=(-0.5, 0.0, 0.0))]
    frac = 38 / 40                              # columns x >= 8 of the stride-4 grid
    for mf, want in ((frac - 1e-9, True), (frac + 1e-9, False)):
        cand, cons, tot, valid = ovg.build([d, d], np.stack([K, K]), P, [0, 0], stride=4,
                                           min_fraction=mf)
        assert valid[0] == want
    # a tighter tau drops nothing here (the round trip is exact up to rounding)
    _, cons2, _, _ = ovg.build([d, d], np.stack([K, K]), P, [0, 0], stride=4, tau=1e-6)
    assert cons2[0] == cons[0]


def test_ring_scene_links_neighbours_not_opposites():
    """Eight cameras on a ring inside the room: neighbours (45 degrees apart)
    are linked, opposite cameras (180 degrees) are not."""
    p = make("c2")
    depth = dense_depth(p)
    maps = [depth[p.view_offset[v]:p.view_offset[v + 1]].reshape(p.height[v], p.width[v])
            for v in range(p.n_views)]
    cand, cons, tot, valid = ovg.build(maps, p.K, p.poses_gt, p.scene_of_view, stride=8)
    link = {(int(i), int(j)): bool(v) for (i, j), v in zip(cand, valid)}
    for i in range(8):
        assert link[tuple(sorted((i, (i + 1) % 8)))]
        assert not link[tuple(sorted((i, (i + 4) % 8)))]
    assert np.all(tot > 0)
