"""GPU: viewgraph estimation by cycle-consistent reprojection against the
oracle: every candidate pair's consistent and total counts bit-exact, the
validity flags, and the directed pair list built from them."""
import numpy as np
import pytest
import torch

from oracle import viewgraph as ovg
from synth.dense import dense_depth
from synth.scenes import config_c1, config_c2, pack
from tests.gpu_helpers import problem, say

pytestmark = pytest.mark.gpu


def run_both(p, poses, depth, **kw):
    from paper_2607_00579_amd.api import build_viewgraph
    g = build_viewgraph(torch.from_numpy(depth).cuda(), p.width, p.height, p.K, p.view_offset,
                        torch.from_numpy(np.ascontiguousarray(poses)).cuda(), p.scene_of_view,
                        **kw)
    maps = [depth[p.view_offset[v]:p.view_offset[v + 1]].reshape(p.height[v], p.width[v])
            for v in range(p.n_views)]
    cand, cons, tot, valid = ovg.build(maps, p.K, poses, p.scene_of_view, **kw)
    assert np.array_equal(g["candidates"], cand)
    gc, gt = g["consistent"].cpu().numpy(), g["total"].cpu().numpy()
    assert np.array_equal(gt, tot)
    assert np.array_equal(gc, cons), np.flatnonzero(gc != cons)
    assert np.array_equal(g["valid"].cpu().numpy(), valid)
    kept = cand[valid]
    want_pairs = np.concatenate([kept, kept[:, ::-1]]) if kept.size else np.zeros((0, 2))
    assert np.array_equal(g["pairs"], want_pairs)
    return g, valid


@pytest.mark.parametrize("which", ["gt", "init"])
def test_ring_scene_counts_equal_the_oracle(gpu, which):
    p = problem("c2")
    poses = p.poses_gt if which == "gt" else p.poses_init
    depth = dense_depth(p, sigma=0.01, seed=3)
    g, valid = run_both(p, poses, depth)
    say(f"c2 viewgraph ({which} poses): {int(valid.sum())} of {valid.size} pairs valid")


def test_two_scenes_other_thresholds(gpu):
    p = pack(list(config_c2().scenes) + list(config_c1().scenes), "c2+c1")
    depth = dense_depth(p)
    run_both(p, p.poses_init, depth, stride=3, tau=1.5, min_fraction=0.3)


def test_many_views(gpu):
    """32 views, 496 candidate pairs."""
    p = problem("c3")
    depth = dense_depth(p, sigma=0.005, seed=1)
    g, valid = run_both(p, p.poses_init, depth, stride=8)
    say(f"c3 viewgraph: {int(valid.sum())} of {valid.size} pairs valid")


def test_viewgraph_feeds_a_plan(gpu):
    """The directed pairs of the valid image pairs make an edge-cost plan."""
    from paper_2607_00579_amd.api import EdgePlan, build_viewgraph
    p = problem("c2")
    depth = dense_depth(p)
    g = build_viewgraph(torch.from_numpy(depth).cuda(), p.width, p.height, p.K, p.view_offset,
                        torch.from_numpy(p.poses_init.copy()).cuda(), p.scene_of_view)
    plan = EdgePlan(p.width, p.height, p.K, p.scene_of_view, p.view_offset, p.edge_flat,
                    p.depth_flat, g["pairs"])
    out = plan.cost(torch.from_numpy(p.poses_init.copy()).cuda(), 10.0, grad=True)
    assert np.isfinite(out["loss"].cpu().numpy()).all()
    assert plan.n_pairs == g["pairs"].shape[0] > 0
