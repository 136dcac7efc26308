"""The oracle's analytic gradient against torch autograd of an independently
written forward (float64, CPU)."""
import numpy as np
import pytest
import torch

from oracle import cost
from paper_2607_00579_amd.autograd_baseline import TorchEdgeCost
from synth import make


def torch_form(p, op, dtype=torch.float64, batch=1 << 20, **kw):
    us, vs, zs, offs = [], [], [], [0]
    for v in range(p.n_views):
        e = p.edge_map(v)
        ys, xs = np.nonzero(e)
        us.append(xs)
        vs.append(ys)
        zs.append(p.depth_map(v)[ys, xs])
        offs.append(offs[-1] + xs.size)
    D = np.concatenate([op.D[v].reshape(-1) for v in range(p.n_views)])
    doff = np.concatenate([[0], np.cumsum([op.D[v].size for v in range(p.n_views)])[:-1]])
    return TorchEdgeCost(p.width, p.height, p.K, p.scene_of_view, p.pairs, p.scene_of_pair,
                         np.concatenate(us), np.concatenate(vs), np.concatenate(zs), offs, D, doff,
                         dtype=dtype, batch_residuals=batch, **kw)


@pytest.mark.parametrize("lam", [10.0, 2.5])
@pytest.mark.parametrize("norm_mode", [0, 1])
def test_c1_autograd_matches_analytic(lam, norm_mode):
    p = make("c1")
    op = cost.OracleProblem(p)
    prm = cost.CostParams(norm_mode=norm_mode)
    r = op.evaluate(p.poses_init, lam, prm)
    tf = torch_form(p, op, norm_mode=norm_mode)
    out = tf.loss_and_grad(p.poses_init, lam)
    assert np.allclose(out["loss"].numpy(), r["loss"], rtol=1e-12)
    g = out["grad"].numpy()
    err = np.abs(g - r["grad"]).max() / np.abs(r["grad"]).max()
    assert err < 1e-10, err


def test_c2_subset_autograd_matches_analytic():
    """Several pairs, batches split mid-list."""
    p = make("c2")
    op = cost.OracleProblem(p)
    r = op.evaluate(p.poses_init, 10.0)
    tf = torch_form(p, op, batch=50000)
    assert len(tf.batches) > 5
    out = tf.loss_and_grad(p.poses_init, 10.0, want_pairs=True)
    assert np.array_equal(out["n"].numpy(), r["n"])
    assert np.allclose(out["S"].numpy(), r["S"], rtol=1e-12)
    err = np.abs(out["grad"].numpy() - r["grad"]).max() / np.abs(r["grad"]).max()
    assert err < 1e-10, err


@pytest.mark.parametrize("lam", [10.0, 2.5])
def test_c1_focal_and_depth_autograd_matches_analytic(lam):
    p = make("c1")
    op = cost.OracleProblem(p)
    r = op.evaluate(p.poses_init, lam)
    tf = torch_form(p, op)
    out = tf.loss_and_grad(p.poses_init, lam, intrinsics_depth=True)
    gf = out["grad_focal"].numpy()
    assert np.abs(gf - r["grad_focal"]).max() < 1e-10 * np.abs(r["grad_focal"]).max()
    gz = out["grad_depth"].numpy()
    want = np.concatenate([r["grad_depth"][v] for v in range(p.n_views)])
    assert np.abs(gz - want).max() < 1e-10 * np.abs(want).max()
    # the pose gradient is unchanged by lifting inside the graph
    assert np.abs(out["grad"].numpy() - r["grad"]).max() < 1e-10 * np.abs(r["grad"]).max()
