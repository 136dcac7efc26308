"""GPU: the hand-written adjoint behind torch.autograd.Function, against
central finite differences of the FP64 oracle and against plain torch
autograd of the same forward (the differentiation workload)."""
import numpy as np
import pytest
import torch

from oracle import cost as ocost
from synth.scenes import pack
from tests.gpu_helpers import problem, rel_norm_err, say

pytestmark = pytest.mark.gpu


def sub_problem(prob, views):
    """The first scene restricted to `views`, with all ordered pairs among them."""
    from synth import fixtures
    idx = list(views)
    pairs = [(a, b) for a in range(len(idx)) for b in range(len(idx)) if a != b]
    return fixtures.problem_from_maps(prob.width[idx], prob.height[idx], prob.K[idx],
                                      [prob.edge_map(v) for v in idx],
                                      [prob.depth_map(v) for v in idx], prob.poses_init[idx],
                                      pairs, name="sub")


def test_autograd_function_fused_and_recompute(gpu):
    from paper_2607_00579_amd.api import EdgeCostFn, EdgePlan
    p = problem("c2")
    plan = EdgePlan.from_problem(p)
    poses = torch.from_numpy(p.poses_init.copy()).cuda()
    grads = []
    for mode in ("fused", "recompute"):
        xi = torch.zeros(p.n_views, 6, dtype=torch.float64, device="cuda", requires_grad=True)
        loss = EdgeCostFn.apply(xi, plan, poses, 10.0, mode)
        (3.0 * loss.sum()).backward()
        grads.append(xi.grad.detach().clone())
    assert torch.equal(grads[0], grads[1])
    ref = ocost.OracleProblem(p).evaluate(p.poses_init, 10.0)
    assert rel_norm_err(grads[0].cpu().numpy(), 3.0 * ref["grad"], axis=1) < 1e-4


def test_adjoint_vs_central_differences_c3_views(gpu):
    """Frozen-branch central differences (h = 1e-6, FP64 oracle) on four views
    of the differentiation workload and all 12 ordered pairs among them."""
    from paper_2607_00579_amd.api import EdgeCostFn, EdgePlan
    q = sub_problem(problem("c3"), [0, 1, 2, 3])
    plan = EdgePlan.from_problem(q)
    xi = torch.zeros(q.n_views, 6, dtype=torch.float64, device="cuda", requires_grad=True)
    poses = torch.from_numpy(q.poses_init.copy()).cuda()
    EdgeCostFn.apply(xi, plan, poses, 10.0).sum().backward()
    g = xi.grad.cpu().numpy()
    op = ocost.OracleProblem(q)
    fd = ocost.fd_gradient(op, q.poses_init, 10.0, h=1e-6)
    e_t = rel_norm_err(g[:, :3], fd[:, :3], axis=1)
    e_r = rel_norm_err(g[:, 3:], fd[:, 3:], axis=1)
    say(f"c3 sub: adjoint vs central differences: t {e_t:.2e} r {e_r:.2e}")
    assert e_t < 1e-4 and e_r < 1e-4


def test_c3_vs_oracle_and_torch_autograd(gpu):
    """Full differentiation workload (32 views, 992 pairs): fused adjoint vs the
    FP64 oracle and vs torch autograd of the plain forward (float64 and float32)
    on the same GPU, with the same distance fields."""
    from paper_2607_00579_amd.api import EdgePlan
    from paper_2607_00579_amd.autograd_baseline import TorchEdgeCost
    p = problem("c3")
    plan = EdgePlan.from_problem(p, keep_fields=True)
    poses = torch.from_numpy(p.poses_init.copy()).cuda()
    g = plan.cost(poses, 10.0, grad=True)
    g_gpu = g["grad"].cpu().numpy()
    loss_gpu = g["loss"].cpu().numpy()
    ref = ocost.OracleProblem(p).evaluate(p.poses_init, 10.0)
    e_or = rel_norm_err(g_gpu, ref["grad"], axis=1)
    us, vs, zs, offs = [], [], [], [0]
    for v in range(p.n_views):
        ys, xs = np.nonzero(p.edge_map(v))
        us.append(xs)
        vs.append(ys)
        zs.append(p.depth_map(v)[ys, xs])
        offs.append(offs[-1] + xs.size)
    res = {}
    for dt in (torch.float64, torch.float32):
        tf = TorchEdgeCost(p.width, p.height, p.K, p.scene_of_view, p.pairs, p.scene_of_pair,
                           np.concatenate(us), np.concatenate(vs), np.concatenate(zs), offs,
                           plan.dtf, p.view_offset[:-1], device="cuda", dtype=dt,
                           batch_residuals=1 << 23)
        o = tf.loss_and_grad(poses, 10.0)
        res[dt] = (o["loss"].double().cpu().numpy(), o["grad"].cpu().numpy())
    e64 = rel_norm_err(g_gpu, res[torch.float64][1], axis=1)
    e32 = rel_norm_err(g_gpu, res[torch.float32][1], axis=1)
    say(f"c3: fused vs oracle {e_or:.2e}, vs torch autograd f64 {e64:.2e}, f32 {e32:.2e}; "
        f"loss {loss_gpu} oracle {ref['loss']}")
    assert abs(loss_gpu[0] - ref["loss"][0]) < 1e-4 * abs(ref["loss"][0])
    assert e_or < 1e-4
    assert e64 < 1e-4
    # float32 autograd rounds the projected coordinate itself, which moves
    # cell-boundary residuals: a looser bound
    assert e32 < 5e-3
