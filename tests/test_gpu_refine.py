"""GPU: focal-scale and per-pixel depth gradients of the joint phase
(f = f0 (1 + gamma), Z = Z0 alpha + beta) against the FP64 oracle, at the
identity and at a seeded non-identity refinement state, through the C-ABI
refinement entry points and the autograd Function."""
import numpy as np
import pytest
import torch

from oracle import cost as ocost
from oracle import sampling as osamp
from tests.gpu_helpers import (check_depth, gather_depth, oracle_index, problem,
                               rel_norm_err, say)

pytestmark = pytest.mark.gpu

TOL = 1e-4


def plan_for(prob, **kw):
    from paper_2607_00579_amd.api import EdgePlan
    return EdgePlan.from_problem(prob, device="cuda:0", **kw)


def run_case(prob, poses, lam, gamma=None, alpha=None, beta=None, sampling=None, options=None):
    """sampling = (budget, seed, step): one sub-sampled step."""
    plan = plan_for(prob, options=options)
    views, idx = oracle_index(prob, plan)
    n = views.size
    z0 = np.zeros(n)
    for v in range(prob.n_views):
        sel = views == v
        ys, xs = np.nonzero(prob.edge_map(v))
        z0[sel] = prob.depth_map(v)[ys, xs].astype(np.float64)[idx[sel]]
    K = prob.K.astype(np.float64).reshape(-1, 4).copy()
    depth = None
    if gamma is not None:
        plan.set_refinement(torch.from_numpy(gamma),
                            None if alpha is None else torch.from_numpy(alpha),
                            None if beta is None else torch.from_numpy(beta))
        # the library's refined values: float32(f0 (1 + gamma)) with the
        # product in float64, float32(Z0 alpha + beta) (Z0 alpha exact)
        K[:, :2] = (prob.K.reshape(-1, 4)[:, :2].astype(np.float64)
                    * (1.0 + gamma)[:, None]).astype(np.float32)
        if alpha is not None:
            z = (z0 * alpha.astype(np.float64) + beta.astype(np.float64)).astype(np.float32)
            depth = {}
            for v in range(prob.n_views):
                sel = views == v
                zv = np.zeros(int(sel.sum()))
                zv[idx[sel]] = z[sel]
                depth[v] = zv.astype(np.float64)
    P = torch.from_numpy(np.ascontiguousarray(poses)).cuda()
    sel = None
    if sampling is not None:
        budget, seed, step = sampling
        plan.set_pair_sampling(budget, seed,
                               torch.full((1,), step, dtype=torch.int32, device="cuda"))
        sel = osamp.selected_pairs(prob.pairs, prob.scene_of_pair, seed, step, budget)
    g = {k: t.cpu().numpy() for k, t in plan.refine(P, lam).items()}
    r = ocost.OracleProblem(prob).evaluate(poses, lam, K=K, depth=depth, selected=sel)
    assert rel_norm_err(g["loss"], r["loss"]) < TOL
    e_t = rel_norm_err(g["grad"][:, :3], r["grad"][:, :3], axis=1)
    e_r = rel_norm_err(g["grad"][:, 3:], r["grad"][:, 3:], axis=1)
    gam = np.zeros(prob.n_views) if gamma is None else gamma
    want_gamma = r["grad_focal"] / (1.0 + gam)
    e_g = rel_norm_err(g["grad_gamma"], want_gamma)
    say(f"{prob.name}: pose grad err t {e_t:.2e} r {e_r:.2e}; focal err {e_g:.2e}")
    assert e_t < TOL and e_r < TOL and e_g < TOL
    want_beta = gather_depth(r["grad_depth"], views, idx, n)
    check_depth(g["grad_beta"], want_beta, f"{prob.name} dL/dbeta")
    check_depth(g["grad_alpha"], z0 * want_beta, f"{prob.name} dL/dalpha")
    assert plan.device_status() == 0
    return plan, g


@pytest.mark.parametrize("name", ["c1", "c2"])
def test_refine_gradients_at_identity(gpu, name):
    p = problem(name)
    plan, g = run_case(p, p.poses_init, 10.0)
    # the refinement variant evaluates the same residual terms and adds them
    # into the same float64 sums in the same order as the pose-only kernel
    # (one residual after the other per thread, the same wave folds), so at
    # the identity refinement loss and pose gradient are bitwise equal
    P = torch.from_numpy(p.poses_init.copy()).cuda()
    o = plan.cost(P, 10.0, grad=True)
    assert np.array_equal(o["loss"].cpu().numpy(), g["loss"])
    assert np.array_equal(o["grad"].cpu().numpy(), g["grad"])


def test_refine_gradients_at_a_refined_state(gpu):
    p = problem("c2")
    rng = np.random.default_rng(11)
    n = sum(int(np.count_nonzero(p.edge_map(v))) for v in range(p.n_views))
    gamma = rng.uniform(-0.02, 0.02, p.n_views)
    alpha = (1.0 + rng.uniform(-0.02, 0.02, n)).astype(np.float32)
    beta = rng.uniform(-0.02, 0.02, n).astype(np.float32)
    run_case(p, p.poses_init, 6.0, gamma, alpha, beta)


@pytest.mark.parametrize("options", [None, dict(texture_format=3, points_per_thread=4,
                                                 tile_order=2, persistent=2)])
def test_refine_with_pair_sub_sampling(gpu, options):
    """A joint-phase call on a sub-sampled step: only the selected pairs'
    tiles run (persistent launch), focal sums and stored depth derivatives
    of the skipped pairs are neither read nor added."""
    p = problem("c2")
    rng = np.random.default_rng(12)
    n = sum(int(np.count_nonzero(p.edge_map(v))) for v in range(p.n_views))
    gamma = rng.uniform(-0.02, 0.02, p.n_views)
    alpha = (1.0 + rng.uniform(-0.02, 0.02, n)).astype(np.float32)
    beta = rng.uniform(-0.02, 0.02, n).astype(np.float32)
    run_case(p, p.poses_init, 8.0, gamma, alpha, beta, sampling=(9, 5, 4), options=options)


def test_refine_small_clamp_and_focal_only(gpu):
    p = problem("c1")
    gamma = np.array([0.03, -0.01])
    run_case(p, p.poses_init, 3.0, gamma)


def test_refinement_reset_and_determinism(gpu):
    p = problem("c2")
    plan = plan_for(p)
    P = torch.from_numpy(p.poses_init.copy()).cuda()
    base = {k: t.cpu().numpy() for k, t in plan.refine(P, 10.0).items()}
    n = plan.n_records
    plan.set_refinement(torch.full((p.n_views,), 0.01, dtype=torch.float64),
                        torch.full((n,), 1.01), torch.full((n,), 0.01))
    moved = {k: t.cpu().numpy() for k, t in plan.refine(P, 10.0).items()}
    assert not np.array_equal(moved["loss"], base["loss"])
    again = {k: t.cpu().numpy() for k, t in plan.refine(P, 10.0).items()}
    for k in base:
        assert np.array_equal(moved[k], again[k]), k
    plan.set_refinement()                       # back to the plan's own values
    back = {k: t.cpu().numpy() for k, t in plan.refine(P, 10.0).items()}
    for k in base:
        assert np.array_equal(back[k], base[k]), k


def test_refine_autograd_function(gpu):
    from paper_2607_00579_amd.api import EdgeRefineFn
    p = problem("c1")
    plan = plan_for(p)
    P = torch.from_numpy(p.poses_init.copy()).cuda()
    n = plan.n_records
    xi = torch.zeros(p.n_views, 6, dtype=torch.float64, device="cuda", requires_grad=True)
    gamma = torch.full((p.n_views,), 0.01, dtype=torch.float64, device="cuda",
                       requires_grad=True)
    alpha = torch.ones(n, dtype=torch.float32, device="cuda", requires_grad=True)
    beta = torch.zeros(n, dtype=torch.float32, device="cuda", requires_grad=True)
    loss = EdgeRefineFn.apply(xi, gamma, alpha, beta, plan, P, 10.0)
    (2.5 * loss.sum()).backward()
    ref = plan.refine(P, 10.0)
    # the kernels apply the upstream factor before their last rounding steps
    assert torch.allclose(xi.grad, 2.5 * ref["grad"], rtol=1e-14, atol=0)
    assert torch.allclose(gamma.grad, 2.5 * ref["grad_gamma"], rtol=1e-14, atol=0)
    assert torch.allclose(alpha.grad, (2.5 * ref["grad_alpha"]).float(), rtol=1e-6, atol=0)
    assert torch.allclose(beta.grad, (2.5 * ref["grad_beta"]).float(), rtol=1e-6, atol=0)


def test_refine_focal_vs_oracle_finite_differences(gpu):
    """GPU dL/dgamma against frozen-branch central differences of the FP64
    oracle (h = 1e-6) on the two-view workload."""
    p = problem("c1")
    plan = plan_for(p)
    P = torch.from_numpy(p.poses_init.copy()).cuda()
    g = plan.refine(P, 10.0, depth=False)["grad_gamma"].cpu().numpy()
    op = ocost.OracleProblem(p)
    fd = ocost.fd_focal(op, p.poses_init, 10.0, h=1e-6)
    e = rel_norm_err(g, fd)
    say(f"c1: focal gradient vs central differences {e:.2e}")
    assert e < TOL


def test_refine_autograd_interleaved_forwards(gpu):
    """Two forwards at different refinements before either backward: each
    backward gives the gradients at its own forward's gamma, alpha, beta
    (bitwise those of a direct call there), whatever the plan holds when it
    runs; changing the poses in place before backward raises."""
    from paper_2607_00579_amd.api import EdgeRefineFn
    p = problem("c1")
    plan = plan_for(p)
    P = torch.from_numpy(p.poses_init.copy()).cuda()
    n, V = plan.n_records, p.n_views
    vals = []
    for k, (g0, a0, b0) in enumerate(((0.01, 1.0, 0.0), (-0.02, 1.03, 0.02))):
        vals.append((torch.full((V,), g0, dtype=torch.float64, device="cuda", requires_grad=True),
                     torch.full((n,), a0, dtype=torch.float32, device="cuda", requires_grad=True),
                     torch.full((n,), b0, dtype=torch.float32, device="cuda", requires_grad=True),
                     torch.zeros(V, 6, dtype=torch.float64, device="cuda", requires_grad=True)))
    losses = [EdgeRefineFn.apply(xi, g, a, b, plan, P, 10.0) for g, a, b, xi in vals]
    # the plan now holds the second refinement; run the first backward first
    for (g, a, b, xi), loss in zip(vals, losses):
        loss.sum().backward()
    for g, a, b, xi in vals:
        plan.set_refinement(g.detach(), a.detach(), b.detach())
        ref = plan.refine(P, 10.0)
        assert torch.equal(xi.grad, ref["grad"])
        assert torch.equal(g.grad, ref["grad_gamma"])
        assert torch.equal(a.grad, ref["grad_alpha"].float())
        assert torch.equal(b.grad, ref["grad_beta"].float())
    g, a, b, xi = vals[0]
    Q = P.clone()
    loss = EdgeRefineFn.apply(xi, g, a, b, plan, Q, 10.0)
    Q.add_(1e-3)
    with pytest.raises(RuntimeError):
        loss.sum().backward()


def test_cost_autograd_recompute_sees_in_place_pose_change(gpu):
    from paper_2607_00579_amd.api import EdgeCostFn
    p = problem("c1")
    plan = plan_for(p)
    Q = torch.from_numpy(p.poses_init.copy()).cuda()
    xi = torch.zeros(p.n_views, 6, dtype=torch.float64, device="cuda", requires_grad=True)
    loss = EdgeCostFn.apply(xi, plan, Q, 10.0, "recompute")
    Q[0, 0, 3] += 1e-3
    with pytest.raises(RuntimeError):
        loss.sum().backward()


@pytest.mark.parametrize("fmt", [2, 3])
def test_depth_pass_stored_and_recomputed_forms_agree_bitwise(gpu, fmt):
    """Before the first refinement update the depth pass re-evaluates every
    residual; afterwards it gathers the derivatives stored by the fused
    refinement kernel.  Same terms in the same order: identical bits."""
    p = problem("c2")
    plan = plan_for(p, options=dict(texture_format=fmt, points_per_thread=4, tile_order=1,
                                    persistent=2))
    P = torch.from_numpy(p.poses_init.copy()).cuda()
    up = torch.tensor([1.5], dtype=torch.float64, device="cuda")
    first = plan.refine(P, 7.0, upstream=up)
    plan.set_refinement()                  # identity state; allocates the derivative buffer
    second = plan.refine(P, 7.0, upstream=up)
    for k in first:
        assert torch.equal(first[k], second[k]), k
    assert float(first["grad_beta"].abs().max()) > 0
