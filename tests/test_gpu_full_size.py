"""GPU: the full-size workloads in the launch configuration the benchmark
times (autotuned schedule), checked on outputs the oracle can compute one by
one: sampled directed pairs (S_d, n_d, L_d and the target-gradient sum G_d),
sampled views of the distance transform, and sampled pixels by brute force.
Also: the captured iteration equals the eager calls bitwise at full size."""
import numpy as np
import pytest
import torch

from oracle import cost as ocost
from oracle import edt as oedt
from tests.gpu_helpers import problem, say

pytestmark = pytest.mark.gpu


def sample_pairs(prob, n, rng, max_px=None):
    """Pairs spread over scenes; targets limited to images of at most max_px
    pixels (the oracle's distance transform is O(W^2 H) per view)."""
    ok = np.ones(prob.n_pairs, bool)
    if max_px is not None:
        px = prob.width.astype(np.int64) * prob.height
        ok &= px[prob.pairs[:, 1]] <= max_px
    cand = np.flatnonzero(ok)
    return np.sort(rng.choice(cand, size=min(n, cand.size), replace=False))


def check_pairs(prob, plan, pair_ids, lam=10.0):
    poses = torch.from_numpy(prob.poses_init.copy()).cuda()
    o = plan.cost(poses, lam, grad=True, pairs=True)
    g = {k: v.cpu().numpy() for k, v in o.items()}
    views = sorted(set(prob.pairs[pair_ids].ravel().tolist()))
    op = ocost.OracleProblem(prob, views=views)
    worst_L, worst_G, dn_max = 0.0, 0.0, 0
    for d in pair_ids:
        r = op.direction(int(d), prob.poses_init, lam, ocost.CostParams())
        dn_max = max(dn_max, abs(int(g["pair_valid"][d]) - r["n"]))
        if r["n"] > 0:
            L = r["S"] / r["n"]
            worst_L = max(worst_L, abs(g["pair_cost"][d] - L) / abs(L))
            Gn = np.linalg.norm(r["G_tgt"])
            if Gn > 0:
                worst_G = max(worst_G, np.linalg.norm(g["pair_grad"][d] - r["G_tgt"]) / Gn)
    return worst_L, worst_G, dn_max, g


@pytest.mark.parametrize("name,n_pairs,max_px", [("c4", 60, 518 * 392), ("c5", 12, None)])
def test_full_size_sampled_pairs(gpu, name, n_pairs, max_px):
    from paper_2607_00579_amd.api import EdgePlan
    prob = problem(name)
    plan = EdgePlan.from_problem(prob)
    poses = torch.from_numpy(prob.poses_init.copy()).cuda()
    chosen = plan.autotune(poses, 10.0, iters=1)
    rng = np.random.default_rng(11)
    ids = sample_pairs(prob, n_pairs, rng, max_px)
    worst_L, worst_G, dn, g = check_pairs(prob, plan, ids)
    say(f"{name} ({plan.n_residuals} residuals, schedule {chosen}): {ids.size} sampled pairs, "
        f"max |dn| {dn}, worst L_d rel err {worst_L:.2e}, worst G_d rel err {worst_G:.2e}")
    assert dn == 0
    assert worst_L < 1e-5
    assert worst_G < 1e-4
    assert np.isfinite(g["loss"]).all() and np.isfinite(g["grad"]).all()
    assert plan.device_status() == 0


def test_full_size_graph_equals_eager_c4(gpu):
    from paper_2607_00579_amd import _lib
    from paper_2607_00579_amd.api import EdgePlan
    prob = problem("c4")
    plan = EdgePlan.from_problem(prob)
    dev = torch.device("cuda:0")
    poses0 = torch.from_numpy(prob.poses_init.copy()).to(dev)
    plan.autotune(poses0, 10.0, iters=1)
    # eager: schedule -> cost + adjoint -> pose step, twice
    P1 = poses0.clone()
    m1 = torch.zeros(prob.n_views, 6, dtype=torch.float64, device=dev)
    v1 = torch.zeros_like(m1)
    s1 = torch.zeros(1, dtype=torch.int32, device=dev)
    lam = torch.zeros(plan.n_scenes, dtype=torch.float32, device=dev)
    lr = torch.zeros(plan.n_scenes, dtype=torch.float64, device=dev)
    st = torch.cuda.current_stream().cuda_stream
    eager_loss = []
    for _ in range(2):
        _lib.schedule(s1, plan.n_scenes, 10.0, 6.0, 1000, 3e-3, 25, 2000, lam, lr, st)
        o = plan.cost(P1, lam, grad=True)
        eager_loss.append(o["loss"].clone())
        plan.pose_step(P1, m1, v1, o["grad"], lr, s1)
    # captured
    P2 = poses0.clone()
    m2 = torch.zeros_like(m1)
    v2 = torch.zeros_like(m1)
    s2 = torch.zeros_like(s1)
    loss = torch.zeros(plan.n_scenes, dtype=torch.float64, device=dev)
    plan.capture_iteration(P2, m2, v2, s2, loss)
    graph_loss = []
    for _ in range(2):
        plan.launch_iteration()
        graph_loss.append(loss.clone())
    torch.cuda.synchronize()
    for a, b in zip(eager_loss, graph_loss):
        assert torch.equal(a, b)
    assert torch.equal(P1, P2) and torch.equal(m1, m2) and torch.equal(v1, v2)
    assert int(s2.item()) == 2


@pytest.mark.parametrize("name,n_views", [("c4", 6), ("c5", 2)])
def test_full_size_edt_sampled(gpu, name, n_views):
    """Whole views bit-exact against the oracle's separable transform (smaller
    views), and 4000 random pixels per view by brute force on the largest."""
    from paper_2607_00579_amd.api import build_distance_fields
    prob = problem(name)
    e = torch.from_numpy(prob.edge_flat).cuda()
    d2, _ = build_distance_fields(e, prob.view_offset[:-1], prob.width, prob.height)
    d2 = d2.cpu().numpy()
    rng = np.random.default_rng(5)
    px = prob.width.astype(np.int64) * prob.height
    small = np.flatnonzero(px <= 518 * 392)
    views = list(rng.choice(small, size=min(n_views, small.size), replace=False)) if small.size else []
    for v in views:
        a, b = prob.view_offset[v], prob.view_offset[v + 1]
        got = d2[a:b].reshape(prob.height[v], prob.width[v])
        assert np.array_equal(got, oedt.edt_separable(prob.edge_map(v))), v
    big = int(np.argmax(px))
    for v in {big, int(rng.integers(prob.n_views))}:
        m = prob.edge_map(v)
        ys, xs = np.nonzero(m)
        a = prob.view_offset[v]
        H, W = m.shape
        qy = rng.integers(0, H, 4000)
        qx = rng.integers(0, W, 4000)
        want = np.array([int(((xs - x) ** 2 + (ys - y) ** 2).min()) for y, x in zip(qy, qx)])
        got = d2[a + qy.astype(np.int64) * W + qx]
        assert np.array_equal(got, want), v
    say(f"{name}: EDT bit-exact on {len(views)} whole views and 2 x 4000 sampled pixels")
