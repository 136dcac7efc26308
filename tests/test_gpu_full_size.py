"""GPU: the full-size workloads in the launch configuration the benchmark
times (autotuned schedule), checked on outputs the oracle can compute one by
one: sampled directed pairs (S_d, n_d, L_d and the target-gradient sum G_d),
sampled views of the distance transform, and sampled pixels by brute force.
Also: the captured iteration equals the eager calls bitwise at full size."""
import numpy as np
import pytest
import torch

from oracle import cost as ocost
from tests.gpu_helpers import check_depth, problem, rel_norm_err, say

pytestmark = pytest.mark.gpu


def sample_pairs(prob, n, rng):
    """n pairs spread over scenes, the same number for every target
    resolution of the workload (256 x 192 up to 1024 x 768 for the batch)."""
    px = prob.width.astype(np.int64) * prob.height
    tpx = px[prob.pairs[:, 1]]
    sizes = np.unique(tpx)
    per = int(np.ceil(n / sizes.size))
    out = []
    for sz in sizes:
        cand = np.flatnonzero(tpx == sz)
        out.append(rng.choice(cand, size=min(per, cand.size), replace=False))
    return np.sort(np.concatenate(out))


def check_pairs(prob, plan, pair_ids, lam=10.0):
    from oracle import parallel as opar
    poses = torch.from_numpy(prob.poses_init.copy()).cuda()
    o = plan.cost(poses, lam, grad=True, pairs=True)
    g = {k: v.cpu().numpy() for k, v in o.items()}
    views = sorted(set(prob.pairs[pair_ids].ravel().tolist()))
    # the oracle's own distance transforms of the views involved, in fresh
    # worker processes (this one holds a GPU context)
    d2 = opar.distance_fields(prob, views=views, context="spawn")
    op = ocost.OracleProblem(prob, d2=d2, views=views)
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


@pytest.mark.parametrize("name,n_pairs", [("c4", 64), ("c5", 12)])
def test_full_size_sampled_pairs(gpu, name, n_pairs):
    """Sampled pairs of the full workloads in the benchmark's launch
    configuration; for the batch, 16 pairs into targets of each of its four
    resolutions."""
    from paper_2607_00579_amd.api import EdgePlan
    prob = problem(name)
    plan = EdgePlan.from_problem(prob)
    poses = torch.from_numpy(prob.poses_init.copy()).cuda()
    chosen = plan.autotune(poses, 10.0, iters=1)
    rng = np.random.default_rng(11)
    ids = sample_pairs(prob, n_pairs, rng)
    tres = sorted({(int(prob.width[j]), int(prob.height[j])) for j in prob.pairs[ids, 1]})
    if name == "c4":
        assert len(tres) == 4, tres
    worst_L, worst_G, dn, g = check_pairs(prob, plan, ids)
    say(f"{name} ({plan.n_residuals} residuals, schedule {chosen}): {ids.size} sampled pairs "
        f"into targets of {tres}, max |dn| {dn}, worst L_d rel err {worst_L:.2e}, "
        f"worst G_d rel err {worst_G:.2e}")
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


@pytest.mark.parametrize("name,per_size", [("c4", 2), ("c5", 6)])
def test_full_size_edt_sampled(gpu, name, per_size):
    """Whole views bit-exact against the oracle's separable transform (for the
    batch, `per_size` views of each of its four resolutions; for the large
    scene six 1024 x 768 views), and 4000 random pixels per view by brute
    force on the largest view and a random one."""
    from oracle import parallel as opar
    from paper_2607_00579_amd.api import build_distance_fields
    prob = problem(name)
    e = torch.from_numpy(prob.edge_flat).cuda()
    d2, _ = build_distance_fields(e, prob.view_offset[:-1], prob.width, prob.height)
    d2 = d2.cpu().numpy()
    rng = np.random.default_rng(5)
    px = prob.width.astype(np.int64) * prob.height
    views = []
    for sz in np.unique(px):
        cand = np.flatnonzero(px == sz)
        views += [int(v) for v in rng.choice(cand, size=min(per_size, cand.size), replace=False)]
    want = opar.distance_fields(prob, views=views, context="spawn")
    for v in views:
        a, b = prob.view_offset[v], prob.view_offset[v + 1]
        got = d2[a:b].reshape(prob.height[v], prob.width[v])
        assert np.array_equal(got, want[v]), v
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


def test_full_size_joint_phase_whole_scenes_c4(gpu):
    """The joint phase on the whole 64-scene batch (autotuned schedule, seeded
    non-identity focal and depth refinement), checked scene by scene: scenes
    are independent, so each sampled scene's loss, pose and focal gradients
    and every one of its records' depth derivatives are the oracle's on that
    scene alone.  Sampled: the scene with the fewest residuals, the one with
    the most image pairs among scenes of at most 2 M residuals and the one
    with the fewest views among scenes of 768 x 576 images or larger."""
    from paper_2607_00579_amd.api import EdgePlan
    prob = problem("c4")
    plan = EdgePlan.from_problem(prob)
    P = torch.from_numpy(prob.poses_init.copy()).cuda()
    chosen = plan.autotune(P, 10.0, iters=1)
    lam = 8.0
    ne = np.array([np.count_nonzero(prob.edge_map(v)) for v in range(prob.n_views)], np.int64)
    off = np.concatenate([[0], np.cumsum(ne)])
    assert plan.n_records == off[-1]
    rng = np.random.default_rng(23)
    gamma = rng.uniform(-0.02, 0.02, prob.n_views)
    alpha = (1.0 + rng.uniform(-0.02, 0.02, off[-1])).astype(np.float32)
    beta = rng.uniform(-0.02, 0.02, off[-1]).astype(np.float32)
    plan.set_refinement(torch.from_numpy(gamma), torch.from_numpy(alpha), torch.from_numpy(beta))
    g = {k: t.cpu().numpy() for k, t in plan.refine(P, lam).items()}
    assert plan.device_status() == 0
    # the library's refined values: float32(f0 (1 + gamma)) with the product
    # in float64, float32(Z0 alpha + beta) (Z0 alpha exact)
    K = prob.K.astype(np.float64).reshape(-1, 4).copy()
    K[:, :2] = (prob.K.reshape(-1, 4)[:, :2].astype(np.float64)
                * (1.0 + gamma)[:, None]).astype(np.float32)

    S = int(prob.scene_of_view.max()) + 1
    R = np.bincount(prob.scene_of_pair, weights=ne[prob.pairs[:, 0]], minlength=S)
    npairs = np.bincount(prob.scene_of_pair, minlength=S)
    px = np.zeros(S, np.int64)
    np.maximum.at(px, prob.scene_of_view, prob.width.astype(np.int64) * prob.height)
    small = np.flatnonzero(R <= 2e6)
    big = np.flatnonzero(px >= 768 * 576)
    nv = np.bincount(prob.scene_of_view, minlength=S)
    scenes = sorted({int(np.argmin(R)), int(small[np.argmax(npairs[small])]),
                     int(big[np.argmin(nv[big])])})
    for s in scenes:
        views = np.flatnonzero(prob.scene_of_view == s)
        pair_ids = np.flatnonzero(prob.scene_of_pair == s)
        depth, z0, rec, order = {}, [], [], []
        for v in views:
            # plan records of view v in plan order -> the oracle's row-major
            # edge-pixel order
            r = plan.view_records(int(v))
            x = (r & 0xFFFF).astype(np.int64)
            y = ((r >> np.uint64(16)) & np.uint64(0xFFFF)).astype(np.int64)
            ys, xs = np.nonzero(prob.edge_map(int(v)))
            keys = ys.astype(np.int64) * int(prob.width[v]) + xs
            pos = np.searchsorted(keys, y * int(prob.width[v]) + x)
            assert np.array_equal(keys[pos], y * int(prob.width[v]) + x)
            idx = np.arange(off[v], off[v + 1])
            zv = prob.depth_map(int(v))[ys, xs].astype(np.float64)[pos]
            zr = np.zeros(ne[v])
            zr[pos] = (zv * alpha[idx].astype(np.float64)
                       + beta[idx].astype(np.float64)).astype(np.float32)
            depth[int(v)] = zr
            z0.append(zv)
            rec.append(idx)
            order.append((int(v), pos))
        op = ocost.OracleProblem(prob, views=views.tolist())
        r = op.evaluate(prob.poses_init, lam, pair_ids=pair_ids.tolist(), K=K, depth=depth)
        e_l = abs(g["loss"][s] - r["loss"][s]) / abs(r["loss"][s])
        e_p = rel_norm_err(g["grad"][views], r["grad"][views], axis=1)
        want_gamma = r["grad_focal"][views] / (1.0 + gamma[views])
        e_g = rel_norm_err(g["grad_gamma"][views], want_gamma)
        say(f"c4 scene {s} ({views.size} views, {pair_ids.size} pairs, {int(R[s])} residuals, "
            f"schedule {chosen}): loss err {e_l:.2e}, pose grad err {e_p:.2e}, "
            f"focal err {e_g:.2e}")
        assert e_l < 1e-4 and e_p < 1e-4 and e_g < 1e-4
        want_beta = np.concatenate([r["grad_depth"][v][pos] for v, pos in order])
        rec = np.concatenate(rec)
        check_depth(g["grad_beta"][rec], want_beta, f"c4 scene {s} dL/dbeta")
        check_depth(g["grad_alpha"][rec], np.concatenate(z0) * want_beta, f"c4 scene {s} dL/dalpha")
    # the other scenes' outputs are finite
    assert np.isfinite(g["loss"]).all() and np.isfinite(g["grad_beta"]).all()


def test_max_side_views(gpu):
    """Two 16384 x 16384 views, the largest side a plan takes: the records'
    uint16 coordinates up to 16383, texel offsets up to 2^30 bytes into a view
    (format 2; format 1 the same in float32 words) and 16-byte texels of a
    4 GiB texture per view (format 3), source pixels on the last rows and
    columns, projections leaving the image there.  Pair 0 -> 1 in every
    texture format against the oracle, whose distance field of the target is
    the grid's closed form at the taps it reads (the GPU's own transform of
    the target goes into the textures); then the refinement variant's loss,
    pose, focal and per-record depth gradients against the oracle's."""
    from oracle import cost as ocost
    from paper_2607_00579_amd.api import EdgePlan
    from synth import fixtures
    from tests.gpu_helpers import GridDTF
    prob = fixtures.max_side_pair()
    S = int(prob.width[0])
    say(f"max side: {S} x {S}, {int(prob.edge_counts()[0])} source edge pixels")
    op = ocost.OracleProblem(prob, d2={0: np.zeros((1, 1), np.int64)}, views=[0])
    op.D[1] = GridDTF(S, fixtures.GRID_PITCH, fixtures.GRID_X0, fixtures.GRID_Y0)
    r = op.direction(0, prob.poses_init, 10.0, ocost.CostParams())
    assert r["n"] > 0.8 * r["n_src"] and r["n"] < r["n_src"]
    plan = EdgePlan.from_problem(prob)
    poses = torch.from_numpy(prob.poses_init.copy()).cuda()
    L = r["S"] / r["n"]
    Gn = np.linalg.norm(r["G_tgt"])
    assert Gn > 0
    for fmt in (1, 2, 3):
        plan.set_options(texture_format=fmt, points_per_thread=16, tile_order=1, persistent=2)
        o = plan.cost(poses, 10.0, grad=True, pairs=True)
        g = {k: v.cpu().numpy() for k, v in o.items()}
        eL = abs(g["pair_cost"][0] - L) / abs(L)
        eG = np.linalg.norm(g["pair_grad"][0] - r["G_tgt"]) / Gn
        say(f"  format {fmt}: n {int(g['pair_valid'][0])} (oracle {r['n']}), L_d rel err "
            f"{eL:.2e}, G_d rel err {eG:.2e}")
        assert int(g["pair_valid"][0]) == r["n"]
        assert eL < 1e-5 and eG < 1e-4
    # the refinement variant (focal sums, per-record depth derivatives) at the
    # identity refinement, with the autotuner's format for the batch
    from tests.gpu_helpers import gather_depth, oracle_index
    plan.set_options(texture_format=2, points_per_thread=16, tile_order=1, persistent=2)
    got = {k: t.cpu().numpy() for k, t in plan.refine(poses, 10.0).items()}
    want = op.evaluate(prob.poses_init, 10.0)
    assert rel_norm_err(got["loss"], want["loss"]) < 1e-4
    assert rel_norm_err(got["grad"], want["grad"], axis=1) < 1e-4
    assert rel_norm_err(got["grad_gamma"], want["grad_focal"]) < 1e-4
    views, idx = oracle_index(prob, plan)
    want_beta = gather_depth(want["grad_depth"], views, idx, views.size)
    z0 = np.zeros(views.size)
    sel = views == 0
    ys, xs = np.nonzero(prob.edge_map(0))
    z0[sel] = prob.depth_map(0)[ys, xs].astype(np.float64)[idx[sel]]
    # the source view's records against the oracle (the target's records are
    # no pair's source here: exactly zero)
    check_depth(got["grad_beta"][sel], want_beta[sel], "max side dL/dbeta")
    check_depth(got["grad_alpha"][sel], z0[sel] * want_beta[sel], "max side dL/dalpha")
    assert not np.any(got["grad_beta"][~sel]) and not np.any(got["grad_alpha"][~sel])
    assert plan.device_status() == 0
