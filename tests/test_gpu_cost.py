"""GPU: fused cost + adjoint against the FP64 oracle on small and medium
workloads, exact-zero fixtures, invariants, formats and determinism."""
import numpy as np
import pytest
import torch

from oracle import cost as ocost
from synth import fixtures
from tests.gpu_helpers import problem, rel_norm_err, say

pytestmark = pytest.mark.gpu

TOL = 1e-4          # relative tolerance on cost and gradient (spec bar)


def plan_for(prob, **kw):
    from paper_2607_00579_amd.api import EdgePlan
    return EdgePlan.from_problem(prob, device="cuda:0", **kw)


def gpu_eval(plan, poses, lam, pairs=True):
    P = torch.from_numpy(np.ascontiguousarray(poses)).cuda()
    o = plan.cost(P, lam, grad=True, pairs=pairs)
    return {k: v.cpu().numpy() for k, v in o.items()}


def check_against_oracle(prob, poses, lam, params=ocost.CostParams(), plan=None, **kw):
    plan = plan or plan_for(prob, norm_mode=params.norm_mode, **kw)
    g = gpu_eval(plan, poses, lam)
    op = ocost.OracleProblem(prob)
    r = op.evaluate(poses, lam, params)
    dn = np.abs(g["pair_valid"] - r["n"])
    assert dn.max() <= max(2, int(1e-4 * r["n"].max())), dn.max()
    assert rel_norm_err(g["loss"], r["loss"]) < TOL, (g["loss"], r["loss"])
    ok = r["n"] > 0
    assert np.allclose(g["pair_cost"][ok], r["L"][ok], rtol=TOL, atol=0)
    e_t = rel_norm_err(g["grad"][:, :3], r["grad"][:, :3], axis=1)
    e_r = rel_norm_err(g["grad"][:, 3:], r["grad"][:, 3:], axis=1)
    say(f"{prob.name}: loss {g['loss']} vs {r['loss']}, grad err t {e_t:.2e} r {e_r:.2e}")
    assert e_t < TOL and e_r < TOL
    return plan, g, r


def test_records_match_edge_pixels(gpu):
    p = problem("c2")
    plan = plan_for(p)
    for v in range(p.n_views):
        rec = plan.view_records(v)
        u = (rec & 0xFFFF).astype(np.int64)
        vv = ((rec >> np.uint64(16)) & np.uint64(0xFFFF)).astype(np.int64)
        z = (rec >> np.uint64(32)).astype(np.uint32).view(np.float32)
        ys, xs = np.nonzero(p.edge_map(v))
        assert rec.size == xs.size
        got = sorted(zip(vv.tolist(), u.tolist()))
        assert got == sorted(zip(ys.tolist(), xs.tolist()))
        assert np.array_equal(z, p.depth_map(v)[vv, u])


def test_zero_cost_shifted_pair_exact(gpu):
    p = fixtures.shifted_pair()
    g = gpu_eval(plan_for(p), p.poses_init, 10.0)
    assert np.array_equal(g["pair_valid"], [160, 160])
    assert g["loss"][0] == 0.0
    assert np.all(g["grad"] == 0.0)


def test_zero_cost_dilated_projection_map(gpu):
    p = problem("c1")
    op = ocost.OracleProblem(p)
    r = op.direction(0, p.poses_init, 10.0, ocost.CostParams(), per_residual=True)
    j = int(p.pairs[0, 1])
    Wj, Hj = int(p.width[j]), int(p.height[j])
    e = np.zeros((Hj, Wj), np.uint8)
    x0 = np.floor(r["up"][r["valid"]]).astype(int)
    y0 = np.floor(r["vp"][r["valid"]]).astype(int)
    for dy in range(-1, 3):
        for dx in range(-1, 3):
            e[np.clip(y0 + dy, 0, Hj - 1), np.clip(x0 + dx, 0, Wj - 1)] = 255
    q = fixtures.problem_from_maps(p.width, p.height, p.K, [p.edge_map(0), e],
                                   [p.depth_map(0), p.depth_map(1)], p.poses_init, [[0, 1]])
    g = gpu_eval(plan_for(q), q.poses_init, 10.0)
    assert abs(int(g["pair_valid"][0]) - r["n"]) <= 2
    assert g["loss"][0] == 0.0
    assert np.all(g["grad"] == 0.0)


@pytest.mark.parametrize("zmin", [1e-4, 0.3])
@pytest.mark.parametrize("fmt", [1, 2, 3])
def test_residuals_behind_the_target_camera(gpu, zmin, fmt):
    """A camera inside the wireframe: hundreds of residuals of the pairs into
    it lie behind it (some of whose negative-depth projections fall inside
    the image) or just in front of it.  Per pair, the valid counts equal the
    oracle's exactly, and L_d, the target gradient sums G_d and the pose
    gradients agree within the bar, with the validity test on z and the
    clamped reciprocal of z both exercised (z_min = 0.3 moves the test)."""
    q = fixtures.camera_inside()
    params = ocost.CostParams(z_min=zmin)
    plan = plan_for(q, z_min=zmin, options=dict(texture_format=fmt, points_per_thread=4,
                                                 tile_order=1, persistent=2))
    g = gpu_eval(plan, q.poses_init, 10.0)
    r = ocost.OracleProblem(q).evaluate(q.poses_init, 10.0, params)
    say(f"camera inside, z_min {zmin}, format {fmt}: valid {g['pair_valid']} (oracle {r['n']})")
    assert np.array_equal(g["pair_valid"], r["n"])
    ok = r["n"] > 0
    assert np.allclose(g["pair_cost"][ok], r["L"][ok], rtol=TOL, atol=0)
    for d in np.flatnonzero(ok):
        assert np.linalg.norm(g["pair_grad"][d] - r["G_tgt"][d]) <= \
            TOL * np.linalg.norm(r["G_tgt"][d]), d
    assert rel_norm_err(g["loss"], r["loss"]) < TOL
    assert rel_norm_err(g["grad"], r["grad"], axis=1) < TOL
    assert plan.device_status() == 0


@pytest.mark.parametrize("name", ["c1", "c2"])
@pytest.mark.parametrize("lam", [10.0, 3.0])
def test_cost_and_gradient_vs_oracle(gpu, name, lam):
    p = problem(name)
    check_against_oracle(p, p.poses_init, lam)


def test_norm_mode_eq_form(gpu):
    p = problem("c1")
    check_against_oracle(p, p.poses_init, 10.0, ocost.CostParams(norm_mode=1))


def test_ground_truth_poses(gpu):
    p = problem("c2")
    check_against_oracle(p, p.poses_gt, 10.0)


@pytest.mark.parametrize("opts", [
    dict(texture_format=1, points_per_thread=1, tile_order=2, persistent=2),
    dict(texture_format=2, points_per_thread=16, tile_order=1, persistent=1),
    dict(texture_format=1, points_per_thread=8, tile_order=1, persistent=1),
    dict(texture_format=2, points_per_thread=2, tile_order=2, persistent=2),
    dict(texture_format=3, points_per_thread=4, tile_order=1, persistent=2),
    dict(texture_format=3, points_per_thread=16, tile_order=2, persistent=1),
])
def test_schedules_agree_with_oracle(gpu, opts):
    p = problem("c2")
    check_against_oracle(p, p.poses_init, 10.0, options=opts)


@pytest.mark.parametrize("fmt", [2, 3])
def test_texture_formats_bitwise_equal(gpu, fmt):
    """The three textures hold the same float32 taps (format 2 through its
    exact square-root table): every output bitwise equal to format 1's."""
    p = problem("c2")
    a = gpu_eval(plan_for(p, options=dict(texture_format=1, points_per_thread=4, tile_order=1,
                                          persistent=2)), p.poses_init, 10.0)
    b = gpu_eval(plan_for(p, options=dict(texture_format=fmt, points_per_thread=4, tile_order=1,
                                          persistent=2)), p.poses_init, 10.0)
    for k in a:
        assert np.array_equal(a[k], b[k]), k


def test_format_switches_rebuild_the_textures(gpu):
    """A plan keeps the float32 texture and the format in use; switching
    formats derives the new one from the float32 texture (and frees the old):
    every output bitwise equal to format 1's, on one plan switched
    1 -> 2 -> 3 -> 1 -> 2 and after an autotune."""
    p = problem("c2")
    base = dict(points_per_thread=4, tile_order=1, persistent=2)
    plan = plan_for(p, options=dict(base, texture_format=1))
    ref = gpu_eval(plan, p.poses_init, 10.0)
    for fmt in (2, 3, 1, 2):
        plan.set_options(**base, texture_format=fmt)
        got = gpu_eval(plan, p.poses_init, 10.0)
        for k in ref:
            assert np.array_equal(got[k], ref[k]), (fmt, k)
    plan.autotune(torch.from_numpy(p.poses_init.copy()).cuda(), 10.0, iters=1)
    plan.set_options(**base, texture_format=3)
    got = gpu_eval(plan, p.poses_init, 10.0)
    for k in ref:
        assert np.array_equal(got[k], ref[k]), k


def test_run_to_run_bitwise(gpu):
    p = problem("c2")
    for opts in (dict(persistent=1), dict(persistent=2)):
        plan = plan_for(p, options=opts)
        a = gpu_eval(plan, p.poses_init, 10.0)
        b = gpu_eval(plan, p.poses_init, 10.0)
        for k in a:
            assert np.array_equal(a[k], b[k]), k


def test_global_rigid_invariance(gpu):
    from oracle import geometry
    p = problem("c2")
    plan = plan_for(p)
    a = gpu_eval(plan, p.poses_init, 10.0)
    G = geometry.se3_exp(np.array([3.0, -7.0, 5.0, 0.4, -1.1, 2.0]))
    Gi = np.linalg.inv(G)
    poses = np.stack([(geometry.to_h(P) @ Gi)[:3] for P in p.poses_init])
    b = gpu_eval(plan, poses, 10.0)
    assert rel_norm_err(b["loss"], a["loss"]) < 1e-6
    assert rel_norm_err(b["grad"], a["grad"], axis=1) < 1e-5


def test_power_of_two_scale_bitwise(gpu):
    p = problem("c1")
    q = fixtures.problem_from_maps(p.width, p.height, p.K, [p.edge_map(0), p.edge_map(1)],
                                   [2 * p.depth_map(0), 2 * p.depth_map(1)], p.poses_init, p.pairs)
    poses2 = p.poses_init.copy()
    poses2[:, :, 3] *= 2
    a = gpu_eval(plan_for(p), p.poses_init, 10.0)
    b = gpu_eval(plan_for(q), poses2, 10.0)
    assert np.array_equal(a["loss"], b["loss"])
    assert np.array_equal(a["grad"][:, 3:], b["grad"][:, 3:])
    assert np.array_equal(a["grad"][:, :3], 2 * b["grad"][:, :3])


def test_gauge_identity(gpu):
    from oracle import geometry
    p = problem("c2")
    g = gpu_eval(plan_for(p), p.poses_init, 10.0)

    def adj(P):
        R, t = P[:, :3], P[:, 3]
        A = np.zeros((6, 6))
        A[:3, :3] = R
        A[:3, 3:] = geometry.hat(t) @ R
        A[3:, 3:] = R
        return A

    tot = sum(adj(p.poses_init[v]).T @ g["grad"][v] for v in range(p.n_views))
    scale = sum(np.abs(adj(p.poses_init[v]).T @ g["grad"][v]).max() for v in range(p.n_views))
    assert np.abs(tot).max() < 1e-9 * scale


def test_empty_target_and_identity_pair(gpu):
    W, H = 40, 30
    K = [32.0, 32.0, 19.5, 14.5]
    e0 = np.zeros((H, W), np.uint8)
    e0[10:20, 15] = 255
    z0 = np.full((H, W), 4.0, np.float32)
    e1 = np.zeros((H, W), np.uint8)
    Pm = np.concatenate([np.eye(3), np.zeros((3, 1))], axis=1)
    q = fixtures.problem_from_maps([W, W], [H, H], [K, K], [e0, e1], [z0, z0], [Pm, Pm],
                                   [[0, 1], [1, 0], [0, 0]])
    g = gpu_eval(plan_for(q), q.poses_init, 10.0)
    assert list(g["pair_valid"]) == [10, 0, 10]
    assert np.isclose(g["pair_cost"][0], 9.5) and g["pair_cost"][1] == 0.0
    assert g["pair_cost"][2] == 0.0
    assert np.all(g["grad"] == 0.0)
    assert np.isclose(g["loss"][0], 2.0 / 3.0 * 9.5)


def test_lambda_outside_plan_range_is_flagged(gpu):
    p = problem("c1")
    plan = plan_for(p)
    plan.device_status()
    gpu_eval(plan, p.poses_init, 12.0)
    assert plan.device_status() & 2
    gpu_eval(plan, p.poses_init, -1.0)
    assert plan.device_status() & 2
    gpu_eval(plan, p.poses_init, 9.0)
    assert plan.device_status() == 0


def test_bwd_matches_fused_and_scales_upstream(gpu):
    p = problem("c2")
    plan = plan_for(p)
    P = torch.from_numpy(p.poses_init.copy()).cuda()
    a = plan.cost(P, 10.0, grad=True)["grad"]
    b = plan.cost_bwd(P, 10.0, upstream=torch.tensor([2.5], dtype=torch.float64, device="cuda"))
    assert torch.equal(b, 2.5 * a)


@pytest.mark.parametrize("fmt", [1, 2, 3])
def test_odd_view_sizes(gpu, fmt):
    """Views whose sides are not multiples of the 8 x 4 texture blocks (down
    to 2 x 2): every format against the oracle and bitwise equal to format 1
    (format 3's per-view texture base counts 16-byte texels)."""
    p = fixtures.odd_size_views()
    opts = dict(texture_format=fmt, points_per_thread=2, tile_order=1, persistent=2)
    plan, g, r = check_against_oracle(p, p.poses_init, 10.0, options=opts)
    assert (r["n"] > 0).sum() >= 10
    if fmt != 1:
        ref = gpu_eval(plan_for(p, options=dict(opts, texture_format=1)), p.poses_init, 10.0)
        for k in ("loss", "grad", "pair_cost", "pair_valid"):
            assert np.array_equal(g[k], ref[k]), k


def _one_view_scene():
    p = fixtures.odd_size_views()
    return fixtures.problem_from_maps([p.width[0]], [p.height[0]], [p.K[0]], [p.edge_map(0)],
                                      [p.depth_map(0)], [p.poses_init[0]], np.zeros((0, 2)),
                                      name="one_view")


def test_scenes_without_pairs(gpu):
    """A scene with one view has no pairs: its loss and gradient are exactly
    zero, alone (a plan with no pairs at all) and batched beside a scene
    that has pairs, whose results are unchanged; the pose step leaves its
    pose where it is."""
    from synth.scenes import config_c1, pack
    one = _one_view_scene()
    g = gpu_eval(plan_for(one), one.poses_init, 10.0)
    assert np.array_equal(g["loss"], np.zeros(1)) and not np.any(g["grad"])
    c1 = pack(list(config_c1().scenes), "c1")
    mix = pack(list(config_c1().scenes) + list(one.scenes), "mix")
    plan, gm, r = check_against_oracle(mix, mix.poses_init, 10.0)
    assert gm["loss"][1] == 0.0 and not np.any(gm["grad"][2])
    alone = gpu_eval(plan_for(c1), c1.poses_init, 10.0)
    assert np.array_equal(gm["loss"][:1], alone["loss"])
    assert np.array_equal(gm["grad"][:2], alone["grad"])
    P = torch.from_numpy(mix.poses_init.copy()).cuda()
    out = plan.cost(P, 10.0, grad=True)
    m = torch.zeros(mix.n_views, 6, dtype=torch.float64, device="cuda")
    v = torch.zeros_like(m)
    step = torch.zeros(1, dtype=torch.int32, device="cuda")
    plan.pose_step(P, m, v, out["grad"], 3e-3, step)
    assert torch.equal(P[2], torch.from_numpy(mix.poses_init[2]).cuda())
    assert int(step.item()) == 1
