"""Pins of the oracle's cost and analytic pose gradient (CPU)."""
import numpy as np
import pytest

from oracle import cost, geometry, edt
from synth import fixtures, make
from synth.scenes import pack

P = cost.CostParams()


def adjoint(Pm):
    """Ad(T) for twists ordered (rho, omega): [[R, [t]x R], [0, R]]."""
    R, t = Pm[:, :3], Pm[:, 3]
    A = np.zeros((6, 6))
    A[:3, :3] = R
    A[:3, 3:] = geometry.hat(t) @ R
    A[3:, 3:] = R
    return A


@pytest.fixture(scope="module")
def c1():
    p = make("c1")
    return p, cost.OracleProblem(p)


def test_zero_cost_shifted_pair_exact():
    """Exact geometry with dyadic disparities: every projection lands on an
    edge pixel, so the loss and gradient are exactly zero (both directions)."""
    p = fixtures.shifted_pair()
    op = cost.OracleProblem(p)
    r = op.evaluate(p.poses_init, 10.0)
    assert (r["n"] == 160).all()
    assert r["loss"][0] == 0.0
    assert np.all(r["grad"] == 0.0)
    # and the shift really is one of 8, 4, 2, 1 pixels: a wrong sign of the
    # translation would leave points off the edges
    bad = p.poses_init.copy()
    bad[1, 0, 3] = +0.5
    assert op.evaluate(bad, 10.0)["loss"][0] > 0.1


def test_zero_cost_dilated_projection_map(c1):
    """Target map = 3x3 dilation of all 2x2 tap sets of the i->j projections:
    every valid sample reads four zero taps."""
    p, op = c1
    r = op.direction(0, p.poses_init, 10.0, P, per_residual=True)
    i, j = p.pairs[0]
    Wj, Hj = int(p.width[j]), int(p.height[j])
    e = np.zeros((Hj, Wj), np.uint8)
    x0 = np.floor(r["up"][r["valid"]]).astype(int)
    y0 = np.floor(r["vp"][r["valid"]]).astype(int)
    for dy in range(-1, 3):
        for dx in range(-1, 3):
            e[np.clip(y0 + dy, 0, Hj - 1), np.clip(x0 + dx, 0, Wj - 1)] = 1
    maps = [p.edge_map(0), e]
    deps = [p.depth_map(0), p.depth_map(1)]
    q = fixtures.problem_from_maps(p.width, p.height, p.K, maps, deps, p.poses_init, [[0, 1]])
    oq = cost.OracleProblem(q)
    rq = oq.evaluate(q.poses_init, 10.0)
    assert rq["n"][0] == r["n"] > 1000
    assert rq["loss"][0] == 0.0
    assert np.all(rq["grad"] == 0.0)


def test_single_column_field_closed_form(c1):
    """DTF of a full column c is |x - c|: off the column the bilinear sample is
    |u' - c| and its slope is sign(u' - c)."""
    p, _ = c1
    W, H = int(p.width[1]), int(p.height[1])
    c = 80
    e1 = np.zeros((H, W), np.uint8)
    e1[:, c] = 1
    q = fixtures.problem_from_maps(p.width, p.height, p.K, [p.edge_map(0), e1],
                                   [p.depth_map(0), p.depth_map(1)], p.poses_init, [[0, 1]])
    oq = cost.OracleProblem(q)
    assert np.array_equal(oq.d2[1], np.broadcast_to((np.arange(W) - c) ** 2, (H, W)))
    r = oq.direction(0, q.poses_init, 1e9, P, per_residual=True)
    v = r["valid"]
    up = r["up"][v]
    x0 = np.floor(up)
    off = (x0 + 1 <= c) | (x0 >= c)
    assert off.sum() > 500
    assert np.allclose(r["Dval"][v][off], np.abs(up[off] - c), rtol=0, atol=1e-9)
    # with lambda = inf and everything on the linear Huber branch beyond 1 px:
    far = off & (np.abs(up - c) > 1.0)
    assert np.allclose(r["rho"][v][far], np.abs(up[far] - c) - 0.5, atol=1e-9)


def test_global_rigid_invariance(c1):
    p, op = c1
    base = op.evaluate(p.poses_init, 10.0)
    rng = np.random.default_rng(3)
    for _ in range(3):
        G = geometry.se3_exp(np.concatenate([rng.uniform(-10, 10, 3), rng.normal(size=3)]))
        Gi = np.linalg.inv(G)
        poses = np.stack([(geometry.to_h(Pm) @ Gi)[:3] for Pm in p.poses_init])
        r = op.evaluate(poses, 10.0)
        assert np.allclose(r["loss"], base["loss"], rtol=1e-12, atol=0)
        assert np.allclose(r["grad"], base["grad"], rtol=1e-9, atol=1e-12)


def test_gauge_identity(c1):
    """A common right perturbation of every pose leaves the cost unchanged, so
    sum_v Ad(T_v)^T g_v = 0, per pair and for the whole problem."""
    p, op = c1
    r = op.evaluate(p.poses_init, 10.0)
    tot = sum(adjoint(p.poses_init[v]).T @ r["grad"][v] for v in range(p.n_views))
    assert np.abs(tot).max() < 1e-12 * np.abs(r["grad"]).max() * 100
    for d in range(p.n_pairs):
        i, j = p.pairs[d]
        per = adjoint(p.poses_init[i]).T @ r["G_src"][d] + adjoint(p.poses_init[j]).T @ r["G_tgt"][d]
        assert np.abs(per).max() < 1e-9 * np.abs(r["G_tgt"][d]).max()


def test_power_of_two_scale_is_exact(c1):
    p, op = c1
    q = fixtures.problem_from_maps(p.width, p.height, p.K, [p.edge_map(0), p.edge_map(1)],
                                   [2 * p.depth_map(0), 2 * p.depth_map(1)], p.poses_init,
                                   p.pairs)
    poses2 = p.poses_init.copy()
    poses2[:, :, 3] *= 2
    oq = cost.OracleProblem(q, d2=op.d2)
    a = op.evaluate(p.poses_init, 10.0)
    b = oq.evaluate(poses2, 10.0)
    assert np.array_equal(a["loss"], b["loss"])
    assert np.array_equal(a["grad"][:, 3:], b["grad"][:, 3:])
    assert np.array_equal(a["grad"][:, :3], 2 * b["grad"][:, :3])


def test_frozen_branch_finite_differences(c1):
    p, op = c1
    for lam in (10.0, 3.0):
        r = op.evaluate(p.poses_init, lam)
        fd = cost.fd_gradient(op, p.poses_init, lam, h=1e-6)
        err = np.abs(fd - r["grad"]).max() / np.abs(r["grad"]).max()
        assert err < 1e-7, err


def test_free_finite_differences_close(c1):
    """Re-evaluating the discrete decisions only adds kink noise."""
    p, op = c1
    r = op.evaluate(p.poses_init, 10.0)
    fd = cost.fd_gradient(op, p.poses_init, 10.0, h=1e-6, frozen_branches=False)
    err = np.abs(fd - r["grad"]).max() / np.abs(r["grad"]).max()
    assert err < 5e-2, err


def test_identity_pair_is_zero(c1):
    p, _ = c1
    q = fixtures.problem_from_maps(p.width[:1], p.height[:1], p.K[:1], [p.edge_map(0)],
                                   [p.depth_map(0)], p.poses_init[:1], [[0, 0]])
    r = cost.OracleProblem(q).evaluate(q.poses_init, 10.0)
    assert r["n"][0] > 0
    assert r["loss"][0] < 1e-20


def test_relabel_and_permute_pairs(c1):
    p, op = c1
    base = op.evaluate(p.poses_init, 10.0)
    # swap the two views and reverse the pair list
    q = fixtures.problem_from_maps(p.width[::-1], p.height[::-1], p.K[::-1],
                                   [p.edge_map(1), p.edge_map(0)],
                                   [p.depth_map(1), p.depth_map(0)], p.poses_init[::-1],
                                   [[0, 1], [1, 0]])
    r = cost.OracleProblem(q).evaluate(q.poses_init, 10.0)
    assert np.allclose(r["loss"], base["loss"], rtol=1e-12)
    assert np.allclose(r["grad"][::-1], base["grad"], rtol=1e-10, atol=1e-14)


def test_huber_branches():
    d = np.array([0.0, 0.5, 1.0, 1.5, 4.0])
    assert np.allclose(cost.huber(d, 1.0), [0.0, 0.125, 0.5, 1.0, 3.5])
    # continuity of value at delta for another delta
    assert np.isclose(cost.huber(np.array([2.0]), 2.0)[0], 2.0)


def test_norm_mode_eq_form(c1):
    """norm_mode 1 divides by |E_i| (the Eq. form) instead of the valid count."""
    p, op = c1
    a = op.evaluate(p.poses_init, 10.0, cost.CostParams(norm_mode=0))
    b = op.evaluate(p.poses_init, 10.0, cost.CostParams(norm_mode=1))
    n_src = np.array([op.pts[int(i)][0].size for i in p.pairs[:, 0]])
    want = np.sum(a["S"] / n_src) * 2 / p.n_pairs
    assert np.isclose(b["loss"][0], want, rtol=1e-12)


def test_multi_scene_losses_are_independent():
    p1 = make("c1")
    f = fixtures.shifted_pair()
    both = pack(list(p1.scenes) + list(f.scenes), "two")
    op = cost.OracleProblem(both)
    r = op.evaluate(both.poses_init, 10.0)
    r1 = cost.OracleProblem(p1).evaluate(p1.poses_init, 10.0)
    assert np.allclose(r["loss"][0], r1["loss"][0], rtol=1e-12)
    assert r["loss"][1] == 0.0
    assert np.allclose(r["grad"][:2], r1["grad"], rtol=1e-12)


def test_empty_target_map_gives_no_valid_cost():
    W, H = 40, 30
    K = [32.0, 32.0, 19.5, 14.5]
    e0 = np.zeros((H, W), np.uint8)
    e0[10:20, 15] = 1
    z0 = np.full((H, W), 4.0, np.float32)
    e1 = np.zeros((H, W), np.uint8)
    Pm = np.concatenate([np.eye(3), np.zeros((3, 1))], axis=1)
    q = fixtures.problem_from_maps([W, W], [H, H], [K, K], [e0, e1], [z0, z0], [Pm, Pm],
                                   [[0, 1], [1, 0]])
    op = cost.OracleProblem(q)
    assert (op.d2[1] == edt.INF_D2).all()
    r = op.evaluate(q.poses_init, 10.0)
    # 0 -> 1: all valid, all clamped at lambda: rho = H(10) = 9.5, zero gradient
    assert r["n"][0] == 10 and np.isclose(r["S"][0], 95.0)
    # 1 -> 0: no source pixels, n = 0, L = 0
    assert r["n"][1] == 0 and r["L"][1] == 0.0
    assert np.all(r["grad"] == 0.0)
    assert np.isclose(r["loss"][0], 9.5)


def test_golden_trajectories_match_generator():
    """The stored oracle trajectories were produced from the current inputs."""
    import os
    from tests.golden.make_golden import input_checksum
    here = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")
    for name in ("c1", "c2"):
        g = np.load(os.path.join(here, f"{name}_trajectory.npz"), allow_pickle=False)
        assert str(g["checksum"]) == input_checksum(make(name)), name


def test_focal_and_depth_gradients_vs_finite_differences(c1):
    """Frozen-branch central differences in each view's focal scale gamma
    (f = f0 (1 + gamma)) and in the depth of single edge pixels."""
    p, op = c1
    for lam in (10.0, 3.0):
        r = op.evaluate(p.poses_init, lam)
        fd = cost.fd_focal(op, p.poses_init, lam)
        assert np.abs(fd - r["grad_focal"]).max() < 1e-7 * np.abs(r["grad_focal"]).max()
        for v in range(p.n_views):
            gz = r["grad_depth"][v]
            idx = np.concatenate([np.argsort(-np.abs(gz))[:4], [0, gz.size - 1]])
            fdz = cost.fd_depth(op, p.poses_init, lam, v, idx)
            assert np.abs(fdz - gz[idx]).max() < 1e-7 * np.abs(gz).max()


def test_depth_gradient_of_a_pure_translation_fixture():
    """Shifted pair at exact zero cost: every residual sits on an edge pixel
    (D = 0, zero slope), so the depth and focal gradients vanish exactly."""
    p = fixtures.shifted_pair()
    r = cost.OracleProblem(p).evaluate(p.poses_init, 10.0)
    assert np.all(r["grad_focal"] == 0.0)
    assert all(np.all(g == 0.0) for g in r["grad_depth"].values())


def test_camera_inside_fixture_has_residuals_behind_the_camera():
    """The behind-camera fixture (a camera inside the wireframe) holds, for
    both pairs into it, residuals behind the camera whose projections with
    the negative depth would land inside the image, and residuals just in
    front of it (0 < z <= 0.3) inside the image: only the depth test decides
    them, and the oracle drops both kinds at z_min = 0.3."""
    q = fixtures.camera_inside()
    op = cost.OracleProblem(q)
    for d in (0, 1):
        i, j = (int(x) for x in q.pairs[d])
        u, v, Z = op.pts[i]
        fx, fy, cx, cy = op.K[i]
        Xc = np.stack([(u - cx) / fx * Z, (v - cy) / fy * Z, Z], 1)
        Pi, Pj = q.poses_init[i], q.poses_init[j]
        Xp = ((Xc - Pi[:, 3]) @ Pi[:, :3]) @ Pj[:, :3].T + Pj[:, 3]
        z = Xp[:, 2]
        fxj, fyj, cxj, cyj = op.K[j]
        with np.errstate(divide="ignore", invalid="ignore"):
            up = fxj * Xp[:, 0] / z + cxj
            vp = fyj * Xp[:, 1] / z + cyj
        inb = (up >= 0) & (up < op.W[j] - 1) & (vp >= 0) & (vp < op.H[j] - 1)
        assert ((z <= 0) & inb).sum() >= 30
        assert ((z > 0) & (z <= 0.3) & inb).sum() >= 20
        for zmin in (1e-4, 0.3):
            r = op.direction(d, q.poses_init, 10.0, cost.CostParams(z_min=zmin),
                             per_residual=True)
            assert r["n"] == int(((z > zmin) & inb).sum())
