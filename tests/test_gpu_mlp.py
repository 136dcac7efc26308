"""GPU: the pose refiner (MLP on bf16 matrix cores, Gram-Schmidt, translation
offsets, AdamW) against the oracle, which rounds to bf16 at the same points
and accumulates exactly.  Tolerances: bit-exact where every sum is exact in
float32; otherwise 2^-7 normwise (two bf16 units: an accumulation-order
difference can move a value across a bf16 rounding boundary)."""
import numpy as np
import pytest
import torch

from oracle import mlp as omlp
from synth import refiner
from tests.gpu_helpers import problem, rel_norm_err, say

pytestmark = pytest.mark.gpu
BF16_TOL = 2.0 ** -7


def plan_for(prob):
    from paper_2607_00579_amd.api import EdgePlan
    return EdgePlan.from_problem(prob, device="cuda:0")


def make_refiner(prob, params):
    from paper_2607_00579_amd.api import PoseRefiner
    plan = plan_for(prob)
    P0 = torch.from_numpy(prob.poses_init.copy()).cuda()
    return plan, PoseRefiner(plan, P0, torch.from_numpy(params))


def scene_rows(prob, s):
    return np.flatnonzero(prob.scene_of_view == s)


def test_zero_last_layer_returns_the_initial_poses(gpu):
    p = problem("c2")
    plan, ref = make_refiner(p, refiner.init_params(np.random.default_rng(0)))
    P = ref.forward().cpu().numpy()
    assert np.abs(P - p.poses_init).max() < 1e-14


def test_forward_exact_on_exact_sums(gpu):
    """Sparse weights in {-1/8, 0, 1/8}, zero biases, small integer inputs:
    every pre-activation is a sum of few multiples of a power of two, exact in
    float32 in any order (checked on the oracle's values), so the device's
    bf16 activations and float32 outputs equal the oracle's and the poses
    agree to float64 rounding."""
    p = problem("c2")
    rng = np.random.default_rng(1)
    th = np.zeros((1, refiner.N_PARAMS), np.float32)
    for (wo, bo), (rows, cols) in zip(refiner.offsets(), refiner.SHAPES):
        th[0, wo:bo] = rng.choice([-1.0, 0.0, 1.0], size=rows * cols, p=[0.05, 0.9, 0.05]) / 8
    plan, ref = make_refiner(p, th)
    P0 = rng.integers(-3, 4, size=(p.n_views, 3, 4)).astype(np.float64)
    P0[:, :, :3] += 8.0 * np.eye(3)              # a well-conditioned rotation block
    ref.poses0.copy_(torch.from_numpy(P0))
    ref.forward()
    o, cache = omlp.forward(th[0].astype(np.float64), P0.reshape(-1, 12))
    for h in cache["h"][1:] + [o]:
        assert np.array_equal(np.asarray(h, np.float32).astype(np.float64), h)
    assert np.abs(o).max() > 0
    want = omlp.assemble(P0, o, np.zeros((p.n_views, 3)))
    got = ref.poses.cpu().numpy()
    say(f"exact-sum fixture: |o| max {np.abs(o).max():.3g}, pose diff {np.abs(got - want).max():.2e}")
    assert np.abs(got - want).max() < 1e-13


def test_forward_and_backward_match_the_oracle(gpu):
    p = problem("c2")
    rng = np.random.default_rng(2)
    th = refiner.init_params(rng, last_std=0.02, bias_std=0.05)
    plan, ref = make_refiner(p, th)
    ref.delta.copy_(torch.from_numpy(0.01 * rng.normal(size=(p.n_views, 3))))
    ref.forward()
    P0 = p.poses_init
    delta = ref.delta.cpu().numpy()
    o, cache = omlp.forward(th[0].astype(np.float64), P0.reshape(-1, 12))
    want = omlp.assemble(P0, o, delta)
    got = ref.poses.cpu().numpy()
    e_pose = np.abs(got - want).max()
    say(f"c2 refiner forward: pose diff {e_pose:.2e}, |o| max {np.abs(o).max():.2e}")
    assert e_pose < BF16_TOL * max(np.abs(o).max(), 1e-30)
    # backward from a seeded twist gradient
    g = rng.normal(size=(p.n_views, 6))
    pg, dg = ref.backward(torch.from_numpy(g).cuda())
    d_o, d_delta = omlp.pose_backward(P0, o, want, g)
    want_pg = omlp.backward(th[0].astype(np.float64), cache, d_o)
    got_pg = pg.cpu().numpy()[0].astype(np.float64)
    assert np.array_equal(dg.cpu().numpy(), d_delta)
    for k, ((wo, bo), (out, inp)) in enumerate(zip(omlp.OFFSETS, omlp.LAYERS)):
        eW = rel_norm_err(got_pg[wo:bo], want_pg[wo:bo])
        eb = rel_norm_err(got_pg[bo:bo + out], want_pg[bo:bo + out])
        say(f"layer {k + 1}: dW err {eW:.2e}, db err {eb:.2e}")
        assert eW < BF16_TOL and eb < BF16_TOL


@pytest.mark.parametrize("name", ["two_scenes", "c5"])
def test_scenes_and_chunks(gpu, name):
    """Two scenes with their own parameters; and one scene of 200 views (four
    64-row chunks per workgroup, weight gradients summed over the chunks)."""
    from paper_2607_00579_amd.api import PoseRefiner
    from synth.scenes import config_c1, config_c2, pack
    prob = pack(list(config_c2().scenes) + list(config_c1().scenes), "two") \
        if name == "two_scenes" else problem("c5")
    rng = np.random.default_rng(3)
    th = refiner.init_params(rng, n_scenes=prob.n_scenes, last_std=0.02, bias_std=0.05)
    plan = plan_for(prob)
    ref = PoseRefiner(plan, torch.from_numpy(prob.poses_init.copy()).cuda(),
                      torch.from_numpy(th))
    ref.forward()
    g = rng.normal(size=(prob.n_views, 6))
    pg, _ = ref.backward(torch.from_numpy(g).cuda())
    got = ref.poses.cpu().numpy()
    pg = pg.cpu().numpy()
    for s in range(prob.n_scenes):
        rows = scene_rows(prob, s)
        P0 = prob.poses_init[rows]
        o, cache = omlp.forward(th[s].astype(np.float64), P0.reshape(-1, 12))
        want = omlp.assemble(P0, o, np.zeros((rows.size, 3)))
        assert np.abs(got[rows] - want).max() < BF16_TOL * np.abs(o).max()
        d_o, _ = omlp.pose_backward(P0, o, want, g[rows])
        want_pg = omlp.backward(th[s].astype(np.float64), cache, d_o)
        e = rel_norm_err(pg[s].astype(np.float64), want_pg)
        say(f"{name} scene {s} ({rows.size} views): param grad err {e:.2e}")
        assert e < BF16_TOL


def test_adamw_step(gpu):
    from paper_2607_00579_amd.api import PoseRefiner
    p = problem("c1")
    rng = np.random.default_rng(4)
    th = refiner.init_params(rng, last_std=0.1, bias_std=0.1)
    plan = plan_for(p)
    ref = PoseRefiner(plan, torch.from_numpy(p.poses_init.copy()).cuda(), torch.from_numpy(th))
    g = rng.normal(size=(1, refiner.N_PARAMS)).astype(np.float32)
    gd = rng.normal(size=(p.n_views, 3))
    d0 = rng.normal(size=(p.n_views, 3))
    ref.grad.copy_(torch.from_numpy(g))
    ref.delta_grad.copy_(torch.from_numpy(gd))
    ref.delta.copy_(torch.from_numpy(d0))
    step = torch.zeros(1, dtype=torch.int32, device="cuda")
    x, m, v = th[0].astype(np.float64), np.zeros(refiner.N_PARAMS), np.zeros(refiner.N_PARAMS)
    d, dm, dv = d0.copy(), np.zeros_like(d0), np.zeros_like(d0)
    for k in range(3):
        ref.step(3e-3, step)
        x, m, v = omlp.adamw(x, m, v, g[0].astype(np.float64), k + 1, 3e-3, 0.01)
        d, dm, dv = omlp.adamw(d, dm, dv, gd, k + 1, 3e-3, 0.1)
    assert int(step.item()) == 3
    assert rel_norm_err(ref.params.cpu().numpy()[0], x) < 1e-6
    assert np.abs(ref.delta.cpu().numpy() - d).max() < 1e-14
