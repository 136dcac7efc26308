"""GPU: stochastic viewgraph sub-sampling on the device against the oracle:
the drawn pair subsets (bit-exact), the loss and gradient of a sub-sampled
step, and a captured loop that draws a fresh subset at every replay."""
import numpy as np
import pytest
import torch

from oracle import cost as ocost
from oracle import loop as oloop
from oracle import sampling as osamp
from synth.scenes import config_c1, config_c2, pack
from tests.gpu_helpers import problem, rel_norm_err, rotation_angle_deg, say

pytestmark = pytest.mark.gpu


def plan_for(prob, **kw):
    from paper_2607_00579_amd.api import EdgePlan
    return EdgePlan.from_problem(prob, device="cuda:0", **kw)


def two_scenes():
    return pack(list(config_c2().scenes) + list(config_c1().scenes), "c2+c1")


def device_selection(plan, poses, step_t, s):
    step_t.fill_(s)
    plan.cost(poses, 10.0, grad=False)
    return plan.sampled_pairs().cpu().numpy()


@pytest.mark.parametrize("name", ["c2", "two"])
def test_device_subsets_equal_the_oracle(gpu, name):
    p = problem("c2") if name == "c2" else two_scenes()
    plan = plan_for(p)
    P = torch.from_numpy(p.poses_init.copy()).cuda()
    step_t = torch.zeros(1, dtype=torch.int32, device="cuda")
    for seed in (0, (1 << 63) + 5):
        for budget in (1, 5, 27, 28, 100):
            plan.set_pair_sampling(budget, seed, step_t)
            for s in (0, 1, 2, 3, 1000):
                got = device_selection(plan, P, step_t, s)
                want = osamp.selected_pairs(p.pairs, p.scene_of_pair, seed, s, budget)
                assert np.array_equal(got, want), (seed, budget, s)
    plan.set_pair_sampling(0)
    plan.cost(P, 10.0, grad=False)
    assert plan.sampled_pairs().all()


def test_device_subsets_on_the_batch_workload(gpu):
    """64 scenes, up to 1128 image pairs each: radix selection with several
    keys per thread."""
    p = problem("c4")
    plan = plan_for(p)
    P = torch.from_numpy(p.poses_init.copy()).cuda()
    step_t = torch.zeros(1, dtype=torch.int32, device="cuda")
    for budget in (1024, 100):
        plan.set_pair_sampling(budget, 12345, step_t)
        for s in (0, 7):
            got = device_selection(plan, P, step_t, s)
            want = osamp.selected_pairs(p.pairs, p.scene_of_pair, 12345, s, budget)
            assert np.array_equal(got, want), (budget, s)
            say(f"c4 budget {budget} step {s}: {int(got.sum())} of {got.size} directed pairs")


@pytest.mark.parametrize("options", [None, dict(persistent=1, points_per_thread=2),
                                     dict(persistent=2, points_per_thread=1, tile_order=2)])
def test_sampled_step_cost_and_gradient(gpu, options):
    """Only the selected pairs' tiles run (compacted tile list), in both launch
    forms and tile sizes."""
    p = problem("c2")
    plan = plan_for(p, options=options)
    P = torch.from_numpy(p.poses_init.copy()).cuda()
    step_t = torch.full((1,), 3, dtype=torch.int32, device="cuda")
    plan.set_pair_sampling(9, 77, step_t)
    g = {k: v.cpu().numpy() for k, v in plan.cost(P, 10.0, grad=True, pairs=True).items()}
    sel = osamp.selected_pairs(p.pairs, p.scene_of_pair, 77, 3, 9)
    r = ocost.OracleProblem(p).evaluate(p.poses_init, 10.0, selected=sel)
    assert rel_norm_err(g["loss"], r["loss"]) < 1e-4
    e_t = rel_norm_err(g["grad"][:, :3], r["grad"][:, :3], axis=1)
    e_r = rel_norm_err(g["grad"][:, 3:], r["grad"][:, 3:], axis=1)
    say(f"c2 sub-sampled step: grad err t {e_t:.2e} r {e_r:.2e}")
    assert e_t < 1e-4 and e_r < 1e-4
    assert np.all(g["pair_valid"][~sel] == 0) and np.all(g["pair_cost"][~sel] == 0)
    assert np.array_equal(g["pair_valid"][sel], r["n"][sel])
    # sub-sampling off again: the full evaluation, bit for bit
    plan.set_pair_sampling(0)
    full = plan.cost(P, 10.0, grad=True)
    plan2 = plan_for(p, options=options)
    ref = plan2.cost(P, 10.0, grad=True)
    assert torch.equal(full["loss"], ref["loss"]) and torch.equal(full["grad"], ref["grad"])


def test_captured_loop_draws_a_fresh_subset_each_step(gpu):
    """Ten replays of the captured iteration with M = 10 of c2's 28 image
    pairs against the oracle loop with the same draws: losses and final
    rotations (the same 10-step window bars as the full-graph loop)."""
    p = problem("c2")
    plan = plan_for(p)
    P = torch.from_numpy(p.poses_init.copy()).cuda()
    m = torch.zeros(p.n_views, 6, dtype=torch.float64, device="cuda")
    v = torch.zeros_like(m)
    step = torch.zeros(1, dtype=torch.int32, device="cuda")
    loss = torch.zeros(1, dtype=torch.float64, device="cuda")
    plan.set_pair_sampling(10, 2024, step)
    plan.capture_iteration(P, m, v, step, loss)
    seen, losses = [], []
    for _ in range(10):
        plan.launch_iteration()
        losses.append(float(loss.item()))
        seen.append(plan.sampled_pairs().cpu().numpy())
    assert int(step.item()) == 10
    assert len({x.tobytes() for x in seen}) == 10
    for s, x in enumerate(seen):
        assert np.array_equal(x, osamp.selected_pairs(p.pairs, p.scene_of_pair, 2024, s, 10))
    h = oloop.run(ocost.OracleProblem(p), p.poses_init, 10, sampling=(2024, 10))
    rel = max(abs(a - b[0]) / b[0] for a, b in zip(losses, h["loss"]))
    got = P.cpu().numpy()
    worst = max(rotation_angle_deg(got[k][:, :3], h["final_poses"][k][:, :3])
                for k in range(p.n_views))
    say(f"c2 sub-sampled loop: worst loss rel err {rel:.2e}, worst rotation diff {worst:.2e} deg")
    assert rel < 1e-5 and worst < 5e-3
