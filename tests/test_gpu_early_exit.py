"""GPU: device-side early exit of stopped scenes in the captured iterations
(convergence mode 2).  From the replay after the dual-phase test stops a
scene, that scene's tiles are left out of the fused launch.  Everything else
the loop computes (poses, phases, the other scenes' losses) is bitwise that of
mode 1, where a stopped scene is still evaluated at learning rate 0; a stopped
scene's loss keeps its last evaluated value; eager calls afterwards evaluate
every pair again."""
import numpy as np
import pytest
import torch

from synth import refiner
from tests.gpu_helpers import say

pytestmark = pytest.mark.gpu


def two_scene_problem():
    from synth.scenes import config_c1, config_c2, pack
    return pack(list(config_c2().scenes) + list(config_c1().scenes), "c2+c1")


def check_modes(runs, n):
    """runs[mode] = (poses per replay, losses per replay, phases per replay)."""
    (P1, L1, H1), (P2, L2, H2) = runs[False], runs[True]
    skipped = 0
    for s in range(n):
        assert np.array_equal(P1[s], P2[s]), s
        assert np.array_equal(H1[s], H2[s]), s
        before = H2[s - 1] if s > 0 else np.zeros_like(H2[0])
        for k in range(before.size):
            if before[k] == 2:
                # skipped this replay: the value of the scene's last evaluation
                assert L2[s][k] == L2[s - 1][k], (s, k)
                skipped += 1
            else:
                assert L2[s][k] == L1[s][k], (s, k)
    return skipped


@pytest.mark.parametrize("budget", [0, 9])
def test_pose_loop_early_exit_equals_the_full_loop(gpu, budget):
    from paper_2607_00579_amd.api import EdgePlan
    prob = two_scene_problem()
    cp = (5, 0.15, 8, 0.1)
    n = 60
    dev = torch.device("cuda:0")
    runs, eager, stopped_sel = {}, {}, None
    for mode in (False, True):
        plan = EdgePlan.from_problem(prob)
        poses = torch.from_numpy(prob.poses_init.copy()).to(dev)
        m = torch.zeros(prob.n_views, 6, dtype=torch.float64, device=dev)
        v = torch.zeros_like(m)
        step = torch.zeros(1, dtype=torch.int32, device=dev)
        loss = torch.zeros(prob.n_scenes, dtype=torch.float64, device=dev)
        if budget:
            plan.set_pair_sampling(budget, 7, step)
        plan.convergence_reset(poses, *cp)
        plan.capture_iteration(poses, m, v, step, loss, convergence=True, early_exit=mode)
        P, L, H = [], [], []
        for _ in range(n):
            plan.launch_iteration()
            P.append(poses.cpu().numpy())
            L.append(loss.cpu().numpy().copy())
            H.append(plan.convergence_query()["phase"].copy())
        runs[mode] = (P, L, H)
        if mode:
            # the last replay's launch skipped the scenes stopped before it
            stopped_sel = (H[-2], plan.sampled_pairs().cpu().numpy())
        # an eager call after the loop evaluates every pair (every sampled
        # pair) of every scene again
        o = plan.cost(poses, 6.0, grad=True)
        eager[mode] = (o["loss"].cpu().numpy(), o["grad"].cpu().numpy())
        assert plan.device_status() == 0
    skipped = check_modes(runs, n)
    switch = [np.flatnonzero(np.array([h[k] for h in runs[True][2]]) == 2)[:1].tolist()
              for k in range(prob.n_scenes)]
    say(f"early exit (budget {budget}): first stopped replay per scene {switch}, "
        f"{skipped} scene-replays skipped")
    assert skipped > 0
    phase, sel = stopped_sel
    for k in np.flatnonzero(phase == 2):
        assert not sel[prob.scene_of_pair == k].any()
    for k in np.flatnonzero(phase != 2):
        assert sel[prob.scene_of_pair == k].any()
    assert np.array_equal(eager[False][0], eager[True][0])
    assert np.array_equal(eager[False][1], eager[True][1])


def test_refiner_loop_early_exit_equals_the_full_loop(gpu):
    from paper_2607_00579_amd.api import EdgePlan, PoseRefiner
    prob = two_scene_problem()
    cp = (3, 3.0, 4, 1.5)
    n = 30
    dev = torch.device("cuda:0")
    th = refiner.init_params(np.random.default_rng(5), n_scenes=prob.n_scenes)
    runs, params = {}, {}
    for mode in (False, True):
        plan = EdgePlan.from_problem(prob)
        ref = PoseRefiner(plan, torch.from_numpy(prob.poses_init.copy()).to(dev),
                          torch.from_numpy(th))
        step = torch.zeros(1, dtype=torch.int32, device=dev)
        loss = torch.zeros(prob.n_scenes, dtype=torch.float64, device=dev)
        ref.capture_iteration(step, loss, convergence=cp, early_exit=mode)
        P, L, H = [], [], []
        for _ in range(n):
            plan.launch_iteration()
            P.append(ref.poses.cpu().numpy())
            L.append(loss.cpu().numpy().copy())
            H.append(plan.convergence_query()["phase"].copy())
        runs[mode] = (P, L, H)
        params[mode] = (ref.params.cpu().numpy(), ref.delta.cpu().numpy())
        assert plan.device_status() == 0
    skipped = check_modes(runs, n)
    say(f"refiner loop early exit: final phases {runs[True][2][-1].tolist()}, "
        f"{skipped} scene-replays skipped")
    assert skipped > 0
    assert np.array_equal(params[False][0], params[True][0])
    assert np.array_equal(params[False][1], params[True][1])
