"""GPU: a captured graph holding several iterations (plan option graph_steps)
runs exactly the iterations of as many one-iteration launches: the poses,
Adam moments, step counter, last loss and convergence phases come out
bitwise equal (the pose loop with the convergence test and early exit, on two
scenes, with and without pair sub-sampling)."""
import numpy as np
import pytest
import torch

from tests.gpu_helpers import say

pytestmark = pytest.mark.gpu


def two_scene_problem():
    from synth.scenes import config_c1, config_c2, pack
    return pack(list(config_c2().scenes) + list(config_c1().scenes), "c2+c1")


def run(prob, graph_steps, launches, budget):
    from paper_2607_00579_amd.api import EdgePlan
    dev = torch.device("cuda:0")
    plan = EdgePlan.from_problem(prob)
    plan.set_options(**dict(plan.info()["options"], graph_steps=graph_steps))
    assert plan.info()["options"]["graph_steps"] == graph_steps
    poses = torch.from_numpy(prob.poses_init.copy()).to(dev)
    m = torch.zeros(prob.n_views, 6, dtype=torch.float64, device=dev)
    v = torch.zeros_like(m)
    step = torch.zeros(1, dtype=torch.int32, device=dev)
    loss = torch.zeros(prob.n_scenes, dtype=torch.float64, device=dev)
    if budget:
        plan.set_pair_sampling(budget, 7, step)
    plan.convergence_reset(poses, 5, 0.15, 8, 0.1)
    plan.capture_iteration(poses, m, v, step, loss, convergence=True, early_exit=True)
    for _ in range(launches):
        plan.launch_iteration()
    torch.cuda.synchronize()
    assert plan.device_status() == 0
    c = plan.convergence_query()
    return (poses.cpu().numpy(), m.cpu().numpy(), v.cpu().numpy(), int(step.item()),
            loss.cpu().numpy(), c["phase"], c["switch_steps"], c["steps"], c["theta_last"])


@pytest.mark.parametrize("budget", [0, 9])
def test_several_steps_per_graph_equal_single_steps(gpu, budget):
    prob = two_scene_problem()
    n = 48
    ref = run(prob, 1, n, budget)
    assert ref[3] == n
    for g in (4, 16):
        got = run(prob, g, n // g, budget)
        say(f"graph_steps {g}: step {got[3]}, phases {got[5].tolist()}")
        for a, b in zip(ref, got):
            assert np.array_equal(np.asarray(a), np.asarray(b)), g


def test_graph_steps_out_of_range_rejected(gpu):
    from paper_2607_00579_amd import _lib
    from paper_2607_00579_amd.api import EdgePlan
    from synth.scenes import config_c1, pack
    plan = EdgePlan.from_problem(pack(list(config_c1().scenes), "c1"))
    for bad in (-1, 65):
        with pytest.raises(_lib.EpoError):
            plan.set_options(**dict(plan.info()["options"], graph_steps=bad))
