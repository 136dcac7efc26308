"""GPU: a captured graph holding several iterations (plan option graph_steps)
runs exactly the iterations of as many one-iteration launches: everything
the loop carries comes out bitwise equal, for the pose loop (convergence
test, early exit, with and without pair sub-sampling), the refiner loop and
the two-phase loop with focal and depth refinement.  And a small plan's
captured iteration, whose reductions and pose step run as one workgroup,
equals eager steps through the separate kernels bitwise."""
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


def _equal(a, b, what):
    if isinstance(a, dict):
        assert a.keys() == b.keys(), what
        for k in a:
            _equal(a[k], b[k], f"{what}.{k}")
    else:
        assert np.array_equal(np.asarray(a), np.asarray(b)), what


def run_refiner(prob, graph_steps, launches):
    from paper_2607_00579_amd.api import EdgePlan, PoseRefiner
    dev = torch.device("cuda:0")
    plan = EdgePlan.from_problem(prob)
    plan.set_options(**dict(plan.info()["options"], graph_steps=graph_steps))
    ref = PoseRefiner(plan, torch.from_numpy(prob.poses_init.copy()).to(dev), seed=0)
    step = torch.zeros(1, dtype=torch.int32, device=dev)
    loss = torch.zeros(prob.n_scenes, dtype=torch.float64, device=dev)
    grad = torch.zeros(prob.n_views, 6, dtype=torch.float64, device=dev)
    ref.capture_iteration(step, loss, grad)
    for _ in range(launches):
        plan.launch_iteration()
    torch.cuda.synchronize()
    state = {k: getattr(ref, k).cpu().numpy().copy()
             for k in ("params", "m", "v", "grad", "delta", "dm", "dv", "delta_grad", "poses")}
    return dict(state=state, step=int(step.item()), loss=loss.cpu().numpy(),
                grad=grad.cpu().numpy())


def test_refiner_loop_several_steps_per_graph(gpu):
    """The refiner loop (MLP forward and backward on matrix cores, AdamW)
    captured 4 or 12 iterations to a graph equals 12 one-iteration launches
    bitwise."""
    from synth.scenes import config_c1, pack
    prob = pack(list(config_c1().scenes), "c1")
    ref = run_refiner(prob, 1, 12)
    assert ref["step"] == 12
    for g in (4, 12):
        _equal(ref, run_refiner(prob, g, 12 // g), f"graph_steps {g}")


def run_joint(prob, graph_steps, launches, early_exit):
    from paper_2607_00579_amd.api import EdgePlan
    dev = torch.device("cuda:0")
    plan = EdgePlan.from_problem(prob, device=dev)
    plan.set_options(**dict(plan.info()["options"], graph_steps=graph_steps))
    poses = torch.from_numpy(prob.poses_init.copy()).to(dev)
    m = torch.zeros(plan.n_views, 6, dtype=torch.float64, device=dev)
    v = torch.zeros_like(m)
    step = torch.zeros(1, dtype=torch.int32, device=dev)
    loss = torch.zeros(plan.n_scenes, dtype=torch.float64, device=dev)
    grad = torch.zeros(plan.n_views, 6, dtype=torch.float64, device=dev)
    state = plan.joint_state()
    plan.convergence_reset(poses, 2, 1e9, 4, 1e9)
    plan.capture_joint_iteration(poses, m, v, step, loss, state, grad=grad, convergence=True,
                                 early_exit=early_exit)
    for _ in range(launches):
        plan.launch_iteration()
    torch.cuda.synchronize()
    assert plan.device_status() == 0
    return dict(poses=poses.cpu().numpy(), m=m.cpu().numpy(), v=v.cpu().numpy(),
                step=int(step.item()), loss=loss.cpu().numpy(), grad=grad.cpu().numpy(),
                state={k: t.detach().cpu().numpy().copy() for k, t in state.items()},
                conv={k: np.asarray(x) for k, x in plan.convergence_query().items()})


@pytest.mark.parametrize("early_exit", [False, True])
def test_joint_loop_several_steps_per_graph(gpu, early_exit):
    """The two-phase loop with focal and depth refinement (the depth step
    switches on after the third iteration, the scenes stop after the
    seventh) captured 4 or 8 iterations to a graph equals 8 one-iteration
    launches bitwise: poses, moments, refinement state, phases."""
    prob = two_scene_problem()
    ref = run_joint(prob, 1, 8, early_exit)
    assert ref["step"] == 8 and ref["conv"]["phase"].tolist() == [2, 2]
    for g in (4, 8):
        _equal(ref, run_joint(prob, g, 8 // g, early_exit), f"graph_steps {g}")


def _eager_and_captured(prob, n):
    """n eager steps (schedule -> cost + adjoint -> separate reductions ->
    pose step) and n replays of the captured iteration, from the same start."""
    from paper_2607_00579_amd import _lib
    from paper_2607_00579_amd.api import EdgePlan
    dev = torch.device("cuda:0")
    plan = EdgePlan.from_problem(prob)
    poses0 = torch.from_numpy(prob.poses_init.copy()).to(dev)
    out = []
    for captured in (False, True):
        P = poses0.clone()
        m = torch.zeros(prob.n_views, 6, dtype=torch.float64, device=dev)
        v = torch.zeros_like(m)
        s = torch.zeros(1, dtype=torch.int32, device=dev)
        loss = torch.zeros(plan.n_scenes, dtype=torch.float64, device=dev)
        grad = torch.zeros(prob.n_views, 6, dtype=torch.float64, device=dev)
        if captured:
            plan.capture_iteration(P, m, v, s, loss, grad)
            for _ in range(n):
                plan.launch_iteration()
        else:
            lam = torch.zeros(plan.n_scenes, dtype=torch.float32, device=dev)
            lr = torch.zeros(plan.n_scenes, dtype=torch.float64, device=dev)
            st = torch.cuda.current_stream().cuda_stream
            for _ in range(n):
                _lib.schedule(s, plan.n_scenes, 10.0, 6.0, 1000, 3e-3, 25, 2000, lam, lr, st)
                o = plan.cost(P, lam, grad=True)
                loss.copy_(o["loss"])
                grad.copy_(o["grad"])
                plan.pose_step(P, m, v, o["grad"], lr, s)
        torch.cuda.synchronize()
        out.append([P.cpu().numpy(), m.cpu().numpy(), v.cpu().numpy(), loss.cpu().numpy(),
                    grad.cpu().numpy(), int(s.item())])
    return out


@pytest.mark.parametrize("case", ["c2", "c1+one-view", "one-view"])
def test_small_plan_epilogue_equals_separate_kernels(gpu, case):
    """A small plan's captured iteration runs its reductions, pose step and
    step count as one workgroup; eager calls run the separate kernels: after
    12 steps the poses, moments, last loss and gradient and the step counter
    are bitwise equal (the 8-view scene, a batch with a scene that has no
    pairs, and a plan with no pair at all: zero loss and gradient, poses
    unchanged)."""
    from synth import fixtures
    from synth.scenes import config_c1, config_c2, pack
    if case == "c2":
        prob = pack(list(config_c2().scenes), "c2")
    else:
        p = fixtures.odd_size_views()
        one = fixtures.problem_from_maps([p.width[0]], [p.height[0]], [p.K[0]], [p.edge_map(0)],
                                         [p.depth_map(0)], [p.poses_init[0]], np.zeros((0, 2)),
                                         name="one_view")
        if case == "one-view":
            prob = one          # no pair at all: the schedule runs as its own kernel
        else:
            prob = pack(list(config_c1().scenes) + list(one.scenes), "c1+one")
    eager, captured = _eager_and_captured(prob, 12)
    assert eager[5] == captured[5] == 12
    if case == "one-view":
        assert not np.any(captured[3]) and not np.any(captured[4])
        assert np.array_equal(captured[0], prob.poses_init)
    for a, b, what in zip(eager, captured, ("poses", "m", "v", "loss", "grad", "step")):
        assert np.array_equal(np.asarray(a), np.asarray(b)), what
