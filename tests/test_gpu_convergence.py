"""GPU: pose-change signal and dual-phase convergence on the device, against
the oracle's (same pose sequences; then inside the captured iteration)."""
import numpy as np
import pytest
import torch
from scipy.spatial.transform import Rotation

from oracle import convergence as oconv
from oracle import cost as ocost
from oracle import loop as oloop
from synth.scenes import pack
from tests.gpu_helpers import problem, say

pytestmark = pytest.mark.gpu


def two_scene_problem():
    # generated here: problems read back from the on-disk input cache carry
    # packed arrays only, not their scenes
    from synth.scenes import config_c1, config_c2
    return pack(list(config_c2().scenes) + list(config_c1().scenes), "c2+c1")


def test_signal_and_phases_on_a_given_pose_sequence(gpu):
    """Feed the same pose sequence to the device and to the oracle: theta_95
    per scene and step agrees to 1e-9 deg, the switch steps are identical."""
    from paper_2607_00579_amd.api import EdgePlan
    prob = two_scene_problem()
    plan = EdgePlan.from_problem(prob)
    rng = np.random.default_rng(3)
    V, S = prob.n_views, 2
    w1, e1, w2, e2 = 4, 0.5, 6, 0.1
    P = prob.poses_init.copy()
    dev = torch.device("cuda:0")
    Pt = torch.from_numpy(P).to(dev)
    plan.convergence_reset(Pt, w1, e1, w2, e2)
    duals = [oconv.DualPhase(w1, e1, w2, e2) for _ in range(S)]
    th_dev = torch.zeros(S, dtype=torch.float64, device=dev)
    ph_dev = torch.zeros(S, dtype=torch.int32, device=dev)
    worst = 0.0
    for s in range(60):
        # rotations and translations shrinking over the run, different per view
        Pn = P.copy()
        for v in range(V):
            ang = 3.0 * 0.93 ** s * rng.uniform(0.2, 1.0)
            Rn = Rotation.from_rotvec(np.radians(ang) * rng.normal(size=3) / np.sqrt(3)).as_matrix()
            Pn[v][:, :3] = Rn @ P[v][:, :3]
            Pn[v][:, 3] = P[v][:, 3] + 0.05 * 0.93 ** s * rng.normal(size=3)
        Pt.copy_(torch.from_numpy(Pn))
        plan.convergence_update(Pt, th_dev, ph_dev)
        th = th_dev.cpu().numpy()
        for k in range(S):
            views = np.flatnonzero(prob.scene_of_view == k)
            want = oconv.theta95(Pn[views], P[views])
            duals[k].update(want)
            worst = max(worst, abs(th[k] - want))
        assert list(ph_dev.cpu().numpy()) == [d.phase for d in duals], s
        P = Pn
    q = plan.convergence_query()
    say(f"convergence on a given sequence: worst theta diff {worst:.2e} deg, switch steps "
        f"{q['switch_steps'].tolist()} (oracle {[d.switch_step for d in duals]})")
    assert worst < 1e-9
    assert q["switch_steps"].tolist() == [[-1 if x is None else x for x in d.switch_step]
                                          for d in duals]
    assert all(d.phase == 2 for d in duals)
    assert list(q["steps"]) == [60, 60]


def test_captured_iteration_with_convergence_c1(gpu):
    """Whole loop on the device: the scene switches phase and stops at the
    oracle's steps, and its poses stay fixed after the stop."""
    from paper_2607_00579_amd.api import EdgePlan
    prob = problem("c1")
    w1, e1, w2, e2 = 5, 0.15, 8, 0.1
    n = 60
    ref = oloop.run_with_convergence(ocost.OracleProblem(prob), prob.poses_init, n,
                                     w1=w1, eps1=e1, w2=w2, eps2=e2)
    dev = torch.device("cuda:0")
    plan = EdgePlan.from_problem(prob)
    poses = torch.from_numpy(prob.poses_init.copy()).to(dev)
    m = torch.zeros(prob.n_views, 6, dtype=torch.float64, device=dev)
    v = torch.zeros_like(m)
    step = torch.zeros(1, dtype=torch.int32, device=dev)
    loss = torch.zeros(1, dtype=torch.float64, device=dev)
    plan.convergence_reset(poses, w1, e1, w2, e2)
    plan.capture_iteration(poses, m, v, step, loss, convergence=True)
    frozen = None
    for s in range(n):
        plan.launch_iteration()
        q = plan.convergence_query()
        if q["phase"][0] == 2 and frozen is None:
            frozen = poses.clone()
    q = plan.convergence_query()
    say(f"c1 loop with convergence: switch steps {q['switch_steps'].tolist()} "
        f"(oracle {ref['switch_steps']})")
    assert q["switch_steps"][0].tolist() == ref["switch_steps"][0]
    assert frozen is not None and torch.equal(frozen, poses)
    ang = max(oconv.rotation_change_deg(poses.cpu().numpy()[k][:, :3],
                                        ref["final_poses"][k][:, :3]) for k in range(2))
    assert ang < 0.01
