"""GPU: the two-phase loop with focal and depth refinement captured as one
graph (schedule -> cost with pose, focal and depth gradients -> joint AdamW
gated by the device phase -> pose step -> convergence test), on a two-scene
batch.  The trajectory is chaotic like the pose loop's, so every replay is
checked against the oracle from the device's own state before it: the
gradients against the oracle evaluated at that refined state, the optimizer
arithmetic (AdamW on gamma, alpha, beta with per-scene step counts; Adam on
the twists) against the oracle's steps fed the device's gradients, and the
phases against the oracle's dual-phase test fed the device's poses."""
import numpy as np
import pytest
import torch

from oracle import convergence as oconv
from oracle import cost as ocost
from oracle import joint as oj
from oracle import loop as oloop
from tests.gpu_helpers import check_depth, oracle_index, problem, rel_norm_err, say

pytestmark = pytest.mark.gpu


def two_scene_problem():
    from synth.scenes import config_c1, config_c2, pack
    return pack(list(config_c2().scenes) + list(config_c1().scenes), "c2+c1")


def to_oracle_order(a, views, idx, op):
    """A plan-order per-record array in the oracle's order (views in order,
    each view's edge pixels row-major)."""
    off = np.cumsum([0] + [op.pts[v][0].size for v in range(op.V)])
    out = np.zeros(off[-1], a.dtype)
    out[off[views] + idx] = a
    return out


def first_moment_ok(got, want, prev_m, g):
    scale = 0.9 * np.abs(prev_m) + 0.1 * np.abs(g)
    return np.all(np.abs(got - want) <= 1e-14 * scale + 1e-13 * np.abs(want))


def host(state):
    return {k: t.detach().cpu().numpy().copy() for k, t in state.items()}


@pytest.mark.parametrize("early_exit", [False, True])
def test_joint_loop_every_replay_against_the_oracle(gpu, early_exit):
    from paper_2607_00579_amd.api import EdgePlan
    prob = two_scene_problem()
    dev = torch.device("cuda:0")
    plan = EdgePlan.from_problem(prob, device=dev)
    S, V, n = plan.n_scenes, plan.n_views, plan.n_records
    views, idx = oracle_index(prob, plan)
    vor = views
    sov = np.asarray(plan.scene_of_view, np.int64)
    op = ocost.OracleProblem(prob)
    off = np.cumsum([0] + [op.pts[x][0].size for x in range(op.V)])
    poses = torch.from_numpy(prob.poses_init.copy()).to(dev)
    m = torch.zeros(V, 6, dtype=torch.float64, device=dev)
    v = torch.zeros_like(m)
    step = torch.zeros(1, dtype=torch.int32, device=dev)
    loss = torch.zeros(S, dtype=torch.float64, device=dev)
    grad = torch.zeros(V, 6, dtype=torch.float64, device=dev)
    state = plan.joint_state()
    # phase 1 once three signals are in (the depth parameters step from the
    # fourth replay), the stop after seven (nothing steps from the eighth)
    conv = (2, 1e9, 4, 1e9)
    plan.convergence_reset(poses, *conv)
    plan.capture_joint_iteration(poses, m, v, step, loss, state, grad=grad, convergence=True,
                                 early_exit=early_exit)
    dual = [oconv.DualPhase(*conv) for _ in range(S)]
    worst = dict(loss=0.0, grad=0.0, gamma_grad=0.0)
    for k in range(9):
        phase = plan.convergence_query()["phase"].copy()
        assert list(phase) == [d.phase for d in dual], (k, phase)
        P0 = poses.cpu().numpy()
        m0, v0 = m.cpu().numpy(), v.cpu().numpy()
        st0 = host(state)
        plan.launch_iteration()
        torch.cuda.synchronize()
        st1 = host(state)
        P1 = poses.cpu().numpy()
        lr = np.array([0.0 if ph == 2 else oloop.learning_rate(k) for ph in phase])
        active = phase != 2
        # gradients against the oracle at the device's refined state
        al = to_oracle_order(st0["alpha"][:n].astype(np.float64), views, idx, op)
        be = to_oracle_order(st0["beta"][:n].astype(np.float64), views, idx, op)
        K, depth = oloop.joint_refinement(op, st0["gamma"], al, be)
        r = op.evaluate(P0, oloop.clamp_lambda(k), ocost.CostParams(), K=K, depth=depth)
        gr = oloop.joint_gradients(op, r, st0["gamma"])
        sc = np.flatnonzero(active)
        rv = np.isin(sov, sc)
        g_pose = grad.cpu().numpy()
        if sc.size == 0:
            e_loss = e_grad = e_gam = 0.0
        else:
            e_loss = float(np.max(np.abs(loss.cpu().numpy()[sc] - r["loss"][sc])
                                  / np.abs(r["loss"][sc])))
            e_grad = rel_norm_err(g_pose[rv], r["grad"][rv], axis=1)
            e_gam = rel_norm_err(st1["grad_gamma"][:V][rv], gr["grad_gamma"][rv])
        assert e_loss < 1e-5 and e_grad < 1e-4 and e_gam < 1e-4, (k, e_loss, e_grad, e_gam)
        worst["loss"] = max(worst["loss"], e_loss)
        worst["grad"] = max(worst["grad"], e_grad)
        worst["gamma_grad"] = max(worst["gamma_grad"], e_gam)
        recs = np.isin(sov[vor], sc)
        if recs.any():
            for name in ("grad_alpha", "grad_beta"):
                want = gr[name][off[views] + idx]          # oracle order -> plan order
                check_depth(st1[name][:n][recs], want[recs], f"replay {k} {name}")
        # optimizer arithmetic: the oracle's steps fed the device's gradients
        g_dev = {"grad_gamma": st1["grad_gamma"][:V], "grad_alpha": st1["grad_alpha"][:n],
                 "grad_beta": st1["grad_beta"][:n]}
        prev = {"gamma": st0["gamma"], "alpha": st0["alpha"][:n], "beta": st0["beta"][:n],
                "m_gamma": st0["m_gamma"], "v_gamma": st0["v_gamma"],
                "m_alpha": st0["m_depth"][:n], "v_alpha": st0["v_depth"][:n],
                "m_beta": st0["m_depth"][n:2 * n], "v_beta": st0["v_depth"][n:2 * n],
                "steps": st0["steps"].reshape(2, S).astype(np.int64)}
        want = oj.joint_step(prev, g_dev, lr, sov, vor, phase=phase)
        assert np.array_equal(st1["steps"], want["steps"].reshape(-1)), k
        np.testing.assert_allclose(st1["gamma"], want["gamma"], rtol=1e-13, atol=1e-300)
        for i, name in enumerate(("alpha", "beta")):
            w = want[name].astype(np.float32)
            err = np.abs(st1[name][:n].astype(np.float64) - w.astype(np.float64))
            assert np.all(err <= np.spacing(np.abs(w)).astype(np.float64)), (k, name)
            assert first_moment_ok(st1["m_depth"][i * n:(i + 1) * n], want["m_" + name],
                                   prev["m_" + name], g_dev["grad_" + name]), (k, name)
        # the pose step from the device's pose gradient
        Pw, mw, vw = oloop.adam_se3_step(P0, m0, v0, g_pose, k + 1, lr, scene_of_view=sov)
        assert np.abs(P1 - Pw).max() < 1e-12 and np.abs(m.cpu().numpy() - mw).max() < 1e-12, k
        # the phases: the oracle's test fed the device's pose change
        for s in range(S):
            vs = np.flatnonzero(sov == s)
            dual[s].update(oconv.theta95(P1[vs], P0[vs]))
    assert [d.phase for d in dual] == [2, 2]
    assert state["steps"].cpu().tolist() == [7, 7, 4, 4]
    say(f"joint loop ({'early exit' if early_exit else 'stopped scenes evaluated'}): 9 replays, "
        f"worst loss {worst['loss']:.2e}, pose grad {worst['grad']:.2e}, "
        f"focal grad {worst['gamma_grad']:.2e}")
    assert plan.device_status() == 0


def test_joint_loop_without_the_test_steps_everything(gpu):
    """with_convergence 0: gamma, alpha and beta all step from the first
    replay (the depth optimizer's step 1 is the closed form), and three
    replays equal three eager calls of the same launches bitwise."""
    from paper_2607_00579_amd import _lib
    from paper_2607_00579_amd.api import EdgePlan
    prob = problem("c1")
    dev = torch.device("cuda:0")
    outs = []
    for mode in ("graph", "eager"):
        plan = EdgePlan.from_problem(prob, device=dev)
        poses = torch.from_numpy(prob.poses_init.copy()).to(dev)
        m = torch.zeros(plan.n_views, 6, dtype=torch.float64, device=dev)
        v = torch.zeros_like(m)
        step = torch.zeros(1, dtype=torch.int32, device=dev)
        loss = torch.zeros(1, dtype=torch.float64, device=dev)
        state = plan.joint_state()
        if mode == "graph":
            plan.capture_joint_iteration(poses, m, v, step, loss, state)
            for _ in range(3):
                plan.launch_iteration()
        else:
            lam = torch.zeros(1, dtype=torch.float32, device=dev)
            lr = torch.zeros(1, dtype=torch.float64, device=dev)
            st = torch.cuda.current_stream().cuda_stream
            plan.set_refinement(state["gamma"], state["alpha"], state["beta"])
            for _ in range(3):
                _lib.schedule(step, 1, 10.0, 6.0, 1000, 3e-3, 25, 2000, lam, lr, st)
                g = plan.refine(poses, lam)
                loss.copy_(g["loss"])
                plan.joint_step(state, g, lr)
                plan.pose_step(poses, m, v, g["grad"], lr, step)
        torch.cuda.synchronize()
        outs.append((poses.cpu().numpy(), host(state), loss.cpu().numpy()))
    (P1, s1, l1), (P2, s2, l2) = outs
    assert np.array_equal(P1, P2) and np.array_equal(l1, l2)
    for k in ("gamma", "alpha", "beta", "m_depth", "v_depth", "steps"):
        assert np.array_equal(s1[k], s2[k]), k
    assert s1["steps"].tolist() == [3, 3]
