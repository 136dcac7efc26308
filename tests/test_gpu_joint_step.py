"""GPU: the joint-phase optimizer step (AdamW on focal scales gamma and the
per-record depth scale alpha and shift beta, with the convergence-phase gate)
through the C-ABI, against the FP64 oracle on the same seeded state and
gradients, on a two-scene batch with one learning rate per scene; and the
refinement it leaves in the plan against an explicit set_refinement."""
import numpy as np
import pytest
import torch

from oracle import joint as oj
from tests.gpu_helpers import say

pytestmark = pytest.mark.gpu


def two_scene_problem():
    from synth.scenes import config_c1, config_c2, pack
    return pack(list(config_c2().scenes) + list(config_c1().scenes), "c2+c1")


def setup(seed=0):
    from paper_2607_00579_amd.api import EdgePlan
    prob = two_scene_problem()
    plan = EdgePlan.from_problem(prob, device="cuda:0")
    V, n = plan.n_views, plan.n_records
    vor = plan.record_pixels()[:, 0]
    sv = np.asarray(plan.scene_of_view, np.int64)
    rng = np.random.default_rng(seed)
    host = oj.initial_state(V, n, plan.n_scenes)
    host["gamma"] = rng.normal(0, 0.02, V)
    host["alpha"] = (1 + rng.normal(0, 0.05, n)).astype(np.float32)
    host["beta"] = rng.normal(0, 0.05, n).astype(np.float32)
    dev = plan.joint_state()
    dev["gamma"].copy_(torch.from_numpy(host["gamma"]))
    dev["alpha"].copy_(torch.from_numpy(host["alpha"]))
    dev["beta"].copy_(torch.from_numpy(host["beta"]))
    return prob, plan, sv, vor, rng, host, dev


def grads_of(rng, V, n):
    return {"grad_gamma": rng.normal(0, 1e-2, V), "grad_alpha": rng.normal(0, 1e-3, n),
            "grad_beta": rng.normal(0, 1e-3, n)}


def check_first_moment(got, want, prev_m, g, tag):
    """m = b1 m_prev + (1 - b1) g can cancel; one side fusing the product
    into the sum changes the result by about 2^-53 of the terms' size, not of
    the result's, and later steps carry that difference on scaled by b1: the
    bound is 1e-14 of the terms' size."""
    scale = 0.9 * np.abs(prev_m) + 0.1 * np.abs(g)
    err = np.abs(got - want)
    assert np.all(err <= 1e-14 * scale + 1e-13 * np.abs(want)), \
        f"{tag}: worst {np.max(err / (scale + 1e-300)):.2e} of the terms' size"


def compare(dev, want, prev, g, n, tag):
    got = {k: t.cpu().numpy() for k, t in dev.items()}
    assert np.array_equal(got["steps"], want["steps"].reshape(-1)), f"{tag} step counts"
    for k in ("gamma", "v_gamma"):
        np.testing.assert_allclose(got[k], want[k], rtol=1e-13, atol=1e-300, err_msg=f"{tag} {k}")
    check_first_moment(got["m_gamma"], want["m_gamma"], prev["m_gamma"], g["grad_gamma"],
                       f"{tag} m_gamma")
    for i, k in enumerate(("alpha", "beta")):
        # float64 step rounded once to float32: at most one float32 ulp apart
        # (the two sides may contract multiply-adds differently)
        w = want[k].astype(np.float32)
        ulp = np.spacing(np.abs(w)).astype(np.float64)
        err = np.abs(got[k].astype(np.float64) - w.astype(np.float64))
        assert np.all(err <= ulp), f"{tag} {k}: {int((err > ulp).sum())} beyond one ulp"
        np.testing.assert_allclose(got["v_depth"][i * n:(i + 1) * n], want["v_" + k],
                                   rtol=1e-13, atol=1e-300, err_msg=f"{tag} v_{k}")
        check_first_moment(got["m_depth"][i * n:(i + 1) * n], want["m_" + k], prev["m_" + k],
                           g["grad_" + k], f"{tag} m_{k}")


def test_joint_step_matches_oracle(gpu):
    """Four steps (two ungated, then phases (0, 1) and (1, 2)) with learning
    rates 3e-3 and 1e-3 by scene and the paper's weight decay."""
    prob, plan, sv, vor, rng, host, dev = setup()
    V, n = plan.n_views, plan.n_records
    say(f"joint step: {V} views, {n} records, {plan.n_scenes} scenes")
    lr = np.array([3e-3, 1e-3])
    lr_t = torch.from_numpy(lr).cuda()
    phases = [None, None, [0, 1], [1, 2]]
    want = host
    for s, ph in enumerate(phases):
        g = grads_of(rng, V, n)
        gt = {k: torch.from_numpy(v).cuda() for k, v in g.items()}
        ph_t = None if ph is None else torch.tensor(ph, dtype=torch.int32, device="cuda")
        plan.joint_step(dev, gt, lr_t, phase=ph_t)
        torch.cuda.synchronize()
        prev, want = want, oj.joint_step(want, g, lr, sv, vor, phase=ph)
        compare(dev, want, prev, g, n, f"step {s}")


def test_depth_steps_count_from_the_switch(gpu):
    """Six gated steps after 40 steps of the pose phase (the focal counts
    start at 40): scene 0 switches to the joint phase at step 2, scene 1 at
    step 0 and stops at step 4.  The depth parameters' bias correction counts
    the depth optimizer's own steps, so a scene's first depth step is the
    closed form -lr g / (|g| + eps) after the decay; every step against the
    oracle."""
    prob, plan, sv, vor, rng, host, dev = setup(seed=2)
    V, n, S = plan.n_views, plan.n_records, plan.n_scenes
    host["steps"][0] = 40
    dev["steps"].copy_(torch.from_numpy(host["steps"].reshape(-1).astype(np.int32)))
    lr = np.array([3e-3, 1e-3])
    lr_t = torch.from_numpy(lr).cuda()
    phases = [[0, 1], [0, 1], [1, 1], [1, 1], [1, 2], [1, 2]]
    want = host
    sr = sv[vor]
    for s, ph in enumerate(phases):
        g = grads_of(rng, V, n)
        gt = {k: torch.from_numpy(v).cuda() for k, v in g.items()}
        before = dev["beta"].cpu().numpy().astype(np.float64)
        plan.joint_step(dev, gt, lr_t, phase=torch.tensor(ph, dtype=torch.int32, device="cuda"))
        torch.cuda.synchronize()
        prev, want = want, oj.joint_step(want, g, lr, sv, vor, phase=ph)
        compare(dev, want, prev, g, n, f"gated step {s}")
        first = [sc for sc in range(S) if ph[sc] == 1 and prev["steps"][1][sc] == 0]
        for sc in first:
            idx = sr == sc
            gb = g["grad_beta"][idx]
            closed = before[idx] * (1 - lr[sc] * 0.01) - lr[sc] * gb / (np.abs(gb) + 1e-8)
            got = dev["beta"].cpu().numpy()[idx].astype(np.float64)
            assert np.all(np.abs(got - closed) <= np.spacing(np.abs(closed).astype(np.float32))), \
                f"first depth step of scene {sc} at iteration {s}"
    assert dev["steps"].cpu().tolist() == [46, 44, 4, 4]


def test_joint_step_sets_refinement(gpu):
    """After each step the plan's refinement is that of the new parameters:
    the loss and gradients equal those after an explicit set_refinement of
    the same arrays (bitwise), and differ from the unrefined ones.  The first
    step of a plan installs the depths through the refinement update, later
    ones rewrite them in the step kernel (phases (1, 0) on the third step:
    one scene's depths stay, the other's move)."""
    prob, plan, sv, vor, rng, host, dev = setup(seed=1)
    V, n = plan.n_views, plan.n_records
    P = torch.from_numpy(prob.poses_init.copy()).cuda()
    for s, ph in enumerate((None, None, [1, 0])):
        g = {k: torch.from_numpy(v).cuda() for k, v in grads_of(rng, V, n).items()}
        ph_t = None if ph is None else torch.tensor(ph, dtype=torch.int32, device="cuda")
        plan.joint_step(dev, g, 1e-2, phase=ph_t)
        after = {k: t.cpu().numpy() for k, t in plan.refine(P, 10.0).items()}
        plan.set_refinement(dev["gamma"], dev["alpha"], dev["beta"])
        explicit = {k: t.cpu().numpy() for k, t in plan.refine(P, 10.0).items()}
        for k in after:
            assert np.array_equal(after[k], explicit[k]), (s, k)
        assert plan.device_status() == 0
    plan.set_refinement()
    base = plan.refine(P, 10.0)["loss"].cpu().numpy()
    assert not np.array_equal(base, after["loss"])


def test_joint_step_rejects_bad_arguments(gpu):
    from paper_2607_00579_amd import _lib
    prob, plan, sv, vor, rng, host, dev = setup()
    g = {k: torch.from_numpy(v).cuda() for k, v in grads_of(rng, plan.n_views, plan.n_records).items()}
    with pytest.raises(RuntimeError):
        plan.joint_step(dev, g, 1e-3, beta1=1.0)
    with pytest.raises(ValueError):
        plan.joint_step(dev, {"grad_gamma": g["grad_gamma"]}, 1e-3)
    with pytest.raises(ValueError):             # fewer phases than scenes
        plan.joint_step(dev, g, 1e-3, phase=torch.zeros(1, dtype=torch.int32, device="cuda"))
    with pytest.raises(ValueError):             # host memory
        plan.joint_step(dev, dict(g, grad_beta=g["grad_beta"].cpu()), 1e-3)
    with pytest.raises(ValueError):             # wrong dtype
        plan.joint_step(dev, dict(g, grad_alpha=g["grad_alpha"].float()), 1e-3)
    with pytest.raises(ValueError):             # step counts for fewer scenes
        plan.joint_step(dict(dev, steps=dev["steps"][:1]), g, 1e-3)
    with pytest.raises(_lib.EpoError):          # null step counts, seen by the C side
        _lib.joint_step(plan.handle, dev["gamma"], dev["alpha"], dev["beta"], dev["m_gamma"],
                        dev["v_gamma"], dev["m_depth"], dev["v_depth"], g["grad_gamma"],
                        g["grad_alpha"], g["grad_beta"],
                        torch.ones(plan.n_scenes, dtype=torch.float64, device="cuda"), None,
                        0.9, 0.999, 1e-8, 0.01, 0.01, None, None)


def test_joint_step_views_without_edges(gpu):
    """Six views of 40x30 with 300, 0, 7, 0, 500, 0 edge pixels (813
    parameters over four workgroups whose boundaries fall inside views, empty
    views in the middle and at the end): two steps (the first installs the
    depths through the refinement update, the second rewrites them itself)
    against the oracle, and the installed refinement against an explicit
    set_refinement."""
    from paper_2607_00579_amd.api import EdgePlan
    from synth import fixtures
    W, H = 40, 30
    K = [32.0, 32.0, 19.5, 14.5]
    rng = np.random.default_rng(11)
    edges, depths = [], []
    for cnt in (300, 0, 7, 0, 500, 0):
        e = np.zeros(W * H, np.uint8)
        e[rng.choice(W * H, cnt, replace=False)] = 255
        edges.append(e.reshape(H, W))
        depths.append(rng.uniform(2.0, 6.0, (H, W)).astype(np.float32))
    P = [np.concatenate([np.eye(3), np.array([[0.05 * v], [0.0], [0.0]])], axis=1)
         for v in range(6)]
    pairs = [[i, j] for i in range(6) for j in range(6) if i != j]
    q = fixtures.problem_from_maps([W] * 6, [H] * 6, [K] * 6, edges, depths, P, pairs)
    plan = EdgePlan.from_problem(q, device="cuda:0")
    V, n = plan.n_views, plan.n_records
    assert (V, n) == (6, 807)
    vor = plan.record_pixels()[:, 0]
    sv = np.asarray(plan.scene_of_view, np.int64)
    host = oj.initial_state(V, n, plan.n_scenes)
    host["gamma"] = rng.normal(0, 0.02, V)
    host["alpha"] = (1 + rng.normal(0, 0.05, n)).astype(np.float32)
    host["beta"] = rng.normal(0, 0.05, n).astype(np.float32)
    dev = plan.joint_state()
    for k in ("gamma", "alpha", "beta"):
        dev[k].copy_(torch.from_numpy(host[k]))
    poses = torch.from_numpy(q.poses_init.copy()).cuda()
    lr = np.array([2e-3])
    want = host
    for s in range(2):
        g = grads_of(rng, V, n)
        plan.joint_step(dev, {k: torch.from_numpy(v).cuda() for k, v in g.items()},
                        torch.from_numpy(lr).cuda())
        after = {k: t.cpu().numpy() for k, t in plan.refine(poses, 10.0).items()}
        prev, want = want, oj.joint_step(want, g, lr, sv, vor)
        compare(dev, want, prev, g, n, f"empty views, step {s}")
        plan.set_refinement(dev["gamma"], dev["alpha"], dev["beta"])
        explicit = {k: t.cpu().numpy() for k, t in plan.refine(poses, 10.0).items()}
        for k in after:
            assert np.array_equal(after[k], explicit[k]), (s, k)
