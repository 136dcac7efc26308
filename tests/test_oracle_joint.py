"""Oracle pins of the joint-phase optimizer step (focal scales gamma, depth
scale alpha and shift beta; AdamW, paper Sec. 4 "Implementation Details"):
against torch.optim.AdamW in float64 over several steps with one learning
rate per scene, with the depth optimizer created at each scene's phase
switch (Alg. EPO.Forward builds one optimizer per module and steps the depth
one only in the joint phase), the first-step closed forms, and the phase
gate (depth steps only in the joint phase, nothing after the stop)."""
import numpy as np
import torch

from oracle import joint as oj


def make_case(seed=0, V=5, per_view=(3, 0, 4, 2, 5), n_scenes=2):
    rng = np.random.default_rng(seed)
    sv = np.array([0, 0, 1, 1, 0][:V], np.int64) % n_scenes
    vor = np.repeat(np.arange(V), per_view)
    n = vor.size
    state = oj.initial_state(V, n, n_scenes)
    state["gamma"] = rng.normal(0, 0.05, V)
    state["alpha"] = (1 + rng.normal(0, 0.1, n)).astype(np.float32)
    state["beta"] = rng.normal(0, 0.1, n).astype(np.float32)
    return rng, sv, vor, state


def grads_of(rng, V, n):
    return {"grad_gamma": rng.normal(0, 1e-2, V), "grad_alpha": rng.normal(0, 1e-3, n),
            "grad_beta": rng.normal(0, 1e-3, n)}


def test_matches_torch_adamw_per_scene_lr():
    """Five ungated steps, wd 0.01, learning rates 3e-3 and 1e-3 by scene:
    the oracle (depth rounding off) against torch.optim.AdamW, one parameter
    group per scene and parameter kind."""
    rng, sv, vor, state = make_case(seed=3)
    V, n = sv.size, vor.size
    lr = np.array([3e-3, 1e-3])
    sr = sv[vor]
    params = {}
    groups = []
    for name, scene_of in (("gamma", sv), ("alpha", sr), ("beta", sr)):
        for s in range(2):
            idx = np.nonzero(scene_of == s)[0]
            p = torch.tensor(np.asarray(state[name], np.float64)[idx], dtype=torch.float64,
                             requires_grad=True)
            params[(name, s)] = (p, idx)
            groups.append({"params": [p], "lr": float(lr[s])})
    opt = torch.optim.AdamW(groups, betas=(0.9, 0.999), eps=1e-8, weight_decay=0.01)
    st = {k: (np.asarray(v, np.float64) if k in ("alpha", "beta") else v) for k, v in state.items()}
    for step in range(5):
        g = grads_of(rng, V, n)
        st = oj.joint_step(st, g, lr, sv, vor, round_depth=False)
        for (name, s), (p, idx) in params.items():
            p.grad = torch.tensor(g["grad_" + name][idx], dtype=torch.float64)
        opt.step()
        for (name, s), (p, idx) in params.items():
            want = p.detach().numpy()
            np.testing.assert_allclose(st[name][idx], want, rtol=1e-13, atol=1e-16)
            ts = opt.state[p]
            np.testing.assert_allclose(st["m_" + name][idx], ts["exp_avg"].numpy(), rtol=1e-13,
                                       atol=1e-20)
            np.testing.assert_allclose(st["v_" + name][idx], ts["exp_avg_sq"].numpy(),
                                       rtol=1e-13, atol=1e-24)
    assert np.array_equal(st["steps"], np.full((2, 2), 5))


def test_focal_optimizer_steps_until_the_stop():
    """Three scenes over eight steps with per-step phases (scene 1 stops at
    step 5) and learning rates changing every step: the focal scales against
    one torch.optim.AdamW per scene, created at step 0 and stepped while the
    scene has not stopped."""
    rng = np.random.default_rng(21)
    V, per_view = 6, (3, 2, 4, 1, 3, 2)
    sv = np.array([0, 1, 2, 0, 1, 2])
    vor = np.repeat(np.arange(V), per_view)
    n = vor.size
    st = oj.initial_state(V, n, 3)
    st["gamma"] = rng.normal(0, 0.05, V)
    phases = [[0, 0, 0], [0, 1, 0], [0, 1, 0], [1, 1, 0], [1, 1, 0], [1, 2, 0], [1, 2, 0],
              [1, 2, 0]]
    focal = {}
    for s in range(3):
        p = torch.tensor(st["gamma"][sv == s], dtype=torch.float64, requires_grad=True)
        focal[s] = (p, torch.optim.AdamW([p], lr=1.0, betas=(0.9, 0.999), eps=1e-8,
                                         weight_decay=0.01))
    for k, ph in enumerate(phases):
        lr = np.array([1e-3, 2e-3, 3e-3]) * (1.0 + 0.1 * k)
        g = grads_of(rng, V, n)
        st = oj.joint_step(st, g, lr, sv, vor, phase=ph, round_depth=False)
        for s in range(3):
            p, opt = focal[s]
            if ph[s] != 2:
                for grp in opt.param_groups:
                    grp["lr"] = float(lr[s])
                p.grad = torch.tensor(g["grad_gamma"][sv == s], dtype=torch.float64)
                opt.step()
            np.testing.assert_allclose(st["gamma"][sv == s], p.detach().numpy(), rtol=1e-13,
                                       atol=1e-18, err_msg=f"step {k} scene {s} gamma")
            np.testing.assert_allclose(st["m_gamma"][sv == s], opt.state[p]["exp_avg"].numpy(),
                                       rtol=1e-13, atol=1e-20)
            assert int(opt.state[p]["step"]) == st["steps"][0][s]


def _depth_reference(phases, lr_of, grads, alpha0, beta0, sr):
    """Per scene a torch AdamW over (alpha, beta) created at the first step
    in phase 1 and stepped only in phase 1."""
    out_a = np.asarray(alpha0, np.float64).copy()
    out_b = np.asarray(beta0, np.float64).copy()
    opts = {}
    for k, ph in enumerate(phases):
        for s, p in enumerate(ph):
            if p != 1:
                continue
            idx = sr == s
            if s not in opts:
                pa = torch.tensor(out_a[idx], dtype=torch.float64, requires_grad=True)
                pb = torch.tensor(out_b[idx], dtype=torch.float64, requires_grad=True)
                opts[s] = (pa, pb, torch.optim.AdamW([pa, pb], lr=1.0, betas=(0.9, 0.999),
                                                     eps=1e-8, weight_decay=0.01))
            pa, pb, opt = opts[s]
            for grp in opt.param_groups:
                grp["lr"] = float(lr_of(k)[s])
            pa.grad = torch.tensor(grads[k]["grad_alpha"][idx], dtype=torch.float64)
            pb.grad = torch.tensor(grads[k]["grad_beta"][idx], dtype=torch.float64)
            opt.step()
            out_a[idx] = pa.detach().numpy()
            out_b[idx] = pb.detach().numpy()
    return out_a, out_b, {s: (o[2].state[o[0]], o[2].state[o[1]]) for s, o in opts.items()}


def test_depth_optimizer_counts_from_the_switch():
    """alpha and beta after eight steps with scenes switching to the joint
    phase at steps 3 and 1 (and the second stopping at step 5) equal a
    torch.optim.AdamW per scene created at the switch; their moments and the
    oracle's depth step counts (5 and 4 steps) match the reference."""
    rng = np.random.default_rng(22)
    V, per_view = 6, (3, 2, 4, 1, 3, 2)
    sv = np.array([0, 1, 2, 0, 1, 2])
    vor = np.repeat(np.arange(V), per_view)
    n = vor.size
    sr = sv[vor]
    st = oj.initial_state(V, n, 3)
    st["alpha"] = (1 + rng.normal(0, 0.1, n))
    st["beta"] = rng.normal(0, 0.1, n)
    a0, b0 = st["alpha"].copy(), st["beta"].copy()
    phases = [[0, 0, 0], [0, 1, 0], [0, 1, 0], [1, 1, 0], [1, 1, 0], [1, 2, 0], [1, 2, 0],
              [1, 2, 0]]

    def lr_of(k):
        return np.array([1e-3, 2e-3, 3e-3]) * (1.0 + 0.1 * k)

    grads = [grads_of(rng, V, n) for _ in phases]
    for k, ph in enumerate(phases):
        st = oj.joint_step(st, grads[k], lr_of(k), sv, vor, phase=ph, round_depth=False)
    ra, rb, states = _depth_reference(phases, lr_of, grads, a0, b0, sr)
    np.testing.assert_allclose(st["alpha"], ra, rtol=1e-13, atol=1e-16)
    np.testing.assert_allclose(st["beta"], rb, rtol=1e-13, atol=1e-16)
    for s, (sa, sb) in states.items():
        idx = sr == s
        np.testing.assert_allclose(st["m_alpha"][idx], sa["exp_avg"].numpy(), rtol=1e-13,
                                   atol=1e-20)
        np.testing.assert_allclose(st["v_beta"][idx], sb["exp_avg_sq"].numpy(), rtol=1e-13,
                                   atol=1e-24)
        assert int(sa["step"]) == st["steps"][1][s]
    assert list(st["steps"][1]) == [5, 4, 0]
    assert list(st["steps"][0]) == [8, 5, 8]
    # scene 2 never switched: its depth parameters are untouched
    assert np.array_equal(st["alpha"][sr == 2], a0[sr == 2])
    # the reading matters: bias correction at the iteration count instead
    # moves the first depth step of a late switch by more than 2x
    late = oj.initial_state(V, n, 3)
    late["steps"][:] = [[900, 900, 900], [0, 0, 0]]
    early = oj.initial_state(V, n, 3)
    early["steps"][:] = [[900, 900, 900], [900, 900, 900]]
    g = grads_of(rng, V, n)
    lr = np.full(3, 1e-3)
    d_late = oj.joint_step(late, g, lr, sv, vor, phase=[1, 1, 1], round_depth=False,
                           wd_depth=0.0)["beta"] - late["beta"]
    d_early = oj.joint_step(early, g, lr, sv, vor, phase=[1, 1, 1], round_depth=False,
                            wd_depth=0.0)["beta"] - early["beta"]
    np.testing.assert_allclose(d_late, -lr[sr] * g["grad_beta"] / (np.abs(g["grad_beta"]) + 1e-8),
                               rtol=1e-12)
    assert np.all(np.abs(d_early) > 2.0 * np.abs(d_late))


def test_first_step_closed_forms():
    """Step 1 from zero moments: m_hat = g, v_hat = g^2, so with wd = 0 the
    update is -lr g / (|g| + eps); with g = 0 only the decay acts."""
    rng, sv, vor, state = make_case(seed=5)
    V, n = sv.size, vor.size
    lr = np.array([2e-3, 5e-4])
    g = grads_of(rng, V, n)
    out = oj.joint_step(state, g, lr, sv, vor, wd_focal=0.0, wd_depth=0.0, round_depth=False)
    gg = g["grad_gamma"]
    np.testing.assert_allclose(out["gamma"], state["gamma"] - lr[sv] * gg / (np.abs(gg) + 1e-8),
                               rtol=1e-15, atol=1e-18)
    ga = g["grad_alpha"]
    want = state["alpha"].astype(np.float64) - lr[sv[vor]] * ga / (np.abs(ga) + 1e-8)
    np.testing.assert_allclose(out["alpha"], want, rtol=1e-15, atol=1e-18)
    zero = {k: np.zeros_like(v) for k, v in g.items()}
    out = oj.joint_step(state, zero, lr, sv, vor, wd_focal=0.01, wd_depth=0.1)
    assert np.array_equal(out["gamma"], state["gamma"] * (1 - lr[sv] * 0.01))
    want = (state["beta"].astype(np.float64) * (1 - lr[sv[vor]] * 0.1)).astype(np.float32)
    assert np.array_equal(out["beta"], want)
    assert out["beta"].dtype == np.float32
    assert not np.any(out["m_gamma"]) and not np.any(out["v_alpha"])


def test_phase_gate():
    """Scene phases (0, 1, 2): phase 0 moves gamma only, phase 1 moves
    everything, phase 2 nothing; gated values, moments and step counts stay
    bitwise."""
    rng, sv, vor, state = make_case(seed=7, V=6, per_view=(2, 3, 1, 4, 2, 3), n_scenes=3)
    sv = np.array([0, 1, 2, 0, 1, 2])
    V, n = sv.size, vor.size
    lr = np.array([1e-3, 2e-3, 3e-3])
    g = grads_of(rng, V, n)
    s1 = oj.joint_step(state, g, lr, sv, vor)
    s1 = oj.joint_step(s1, grads_of(rng, V, n), lr, sv, vor)
    out = oj.joint_step(s1, grads_of(rng, V, n), lr, sv, vor, phase=[0, 1, 2])
    sr = sv[vor]
    for k in ("gamma", "m_gamma", "v_gamma"):
        assert np.array_equal(out[k][sv == 2], s1[k][sv == 2]), k
        assert not np.any(out[k][sv != 2] == s1[k][sv != 2]), k
    for k in ("alpha", "beta", "m_alpha", "v_alpha", "m_beta", "v_beta"):
        assert np.array_equal(out[k][sr != 1], s1[k][sr != 1]), k
        assert not np.any(out[k][sr == 1] == s1[k][sr == 1]), k
    assert list(out["steps"][0]) == [3, 3, 2]
    assert list(out["steps"][1]) == [2, 3, 2]


def test_joint_loop_first_step_on_the_zero_fixture():
    """Exact-zero fixture (shifted edges, loss and every gradient exactly 0):
    the joint loop's first step, everything ungated, is pure weight decay:
    the poses and gamma stay (0 decays to 0), alpha becomes float32(1 - lr(0)
    wd), beta stays 0, the moments stay 0 and both step counts advance."""
    from oracle import cost, loop
    from synth import fixtures
    p = fixtures.shifted_pair()
    op = cost.OracleProblem(p)
    n = sum(op.pts[v][0].size for v in range(op.V))
    st = oj.initial_state(op.V, n, 1)
    m, v = np.zeros((op.V, 6)), np.zeros((op.V, 6))
    new, m1, v1, st1, r = loop.joint_loop_step(op, 0, p.poses_init, m, v, st, phase=None)
    assert r["loss"][0] == 0.0 and not np.any(r["grad"]) and not np.any(r["grad_focal"])
    assert np.array_equal(new, p.poses_init)
    assert not np.any(st1["gamma"]) and not np.any(st1["beta"])
    lr0 = loop.learning_rate(0)
    assert np.all(st1["alpha"] == np.float32(1.0 * (1.0 - lr0 * 0.01)))
    for k in ("m_gamma", "v_gamma", "m_alpha", "v_alpha", "m_beta", "v_beta"):
        assert not np.any(st1[k]), k
    assert st1["steps"].tolist() == [[1], [1]]


def test_joint_loop_gradients_against_central_differences():
    """At a seeded refined state (|gamma|, |alpha - 1|, |beta| <= 0.02, poses
    of the small workload) the loop's dL/dgamma, dL/dalpha, dL/dbeta against
    frozen-branch central differences of the scene loss in gamma and in
    single pixels' alpha and beta (h = 1e-6, unrounded refinement)."""
    from oracle import cost, loop
    from synth import make
    p = make("c1")
    op = cost.OracleProblem(p)
    rng = np.random.default_rng(3)
    n = sum(op.pts[v][0].size for v in range(op.V))
    gam = rng.uniform(-0.02, 0.02, op.V)
    al = 1.0 + rng.uniform(-0.02, 0.02, n)
    be = rng.uniform(-0.02, 0.02, n)
    params = cost.CostParams()
    K, depth = loop.joint_refinement(op, gam, al, be, rounded=False)
    base = op.evaluate(p.poses_init, 10.0, params, K=K, depth=depth)
    g = loop.joint_gradients(op, base, gam)
    frozen = base["decisions"]
    h = 1e-6

    def loss_at(gm, a, b):
        Kx, dx = loop.joint_refinement(op, gm, a, b, rounded=False)
        return cost._frozen_loss(op, p.poses_init, 10.0, params, frozen, base, K=Kx,
                                 depth=dx)[0]

    for vv in range(op.V):
        gp, gm_ = gam.copy(), gam.copy()
        gp[vv] += h
        gm_[vv] -= h
        fd = (loss_at(gp, al, be) - loss_at(gm_, al, be)) / (2 * h)
        assert abs(fd - g["grad_gamma"][vv]) <= 1e-6 * abs(fd), (vv, fd, g["grad_gamma"][vv])
    views = loop.record_views(op)
    for k in rng.choice(np.flatnonzero(views == 0), 6, replace=False):
        for name, arr in (("grad_alpha", al), ("grad_beta", be)):
            ap, am = arr.copy(), arr.copy()
            ap[k] += h
            am[k] -= h
            if name == "grad_alpha":
                fd = (loss_at(gam, ap, be) - loss_at(gam, am, be)) / (2 * h)
            else:
                fd = (loss_at(gam, al, ap) - loss_at(gam, al, am)) / (2 * h)
            want = g[name][k]
            assert abs(fd - want) <= 1e-6 * max(abs(want), 1e-3 * np.abs(g[name]).max()), \
                (name, k, fd, want)


def test_joint_loop_depth_waits_for_the_switch():
    """Phases (0, 0, 0, 1, 1) over five steps of the small workload: the
    depth parameters keep their identity values through the pose phase; the
    first step of the joint phase, at iteration 3, is the depth optimizer's
    step 1 (closed form after the decay), while gamma has stepped at every
    iteration (its count 5)."""
    from oracle import cost, loop
    from synth import make
    p = make("c1")
    op = cost.OracleProblem(p)
    n = sum(op.pts[v][0].size for v in range(op.V))
    st = oj.initial_state(op.V, n, 1)
    poses, m, v = p.poses_init.copy(), np.zeros((op.V, 6)), np.zeros((op.V, 6))
    for s, ph in enumerate((0, 0, 0, 1, 1)):
        before = st
        poses, m, v, st, r = loop.joint_loop_step(op, s, poses, m, v, st, phase=[ph])
        if s < 3:
            assert np.all(st["alpha"] == 1.0) and np.all(st["beta"] == 0.0)
            assert not np.any(st["m_alpha"])
        if s == 3:
            gb = loop.joint_gradients(op, r, before["gamma"])["grad_beta"]
            lr = loop.learning_rate(3)
            want = (-lr * gb / (np.abs(gb) + 1e-8)).astype(np.float32)
            assert np.all(np.abs(st["beta"] - want) <= np.spacing(np.abs(want)))
            assert not np.array_equal(st["gamma"], before["gamma"])
    assert st["steps"].tolist() == [[5], [2]]
