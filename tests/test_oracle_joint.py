"""Oracle pins of the joint-phase optimizer step (focal scales gamma, depth
scale alpha and shift beta; AdamW, paper Sec. 4 "Implementation Details"):
against torch.optim.AdamW in float64 over several steps with one learning
rate per scene, the first-step closed forms, and the phase gate of Alg.
EPO.Forward (depth steps only in the joint phase, nothing after the stop)."""
import numpy as np
import torch

from oracle import joint as oj


def make_case(seed=0, V=5, per_view=(3, 0, 4, 2, 5), n_scenes=2):
    rng = np.random.default_rng(seed)
    sv = np.array([0, 0, 1, 1, 0][:V], np.int64) % n_scenes
    vor = np.repeat(np.arange(V), per_view)
    n = vor.size
    state = {"gamma": rng.normal(0, 0.05, V), "alpha": (1 + rng.normal(0, 0.1, n)).astype(np.float32),
             "beta": rng.normal(0, 0.1, n).astype(np.float32),
             "m_gamma": np.zeros(V), "v_gamma": np.zeros(V)}
    for k in ("alpha", "beta"):
        state["m_" + k] = np.zeros(n)
        state["v_" + k] = np.zeros(n)
    return rng, sv, vor, state


def grads_of(rng, V, n):
    return {"grad_gamma": rng.normal(0, 1e-2, V), "grad_alpha": rng.normal(0, 1e-3, n),
            "grad_beta": rng.normal(0, 1e-3, n)}


def test_matches_torch_adamw_per_scene_lr():
    """Five steps, wd 0.01, learning rates 3e-3 and 1e-3 by scene: the
    oracle (depth rounding off) against torch.optim.AdamW, one parameter group
    per scene and parameter kind."""
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
        st = oj.joint_step(st, g, lr, sv, vor, step, round_depth=False)
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


def test_first_step_closed_forms():
    """Step 1 from zero moments: m_hat = g, v_hat = g^2, so with wd = 0 the
    update is -lr g / (|g| + eps); with g = 0 only the decay acts."""
    rng, sv, vor, state = make_case(seed=5)
    V, n = sv.size, vor.size
    lr = np.array([2e-3, 5e-4])
    g = grads_of(rng, V, n)
    out = oj.joint_step(state, g, lr, sv, vor, 0, wd_focal=0.0, wd_depth=0.0, round_depth=False)
    gg = g["grad_gamma"]
    np.testing.assert_allclose(out["gamma"], state["gamma"] - lr[sv] * gg / (np.abs(gg) + 1e-8),
                               rtol=1e-15, atol=1e-18)
    ga = g["grad_alpha"]
    want = state["alpha"].astype(np.float64) - lr[sv[vor]] * ga / (np.abs(ga) + 1e-8)
    np.testing.assert_allclose(out["alpha"], want, rtol=1e-15, atol=1e-18)
    zero = {k: np.zeros_like(v) for k, v in g.items()}
    out = oj.joint_step(state, zero, lr, sv, vor, 0, wd_focal=0.01, wd_depth=0.1)
    assert np.array_equal(out["gamma"], state["gamma"] * (1 - lr[sv] * 0.01))
    want = (state["beta"].astype(np.float64) * (1 - lr[sv[vor]] * 0.1)).astype(np.float32)
    assert np.array_equal(out["beta"], want)
    assert out["beta"].dtype == np.float32
    assert not np.any(out["m_gamma"]) and not np.any(out["v_alpha"])


def test_phase_gate():
    """Scene phases (0, 1, 2): phase 0 moves gamma only, phase 1 moves
    everything, phase 2 nothing; gated values and moments stay bitwise."""
    rng, sv, vor, state = make_case(seed=7, V=6, per_view=(2, 3, 1, 4, 2, 3), n_scenes=3)
    sv = np.array([0, 1, 2, 0, 1, 2])
    V, n = sv.size, vor.size
    lr = np.array([1e-3, 2e-3, 3e-3])
    g = grads_of(rng, V, n)
    s1 = oj.joint_step(state, g, lr, sv, vor, 0)
    s1 = oj.joint_step(s1, grads_of(rng, V, n), lr, sv, vor, 1)
    out = oj.joint_step(s1, grads_of(rng, V, n), lr, sv, vor, 2, phase=[0, 1, 2])
    ref = oj.joint_step(s1, grads_of(np.random.default_rng(99), V, n), lr, sv, vor, 2)
    sr = sv[vor]
    for k in ("gamma", "m_gamma", "v_gamma"):
        assert np.array_equal(out[k][sv == 2], s1[k][sv == 2]), k
        assert not np.any(out[k][sv != 2] == s1[k][sv != 2]), k
    for k in ("alpha", "beta", "m_alpha", "v_alpha", "m_beta", "v_beta"):
        assert np.array_equal(out[k][sr != 1], s1[k][sr != 1]), k
        assert not np.any(out[k][sr == 1] == s1[k][sr == 1]), k
    assert ref["gamma"].shape == out["gamma"].shape
