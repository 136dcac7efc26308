"""Pins of the oracle's SE(3) exponential, schedules and Adam step (CPU)."""
import math

import numpy as np
import torch
from scipy.linalg import expm

from oracle import geometry, loop, mlp


def twist_matrix(xi):
    T = np.zeros((4, 4))
    T[:3, :3] = geometry.hat(xi[3:])
    T[:3, 3] = xi[:3]
    return T


def test_exp_matches_matrix_exponential():
    rng = np.random.default_rng(0)
    for scale in (1e-7, 1e-5, 1e-3, 0.3, 2.0, 3.0):
        for _ in range(10):
            xi = rng.normal(size=6) * scale
            assert np.allclose(geometry.se3_exp(xi), expm(twist_matrix(xi)), atol=1e-13, rtol=1e-12)


def test_exp_log_roundtrip():
    rng = np.random.default_rng(1)
    for _ in range(50):
        xi = rng.normal(size=6)
        xi[3:] *= rng.uniform(1e-6, 3.0) / np.linalg.norm(xi[3:])   # angle below pi: Log is unique
        assert np.allclose(geometry.se3_log(geometry.se3_exp(xi)), xi, atol=1e-10)


def test_pure_translation_and_rotation():
    T = geometry.se3_exp(np.array([1.0, -2.0, 3.0, 0, 0, 0]))
    assert np.allclose(T[:3, :3], np.eye(3)) and np.allclose(T[:3, 3], [1, -2, 3])
    th = 0.7
    R = geometry.se3_exp(np.array([0, 0, 0, 0, 0, th]))[:3, :3]
    assert np.allclose(R, [[math.cos(th), -math.sin(th), 0], [math.sin(th), math.cos(th), 0],
                           [0, 0, 1]])


def test_small_angle_branch_continuous():
    a = geometry.se3_exp(np.array([0.3, 0.1, -0.2, 0.99999e-4, 0, 0]))
    b = geometry.se3_exp(np.array([0.3, 0.1, -0.2, 1.00001e-4, 0, 0]))
    assert np.abs(a - b).max() < 1e-8


def test_schedules():
    assert loop.clamp_lambda(0) == 10.0 and loop.clamp_lambda(1000) == 6.0
    assert loop.clamp_lambda(5000) == 6.0 and loop.clamp_lambda(500) == 8.0
    assert math.isclose(loop.learning_rate(24), 3e-3)
    assert math.isclose(loop.learning_rate(0), 3e-3 / 25)
    assert math.isclose(loop.learning_rate(25), 3e-3)
    assert loop.learning_rate(1999) < 1e-8 + 3e-3 * 0.5 * (1 + math.cos(math.pi * 1974 / 1975))


def test_first_adam_step_closed_form():
    """After one step m^ = g and v^ = g^2, so the twist is -lr g / (|g| + eps)."""
    rng = np.random.default_rng(2)
    poses = np.stack([np.concatenate([np.eye(3), rng.normal(size=(3, 1))], 1) for _ in range(3)])
    g = rng.normal(size=(3, 6))
    lr = 1e-2
    new, m, v = loop.adam_se3_step(poses, np.zeros((3, 6)), np.zeros((3, 6)), g, 1, lr)
    for k in range(3):
        xi = -lr * g[k] / (np.abs(g[k]) + 1e-8)
        assert np.allclose(new[k], geometry.left_update(poses[k], xi), atol=1e-15)
    assert np.allclose(m, 0.1 * g) and np.allclose(v, 0.001 * g * g)


def test_fixed_mask_and_zero_gradient():
    poses = np.stack([np.concatenate([np.eye(3), np.ones((3, 1))], 1)] * 2)
    g = np.ones((2, 6))
    new, m, v = loop.adam_se3_step(poses, np.zeros((2, 6)), np.zeros((2, 6)), g, 1, 1e-2,
                                   fixed=np.array([True, False]))
    assert np.array_equal(new[0], poses[0]) and np.all(m[0] == 0)
    assert not np.array_equal(new[1], poses[1])
    new, _, _ = loop.adam_se3_step(poses, np.zeros((2, 6)), np.zeros((2, 6)), np.zeros((2, 6)),
                                   1, 1e-2)
    assert np.array_equal(new, poses)


def test_log_near_pi():
    """Angles within 1e-6 of pi take the symmetric-part branch of Log: the
    axis and its sign come back (against expm of the twist), and at exactly
    pi either sign is a valid logarithm."""
    rng = np.random.default_rng(3)
    for gap in (5e-7, 1e-8, 1e-11, 0.0):
        for _ in range(20):
            n = rng.normal(size=3)
            n /= np.linalg.norm(n)
            th = np.pi - gap
            R = expm(geometry.hat(th * n))
            w = geometry.so3_log(R)
            assert abs(np.linalg.norm(w) - th) < 1e-9
            assert np.allclose(expm(geometry.hat(w)), R, atol=1e-9)
            if gap >= 1e-8:
                # the sign is recoverable while sin(th) dominates the rounding
                assert np.allclose(w, th * n, atol=1e-7), (gap, w, th * n)
    xi = np.concatenate([rng.normal(size=3), (np.pi - 1e-7) * np.array([0.0, 0.6, -0.8])])
    assert np.allclose(geometry.se3_log(geometry.se3_exp(xi)), xi, atol=1e-7)


def test_adam_twists_match_torch_adam_over_many_steps():
    """Seven steps of the twist optimizer from a resumed state (start step 5,
    nonzero moments) with one learning rate per scene changing every step and
    one fixed pose, against torch.optim.Adam (float64) stepping the twist of
    every free pose: after every step the moments equal torch's exp_avg and
    exp_avg_sq, and the applied twist, read back as Log(P_new P_old^-1),
    equals torch's parameter change.  A fixed pose neither moves nor updates
    its moments."""
    rng = np.random.default_rng(4)
    V, sov = 5, np.array([0, 1, 0, 1, 1])
    fixed = np.array([False, False, True, False, False])
    poses = np.stack([geometry.left_update(np.concatenate([np.eye(3), np.zeros((3, 1))], 1),
                                           rng.normal(size=6) * 0.3) for _ in range(V)])
    m = rng.normal(size=(V, 6)) * 1e-3
    v = np.abs(rng.normal(size=(V, 6))) * 1e-6
    m[fixed] = 0.0
    v[fixed] = 0.0
    s0 = 5
    params, opts = {}, {}
    for k in np.flatnonzero(~fixed):
        p = torch.zeros(6, dtype=torch.float64, requires_grad=True)
        opt = torch.optim.Adam([p], lr=1.0, betas=(0.9, 0.999), eps=1e-8)
        opt.state[p] = {"step": torch.tensor(float(s0 - 1), dtype=torch.float64),
                        "exp_avg": torch.tensor(m[k]), "exp_avg_sq": torch.tensor(v[k])}
        params[k], opts[k] = p, opt
    for s in range(s0, s0 + 7):
        g = rng.normal(size=(V, 6)) * 10.0 ** rng.uniform(-4, 0, size=(V, 1))
        g[1, 2] = 0.0                                   # a zero component
        lr = np.array([3e-3, 1e-3]) * (1.0 + 0.05 * s)
        new, m_new, v_new = loop.adam_se3_step(poses, m, v, g, s, lr, fixed=fixed,
                                               scene_of_view=sov)
        for k in range(V):
            if fixed[k]:
                assert np.array_equal(new[k], poses[k])
                assert not np.any(m_new[k]) and not np.any(v_new[k])
                continue
            p, opt = params[k], opts[k]
            before = p.detach().clone()
            opt.param_groups[0]["lr"] = float(lr[sov[k]])
            p.grad = torch.tensor(g[k])
            opt.step()
            st = opt.state[p]
            scale = 0.9 * np.abs(m[k]) + 0.1 * np.abs(g[k])
            assert np.all(np.abs(m_new[k] - st["exp_avg"].numpy()) <= 1e-14 * scale + 1e-300)
            np.testing.assert_allclose(v_new[k], st["exp_avg_sq"].numpy(), rtol=1e-13, atol=0)
            want = (p.detach() - before).numpy()
            T = geometry.to_h(new[k]) @ np.linalg.inv(geometry.to_h(poses[k]))
            got = geometry.se3_log(T)
            np.testing.assert_allclose(got, want, rtol=1e-9, atol=1e-15)
            assert int(st["step"]) == s
        poses, m, v = new, m_new, v_new


def test_mlp_adamw_matches_torch_adamw_over_many_steps():
    """Six AdamW steps of the refiner's optimizer (decoupled decay, then Adam
    at the 1-based step) from a resumed state, with the learning rate changing
    every step and the two weight decays of the refiner loop (0.01 on the MLP,
    0.1 on the translation offsets), against torch.optim.AdamW in float64."""
    rng = np.random.default_rng(5)
    for wd in (0.01, 0.1):
        x = rng.normal(size=40)
        m = rng.normal(size=40) * 1e-3
        v = np.abs(rng.normal(size=40)) * 1e-6
        s0 = 3
        p = torch.tensor(x.copy(), requires_grad=True)
        opt = torch.optim.AdamW([p], lr=1.0, betas=(0.9, 0.999), eps=1e-8, weight_decay=wd)
        opt.state[p] = {"step": torch.tensor(float(s0 - 1), dtype=torch.float64),
                        "exp_avg": torch.tensor(m.copy()), "exp_avg_sq": torch.tensor(v.copy())}
        for s in range(s0, s0 + 6):
            g = rng.normal(size=40) * 10.0 ** rng.uniform(-3, 0)
            lr = 2e-3 * (1.0 + 0.1 * s)
            scale = 0.9 * np.abs(m) + 0.1 * np.abs(g)
            x, m, v = mlp.adamw(x, m, v, g, s, lr, wd)
            opt.param_groups[0]["lr"] = lr
            p.grad = torch.tensor(g)
            opt.step()
            st = opt.state[p]
            np.testing.assert_allclose(x, p.detach().numpy(), rtol=1e-13, atol=1e-16)
            assert np.all(np.abs(m - st["exp_avg"].numpy()) <= 1e-14 * scale + 1e-300)
            np.testing.assert_allclose(v, st["exp_avg_sq"].numpy(), rtol=1e-13, atol=0)
