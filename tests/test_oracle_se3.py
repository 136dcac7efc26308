"""Pins of the oracle's SE(3) exponential, schedules and Adam step (CPU)."""
import math

import numpy as np
from scipy.linalg import expm

from oracle import geometry, loop


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
