"""Pins of the oracle's pose-change signal and dual-phase convergence (CPU)."""
import math

import numpy as np
import pytest
from scipy.spatial.transform import Rotation

from oracle import convergence as oc


def test_rotation_change_closed_form():
    rng = np.random.default_rng(0)
    for ang in (0.0, 1e-3, 0.5, 7.0, 90.0, 179.0):
        R0 = Rotation.random(random_state=rng.integers(1 << 31)).as_matrix()
        axis = rng.normal(size=3)
        axis /= np.linalg.norm(axis)
        R1 = Rotation.from_rotvec(axis * math.radians(ang)).as_matrix() @ R0
        assert abs(oc.rotation_change_deg(R1, R0) - ang) < 1e-5


def test_translation_change_closed_form():
    t0 = np.array([3.0, 0.0, 0.0])
    for ang in (0.0, 0.25, 30.0, 120.0):
        a = math.radians(ang)
        t1 = 2.5 * np.array([math.cos(a), math.sin(a), 0.0])   # length does not matter
        assert abs(oc.translation_change_deg(t1, t0) - ang) < 1e-6


@pytest.mark.parametrize("n", [1, 2, 3, 8, 20, 48, 200])
def test_percentile_matches_numpy(n):
    rng = np.random.default_rng(n)
    x = rng.exponential(size=n)
    for q in (0, 50, 95, 100):
        assert abs(oc.percentile(x, q) - np.percentile(x, q)) < 1e-12


def test_percentile_hand_example():
    # 21 values 0..20: rank 0.95 * 20 = 19 exactly
    assert oc.percentile(list(range(21)), 95) == 19.0
    # 5 values: rank 3.8 between 30 and 40
    assert abs(oc.percentile([10, 20, 30, 40, 50], 95) - 48.0) < 1e-12


def test_theta95_takes_the_larger_percentile():
    V = 10
    poses_old = np.stack([np.concatenate([np.eye(3), [[1.0], [0.0], [0.0]]], 1)] * V)
    poses_new = poses_old.copy()
    # rotate pose k by k degrees about z; translations unchanged
    for k in range(V):
        poses_new[k][:, :3] = Rotation.from_rotvec([0, 0, math.radians(k)]).as_matrix()
    # dR = 0..9: 95th percentile at rank 8.55 -> 8.55; dt = 0
    assert abs(oc.theta95(poses_new, poses_old) - 8.55) < 1e-6


def test_converged_fires_at_known_step():
    w, eps = 3, 1.0
    theta = [5.0, 5.0, 5.0, 0.1, 0.1, 0.1, 0.1, 0.1, 0.1]
    # moving averages (from step 2): 5, 3.4, 1.8, 0.1, 0.1, 0.1, 0.1
    fired = [oc.converged(theta[:s + 1], w, eps) for s in range(len(theta))]
    # steps 5, 6, 7 have MA 0.1 -> first s whose last 3 MAs (s-2..s) are < 1 is s = 7
    assert fired.index(True) == 7
    assert not any(fired[:7])


def test_dual_phase_switches_then_stops():
    dp = oc.DualPhase(w1=2, eps1=1.0, w2=3, eps2=0.1)
    seq = [3.0, 3.0, 0.5, 0.5, 0.5, 0.05, 0.05, 0.05, 0.05, 0.05, 0.05]
    phases = [dp.update(t) for t in seq]
    # phase 1: MA_s = mean(theta[s-1:s+1]); fires when MA_{s-1}, MA_s < 1 -> s = 4
    assert dp.switch_step[0] == 4
    # phase 2 (whole history, w = 3): MAs from s = 2; need MA_{s-2..s} < 0.1:
    # MA_7 = mean(.05,.05,.05) ... first s with three such = 9
    assert dp.switch_step[1] == 9
    assert phases[-1] == 2 and phases[4] == 1 and phases[3] == 0


def test_loop_with_convergence_freezes_a_stopped_scene():
    from oracle import cost, loop
    from synth import make
    p = make("c1")
    h = loop.run_with_convergence(cost.OracleProblem(p), p.poses_init, 60, w1=5, eps1=0.15,
                                  w2=8, eps2=0.1)
    stop = h["switch_steps"][0][1]
    assert stop is not None and h["switch_steps"][0][0] < stop
    th = np.array(h["theta"])[:, 0]
    # the steps after the stop move nothing (Exp(0) P = P bitwise); theta of
    # identical rotations is not exactly 0 only because acos amplifies the
    # rounding of tr(R R^T) next to 3
    assert np.all(th[stop + 1:] < 1e-5)
    assert np.all(np.array(h["phase"])[stop:, 0] == 2)
