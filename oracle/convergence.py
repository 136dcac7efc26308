"""Oracle: pose-change signal and the dual-phase convergence test.

Test infrastructure only (see the package header).

Paper Sec. 3 "Optimization Schedule", Alg. 2 and Sec. A1.1:
  * per pose i between steps s-1 and s, in degrees,
      dR_i = (180/pi) arccos((tr(R_i^s (R_i^{s-1})^T) - 1) / 2)
      dt_i = (180/pi) arccos(t_i^s / |t_i^s| . t_i^{s-1} / |t_i^{s-1}|)
    (t is the translation of the world->camera matrix [R | t]); the arccos
    argument is clipped to [-1, 1];
  * dR_95, dt_95 = 95th percentiles over the poses (of one scene), and
    theta_95 = max(dR_95, dt_95);
  * Converged(theta^{0:s}; w, eps): the signal is smoothed by a moving average
    over w steps, and the test fires when every smoothed value in the last w
    steps is below eps;
  * phase 1 (w1 = 25, eps1 = 0.5) ends the pose-only phase; phase 2
    (w2 = 50, eps2 = 0.1) then stops the run.

Readings:
  * percentile: linear interpolation between order statistics at rank
    (n - 1) q of the ascending values (NumPy's default method);
  * the moving average at step s is the mean of theta at steps s-w+1 .. s and
    exists from step w-1 on; Converged at step s therefore needs s >= 2w - 2
    (w smoothed values);
  * both tests read the whole history theta^{0:s}, as Alg. 2 passes it; the
    phase-2 test starts at the step after the phase-1 switch (Alg. 2's
    if / else-if).

Pins: closed-form rotations and translations, the percentile against
numpy.percentile (an independent library routine), hand-built signals with a
known firing step.
"""
from __future__ import annotations

import math

import numpy as np


def rotation_change_deg(R_new: np.ndarray, R_old: np.ndarray) -> float:
    c = (np.trace(R_new @ R_old.T) - 1.0) / 2.0
    return math.degrees(math.acos(min(1.0, max(-1.0, c))))


def translation_change_deg(t_new: np.ndarray, t_old: np.ndarray) -> float:
    a = t_new / np.linalg.norm(t_new)
    b = t_old / np.linalg.norm(t_old)
    c = float(a @ b)
    return math.degrees(math.acos(min(1.0, max(-1.0, c))))


def percentile(values, q: float) -> float:
    """q in [0, 100]; linear interpolation at rank (n - 1) q / 100."""
    x = sorted(float(v) for v in values)
    n = len(x)
    if n == 1:
        return x[0]
    r = (n - 1) * q / 100.0
    lo = int(math.floor(r))
    hi = min(lo + 1, n - 1)
    return x[lo] + (r - lo) * (x[hi] - x[lo])


def theta95(poses_new: np.ndarray, poses_old: np.ndarray) -> float:
    dR = [rotation_change_deg(poses_new[k][:, :3], poses_old[k][:, :3])
          for k in range(poses_new.shape[0])]
    dt = [translation_change_deg(poses_new[k][:, 3], poses_old[k][:, 3])
          for k in range(poses_new.shape[0])]
    return max(percentile(dR, 95.0), percentile(dt, 95.0))


def converged(theta_hist, w: int, eps: float) -> bool:
    """Every moving average (window w) over the last w steps is below eps."""
    n = len(theta_hist)
    if n < 2 * w - 1:
        return False
    for s in range(n - w, n):
        ma = sum(theta_hist[s - w + 1:s + 1]) / w
        if not ma < eps:
            return False
    return True


class DualPhase:
    """Phase 0: poses only; phase 1: joint (depth) phase; phase 2: stopped."""

    def __init__(self, w1=25, eps1=0.5, w2=50, eps2=0.1):
        self.w1, self.eps1, self.w2, self.eps2 = w1, eps1, w2, eps2
        self.phase = 0
        self.hist = []          # theta^{0:s}
        self.switch_step = [None, None]
        self.step = 0

    def update(self, theta: float) -> int:
        self.hist.append(float(theta))
        if self.phase == 0:
            if converged(self.hist, self.w1, self.eps1):
                self.phase, self.switch_step[0] = 1, self.step
        elif self.phase == 1 and converged(self.hist, self.w2, self.eps2):
            self.phase, self.switch_step[1] = 2, self.step
        self.step += 1
        return self.phase
