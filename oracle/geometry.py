"""Oracle: SE(3) helpers in float64.

Test infrastructure only (see the package header).

Poses are world->camera matrices P = [R | t] (Sec. 3 "Preliminaries": the
camera head predicts P = [R | t]).  The optimised variables are left twists
xi = (rho, omega) in se(3) (translation first, rotation second), applied as
P <- Exp(xi) P.  Exp is the closed-form SE(3) exponential: Rodrigues' formula
for the rotation and the left Jacobian V(omega) for the translation,

  Exp(rho, omega) = [ R(omega) | V(omega) rho ],
  R = I + sin(th)/th [w]x + (1 - cos th)/th^2 [w]x^2,
  V = I + (1 - cos th)/th^2 [w]x + (th - sin th)/th^3 [w]x^2,

with Taylor expansions below th = 1e-4.  Log is its inverse (tests only).

Pins: Exp(Log T) = T on random poses and at angles within 1e-6 of pi (the
near-pi branch of Log), Rodrigues against the matrix exponential of the
twist (scipy.linalg.expm), pure translations, continuity of the small-angle
branch.
"""
from __future__ import annotations

import numpy as np

SMALL = 1e-4


def hat(w: np.ndarray) -> np.ndarray:
    wx, wy, wz = w
    return np.array([[0.0, -wz, wy], [wz, 0.0, -wx], [-wy, wx, 0.0]])


def _coeffs(th: float):
    """a = sin/th, b = (1-cos)/th^2, c = (th - sin)/th^3."""
    if th < SMALL:
        t2 = th * th
        return 1.0 - t2 / 6.0, 0.5 - t2 / 24.0, 1.0 / 6.0 - t2 / 120.0
    return np.sin(th) / th, (1.0 - np.cos(th)) / th ** 2, (th - np.sin(th)) / th ** 3


def se3_exp(xi: np.ndarray) -> np.ndarray:
    """4x4 homogeneous matrix of Exp(xi), xi = (rho, omega)."""
    rho, w = np.asarray(xi[:3], float), np.asarray(xi[3:], float)
    th = float(np.linalg.norm(w))
    a, b, c = _coeffs(th)
    W = hat(w)
    W2 = W @ W
    R = np.eye(3) + a * W + b * W2
    V = np.eye(3) + b * W + c * W2
    T = np.eye(4)
    T[:3, :3] = R
    T[:3, 3] = V @ rho
    return T


def so3_log(R: np.ndarray) -> np.ndarray:
    # the angle from both parts of R = I + sin(th) [n]x + (1 - cos th) [n]x^2:
    # (trace - 1)/2 = cos th and the antisymmetric part's vee = 2 sin(th) n,
    # so atan2 keeps full precision near 0 and near pi (arccos alone loses
    # half the digits there)
    anti = np.array([R[2, 1] - R[1, 2], R[0, 2] - R[2, 0], R[1, 0] - R[0, 1]])
    th = float(np.arctan2(0.5 * np.linalg.norm(anti), (np.trace(R) - 1.0) / 2.0))
    if th < SMALL:
        return 0.5 * anti
    if np.pi - th < 1e-6:
        # near pi the antisymmetric part sin(th) [n]x vanishes: the axis up
        # to its sign comes from the symmetric part, (R + R^T)/4 + I/2 =
        # n n^T + O((pi - th)^2), the column of its largest diagonal entry;
        # the sign is that of the (small) antisymmetric part, either sign at
        # exactly pi
        M = ((R + R.T) / 2.0 + np.eye(3)) / 2.0
        k = int(np.argmax(np.diag(M)))
        axis = M[:, k] / np.linalg.norm(M[:, k])
        if axis @ anti < 0.0:
            axis = -axis
        return th * axis
    return th / (2.0 * np.sin(th)) * anti


def se3_log(T: np.ndarray) -> np.ndarray:
    R, t = T[:3, :3], T[:3, 3]
    w = so3_log(R)
    th = float(np.linalg.norm(w))
    a, b, c = _coeffs(th)
    V = np.eye(3) + b * hat(w) + c * hat(w) @ hat(w)
    return np.concatenate([np.linalg.solve(V, t), w])


def to_h(P: np.ndarray) -> np.ndarray:
    T = np.eye(4)
    T[:3, :] = P
    return T


def left_update(P: np.ndarray, xi: np.ndarray) -> np.ndarray:
    """[R | t] <- Exp(xi) [R | t]."""
    return (se3_exp(xi) @ to_h(P))[:3, :]


def rotation_angle_deg(Ra: np.ndarray, Rb: np.ndarray) -> float:
    cos = np.clip((np.trace(Ra @ Rb.T) - 1.0) / 2.0, -1.0, 1.0)
    return float(np.degrees(np.arccos(cos)))


def camera_center(P: np.ndarray) -> np.ndarray:
    return -P[:, :3].T @ P[:, 3]
