"""Oracle: the paper's pose parameterization (Sec. 3 "Pose Refinement",
Sec. 4 "Implementation Details"): a pose refiner MLP, the continuous 6D
rotation representation with Gram-Schmidt, a translation offset, AdamW.

Test infrastructure only (see the package header).

Per scene, every pose is produced from its initial pose P0 = [R0 | t0]:

    P = phi(P0 + MLP(P0)) + [0 | delta]

  * MLP: 12 inputs (P0 flattened row-major), six linear layers 12 -> 128 ->
    128 -> 128 -> 128 -> 128 -> 12, ReLU after the first five, a skip
    connection after the third (reading: the first layer's output is added to
    the third's, h3 = relu(W3 h2 + b3) + h1), 12 outputs (an offset of the
    flattened pose).  Kaiming-normal weights, zero biases, the last layer all
    zero (the initial pose is returned at the first step).
  * phi: the rotation block A of P0 + MLP(P0) is read in the 6D representation
    of Zhou et al. (its first two columns a1, a2) and orthonormalised by
    Gram-Schmidt: b1 = a1/|a1|, b2 = u2/|u2| with u2 = a2 - (b1.a2) b1,
    b3 = b1 x b2, R = [b1 b2 b3]; the translation is t0 + MLP's translation
    entries + delta.
  * precision (the paper runs the MLP in BF16): every matrix product takes
    bf16 operands (weights rounded from their float32 values, activations and
    activation gradients stored in bf16) and accumulates exactly here (float32
    on the device); bias, ReLU, skip sums and masks act on the accumulated
    values, which are rounded to bf16 once, where stored as the next
    product's operand; weight and bias gradients and the MLP output are not
    rounded.  The pose algebra (phi, its gradient) is float64.
  * gradient: from the left-twist gradient g = (g_rho, g_omega) of the pose
    P = [R | t]: dL/dt = g_rho and, for tangent changes dR = [w]x R,
    dL/dR = 1/2 [g_omega - t x g_rho]x R; back through Gram-Schmidt to dL/dA
    (its third column gets none), then through the MLP; dL/ddelta = g_rho.
  * AdamW (decoupled weight decay, as in Sec. 4): x <- x (1 - lr wd), then the
    Adam step with beta = (0.9, 0.999), eps = 1e-8; wd = 0.01 for the MLP and
    0.1 for delta.
"""
from __future__ import annotations

import numpy as np

HIDDEN = 128
N_IN = 12
N_OUT = 12
LAYERS = [(HIDDEN, N_IN), (HIDDEN, HIDDEN), (HIDDEN, HIDDEN), (HIDDEN, HIDDEN),
          (HIDDEN, HIDDEN), (N_OUT, HIDDEN)]          # (out, in) of each linear layer


def param_layout():
    """Offsets of W1, b1, ..., W6, b6 in one scene's flat parameter vector."""
    off, o = [], 0
    for out, inp in LAYERS:
        off.append((o, o + out * inp))
        o += out * inp + out
    return off, o


OFFSETS, N_PARAMS = param_layout()


def unpack(theta):
    Ws, bs = [], []
    for (wo, bo), (out, inp) in zip(OFFSETS, LAYERS):
        Ws.append(np.asarray(theta[wo:wo + out * inp], np.float64).reshape(out, inp))
        bs.append(np.asarray(theta[bo:bo + out], np.float64))
    return Ws, bs


def init_params(rng: np.random.Generator) -> np.ndarray:
    """Kaiming-normal weights (std sqrt(2 / fan_in)), zero biases, zero last
    layer; float32 like the device's parameters."""
    theta = np.zeros(N_PARAMS, np.float32)
    for k, ((wo, bo), (out, inp)) in enumerate(zip(OFFSETS, LAYERS)):
        if k < len(LAYERS) - 1:
            theta[wo:wo + out * inp] = rng.normal(0.0, np.sqrt(2.0 / inp), out * inp)
    return theta


def bf16(x):
    """Round to the nearest bfloat16 (ties to even), returned as float64."""
    f = np.asarray(x, np.float64).astype(np.float32)
    u = f.view(np.uint32).astype(np.uint64)
    lsb = (u >> np.uint64(16)) & np.uint64(1)
    u = (u + np.uint64(0x7FFF) + lsb) & np.uint64(0xFFFF0000)
    return u.astype(np.uint32).view(np.float32).astype(np.float64)


def exact(x):
    """No rounding (the smooth function the finite-difference pins use)."""
    return np.asarray(x, np.float64)


def forward(theta, P0, rnd=bf16):
    """MLP offsets o (n x 12, float64 holding the unrounded outputs) and the
    cache of stored activations (rounded by `rnd`, bf16 by default)."""
    Ws, bs = unpack(theta)
    Wq = [rnd(W) for W in Ws]
    h0 = rnd(np.asarray(P0, np.float64).reshape(-1, 12))
    h1 = rnd(np.maximum(h0 @ Wq[0].T + bs[0], 0.0))
    h2 = rnd(np.maximum(h1 @ Wq[1].T + bs[1], 0.0))
    y3 = np.maximum(h2 @ Wq[2].T + bs[2], 0.0)
    r3 = rnd(y3)
    h3 = rnd(y3 + h1)
    h4 = rnd(np.maximum(h3 @ Wq[3].T + bs[3], 0.0))
    h5 = rnd(np.maximum(h4 @ Wq[4].T + bs[4], 0.0))
    o = h5 @ Wq[5].T + bs[5]
    return o, dict(h=[h0, h1, h2, h3, h4, h5], r3=r3, Wq=Wq, rnd=rnd)


def backward(theta, cache, d_o):
    """Parameter gradient (flat, float64) from dL/do (n x 12)."""
    h0, h1, h2, h3, h4, h5 = cache["h"]
    Wq = cache["Wq"]
    bf16 = cache["rnd"]
    g = np.zeros(N_PARAMS)

    def put(k, dY, h_in):
        wo, bo = OFFSETS[k]
        out, inp = LAYERS[k]
        g[wo:wo + out * inp] = (dY.T @ h_in).ravel()
        g[bo:bo + out] = dY.sum(axis=0)

    dY6 = bf16(d_o)
    put(5, dY6, h5)
    dY5 = bf16((dY6 @ Wq[5]) * (h5 > 0))
    put(4, dY5, h4)
    dY4 = bf16((dY5 @ Wq[4]) * (h4 > 0))
    put(3, dY4, h3)
    dh3 = dY4 @ Wq[3]                              # kept unrounded for the skip
    dY3 = bf16(dh3 * (cache["r3"] > 0))
    put(2, dY3, h2)
    dY2 = bf16((dY3 @ Wq[2]) * (h2 > 0))
    put(1, dY2, h1)
    dY1 = bf16((dY2 @ Wq[1] + dh3) * (h1 > 0))
    put(0, dY1, h0)
    return g


def gram_schmidt(A):
    """phi: 3 x 3 block -> rotation from its first two columns."""
    a1, a2 = A[:, 0], A[:, 1]
    b1 = a1 / np.linalg.norm(a1)
    u2 = a2 - (b1 @ a2) * b1
    b2 = u2 / np.linalg.norm(u2)
    b3 = np.cross(b1, b2)
    return np.stack([b1, b2, b3], axis=1)


def gram_schmidt_backward(A, G):
    """dL/dA from dL/dR = G (columns g1, g2, g3) through phi."""
    a1, a2 = A[:, 0], A[:, 1]
    n1 = np.linalg.norm(a1)
    b1 = a1 / n1
    c = b1 @ a2
    u2 = a2 - c * b1
    n2 = np.linalg.norm(u2)
    b2 = u2 / n2
    g1, g2, g3 = G[:, 0], G[:, 1], G[:, 2]
    # b3 = b1 x b2
    gb1 = g1 + np.cross(b2, g3)
    gb2 = g2 + np.cross(g3, b1)
    # b2 = u2 / |u2|
    gu2 = (gb2 - b2 * (b2 @ gb2)) / n2
    # u2 = a2 - (b1 . a2) b1
    ga2 = gu2 - b1 * (b1 @ gu2)
    gb1 = gb1 - (c * gu2 + (b1 @ gu2) * a2)
    # b1 = a1 / |a1|
    ga1 = (gb1 - b1 * (b1 @ gb1)) / n1
    dA = np.zeros((3, 3))
    dA[:, 0] = ga1
    dA[:, 1] = ga2
    return dA


def hat(w):
    return np.array([[0.0, -w[2], w[1]], [w[2], 0.0, -w[0]], [-w[1], w[0], 0.0]])


def assemble(P0, o, delta):
    """Poses P = phi(P0 + o) + [0 | delta] (n x 3 x 4)."""
    P0 = np.asarray(P0, np.float64).reshape(-1, 3, 4)
    M = P0 + np.asarray(o, np.float64).reshape(-1, 3, 4)
    out = np.empty_like(P0)
    for k in range(P0.shape[0]):
        out[k, :, :3] = gram_schmidt(M[k, :, :3])
        out[k, :, 3] = M[k, :, 3] + delta[k]
    return out


def pose_backward(P0, o, poses, grad):
    """dL/do (n x 12) and dL/ddelta (n x 3) from the left-twist gradients."""
    P0 = np.asarray(P0, np.float64).reshape(-1, 3, 4)
    M = P0 + np.asarray(o, np.float64).reshape(-1, 3, 4)
    d_o = np.zeros((P0.shape[0], 3, 4))
    d_delta = np.zeros((P0.shape[0], 3))
    for k in range(P0.shape[0]):
        R, t = poses[k][:, :3], poses[k][:, 3]
        g_rho, g_omega = grad[k][:3], grad[k][3:]
        GR = 0.5 * hat(g_omega - np.cross(t, g_rho)) @ R
        d_o[k, :, :3] = gram_schmidt_backward(M[k, :, :3], GR)
        d_o[k, :, 3] = g_rho
        d_delta[k] = g_rho
    return d_o.reshape(-1, 12), d_delta


def adamw(x, m, v, g, step, lr, wd, b1=0.9, b2=0.999, eps=1e-8):
    """One AdamW step (decoupled weight decay, then Adam) at 1-based step."""
    x = x * (1.0 - lr * wd)
    m = b1 * m + (1.0 - b1) * g
    v = b2 * v + (1.0 - b2) * g * g
    mh = m / (1.0 - b1 ** step)
    vh = v / (1.0 - b2 ** step)
    return x - lr * mh / (np.sqrt(vh) + eps), m, v
