"""CPU: the oracle's pose parameterization (MLP refiner, 6D rotation with
Gram-Schmidt, translation offset, AdamW) against closed forms and finite
differences."""
import numpy as np
import pytest
from scipy.spatial.transform import Rotation

from oracle import mlp


def test_bf16_rounding_closed_forms():
    u = 2.0 ** -7                       # bf16 spacing just above 1
    cases = [(1.0, 1.0), (1 + u / 2, 1.0), (1 + 1.5 * u, 1 + 2 * u),
             (1 + u / 2 + 2.0 ** -20, 1 + u), (-(1 + 1.5 * u), -(1 + 2 * u)),
             (3.0, 3.0), (0.0, 0.0), (2.0 ** -130, 2.0 ** -130), (65504.0, 65536.0),
             (1 + u / 2 - 2.0 ** -20, 1.0)]
    for x, want in cases:
        assert mlp.bf16(x) == want, (x, mlp.bf16(x), want)
    # every bfloat16 value is a fixed point
    v = np.arange(0, 1 << 16, 7, dtype=np.uint32) << np.uint32(16)
    f32 = v.view(np.float32)
    f = f32[np.isfinite(f32)].astype(np.float64)
    assert np.array_equal(mlp.bf16(f), f)


def test_layout_and_init():
    assert mlp.N_PARAMS == 12 * 128 + 128 + 4 * (128 * 128 + 128) + 128 * 12 + 12
    rng = np.random.default_rng(0)
    th = mlp.init_params(rng)
    Ws, bs = mlp.unpack(th)
    assert all(np.all(b == 0) for b in bs) and np.all(Ws[5] == 0)
    for W, (out, inp) in zip(Ws[:5], mlp.LAYERS[:5]):
        assert abs(W.std() / np.sqrt(2.0 / inp) - 1) < 0.05
    P0 = np.stack([np.concatenate([Rotation.random(random_state=k).as_matrix(),
                                   rng.normal(size=(3, 1))], axis=1) for k in range(5)])
    o, _ = mlp.forward(th, P0)
    assert np.all(o == 0.0)                     # the zero last layer returns P0
    P = mlp.assemble(P0, o, np.zeros((5, 3)))
    assert np.abs(P - P0).max() < 1e-14


def test_gram_schmidt_properties():
    rng = np.random.default_rng(1)
    for _ in range(20):
        R = Rotation.random(random_state=rng).as_matrix()
        assert np.abs(mlp.gram_schmidt(R) - R).max() < 1e-15
        A = rng.normal(size=(3, 3))
        Q = mlp.gram_schmidt(A)
        assert np.abs(Q.T @ Q - np.eye(3)).max() < 1e-14 and np.linalg.det(Q) > 0
        # invariant to scaling a1 and to adding a1 to a2; ignores the 3rd column
        B = A.copy()
        B[:, 0] *= 3.7
        B[:, 1] += 2.0 * A[:, 0]
        B[:, 2] = rng.normal(size=3)
        assert np.abs(mlp.gram_schmidt(B) - Q).max() < 1e-14


def test_gram_schmidt_backward_vs_finite_differences():
    rng = np.random.default_rng(2)
    A = rng.normal(size=(3, 3))
    G = rng.normal(size=(3, 3))
    dA = mlp.gram_schmidt_backward(A, G)
    h = 1e-6
    fd = np.zeros((3, 3))
    for i in range(3):
        for j in range(3):
            Ap, Am = A.copy(), A.copy()
            Ap[i, j] += h
            Am[i, j] -= h
            fd[i, j] = (np.sum(G * mlp.gram_schmidt(Ap)) - np.sum(G * mlp.gram_schmidt(Am))) / (2 * h)
    assert np.abs(dA - fd).max() < 1e-8 * np.abs(fd).max()
    assert np.all(dA[:, 2] == 0)


def _exp_left(xi, P):
    """Exp(xi) P for a left twist xi = (rho, omega) (first order is enough
    for central differences of size 1e-6)."""
    rho, om = xi[:3], xi[3:]
    Rw = Rotation.from_rotvec(om).as_matrix()
    th = np.linalg.norm(om)
    K = mlp.hat(om)
    V = np.eye(3) if th < 1e-12 else (np.eye(3) + (1 - np.cos(th)) / th ** 2 * K
                                      + (th - np.sin(th)) / th ** 3 * K @ K)
    return np.concatenate([Rw @ P[:, :3], (Rw @ P[:, 3] + V @ rho)[:, None]], axis=1)


def test_pose_chain_vs_finite_differences():
    """For a smooth function f of the 12 pose entries: its left-twist gradient
    (by central differences on twists), pushed back by pose_backward, equals
    central differences of f(assemble(P0, o, delta)) in o and delta."""
    rng = np.random.default_rng(3)
    C = rng.normal(size=(3, 4))
    D = rng.normal(size=(3, 4))
    f = lambda P: float(np.sum(C * P) + 0.5 * np.sum(D * P * P))
    P0 = np.concatenate([Rotation.random(random_state=4).as_matrix(), rng.normal(size=(3, 1))], 1)
    o = 0.05 * rng.normal(size=12)
    delta = 0.1 * rng.normal(size=3)
    P = mlp.assemble(P0[None], o[None], delta[None])[0]
    h = 1e-6
    g = np.zeros(6)
    for k in range(6):
        e = np.zeros(6)
        e[k] = h
        g[k] = (f(_exp_left(e, P)) - f(_exp_left(-e, P))) / (2 * h)
    d_o, d_delta = mlp.pose_backward(P0[None], o[None], P[None], g[None])
    fd_o = np.zeros(12)
    for k in range(12):
        e = np.zeros(12)
        e[k] = h
        fd_o[k] = (f(mlp.assemble(P0[None], (o + e)[None], delta[None])[0])
                   - f(mlp.assemble(P0[None], (o - e)[None], delta[None])[0])) / (2 * h)
    fd_d = np.zeros(3)
    for k in range(3):
        e = np.zeros(3)
        e[k] = h
        fd_d[k] = (f(mlp.assemble(P0[None], o[None], (delta + e)[None])[0])
                   - f(mlp.assemble(P0[None], o[None], (delta - e)[None])[0])) / (2 * h)
    assert np.abs(d_o[0] - fd_o).max() < 1e-7 * np.abs(fd_o).max()
    assert np.abs(d_delta[0] - fd_d).max() < 1e-7 * np.abs(fd_d).max()


def test_mlp_backward_vs_finite_differences():
    """Without rounding the MLP is smooth away from ReLU kinks: its backward
    equals central differences of a linear function of the outputs."""
    rng = np.random.default_rng(5)
    th = mlp.init_params(rng).astype(np.float64)
    Ws, _ = mlp.unpack(th)
    wo, bo = mlp.OFFSETS[5]
    th[wo:bo] = rng.normal(0, 0.1, bo - wo)          # a non-zero last layer
    for (w0, b0), (out, inp) in zip(mlp.OFFSETS, mlp.LAYERS):
        th[b0:b0 + out] = rng.normal(0, 0.05, out)
    P0 = rng.normal(size=(6, 12))
    C = rng.normal(size=(6, 12))
    o, cache = mlp.forward(th, P0, rnd=mlp.exact)
    g = mlp.backward(th, cache, C)
    idx = np.concatenate([rng.choice(mlp.N_PARAMS, 60, replace=False),
                          [mlp.OFFSETS[0][0], mlp.OFFSETS[2][1], mlp.N_PARAMS - 1]])
    h = 1e-6
    for k in idx:
        tp, tm = th.copy(), th.copy()
        tp[k] += h
        tm[k] -= h
        fd = (np.sum(C * mlp.forward(tp, P0, rnd=mlp.exact)[0])
              - np.sum(C * mlp.forward(tm, P0, rnd=mlp.exact)[0])) / (2 * h)
        assert abs(fd - g[k]) < 1e-6 * max(1.0, abs(fd)), (k, fd, g[k])


def test_adamw_first_step_closed_form():
    rng = np.random.default_rng(6)
    x = rng.normal(size=50)
    g = rng.normal(size=50)
    lr, wd = 3e-3, 0.01
    x1, m, v = mlp.adamw(x, np.zeros(50), np.zeros(50), g, 1, lr, wd)
    np.testing.assert_allclose(x1, x * (1 - lr * wd) - lr * g / (np.abs(g) + 1e-8), rtol=1e-12)
    # zero learning rate: nothing moves, moments still update
    x2, m2, v2 = mlp.adamw(x, m, v, g, 2, 0.0, wd)
    assert np.array_equal(x2, x) and not np.array_equal(m2, m)


def test_generator_and_library_agree_on_the_layout():
    import re
    from synth import refiner
    hdr = open(__import__("os").path.join(__import__("os").path.dirname(__file__), "..",
                                          "include", "epo.h")).read()
    n = int(re.search(r"#define EPO_MLP_PARAMS (\d+)", hdr).group(1))
    assert n == mlp.N_PARAMS == refiner.N_PARAMS
    assert refiner.offsets() == mlp.OFFSETS


def test_loop_first_step_closed_form():
    """The loop with this parameterization, pinned by what its first step must
    do.  With the last layer zero the first poses are the initial ones and
    the loss is the plain loss there; only the last layer and delta receive
    gradient (the hidden layers see a zero backward signal through W6 = 0).
    Adam's first step moves every parameter by -lr g/(|g| + eps), so b6's
    translation entries move by -lr sign(sum_v g_rho) and each delta by
    -lr sign(g_rho) with g_rho the cost's own gradient at the initial poses;
    the hidden layers do not move."""
    from oracle import cost as ocost
    from oracle import loop as oloop
    from synth import make
    p = make("c1")
    op = ocost.OracleProblem(p)
    th = mlp.init_params(np.random.default_rng(0))[None].astype(np.float64)
    h = oloop.run_mlp(op, p.poses_init, th, 1)
    # Gram-Schmidt returns a rotation block up to rounding
    assert np.abs(h["poses"][0] - p.poses_init).max() < 1e-14
    r = op.evaluate(h["poses"][0], oloop.clamp_lambda(0))
    assert np.array_equal(h["loss"][0], r["loss"])
    lr = oloop.learning_rate(0)
    g_rho = r["grad"][:, :3]
    want_delta = -lr * g_rho / (np.abs(g_rho) + 1e-8)
    assert np.allclose(h["delta"], want_delta, rtol=1e-12, atol=0)
    (wo6, bo6) = mlp.OFFSETS[5]
    b6 = h["params"][0][bo6:bo6 + 12].reshape(3, 4)
    gs = g_rho.sum(axis=0)
    # the bias gradient sums bf16-rounded d_o, which moves g/(|g| + eps) by
    # about eps |dg| / g^2 < 1e-9 relative here
    assert np.allclose(b6[:, 3], -lr * gs / (np.abs(gs) + 1e-8), rtol=1e-9, atol=0)
    assert np.array_equal(h["params"][0][:wo6], th[0][:wo6] * (1.0 - lr * 0.01))


def test_loop_decreases_the_loss_c1():
    from oracle import cost as ocost
    from oracle import loop as oloop
    from synth import make
    p = make("c1")
    op = ocost.OracleProblem(p)
    th = mlp.init_params(np.random.default_rng(0))[None].astype(np.float64)
    h = oloop.run_mlp(op, p.poses_init, th, 60)
    assert h["loss"][-1][0] < 0.1 * h["loss"][0][0]
