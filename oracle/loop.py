"""Oracle: schedules, the Adam step on se(3) twists and the iteration loop.

Test infrastructure only (see the package header).

  * clamp annealing: lambda goes from 10 to 6 over the first 1000 steps
    (Alg. 3, AnnealClamp); read as linear, lambda(s) = 10 - 4 min(s, 1000)/1000;
  * learning rate: linear warm-up to 3e-3 over 25 steps, then cosine decay
    over N = 2000 iterations (Sec. 4 "Implementation Details"); read as
    lr(s) = 3e-3 (s + 1)/25 for s < 25, else
    3e-3 (1 + cos(pi (s - 25)/(2000 - 25)))/2;
  * optimizer: Adam with beta = (0.9, 0.999) (Sec. 4), eps = 1e-8, no weight
    decay (the paper's decay acts on network parameters that a direct twist
    parameterization does not have), on left twists of each pose:
      m <- b1 m + (1 - b1) g,  v <- b2 v + (1 - b2) g^2,
      step = -lr (m / (1 - b1^s)) / (sqrt(v / (1 - b2^s)) + eps),
      P <- Exp(step) P;
    poses in `fixed` skip both the moment update and the step.

Pins: first Adam step equals -lr g/(|g| + eps) componentwise (closed form),
zero gradient leaves poses unchanged.
"""
from __future__ import annotations

import math

import numpy as np

from .cost import CostParams, OracleProblem
from .geometry import left_update


def clamp_lambda(step: int) -> float:
    return 10.0 - 4.0 * min(step, 1000) / 1000.0


def learning_rate(step: int, peak: float = 3e-3, warmup: int = 25, total: int = 2000) -> float:
    if step < warmup:
        return peak * (step + 1) / warmup
    return peak * 0.5 * (1.0 + math.cos(math.pi * (step - warmup) / (total - warmup)))


def adam_se3_step(poses, m, v, g, step: int, lr, b1=0.9, b2=0.999, eps=1e-8, fixed=None,
                  scene_of_view=None):
    """One Adam update of every pose; `step` counts from 1.  `lr` is a scalar
    or one value per scene (with scene_of_view)."""
    poses = poses.copy()
    m = m.copy()
    v = v.copy()
    V = poses.shape[0]
    lr = np.asarray(lr, np.float64)
    for k in range(V):
        if fixed is not None and fixed[k]:
            continue
        m[k] = b1 * m[k] + (1.0 - b1) * g[k]
        v[k] = b2 * v[k] + (1.0 - b2) * g[k] * g[k]
        mhat = m[k] / (1.0 - b1 ** step)
        vhat = v[k] / (1.0 - b2 ** step)
        lr_k = float(lr) if lr.ndim == 0 else float(lr[scene_of_view[k]])
        delta = -lr_k * mhat / (np.sqrt(vhat) + eps)
        poses[k] = left_update(poses[k], delta)
    return poses, m, v


def run(op: OracleProblem, poses0: np.ndarray, n_iters: int, params: CostParams = CostParams(),
        fixed=None, start_step: int = 0, record_every: int = 1, m0=None, v0=None,
        sampling=None, evaluate=None):
    """The optimisation loop: for s = start .. start + n - 1 evaluate lambda(s)
    and lr(s), the loss and the gradient at the current poses, then step.
    Recorded per iteration: the loss, the gradient norm, and the state the
    iteration starts from (poses and Adam moments).  `sampling = (seed, M)`
    evaluates each step on the fresh pair subset of that step (stochastic
    viewgraph sub-sampling).  `evaluate` replaces op.evaluate (same
    arguments and result; a process-parallel form of it)."""
    from .sampling import selected_pairs
    evaluate = op.evaluate if evaluate is None else evaluate
    poses = poses0.copy()
    m = np.zeros((op.V, 6)) if m0 is None else m0.copy()
    v = np.zeros((op.V, 6)) if v0 is None else v0.copy()
    hist = dict(loss=[], grad_norm=[], poses=[], m_hist=[], v_hist=[])
    for s in range(start_step, start_step + n_iters):
        sel = None
        if sampling is not None:
            sel = selected_pairs(op.pairs, op.scene_of_pair, sampling[0], s, sampling[1])
        r = evaluate(poses, clamp_lambda(s), params, selected=sel)
        if (s - start_step) % record_every == 0:
            hist["loss"].append(r["loss"].copy())
            hist["grad_norm"].append(float(np.linalg.norm(r["grad"])))
            hist["poses"].append(poses.copy())
            hist["m_hist"].append(m.copy())
            hist["v_hist"].append(v.copy())
        poses, m, v = adam_se3_step(poses, m, v, r["grad"], s + 1, learning_rate(s),
                                    fixed=fixed)
    hist["final_poses"] = poses
    hist["m"], hist["v"] = m, v
    return hist


def run_with_convergence(op: OracleProblem, poses0: np.ndarray, n_iters: int,
                         params: CostParams = CostParams(), w1=25, eps1=0.5, w2=50, eps2=0.1):
    """The loop of Alg. 2 with the pose-change signal and the dual-phase test
    kept per scene: after every step theta_95 of each scene is recorded; a
    scene whose phase-2 test has fired stops moving (its learning rate is 0
    from the next step on), which is what ending the loop means for it."""
    from .convergence import DualPhase, theta95
    poses = poses0.copy()
    m = np.zeros((op.V, 6))
    v = np.zeros((op.V, 6))
    sov = op.scene_of_view
    dual = [DualPhase(w1, eps1, w2, eps2) for _ in range(op.n_scenes)]
    hist = dict(loss=[], theta=[], phase=[])
    for s in range(n_iters):
        lr = np.array([0.0 if d.phase == 2 else learning_rate(s) for d in dual])
        r = op.evaluate(poses, clamp_lambda(s), params)
        new, m, v = adam_se3_step(poses, m, v, r["grad"], s + 1, lr, scene_of_view=sov)
        th = []
        for k, d in enumerate(dual):
            views = np.flatnonzero(sov == k)
            t = theta95(new[views], poses[views])
            d.update(t)
            th.append(t)
        poses = new
        hist["loss"].append(r["loss"].copy())
        hist["theta"].append(th)
        hist["phase"].append([d.phase for d in dual])
    hist["final_poses"] = poses
    hist["switch_steps"] = [list(d.switch_step) for d in dual]
    return hist



def run_mlp(op: OracleProblem, P0: np.ndarray, theta0: np.ndarray, n_iters: int,
            params: CostParams = CostParams(), wd_mlp: float = 0.01, wd_delta: float = 0.1,
            convergence=None):
    """The loop with the paper's pose parameterization (Sec. 3 "Pose
    Refinement", Sec. 4): the poses are phi(P0 + MLP(P0)) + [0 | delta] per
    scene (P0: the initial poses, theta0: one parameter row per scene, delta
    starting at zero); at step s the loss and its left-twist gradient are
    evaluated at the current poses with lambda(s), the gradient goes back
    through phi and the MLP, and AdamW steps the MLP parameters and delta with
    lr(s).  `convergence = (w1, eps1, w2, eps2)` adds the dual-phase test on
    theta_95 of consecutive poses per scene, as in run_with_convergence."""
    from . import mlp
    from .convergence import DualPhase, theta95
    P0 = np.asarray(P0, np.float64)
    S, sov = op.n_scenes, op.scene_of_view
    rows = [np.flatnonzero(sov == k) for k in range(S)]
    theta = np.asarray(theta0, np.float64).copy()
    m = np.zeros_like(theta)
    v = np.zeros_like(theta)
    delta = np.zeros((op.V, 3))
    dm = np.zeros_like(delta)
    dv = np.zeros_like(delta)
    dual = [DualPhase(*convergence) for _ in range(S)] if convergence else None

    def poses_of(theta, delta):
        out = np.zeros((op.V, 3, 4))
        fw = []
        for k in range(S):
            o, cache = mlp.forward(theta[k], P0[rows[k]].reshape(-1, 12))
            out[rows[k]] = mlp.assemble(P0[rows[k]], o, delta[rows[k]])
            fw.append((o, cache))
        return out, fw

    poses, fw = poses_of(theta, delta)
    hist = dict(loss=[], poses=[], theta=[], phase=[])
    for s in range(n_iters):
        lr = np.array([0.0 if dual and dual[k].phase == 2 else learning_rate(s)
                       for k in range(S)])
        r = op.evaluate(poses, clamp_lambda(s), params)
        hist["loss"].append(r["loss"].copy())
        hist["poses"].append(poses.copy())
        g_delta = np.zeros_like(delta)
        for k in range(S):
            o, cache = fw[k]
            d_o, g_delta[rows[k]] = mlp.pose_backward(P0[rows[k]], o, poses[rows[k]],
                                                      r["grad"][rows[k]])
            g = mlp.backward(theta[k], cache, d_o)
            theta[k], m[k], v[k] = mlp.adamw(theta[k], m[k], v[k], g, s + 1, lr[k], wd_mlp)
        delta, dm, dv = mlp.adamw(delta, dm, dv, g_delta, s + 1, lr[sov][:, None], wd_delta)
        new, fw = poses_of(theta, delta)
        if dual:
            th = [theta95(new[rows[k]], poses[rows[k]]) for k in range(S)]
            for k in range(S):
                dual[k].update(th[k])
            hist["theta"].append(th)
            hist["phase"].append([d.phase for d in dual])
        poses = new
    hist["final_poses"] = poses
    hist["params"], hist["delta"] = theta, delta
    return hist
