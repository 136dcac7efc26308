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

The joint loop (run_joint) adds the focal and depth refinement of Sec. 3
"Camera Refinement" / "Depth Refinement" to the loop of Alg. 2: each step
evaluates the cost at the refined intrinsics f = f0 (1 + gamma) and edge
depths Z = Z0 alpha + beta (each formed in float64 and rounded to float32
once: the paper's FP32 parameters), then the joint-phase AdamW step of
oracle.joint (gamma in both phases, alpha and beta in the joint phase only,
each with its own step count), the Adam twist step and the dual-phase test.

Pins: first Adam step equals -lr g/(|g| + eps) componentwise (closed form),
zero gradient leaves poses unchanged; the joint loop on the exact-zero
fixture takes pure weight-decay steps (closed form), its focal and depth
gradients against central differences of the loss in gamma, alpha and beta,
and its depth parameters stay put until their scene's switch, whose first
depth step is the closed form.
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


def joint_refinement(op: OracleProblem, gamma, alpha, beta, rounded: bool = True):
    """Intrinsics and edge depths the cost sees under the refinement (gamma
    per view; alpha, beta per edge pixel in the oracle's order: views in
    order, each view's edge pixels row-major): f = f0 (1 + gamma) and
    Z = Z0 alpha + beta in float64, rounded to float32 unless `rounded` is
    False (used by finite differences)."""
    K = op.K.copy()
    f = op.K[:, :2] * (1.0 + np.asarray(gamma, np.float64))[:, None]
    K[:, :2] = f.astype(np.float32) if rounded else f
    depth = {}
    o = 0
    for v in range(op.V):
        z0 = op.pts[v][2]
        n = z0.size
        z = z0 * np.asarray(alpha[o:o + n], np.float64) + np.asarray(beta[o:o + n], np.float64)
        depth[v] = z.astype(np.float32).astype(np.float64) if rounded else z
        o += n
    return K, depth


def record_views(op: OracleProblem) -> np.ndarray:
    """View of every edge pixel in the oracle's order."""
    return np.concatenate([np.full(op.pts[v][0].size, v, np.int64) for v in range(op.V)])


def joint_gradients(op: OracleProblem, r, gamma):
    """dL/dgamma, dL/dalpha, dL/dbeta from an evaluation at the refined state:
    f dL/df per view (the cost's focal term) times f0/f = 1/(1 + gamma), and
    by Z = Z0 alpha + beta, dL/dbeta = dL/dZ and dL/dalpha = Z0 dL/dZ."""
    gz = np.concatenate([r["grad_depth"].get(v, np.zeros(op.pts[v][0].size))
                         for v in range(op.V)])
    z0 = np.concatenate([op.pts[v][2] for v in range(op.V)])
    return {"grad_gamma": r["grad_focal"] / (1.0 + np.asarray(gamma, np.float64)),
            "grad_alpha": z0 * gz, "grad_beta": gz}


def joint_loop_step(op: OracleProblem, s: int, poses, m, v, jstate, phase=None,
                    params: CostParams = CostParams(), wd_focal=0.01, wd_depth=0.01,
                    b1=0.9, b2=0.999, eps=1e-8):
    """Step s of the joint loop from the given state.  `phase` (per scene:
    0 pose phase, 1 joint phase, 2 stopped) gates the step as in Alg. 2:
    a stopped scene's learning rate is 0, the focal scales step unless it
    stopped, the depth parameters only in the joint phase; None steps every
    parameter.  Returns the new poses, moments, joint state and the
    evaluation."""
    from . import joint
    S = op.n_scenes
    ph = None if phase is None else np.asarray(phase)
    lr = np.array([0.0 if (ph is not None and ph[k] == 2) else learning_rate(s) for k in range(S)])
    K, depth = joint_refinement(op, jstate["gamma"], jstate["alpha"], jstate["beta"])
    r = op.evaluate(poses, clamp_lambda(s), params, K=K, depth=depth)
    g = joint_gradients(op, r, jstate["gamma"])
    jstate = joint.joint_step(jstate, g, lr, op.scene_of_view, record_views(op), phase=ph,
                              b1=b1, b2=b2, eps=eps, wd_focal=wd_focal, wd_depth=wd_depth)
    new, m, v = adam_se3_step(poses, m, v, r["grad"], s + 1, lr, b1, b2, eps,
                              scene_of_view=op.scene_of_view)
    return new, m, v, jstate, r


def run_joint(op: OracleProblem, poses0: np.ndarray, n_iters: int,
              params: CostParams = CostParams(), convergence=(25, 0.5, 50, 0.1),
              wd_focal=0.01, wd_depth=0.01):
    """The two-phase loop of Alg. 2 with focal and depth refinement: per step
    the phase of each scene at the start of the step gates that step
    (joint_loop_step), then theta_95 of the scene's pose change updates its
    dual-phase test.  convergence=None steps every parameter from step 0 with
    no test."""
    from . import joint
    from .convergence import DualPhase, theta95
    poses = poses0.copy()
    m = np.zeros((op.V, 6))
    v = np.zeros((op.V, 6))
    n_rec = sum(op.pts[k][0].size for k in range(op.V))
    jstate = joint.initial_state(op.V, n_rec, op.n_scenes)
    dual = [DualPhase(*convergence) for _ in range(op.n_scenes)] if convergence else None
    hist = dict(loss=[], theta=[], phase=[], gamma=[])
    for s in range(n_iters):
        phase = [d.phase for d in dual] if dual else None
        new, m, v, jstate, r = joint_loop_step(op, s, poses, m, v, jstate, phase, params,
                                               wd_focal, wd_depth)
        hist["loss"].append(r["loss"].copy())
        hist["gamma"].append(jstate["gamma"].copy())
        if dual:
            th = []
            for k, d in enumerate(dual):
                views = np.flatnonzero(op.scene_of_view == k)
                t = theta95(new[views], poses[views])
                d.update(t)
                th.append(t)
            hist["theta"].append(th)
            hist["phase"].append([d.phase for d in dual])
        poses = new
    hist["final_poses"] = poses
    hist["m"], hist["v"], hist["joint"] = m, v, jstate
    hist["switch_steps"] = [list(d.switch_step) for d in dual] if dual else None
    return hist
