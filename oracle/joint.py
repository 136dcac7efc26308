"""Oracle: the optimizer step of the joint phase (focal scales and per-pixel
depth scale and shift).

Test infrastructure only (see the package header).

Paper Sec. 3 "Camera Refinement" and "Depth Refinement": the refined focal
length of view v is f0_v (1 + gamma_v) and the refined depth of edge pixel p
is Z0_p alpha_p + beta_p.  Sec. 4 "Implementation Details": every parameter
is trained with AdamW, beta = (0.9, 0.999), weight decay 0.01.  Alg.
EPO.Forward builds one optimizer per module; the depth optimizer steps only
once the pose-phase criterion holds (phase 2 of the paper, phase 1 of the
convergence state here), and the loop stops after the second criterion
(phase 2 here), when nothing steps.

Readings (where the paper is silent):
  * AdamW as decoupled weight decay x <- x (1 - lr wd) followed by Adam with
    bias correction at the 1-based step t of the optimizer that owns the
    parameter; the decay acts on the parameter itself (alpha decays towards
    0, not towards its identity value 1), as the paper's optimizer does;
  * each scene's focal scales and its depth parameters count their own
    steps, as separate optimizers do: the focal count advances at every step
    the scene's focal scales take (both phases), the depth count only at the
    steps its depth parameters take (the joint phase), so the depth
    optimizer's first step after the phase switch is its step 1;
  * a parameter that does not step keeps its value, its moments and its
    step count (no decay either);
  * alpha and beta are float32 parameters (the paper computes in FP32 outside
    the MLP); each step is formed in float64 from the stored value and
    rounded to float32 once.

Pinned by tests/test_oracle_joint.py against torch.optim.AdamW (float64,
several steps, one learning rate per scene, the depth optimizer created at
each scene's phase switch), the first-step closed forms and the phase gate.
"""
import numpy as np


def adamw_update(x, m, v, g, t, lr, wd, b1=0.9, b2=0.999, eps=1e-8):
    """One AdamW step of float64 arrays at 1-based step t; lr and t
    broadcast."""
    x = x * (1.0 - lr * wd)
    m = b1 * m + (1.0 - b1) * g
    v = b2 * v + (1.0 - b2) * g * g
    m_hat = m / (1.0 - b1 ** t)
    v_hat = v / (1.0 - b2 ** t)
    return x - lr * m_hat / (np.sqrt(v_hat) + eps), m, v


def initial_state(n_views, n_records, n_scenes):
    """Identity refinement (gamma 0, alpha 1, beta 0), zero moments, no
    steps taken."""
    st = {"gamma": np.zeros(n_views), "alpha": np.ones(n_records, np.float32),
          "beta": np.zeros(n_records, np.float32), "m_gamma": np.zeros(n_views),
          "v_gamma": np.zeros(n_views), "steps": np.zeros((2, n_scenes), np.int64)}
    for k in ("alpha", "beta"):
        st["m_" + k] = np.zeros(n_records)
        st["v_" + k] = np.zeros(n_records)
    return st


def joint_step(state, grads, lr, scene_of_view, view_of_record, phase=None, b1=0.9,
               b2=0.999, eps=1e-8, wd_focal=0.01, wd_depth=0.01, round_depth=True):
    """One joint-phase step.

    state: dict of gamma [V] f64, alpha, beta [n] f32, m_gamma, v_gamma [V],
    m_alpha, v_alpha, m_beta, v_beta [n] (float64), steps [2, n_scenes]
    (steps taken so far by each scene's focal scales, then by its depth
    parameters); returns a new dict with the steps that were taken counted.
    grads: grad_gamma [V], grad_alpha, grad_beta [n] (float64).
    lr: [n_scenes]; phase: [n_scenes] ints or None (everything steps)."""
    sv = np.asarray(scene_of_view, np.int64)
    sr = sv[np.asarray(view_of_record, np.int64)]
    lr = np.asarray(lr, np.float64)
    out = {k: np.array(val, copy=True) for k, val in state.items()}
    n_scenes = out["steps"].shape[1]
    if phase is None:
        focal_s = np.ones(n_scenes, bool)
        depth_s = np.ones(n_scenes, bool)
    else:
        ph = np.asarray(phase)
        focal_s = ph != 2
        depth_s = ph == 1
    t_focal = (out["steps"][0] + 1).astype(np.float64)
    t_depth = (out["steps"][1] + 1).astype(np.float64)
    step_v = focal_s[sv]
    step_r = depth_s[sr]

    x, m, v = adamw_update(np.asarray(state["gamma"], np.float64), state["m_gamma"],
                           state["v_gamma"], grads["grad_gamma"], t_focal[sv], lr[sv], wd_focal,
                           b1, b2, eps)
    out["gamma"][step_v] = x[step_v]
    out["m_gamma"][step_v] = m[step_v]
    out["v_gamma"][step_v] = v[step_v]

    for name in ("alpha", "beta"):
        x, m, v = adamw_update(np.asarray(state[name], np.float64), state["m_" + name],
                               state["v_" + name], grads["grad_" + name], t_depth[sr], lr[sr],
                               wd_depth, b1, b2, eps)
        if round_depth:
            out[name][step_r] = x[step_r].astype(np.float32)
        else:
            out[name] = np.asarray(out[name], np.float64)
            out[name][step_r] = x[step_r]
        out["m_" + name][step_r] = m[step_r]
        out["v_" + name][step_r] = v[step_r]
    out["steps"][0] += focal_s
    out["steps"][1] += depth_s
    return out
