"""Oracle: the optimizer step of the joint phase (focal scales and per-pixel
depth scale and shift).

Test infrastructure only (see the package header).

Paper Sec. 3 "Camera Refinement" and "Depth Refinement": the refined focal
length of view v is f0_v (1 + gamma_v) and the refined depth of edge pixel p
is Z0_p alpha_p + beta_p.  Sec. 4 "Implementation Details": every parameter
is trained with AdamW, beta = (0.9, 0.999), weight decay 0.01.  Alg.
EPO.Forward: the depth optimizer steps only once the pose-phase criterion
holds (phase 2 of the paper, phase 1 of the convergence state here), and the
loop stops after the second criterion (phase 2 here), when nothing steps.

Readings (where the paper is silent):
  * AdamW as decoupled weight decay x <- x (1 - lr wd) followed by Adam with
    bias correction at the 1-based step t; the decay acts on the parameter
    itself (alpha decays towards 0, not towards its identity value 1), as the
    paper's optimizer does;
  * the focal scales step in both optimization phases, the depth parameters
    only in the joint phase; a parameter that does not step keeps its value
    and its moments (no decay either);
  * alpha and beta are float32 parameters (the paper computes in FP32 outside
    the MLP); each step is formed in float64 from the stored value and
    rounded to float32 once.

Pinned by tests/test_oracle_joint.py against torch.optim.AdamW (float64,
several steps, one learning rate per scene), the first-step closed forms and
the phase gate.
"""
import numpy as np


def adamw_update(x, m, v, g, t, lr, wd, b1=0.9, b2=0.999, eps=1e-8):
    """One AdamW step of float64 arrays at 1-based step t; lr broadcasts."""
    x = x * (1.0 - lr * wd)
    m = b1 * m + (1.0 - b1) * g
    v = b2 * v + (1.0 - b2) * g * g
    m_hat = m / (1.0 - b1 ** t)
    v_hat = v / (1.0 - b2 ** t)
    return x - lr * m_hat / (np.sqrt(v_hat) + eps), m, v


def joint_step(state, grads, lr, scene_of_view, view_of_record, step, phase=None, b1=0.9,
               b2=0.999, eps=1e-8, wd_focal=0.01, wd_depth=0.01, round_depth=True):
    """One joint-phase step.

    state: dict of gamma [V] f64, alpha, beta [n] f32, m_gamma, v_gamma [V],
    m_alpha, v_alpha, m_beta, v_beta [n] (float64); returns a new dict.
    grads: grad_gamma [V], grad_alpha, grad_beta [n] (float64).
    lr: [n_scenes]; step: steps taken before this one (t = step + 1);
    phase: [n_scenes] ints or None (everything steps)."""
    sv = np.asarray(scene_of_view, np.int64)
    sr = sv[np.asarray(view_of_record, np.int64)]
    lr = np.asarray(lr, np.float64)
    t = float(step + 1)
    out = {k: np.array(val, copy=True) for k, val in state.items()}
    if phase is None:
        step_v = np.ones(sv.size, bool)
        step_r = np.ones(sr.size, bool)
    else:
        ph = np.asarray(phase)
        step_v = ph[sv] != 2
        step_r = ph[sr] == 1

    x, m, v = adamw_update(np.asarray(state["gamma"], np.float64), state["m_gamma"],
                           state["v_gamma"], grads["grad_gamma"], t, lr[sv], wd_focal, b1, b2, eps)
    out["gamma"][step_v] = x[step_v]
    out["m_gamma"][step_v] = m[step_v]
    out["v_gamma"][step_v] = v[step_v]

    for name in ("alpha", "beta"):
        x, m, v = adamw_update(np.asarray(state[name], np.float64), state["m_" + name],
                               state["v_" + name], grads["grad_" + name], t, lr[sr], wd_depth,
                               b1, b2, eps)
        if round_depth:
            out[name][step_r] = x[step_r].astype(np.float32)
        else:
            out[name] = np.asarray(out[name], np.float64)
            out[name][step_r] = x[step_r]
        out["m_" + name][step_r] = m[step_r]
        out["v_" + name][step_r] = v[step_r]
    return out
