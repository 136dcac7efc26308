"""ctypes binding of libepo.so: argument marshalling only.

Every function of include/epo.h is exposed under the same name without the
`epo_` prefix.  Pointers are plain integers (device addresses from
torch.Tensor.data_ptr(), host addresses from NumPy arrays); streams are the
integer handle of a HIP stream.  A non-OK status raises EpoError with the
library's message.  There is no fallback: if the library is missing the first
call raises.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

LIB_PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "libepo.so")

OK, ERR_INVALID_ARG, ERR_HIP, ERR_UNSUPPORTED, ERR_NONFINITE = 0, -1, -2, -3, -4
D2_EMPTY = 1 << 30
MAX_SIDE = 16384


class EpoError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"epo status {status}: {msg}")
        self.status = status


class CostParams(C.Structure):
    _fields_ = [("huber_delta", C.c_float), ("z_min", C.c_float), ("norm_mode", C.c_int32),
                ("lambda_max", C.c_float)]


class JointState(C.Structure):
    """epo_joint_state: device addresses of the joint phase's buffers."""
    _fields_ = [("gamma", C.c_void_p), ("alpha", C.c_void_p), ("beta", C.c_void_p),
                ("m_gamma", C.c_void_p), ("v_gamma", C.c_void_p), ("m_depth", C.c_void_p),
                ("v_depth", C.c_void_p), ("steps", C.c_void_p), ("grad_gamma", C.c_void_p),
                ("grad_alpha", C.c_void_p), ("grad_beta", C.c_void_p), ("wd_focal", C.c_double),
                ("wd_depth", C.c_double)]


class PlanOptions(C.Structure):
    _fields_ = [("texture_format", C.c_int32), ("points_per_thread", C.c_int32),
                ("tile_order", C.c_int32), ("persistent", C.c_int32),
                ("record_order", C.c_int32), ("resort_interval", C.c_int32),
                ("graph_steps", C.c_int32)]

    def as_dict(self):
        return {k: int(getattr(self, k)) for k, _ in self._fields_}


P, I32, I64, F32, F64 = C.c_void_p, C.c_int32, C.c_int64, C.c_float, C.c_double

_SIGS = {
    "epo_build_distance_fields": [P, P, P, P, I32, P, P, P],
    "epo_plan_create": [C.POINTER(C.c_void_p), I32, P, P, P, P, P, P, P, P, P, I32,
                        C.POINTER(CostParams), C.POINTER(PlanOptions), P],
    "epo_plan_destroy": [P],
    "epo_plan_info": [P, P, P, P, P, C.POINTER(PlanOptions)],
    "epo_plan_view_records": [P, I32, P, I64, P],
    "epo_edge_cost_fwd": [P, P, P, P, P, P, P, P, P],
    "epo_edge_cost_bwd": [P, P, P, P, P, P],
    "epo_plan_set_refinement": [P, P, P, P, P],
    "epo_plan_set_pair_sampling": [P, I32, C.c_uint64, P, P],
    "epo_build_viewgraph": [I32, P, P, P, P, P, P, P, I32, I32, F64, F64, F64, P, P, P, P],
    "epo_build_viewgraph_noalloc": [I32, P, P, P, P, P, P, P, I32, I32, F64, F64, F64, P, P, P, P],
    "epo_mlp_setup": [P, P],
    "epo_mlp_forward": [P, P, P, P, P, P],
    "epo_mlp_backward": [P, P, P, P, P, P, P, P],
    "epo_mlp_step": [P, P, P, P, P, P, P, P, P, P, F64, F64, F64, F64, F64, P, P],
    "epo_mlp_iteration_capture": [P, P, P, P, P, P, P, P, P, P, P, P, P, P, F32, F32, I32, F64,
                                  I32, I32, F64, F64, F64, F64, F64, I32, P],
    "epo_plan_sampled_pairs": [P, P, P],
    "epo_edge_cost_refine": [P, P, P, P, P, P, P, P, P, P],
    "epo_pose_step": [P, P, P, P, I32, P, P, P, F64, F64, F64, P, P],
    "epo_joint_step": [P, P, P, P, P, P, P, P, P, P, P, P, P, F64, F64, F64, F64, F64, P, P],
    "epo_schedule": [P, I32, F32, F32, I32, F64, I32, I32, P, P, P],
    "epo_iteration_capture": [P, P, P, P, P, P, P, P, F32, F32, I32, F64, I32, I32, F64, F64,
                              F64, I32, P],
    "epo_joint_iteration_capture": [P, P, P, P, P, P, P, C.POINTER(JointState), F32, F32, I32,
                                    F64, I32, I32, F64, F64, F64, I32, P],
    "epo_convergence_reset": [P, P, P, P],
    "epo_convergence_update": [P, P, P, P, P],
    "epo_convergence_query": [P, P, P, P, P, P],
    "epo_iteration_launch": [P, P],
    "epo_plan_autotune": [P, P, P, I32, C.POINTER(PlanOptions), P],
    "epo_plan_set_options": [P, C.POINTER(PlanOptions), P],
    "epo_plan_resort": [P, P, P, I32, P],
    "epo_plan_pair_records": [P, I32, P, I64, P],
    "epo_get_device_status": [P, P, P],
    "epo_plan_enable_timing": [P, I32],
    "epo_plan_last_kernel_ms": [P, P],
    "epo_plan_time_kernel": [P, P, P, I32, P, P],
}
EXPORTS = sorted(list(_SIGS) + ["epo_last_error", "epo_version"])

_lib = None


def load():
    """Load libepo.so (built in-tree by paper_2607_00579_amd.build)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is missing: build it with "
                           "`python -m paper_2607_00579_amd.build` (there is no fallback path)")
    lib = C.CDLL(LIB_PATH)
    for name, args in _SIGS.items():
        fn = getattr(lib, name)
        fn.argtypes = args
        fn.restype = C.c_int
    lib.epo_last_error.restype = C.c_char_p
    lib.epo_last_error.argtypes = []
    lib.epo_version.restype = C.c_char_p
    lib.epo_version.argtypes = []
    _lib = lib
    return lib


def _check(status: int):
    if status != OK:
        raise EpoError(status, load().epo_last_error().decode())


def _ptr(x):
    """Address of a NumPy array, a torch tensor, an int, or None."""
    if x is None:
        return None
    if isinstance(x, int):
        return x
    if isinstance(x, np.ndarray):
        assert x.flags["C_CONTIGUOUS"], "host arrays must be C-contiguous"
        return x.ctypes.data
    if hasattr(x, "data_ptr"):
        assert x.is_contiguous(), "tensors must be contiguous"
        return x.data_ptr()
    raise TypeError(f"cannot take the address of {type(x)}")


def version() -> str:
    return load().epo_version().decode()


def build_distance_fields(edge_maps, view_offset, width, height, n_views, d2_out, dtf_out, stream):
    _check(load().epo_build_distance_fields(_ptr(edge_maps), _ptr(view_offset), _ptr(width),
                                            _ptr(height), n_views, _ptr(d2_out), _ptr(dtf_out),
                                            stream))


def plan_create(n_views, width, height, K, scene_of_view, view_offset, edge_maps, depth, d2, pairs,
                n_pairs, params: CostParams | None, options: PlanOptions | None, stream):
    h = C.c_void_p()
    _check(load().epo_plan_create(C.byref(h), n_views, _ptr(width), _ptr(height), _ptr(K),
                                  _ptr(scene_of_view), _ptr(view_offset), _ptr(edge_maps),
                                  _ptr(depth), _ptr(d2), _ptr(pairs), n_pairs,
                                  C.byref(params) if params is not None else None,
                                  C.byref(options) if options is not None else None, stream))
    return h.value


def plan_destroy(plan):
    _check(load().epo_plan_destroy(plan))


def plan_info(plan):
    s, r, n, t = C.c_int32(), C.c_int64(), C.c_int64(), C.c_int64()
    o = PlanOptions()
    _check(load().epo_plan_info(plan, C.byref(s), C.byref(r), C.byref(n), C.byref(t), C.byref(o)))
    return dict(n_scenes=s.value, n_records=r.value, n_residuals=n.value, n_tiles=t.value,
                options=o.as_dict())


def plan_view_records(plan, v):
    cnt = C.c_int64()
    _check(load().epo_plan_view_records(plan, v, None, 0, C.byref(cnt)))
    out = np.empty(max(cnt.value, 1), np.uint64)
    _check(load().epo_plan_view_records(plan, v, out.ctypes.data, out.size, C.byref(cnt)))
    return out[:cnt.value]


def edge_cost_fwd(plan, poses, lam, loss, pair_cost, pair_valid, pair_grad, grad, stream):
    _check(load().epo_edge_cost_fwd(plan, _ptr(poses), _ptr(lam), _ptr(loss), _ptr(pair_cost),
                                    _ptr(pair_valid), _ptr(pair_grad), _ptr(grad), stream))


def edge_cost_bwd(plan, poses, lam, upstream, grad, stream):
    _check(load().epo_edge_cost_bwd(plan, _ptr(poses), _ptr(lam), _ptr(upstream), _ptr(grad),
                                    stream))


def plan_set_refinement(plan, gamma, alpha, beta, stream):
    _check(load().epo_plan_set_refinement(plan, _ptr(gamma), _ptr(alpha), _ptr(beta), stream))


def build_viewgraph(n_views, width, height, K, view_offset, depth, poses, candidates,
                    n_candidates, stride, tau, min_fraction, z_min, consistent, total, valid,
                    stream):
    _check(load().epo_build_viewgraph(n_views, _ptr(width), _ptr(height), _ptr(K),
                                      _ptr(view_offset), _ptr(depth), _ptr(poses),
                                      _ptr(candidates), n_candidates, stride, tau, min_fraction,
                                      z_min, _ptr(consistent), _ptr(total), _ptr(valid), stream))


def build_viewgraph_noalloc(n_views, width, height, K, view_offset, depth, poses, candidates,
                            n_candidates, stride, tau, min_fraction, z_min, consistent, total,
                            valid, stream):
    _check(load().epo_build_viewgraph_noalloc(n_views, _ptr(width), _ptr(height), _ptr(K),
                                              _ptr(view_offset), _ptr(depth), _ptr(poses),
                                              _ptr(candidates), n_candidates, stride, tau,
                                              min_fraction, z_min, _ptr(consistent), _ptr(total),
                                              _ptr(valid), stream))


MLP_PARAMS = 69260


def mlp_setup(plan, stream):
    _check(load().epo_mlp_setup(plan, stream))


def mlp_forward(plan, params, poses0, delta, poses, stream):
    _check(load().epo_mlp_forward(plan, _ptr(params), _ptr(poses0), _ptr(delta), _ptr(poses),
                                  stream))


def mlp_backward(plan, params, poses0, poses, grad, param_grad, delta_grad, stream):
    _check(load().epo_mlp_backward(plan, _ptr(params), _ptr(poses0), _ptr(poses), _ptr(grad),
                                   _ptr(param_grad), _ptr(delta_grad), stream))


def mlp_step(plan, params, m, v, param_grad, delta, dm, dv, delta_grad, lr, beta1, beta2, eps,
             wd_mlp, wd_delta, step, stream):
    _check(load().epo_mlp_step(plan, _ptr(params), _ptr(m), _ptr(v), _ptr(param_grad),
                               _ptr(delta), _ptr(dm), _ptr(dv), _ptr(delta_grad), _ptr(lr),
                               beta1, beta2, eps, wd_mlp, wd_delta, _ptr(step), stream))


def mlp_iteration_capture(plan, params, m, v, param_grad, delta, dm, dv, delta_grad, poses0,
                          poses, step, loss, grad, lambda0, lambda1, anneal_steps, peak_lr, warmup,
                          total, beta1, beta2, eps, wd_mlp, wd_delta, with_convergence, stream):
    _check(load().epo_mlp_iteration_capture(
        plan, _ptr(params), _ptr(m), _ptr(v), _ptr(param_grad), _ptr(delta), _ptr(dm), _ptr(dv),
        _ptr(delta_grad), _ptr(poses0), _ptr(poses), _ptr(step), _ptr(loss), _ptr(grad), lambda0,
        lambda1, anneal_steps, peak_lr, warmup, total, beta1, beta2, eps, wd_mlp, wd_delta,
        int(with_convergence), stream))


def plan_set_pair_sampling(plan, budget, seed, step, stream):
    _check(load().epo_plan_set_pair_sampling(plan, budget, seed, _ptr(step), stream))


def plan_sampled_pairs(plan, selected, stream):
    _check(load().epo_plan_sampled_pairs(plan, _ptr(selected), stream))


def edge_cost_refine(plan, poses, lam, upstream, loss, grad, grad_gamma, grad_alpha, grad_beta,
                     stream):
    _check(load().epo_edge_cost_refine(plan, _ptr(poses), _ptr(lam), _ptr(upstream), _ptr(loss),
                                       _ptr(grad), _ptr(grad_gamma), _ptr(grad_alpha),
                                       _ptr(grad_beta), stream))


def joint_step(plan, gamma, alpha, beta, m_gamma, v_gamma, m_depth, v_depth, grad_gamma,
               grad_alpha, grad_beta, lr, phase, beta1, beta2, eps, wd_focal, wd_depth, steps,
               stream):
    _check(load().epo_joint_step(plan, _ptr(gamma), _ptr(alpha), _ptr(beta), _ptr(m_gamma),
                                 _ptr(v_gamma), _ptr(m_depth), _ptr(v_depth), _ptr(grad_gamma),
                                 _ptr(grad_alpha), _ptr(grad_beta), _ptr(lr), _ptr(phase), beta1,
                                 beta2, eps, wd_focal, wd_depth, _ptr(steps), stream))


def pose_step(poses, m, v, grad, n_views, scene_of_view, fixed_mask, lr, beta1, beta2, eps, step,
              stream):
    _check(load().epo_pose_step(_ptr(poses), _ptr(m), _ptr(v), _ptr(grad), n_views,
                                _ptr(scene_of_view), _ptr(fixed_mask), _ptr(lr), beta1, beta2,
                                eps, _ptr(step), stream))


def schedule(step, n_scenes, lambda0, lambda1, anneal_steps, peak_lr, warmup, total, lambda_out,
             lr_out, stream):
    _check(load().epo_schedule(_ptr(step), n_scenes, lambda0, lambda1, anneal_steps, peak_lr,
                               warmup, total, _ptr(lambda_out), _ptr(lr_out), stream))


def iteration_capture(plan, poses, m, v, step, loss, grad, fixed_mask, lambda0, lambda1,
                      anneal_steps, peak_lr, warmup, total, beta1, beta2, eps, with_convergence,
                      stream):
    _check(load().epo_iteration_capture(plan, _ptr(poses), _ptr(m), _ptr(v), _ptr(step),
                                        _ptr(loss), _ptr(grad), _ptr(fixed_mask), lambda0,
                                        lambda1, anneal_steps, peak_lr, warmup, total, beta1,
                                        beta2, eps, int(with_convergence), stream))


def joint_iteration_capture(plan, poses, m, v, step, loss, grad, joint: dict, wd_focal, wd_depth,
                            lambda0, lambda1, anneal_steps, peak_lr, warmup, total, beta1, beta2,
                            eps, with_convergence, stream):
    js = JointState(*[_ptr(joint.get(k)) for k in ("gamma", "alpha", "beta", "m_gamma",
                                                   "v_gamma", "m_depth", "v_depth", "steps",
                                                   "grad_gamma", "grad_alpha", "grad_beta")],
                    float(wd_focal), float(wd_depth))
    _check(load().epo_joint_iteration_capture(plan, _ptr(poses), _ptr(m), _ptr(v), _ptr(step),
                                              _ptr(loss), _ptr(grad), C.byref(js), lambda0,
                                              lambda1, anneal_steps, peak_lr, warmup, total,
                                              beta1, beta2, eps, int(with_convergence), stream))


class ConvergenceParams(C.Structure):
    _fields_ = [("w1", C.c_int32), ("eps1", C.c_float), ("w2", C.c_int32), ("eps2", C.c_float)]


def convergence_reset(plan, poses, params: ConvergenceParams | None, stream):
    _check(load().epo_convergence_reset(plan, _ptr(poses),
                                        C.byref(params) if params is not None else None, stream))


def convergence_update(plan, poses, theta95, phase, stream):
    _check(load().epo_convergence_update(plan, _ptr(poses), _ptr(theta95), _ptr(phase), stream))


def convergence_query(plan, n_scenes, stream):
    phase = np.zeros(n_scenes, np.int32)
    theta = np.zeros(n_scenes, np.float64)
    sw = np.zeros((n_scenes, 2), np.int32)
    steps = np.zeros(n_scenes, np.int32)
    _check(load().epo_convergence_query(plan, phase.ctypes.data, theta.ctypes.data,
                                        sw.ctypes.data, steps.ctypes.data, stream))
    return dict(phase=phase, theta_last=theta, switch_steps=sw, steps=steps)


def iteration_launch(plan, stream):
    _check(load().epo_iteration_launch(plan, stream))


def plan_autotune(plan, poses, lam, iters, stream):
    o = PlanOptions()
    _check(load().epo_plan_autotune(plan, _ptr(poses), _ptr(lam), iters, C.byref(o), stream))
    return o.as_dict()


def plan_set_options(plan, options: dict, stream):
    o = PlanOptions(**{k: int(options.get(k, 0)) for k, _ in PlanOptions._fields_})
    _check(load().epo_plan_set_options(plan, C.byref(o), stream))


def plan_resort(plan, poses, step, every, stream):
    _check(load().epo_plan_resort(plan, _ptr(poses), _ptr(step) if step is not None else None,
                                  every, stream))


def plan_pair_records(plan, d):
    n = C.c_int64()
    _check(load().epo_plan_pair_records(plan, d, None, 0, C.byref(n)))
    out = np.zeros(n.value, np.uint64)
    _check(load().epo_plan_pair_records(plan, d, _ptr(out), n.value, C.byref(n)))
    return out


def get_device_status(plan, stream) -> int:
    f = C.c_int32()
    _check(load().epo_get_device_status(plan, C.byref(f), stream))
    return f.value


def plan_enable_timing(plan, enable: bool):
    _check(load().epo_plan_enable_timing(plan, 1 if enable else 0))


def plan_time_kernel(plan, poses, lam, reps: int, stream) -> float:
    ms = C.c_float(0.0)
    _check(load().epo_plan_time_kernel(plan, _ptr(poses), _ptr(lam), int(reps), C.byref(ms),
                                       stream))
    return float(ms.value)


def plan_last_kernel_ms(plan) -> float:
    ms = C.c_float()
    _check(load().epo_plan_last_kernel_ms(plan, C.byref(ms)))
    return ms.value
