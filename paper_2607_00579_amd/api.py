"""Python-level objects over the C-ABI: device buffers from torch, calls into
libepo.so.  No arithmetic of the method happens here.

    plan = EdgePlan.from_problem(problem, device="cuda:0")
    out = plan.cost(poses, lam, grad=True)           # fused forward + adjoint
    plan.pose_step(poses, m, v, out["grad"], lr, step)

`EdgeCostFn` puts the fused adjoint behind torch.autograd.
"""
from __future__ import annotations

import numpy as np
import torch

from . import _lib


def _stream(device=None) -> int:
    return torch.cuda.current_stream(device).cuda_stream


def _require_gpu(device):
    dev = torch.device(device)
    if dev.type != "cuda" or not torch.cuda.is_available():
        raise RuntimeError("the HIP path needs a ROCm GPU (no CPU fallback exists)")
    _lib.load()
    return dev


def build_distance_fields(edge_flat: torch.Tensor, view_offset, width, height):
    """Exact d2 (int32) and DTF (float32) of packed uint8 edge maps on the GPU."""
    dev = edge_flat.device
    n = edge_flat.numel()
    d2 = torch.empty(n, dtype=torch.int32, device=dev)
    dtf = torch.empty(n, dtype=torch.float32, device=dev)
    vo = np.ascontiguousarray(view_offset, np.int64)
    w = np.ascontiguousarray(width, np.int32)
    h = np.ascontiguousarray(height, np.int32)
    _lib.build_distance_fields(edge_flat, vo, w, h, int(w.size), d2, dtf, _stream(dev))
    return d2, dtf


def build_viewgraph(depth_flat: torch.Tensor, width, height, K, view_offset, poses: torch.Tensor,
                    scene_of_view, stride=4, tau=3.0, min_fraction=0.125, z_min=1e-4):
    """Cycle-consistent reprojection test of every pair (i < j) of views of the
    same scene.  Returns the candidates (int32 [n, 2], host), the device
    counts (consistent, total), the validity flags and the directed pair list
    (both directions of every valid pair, host int32 [m, 2])."""
    dev = depth_flat.device
    w = np.ascontiguousarray(width, np.int32)
    h = np.ascontiguousarray(height, np.int32)
    k = np.ascontiguousarray(K, np.float32).reshape(-1, 4)
    vo = np.ascontiguousarray(view_offset, np.int64)[: w.size]
    sov = np.ascontiguousarray(scene_of_view, np.int64)
    n = w.size
    iu, ju = np.triu_indices(n, 1)
    same = sov[iu] == sov[ju]
    cand = np.ascontiguousarray(np.stack([iu[same], ju[same]], axis=1).astype(np.int32))
    nc = cand.shape[0]
    cons = torch.zeros(max(nc, 1), dtype=torch.int32, device=dev)
    tot = torch.zeros(max(nc, 1), dtype=torch.int32, device=dev)
    valid = torch.zeros(max(nc, 1), dtype=torch.uint8, device=dev)
    _lib.build_viewgraph(n, w, h, k, vo, depth_flat.contiguous(), poses.contiguous(), cand, nc,
                         int(stride), float(tau), float(min_fraction), float(z_min), cons, tot,
                         valid, _stream(dev))
    v = valid[:nc].bool().cpu().numpy()
    kept = cand[v]
    directed = np.concatenate([kept, kept[:, ::-1]]).astype(np.int32) if kept.size else \
        np.zeros((0, 2), np.int32)
    return dict(candidates=cand, consistent=cons[:nc], total=tot[:nc], valid=valid[:nc].bool(),
                pairs=np.ascontiguousarray(directed))


class EdgePlan:
    """A problem resident on one GPU: edge records, sampling textures, tile
    schedule and per-iteration buffers, owned by a libepo plan."""

    def __init__(self, width, height, K, scene_of_view, view_offset, edge_flat, depth_flat, pairs,
                 huber_delta=1.0, z_min=1e-4, norm_mode=0, lambda_max=10.0, options=None,
                 device="cuda:0", keep_fields=False):
        dev = _require_gpu(device)
        self.device = dev
        self.width = np.ascontiguousarray(width, np.int32)
        self.height = np.ascontiguousarray(height, np.int32)
        self.K = np.ascontiguousarray(K, np.float32).reshape(-1, 4)
        self.scene_of_view = np.ascontiguousarray(scene_of_view, np.int32)
        self.view_offset = np.ascontiguousarray(view_offset, np.int64)[: self.width.size]
        self.pairs = np.ascontiguousarray(pairs, np.int32).reshape(-1, 2)
        self.n_views = int(self.width.size)
        self.n_pairs = int(self.pairs.shape[0])
        with torch.cuda.device(dev):
            e = edge_flat if torch.is_tensor(edge_flat) else torch.from_numpy(np.asarray(edge_flat))
            z = depth_flat if torch.is_tensor(depth_flat) else torch.from_numpy(np.asarray(depth_flat))
            e = e.to(dev, torch.uint8).contiguous()
            z = z.to(dev, torch.float32).contiguous()
            d2, dtf = build_distance_fields(e, self.view_offset, self.width, self.height)
            self.params = _lib.CostParams(huber_delta, z_min, norm_mode, lambda_max)
            opts = None
            if options is not None:
                opts = _lib.PlanOptions(**{k: int(options.get(k, 0))
                                           for k, _ in _lib.PlanOptions._fields_})
            self.handle = _lib.plan_create(self.n_views, self.width, self.height, self.K,
                                           self.scene_of_view, self.view_offset, e, z, d2,
                                           self.pairs, self.n_pairs, self.params, opts,
                                           _stream(dev))
            self.d2 = d2 if keep_fields else None
            self.dtf = dtf if keep_fields else None
            del e, z
        info = _lib.plan_info(self.handle)
        self.n_scenes = info["n_scenes"]
        self.n_residuals = info["n_residuals"]
        self.n_records = info["n_records"]
        self.scene_of_view_t = torch.from_numpy(self.scene_of_view.astype(np.int64)).to(dev)
        self.scene_of_view_i32 = torch.from_numpy(self.scene_of_view).to(dev)

    @classmethod
    def from_problem(cls, prob, device="cuda:0", **kw):
        return cls(prob.width, prob.height, prob.K, prob.scene_of_view, prob.view_offset,
                   prob.edge_flat, prob.depth_flat, prob.pairs, device=device, **kw)

    def __del__(self):
        h = getattr(self, "handle", None)
        if h:
            try:
                _lib.plan_destroy(h)
            except Exception:
                pass
            self.handle = None

    # ------------------------------------------------------------------
    def info(self):
        return _lib.plan_info(self.handle)

    def view_records(self, v: int) -> np.ndarray:
        return _lib.plan_view_records(self.handle, v)

    def _f64(self, *shape):
        return torch.empty(*shape, dtype=torch.float64, device=self.device)

    def lam_tensor(self, lam):
        if torch.is_tensor(lam):
            return lam.to(self.device, torch.float32).contiguous()
        a = np.broadcast_to(np.asarray(lam, np.float32), (self.n_scenes,)).copy()
        return torch.from_numpy(a).to(self.device)

    def cost(self, poses: torch.Tensor, lam, grad=True, pairs=False, out=None):
        """Fused forward (+ adjoint).  Returns device tensors: loss [S], grad
        [V, 6] (if grad), and per-pair cost / valid count / target gradient
        sums (if pairs)."""
        lam_t = self.lam_tensor(lam)
        o = out if out is not None else {}
        if "loss" not in o:
            o["loss"] = self._f64(self.n_scenes)
        if grad and "grad" not in o:
            o["grad"] = self._f64(self.n_views, 6)
        if pairs:
            o.setdefault("pair_cost", self._f64(self.n_pairs))
            o.setdefault("pair_valid", torch.empty(self.n_pairs, dtype=torch.int32,
                                                   device=self.device))
            o.setdefault("pair_grad", self._f64(self.n_pairs, 6))
        _lib.edge_cost_fwd(self.handle, poses, lam_t, o["loss"], o.get("pair_cost") if pairs else None,
                           o.get("pair_valid") if pairs else None,
                           o.get("pair_grad") if pairs else None, o.get("grad") if grad else None,
                           _stream(self.device))
        return o

    def cost_bwd(self, poses, lam, upstream=None, grad=None):
        lam_t = self.lam_tensor(lam)
        g = grad if grad is not None else self._f64(self.n_views, 6)
        up = None if upstream is None else upstream.to(self.device, torch.float64).contiguous()
        _lib.edge_cost_bwd(self.handle, poses, lam_t, up, g, _stream(self.device))
        return g

    # ------------------------------------------------------------------
    # focal-length and depth refinement
    def record_pixels(self) -> np.ndarray:
        """(n_records, 3) int64 rows (view, x, y) of the edge records in the
        plan's order, the order of alpha, beta and the depth gradients."""
        out = []
        for v in range(self.n_views):
            r = self.view_records(v)
            out.append(np.stack([np.full(r.size, v, np.int64), (r & 0xFFFF).astype(np.int64),
                                 ((r >> np.uint64(16)) & np.uint64(0xFFFF)).astype(np.int64)],
                                axis=1))
        return np.concatenate(out) if out else np.zeros((0, 3), np.int64)

    def set_refinement(self, gamma=None, alpha=None, beta=None):
        """f_v = f0_v (1 + gamma_v) and Z_p = Z0_p alpha_p + beta_p on the
        device (gamma float64 [V]; alpha, beta float32 [n_records]); None
        restores the values the plan was built with."""
        if gamma is not None and gamma.numel() != self.n_views:
            raise ValueError(f"gamma needs {self.n_views} values, got {gamma.numel()}")
        for name, t in (("alpha", alpha), ("beta", beta)):
            if t is not None and t.numel() != self.n_records:
                raise ValueError(f"{name} needs {self.n_records} values, got {t.numel()}")
        g = None if gamma is None else gamma.to(self.device, torch.float64).contiguous()
        a = None if alpha is None else alpha.to(self.device, torch.float32).contiguous()
        b = None if beta is None else beta.to(self.device, torch.float32).contiguous()
        _lib.plan_set_refinement(self.handle, g, a, b, _stream(self.device))

    def refine(self, poses, lam, upstream=None, loss=True, grad=True, focal=True, depth=True):
        """Loss and the gradients of the joint phase: pose twists [V, 6],
        focal scales gamma [V], per-record depth scale alpha and shift beta
        [n_records]."""
        lam_t = self.lam_tensor(lam)
        o = {}
        if loss:
            o["loss"] = self._f64(self.n_scenes)
        if grad:
            o["grad"] = self._f64(self.n_views, 6)
        if focal:
            o["grad_gamma"] = self._f64(self.n_views)
        if depth:
            o["grad_alpha"] = self._f64(self.n_records)
            o["grad_beta"] = self._f64(self.n_records)
        up = None if upstream is None else upstream.to(self.device, torch.float64).contiguous()
        _lib.edge_cost_refine(self.handle, poses, lam_t, up, o.get("loss"), o.get("grad"),
                              o.get("grad_gamma"), o.get("grad_alpha"), o.get("grad_beta"),
                              _stream(self.device))
        return o

    # ------------------------------------------------------------------
    # stochastic viewgraph sub-sampling
    def set_pair_sampling(self, budget: int, seed: int = 0, step=None):
        """Evaluate min(|E_scene|, budget) random image pairs per scene per
        launch (0 = every pair).  `step` is the int32 device counter the draw
        reads in eager launches (a captured iteration uses its own)."""
        if budget and step is None:
            raise ValueError("sub-sampling needs a device step counter")
        if step is not None:
            if step.dtype != torch.int32 or step.device != self.device or step.numel() != 1:
                raise ValueError("step must be one int32 on the plan's device")
            self._sample_step = step               # keep it alive while in use
        _lib.plan_set_pair_sampling(self.handle, int(budget), int(seed) & ((1 << 64) - 1),
                                    step if budget else None, _stream(self.device))

    def sampled_pairs(self) -> torch.Tensor:
        """Directed pairs evaluated by the last cost launch (bool [n_pairs])."""
        out = torch.empty(max(self.n_pairs, 1), dtype=torch.uint8, device=self.device)
        _lib.plan_sampled_pairs(self.handle, out, _stream(self.device))
        return out[: self.n_pairs].bool()

    def joint_state(self):
        """Parameters of the joint phase at their identity values (gamma 0,
        alpha 1, beta 0), zero AdamW moments and step counts (per scene, the
        focal scales' then the depth parameters'), on the plan's device."""
        d, n, V = self.device, self.n_records, self.n_views
        return {"steps": torch.zeros(2 * self.n_scenes, dtype=torch.int32, device=d),
                "gamma": torch.zeros(V, dtype=torch.float64, device=d),
                "alpha": torch.ones(max(n, 1), dtype=torch.float32, device=d)[:n],
                "beta": torch.zeros(max(n, 1), dtype=torch.float32, device=d)[:n],
                "m_gamma": torch.zeros(V, dtype=torch.float64, device=d),
                "v_gamma": torch.zeros(V, dtype=torch.float64, device=d),
                "m_depth": torch.zeros(max(2 * n, 1), dtype=torch.float64, device=d),
                "v_depth": torch.zeros(max(2 * n, 1), dtype=torch.float64, device=d)}

    def joint_step(self, state, grads, lr, phase=None, beta1=0.9, beta2=0.999, eps=1e-8,
                   wd_focal=0.01, wd_depth=0.01):
        """One AdamW step of gamma, alpha, beta (state from joint_state,
        updated in place, its step counts included; grads from refine()),
        then the plan's refinement is set to the new values.  phase: int32
        [n_scenes] device tensor of convergence phases (depth steps only in
        phase 1, nothing in phase 2) or None (every parameter steps)."""
        if not torch.is_tensor(lr):
            lr = torch.full((self.n_scenes,), float(lr), dtype=torch.float64, device=self.device)
        for k in ("grad_gamma", "grad_alpha", "grad_beta"):
            if k not in grads:
                raise ValueError(f"joint_step needs {k} (refine(..., focal=True, depth=True))")
        V, n = self.n_views, self.n_records
        want = {"gamma": (torch.float64, V), "alpha": (torch.float32, n),
                "beta": (torch.float32, n), "m_gamma": (torch.float64, V),
                "v_gamma": (torch.float64, V), "m_depth": (torch.float64, 2 * n),
                "v_depth": (torch.float64, 2 * n)}
        checks = [(f"state[{k!r}]", state.get(k), dt, size) for k, (dt, size) in want.items()]
        checks += [("grad_gamma", grads["grad_gamma"], torch.float64, V),
                   ("grad_alpha", grads["grad_alpha"], torch.float64, n),
                   ("grad_beta", grads["grad_beta"], torch.float64, n),
                   ("lr", lr, torch.float64, self.n_scenes),
                   ("state['steps']", state.get("steps"), torch.int32, 2 * self.n_scenes)]
        if phase is not None:
            checks.append(("phase", phase, torch.int32, self.n_scenes))
        for name, t, dt, size in checks:
            if (not torch.is_tensor(t) or not t.is_cuda
                    or t.device.index != (self.device.index or 0) or t.dtype != dt
                    or t.numel() < size or not t.is_contiguous()):
                raise ValueError(f"{name} must be a contiguous {dt} tensor of at least {size} "
                                 f"values on {self.device}")
        _lib.joint_step(self.handle, state["gamma"], state["alpha"], state["beta"],
                        state["m_gamma"], state["v_gamma"], state["m_depth"], state["v_depth"],
                        grads["grad_gamma"], grads["grad_alpha"], grads["grad_beta"],
                        lr, phase, beta1, beta2,
                        eps, wd_focal, wd_depth, state["steps"], _stream(self.device))

    def _check_joint_state(self, state):
        V, n = self.n_views, self.n_records
        want = {"gamma": (torch.float64, V), "alpha": (torch.float32, n),
                "beta": (torch.float32, n), "m_gamma": (torch.float64, V),
                "v_gamma": (torch.float64, V), "m_depth": (torch.float64, 2 * n),
                "v_depth": (torch.float64, 2 * n), "steps": (torch.int32, 2 * self.n_scenes)}
        for k, (dt, size) in want.items():
            t = state.get(k)
            if (not torch.is_tensor(t) or not t.is_cuda
                    or t.device.index != (self.device.index or 0) or t.dtype != dt
                    or t.numel() < size or not t.is_contiguous()):
                raise ValueError(f"state[{k!r}] must be a contiguous {dt} tensor of at least "
                                 f"{size} values on {self.device}")

    def capture_joint_iteration(self, poses, m, v, step, loss, state, grad=None, lambda0=10.0,
                                lambda1=6.0, anneal_steps=1000, peak_lr=3e-3, warmup=25,
                                total=2000, beta1=0.9, beta2=0.999, eps=1e-8, wd_focal=0.01,
                                wd_depth=0.01, convergence=False, early_exit=False):
        """Capture one iteration of the two-phase loop with focal and depth
        refinement (schedule -> cost with pose, focal and depth gradients ->
        joint AdamW gated by the device phase -> pose step [-> convergence
        test]); replay with launch_iteration().  `state` is joint_state()'s
        dict; its gradient buffers (grad_gamma, grad_alpha, grad_beta) are
        added if missing and rewritten at every replay.  Without the test
        every parameter steps at every replay; with it (reset beforehand with
        convergence_reset) the depth parameters step only in the joint phase
        and nothing after the stop; early_exit as for capture_iteration."""
        self._check_joint_state(state)
        d, n, V = self.device, self.n_records, self.n_views
        for k, size in (("grad_gamma", V), ("grad_alpha", n), ("grad_beta", n)):
            if k not in state:
                state[k] = torch.zeros(max(size, 1), dtype=torch.float64, device=d)
        self._graph_refs = (poses, m, v, step, loss, grad, dict(state))
        mode = (2 if early_exit else 1) if convergence else 0
        _lib.joint_iteration_capture(self.handle, poses, m, v, step, loss, grad, state, wd_focal,
                                     wd_depth, lambda0, lambda1, anneal_steps, peak_lr, warmup,
                                     total, beta1, beta2, eps, mode, _stream(self.device))

    def pose_step(self, poses, m, v, grad, lr, step, fixed_mask=None, beta1=0.9, beta2=0.999,
                  eps=1e-8):
        if not torch.is_tensor(lr):
            lr = torch.full((self.n_scenes,), float(lr), dtype=torch.float64, device=self.device)
        _lib.pose_step(poses, m, v, grad, self.n_views, self.scene_of_view_i32, fixed_mask, lr,
                       beta1, beta2, eps, step, _stream(self.device))

    def autotune(self, poses, lam, iters=3):
        return _lib.plan_autotune(self.handle, poses, self.lam_tensor(lam), iters,
                                  _stream(self.device))

    def set_options(self, **options):
        _lib.plan_set_options(self.handle, options, _stream(self.device))

    def resort(self, poses, step=None, every=1):
        """Re-sort the per-pair record copies (record_order 2) at `poses`:
        all of them, or (with a device step counter) the chunks c with
        c mod every == step mod every, as a captured iteration does."""
        _lib.plan_resort(self.handle, poses, step, every, _stream(self.device))

    def pair_records(self, d: int) -> np.ndarray:
        """The records pair d reads, in its reading order (host copy)."""
        return _lib.plan_pair_records(self.handle, d)

    def capture_iteration(self, poses, m, v, step, loss, grad=None, fixed_mask=None,
                          lambda0=10.0, lambda1=6.0, anneal_steps=1000, peak_lr=3e-3, warmup=25,
                          total=2000, beta1=0.9, beta2=0.999, eps=1e-8, convergence=False,
                          early_exit=False):
        """Capture one iteration (schedule -> cost + adjoint -> reductions ->
        pose step [-> convergence test]), graph_steps times in a row (plan
        option, default 1); replay with launch_iteration(), which runs that
        many steps.  With the test, early_exit=True leaves a stopped scene's
        tiles out of the following iterations (its loss keeps its last
        value)."""
        self._graph_refs = (poses, m, v, step, loss, grad, fixed_mask)   # keep buffers alive
        mode = (2 if early_exit else 1) if convergence else 0
        _lib.iteration_capture(self.handle, poses, m, v, step, loss, grad, fixed_mask, lambda0,
                               lambda1, anneal_steps, peak_lr, warmup, total, beta1, beta2, eps,
                               mode, _stream(self.device))

    def convergence_reset(self, poses, w1=25, eps1=0.5, w2=50, eps2=0.1):
        _lib.convergence_reset(self.handle, poses, _lib.ConvergenceParams(w1, eps1, w2, eps2),
                               _stream(self.device))

    def convergence_update(self, poses, theta95=None, phase=None):
        _lib.convergence_update(self.handle, poses, theta95, phase, _stream(self.device))

    def convergence_query(self):
        return _lib.convergence_query(self.handle, self.n_scenes, _stream(self.device))

    def launch_iteration(self):
        _lib.iteration_launch(self.handle, _stream(self.device))

    def device_status(self) -> int:
        return _lib.get_device_status(self.handle, _stream(self.device))

    def enable_timing(self, on=True):
        _lib.plan_enable_timing(self.handle, on)

    def last_kernel_ms(self) -> float:
        return _lib.plan_last_kernel_ms(self.handle)

    def time_kernel(self, poses, lam, reps=20) -> float:
        """Mean duration (ms) of the fused kernel over `reps` back-to-back
        launches at these poses (HIP events on the current stream)."""
        return _lib.plan_time_kernel(self.handle, poses, self.lam_tensor(lam), reps,
                                     _stream(self.device))


class EdgeCostFn(torch.autograd.Function):
    """loss[s] of every scene as a differentiable function of left twists xi
    (V x 6, float64) at the current poses; the gradient is the derivative at
    xi = 0 and comes from the hand-written adjoint kernel.

    mode "fused": the forward pass runs forward + adjoint together and keeps
    the gradient; mode "recompute": backward calls the adjoint-only entry
    point with the upstream gradient."""

    @staticmethod
    def forward(ctx, xi, plan: EdgePlan, poses, lam, mode="fused"):
        ctx.plan, ctx.mode = plan, mode
        if mode == "fused":
            o = plan.cost(poses, lam, grad=True)
            ctx.save_for_backward(o["grad"])
        else:
            o = plan.cost(poses, lam, grad=False)
            # saved through autograd, so an in-place change of the poses
            # before backward raises instead of differentiating elsewhere
            ctx.save_for_backward(poses)
            ctx.lam = lam.clone() if torch.is_tensor(lam) else lam
        return o["loss"]

    @staticmethod
    def backward(ctx, grad_loss):
        plan = ctx.plan
        if ctx.mode == "fused":
            (g,) = ctx.saved_tensors
            scale = grad_loss.to(torch.float64)[plan.scene_of_view_t].unsqueeze(1)
            return scale * g, None, None, None, None
        (poses,) = ctx.saved_tensors
        g = plan.cost_bwd(poses, ctx.lam, upstream=grad_loss.to(torch.float64).contiguous())
        return g, None, None, None, None


class EdgeRefineFn(torch.autograd.Function):
    """loss[s] of every scene as a differentiable function of the pose twists
    xi (V x 6, derivative at xi = 0), the focal scales gamma [V] and the
    per-record depth scale alpha and shift beta [n_records] (derivatives at
    the given values, which the forward pass installs in the plan).  The
    backward pass is the hand-written adjoint: one refinement call with the
    upstream gradient (recompute), after installing the forward's gamma,
    alpha and beta again (another forward or joint step may have changed the
    plan's refinement in between).  Poses and refinement values are saved
    through autograd, so changing them in place before backward raises."""

    @staticmethod
    def forward(ctx, xi, gamma, alpha, beta, plan: EdgePlan, poses, lam):
        plan.set_refinement(gamma.detach(), alpha.detach(), beta.detach())
        ctx.plan = plan
        ctx.lam = lam.clone() if torch.is_tensor(lam) else lam
        ctx.save_for_backward(poses, gamma, alpha, beta)
        return plan.refine(poses, lam, grad=False, focal=False, depth=False)["loss"]

    @staticmethod
    def backward(ctx, grad_loss):
        poses, gamma, alpha, beta = ctx.saved_tensors
        ctx.plan.set_refinement(gamma.detach(), alpha.detach(), beta.detach())
        o = ctx.plan.refine(poses, ctx.lam, upstream=grad_loss.to(torch.float64).contiguous(),
                            loss=False)
        return (o["grad"], o["grad_gamma"], o["grad_alpha"], o["grad_beta"], None, None, None)


class PoseRefiner:
    """The paper's pose parameterization on a plan: per scene a refiner MLP
    (float32 parameters, bf16 matrix products) and per view a translation
    offset, P = phi(P0 + MLP(P0)) + [0 | delta], trained with AdamW.  All
    state is device tensors; forward / backward / step launch the library's
    kernels on the current stream."""

    def __init__(self, plan: EdgePlan, poses0: torch.Tensor, params: torch.Tensor | None = None,
                 seed: int = 0):
        dev = plan.device
        self.plan = plan
        self.poses0 = poses0.to(dev, torch.float64).contiguous()
        if params is None:
            params = torch.from_numpy(self.init_params(plan.n_scenes, seed))
        if tuple(params.shape) != (plan.n_scenes, _lib.MLP_PARAMS):
            raise ValueError(f"params must be ({plan.n_scenes}, {_lib.MLP_PARAMS})")
        self.params = params.to(dev, torch.float32).contiguous()
        self.m = torch.zeros_like(self.params)
        self.v = torch.zeros_like(self.params)
        self.grad = torch.zeros_like(self.params)
        self.delta = torch.zeros(plan.n_views, 3, dtype=torch.float64, device=dev)
        self.dm = torch.zeros_like(self.delta)
        self.dv = torch.zeros_like(self.delta)
        self.delta_grad = torch.zeros_like(self.delta)
        self.poses = self.poses0.clone()
        _lib.mlp_setup(plan.handle, _stream(dev))

    @staticmethod
    def init_params(n_scenes: int, seed: int = 0) -> np.ndarray:
        """Kaiming-normal weights, zero biases, zero last layer (float32)."""
        rng = np.random.default_rng(seed)
        shapes = [(128, 12), (128, 128), (128, 128), (128, 128), (128, 128), (12, 128)]
        th = np.zeros((n_scenes, _lib.MLP_PARAMS), np.float32)
        for s in range(n_scenes):
            o = 0
            for k, (rows, cols) in enumerate(shapes):
                if k < len(shapes) - 1:
                    th[s, o:o + rows * cols] = rng.normal(0.0, np.sqrt(2.0 / cols), rows * cols)
                o += rows * cols + rows
        return th

    def forward(self):
        _lib.mlp_forward(self.plan.handle, self.params, self.poses0, self.delta, self.poses,
                         _stream(self.plan.device))
        return self.poses

    def backward(self, grad: torch.Tensor):
        _lib.mlp_backward(self.plan.handle, self.params, self.poses0, self.poses,
                          grad.to(torch.float64).contiguous(), self.grad, self.delta_grad,
                          _stream(self.plan.device))
        return self.grad, self.delta_grad

    def capture_iteration(self, step: torch.Tensor, loss: torch.Tensor, grad=None,
                          lambda0=10.0, lambda1=6.0, anneal_steps=1000, peak_lr=3e-3, warmup=25,
                          total=2000, beta1=0.9, beta2=0.999, eps=1e-8, wd_mlp=0.01,
                          wd_delta=0.1, convergence=False, early_exit=False):
        """Capture one iteration of the loop with this parameterization;
        replay it with plan.launch_iteration().  Runs the forward once so
        that `poses` and the stored activations belong to the current
        parameters (and, with the convergence test, resets it there;
        `convergence` is True or (w1, eps1, w2, eps2); early_exit=True
        leaves a stopped scene's tiles out of the following replays)."""
        self.forward()
        if convergence:
            cp = tuple(convergence) if isinstance(convergence, (tuple, list)) else ()
            self.plan.convergence_reset(self.poses, *cp)
        self._graph_refs = (step, loss, grad)
        _lib.mlp_iteration_capture(self.plan.handle, self.params, self.m, self.v, self.grad,
                                   self.delta, self.dm, self.dv, self.delta_grad, self.poses0,
                                   self.poses, step, loss, grad, lambda0, lambda1, anneal_steps,
                                   peak_lr, warmup, total, beta1, beta2, eps, wd_mlp, wd_delta,
                                   (2 if early_exit else 1) if convergence else 0,
                                   _stream(self.plan.device))

    def step(self, lr, step: torch.Tensor, beta1=0.9, beta2=0.999, eps=1e-8, wd_mlp=0.01,
             wd_delta=0.1):
        if not torch.is_tensor(lr):
            lr = torch.full((self.plan.n_scenes,), float(lr), dtype=torch.float64,
                            device=self.plan.device)
        _lib.mlp_step(self.plan.handle, self.params, self.m, self.v, self.grad, self.delta,
                      self.dm, self.dv, self.delta_grad, lr, beta1, beta2, eps, wd_mlp, wd_delta,
                      step, _stream(self.plan.device))
