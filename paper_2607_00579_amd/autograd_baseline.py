"""Plain torch-autograd form of the edge-alignment cost (comparison baseline).

This is the "reference PyTorch" form the paper's fused kernels replace
(supplementary Sec. A1.2: each kernel expands into a chain of ordinary tensor
operations, each with its own launch, autograd node and intermediate tensor).
It is used for two things only:
  * the throughput baseline the fused HIP adjoint is compared against
    (float32, on the GPU, same inputs, same per-iteration work);
  * an independent gradient in float64 (autograd of the forward, on the CPU)
    against which the analytic gradients are checked.
The HIP path never calls it.

The forward follows Alg. 3's batched step: pairs are split into batches of
whole directed pairs; each batch gathers the source edge points X_i (lifted
once, pose-free, in the source camera frame), the relative pose and K_j of its
target, projects, bilinearly samples DTF_j from a flat tensor, clamps and
applies the Huber loss, and reduces the per-direction mean over valid
residuals.  Poses enter as T_v = Exp(xi_v) T_v^0 with torch.linalg.matrix_exp,
so autograd gives the left-twist gradient at xi = 0.  Because the loss is a sum
over pairs, each batch is back-propagated on its own and the twist gradient
accumulates, which bounds memory by the batch size.
"""
from __future__ import annotations

import numpy as np
import torch


class TorchEdgeCost:
    def __init__(self, width, height, K, scene_of_view, pairs, scene_of_pair, pts_u, pts_v, pts_z,
                 pts_offset, dtf_flat, dtf_offset, device="cpu", dtype=torch.float32,
                 huber_delta=1.0, z_min=1e-4, norm_mode=0, batch_residuals=1 << 24):
        """All array arguments are NumPy or torch tensors:
        width/height (V,), K (V, 4) fx fy cx cy, scene_of_view (V,), pairs (D, 2),
        scene_of_pair (D,), edge points of all views concatenated (u, v, Z) with
        pts_offset (V + 1,), distance fields concatenated with dtf_offset (V,)."""
        dev = torch.device(device)
        self.device, self.dtype = dev, dtype
        t = lambda a, dt: torch.as_tensor(np.asarray(a) if not torch.is_tensor(a) else a,
                                          device=dev).to(dt)
        self.W = t(width, torch.int64)
        self.H = t(height, torch.int64)
        self.K = t(K, torch.float64).to(dtype)
        self.scene_of_view = t(scene_of_view, torch.int64)
        self.pairs = t(pairs, torch.int64)
        self.scene_of_pair = t(scene_of_pair, torch.int64)
        self.pts_offset = np.asarray(pts_offset if not torch.is_tensor(pts_offset)
                                     else pts_offset.cpu().numpy(), np.int64)
        self.D = t(dtf_flat, dtype)
        self.D_off = t(dtf_offset, torch.int64)
        self.n_views = int(self.W.shape[0])
        self.n_scenes = int(self.scene_of_view.max().item()) + 1
        self.delta, self.z_min, self.norm_mode = float(huber_delta), float(z_min), int(norm_mode)
        per_scene = torch.bincount(self.scene_of_pair, minlength=self.n_scenes)
        self.pair_scale = (2.0 / per_scene[self.scene_of_pair].to(torch.float64)).to(dtype)
        # lift once: camera-frame points of every edge pixel (pose independent)
        u, v, z = t(pts_u, torch.float64), t(pts_v, torch.float64), t(pts_z, torch.float64)
        view_of_pt = torch.repeat_interleave(
            torch.arange(self.n_views, device=dev),
            torch.as_tensor(np.diff(self.pts_offset), device=dev))
        Kp = t(K, torch.float64)[view_of_pt]
        self.Xc = torch.stack([(u - Kp[:, 2]) / Kp[:, 0] * z, (v - Kp[:, 3]) / Kp[:, 1] * z, z],
                              dim=1).to(dtype)
        # batches of whole pairs
        n_src = np.diff(self.pts_offset)[self.pairs[:, 0].cpu().numpy()]
        self.n_src = n_src
        self.batches = []
        a, acc = 0, 0
        for d in range(len(n_src)):
            if acc > 0 and acc + n_src[d] > batch_residuals:
                self.batches.append((a, d))
                a, acc = d, 0
            acc += int(n_src[d])
        if len(n_src):
            self.batches.append((a, len(n_src)))

    # ------------------------------------------------------------------
    def poses_from_twists(self, xi, poses0):
        A = torch.zeros(xi.shape[0], 4, 4, dtype=xi.dtype, device=xi.device)
        w = xi[:, 3:]
        A[:, 0, 1], A[:, 0, 2], A[:, 1, 2] = -w[:, 2], w[:, 1], -w[:, 0]
        A[:, 1, 0], A[:, 2, 0], A[:, 2, 1] = w[:, 2], -w[:, 1], w[:, 0]
        A[:, :3, 3] = xi[:, :3]
        T0 = torch.zeros(xi.shape[0], 4, 4, dtype=xi.dtype, device=xi.device)
        T0[:, :3, :] = poses0
        T0[:, 3, 3] = 1.0
        return torch.linalg.matrix_exp(A) @ T0

    def _batch(self, T, lam, a, b, want_pair=False):
        dev, dt = self.device, self.dtype
        pi, pj = self.pairs[a:b, 0], self.pairs[a:b, 1]
        Ri, ti = T[pi, :3, :3], T[pi, :3, 3]
        Rj, tj = T[pj, :3, :3], T[pj, :3, 3]
        Rji = (Rj @ Ri.transpose(1, 2).contiguous()).to(dt)
        tji = (tj - (Rji.to(T.dtype) @ ti.unsqueeze(-1)).squeeze(-1)).to(dt)
        cnt = torch.as_tensor(self.n_src[a:b], device=dev)
        res_pair = torch.repeat_interleave(torch.arange(b - a, device=dev), cnt)
        starts = torch.as_tensor(self.pts_offset[self.pairs[a:b, 0].cpu().numpy()], device=dev)
        first = torch.cumsum(cnt, 0) - cnt
        res_pt = starts[res_pair] + (torch.arange(res_pair.shape[0], device=dev) - first[res_pair])
        Xc = self.Xc[res_pt]
        Xp = (Rji[res_pair] @ Xc.unsqueeze(-1)).squeeze(-1) + tji[res_pair]
        Kj = self.K[pj][res_pair]
        Wj = self.W[pj][res_pair]
        Hj = self.H[pj][res_pair]
        z = Xp[:, 2]
        front = z > self.z_min
        zs = torch.where(front, z, torch.ones_like(z))
        up = Kj[:, 0] * Xp[:, 0] / zs + Kj[:, 2]
        vp = Kj[:, 1] * Xp[:, 1] / zs + Kj[:, 3]
        valid = front & (up >= 0) & (up < (Wj - 1).to(dt)) & (vp >= 0) & (vp < (Hj - 1).to(dt))
        x0 = torch.where(valid, torch.floor(up.detach()), torch.zeros_like(up)).to(torch.int64)
        y0 = torch.where(valid, torch.floor(vp.detach()), torch.zeros_like(vp)).to(torch.int64)
        al = torch.where(valid, up - x0.to(dt), torch.zeros_like(up))
        be = torch.where(valid, vp - y0.to(dt), torch.zeros_like(vp))
        base = self.D_off[pj][res_pair] + y0 * Wj + x0
        step_x = valid.to(torch.int64)
        step_y = Wj * valid.to(torch.int64)
        D00 = self.D[base]
        D10 = self.D[base + step_x]
        D01 = self.D[base + step_y]
        D11 = self.D[base + step_y + step_x]
        Dv = (1 - be) * ((1 - al) * D00 + al * D10) + be * ((1 - al) * D01 + al * D11)
        lam_r = lam[self.scene_of_pair[a:b]][res_pair]
        dhat = torch.where(Dv < lam_r, Dv, lam_r)
        rho = torch.where(dhat <= self.delta, 0.5 * dhat * dhat,
                          self.delta * (dhat - 0.5 * self.delta))
        rho = torch.where(valid, rho, torch.zeros_like(rho))
        S = torch.zeros(b - a, dtype=dt, device=dev).index_add(0, res_pair, rho)
        n = torch.zeros(b - a, dtype=torch.int64, device=dev).index_add(0, res_pair,
                                                                         valid.to(torch.int64))
        den = n if self.norm_mode == 0 else cnt
        L = torch.where(den > 0, S / den.clamp(min=1).to(dt), torch.zeros_like(S))
        return S, n, L

    def loss_and_grad(self, poses0, lam, want_pairs=False):
        """Loss per scene and d(loss)/d(xi) per view at xi = 0 (autograd)."""
        dev = self.device
        poses0 = torch.as_tensor(np.asarray(poses0) if not torch.is_tensor(poses0) else poses0,
                                 device=dev, dtype=torch.float64)
        lam = torch.as_tensor(np.broadcast_to(np.asarray(lam, np.float64), (self.n_scenes,)).copy()
                              if not torch.is_tensor(lam) else lam, device=dev).to(self.dtype)
        xi = torch.zeros(self.n_views, 6, dtype=torch.float64, device=dev, requires_grad=True)
        loss = torch.zeros(self.n_scenes, dtype=self.dtype, device=dev)
        pair_S, pair_n = [], []
        for (a, b) in self.batches:
            T = self.poses_from_twists(xi, poses0)
            S, n, L = self._batch(T, lam, a, b)
            contrib = self.pair_scale[a:b] * L
            per_scene = torch.zeros(self.n_scenes, dtype=self.dtype, device=dev).index_add(
                0, self.scene_of_pair[a:b], contrib)
            per_scene.sum().backward()
            loss += per_scene.detach()
            if want_pairs:
                pair_S.append(S.detach())
                pair_n.append(n)
        out = dict(loss=loss, grad=xi.grad.detach() if xi.grad is not None
                   else torch.zeros_like(xi))
        if want_pairs:
            out["S"] = torch.cat(pair_S)
            out["n"] = torch.cat(pair_n)
        return out
