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

The forward follows Alg. 3's batched step: the directed pairs are split into
batches; CreateBatchedInputs becomes padded tensors [pairs, points] of the
source edge points (lifted once, pose-free, in the source camera frame) with a
mask, and per-pair relative poses, intrinsics and distance-field offsets
broadcast along the points.  Projection, bilinear sampling of DTF_j from a
flat tensor, clamp and Huber are elementwise; the per-direction mean over valid
residuals is a sum over the points axis.  Poses enter as
T_v = (I + hat(xi_v)) T_v^0, whose derivative at xi = 0 is that of the SE(3)
exponential, so autograd returns the left-twist gradient.  Every product is
written out elementwise (no batched matmul).  Because the loss is a sum over
pairs, each batch is back-propagated on its own and the twist gradient
accumulates, which bounds memory by the batch size.
"""
from __future__ import annotations

import numpy as np
import torch

_MAX_ELEMS = 1 << 28          # keep every padded tensor well below 2 GiB


class TorchEdgeCost:
    def __init__(self, width, height, K, scene_of_view, pairs, scene_of_pair, pts_u, pts_v, pts_z,
                 pts_offset, dtf_flat, dtf_offset, device="cpu", dtype=torch.float32,
                 huber_delta=1.0, z_min=1e-4, norm_mode=0, batch_residuals=1 << 24):
        """width/height (V,), K (V, 4) fx fy cx cy, scene_of_view (V,), pairs
        (D, 2) directed (source, target), scene_of_pair (D,), edge points of all
        views concatenated (u, v, Z) with pts_offset (V + 1,), distance fields
        concatenated (flat) with dtf_offset (V,) element offsets."""
        dev = torch.device(device)
        self.device, self.dtype = dev, dtype
        asnp = lambda a: a.detach().cpu().numpy() if torch.is_tensor(a) else np.asarray(a)
        self.W_np = asnp(width).astype(np.int64)
        self.H_np = asnp(height).astype(np.int64)
        K64 = asnp(K).astype(np.float64).reshape(-1, 4)
        self.K = torch.as_tensor(K64, device=dev).to(dtype)
        self.scene_of_view = asnp(scene_of_view).astype(np.int64)
        self.pairs_np = asnp(pairs).astype(np.int64).reshape(-1, 2)
        self.scene_of_pair_np = asnp(scene_of_pair).astype(np.int64)
        self.pts_offset = asnp(pts_offset).astype(np.int64)
        self.D = dtf_flat.to(dev, dtype) if torch.is_tensor(dtf_flat) else \
            torch.as_tensor(np.asarray(dtf_flat), device=dev).to(dtype)
        self.D_off = asnp(dtf_offset).astype(np.int64)
        self.n_views = int(self.W_np.shape[0])
        self.n_scenes = int(self.scene_of_view.max()) + 1
        self.delta, self.z_min, self.norm_mode = float(huber_delta), float(z_min), int(norm_mode)
        per_scene = np.bincount(self.scene_of_pair_np, minlength=self.n_scenes)
        self.pair_scale = torch.as_tensor(2.0 / per_scene[self.scene_of_pair_np],
                                          device=dev).to(dtype)
        # lift once: camera-frame points of every edge pixel (pose independent)
        u = torch.as_tensor(asnp(pts_u).astype(np.float64), device=dev)
        v = torch.as_tensor(asnp(pts_v).astype(np.float64), device=dev)
        z = torch.as_tensor(asnp(pts_z).astype(np.float64), device=dev)
        counts = np.diff(self.pts_offset)
        view_of_pt = torch.repeat_interleave(torch.arange(self.n_views, device=dev),
                                             torch.as_tensor(counts, device=dev))
        Kp = torch.as_tensor(K64, device=dev)[view_of_pt]
        self.Xc = torch.stack([(u - Kp[:, 2]) / Kp[:, 0] * z, (v - Kp[:, 3]) / Kp[:, 1] * z, z],
                              dim=0).to(dtype)                       # (3, P)
        # the unlifted points, for the form with focal and depth leaves
        self.uvz = torch.stack([u, v, z], dim=0).to(dtype)
        self.K0 = torch.as_tensor(K64, device=dev).to(dtype)
        self.view_of_pt = view_of_pt
        # batches of whole pairs, padded to the longest source in the batch
        self.n_src = counts[self.pairs_np[:, 0]]
        self.batches = []
        a = 0
        D = len(self.n_src)
        while a < D:
            b, nmax = a, 0
            while b < D:
                nm = max(nmax, int(self.n_src[b]))
                if b > a and (nm * (b + 1 - a) > batch_residuals or nm * (b + 1 - a) > _MAX_ELEMS):
                    break
                nmax, b = nm, b + 1
            self.batches.append((a, b, nmax))
            a = b
        self._idx_cache = {}

    # ------------------------------------------------------------------
    def _indices(self, a, b, nmax):
        key = (a, b)
        if key not in self._idx_cache:
            dev = self.device
            starts = torch.as_tensor(self.pts_offset[self.pairs_np[a:b, 0]], device=dev)
            cnt = torch.as_tensor(self.n_src[a:b], device=dev)
            col = torch.arange(max(nmax, 1), device=dev)
            mask = col[None, :] < cnt[:, None]
            idx = torch.where(mask, starts[:, None] + col[None, :], torch.zeros_like(mask,
                                                                                   dtype=torch.int64))
            self._idx_cache = {key: (idx, mask, cnt)}     # one batch cached at a time
        return self._idx_cache[key]

    @staticmethod
    def _poses(xi, poses0):
        """(I + hat(xi)) [R | t] for every view: R (V,3,3) and t (V,3)."""
        rho, w = xi[:, :3], xi[:, 3:]
        R0, t0 = poses0[:, :, :3], poses0[:, :, 3]
        z = torch.zeros_like(w[:, 0])
        Wh = torch.stack([torch.stack([z, -w[:, 2], w[:, 1]], 1),
                          torch.stack([w[:, 2], z, -w[:, 0]], 1),
                          torch.stack([-w[:, 1], w[:, 0], z], 1)], 1)          # (V,3,3)
        R = R0 + (Wh[:, :, :, None] * R0[:, None, :, :]).sum(2)
        t = t0 + (Wh * t0[:, None, :]).sum(2) + rho
        return R, t

    def _batch(self, R, t, lam, a, b, nmax, gamma=None, dz=None):
        dt = self.dtype
        dev = self.device
        pi = torch.as_tensor(self.pairs_np[a:b, 0], device=dev)
        pj = torch.as_tensor(self.pairs_np[a:b, 1], device=dev)
        Ri, ti, Rj, tj = R[pi], t[pi], R[pj], t[pj]
        # R_ji = R_j R_i^T, t_ji = t_j - R_ji t_i (written out elementwise)
        Rji = (Rj[:, :, None, :] * Ri[:, None, :, :]).sum(-1)
        tji = tj - (Rji * ti[:, None, :]).sum(-1)
        Rji, tji = Rji.to(dt), tji.to(dt)
        idx, mask, cnt = self._indices(a, b, nmax)
        if gamma is None:
            X, Y, Z = self.Xc[0][idx], self.Xc[1][idx], self.Xc[2][idx]   # (b, n)
            Kj = self.K[pj]
        else:
            # lift inside the graph: f = f0 (1 + gamma), Z = Z0 + dz
            Ks = self.K0 * torch.stack([1 + gamma, 1 + gamma, torch.ones_like(gamma),
                                        torch.ones_like(gamma)], dim=1).to(dt)
            Ki = Ks[pi]
            Kj = Ks[pj]
            Z = (self.uvz[2] + dz.to(dt))[idx]
            X = (self.uvz[0][idx] - Ki[:, 2:3]) / Ki[:, 0:1] * Z
            Y = (self.uvz[1][idx] - Ki[:, 3:4]) / Ki[:, 1:2] * Z
        xp = Rji[:, 0, 0:1] * X + Rji[:, 0, 1:2] * Y + Rji[:, 0, 2:3] * Z + tji[:, 0:1]
        yp = Rji[:, 1, 0:1] * X + Rji[:, 1, 1:2] * Y + Rji[:, 1, 2:3] * Z + tji[:, 1:2]
        zp = Rji[:, 2, 0:1] * X + Rji[:, 2, 1:2] * Y + Rji[:, 2, 2:3] * Z + tji[:, 2:3]
        Wj = torch.as_tensor(self.W_np[self.pairs_np[a:b, 1]], device=dev)[:, None]
        Hj = torch.as_tensor(self.H_np[self.pairs_np[a:b, 1]], device=dev)[:, None]
        front = zp > self.z_min
        zs = torch.where(front, zp, torch.ones_like(zp))
        up = Kj[:, 0:1] * xp / zs + Kj[:, 2:3]
        vp = Kj[:, 1:2] * yp / zs + Kj[:, 3:4]
        valid = mask & front & (up >= 0) & (up < (Wj - 1).to(dt)) & (vp >= 0) & (vp < (Hj - 1).to(dt))
        x0 = torch.where(valid, torch.floor(up.detach()), torch.zeros_like(up)).to(torch.int64)
        y0 = torch.where(valid, torch.floor(vp.detach()), torch.zeros_like(vp)).to(torch.int64)
        al = torch.where(valid, up - x0.to(dt), torch.zeros_like(up))
        be = torch.where(valid, vp - y0.to(dt), torch.zeros_like(vp))
        off = torch.as_tensor(self.D_off[self.pairs_np[a:b, 1]], device=dev)[:, None]
        base = off + y0 * Wj + x0
        sx = valid.to(torch.int64)
        sy = Wj * sx
        D00 = self.D[base]
        D10 = self.D[base + sx]
        D01 = self.D[base + sy]
        D11 = self.D[base + sy + sx]
        Dv = (1 - be) * ((1 - al) * D00 + al * D10) + be * ((1 - al) * D01 + al * D11)
        lam_p = lam[torch.as_tensor(self.scene_of_pair_np[a:b], device=dev)][:, None]
        dhat = torch.where(Dv < lam_p, Dv, lam_p)
        rho = torch.where(dhat <= self.delta, 0.5 * dhat * dhat,
                          self.delta * (dhat - 0.5 * self.delta))
        rho = torch.where(valid, rho, torch.zeros_like(rho))
        S = rho.sum(1)
        n = valid.sum(1)
        den = n if self.norm_mode == 0 else cnt
        L = torch.where(den > 0, S / den.clamp(min=1).to(dt), torch.zeros_like(S))
        return S, n, L

    def loss_and_grad(self, poses0, lam, want_pairs=False, intrinsics_depth=False):
        """Loss per scene and d(loss)/d(xi) per view at xi = 0 (autograd).
        With intrinsics_depth, also d(loss)/d(gamma) per view (focal scale,
        f = f0 (1 + gamma)) and d(loss)/dZ per edge point, at gamma = 0 and
        the given depths."""
        dev = self.device
        poses0 = torch.as_tensor(np.asarray(poses0) if not torch.is_tensor(poses0) else poses0,
                                 device=dev, dtype=torch.float64)
        if torch.is_tensor(lam):
            lam_t = lam.to(dev, self.dtype)
        else:
            lam_t = torch.as_tensor(np.broadcast_to(np.asarray(lam, np.float64),
                                                    (self.n_scenes,)).copy(), device=dev).to(self.dtype)
        xi = torch.zeros(self.n_views, 6, dtype=torch.float64, device=dev, requires_grad=True)
        gamma = dz = None
        if intrinsics_depth:
            gamma = torch.zeros(self.n_views, dtype=torch.float64, device=dev, requires_grad=True)
            dz = torch.zeros(self.uvz.shape[1], dtype=torch.float64, device=dev,
                             requires_grad=True)
        loss = torch.zeros(self.n_scenes, dtype=self.dtype, device=dev)
        sop = torch.as_tensor(self.scene_of_pair_np, device=dev)
        pair_S, pair_n = [], []
        for (a, b, nmax) in self.batches:
            R, t = self._poses(xi, poses0)
            S, n, L = self._batch(R, t, lam_t, a, b, nmax, gamma, dz)
            contrib = self.pair_scale[a:b] * L
            per_scene = torch.zeros(self.n_scenes, dtype=self.dtype, device=dev).index_add(
                0, sop[a:b], contrib)
            per_scene.sum().backward()
            loss += per_scene.detach()
            if want_pairs:
                pair_S.append(S.detach())
                pair_n.append(n)
        out = dict(loss=loss, grad=xi.grad.detach() if xi.grad is not None
                   else torch.zeros_like(xi))
        if intrinsics_depth:
            out["grad_focal"] = gamma.grad.detach() if gamma.grad is not None else \
                torch.zeros_like(gamma)
            out["grad_depth"] = dz.grad.detach() if dz.grad is not None else torch.zeros_like(dz)
        if want_pairs:
            out["S"] = torch.cat(pair_S)
            out["n"] = torch.cat(pair_n)
        return out
