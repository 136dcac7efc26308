"""Oracle: edge reprojection cost, per-direction means, loss and the analytic
left-twist pose gradient, in float64.

Test infrastructure only (see the package header).

What is computed (paper Sec. 3 "Method", Eqs. pi, L, L_ij, d_ij; supplementary
Alg. 3 and Sec. A1.1), for every directed pair d = (i -> j) and every edge
pixel p = (u, v) of view i:

  1. lift (UnprojectEdgesTo3D):   X_i = P_i^-1 K_i^-1 [u, v, 1]^T Z_i(u, v)
     i.e. camera point X_c = Z ((u - cx_i)/fx_i, (v - cy_i)/fy_i, 1) and world
     point X_w = R_i^T (X_c - t_i);
  2. target camera:               X' = R_j X_w + t_j;
  3. pinhole projection:          u' = fx_j X'_x / X'_z + cx_j,
                                  v' = fy_j X'_y / X'_z + cy_j;
  4. validity: X'_z > z_min and 0 <= u' < W_j - 1 and 0 <= v' < H_j - 1, so
     that all four bilinear taps lie inside the target image;
  5. bilinear sample of DTF_j at (u', v') from the cell x0 = floor(u'),
     y0 = floor(v') (integer pixel centres);
  6. clamp d^ = min(d, lambda) and Huber H(d^) = d^2/2 if d^ <= delta, else
     delta (d^ - delta/2);
  7. per direction: S_d = sum of H over valid residuals, n_d = number of valid
     residuals, L_d = S_d / n_d (0 if n_d = 0)  -- Alg. 3's mean over valid;
     norm_mode 1 divides by |E_i| instead (the form of Eq. L_ij);
  8. per scene: L = (2 / |D|) sum_d L_d over its |D| directed pairs, which for a
     pair list holding both directions of every undirected pair equals the
     paper's (1/|E|) sum over pairs of (L_ij + L_ji).

The gradient is with respect to left twists xi_v = (rho, omega) of every pose,
P_v <- Exp(xi_v) P_v, at xi = 0, with n_d held fixed (it is piecewise
constant).  For one valid residual with r = dH/dd^ (0 when d >= lambda) and the
bilinear slopes (dD/du', dD/dv'), the chain rule gives

  a   = dH/dX' = r [dD/du' fx_j / z, dD/dv' fy_j / z,
                    -(dD/du' fx_j X'_x + dD/dv' fy_j X'_y) / z^2]
  target pose j: dX' = rho_j + omega_j x X'           -> g_j = (a, X' x a)
  source pose i: dX_w = -R_i^T (rho_i + omega_i x X_c) -> with b = R_i R_j^T a,
                                                          g_i = -(b, X_c x b)

Readings where the paper is silent (kept identical on the GPU side): Huber
delta = 1 px, invalid projections dropped, bounds as in step 4, pixel centres
at integers, the right/lower cell at exact integers, clamp derivative 0 at
d = lambda, empty edge maps give d2 = 2^30.

Pins: exact-zero fixtures (shifted edges, dilated projections), a single-column
distance field (closed form), global rigid invariance, the gauge identity,
power-of-two scale invariance, frozen-branch central finite differences, an
independent plain torch-autograd evaluation in float64.
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np

from . import edt as _edt


@dataclass(frozen=True)
class CostParams:
    huber_delta: float = 1.0
    z_min: float = 1e-4
    norm_mode: int = 0          # 0: sum rho / sum valid (Alg. 3); 1: sum rho / |E_i|


def huber(dhat: np.ndarray, delta: float) -> np.ndarray:
    return np.where(dhat <= delta, 0.5 * dhat * dhat, delta * (dhat - 0.5 * delta))


def edge_pixels(edge: np.ndarray, depth: np.ndarray):
    """Edge pixels (u = column, v = row) in row-major order and their depth."""
    ys, xs = np.nonzero(edge)
    return xs.astype(np.float64), ys.astype(np.float64), depth[ys, xs].astype(np.float64)


class OracleProblem:
    """Per-view edge pixels and float64 distance fields of a packed problem.

    `prob` is any object with the packed arrays of the input generator
    (width, height, K, scene_of_view, edge_map(v), depth_map(v), pairs,
    scene_of_pair)."""

    def __init__(self, prob, d2=None, views=None):
        self.prob = prob
        V = prob.n_views
        self.V = V
        self.W = prob.width.astype(np.int64)
        self.H = prob.height.astype(np.int64)
        self.K = prob.K.astype(np.float64)          # f32 values, upcast
        self.scene_of_view = prob.scene_of_view.astype(np.int64)
        self.pairs = prob.pairs.astype(np.int64)
        self.scene_of_pair = prob.scene_of_pair.astype(np.int64)
        self.n_scenes = int(self.scene_of_view.max()) + 1 if V else 0
        self.pairs_per_scene = np.bincount(self.scene_of_pair, minlength=self.n_scenes)
        need = set(range(V)) if views is None else set(views)
        self.pts = {}
        self.D = {}
        self.d2 = {}
        for v in need:
            self.pts[v] = edge_pixels(prob.edge_map(v), prob.depth_map(v))
            if d2 is not None and v in d2:
                dv = np.asarray(d2[v], np.int64)
            else:
                dv = _edt.edt_separable(prob.edge_map(v))
            self.d2[v] = dv
            self.D[v] = np.sqrt(dv.astype(np.float64))

    # ------------------------------------------------------------------
    def direction(self, d: int, poses: np.ndarray, lam: float, params: CostParams,
                  frozen=None, per_residual=False, K=None, depth=None):
        """Residual sums of directed pair d.  Returns a dict with S, n, G_tgt,
        G_src (6-vectors, left twists of the target and source pose), the
        focal-scale sums F_tgt, F_src, the per-pixel depth derivatives dZ of the
        source edge pixels, and the discrete decisions taken (for frozen-branch
        finite differences).  `K` (V x 4) and `depth` ({view: Z array}) replace
        the problem's intrinsics / edge depths when given."""
        i, j = int(self.pairs[d, 0]), int(self.pairs[d, 1])
        u, v, Z = self.pts[i]
        if depth is not None and i in depth:
            Z = depth[i]
        Kx = self.K if K is None else K
        fxi, fyi, cxi, cyi = Kx[i]
        fxj, fyj, cxj, cyj = Kx[j]
        Wj, Hj = int(self.W[j]), int(self.H[j])
        Dj = self.D[j]
        Ri, ti = poses[i][:, :3], poses[i][:, 3]
        Rj, tj = poses[j][:, :3], poses[j][:, 3]
        delta = params.huber_delta

        # 1. lift to the camera frame of i, then to the world frame
        Xc = np.stack([(u - cxi) / fxi * Z, (v - cyi) / fyi * Z, Z], axis=1)
        Xw = (Xc - ti) @ Ri                        # rows: R_i^T (X_c - t_i)
        # 2. into the camera frame of j
        Xp = Xw @ Rj.T + tj
        z = Xp[:, 2]
        if frozen is None:
            front = z > params.z_min
            zs = np.where(front, z, 1.0)
            up = fxj * Xp[:, 0] / zs + cxj
            vp = fyj * Xp[:, 1] / zs + cyj
            valid = front & (up >= 0) & (up < Wj - 1) & (vp >= 0) & (vp < Hj - 1)
            x0 = np.where(valid, np.floor(up), 0).astype(np.int64)
            y0 = np.where(valid, np.floor(vp), 0).astype(np.int64)
        else:
            valid, x0, y0 = frozen["valid"], frozen["x0"], frozen["y0"]
            zs = np.where(valid, z, 1.0)
            up = fxj * Xp[:, 0] / zs + cxj
            vp = fyj * Xp[:, 1] / zs + cyj
        # 5. bilinear sample of DTF_j
        al = np.where(valid, up - x0, 0.0)
        be = np.where(valid, vp - y0, 0.0)
        D00 = Dj[y0, x0]
        D10 = Dj[y0, np.minimum(x0 + 1, Wj - 1)]
        D01 = Dj[np.minimum(y0 + 1, Hj - 1), x0]
        D11 = Dj[np.minimum(y0 + 1, Hj - 1), np.minimum(x0 + 1, Wj - 1)]
        Dval = (1 - be) * ((1 - al) * D00 + al * D10) + be * ((1 - al) * D01 + al * D11)
        dDdu = (1 - be) * (D10 - D00) + be * (D11 - D01)
        dDdv = (1 - al) * (D01 - D00) + al * (D11 - D10)
        # 6. clamp and Huber
        if frozen is None:
            unclamped = Dval < lam
            dhat = np.minimum(Dval, lam)
            quad = dhat <= delta
        else:
            unclamped, quad = frozen["unclamped"], frozen["quad"]
            dhat = np.where(unclamped, Dval, lam)
        rho = np.where(quad, 0.5 * dhat * dhat, delta * (dhat - 0.5 * delta))
        drho = np.where(unclamped, np.where(quad, dhat, delta), 0.0)
        rho = np.where(valid, rho, 0.0)
        drho = np.where(valid, drho, 0.0)
        # gradient with respect to X'
        zz = zs
        a = np.stack([drho * dDdu * fxj / zz,
                      drho * dDdv * fyj / zz,
                      -drho * (dDdu * fxj * Xp[:, 0] + dDdv * fyj * Xp[:, 1]) / (zz * zz)], axis=1)
        g_tgt = np.concatenate([a, np.cross(Xp, a)], axis=1)
        b = a @ (Rj @ Ri.T)                        # rows: R_i R_j^T a
        g_src = -np.concatenate([b, np.cross(Xc, b)], axis=1)
        # depth of the source pixel: X_c = Z r, so dX'/dZ = R_j R_i^T r, and
        # dH/dZ = a . (R_j R_i^T r) = b . r
        r = np.stack([(u - cxi) / fxi, (v - cyi) / fyi, np.ones_like(u)], axis=1)
        dZ = np.einsum("nk,nk->n", b, r)
        # focal scales f = f0 (1 + gamma), derivatives at gamma = 0:
        #   target: u' = f_j X'_x / z + cx_j, so du'/dgamma_j = f_j X'_x / z
        #   source: dX_c/dgamma_i = -Z ((u - cx)/f_i, (v - cy)/f_i, 0)
        F_tgt = drho * (dDdu * fxj * Xp[:, 0] + dDdv * fyj * Xp[:, 1]) / zz
        dXc = np.stack([-Z * (u - cxi) / fxi, -Z * (v - cyi) / fyi, np.zeros_like(u)], axis=1)
        F_src = np.einsum("nk,nk->n", b, dXc)
        out = dict(S=float(rho.sum()), n=int(valid.sum()), n_src=int(u.size),
                   G_tgt=g_tgt.sum(axis=0), G_src=g_src.sum(axis=0),
                   F_tgt=float(F_tgt.sum()), F_src=float(F_src.sum()), dZ=dZ,
                   decisions=dict(valid=valid, x0=x0, y0=y0, unclamped=unclamped, quad=quad))
        if per_residual:
            out.update(rho=rho, valid=valid, up=up, vp=vp, Dval=Dval, g_tgt=g_tgt, g_src=g_src)
        return out

    # ------------------------------------------------------------------
    def weights(self, S, n, n_src, params: CostParams, selected=None):
        """Per-pair mean L_d and weight w_d = (2/|D_scene|) / denominator.
        With a boolean mask `selected` over directed pairs (a sub-sampled
        step), |D_scene| counts the selected pairs of the scene and an
        unselected pair has scale and weight 0."""
        den = n if params.norm_mode == 0 else n_src
        den = np.asarray(den, np.float64)
        L = np.where(den > 0, np.asarray(S) / np.where(den > 0, den, 1.0), 0.0)
        if selected is None:
            count = self.pairs_per_scene
            scale = 2.0 / count[self.scene_of_pair].astype(np.float64)
        else:
            selected = np.asarray(selected, bool)
            count = np.bincount(self.scene_of_pair[selected], minlength=self.n_scenes)
            scale = np.where(selected, 2.0 / np.maximum(count[self.scene_of_pair], 1), 0.0)
        w = np.where(den > 0, scale / np.where(den > 0, den, 1.0), 0.0)
        return L, w, scale

    def evaluate(self, poses: np.ndarray, lam, params: CostParams = CostParams(),
                 frozen=None, pair_ids=None, K=None, depth=None, selected=None,
                 pair_results=None):
        """Loss per scene, per-pair S, n, L_d, G, the gradient per view, the
        focal-scale gradient per view (grad_focal) and the depth gradient of
        every edge pixel (grad_depth: {view: array in edge-pixel order}).
        `selected` (boolean mask over directed pairs) evaluates one
        sub-sampled step: only those pairs, each scene's loss the mean over
        its selected pairs.  `pair_results` ({d: the sums direction() returns
        for pair d at these arguments}) supplies the per-pair sums computed
        elsewhere (worker processes); they are combined here in the same
        order, so the result is the same bits (without grad_depth unless the
        results carry dZ)."""
        lam = np.broadcast_to(np.asarray(lam, np.float64), (self.n_scenes,))
        D = self.pairs.shape[0]
        ids = range(D) if pair_ids is None else pair_ids
        if selected is not None:
            ids = [d for d in ids if selected[d]]
        S = np.zeros(D)
        n = np.zeros(D, np.int64)
        n_src = np.zeros(D, np.int64)
        G_tgt = np.zeros((D, 6))
        G_src = np.zeros((D, 6))
        F_tgt = np.zeros(D)
        F_src = np.zeros(D)
        dZ = {}
        decisions = {}
        for d in ids:
            s = int(self.scene_of_pair[d])
            if pair_results is not None:
                r = pair_results[d]
            else:
                r = self.direction(d, poses, float(lam[s]), params,
                                   frozen=None if frozen is None else frozen[d], K=K, depth=depth)
            S[d], n[d], n_src[d] = r["S"], r["n"], r["n_src"]
            G_tgt[d], G_src[d] = r["G_tgt"], r["G_src"]
            F_tgt[d], F_src[d] = r["F_tgt"], r["F_src"]
            dZ[d] = r.get("dZ")
            decisions[d] = r.get("decisions")
        L, w, scale = self.weights(S, n, n_src, params, selected)
        loss = np.zeros(self.n_scenes)
        grad = np.zeros((self.V, 6))
        grad_focal = np.zeros(self.V)
        grad_depth = {}
        for d in ids:
            s = int(self.scene_of_pair[d])
            i, j = int(self.pairs[d, 0]), int(self.pairs[d, 1])
            loss[s] += scale[d] * L[d]
            grad[j] += w[d] * G_tgt[d]
            grad[i] += w[d] * G_src[d]
            grad_focal[j] += w[d] * F_tgt[d]
            grad_focal[i] += w[d] * F_src[d]
            if dZ[d] is None:
                continue
            if i not in grad_depth:
                grad_depth[i] = np.zeros(self.pts[i][0].size)
            grad_depth[i] += w[d] * dZ[d]
        return dict(loss=loss, grad=grad, grad_focal=grad_focal, grad_depth=grad_depth, S=S, n=n,
                    L=L, w=w, G_tgt=G_tgt, G_src=G_src, F_tgt=F_tgt, F_src=F_src,
                    decisions=decisions)


def fd_gradient(op: OracleProblem, poses: np.ndarray, lam, params: CostParams = CostParams(),
                h: float = 1e-6, views=None, frozen_branches=True):
    """Central differences of the scene loss in every left-twist component.

    With frozen_branches the discrete decisions of the base point (valid mask,
    n_d, bilinear cell, clamp and Huber branch) are kept, so the function is
    smooth and is exactly the one the analytic gradient differentiates."""
    from .geometry import left_update
    base = op.evaluate(poses, lam, params)
    frozen = base["decisions"] if frozen_branches else None
    views = range(op.V) if views is None else views
    g = np.zeros((op.V, 6))
    for v in views:
        s = int(op.scene_of_view[v])
        for k in range(6):
            xi = np.zeros(6)
            xi[k] = h
            pp = poses.copy()
            pm = poses.copy()
            pp[v] = left_update(poses[v], xi)
            pm[v] = left_update(poses[v], -xi)
            if frozen_branches:
                # n_d stays that of the base point
                lp = _frozen_loss(op, pp, lam, params, frozen, base)
                lm = _frozen_loss(op, pm, lam, params, frozen, base)
            else:
                lp = op.evaluate(pp, lam, params)["loss"]
                lm = op.evaluate(pm, lam, params)["loss"]
            g[v, k] = (lp[s] - lm[s]) / (2.0 * h)
    return g


def fd_focal(op: OracleProblem, poses: np.ndarray, lam, params: CostParams = CostParams(),
             h: float = 1e-6, views=None):
    """Frozen-branch central differences of the scene loss in each view's
    focal scale gamma (fx and fy multiplied by 1 + gamma)."""
    base = op.evaluate(poses, lam, params)
    frozen = base["decisions"]
    views = range(op.V) if views is None else views
    g = np.zeros(op.V)
    for v in views:
        s = int(op.scene_of_view[v])
        Kp, Km = op.K.copy(), op.K.copy()
        Kp[v, :2] *= 1.0 + h
        Km[v, :2] *= 1.0 - h
        lp = _frozen_loss(op, poses, lam, params, frozen, base, K=Kp)
        lm = _frozen_loss(op, poses, lam, params, frozen, base, K=Km)
        g[v] = (lp[s] - lm[s]) / (2.0 * h)
    return g


def fd_depth(op: OracleProblem, poses: np.ndarray, lam, view: int, pixels,
             params: CostParams = CostParams(), h: float = 1e-6):
    """Frozen-branch central differences of the scene loss in the depth of the
    given edge pixels (indices into the view's edge-pixel order)."""
    base = op.evaluate(poses, lam, params)
    frozen = base["decisions"]
    s = int(op.scene_of_view[view])
    Z = op.pts[view][2]
    out = []
    for p in pixels:
        Zp, Zm = Z.copy(), Z.copy()
        step = h * Z[p]
        Zp[p] += step
        Zm[p] -= step
        lp = _frozen_loss(op, poses, lam, params, frozen, base, depth={view: Zp})
        lm = _frozen_loss(op, poses, lam, params, frozen, base, depth={view: Zm})
        out.append((lp[s] - lm[s]) / (2.0 * step))
    return np.array(out)


def _frozen_loss(op, poses, lam, params, frozen, base, K=None, depth=None):
    r = op.evaluate(poses, lam, params, frozen=frozen, K=K, depth=depth)
    # denominators fixed at the base point
    L, w, scale = op.weights(r["S"], base["n"], op_n_src(op, base), params)
    loss = np.zeros(op.n_scenes)
    for d in range(op.pairs.shape[0]):
        loss[int(op.scene_of_pair[d])] += scale[d] * L[d]
    return loss


def op_n_src(op, base):
    return np.array([op.pts[int(i)][0].size for i in op.pairs[:, 0]], np.int64)
