// Float64 reductions above the fused kernel's tile partials, all in a fixed
// order (bitwise reproducible whatever the launch schedule):
//   per pair   S_d, n_d, G_d = sum of its tiles in tile order; L_d = S_d / n_d
//              (Alg. 3 mean over valid residuals; |E_i| in norm mode 1) and the
//              pose weight w_d = (2 / |D_scene|) / n_d, where |D_scene| counts
//              the pairs evaluated in this step (all of them, or the
//              sub-sampled ones; a skipped pair has scale and weight 0)
//   per pose   g_v = sum over pairs into v of w_d G_d
//                  - sum over pairs out of v of w_d Ad(T_ji)^T G_d
//              (the source pose sees the target's left perturbation moved
//              through the relative pose: T_ji Exp(-xi_i) = Exp(-Ad(T_ji) xi_i) T_ji)
//   per scene  loss = sum over its pairs of (2 / |D_scene|) L_d (Eqs. L, L_ij);
//              in an iteration that skips stopped scenes, theirs is kept
//   refinement (Sec. 3 Camera Refinement): with the per-pair focal sums F_t
//              (target) and F_s (source), each f dH/df,
//              dL/dgamma_v = (sum over pairs into v of w_d F_t
//                             + sum over pairs out of v of w_d F_s) / (1 + gamma_v)
//              (f = f0 (1 + gamma), so dL/dgamma = f0 dL/df = f dL/df / (1 + gamma))
// One thread per pair; one wave64 per pose (lanes stride over the pose's pairs,
// then a butterfly); one workgroup per scene (threads stride over its pairs,
// then wave butterflies and an LDS step).
#include "epo_internal.h"

namespace epo {
#include "pose_update.h"
namespace {

__device__ inline double wave_sum64(double x) {
#pragma unroll
    for (int m = 32; m >= 1; m >>= 1) x += __shfl_xor(x, m, 64);
    return x;
}

// pair d's sums (one thread)
__device__ inline void reduce_pair(
    int d, const Partial* __restrict__ partials, const double* __restrict__ ext_partials,
    const PairStatic* __restrict__ ps, const double* __restrict__ pair_scale, int32_t norm_mode,
    double* __restrict__ pair_sum, double* __restrict__ pair_w, double* __restrict__ pair_ext,
    double* __restrict__ pair_cost, int32_t* __restrict__ pair_valid,
    double* __restrict__ pair_grad, int32_t* __restrict__ status) {
    const PairStatic st = ps[d];
    const double scale = pair_scale[d];
    // a pair skipped by the sub-sampling of this step ran no tiles: all zero
    const int n_tiles = scale != 0.0 ? st.n_tiles : 0;
    // the tiles' partials four at a time (their loads in flight together),
    // added one after another in tile order as before
    double s[8] = {0, 0, 0, 0, 0, 0, 0, 0};
    const Partial* pp = partials + st.first_tile;
    int k = 0;
    for (; k + 4 <= n_tiles; k += 4) {
        Partial pt[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) pt[u] = pp[k + u];
#pragma unroll
        for (int u = 0; u < 4; ++u)
#pragma unroll
            for (int c = 0; c < 8; ++c) s[c] += pt[u].v[c];
    }
    for (; k < n_tiles; ++k) {
        const Partial pt = pp[k];
#pragma unroll
        for (int c = 0; c < 8; ++c) s[c] += pt.v[c];
    }
    if (ext_partials) {
        double ft = 0.0, fs = 0.0;
        const double* ep = ext_partials + 2 * (int64_t)st.first_tile;
        int q = 0;
        for (; q + 4 <= n_tiles; q += 4) {
            double e[8];
#pragma unroll
            for (int u = 0; u < 8; ++u) e[u] = ep[2 * q + u];
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                ft += e[2 * u];
                fs += e[2 * u + 1];
            }
        }
        for (; q < n_tiles; ++q) {
            ft += ep[2 * q];
            fs += ep[2 * q + 1];
        }
        if (!isfinite(ft) || !isfinite(fs)) atomicOr(status, 1);
        pair_ext[2 * d] = ft;
        pair_ext[2 * d + 1] = fs;
    }
    const double den = norm_mode == 0 ? s[1] : (double)st.n_src;
    const double L = den > 0 ? s[0] / den : 0.0;
    const double w = den > 0 ? scale / den : 0.0;
    if (!isfinite(s[0]) || !isfinite(s[2]) || !isfinite(s[5])) atomicOr(status, 1);
#pragma unroll
    for (int c = 0; c < 8; ++c) pair_sum[8 * d + c] = s[c];
    pair_w[d] = w;
    if (pair_cost) pair_cost[d] = L;
    if (pair_valid) pair_valid[d] = (int32_t)s[1];
    if (pair_grad) {
#pragma unroll
        for (int c = 0; c < 6; ++c) pair_grad[6 * d + c] = s[2 + c];
    }
}

__global__ __launch_bounds__(256) void reduce_pairs_kernel(
    const Partial* __restrict__ partials, const double* __restrict__ ext_partials,
    const PairStatic* __restrict__ ps, const double* __restrict__ pair_scale, int32_t D,
    int32_t norm_mode, double* __restrict__ pair_sum, double* __restrict__ pair_w,
    double* __restrict__ pair_ext, double* __restrict__ pair_cost,
    int32_t* __restrict__ pair_valid, double* __restrict__ pair_grad,
    int32_t* __restrict__ status) {
    const int d = blockIdx.x * blockDim.x + threadIdx.x;
    if (d >= D) return;
    reduce_pair(d, partials, ext_partials, ps, pair_scale, norm_mode, pair_sum, pair_w, pair_ext,
                pair_cost, pair_valid, pair_grad, status);
}

// pose v's gradient (one wave: lanes stride over the pose's pairs, then a
// butterfly)
__device__ inline void reduce_view(
    int v, int lane, const double* __restrict__ pair_sum, const double* __restrict__ pair_w,
    const double* __restrict__ rel, const int32_t* __restrict__ in_ptr,
    const int32_t* __restrict__ in_idx, const int32_t* __restrict__ out_ptr,
    const int32_t* __restrict__ out_idx, const int32_t* __restrict__ scene_of_view,
    const double* __restrict__ upstream, double* __restrict__ grad,
    const double* __restrict__ pair_ext, const double* __restrict__ gamma,
    double* __restrict__ grad_gamma) {
    double g[6] = {0, 0, 0, 0, 0, 0};
    double gf = 0.0;
    for (int k = in_ptr[v] + lane; k < in_ptr[v + 1]; k += 64) {
        const int d = in_idx[k];
        const double w = pair_w[d];
#pragma unroll
        for (int c = 0; c < 6; ++c) g[c] += w * pair_sum[8 * d + 2 + c];
        if (grad_gamma) gf += w * pair_ext[2 * d];
    }
    //   Ad^T (G_r, G_w) = (R^T G_r, R^T (G_w - t x G_r))
    for (int k = out_ptr[v] + lane; k < out_ptr[v + 1]; k += 64) {
        const int d = out_idx[k];
        const double w = pair_w[d];
        const double* R = rel + 12 * d;
        const double* t = R + 9;
        const double* G = pair_sum + 8 * d + 2;
        const double c0 = G[3] - (t[1] * G[2] - t[2] * G[1]);
        const double c1 = G[4] - (t[2] * G[0] - t[0] * G[2]);
        const double c2 = G[5] - (t[0] * G[1] - t[1] * G[0]);
#pragma unroll
        for (int r = 0; r < 3; ++r) {
            g[r] -= w * (R[0 + r] * G[0] + R[3 + r] * G[1] + R[6 + r] * G[2]);
            g[3 + r] -= w * (R[0 + r] * c0 + R[3 + r] * c1 + R[6 + r] * c2);
        }
        if (grad_gamma) gf += w * pair_ext[2 * d + 1];
    }
    const double up = upstream ? upstream[scene_of_view[v]] : 1.0;
    if (grad) {
#pragma unroll
        for (int c = 0; c < 6; ++c) g[c] = wave_sum64(g[c]);
        if (lane < 6) {
            double x = g[0];
#pragma unroll
            for (int c = 1; c < 6; ++c) x = lane == c ? g[c] : x;
            grad[6 * v + lane] = up * x;
        }
    }
    if (grad_gamma) {
        gf = wave_sum64(gf);
        if (lane == 0) grad_gamma[v] = up * gf / (1.0 + gamma[v]);
    }
}

// one wave per pose
__global__ __launch_bounds__(256) void reduce_views_kernel(
    const double* __restrict__ pair_sum, const double* __restrict__ pair_w,
    const double* __restrict__ rel, const int32_t* __restrict__ in_ptr,
    const int32_t* __restrict__ in_idx, const int32_t* __restrict__ out_ptr,
    const int32_t* __restrict__ out_idx, const int32_t* __restrict__ scene_of_view, int32_t V,
    const double* __restrict__ upstream, double* __restrict__ grad,
    const double* __restrict__ pair_ext, const double* __restrict__ gamma,
    double* __restrict__ grad_gamma) {
    const int v = blockIdx.x * 4 + (threadIdx.x >> 6);
    const int lane = threadIdx.x & 63;
    if (v >= V) return;                       // whole wave leaves together
    reduce_view(v, lane, pair_sum, pair_w, rel, in_ptr, in_idx, out_ptr, out_idx, scene_of_view,
                upstream, grad, pair_ext, gamma, grad_gamma);
}

// scene s's loss (a 256-thread workgroup: threads stride over its pairs, then
// wave butterflies and an LDS step; `part` holds 4 doubles of LDS)
__device__ inline void reduce_scene(int s, const double* __restrict__ pair_sum,
                                    const PairStatic* __restrict__ ps,
                                    const double* __restrict__ pair_scale,
                                    const int32_t* __restrict__ scene_ptr,
                                    const int32_t* __restrict__ scene_pairs, int32_t norm_mode,
                                    double* __restrict__ loss, double* part) {
    // the thread's pairs k = first + tid, + blockDim, ... four at a time (the
    // index and value loads of the four in flight together), added in order
    double L = 0.0;
    const int k1 = scene_ptr[s + 1], step = blockDim.x;
    int k = scene_ptr[s] + threadIdx.x;
    for (; k + 3 * step < k1; k += 4 * step) {
        int d[4];
        double den[4], num[4], sc[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) d[u] = scene_pairs[k + u * step];
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            den[u] = norm_mode == 0 ? pair_sum[8 * d[u] + 1] : (double)ps[d[u]].n_src;
            num[u] = pair_sum[8 * d[u] + 0];
            sc[u] = pair_scale[d[u]];
        }
#pragma unroll
        for (int u = 0; u < 4; ++u)
            if (den[u] > 0) L += sc[u] * (num[u] / den[u]);
    }
    for (; k < k1; k += step) {
        const int d = scene_pairs[k];
        const PairStatic st = ps[d];
        const double den = norm_mode == 0 ? pair_sum[8 * d + 1] : (double)st.n_src;
        if (den > 0) L += pair_scale[d] * (pair_sum[8 * d + 0] / den);
    }
    L = wave_sum64(L);
    if ((threadIdx.x & 63) == 0) part[threadIdx.x >> 6] = L;
    __syncthreads();
    if (threadIdx.x == 0) loss[s] = (part[0] + part[1]) + (part[2] + part[3]);
}

// one workgroup per scene; a scene the convergence test has stopped (phase
// 2, when phases are given) evaluated nothing and keeps its last loss
__global__ __launch_bounds__(256) void reduce_scenes_kernel(
    const double* __restrict__ pair_sum, const PairStatic* __restrict__ ps,
    const double* __restrict__ pair_scale, const int32_t* __restrict__ scene_ptr,
    const int32_t* __restrict__ scene_pairs, int32_t norm_mode, const int32_t* __restrict__ phase,
    double* __restrict__ loss) {
    __shared__ double part[4];
    const int s = blockIdx.x;
    if (phase && phase[s] == 2) return;
    reduce_scene(s, pair_sum, ps, pair_scale, scene_ptr, scene_pairs, norm_mode, loss, part);
}

// The whole step after the fused kernel, for plans whose launches rather than
// their work set the step time: pair sums, pose gradients, pose update, scene
// losses and the step count in one 256-thread workgroup, phases separated by
// barriers (the waves of one workgroup share a CU and its L1, so the sums a
// phase stores are visible to the next).  Every pair, pose and scene goes
// through the same device code as in the separate kernels, in the same
// order: the same bits.
__global__ __launch_bounds__(256) void step_epilogue_kernel(
    const Partial* __restrict__ partials, const PairStatic* __restrict__ ps,
    const double* __restrict__ pair_scale, int32_t D, int32_t norm_mode,
    double* __restrict__ pair_sum, double* __restrict__ pair_w, const double* __restrict__ rel,
    const int32_t* __restrict__ in_ptr, const int32_t* __restrict__ in_idx,
    const int32_t* __restrict__ out_ptr, const int32_t* __restrict__ out_idx,
    const int32_t* __restrict__ scene_of_view, int32_t V, double* __restrict__ grad,
    const int32_t* __restrict__ scene_ptr, const int32_t* __restrict__ scene_pairs, int32_t S,
    const int32_t* __restrict__ phase, double* __restrict__ loss, double* __restrict__ poses,
    double* __restrict__ m, double* __restrict__ w2, const uint8_t* __restrict__ fixed,
    const double* __restrict__ lr, double b1, double b2, double eps,
    int32_t* __restrict__ step, int32_t* __restrict__ status) {
    __shared__ double part[4];
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    for (int d = tid; d < D; d += blockDim.x)
        reduce_pair(d, partials, nullptr, ps, pair_scale, norm_mode, pair_sum, pair_w, nullptr,
                    nullptr, nullptr, nullptr, status);
    __syncthreads();
    for (int v = wave; v < V; v += blockDim.x >> 6)
        reduce_view(v, lane, pair_sum, pair_w, rel, in_ptr, in_idx, out_ptr, out_idx,
                    scene_of_view, nullptr, grad, nullptr, nullptr, nullptr);
    __syncthreads();
    const int st = step[0] + 1;
    const double bc1 = 1.0 - pow(b1, (double)st);
    const double bc2 = 1.0 - pow(b2, (double)st);
    for (int v = tid; v < V; v += blockDim.x)
        pose_update(v, poses, m, w2, grad, V, scene_of_view, fixed, lr, b1, b2, eps, bc1, bc2);
    for (int sc = 0; sc < S; ++sc) {
        if (phase && phase[sc] == 2) continue;        // the same for every thread
        reduce_scene(sc, pair_sum, ps, pair_scale, scene_ptr, scene_pairs, norm_mode, loss, part);
        __syncthreads();                              // part is reused by the next scene
    }
    __syncthreads();                                  // every thread has read the step
    if (tid == 0) step[0] = st;
}

}  // namespace

void launch_reductions(Plan& p, double* loss, double* pair_cost, int32_t* pair_valid,
                       double* pair_grad, double* grad, const double* upstream, hipStream_t s,
                       double* grad_gamma) {
    if (p.D > 0) {
        reduce_pairs_kernel<<<(unsigned)ceil_div(p.D, 256), 256, 0, s>>>(
            p.partials.p, grad_gamma ? p.ext_partials.p : nullptr, p.pair_static.p,
            p.pair_scale.p, p.D, p.params.norm_mode, p.pair_sum.p, p.pair_w.p, p.pair_ext.p,
            pair_cost, pair_valid, pair_grad, p.status.p);
        EPO_CHECK_LAUNCH();
    }
    if (grad || grad_gamma) {
        reduce_views_kernel<<<(unsigned)ceil_div(p.V, 4), 256, 0, s>>>(
            p.pair_sum.p, p.pair_w.p, p.pair_rel.p, p.view_in_ptr.p, p.view_in_idx.p,
            p.view_out_ptr.p, p.view_out_idx.p, p.scene_of_view_d.p, p.V, upstream, grad,
            p.pair_ext.p, p.gamma_d.p, grad_gamma);
        EPO_CHECK_LAUNCH();
    }
    if (loss) {
        reduce_scenes_kernel<<<(unsigned)p.S, 256, 0, s>>>(p.pair_sum.p, p.pair_static.p,
                                                            p.pair_scale.p, p.scene_ptr.p,
                                                            p.scene_pairs.p, p.params.norm_mode,
                                                            p.gate_phase, loss);
        EPO_CHECK_LAUNCH();
    }
}

// bounds of the small-plan epilogue: at most one pair per thread (each thread
// then sums one pair's tiles, the same dependent chain as in the pair
// kernel) and 16 poses per wave.  On the 8-view scene (56 pairs) it takes
// the step from 28 to 24 us; on the 32-view one (992 pairs, four pairs'
// tile chains per thread in a row) it was 15 us slower than the separate
// launches
constexpr int32_t kEpilogueMaxPairs = 256;
constexpr int32_t kEpilogueMaxViews = 64;
constexpr int64_t kEpilogueMaxTiles = 16384;
constexpr int32_t kEpilogueMaxScenes = 64;

// The small-plan epilogue: the reductions, pose step and step count of a
// captured pose iteration in one launch, when the plan is small enough for
// one workgroup (the bounds above); returns false (nothing launched)
// otherwise.
bool launch_step_epilogue(Plan& p, double* loss, double* grad, double* poses, double* m,
                          double* v, const uint8_t* fixed, const double* lr, double b1,
                          double b2, double eps, int32_t* step, hipStream_t s) {
    if (p.D > kEpilogueMaxPairs || p.V > kEpilogueMaxViews || p.n_tiles > kEpilogueMaxTiles ||
        p.S > kEpilogueMaxScenes)
        return false;
    step_epilogue_kernel<<<1, 256, 0, s>>>(
        p.partials.p, p.pair_static.p, p.pair_scale.p, p.D, p.params.norm_mode, p.pair_sum.p,
        p.pair_w.p, p.pair_rel.p, p.view_in_ptr.p, p.view_in_idx.p, p.view_out_ptr.p,
        p.view_out_idx.p, p.scene_of_view_d.p, p.V, grad, p.scene_ptr.p, p.scene_pairs.p, p.S,
        p.gate_phase, loss, poses, m, v, fixed, lr, b1, b2, eps, step, p.status.p);
    EPO_CHECK_LAUNCH();
    return true;
}

}  // namespace epo
