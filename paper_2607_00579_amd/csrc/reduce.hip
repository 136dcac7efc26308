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
// One launch: one thread per pair; one wave64 per pose (lanes stride over
// the pose's pairs, then a butterfly); one workgroup per scene (threads stride
// over its pairs, then wave butterflies and an LDS step).  The pose and scene
// parts form the pair sums from the tiles themselves, so no part waits for
// another.
#include "epo_internal.h"

namespace epo {
namespace {

__device__ inline double wave_sum64(double x) {
#pragma unroll
    for (int m = 32; m >= 1; m >>= 1) x += __shfl_xor(x, m, 64);
    return x;
}

// the sums of pair d over its tiles, in tile order (S, n, G[6]); a pair
// skipped by the sub-sampling of this step ran no tiles: all zero
__device__ __forceinline__ void pair_tile_sums(const Partial* __restrict__ partials,
                                               const PairStatic& st, double scale, double* s) {
    const int n_tiles = scale != 0.0 ? st.n_tiles : 0;
#pragma unroll
    for (int c = 0; c < 8; ++c) s[c] = 0.0;
    for (int k = 0; k < n_tiles; ++k) {
        const Partial pt = partials[st.first_tile + k];
#pragma unroll
        for (int c = 0; c < 8; ++c) s[c] += pt.v[c];
    }
}

// the focal sums F_t, F_s of pair d over its tiles, in tile order
__device__ __forceinline__ void pair_tile_ext(const double* __restrict__ ext_partials,
                                              const PairStatic& st, double scale, double& ft,
                                              double& fs) {
    const int n_tiles = scale != 0.0 ? st.n_tiles : 0;
    ft = fs = 0.0;
    for (int k = 0; k < n_tiles; ++k) {
        ft += ext_partials[2 * (int64_t)(st.first_tile + k)];
        fs += ext_partials[2 * (int64_t)(st.first_tile + k) + 1];
    }
}

// the pose weight w_d = scale / (n_d or |E_i|) (0 for a pair without residuals)
__device__ __forceinline__ double pair_weight(const double* s, const PairStatic& st, double scale,
                                              int32_t norm_mode) {
    const double den = norm_mode == 0 ? s[1] : (double)st.n_src;
    return den > 0 ? scale / den : 0.0;
}

struct ReduceArgs {
    const Partial* partials;
    const double* ext_partials;              // null: no focal sums
    const PairStatic* ps;
    const double* pair_scale;
    int32_t D, V, S, norm_mode;
    // pairs
    double* pair_sum;
    double* pair_w;
    double* pair_ext;
    double* pair_cost;
    int32_t* pair_valid;
    double* pair_grad;
    int32_t* status;
    // poses
    const double* rel;
    const int32_t *in_ptr, *in_idx, *out_ptr, *out_idx, *scene_of_view;
    const double* upstream;
    double* grad;
    const double* gamma;
    double* grad_gamma;
    // scenes
    const int32_t *scene_ptr, *scene_pairs, *phase;
    double* loss;
    // block ranges
    int32_t pair_blocks, view_blocks;
};

// one thread per pair: its sums, weight and outputs
__device__ void reduce_pair(const ReduceArgs& a, int d) {
    if (d >= a.D) return;
    const PairStatic st = a.ps[d];
    const double scale = a.pair_scale[d];
    double s[8];
    pair_tile_sums(a.partials, st, scale, s);
    if (a.ext_partials) {
        double ft, fs;
        pair_tile_ext(a.ext_partials, st, scale, ft, fs);
        if (!isfinite(ft) || !isfinite(fs)) atomicOr(a.status, 1);
        a.pair_ext[2 * d] = ft;
        a.pair_ext[2 * d + 1] = fs;
    }
    const double den = a.norm_mode == 0 ? s[1] : (double)st.n_src;
    const double L = den > 0 ? s[0] / den : 0.0;
    if (!isfinite(s[0]) || !isfinite(s[2]) || !isfinite(s[5])) atomicOr(a.status, 1);
#pragma unroll
    for (int c = 0; c < 8; ++c) a.pair_sum[8 * d + c] = s[c];
    a.pair_w[d] = pair_weight(s, st, scale, a.norm_mode);
    if (a.pair_cost) a.pair_cost[d] = L;
    if (a.pair_valid) a.pair_valid[d] = (int32_t)s[1];
    if (a.pair_grad) {
#pragma unroll
        for (int c = 0; c < 6; ++c) a.pair_grad[6 * d + c] = s[2 + c];
    }
}

// one wave per pose: its pairs' sums are formed again from the tiles (the
// same additions in the same order as the pair threads'), so the three
// parts of the reduction need no ordering among each other
__device__ void reduce_view(const ReduceArgs& a, int v, int lane) {
    if (v >= a.V) return;                     // whole wave leaves together
    double g[6] = {0, 0, 0, 0, 0, 0};
    double gf = 0.0;
    for (int k = a.in_ptr[v] + lane; k < a.in_ptr[v + 1]; k += 64) {
        const int d = a.in_idx[k];
        const PairStatic st = a.ps[d];
        const double scale = a.pair_scale[d];
        double s[8];
        pair_tile_sums(a.partials, st, scale, s);
        const double w = pair_weight(s, st, scale, a.norm_mode);
#pragma unroll
        for (int c = 0; c < 6; ++c) g[c] += w * s[2 + c];
        if (a.grad_gamma) {
            double ft, fs;
            pair_tile_ext(a.ext_partials, st, scale, ft, fs);
            gf += w * ft;
        }
    }
    //   Ad^T (G_r, G_w) = (R^T G_r, R^T (G_w - t x G_r))
    for (int k = a.out_ptr[v] + lane; k < a.out_ptr[v + 1]; k += 64) {
        const int d = a.out_idx[k];
        const PairStatic st = a.ps[d];
        const double scale = a.pair_scale[d];
        double s[8];
        pair_tile_sums(a.partials, st, scale, s);
        const double w = pair_weight(s, st, scale, a.norm_mode);
        const double* R = a.rel + 12 * d;
        const double* t = R + 9;
        const double* G = s + 2;
        const double c0 = G[3] - (t[1] * G[2] - t[2] * G[1]);
        const double c1 = G[4] - (t[2] * G[0] - t[0] * G[2]);
        const double c2 = G[5] - (t[0] * G[1] - t[1] * G[0]);
#pragma unroll
        for (int r = 0; r < 3; ++r) {
            g[r] -= w * (R[0 + r] * G[0] + R[3 + r] * G[1] + R[6 + r] * G[2]);
            g[3 + r] -= w * (R[0 + r] * c0 + R[3 + r] * c1 + R[6 + r] * c2);
        }
        if (a.grad_gamma) {
            double ft, fs;
            pair_tile_ext(a.ext_partials, st, scale, ft, fs);
            gf += w * fs;
        }
    }
    const double up = a.upstream ? a.upstream[a.scene_of_view[v]] : 1.0;
    if (a.grad) {
#pragma unroll
        for (int c = 0; c < 6; ++c) g[c] = wave_sum64(g[c]);
        if (lane < 6) {
            double x = g[0];
#pragma unroll
            for (int c = 1; c < 6; ++c) x = lane == c ? g[c] : x;
            a.grad[6 * v + lane] = up * x;
        }
    }
    if (a.grad_gamma) {
        gf = wave_sum64(gf);
        if (lane == 0) a.grad_gamma[v] = up * gf / (1.0 + a.gamma[v]);
    }
}

// one workgroup per scene; a scene the convergence test has stopped (phase
// 2, when phases are given) evaluated nothing and keeps its last loss
__device__ void reduce_scene(const ReduceArgs& a, int sc, double* part) {
    if (a.phase && a.phase[sc] == 2) return;
    double L = 0.0;
    for (int k = a.scene_ptr[sc] + threadIdx.x; k < a.scene_ptr[sc + 1]; k += blockDim.x) {
        const int d = a.scene_pairs[k];
        const PairStatic st = a.ps[d];
        const double scale = a.pair_scale[d];
        double s[8];
        pair_tile_sums(a.partials, st, scale, s);
        const double den = a.norm_mode == 0 ? s[1] : (double)st.n_src;
        if (den > 0) L += scale * (s[0] / den);
    }
    L = wave_sum64(L);
    if ((threadIdx.x & 63) == 0) part[threadIdx.x >> 6] = L;
    __syncthreads();
    if (threadIdx.x == 0) a.loss[sc] = (part[0] + part[1]) + (part[2] + part[3]);
}

// the three parts in one launch: blocks [0, pair_blocks) take 256 pairs
// each, the next view_blocks four poses each, the rest one scene each
__global__ __launch_bounds__(256) void reduce_kernel(ReduceArgs a) {
    __shared__ double part[4];
    const int b = (int)blockIdx.x;
    if (b < a.pair_blocks) {
        reduce_pair(a, b * 256 + (int)threadIdx.x);
    } else if (b < a.pair_blocks + a.view_blocks) {
        reduce_view(a, (b - a.pair_blocks) * 4 + ((int)threadIdx.x >> 6), (int)threadIdx.x & 63);
    } else {
        reduce_scene(a, b - a.pair_blocks - a.view_blocks, part);
    }
}

}  // namespace

void launch_reductions(Plan& p, double* loss, double* pair_cost, int32_t* pair_valid,
                       double* pair_grad, double* grad, const double* upstream, hipStream_t s,
                       double* grad_gamma) {
    ReduceArgs a{};
    a.partials = p.partials.p;
    a.ext_partials = grad_gamma ? p.ext_partials.p : nullptr;
    a.ps = p.pair_static.p;
    a.pair_scale = p.pair_scale.p;
    a.D = p.D;
    a.V = p.V;
    a.S = p.S;
    a.norm_mode = p.params.norm_mode;
    a.pair_sum = p.pair_sum.p;
    a.pair_w = p.pair_w.p;
    a.pair_ext = p.pair_ext.p;
    a.pair_cost = pair_cost;
    a.pair_valid = pair_valid;
    a.pair_grad = pair_grad;
    a.status = p.status.p;
    a.rel = p.pair_rel.p;
    a.in_ptr = p.view_in_ptr.p;
    a.in_idx = p.view_in_idx.p;
    a.out_ptr = p.view_out_ptr.p;
    a.out_idx = p.view_out_idx.p;
    a.scene_of_view = p.scene_of_view_d.p;
    a.upstream = upstream;
    a.grad = grad;
    a.gamma = p.gamma_d.p;
    a.grad_gamma = grad_gamma;
    a.scene_ptr = p.scene_ptr.p;
    a.scene_pairs = p.scene_pairs.p;
    a.phase = p.gate_phase;
    a.loss = loss;
    a.pair_blocks = p.D > 0 ? (int32_t)ceil_div(p.D, 256) : 0;
    a.view_blocks = (grad || grad_gamma) ? (int32_t)ceil_div(p.V, 4) : 0;
    const int scene_blocks = loss ? p.S : 0;
    const int blocks = a.pair_blocks + a.view_blocks + scene_blocks;
    if (blocks == 0) return;
    reduce_kernel<<<(unsigned)blocks, 256, 0, s>>>(a);
    EPO_CHECK_LAUNCH();
}

}  // namespace epo
