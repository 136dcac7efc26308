// Focal-length and depth refinement on the device (paper Sec. 3 "Camera
// Refinement" and "Depth Refinement"; the intrinsics update and the depth
// module of Alg. EPO.Forward):
//   f_v = f0_v (1 + gamma_v)        (fx and fy of view v scale together)
//   Z_p = Z0_p alpha_p + beta_p     (per edge pixel p of every view)
// The plan keeps the intrinsics and depths it was built with (f0, Z0); an
// update rewrites the intrinsics used by the pair set-up and the depth field
// of the edge records in place, so every later cost launch (and a captured
// iteration) sees the refined values.
//
// Depth gradient, source-major: the per-pixel derivative
//   dL/dZ_p = sum over pairs d out of view i of w_d (dH/dX') . m_d(p)
// (X' = Z m + t, m = R_ji K_i^-1 (u, v, 1)^T) needs the pair weights w_d, which
// exist only after the pair-major pass has counted the valid residuals.  So
// a second pass gives one thread to each edge record of view i and walks the
// pairs out of i in a fixed order, adding in float64: no atomics, bitwise
// reproducible.  dL/dbeta_p = dL/dZ_p and dL/dalpha_p = Z0_p dL/dZ_p.
// Two forms of that pass, with bitwise identical results:
//   stored     the pair-major refinement kernel has written every residual's
//              dH/dZ (float32, 4 bytes per residual) source-major: each
//              256-record block of a source holds one 1 KB chunk per pair out
//              of it, so the pass reads one contiguous run per block
//   recompute  no room for that buffer: the pass evaluates every residual
//              again from the record, the pair descriptor and the texture.
#include "residual.h"

namespace epo {
namespace {

constexpr int kBlock = 256;

__global__ __launch_bounds__(256) void refine_intrinsics_kernel(
    const float* __restrict__ K0, const double* __restrict__ gamma, float* __restrict__ K,
    double* __restrict__ gamma_state, int32_t V, int32_t* __restrict__ status) {
    const int v = blockIdx.x * blockDim.x + threadIdx.x;
    if (v >= V) return;
    const double g = gamma ? gamma[v] : 0.0;
    const double s = 1.0 + g;
    // float64 product of the float32 focal length, rounded once to float32
    const float fx = (float)((double)K0[4 * v] * s);
    const float fy = (float)((double)K0[4 * v + 1] * s);
    if (!(fx > 0.0f) || !(fy > 0.0f) || !isfinite(fx) || !isfinite(fy)) atomicOr(status, 4);
    K[4 * v] = fx;
    K[4 * v + 1] = fy;
    K[4 * v + 2] = K0[4 * v + 2];
    K[4 * v + 3] = K0[4 * v + 3];
    gamma_state[v] = g;
}

__global__ __launch_bounds__(256) void snapshot_depth_kernel(const uint2* __restrict__ records,
                                                             float* __restrict__ z0, int64_t n) {
    const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k < n) z0[k] = __uint_as_float(records[k].y);
}

// Z0 alpha is exact in float64 (two float32 factors), so this is one
// rounding to float64 followed by one to float32
__device__ inline float refined_depth(float z0, float alpha, float beta) {
    return (float)fma((double)z0, (double)alpha, (double)beta);
}

__global__ __launch_bounds__(256) void refine_depth_kernel(const float* __restrict__ z0,
                                                           const float* __restrict__ alpha,
                                                           const float* __restrict__ beta,
                                                           uint2* __restrict__ records, int64_t n,
                                                           int32_t* __restrict__ status) {
    const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= n) return;
    const float z = alpha ? refined_depth(z0[k], alpha[k], beta[k]) : z0[k];
    if (!isfinite(z)) atomicOr(status, 4);
    records[k].y = __float_as_uint(z);
}

template <int FMT>
__global__ __launch_bounds__(kBlock) void depth_grad_kernel(
    const uint2* __restrict__ records, const uint32_t* __restrict__ tex,
    const Tile* __restrict__ vblocks, const PairDesc* __restrict__ desc,
    const double* __restrict__ pair_w, const int32_t* __restrict__ out_ptr,
    const int32_t* __restrict__ out_idx, const int32_t* __restrict__ scene_of_view,
    const double* __restrict__ upstream, const float* __restrict__ z0, float delta, double zmin,
    double* __restrict__ grad_alpha, double* __restrict__ grad_beta) {
    __shared__ float lut[256];
    if (FMT == 2) lut[threadIdx.x] = sqrtf((float)threadIdx.x);
    __syncthreads();
    const Tile b = vblocks[blockIdx.x];
    const int i = b.pair;                       // source view of this block
    const bool active = (int)threadIdx.x < b.count;
    const int64_t k = b.rec + threadIdx.x;
    const uint2 rec = active ? records[k] : make_uint2(0u, 0u);
    double acc = 0.0;
    const int e1 = out_ptr[i + 1];
    for (int e = out_ptr[i]; e < e1; ++e) {
        const int d = out_idx[e];
        const double wd = pair_w[d];
        if (wd == 0.0) continue;                // no valid residual in pair d
        const PairDesc pd = desc[d];
        const Residual r = eval_residual<FMT>(rec, active, pd, view_texture<FMT>(tex, pd.tex_off),
                                              lut, delta, zmin);
        acc = fma(wd, (double)depth_derivative(r), acc);
    }
    if (!active) return;
    const double g = (upstream ? upstream[scene_of_view[i]] : 1.0) * acc;
    if (grad_beta) grad_beta[k] = g;
    if (grad_alpha) grad_alpha[k] = g * (double)(z0 ? z0[k] : __uint_as_float(rec.y));
}

__global__ __launch_bounds__(256) void depth_gather_kernel(
    const float* __restrict__ dz, const int64_t* __restrict__ dz_index,
    const Tile* __restrict__ vblocks, const double* __restrict__ pair_w,
    const int32_t* __restrict__ out_ptr, const int32_t* __restrict__ out_idx,
    const int32_t* __restrict__ scene_of_view, const double* __restrict__ upstream,
    const float* __restrict__ z0, const uint2* __restrict__ records,
    double* __restrict__ grad_alpha, double* __restrict__ grad_beta) {
    const Tile b = vblocks[blockIdx.x];
    const int i = b.pair;
    if ((int)threadIdx.x >= b.count) return;
    const int64_t k = b.rec + threadIdx.x;
    double acc = 0.0;
    const int e0 = out_ptr[i], n = out_ptr[i + 1] - e0;
    if (n > 0) {
        // the block's derivative chunks are contiguous, one of 256 per pair
        // out of i in CSR order, so the loads need no per-pair look-up and
        // go out eight at a time ahead of the (ordered) sums.  Same pairs,
        // same order and same float32 terms as the recompute form
        const float* __restrict__ g = dz + dz_index[2 * out_idx[e0]] + b.rec * n + threadIdx.x;
        constexpr int B = 8;
        int q = 0;
        for (; q + B <= n; q += B) {
            float gq[B];
#pragma unroll
            for (int u = 0; u < B; ++u) gq[u] = g[(int64_t)(q + u) * 256];
#pragma unroll
            for (int u = 0; u < B; ++u) {
                const double wd = pair_w[out_idx[e0 + q + u]];
                // a pair with zero weight (no valid residual, or skipped by
                // this step's sub-sampling) holds no derivatives this step
                acc = wd != 0.0 ? fma(wd, (double)gq[u], acc) : acc;
            }
        }
        for (; q < n; ++q) {
            const double wd = pair_w[out_idx[e0 + q]];
            const float gq = g[(int64_t)q * 256];
            acc = wd != 0.0 ? fma(wd, (double)gq, acc) : acc;
        }
    }
    const double gr = (upstream ? upstream[scene_of_view[i]] : 1.0) * acc;
    if (grad_beta) grad_beta[k] = gr;
    if (grad_alpha) grad_alpha[k] = gr * (double)(z0 ? z0[k] : __uint_as_float(records[k].y));
}

template <int FMT>
void launch_depth_fmt(Plan& p, const uint32_t* tex, const double* upstream, double* grad_alpha,
                      double* grad_beta, hipStream_t s) {
    depth_grad_kernel<FMT><<<(unsigned)p.n_vblocks, kBlock, 0, s>>>(
        reinterpret_cast<const uint2*>(p.records.p), tex, p.vblocks.p, p.pair_desc.p, p.pair_w.p,
        p.view_out_ptr.p, p.view_out_idx.p, p.scene_of_view_d.p, upstream, p.z0.p,
        p.params.huber_delta, p.params.z_min, grad_alpha, grad_beta);
    EPO_CHECK_LAUNCH();
}

// AdamW step of the joint phase's parameters (decoupled weight decay, then
// Adam with bias correction at the 1-based step of the optimizer that owns
// the parameter), one thread per view (its focal scale gamma, float64) and
// one per edge record (its alpha and beta, float32 parameters: the update is
// formed in float64 from the stored value and rounded once).  Each scene's
// focal scales and depth parameters count their own steps: steps[s] and
// steps[S + s] hold the steps taken so far (advanced afterwards by
// count_joint_steps_kernel), so a scene's first depth step after its switch
// to the joint phase is its depth optimizer's step 1.  Moments are float64:
// m_depth / v_depth hold alpha's at [0, n) and beta's at [n, 2n).  With a
// phase array, the scene's phase gates the step: gamma moves unless the
// scene has stopped (phase 2), alpha and beta only in the joint phase
// (phase 1); a gated parameter and its moments are left as they are.  With
// z0 and records, each record's depth is then rewritten from the current
// alpha and beta, as the refinement update does.
__global__ __launch_bounds__(256) void joint_step_kernel(
    double* __restrict__ gamma, float* __restrict__ alpha, float* __restrict__ beta,
    double* __restrict__ m_gamma, double* __restrict__ v_gamma, double* __restrict__ m_depth,
    double* __restrict__ v_depth, const double* __restrict__ g_gamma,
    const double* __restrict__ g_alpha, const double* __restrict__ g_beta,
    const int64_t* __restrict__ rec_off, const int32_t* __restrict__ scene_of_view, int32_t V,
    int64_t n, int32_t S, const double* __restrict__ lr, const int32_t* __restrict__ phase,
    double b1, double b2, double eps, double wd_focal, double wd_depth,
    const int32_t* __restrict__ steps, const float* __restrict__ z0, uint2* __restrict__ records,
    int32_t* __restrict__ status) {
    const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    // the view of the workgroup's first record, found once (records are in
    // view order, so each thread then advances a few views at most)
    __shared__ int view0;
    if (threadIdx.x == 0) {
        const int64_t r0 = std::max<int64_t>((int64_t)blockIdx.x * blockDim.x - V, 0);
        int lo = 0, hi = V - 1;              // last view whose first record is <= r0
        while (lo < hi) {
            const int mid = (lo + hi + 1) >> 1;
            if (rec_off[mid] <= r0) lo = mid; else hi = mid - 1;
        }
        view0 = lo;
    }
    __syncthreads();
    if (k >= (int64_t)V + n) return;
    if (k < V) {
        const int sc = scene_of_view[k];
        if (phase && phase[sc] == 2) return;
        const double t = (double)(steps[sc] + 1);
        const double c1 = 1.0 - pow(b1, t), c2 = 1.0 - pow(b2, t);
        const double a = lr[sc];
        const double g = g_gamma[k];
        const double mk = b1 * m_gamma[k] + (1.0 - b1) * g;
        const double vk = b2 * v_gamma[k] + (1.0 - b2) * g * g;
        m_gamma[k] = mk;
        v_gamma[k] = vk;
        gamma[k] = gamma[k] * (1.0 - a * wd_focal) - a * (mk / c1) / (sqrt(vk / c2) + eps);
        return;
    }
    const int64_t r = k - V;
    int view = view0;                        // rec_off[view] <= r0 <= r < n = rec_off[V]
    while (rec_off[view + 1] <= r) ++view;
    const int sc = scene_of_view[view];
    float xa = alpha[r], xb = beta[r];
    if (!phase || phase[sc] == 1) {
        const double t = (double)(steps[S + sc] + 1);
        const double c1 = 1.0 - pow(b1, t), c2 = 1.0 - pow(b2, t);
        const double a = lr[sc];
        const double ga = g_alpha[r], gb = g_beta[r];
        const double ma = b1 * m_depth[r] + (1.0 - b1) * ga;
        const double va = b2 * v_depth[r] + (1.0 - b2) * ga * ga;
        const double mb = b1 * m_depth[n + r] + (1.0 - b1) * gb;
        const double vb = b2 * v_depth[n + r] + (1.0 - b2) * gb * gb;
        m_depth[r] = ma;
        v_depth[r] = va;
        m_depth[n + r] = mb;
        v_depth[n + r] = vb;
        xa = (float)((double)xa * (1.0 - a * wd_depth) - a * (ma / c1) / (sqrt(va / c2) + eps));
        xb = (float)((double)xb * (1.0 - a * wd_depth) - a * (mb / c1) / (sqrt(vb / c2) + eps));
        alpha[r] = xa;
        beta[r] = xb;
    }
    if (records) {
        const float z = refined_depth(z0[r], xa, xb);
        if (!isfinite(z)) atomicOr(status, 4);
        records[r].y = __float_as_uint(z);
    }
}

// the steps the joint step just took: a scene's focal count advances unless
// it has stopped, its depth count only in the joint phase (every count when
// no phases are given)
__global__ __launch_bounds__(256) void count_joint_steps_kernel(int32_t* __restrict__ steps,
                                                                const int32_t* __restrict__ phase,
                                                                int32_t S) {
    const int s = blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= S) return;
    const int ph = phase ? phase[s] : 1;
    if (ph != 2) steps[s] += 1;
    if (ph == 1) steps[S + s] += 1;
}

}  // namespace

void launch_depth_grad(Plan& p, const double* upstream, double* grad_alpha, double* grad_beta,
                       bool stored, hipStream_t s) {
    if (p.n_vblocks == 0) return;
    if (stored) {
        depth_gather_kernel<<<(unsigned)p.n_vblocks, kBlock, 0, s>>>(
            p.dz.p, p.dz_index.p, p.vblocks.p, p.pair_w.p, p.view_out_ptr.p,
            p.view_out_idx.p, p.scene_of_view_d.p, upstream, p.z0.p,
            reinterpret_cast<const uint2*>(p.records.p), grad_alpha, grad_beta);
        EPO_CHECK_LAUNCH();
        return;
    }
    if (p.opt.texture_format == 2)
        launch_depth_fmt<2>(p, p.tex.p, upstream, grad_alpha, grad_beta, s);
    else if (p.opt.texture_format == 3)
        launch_depth_fmt<3>(p, reinterpret_cast<const uint32_t*>(p.tex_q32.p), upstream,
                            grad_alpha, grad_beta, s);
    else
        launch_depth_fmt<1>(p, reinterpret_cast<const uint32_t*>(p.tex_f32.p), upstream,
                            grad_alpha, grad_beta, s);
}

}  // namespace epo

using namespace epo;

namespace epo {

void install_refinement(Plan& p, const double* gamma, const float* alpha, const float* beta,
                        hipStream_t s) {
    if (!p.dz.p && p.dz_size > 0 && !p.dz_declined) {
        // room for the per-residual depth derivatives: use at most half
        // of the free device memory, else keep recomputing them
        size_t free_b = 0, total_b = 0;
        EPO_HIP(hipMemGetInfo(&free_b, &total_b));
        if ((uint64_t)p.dz_size * sizeof(float) <= free_b / 2)
            p.dz.alloc((size_t)p.dz_size);
        else
            p.dz_declined = true;
    }
    refine_intrinsics_kernel<<<(unsigned)ceil_div(p.V, 256), 256, 0, s>>>(
        p.K0_d.p, gamma, p.K_d.p, p.gamma_d.p, p.V, p.status.p);
    EPO_CHECK_LAUNCH();
    const int64_t n = p.rec_off.back();
    if (n == 0) return;
    if (!p.z0.p) {
        // first depth update: keep the depths the plan was built with
        if (!alpha) return;
        p.z0.alloc((size_t)n);
        snapshot_depth_kernel<<<(unsigned)ceil_div(n, 256), 256, 0, s>>>(
            reinterpret_cast<const uint2*>(p.records.p), p.z0.p, n);
        EPO_CHECK_LAUNCH();
    }
    refine_depth_kernel<<<(unsigned)ceil_div(n, 256), 256, 0, s>>>(
        p.z0.p, alpha, beta, reinterpret_cast<uint2*>(p.records.p), n, p.status.p);
    EPO_CHECK_LAUNCH();
}

void launch_joint_step(Plan& p, const epo_joint_state& j, const double* lr, const int32_t* phase,
                       double b1, double b2, double eps, hipStream_t s) {
    const int64_t n = p.rec_off.back();
    const bool installed = p.z0.p != nullptr;
    const int64_t total = (int64_t)p.V + n;
    joint_step_kernel<<<(unsigned)ceil_div(total, 256), 256, 0, s>>>(
        j.gamma, j.alpha, j.beta, j.m_gamma, j.v_gamma, j.m_depth, j.v_depth, j.grad_gamma,
        j.grad_alpha, j.grad_beta, p.rec_off_d.p, p.scene_of_view_d.p, p.V, n, p.S, lr, phase, b1,
        b2, eps, j.wd_focal, j.wd_depth, j.steps, installed ? p.z0.p : nullptr,
        installed ? reinterpret_cast<uint2*>(p.records.p) : nullptr, p.status.p);
    EPO_CHECK_LAUNCH();
    count_joint_steps_kernel<<<(unsigned)ceil_div(p.S, 256), 256, 0, s>>>(j.steps, phase, p.S);
    EPO_CHECK_LAUNCH();
    if (installed) {
        refine_intrinsics_kernel<<<(unsigned)ceil_div(p.V, 256), 256, 0, s>>>(
            p.K0_d.p, j.gamma, p.K_d.p, p.gamma_d.p, p.V, p.status.p);
        EPO_CHECK_LAUNCH();
    }
}

void ensure_record_offsets(Plan& p, hipStream_t s) {
    if (p.rec_off_d.p) return;
    p.rec_off_d.alloc(p.rec_off.size());
    EPO_HIP(hipMemcpyAsync(p.rec_off_d.p, p.rec_off.data(), p.rec_off.size() * sizeof(int64_t),
                           hipMemcpyHostToDevice, s));
    EPO_HIP(hipStreamSynchronize(s));
}

}  // namespace epo

extern "C" epo_status epo_plan_set_refinement(epo_plan plan, const double* gamma,
                                              const float* alpha, const float* beta,
                                              void* stream) {
    return guarded([&] {
        EPO_REQUIRE(plan, "null plan");
        EPO_REQUIRE((alpha == nullptr) == (beta == nullptr),
                    "alpha and beta must be given together");
        Plan& p = *reinterpret_cast<Plan*>(plan);
        EPO_HIP(hipSetDevice(p.device));
        install_refinement(p, gamma, alpha, beta, as_stream(stream));
    });
}

extern "C" epo_status epo_edge_cost_refine(epo_plan plan, const double* poses,
                                           const float* lambda, const double* upstream,
                                           double* loss, double* grad, double* grad_gamma,
                                           double* grad_alpha, double* grad_beta, void* stream) {
    return guarded([&] {
        EPO_REQUIRE(plan, "null plan");
        EPO_REQUIRE(poses && lambda, "poses and lambda are required");
        Plan& p = *reinterpret_cast<Plan*>(plan);
        EPO_HIP(hipSetDevice(p.device));
        const RefineOut out{grad_gamma, grad_alpha, grad_beta};
        launch_cost(p, poses, lambda, loss, nullptr, nullptr, nullptr, grad, upstream,
                    as_stream(stream), &out);
    });
}

extern "C" epo_status epo_joint_step(epo_plan plan, double* gamma, float* alpha, float* beta,
                                     double* m_gamma, double* v_gamma, double* m_depth,
                                     double* v_depth, const double* grad_gamma,
                                     const double* grad_alpha, const double* grad_beta,
                                     const double* lr, const int32_t* phase, double beta1,
                                     double beta2, double eps, double wd_focal, double wd_depth,
                                     int32_t* steps, void* stream) {
    return guarded([&] {
        EPO_REQUIRE(plan, "null plan");
        EPO_REQUIRE(gamma && alpha && beta && m_gamma && v_gamma && m_depth && v_depth &&
                        grad_gamma && grad_alpha && grad_beta && lr && steps,
                    "null pointer argument (only phase may be null)");
        EPO_REQUIRE(beta1 >= 0.0 && beta1 < 1.0 && beta2 >= 0.0 && beta2 < 1.0 && eps > 0.0,
                    "beta1, beta2 must be in [0, 1) and eps > 0");
        Plan& p = *reinterpret_cast<Plan*>(plan);
        EPO_HIP(hipSetDevice(p.device));
        hipStream_t s = as_stream(stream);
        ensure_record_offsets(p, s);
        // once the plan holds its original depths (after the first depth
        // update), the step kernel rewrites the records' depths itself
        const bool installed = p.z0.p != nullptr;
        const epo_joint_state j{gamma,  alpha,      beta,       m_gamma,   v_gamma,
                                m_depth, v_depth,   steps,      const_cast<double*>(grad_gamma),
                                const_cast<double*>(grad_alpha),
                                const_cast<double*>(grad_beta), wd_focal, wd_depth};
        launch_joint_step(p, j, lr, phase, beta1, beta2, eps, s);
        // first depth update of the plan: the refinement update keeps its depths
        if (!installed) install_refinement(p, gamma, alpha, beta, s);
    });
}
