// Per-iteration hot path on gfx950: relative poses and the fused residual +
// adjoint kernel (paper Eqs. pi, L, L_ij, d_ij; supplementary Alg. 3 and
// Sec. A1.2 "Per-iteration kernels").  The float64 reductions above the tile
// partials are in reduce.hip.
//
// Fused kernel, per residual (source edge pixel p = (u, v) with depth Z of
// view i, directed pair i -> j):
//   lift + warp in one step: X' = Z M (u, v, 1)^T + t_ji with M = R_ji K_i^-1
//     (the paper lifts to the world once per image and projects per pair;
//     folding the pose-free lift into one 3x3 per pair gives the same point
//     with fewer operations), z = X'_z, x_n = X'_x / z, y_n = X'_y / z,
//     u' = fx_j x_n + cx_j, v' = fy_j y_n + cy_j; this coordinate, the
//     validity test and the cell split are float64, the rest of the residual
//     and its adjoint float32;
//   valid iff z > z_min and 0 <= u' < W_j - 1 and 0 <= v' < H_j - 1;
//   bilinear D from the cell floor(u'), floor(v'); d^ = min(D, lambda);
//   rho = Huber(d^); rho' = dHuber/dd^ if D < lambda else 0;
//   adjoint: with A_u = rho' dD/du' fx_j, A_v = rho' dD/dv' fy_j, the
//   normalised target coordinates x_n, y_n and
//   w = -(A_u x_n + A_v y_n), the left-twist gradient of the target pose is
//     (A_u, A_v, w) / z   and   (y_n w - A_v, A_u - x_n w, x_n A_v - y_n A_u)
//   (the translation block is dH/dX', the rotation block X' x dH/dX', in
//   which the depth cancels).
// A refinement variant of the same kernel also sums the focal-scale terms of
// both views (Sec. 3 Camera Refinement); the per-pixel depth gradient comes
// from a second, source-major pass in refine.hip.
// Each thread adds its float32 residual terms in float64; each workgroup
// reduces its tile to eight float64 partial sums (S, n, G[6]) with wave64
// butterflies and an LDS step across its four waves.  Everything above the
// tile is float64 in a fixed order too: per pair (tiles in order), per
// pose (g_j += w_d G_d, g_i += -w_d Ad(T_ji)^T G_d), per scene.
#include "fused_kernel.h"

namespace epo {
namespace {

using fused::edge_cost_kernel;
using fused::kBlock;

// ---------------------------------------------------------------------------
// relative poses and pair descriptors (one thread per directed pair)
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void pair_setup_kernel(
    const double* __restrict__ poses, const float* __restrict__ K, const int32_t* __restrict__ wh,
    const int64_t* __restrict__ view_off, const int64_t* __restrict__ blk_off,
    const PairStatic* __restrict__ ps,
    const float* __restrict__ lambda, float lambda_max, PairDesc* __restrict__ desc,
    double* __restrict__ rel, int32_t D, int32_t* __restrict__ counters, int32_t n_counters,
    int32_t* __restrict__ status, ScheduleArgs sched) {
    const int d = blockIdx.x * blockDim.x + threadIdx.x;
    if (d < n_counters) counters[d] = 0;      // work queues of the next cost launch
    // the schedule of this step, when this launch takes the schedule
    // kernel's place: lambda for every pair, each scene's lambda and rate
    // written for the kernels after it
    float lv = 0.0f;
    if (sched.step) {
        double r;
        schedule_at(sched, sched.step[0], lv, r);
        if (d < sched.S) {
            if (sched.lam) sched.lam[d] = lv;
            if (sched.lr) sched.lr[d] = (sched.phase && sched.phase[d] == 2) ? 0.0 : r;
        }
    }
    if (d >= D) return;
    const PairStatic st = ps[d];
    const int i = st.src, j = st.tgt;
    double R[9], t[3], M[9];
    relative_pose(poses, K, i, j, R, t, M);
    const double fxj = K[4 * j + 0], fyj = K[4 * j + 1], cxj = K[4 * j + 2], cyj = K[4 * j + 3];
    PairDesc o;
    for (int k = 0; k < 9; ++k) o.M[k] = M[k];
    for (int k = 0; k < 3; ++k) o.t[k] = t[k];
    o.fxd = fxj;
    o.fyd = fyj;
    o.cxd = cxj;
    o.cyd = cyj;
    o.fx = (float)fxj;
    o.fy = (float)fyj;
    o.wcells = wh[2 * j + 0] - 1;
    o.hcells = wh[2 * j + 1] - 1;
    const float lam = sched.step ? lv : lambda[st.scene];
    if (!(lam >= 0.0f && lam <= lambda_max)) atomicOr(status, 2);
    o.lambda = lam;
    // texture addressing of the format in use: blocked u8 quads (blk_off
    // given: width = 128 (blocks per row - 1), the row-of-blocks stride less
    // the part that 32 y0 covers) or row-major per-pixel texels
    o.width = blk_off ? 128 * ((wh[2 * j + 0] + kQuadBlockW - 1) / kQuadBlockW - 1)
                      : wh[2 * j + 0];
    o.tex_off = blk_off ? blk_off[j] : view_off[j];
    desc[d] = o;
    for (int k = 0; k < 9; ++k) rel[12 * d + k] = R[k];
    for (int k = 0; k < 3; ++k) rel[12 * d + 9 + k] = t[k];
}

template <int FMT, int P, bool EXT>
void launch_cost_kernel(Plan& p, float* dz, hipStream_t s) {
    const uint32_t* tex = FMT == 2   ? p.tex.p
                          : FMT == 3 ? reinterpret_cast<const uint32_t*>(p.tex_q32.p)
                                     : reinterpret_cast<const uint32_t*>(p.tex_f32.p);
    const int nq = p.n_xcd_queues;
    const bool persistent = p.opt.persistent == 1;
    unsigned grid;
    if (persistent) {
        int64_t want = (int64_t)p.n_cu * 8;
        want = std::min<int64_t>(want, ceil_div(p.n_tiles, 1) + nq);
        grid = (unsigned)(ceil_div(want, nq) * nq);
    } else if (compacted_launch(p)) {
        // with pair sub-sampling (or stopped scenes skipped) the step's tile
        // count is known only on the device: enough workgroups for every
        // tile, split as the compacted list is (nq equal queues); those past
        // a queue's end exit at once
        grid = (unsigned)(ceil_div(p.n_tiles, nq) * nq);
    } else {
        int64_t per_q = 0;
        for (int q = 0; q < nq; ++q)
            per_q = std::max<int64_t>(per_q, p.xcd_begin[q + 1] - p.xcd_begin[q]);
        grid = (unsigned)(per_q * nq);
    }
    if (grid == 0) return;
    auto kernel = persistent ? edge_cost_kernel<FMT, P, EXT, true>
                             : edge_cost_kernel<FMT, P, EXT, false>;
    // the pose-only variant reads the per-pair sorted copies under record
    // order 2; the refinement variant stores depth derivatives by source
    // record and keeps the source order
    const bool own = !EXT && p.opt.record_order == 2 && p.sorted_records.p;
    kernel<<<grid, kBlock, 0, s>>>(
        reinterpret_cast<const uint2*>(own ? p.sorted_records.p : p.records.p), tex, p.tiles.p,
        p.pair_desc.p, p.pair_rel.p, p.partials.p, EXT ? p.ext_partials.p : nullptr,
        p.dz_index.p, dz, p.pair_scale.p, own ? p.pair_shift.p : nullptr,
        compacted_launch(p) ? p.qbegin_d.p : p.xcd_begin_d.p,
        compacted_launch(p) ? p.tile_list.p : nullptr, nq, p.counters.p,
        std::max(1, 16384 / p.tile_size), p.params.huber_delta, p.params.z_min);
    EPO_CHECK_LAUNCH();
}

template <int FMT, bool EXT>
void launch_cost_fmt(Plan& p, float* dz, hipStream_t s) {
    switch (p.opt.points_per_thread) {
        case 1: launch_cost_kernel<FMT, 1, EXT>(p, dz, s); break;
        case 2: launch_cost_kernel<FMT, 2, EXT>(p, dz, s); break;
        case 4: launch_cost_kernel<FMT, 4, EXT>(p, dz, s); break;
        case 8: launch_cost_kernel<FMT, 8, EXT>(p, dz, s); break;
        case 16: launch_cost_kernel<FMT, 16, EXT>(p, dz, s); break;
        default: throw Failure{EPO_ERR_UNSUPPORTED, "points_per_thread must be 1, 2, 4, 8 or 16"};
    }
}

template <bool EXT>
void launch_cost_variant(Plan& p, float* dz, hipStream_t s) {
    if (p.opt.texture_format == 2)
        launch_cost_fmt<2, EXT>(p, dz, s);
    else if (p.opt.texture_format == 3)
        launch_cost_fmt<3, EXT>(p, dz, s);
    else
        launch_cost_fmt<1, EXT>(p, dz, s);
}

}  // namespace

// this step's pair subset (stochastic sub-sampling, stopped scenes skipped),
// if enabled, the compacted list of its tiles, and the pair descriptors
static void launch_pair_setup(Plan& p, const double* poses, const float* lambda, hipStream_t s,
                              const ScheduleArgs* sched) {
    launch_pair_selection(p, p.capture_step ? p.capture_step : p.sample_step, s);
    const int threads = std::max({p.D, 16, sched ? sched->S : 0});
    pair_setup_kernel<<<(unsigned)ceil_div(threads, 256), 256, 0, s>>>(
        poses, p.K_d.p, p.wh_d.p, p.view_offset_d.p,
        p.opt.texture_format == 2 ? p.blk_off_d.p : nullptr, p.pair_static.p, lambda,
        p.params.lambda_max, p.pair_desc.p, p.pair_rel.p, p.D, p.counters.p, 8, p.status.p,
        sched ? *sched : ScheduleArgs{});
    EPO_CHECK_LAUNCH();
}

void launch_tiles(Plan& p, const double* poses, const float* lambda, hipStream_t s,
                  const RefineOut* ext, const ScheduleArgs* sched) {
    if (p.D == 0) return;
    launch_pair_setup(p, poses, lambda, s, sched);
    const bool timed = p.timing;
    if (timed) EPO_HIP(hipEventRecord(p.ev0, s));
    // the refinement variant runs for focal gradients, and for depth
    // gradients when the per-residual derivatives can be stored
    const bool depth = ext && (ext->grad_alpha || ext->grad_beta);
    float* dz = depth && p.dz.p ? p.dz.p : nullptr;
    if (ext && (ext->grad_gamma || dz))
        launch_cost_variant<true>(p, dz, s);
    else
        launch_cost_variant<false>(p, nullptr, s);
    if (timed) {
        EPO_HIP(hipEventRecord(p.ev1, s));
        p.timed_once = true;
    }
}

void launch_cost(Plan& p, const double* poses, const float* lambda, double* loss,
                 double* pair_cost, int32_t* pair_valid, double* pair_grad, double* grad,
                 const double* upstream, hipStream_t s, const RefineOut* ext,
                 const ScheduleArgs* sched) {
    launch_tiles(p, poses, lambda, s, ext, sched);
    launch_reductions(p, loss, pair_cost, pair_valid, pair_grad, grad, upstream, s,
                      ext ? ext->grad_gamma : nullptr);
    if (ext && (ext->grad_alpha || ext->grad_beta))
        launch_depth_grad(p, upstream, ext->grad_alpha, ext->grad_beta, p.D > 0 && p.dz.p, s);
}

}  // namespace epo

extern "C" epo_status epo_edge_cost_fwd(epo_plan plan, const double* poses, const float* lambda,
                                        double* loss, double* pair_cost, int32_t* pair_valid,
                                        double* pair_grad, double* grad, void* stream) {
    using namespace epo;
    return guarded([&] {
        EPO_REQUIRE(plan, "null plan");
        EPO_REQUIRE(poses && lambda && loss, "poses, lambda and loss are required");
        Plan& p = *reinterpret_cast<Plan*>(plan);
        EPO_HIP(hipSetDevice(p.device));
        launch_cost(p, poses, lambda, loss, pair_cost, pair_valid, pair_grad, grad, nullptr,
                    as_stream(stream));
    });
}

extern "C" epo_status epo_plan_time_kernel(epo_plan plan, const double* poses,
                                           const float* lambda, int32_t reps, float* ms,
                                           void* stream) {
    using namespace epo;
    return guarded([&] {
        EPO_REQUIRE(plan && poses && lambda && ms, "null argument");
        EPO_REQUIRE(reps >= 1 && reps <= 100000, "reps must be in [1, 100000]");
        Plan& p = *reinterpret_cast<Plan*>(plan);
        EPO_HIP(hipSetDevice(p.device));
        hipStream_t s = as_stream(stream);
        *ms = 0.0f;
        if (p.D == 0) return;
        launch_pair_setup(p, poses, lambda, s, nullptr);
        EPO_HIP(hipStreamSynchronize(s));
        // `reps` launches of the kernel captured as one graph (the way a
        // captured iteration launches it), replayed once to warm up and once
        // between two events on `stream`
        hipStream_t cs = nullptr;
        hipGraph_t g = nullptr;
        hipGraphExec_t ge = nullptr;
        hipEvent_t a = nullptr, b = nullptr;
        auto cleanup = [&] {
            if (ge) (void)hipGraphExecDestroy(ge);
            if (g) (void)hipGraphDestroy(g);
            if (cs) (void)hipStreamDestroy(cs);
            if (a) (void)hipEventDestroy(a);
            if (b) (void)hipEventDestroy(b);
        };
        try {
            EPO_HIP(hipStreamCreateWithFlags(&cs, hipStreamNonBlocking));
            EPO_HIP(hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal));
            try {
                for (int k = 0; k < reps; ++k) launch_cost_variant<false>(p, nullptr, cs);
            } catch (...) {
                hipGraph_t junk = nullptr;
                (void)hipStreamEndCapture(cs, &junk);
                if (junk) (void)hipGraphDestroy(junk);
                throw;
            }
            EPO_HIP(hipStreamEndCapture(cs, &g));
            EPO_HIP(hipGraphInstantiate(&ge, g, nullptr, nullptr, 0));
            EPO_HIP(hipEventCreate(&a));
            EPO_HIP(hipEventCreate(&b));
            EPO_HIP(hipGraphLaunch(ge, s));
            EPO_HIP(hipEventRecord(a, s));
            EPO_HIP(hipGraphLaunch(ge, s));
            EPO_HIP(hipEventRecord(b, s));
            EPO_HIP(hipEventSynchronize(b));
            float total = 0.0f;
            EPO_HIP(hipEventElapsedTime(&total, a, b));
            *ms = total / (float)reps;
        } catch (...) {
            cleanup();
            throw;
        }
        cleanup();
    });
}

extern "C" epo_status epo_edge_cost_bwd(epo_plan plan, const double* poses, const float* lambda,
                                        const double* upstream, double* grad, void* stream) {
    using namespace epo;
    return guarded([&] {
        EPO_REQUIRE(plan, "null plan");
        EPO_REQUIRE(poses && lambda && grad, "poses, lambda and grad are required");
        Plan& p = *reinterpret_cast<Plan*>(plan);
        EPO_HIP(hipSetDevice(p.device));
        launch_cost(p, poses, lambda, nullptr, nullptr, nullptr, nullptr, grad, upstream,
                    as_stream(stream));
    });
}
