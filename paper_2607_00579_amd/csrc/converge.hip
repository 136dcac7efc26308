// Pose-change signal and dual-phase convergence on the device (paper Sec. 3
// "Optimization Schedule", Alg. 2, Sec. A1.1), one workgroup per scene:
//   dR_v = (180/pi) acos((tr(R_v R_v'^T) - 1)/2),
//   dt_v = (180/pi) acos(t_v . t_v' / (|t_v| |t_v'|))      (' = previous step)
//   theta_95 = max(95th percentile of dR, 95th percentile of dt) over the
//              scene's poses (linear interpolation at rank (n - 1) 0.95);
//   Converged(w, eps): the w moving averages (window w) ending at the current
//   step are all below eps (needs 2w - 1 recorded steps).
// Phase 0 -> 1 when Converged(w1, eps1); phase 1 -> 2 (stopped) when
// Converged(w2, eps2) at a later step.  A stopped scene's learning rate is
// set to zero by the schedule kernel, so its poses stay fixed.
#include "epo_internal.h"

namespace epo {
namespace {

constexpr double kRadToDeg = 57.29577951308232;

__device__ inline double clamp1(double x) { return fmin(1.0, fmax(-1.0, x)); }

// value at ascending rank r (ties broken by index) of vals[0..n)
__device__ inline void rank_pick(const double* vals, int n, int r_lo, int r_hi, double* out) {
    for (int k = threadIdx.x; k < n; k += blockDim.x) {
        const double x = vals[k];
        int r = 0;
        for (int j = 0; j < n; ++j) {
            const double y = vals[j];
            r += (y < x) || (y == x && j < k);
        }
        if (r == r_lo) out[0] = x;
        if (r == r_hi) out[1] = x;
    }
}

__global__ __launch_bounds__(256) void convergence_kernel(
    const double* __restrict__ poses, double* __restrict__ prev,
    const int32_t* __restrict__ view_ptr, const int32_t* __restrict__ view_idx,
    ConvState* __restrict__ state, int32_t* __restrict__ phase, double* __restrict__ theta_out,
    int32_t w1, double eps1, int32_t w2, double eps2) {
    extern __shared__ double lds[];
    __shared__ double pick[4];
    __shared__ int below;
    const int s = blockIdx.x;
    const int a = view_ptr[s], n = view_ptr[s + 1] - a;
    double* dR = lds;
    double* dt = lds + n;
    for (int k = threadIdx.x; k < n; k += blockDim.x) {
        const int v = view_idx[a + k];
        const double* P = poses + 12 * v;
        double* Q = prev + 12 * v;
        double tr = 0.0, tp = 0.0, nn = 0.0, no = 0.0;
        for (int r = 0; r < 3; ++r)
            for (int c = 0; c < 3; ++c) tr += P[4 * r + c] * Q[4 * r + c];   // tr(R R'^T)
        for (int r = 0; r < 3; ++r) {
            tp += P[4 * r + 3] * Q[4 * r + 3];
            nn += P[4 * r + 3] * P[4 * r + 3];
            no += Q[4 * r + 3] * Q[4 * r + 3];
        }
        dR[k] = kRadToDeg * acos(clamp1((tr - 1.0) * 0.5));
        dt[k] = kRadToDeg * acos(clamp1(tp / (sqrt(nn) * sqrt(no))));
    }
    __syncthreads();
    const double r = (n - 1) * 0.95;
    const int lo = (int)floor(r);
    const int hi = min(lo + 1, n - 1);
    const double frac = r - lo;
    rank_pick(dR, n, lo, hi, pick);
    rank_pick(dt, n, lo, hi, pick + 2);
    __syncthreads();
    // the current poses become the previous ones
    for (int k = threadIdx.x; k < 12 * n; k += blockDim.x) {
        const int v = view_idx[a + k / 12];
        prev[12 * v + k % 12] = poses[12 * v + k % 12];
    }
    ConvState& st = state[s];
    if (threadIdx.x == 0) {
        const double pR = pick[0] + frac * (pick[1] - pick[0]);
        const double pt = pick[2] + frac * (pick[3] - pick[2]);
        const double th = fmax(pR, pt);
        st.theta[st.count % kConvRing] = th;
        st.count += 1;
        if (theta_out) theta_out[s] = th;
        below = 1;
    }
    __syncthreads();
    const int ph = st.phase;
    if (ph < 2) {
        const int w = ph == 0 ? w1 : w2;
        const double eps = ph == 0 ? eps1 : eps2;
        const int cnt = st.count;
        // the w moving averages ending at steps cnt-w .. cnt-1, one per thread
        int ok = 1;
        if (cnt < 2 * w - 1) {
            ok = 0;
        } else if ((int)threadIdx.x < w) {
            const int e = cnt - 1 - (int)threadIdx.x;      // last step of this window
            double sum = 0.0;
            for (int j = 0; j < w; ++j) sum += st.theta[(e - j) % kConvRing];
            ok = (sum / w) < eps;
        }
        const int all = __syncthreads_and(ok);
        if (threadIdx.x == 0 && all) {
            // phase 1 -> 2 is tested from the step after the 0 -> 1 switch
            if (ph == 0 || st.switch_step[0] < cnt - 1) {
                st.phase = ph + 1;
                st.switch_step[ph] = cnt - 1;
            }
        }
    }
    __syncthreads();
    if (threadIdx.x == 0) phase[s] = st.phase;
}

__global__ void convergence_reset_kernel(const double* __restrict__ poses,
                                         double* __restrict__ prev, int32_t n12,
                                         ConvState* __restrict__ state,
                                         int32_t* __restrict__ phase, int32_t S) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n12) prev[i] = poses[i];
    if (i < S) {
        state[i].phase = 0;
        state[i].count = 0;
        state[i].switch_step[0] = -1;
        state[i].switch_step[1] = -1;
        phase[i] = 0;
    }
}

}  // namespace

void launch_convergence(Plan& p, const double* poses, double* theta_out, hipStream_t s) {
    const size_t lds = 2 * sizeof(double) * (size_t)std::max(p.max_views_per_scene, 1);
    convergence_kernel<<<(unsigned)p.S, 256, lds, s>>>(
        poses, p.conv_prev.p, p.scene_view_ptr.p, p.scene_view_idx.p, p.conv_state.p,
        p.conv_phase.p, theta_out, p.conv.w1, (double)p.conv.eps1, p.conv.w2,
        (double)p.conv.eps2);
    EPO_CHECK_LAUNCH();
}

void launch_convergence_reset(Plan& p, const double* poses, hipStream_t s) {
    const int n = std::max(12 * p.V, p.S);
    convergence_reset_kernel<<<(unsigned)ceil_div(n, 256), 256, 0, s>>>(
        poses, p.conv_prev.p, 12 * p.V, p.conv_state.p, p.conv_phase.p, p.S);
    EPO_CHECK_LAUNCH();
}

}  // namespace epo

using namespace epo;

extern "C" epo_status epo_convergence_reset(epo_plan plan, const double* poses,
                                            const epo_convergence_params* params, void* stream) {
    return guarded([&] {
        EPO_REQUIRE(plan && poses, "null argument");
        Plan& p = *reinterpret_cast<Plan*>(plan);
        epo_convergence_params c = params ? *params : epo_convergence_params{25, 0.5f, 50, 0.1f};
        EPO_REQUIRE(c.w1 >= 1 && c.w2 >= 1 && 2 * std::max(c.w1, c.w2) - 1 <= kConvRing,
                    "convergence windows must be in [1, 64]");
        EPO_REQUIRE(c.eps1 > 0 && c.eps2 > 0, "convergence thresholds must be > 0");
        EPO_REQUIRE(p.max_views_per_scene <= kConvMaxViews,
                    "a scene has more views than the convergence kernel supports");
        EPO_HIP(hipSetDevice(p.device));
        p.conv = c;
        launch_convergence_reset(p, poses, as_stream(stream));
    });
}

extern "C" epo_status epo_convergence_update(epo_plan plan, const double* poses,
                                             double* theta95, int32_t* phase, void* stream) {
    return guarded([&] {
        EPO_REQUIRE(plan && poses, "null argument");
        Plan& p = *reinterpret_cast<Plan*>(plan);
        EPO_REQUIRE(p.max_views_per_scene <= kConvMaxViews,
                    "a scene has more views than the convergence kernel supports");
        EPO_HIP(hipSetDevice(p.device));
        hipStream_t s = as_stream(stream);
        launch_convergence(p, poses, theta95, s);
        if (phase)
            EPO_HIP(hipMemcpyAsync(phase, p.conv_phase.p, sizeof(int32_t) * p.S,
                                   hipMemcpyDeviceToDevice, s));
    });
}

extern "C" epo_status epo_convergence_query(epo_plan plan, int32_t* phase, double* theta_last,
                                            int32_t* switch_steps, int32_t* steps, void* stream) {
    return guarded([&] {
        EPO_REQUIRE(plan, "null plan");
        Plan& p = *reinterpret_cast<Plan*>(plan);
        EPO_HIP(hipSetDevice(p.device));
        hipStream_t s = as_stream(stream);
        std::vector<ConvState> st(p.S);
        EPO_HIP(hipMemcpyAsync(st.data(), p.conv_state.p, sizeof(ConvState) * p.S,
                               hipMemcpyDeviceToHost, s));
        EPO_HIP(hipStreamSynchronize(s));
        for (int k = 0; k < p.S; ++k) {
            if (phase) phase[k] = st[k].phase;
            if (steps) steps[k] = st[k].count;
            if (theta_last)
                theta_last[k] = st[k].count ? st[k].theta[(st[k].count - 1) % kConvRing] : 0.0;
            if (switch_steps) {
                switch_steps[2 * k] = st[k].switch_step[0];
                switch_steps[2 * k + 1] = st[k].switch_step[1];
            }
        }
    });
}
