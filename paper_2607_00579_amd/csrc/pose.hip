// Float64 pose update (Adam on left se(3) twists + SE(3) exponential) and the
// paper's clamp / learning-rate schedules evaluated on the device.
//
// Adam with beta = (0.9, 0.999) is the paper's optimizer (Sec. 4
// "Implementation Details"); the twist parameterization replaces its pose
// refiner network.  For every pose v not held fixed:
//   m <- b1 m + (1 - b1) g,  w <- b2 w + (1 - b2) g^2,
//   xi = -lr (m / (1 - b1^s)) / (sqrt(w / (1 - b2^s)) + eps),
//   [R | t] <- Exp(xi) [R | t],  Exp(rho, omega) = [R(omega) | V(omega) rho]
// with R(omega) = I + a [w]x + b [w]x^2, V = I + b [w]x + c [w]x^2,
// a = sin th / th, b = (1 - cos th)/th^2, c = (th - sin th)/th^3 (Taylor
// series below th = 1e-4).
#include "epo_internal.h"

namespace epo {
namespace {

__device__ inline void exp_coeffs(double th, double& a, double& b, double& c) {
    if (th < 1e-4) {
        const double t2 = th * th;
        a = 1.0 - t2 / 6.0;
        b = 0.5 - t2 / 24.0;
        c = 1.0 / 6.0 - t2 / 120.0;
    } else {
        const double s = sin(th), co = cos(th);
        a = s / th;
        b = (1.0 - co) / (th * th);
        c = (th - s) / (th * th * th);
    }
}

// one thread per view; every thread reads the step counter, which
// advance_step_kernel increments afterwards
__global__ __launch_bounds__(64) void pose_step_kernel(
    double* __restrict__ poses, double* __restrict__ m, double* __restrict__ w2,
    const double* __restrict__ grad, int32_t V, const int32_t* __restrict__ scene_of_view,
    const uint8_t* __restrict__ fixed, const double* __restrict__ lr, double b1, double b2,
    double eps, const int32_t* __restrict__ step) {
    const int s = step[0] + 1;
    const double bc1 = 1.0 - pow(b1, (double)s);
    const double bc2 = 1.0 - pow(b2, (double)s);
    const int v = blockIdx.x * blockDim.x + threadIdx.x;
    if (v < V && !(fixed && fixed[v])) {
        const double lr_v = lr[scene_of_view ? scene_of_view[v] : 0];
        double xi[6];
        for (int k = 0; k < 6; ++k) {
            const double g = grad[6 * v + k];
            const double mk = b1 * m[6 * v + k] + (1.0 - b1) * g;
            const double wk = b2 * w2[6 * v + k] + (1.0 - b2) * g * g;
            m[6 * v + k] = mk;
            w2[6 * v + k] = wk;
            xi[k] = -lr_v * (mk / bc1) / (sqrt(wk / bc2) + eps);
        }
        const double wx = xi[3], wy = xi[4], wz = xi[5];
        const double th = sqrt(wx * wx + wy * wy + wz * wz);
        double a, b, c;
        exp_coeffs(th, a, b, c);
        const double W[9] = {0.0, -wz, wy, wz, 0.0, -wx, -wy, wx, 0.0};
        double W2[9];
        for (int r = 0; r < 3; ++r)
            for (int q = 0; q < 3; ++q)
                W2[3 * r + q] = W[3 * r + 0] * W[0 + q] + W[3 * r + 1] * W[3 + q] +
                                W[3 * r + 2] * W[6 + q];
        double R[9], Vm[9];
        for (int k = 0; k < 9; ++k) {
            const double I = (k % 4 == 0) ? 1.0 : 0.0;
            R[k] = I + a * W[k] + b * W2[k];
            Vm[k] = I + b * W[k] + c * W2[k];
        }
        double tv[3];
        for (int r = 0; r < 3; ++r)
            tv[r] = Vm[3 * r + 0] * xi[0] + Vm[3 * r + 1] * xi[1] + Vm[3 * r + 2] * xi[2];
        // [R | tv] * [P ; 0 0 0 1]
        double P[12];
        for (int k = 0; k < 12; ++k) P[k] = poses[12 * v + k];
        for (int r = 0; r < 3; ++r) {
            for (int q = 0; q < 4; ++q) {
                double x = R[3 * r + 0] * P[0 + q] + R[3 * r + 1] * P[4 + q] +
                           R[3 * r + 2] * P[8 + q];
                if (q == 3) x += tv[r];
                poses[12 * v + 4 * r + q] = x;
            }
        }
    }
}

// the step counter advances after every view has read it (its own launch)
__global__ void advance_step_kernel(int32_t* step) { step[0] += 1; }

__global__ __launch_bounds__(256) void schedule_kernel(const int32_t* __restrict__ step,
                                                       int32_t S, float l0, float l1,
                                                       int32_t anneal, double peak,
                                                       int32_t warmup, int32_t total,
                                                       float* __restrict__ lam,
                                                       double* __restrict__ lr,
                                                       const int32_t* __restrict__ phase) {
    const int s = step[0];
    const double frac = anneal > 0 ? (double)min(s, anneal) / (double)anneal : 1.0;
    const float lv = (float)((double)l0 - ((double)l0 - (double)l1) * frac);
    double r;
    if (s < warmup)
        r = peak * (double)(s + 1) / (double)warmup;
    else
        r = peak * 0.5 * (1.0 + cos(M_PI * (double)(s - warmup) / (double)(total - warmup)));
    for (int k = threadIdx.x; k < S; k += blockDim.x) {
        if (lam) lam[k] = lv;
        // a scene whose run has stopped (phase 2) keeps its poses
        if (lr) lr[k] = (phase && phase[k] == 2) ? 0.0 : r;
    }
}

}  // namespace

void launch_pose_step(double* poses, double* m, double* v, const double* grad, int32_t n_views,
                      const int32_t* scene_of_view, const uint8_t* fixed, const double* lr,
                      double b1, double b2, double eps, int32_t* step, hipStream_t s) {
    // one view per thread over the whole chip (the float64 exponential map is
    // a long dependent chain, so views are spread rather than looped over)
    if (n_views > 0) {
        pose_step_kernel<<<(unsigned)ceil_div(n_views, 64), 64, 0, s>>>(
            poses, m, v, grad, n_views, scene_of_view, fixed, lr, b1, b2, eps, step);
        EPO_CHECK_LAUNCH();
    }
    advance_step_kernel<<<1, 1, 0, s>>>(step);
    EPO_CHECK_LAUNCH();
}

void launch_schedule(const int32_t* step, int32_t n_scenes, float lambda0, float lambda1,
                     int32_t anneal_steps, double peak_lr, int32_t warmup, int32_t total,
                     float* lambda_out, double* lr_out, const int32_t* phase, hipStream_t s) {
    schedule_kernel<<<1, 256, 0, s>>>(step, n_scenes, lambda0, lambda1, anneal_steps, peak_lr,
                                      warmup, total, lambda_out, lr_out, phase);
    EPO_CHECK_LAUNCH();
}

}  // namespace epo

extern "C" epo_status epo_pose_step(double* poses, double* adam_m, double* adam_v,
                                    const double* grad, int32_t n_views,
                                    const int32_t* scene_of_view, const uint8_t* fixed_mask,
                                    const double* lr, double beta1, double beta2, double eps,
                                    int32_t* step, void* stream) {
    using namespace epo;
    return guarded([&] {
        EPO_REQUIRE(n_views >= 0, "n_views must be >= 0");
        EPO_REQUIRE(poses && adam_m && adam_v && grad && lr && step, "null pointer argument");
        EPO_REQUIRE(beta1 >= 0 && beta1 < 1 && beta2 >= 0 && beta2 < 1 && eps >= 0,
                    "Adam constants out of range");
        launch_pose_step(poses, adam_m, adam_v, grad, n_views, scene_of_view, fixed_mask, lr,
                         beta1, beta2, eps, step, as_stream(stream));
    });
}

extern "C" epo_status epo_schedule(const int32_t* step, int32_t n_scenes, float lambda0,
                                   float lambda1, int32_t anneal_steps, double peak_lr,
                                   int32_t warmup, int32_t total, float* lambda_out,
                                   double* lr_out, void* stream) {
    using namespace epo;
    return guarded([&] {
        EPO_REQUIRE(step && n_scenes >= 1, "step pointer and n_scenes >= 1 required");
        EPO_REQUIRE(lambda_out || lr_out, "nothing to write");
        EPO_REQUIRE(warmup >= 1 && total > warmup && anneal_steps >= 0,
                    "schedule lengths out of range");
        launch_schedule(step, n_scenes, lambda0, lambda1, anneal_steps, peak_lr, warmup, total,
                        lambda_out, lr_out, nullptr, as_stream(stream));
    });
}
