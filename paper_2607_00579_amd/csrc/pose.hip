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
#include "pose_update.h"
namespace {

// one thread per view; every thread reads the step counter, which is
// advanced after every workgroup has read it: by the last workgroup to
// finish when `done` is given (a counter at 0, rearmed here), else by
// advance_step_kernel in a launch of its own
__global__ __launch_bounds__(64) void pose_step_kernel(
    double* __restrict__ poses, double* __restrict__ m, double* __restrict__ w2,
    const double* __restrict__ grad, int32_t V, const int32_t* __restrict__ scene_of_view,
    const uint8_t* __restrict__ fixed, const double* __restrict__ lr, double b1, double b2,
    double eps, int32_t* __restrict__ step, int32_t* __restrict__ done) {
    const int s = step[0] + 1;
    const double bc1 = 1.0 - pow(b1, (double)s);
    const double bc2 = 1.0 - pow(b2, (double)s);
    const int v = blockIdx.x * blockDim.x + threadIdx.x;
    pose_update(v, poses, m, w2, grad, V, scene_of_view, fixed, lr, b1, b2, eps, bc1, bc2);
    if (done) {
        __shared__ int last;
        __syncthreads();                      // the workgroup has read the step
        if (threadIdx.x == 0) {
            __threadfence();
            last = atomicAdd(done, 1) == (int)gridDim.x - 1;
        }
        __syncthreads();
        if (last && threadIdx.x == 0) {
            step[0] = s;
            done[0] = 0;
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
    const ScheduleArgs a{step, l0, l1, anneal, peak, warmup, total, lam, lr, phase, S};
    float lv;
    double r;
    schedule_at(a, step[0], lv, r);
    for (int k = threadIdx.x; k < S; k += blockDim.x) {
        if (lam) lam[k] = lv;
        // a scene whose run has stopped (phase 2) keeps its poses
        if (lr) lr[k] = (phase && phase[k] == 2) ? 0.0 : r;
    }
}

}  // namespace

void launch_pose_step(double* poses, double* m, double* v, const double* grad, int32_t n_views,
                      const int32_t* scene_of_view, const uint8_t* fixed, const double* lr,
                      double b1, double b2, double eps, int32_t* step, hipStream_t s,
                      int32_t* done) {
    // one view per thread over the whole chip (the float64 exponential map is
    // a long dependent chain, so views are spread rather than looped over)
    if (n_views > 0) {
        pose_step_kernel<<<(unsigned)ceil_div(n_views, 64), 64, 0, s>>>(
            poses, m, v, grad, n_views, scene_of_view, fixed, lr, b1, b2, eps, step, done);
        EPO_CHECK_LAUNCH();
        if (done) return;
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
