// The float64 pose update of one view (Adam on its left se(3) twist, then
// the SE(3) exponential), shared by the pose-step kernel and the small-plan
// step epilogue so that both give the same bits.  Included inside
// namespace epo.
#pragma once

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

// view v at the bias corrections bc1 = 1 - b1^s, bc2 = 1 - b2^s of step s
__device__ inline void pose_update(int v, double* __restrict__ poses, double* __restrict__ m,
                                   double* __restrict__ w2, const double* __restrict__ grad,
                                   int32_t V, const int32_t* __restrict__ scene_of_view,
                                   const uint8_t* __restrict__ fixed,
                                   const double* __restrict__ lr, double b1, double b2,
                                   double eps, double bc1, double bc2) {
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
