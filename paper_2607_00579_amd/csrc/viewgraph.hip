// Viewgraph estimation by cycle-consistent reprojection (paper Sec. 3
// "Viewgraph Estimation", Sec. 4 "Implementation Details"; supplementary
// construction kernels): for a candidate pair (i, j) every pixel p of a grid
// over image i with a depth is projected into j, p_ij = pi(K_i, K_j, P_i, P_j,
// Z_i; p), and back, p_iji = pi(K_j, K_i, P_j, P_i, Z_j; p_ij) with Z_j read at
// the pixel nearest to p_ij; p is consistent when |p - p_iji|^2 < tau^2, and
// the pair is valid when at least min_fraction of its grid points with depth
// are consistent.
//
// The decisions (inside, depth present, consistent) are integers decided by
// floating point, so they are taken in float64 with contraction off and the
// operations in a fixed order: every step is one correctly rounded IEEE
// operation, the same ones a plain float64 evaluation in that order performs.
//
// One workgroup per (candidate, chunk of 1024 grid points), four points per
// thread; per-workgroup counts are added to the candidate's integer counters
// with atomics (integer sums: the result does not depend on the order).
#include <mutex>
#include <vector>

#include "epo_internal.h"

namespace epo {
namespace {

constexpr int kChunk = 1024;

struct Cam {
    double fx, fy, cx, cy;
    double R[9], t[3];
};

__device__ inline Cam load_cam(const float* __restrict__ K, const double* __restrict__ poses,
                               int v) {
    Cam c;
    c.fx = (double)K[4 * v];
    c.fy = (double)K[4 * v + 1];
    c.cx = (double)K[4 * v + 2];
    c.cy = (double)K[4 * v + 3];
    for (int r = 0; r < 3; ++r) {
        for (int k = 0; k < 3; ++k) c.R[3 * r + k] = poses[12 * v + 4 * r + k];
        c.t[r] = poses[12 * v + 4 * r + 3];
    }
    return c;
}

// pi(K_s, K_t, P_s, P_t, Z; (x, y)) -> (u', v') and the target depth z'
__device__ inline void project(double x, double y, double Z, const Cam& s, const Cam& t,
                               double& u, double& v, double& z) {
#pragma clang fp contract(off)
    const double X0 = (x - s.cx) / s.fx * Z;
    const double X1 = (y - s.cy) / s.fy * Z;
    const double X2 = Z;
    const double d0 = X0 - s.t[0], d1 = X1 - s.t[1], d2 = X2 - s.t[2];
    // world point R_s^T (X_c - t_s)
    const double W0 = (s.R[0] * d0 + s.R[3] * d1) + s.R[6] * d2;
    const double W1 = (s.R[1] * d0 + s.R[4] * d1) + s.R[7] * d2;
    const double W2 = (s.R[2] * d0 + s.R[5] * d1) + s.R[8] * d2;
    // target camera R_t X_w + t_t
    const double Y0 = ((t.R[0] * W0 + t.R[1] * W1) + t.R[2] * W2) + t.t[0];
    const double Y1 = ((t.R[3] * W0 + t.R[4] * W1) + t.R[5] * W2) + t.t[1];
    const double Y2 = ((t.R[6] * W0 + t.R[7] * W1) + t.R[8] * W2) + t.t[2];
    u = t.fx * (Y0 / Y2) + t.cx;
    v = t.fy * (Y1 / Y2) + t.cy;
    z = Y2;
}

__global__ __launch_bounds__(256) void viewgraph_kernel(
    const int2* __restrict__ blocks, const int2* __restrict__ cand,
    const int32_t* __restrict__ wh, const int64_t* __restrict__ view_off,
    const float* __restrict__ K, const double* __restrict__ poses,
    const float* __restrict__ depth, int32_t stride, double tau2, double z_min,
    int32_t* __restrict__ consistent, int32_t* __restrict__ total) {
#pragma clang fp contract(off)
    __shared__ int part[2][4];
    const int2 b = blocks[blockIdx.x];            // (candidate, chunk)
    const int2 ij = cand[b.x];
    const int i = ij.x, j = ij.y;
    const int Wi = wh[2 * i], Hi = wh[2 * i + 1];
    const int Wj = wh[2 * j], Hj = wh[2 * j + 1];
    const int nx = (Wi + stride - 1) / stride, ny = (Hi + stride - 1) / stride;
    const Cam ci = load_cam(K, poses, i), cj = load_cam(K, poses, j);
    const float* __restrict__ Zi = depth + view_off[i];
    const float* __restrict__ Zj = depth + view_off[j];
    int n_cons = 0, n_tot = 0;
    for (int r = 0; r < kChunk / 256; ++r) {
        const int k = b.y * kChunk + r * 256 + (int)threadIdx.x;
        if (k >= nx * ny) break;
        const int gx = (k % nx) * stride, gy = (k / nx) * stride;
        const float zf = Zi[(int64_t)gy * Wi + gx];
        if (!(isfinite(zf) && zf > 0.0f)) continue;
        ++n_tot;
        const double x = (double)gx, y = (double)gy;
        double u, v, z;
        project(x, y, (double)zf, ci, cj, u, v, z);
        if (!(z > z_min)) continue;
        const double ur = floor(u + 0.5), vr = floor(v + 0.5);
        if (!(ur >= 0.0 && ur < (double)Wj && vr >= 0.0 && vr < (double)Hj)) continue;
        const float zj = Zj[(int64_t)vr * Wj + (int64_t)ur];
        if (!(isfinite(zj) && zj > 0.0f)) continue;
        double u2, v2, z2;
        project(u, v, (double)zj, cj, ci, u2, v2, z2);
        if (!(z2 > z_min)) continue;
        const double e0 = u2 - x, e1 = v2 - y;
        if (e0 * e0 + e1 * e1 < tau2) ++n_cons;
    }
#pragma unroll
    for (int m = 32; m >= 1; m >>= 1) {
        n_cons += __shfl_xor(n_cons, m, 64);
        n_tot += __shfl_xor(n_tot, m, 64);
    }
    if ((threadIdx.x & 63) == 0) {
        part[0][threadIdx.x >> 6] = n_cons;
        part[1][threadIdx.x >> 6] = n_tot;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        const int c = part[0][0] + part[0][1] + part[0][2] + part[0][3];
        const int t = part[1][0] + part[1][1] + part[1][2] + part[1][3];
        if (c) atomicAdd(&consistent[b.x], c);
        if (t) atomicAdd(&total[b.x], t);
    }
}

__global__ __launch_bounds__(256) void viewgraph_zero_kernel(int32_t* __restrict__ a,
                                                             int32_t* __restrict__ b, int32_t n) {
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k < n) {
        a[k] = 0;
        b[k] = 0;
    }
}

__global__ __launch_bounds__(256) void viewgraph_valid_kernel(const int32_t* __restrict__ cons,
                                                              const int32_t* __restrict__ tot,
                                                              double min_fraction, int32_t n,
                                                              uint8_t* __restrict__ valid) {
#pragma clang fp contract(off)
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k < n) valid[k] = (tot[k] > 0 && (double)cons[k] >= min_fraction * (double)tot[k]) ? 1 : 0;
}

// host-side staging of one call: validated arguments, per-view sizes, the
// candidates and the (candidate, grid chunk) work list
struct ViewgraphStaging {
    std::vector<int32_t> wh;
    std::vector<int2> cand, blocks;
};

void prepare_viewgraph(int32_t n_views, const int32_t* width, const int32_t* height,
                       const float* K, const int64_t* view_offset, const float* depth,
                       const double* poses, const int32_t* candidates, int32_t n_candidates,
                       int32_t stride, double tau, double min_fraction, double z_min,
                       int32_t* consistent, int32_t* total, ViewgraphStaging& h) {
    EPO_REQUIRE(n_views >= 1, "n_views must be >= 1");
    EPO_REQUIRE(n_candidates >= 0, "n_candidates must be >= 0");
    EPO_REQUIRE(width && height && K && view_offset, "null host argument");
    EPO_REQUIRE(n_candidates == 0 || (candidates && depth && poses && consistent && total),
                "null argument");
    EPO_REQUIRE(stride >= 1 && stride <= 1024, "stride must be in [1, 1024]");
    EPO_REQUIRE(tau > 0 && std::isfinite(tau), "tau must be > 0");
    EPO_REQUIRE(min_fraction >= 0 && min_fraction <= 1, "min_fraction must be in [0, 1]");
    EPO_REQUIRE(z_min > 0 && std::isfinite(z_min), "z_min must be > 0");
    h.wh.assign(2 * (size_t)n_views, 0);
    for (int v = 0; v < n_views; ++v) {
        EPO_REQUIRE(width[v] >= 1 && width[v] <= EPO_MAX_SIDE && height[v] >= 1 &&
                        height[v] <= EPO_MAX_SIDE,
                    "view " + std::to_string(v) + ": side out of [1, 16384]");
        EPO_REQUIRE(view_offset[v] >= 0, "view " + std::to_string(v) + ": negative offset");
        EPO_REQUIRE(std::isfinite(K[4 * v]) && std::isfinite(K[4 * v + 1]) &&
                        K[4 * v] != 0.0f && K[4 * v + 1] != 0.0f &&
                        std::isfinite(K[4 * v + 2]) && std::isfinite(K[4 * v + 3]),
                    "view " + std::to_string(v) + ": intrinsics must be finite, focal != 0");
        h.wh[2 * v] = width[v];
        h.wh[2 * v + 1] = height[v];
    }
    h.cand.assign((size_t)n_candidates, make_int2(0, 0));
    h.blocks.clear();
    for (int c = 0; c < n_candidates; ++c) {
        const int i = candidates[2 * c], j = candidates[2 * c + 1];
        EPO_REQUIRE(i >= 0 && i < n_views && j >= 0 && j < n_views,
                    "candidate " + std::to_string(c) + ": view index out of range");
        h.cand[c] = make_int2(i, j);
        const int64_t pts = (int64_t)((width[i] + stride - 1) / stride) *
                            ((height[i] + stride - 1) / stride);
        for (int64_t k = 0; k < pts; k += kChunk) h.blocks.push_back(make_int2(c, (int)(k / kChunk)));
    }
    EPO_REQUIRE((int64_t)h.blocks.size() < (int64_t)INT32_MAX, "too many grid chunks");
}

// device copies of the staging arrays (wherever they live), then the kernels;
// synchronises the stream (the host staging is freed on return)
void run_viewgraph(const ViewgraphStaging& h, int32_t n_views, const float* K,
                   const int64_t* view_offset, const float* depth, const double* poses,
                   int32_t n_candidates, int32_t stride, double tau, double min_fraction,
                   double z_min, int32_t* consistent, int32_t* total, uint8_t* valid, int2* cand_d,
                   int2* blocks_d, int32_t* wh_d, int64_t* off_d, float* K_d, hipStream_t s) {
    EPO_HIP(hipMemcpyAsync(cand_d, h.cand.data(), sizeof(int2) * h.cand.size(),
                           hipMemcpyHostToDevice, s));
    if (!h.blocks.empty())
        EPO_HIP(hipMemcpyAsync(blocks_d, h.blocks.data(), sizeof(int2) * h.blocks.size(),
                               hipMemcpyHostToDevice, s));
    EPO_HIP(hipMemcpyAsync(wh_d, h.wh.data(), sizeof(int32_t) * h.wh.size(),
                           hipMemcpyHostToDevice, s));
    EPO_HIP(hipMemcpyAsync(off_d, view_offset, sizeof(int64_t) * n_views, hipMemcpyHostToDevice,
                           s));
    EPO_HIP(hipMemcpyAsync(K_d, K, sizeof(float) * 4 * n_views, hipMemcpyHostToDevice, s));
    viewgraph_zero_kernel<<<(unsigned)ceil_div(n_candidates, 256), 256, 0, s>>>(
        consistent, total, n_candidates);
    EPO_CHECK_LAUNCH();
    if (!h.blocks.empty()) {
        viewgraph_kernel<<<(unsigned)h.blocks.size(), 256, 0, s>>>(
            blocks_d, cand_d, wh_d, off_d, K_d, poses, depth, stride, tau * tau, z_min,
            consistent, total);
        EPO_CHECK_LAUNCH();
    }
    if (valid) {
        viewgraph_valid_kernel<<<(unsigned)ceil_div(n_candidates, 256), 256, 0, s>>>(
            consistent, total, min_fraction, n_candidates, valid);
        EPO_CHECK_LAUNCH();
    }
    EPO_HIP(hipStreamSynchronize(s));
}

// ---------------------------------------------------------------------------
// staging without allocation: a file-scope device array of a fixed size.
// Host code never passes the array's name to a kernel or a copy (there it is
// a host-side stand-in); it takes the array's device address once per device
// with hipGetSymbolAddress and uses that address.
// ---------------------------------------------------------------------------
constexpr size_t kStaticStagingBytes = size_t(4) << 20;
constexpr int kMaxDevices = 64;
std::mutex g_staging_mu;
void* g_staging_ptr[kMaxDevices] = {};

}  // namespace

static __device__ __align__(256) unsigned char scratch[kStaticStagingBytes];

namespace {

// the current device's copy of `scratch` (each GPU holds its own, at its own
// address), looked up on the first call on that device
char* static_staging() {
    int dev = 0;
    EPO_HIP(hipGetDevice(&dev));
    EPO_REQUIRE(dev >= 0 && dev < kMaxDevices, "device index out of range");
    std::lock_guard<std::mutex> lock(g_staging_mu);
    if (!g_staging_ptr[dev]) {
        void* ptr = nullptr;
        EPO_HIP(hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)));
        EPO_REQUIRE(ptr != nullptr, "no device address for the static staging array");
        g_staging_ptr[dev] = ptr;
    }
    return static_cast<char*>(g_staging_ptr[dev]);
}

size_t align256(size_t x) { return (x + 255) & ~size_t(255); }

}  // namespace
}  // namespace epo

using namespace epo;

extern "C" epo_status epo_build_viewgraph(int32_t n_views, const int32_t* width,
                                          const int32_t* height, const float* K,
                                          const int64_t* view_offset, const float* depth,
                                          const double* poses, const int32_t* candidates,
                                          int32_t n_candidates, int32_t stride, double tau,
                                          double min_fraction, double z_min,
                                          int32_t* consistent, int32_t* total, uint8_t* valid,
                                          void* stream) {
    return guarded([&] {
        ViewgraphStaging h;
        prepare_viewgraph(n_views, width, height, K, view_offset, depth, poses, candidates,
                          n_candidates, stride, tau, min_fraction, z_min, consistent, total, h);
        if (n_candidates == 0) return;
        DevBuf<int2> cand_d, blocks_d;
        DevBuf<int32_t> wh_d;
        DevBuf<int64_t> off_d;
        DevBuf<float> K_d;
        cand_d.alloc(h.cand.size());
        blocks_d.alloc(std::max<size_t>(h.blocks.size(), 1));
        wh_d.alloc(h.wh.size());
        off_d.alloc(n_views);
        K_d.alloc(4 * (size_t)n_views);
        run_viewgraph(h, n_views, K, view_offset, depth, poses, n_candidates, stride, tau,
                      min_fraction, z_min, consistent, total, valid, cand_d.p, blocks_d.p, wh_d.p,
                      off_d.p, K_d.p, as_stream(stream));
    });
}

extern "C" epo_status epo_build_viewgraph_noalloc(
    int32_t n_views, const int32_t* width, const int32_t* height, const float* K,
    const int64_t* view_offset, const float* depth, const double* poses,
    const int32_t* candidates, int32_t n_candidates, int32_t stride, double tau,
    double min_fraction, double z_min, int32_t* consistent, int32_t* total, uint8_t* valid,
    void* stream) {
    return guarded([&] {
        ViewgraphStaging h;
        prepare_viewgraph(n_views, width, height, K, view_offset, depth, poses, candidates,
                          n_candidates, stride, tau, min_fraction, z_min, consistent, total, h);
        if (n_candidates == 0) return;
        // the staging arrays one after another, each 256-byte aligned
        const size_t o_cand = 0;
        const size_t o_blk = align256(o_cand + sizeof(int2) * h.cand.size());
        const size_t o_wh = align256(o_blk + sizeof(int2) * std::max<size_t>(h.blocks.size(), 1));
        const size_t o_off = align256(o_wh + sizeof(int32_t) * h.wh.size());
        const size_t o_K = align256(o_off + sizeof(int64_t) * (size_t)n_views);
        const size_t need = o_K + sizeof(float) * 4 * (size_t)n_views;
        EPO_REQUIRE(need <= kStaticStagingBytes,
                    "the call needs " + std::to_string(need) + " bytes of staging (" +
                        std::to_string(n_candidates) + " candidates, " +
                        std::to_string(h.blocks.size()) + " grid chunks, " +
                        std::to_string(n_views) + " views), more than the " +
                        std::to_string(kStaticStagingBytes) +
                        " of the no-allocation form: use epo_build_viewgraph, fewer "
                        "candidates or a larger stride");
        char* base = static_staging();
        run_viewgraph(h, n_views, K, view_offset, depth, poses, n_candidates, stride, tau,
                      min_fraction, z_min, consistent, total, valid,
                      reinterpret_cast<int2*>(base + o_cand), reinterpret_cast<int2*>(base + o_blk),
                      reinterpret_cast<int32_t*>(base + o_wh),
                      reinterpret_cast<int64_t*>(base + o_off), reinterpret_cast<float*>(base + o_K),
                      as_stream(stream));
    });
}
