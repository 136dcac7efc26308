// Exact squared Euclidean distance transform on gfx950 (two separable 1-D
// passes, the structure of Felzenszwalb-Huttenlocher), the distance transform
// field of the paper's Sec. 3 and supplementary Sec. A1.2 "Construction
// kernels".
//
//   column pass  f(x, y) = squared distance to the nearest edge pixel of
//                column x (EPO_D2_EMPTY if the column has none).  One thread
//                per (column, 64-row segment): it looks up and down from its
//                segment for the nearest edge outside it, then sweeps the
//                segment down and up.  The 64 threads of a wave take 64
//                adjacent columns, so every step is one coalesced access, and
//                the segments give every view H/64 times the waves of a
//                thread-per-column pass.
//   row pass     d2(x, y) = min over q of f(q, y) + (x - q)^2.  One workgroup
//                per row stages f of the row in LDS; for each x the search
//                widens r = 1, 2, ... on both sides while r^2 is below the
//                best value found so far (every q at distance r adds at
//                least r^2), so a pixel costs about twice its distance to
//                the nearest edge instead of a sequential envelope per row.
//                Integer arithmetic throughout: the exact minimum.  The same
//                kernel writes DTF = sqrt(d2) in float32.
//
// Views are processed in batches whose descriptors travel as a kernel
// argument, so the call needs no device allocation.
#include "epo_internal.h"

namespace epo {
namespace {

// views per launch: their descriptors (16 B each) fill most of the 4 KB of
// kernel arguments
constexpr int kEdtBatch = 240;
constexpr int32_t kInf = EPO_D2_EMPTY;
constexpr int kSeg = 64;                 // rows per column-pass thread

struct EdtBatch {
    int32_t n;
    int32_t w[kEdtBatch];
    int32_t h[kEdtBatch];
    int64_t off[kEdtBatch];
};
static_assert(sizeof(EdtBatch) <= 4000, "EDT batch descriptors exceed the kernel-argument space");

__global__ __launch_bounds__(64) void edt_columns(const uint8_t* __restrict__ edge,
                                                  int32_t* __restrict__ colsq, EdtBatch b) {
    const int k = blockIdx.z;
    const int W = b.w[k], H = b.h[k];
    const int x = blockIdx.x * blockDim.x + threadIdx.x;
    const int y0 = blockIdx.y * kSeg;
    if (x >= W || y0 >= H) return;
    const int y1 = min(y0 + kSeg, H);
    const uint8_t* e = edge + b.off[k] + x;
    int32_t* out = colsq + b.off[k] + x;
    int last = -1;                       // row of the nearest edge at or above
    for (int y = y0 - 1; y >= 0; --y) {
        if (e[(int64_t)y * W]) {
            last = y;
            break;
        }
    }
#pragma unroll 8
    for (int y = y0; y < y1; ++y) {
        const int64_t o = (int64_t)y * W;
        if (e[o]) last = y;
        out[o] = last >= 0 ? (y - last) : -1;
    }
    int next = -1;                       // row of the nearest edge at or below
    for (int y = y1; y < H; ++y) {
        if (e[(int64_t)y * W]) {
            next = y;
            break;
        }
    }
#pragma unroll 8
    for (int y = y1 - 1; y >= y0; --y) {
        const int64_t o = (int64_t)y * W;
        if (e[o]) next = y;
        int best = out[o];
        if (next >= 0 && (best < 0 || next - y < best)) best = next - y;
        out[o] = best >= 0 ? best * best : kInf;
    }
}

// One workgroup per row.  The row's column-pass values live in dtf (the
// call's scratch); the workgroup reads all of them into LDS before any of its
// threads writes the row's DTF, and no other workgroup touches the row.
__global__ __launch_bounds__(256) void edt_rows(const int32_t* __restrict__ colsq,
                                               int32_t* __restrict__ d2, float* __restrict__ dtf,
                                               EdtBatch b) {
    extern __shared__ int32_t row[];
    const int k = blockIdx.y;
    const int W = b.w[k], H = b.h[k];
    const int y = blockIdx.x;
    if (y >= H) return;                  // whole workgroup
    const int64_t base = b.off[k] + (int64_t)y * W;
    for (int x = threadIdx.x; x < W; x += blockDim.x) row[x] = colsq[base + x];
    __syncthreads();
    for (int x = threadIdx.x; x < W; x += blockDim.x) {
        // f <= (H - 1)^2 < 2^28 or kInf = 2^30, r^2 < 2^28: no int32 overflow
        int32_t best = row[x];
        for (int r = 1; r * r < best && (x - r >= 0 || x + r < W); ++r) {
            if (x - r >= 0) best = min(best, row[x - r] + r * r);
            if (x + r < W) best = min(best, row[x + r] + r * r);
        }
        d2[base + x] = best;
        dtf[base + x] = sqrtf((float)best);
    }
}

}  // namespace
}  // namespace epo

extern "C" epo_status epo_build_distance_fields(const uint8_t* edge_maps, const int64_t* view_offset,
                                                const int32_t* width, const int32_t* height,
                                                int32_t n_views, int32_t* d2_out, float* dtf_out,
                                                void* stream) {
    using namespace epo;
    return guarded([&] {
        EPO_REQUIRE(n_views >= 0, "n_views must be >= 0");
        if (n_views == 0) return;
        EPO_REQUIRE(edge_maps && view_offset && width && height && d2_out && dtf_out,
                    "null pointer argument");
        for (int32_t v = 0; v < n_views; ++v) {
            EPO_REQUIRE(width[v] >= 1 && width[v] <= EPO_MAX_SIDE && height[v] >= 1 &&
                            height[v] <= EPO_MAX_SIDE,
                        "view " + std::to_string(v) + ": side out of [1, 16384]");
            EPO_REQUIRE(view_offset[v] >= 0, "view " + std::to_string(v) + ": negative offset");
        }
        hipStream_t s = as_stream(stream);
        int32_t* colsq = reinterpret_cast<int32_t*>(dtf_out);   // column-pass scratch
        for (int32_t a = 0; a < n_views; a += kEdtBatch) {
            EdtBatch b{};
            b.n = std::min(kEdtBatch, n_views - a);
            int maxW = 1, maxH = 1;
            for (int k = 0; k < b.n; ++k) {
                b.w[k] = width[a + k];
                b.h[k] = height[a + k];
                b.off[k] = view_offset[a + k];
                maxW = std::max(maxW, b.w[k]);
                maxH = std::max(maxH, b.h[k]);
            }
            edt_columns<<<dim3((unsigned)ceil_div(maxW, 64), (unsigned)ceil_div(maxH, kSeg), b.n),
                          64, 0, s>>>(edge_maps, colsq, b);
            EPO_CHECK_LAUNCH();
            edt_rows<<<dim3((unsigned)maxH, b.n), 256, (size_t)maxW * sizeof(int32_t), s>>>(
                colsq, d2_out, dtf_out, b);
            EPO_CHECK_LAUNCH();
        }
    });
}
