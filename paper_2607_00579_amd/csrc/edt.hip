// Exact squared Euclidean distance transform on gfx950 (Felzenszwalb-
// Huttenlocher, two 1-D passes), the distance transform field of the paper's
// Sec. 3 and supplementary Sec. A1.2 "Construction kernels".
//
//   column pass  one thread per image column, two sweeps: distance to the
//                nearest edge pixel above and below, squared (EPO_D2_EMPTY if
//                the column has none).  Threads of a wave read 64 adjacent
//                bytes of a row, so every sweep step is one coalesced access.
//   row pass     one thread per image row builds the lower envelope of the
//                parabolas f(q) + (x - q)^2 of its row; the stack of parabola
//                apexes lives in LDS (int16, padded row stride against bank
//                conflicts) and every breakpoint test is an exact int64
//                cross-multiplication, so the result is the exact integer
//                minimum.
//   sqrt pass    DTF = sqrt(d2) in float32.
//
// Views are processed in batches whose descriptors travel as a kernel
// argument, so the call needs no device allocation.
#include "epo_internal.h"

namespace epo {
namespace {

constexpr int kEdtBatch = 64;
constexpr int32_t kInf = EPO_D2_EMPTY;
constexpr int kRowLdsBudget = 64 * 1024;

struct EdtBatch {
    int32_t n;
    int32_t w[kEdtBatch];
    int32_t h[kEdtBatch];
    int64_t off[kEdtBatch];
};

__global__ __launch_bounds__(64) void edt_columns(const uint8_t* __restrict__ edge,
                                                  int32_t* __restrict__ colsq, EdtBatch b) {
    const int k = blockIdx.y;
    const int W = b.w[k], H = b.h[k];
    const int x = blockIdx.x * blockDim.x + threadIdx.x;
    if (x >= W) return;
    const uint8_t* e = edge + b.off[k] + x;
    int32_t* out = colsq + b.off[k] + x;
    int last = -1;                       // row of the nearest edge at or above
    for (int y = 0; y < H; ++y) {
        const int64_t o = (int64_t)y * W;
        if (e[o]) last = y;
        out[o] = last >= 0 ? (y - last) : -1;
    }
    int next = -1;                       // row of the nearest edge at or below
    for (int y = H - 1; y >= 0; --y) {
        const int64_t o = (int64_t)y * W;
        if (e[o]) next = y;
        int best = out[o];
        if (next >= 0 && (best < 0 || next - y < best)) best = next - y;
        out[o] = best >= 0 ? best * best : kInf;
    }
}

__global__ __launch_bounds__(64) void edt_rows(const int32_t* __restrict__ colsq,
                                               int32_t* __restrict__ d2, EdtBatch b,
                                               int rows_per_block, int stride16) {
    extern __shared__ int16_t stack_mem[];
    const int k = blockIdx.y;
    const int W = b.w[k], H = b.h[k];
    const int r = threadIdx.x;
    const int y = blockIdx.x * rows_per_block + r;
    if (r >= rows_per_block || y >= H) return;
    const int32_t* f = colsq + b.off[k] + (int64_t)y * W;
    int32_t* out = d2 + b.off[k] + (int64_t)y * W;
    int16_t* v = stack_mem + r * stride16;

    // lower envelope of the parabolas with finite height
    int n = 0;
    for (int q = 0; q < W; ++q) {
        const int32_t fq = f[q];
        if (fq >= kInf) continue;
        const int64_t Fq = (int64_t)fq + (int64_t)q * q;
        while (n >= 2) {
            const int p = v[n - 1], pp = v[n - 2];
            const int64_t Fp = (int64_t)f[p] + (int64_t)p * p;
            const int64_t Fpp = (int64_t)f[pp] + (int64_t)pp * pp;
            // meet(p, q) <= meet(pp, p): parabola p is nowhere lowest
            if ((Fq - Fp) * (int64_t)(p - pp) <= (Fp - Fpp) * (int64_t)(q - p)) {
                --n;
            } else {
                break;
            }
        }
        v[n++] = (int16_t)q;
    }
    if (n == 0) {
        for (int x = 0; x < W; ++x) out[x] = kInf;
        return;
    }
    int j = 0;
    int p = v[0];
    int64_t Fp = (int64_t)f[p] + (int64_t)p * p;
    for (int x = 0; x < W; ++x) {
        while (j + 1 < n) {
            const int q = v[j + 1];
            const int64_t Fq = (int64_t)f[q] + (int64_t)q * q;
            // meet(p, q) < x  <=>  Fq - Fp < 2 x (q - p)
            if (Fq - Fp < 2 * (int64_t)x * (q - p)) {
                ++j;
                p = q;
                Fp = Fq;
            } else {
                break;
            }
        }
        out[x] = f[p] + (x - p) * (x - p);
    }
}

__global__ __launch_bounds__(256) void edt_sqrt(const int32_t* __restrict__ d2,
                                                float* __restrict__ dtf, EdtBatch b) {
    const int k = blockIdx.y;
    const int64_t n = (int64_t)b.w[k] * b.h[k];
    const int64_t base = b.off[k];
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x) {
        dtf[base + i] = sqrtf((float)d2[base + i]);
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
            int64_t maxWH = 1;
            for (int k = 0; k < b.n; ++k) {
                b.w[k] = width[a + k];
                b.h[k] = height[a + k];
                b.off[k] = view_offset[a + k];
                maxW = std::max(maxW, b.w[k]);
                maxH = std::max(maxH, b.h[k]);
                maxWH = std::max(maxWH, (int64_t)b.w[k] * b.h[k]);
            }
            edt_columns<<<dim3((unsigned)ceil_div(maxW, 64), b.n), 64, 0, s>>>(edge_maps, colsq, b);
            EPO_CHECK_LAUNCH();
            // int16 stack per row, stride chosen so that the dword stride is odd
            int stride16 = (int)(2 * ceil_div(maxW, 2));
            if (((stride16 / 2) & 1) == 0) stride16 += 2;
            int rows = std::max(1, std::min(64, kRowLdsBudget / (2 * stride16)));
            size_t lds = (size_t)rows * stride16 * sizeof(int16_t);
            edt_rows<<<dim3((unsigned)ceil_div(maxH, rows), b.n), 64, lds, s>>>(colsq, d2_out, b,
                                                                                rows, stride16);
            EPO_CHECK_LAUNCH();
            unsigned gx = (unsigned)std::min<int64_t>(ceil_div(maxWH, 256), 2048);
            edt_sqrt<<<dim3(gx, b.n), 256, 0, s>>>(d2_out, dtf_out, b);
            EPO_CHECK_LAUNCH();
        }
    });
}
