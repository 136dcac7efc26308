// Exact squared Euclidean distance transform on gfx950 (two separable 1-D
// passes, the structure of Felzenszwalb-Huttenlocher), the distance transform
// field of the paper's Sec. 3 and supplementary Sec. A1.2 "Construction
// kernels".
//
//   column pass  f(x, y) = squared distance to the nearest edge pixel of
//                column x (EPO_D2_EMPTY if the column has none).  One thread
//                per (column, 64-row segment), in two kernels: the first
//                records each segment's first and last edge row (in d2, not
//                yet written); the second takes the nearest edge above and
//                below its segment from those records, then sweeps the
//                segment down and up, holding it in registers in between.  The 64 threads of a wave take 64
//                adjacent columns, so every step is one coalesced access, and
//                the segments give every view H/64 times the waves of a
//                thread-per-column pass.
//   row pass     d2(x, y) = min over q of f(q, y) + (x - q)^2.  One workgroup
//                per row stages f of the row and its minimum per 16-pixel
//                block in LDS; each x searches outward block by block,
//                scanning only blocks whose minimum plus the squared
//                distance could beat its best value, and stops when the
//                distance alone cannot (a parallel bounded search instead of
//                a sequential envelope per row).  Integer arithmetic
//                throughout: the exact minimum.  The same kernel writes
//                DTF = sqrt(d2) in float32.
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

// First pass over each (column, segment): the rows of its first and last
// edge pixel (-1 if none), packed as (first + 1) | (last + 1) << 16 into the
// segment's first row of d2, which is free until the row pass.
__global__ __launch_bounds__(64) void edt_segments(const uint8_t* __restrict__ edge,
                                                   int32_t* __restrict__ seg, EdtBatch b) {
    const int k = blockIdx.z;
    const int W = b.w[k], H = b.h[k];
    const int x = blockIdx.x * blockDim.x + threadIdx.x;
    const int y0 = blockIdx.y * kSeg;
    if (x >= W || y0 >= H) return;
    const int y1 = min(y0 + kSeg, H);
    const uint8_t* e = edge + b.off[k] + x;
    int first = -1, last = -1;
#pragma unroll 8
    for (int y = y0; y < y1; ++y) {
        if (e[(int64_t)y * W]) {
            if (first < 0) first = y;
            last = y;
        }
    }
    seg[b.off[k] + (int64_t)y0 * W + x] = (first + 1) | ((last + 1) << 16);
}

// The nearest edge above and below a segment comes from the other segments'
// summaries (at most H/64 coalesced reads, however far the edge is), then
// the segment is swept down and up.
__global__ __launch_bounds__(64) void edt_columns(const uint8_t* __restrict__ edge,
                                                  const int32_t* __restrict__ seg,
                                                  int32_t* __restrict__ colsq, EdtBatch b) {
    const int k = blockIdx.z;
    const int W = b.w[k], H = b.h[k];
    const int x = blockIdx.x * blockDim.x + threadIdx.x;
    const int s0 = blockIdx.y, y0 = s0 * kSeg;
    if (x >= W || y0 >= H) return;
    const int y1 = min(y0 + kSeg, H);
    const int n_seg = (H + kSeg - 1) / kSeg;
    const uint8_t* e = edge + b.off[k] + x;
    const int32_t* sm = seg + b.off[k] + x;
    int32_t* out = colsq + b.off[k] + x;
    int last = -1;                       // row of the nearest edge at or above
    for (int q = s0 - 1; q >= 0; --q) {
        const int32_t v = sm[(int64_t)q * kSeg * W];
        if (v >> 16) {
            last = (v >> 16) - 1;
            break;
        }
    }
    // the segment stays in registers between the two sweeps: the distance
    // to the edge above (-1: none) per row, and the rows' edge flags as bits
    int up[kSeg];
    uint64_t emask = 0;
#pragma unroll
    for (int i = 0; i < kSeg; ++i) {
        const int y = y0 + i;
        if (y < y1) {
            if (e[(int64_t)y * W]) {
                last = y;
                emask |= 1ull << i;
            }
            up[i] = last >= 0 ? (y - last) : -1;
        }
    }
    int next = -1;                       // row of the nearest edge at or below
    for (int q = s0 + 1; q < n_seg; ++q) {
        const int32_t v = sm[(int64_t)q * kSeg * W];
        if (v & 0xFFFF) {
            next = (v & 0xFFFF) - 1;
            break;
        }
    }
#pragma unroll
    for (int i = kSeg - 1; i >= 0; --i) {
        const int y = y0 + i;
        if (y < y1) {
            if ((emask >> i) & 1ull) next = y;
            int best = up[i];
            if (next >= 0 && (best < 0 || next - y < best)) best = next - y;
            out[(int64_t)y * W] = best >= 0 ? best * best : kInf;
        }
    }
}

// One workgroup per row.  The row's column-pass values live in dtf (the
// call's scratch); the workgroup reads all of them into LDS before any of its
// threads writes the row's DTF, and no other workgroup touches the row.
// The row is split into blocks of 16 pixels with their minimum f in LDS; a
// pixel scans its own block, then the blocks at block distance R = 1, 2, ...
// on both sides: a block is scanned only if its minimum plus the squared
// distance to its nearest pixel is below the best value so far, and the
// search ends once the nearer of the two blocks is at least sqrt(best) away
// (every farther pixel adds more).  Every pixel that can attain the minimum
// is scanned, so the result is the exact minimum, at about D/16 block tests
// per pixel (D its distance to the nearest edge).
constexpr int kRowBlk = 16;

__global__ __launch_bounds__(256) void edt_rows(const int32_t* __restrict__ colsq,
                                               int32_t* __restrict__ d2, float* __restrict__ dtf,
                                               EdtBatch b) {
    extern __shared__ int32_t lds[];
    const int k = blockIdx.y;
    const int W = b.w[k], H = b.h[k];
    const int y = blockIdx.x;
    if (y >= H) return;                  // whole workgroup
    const int nb = (W + kRowBlk - 1) / kRowBlk;
    int32_t* row = lds;
    int32_t* bmin = lds + W;
    const int64_t base = b.off[k] + (int64_t)y * W;
    for (int x = threadIdx.x; x < W; x += blockDim.x) row[x] = colsq[base + x];
    __syncthreads();
    for (int j = threadIdx.x; j < nb; j += blockDim.x) {
        int32_t m = row[kRowBlk * j];
        for (int q = kRowBlk * j + 1; q < min(kRowBlk * j + kRowBlk, W); ++q) m = min(m, row[q]);
        bmin[j] = m;
    }
    __syncthreads();
    // f <= (H - 1)^2 < 2^28 or kInf = 2^30, distances < 2^14: no int32 overflow
    for (int x = threadIdx.x; x < W; x += blockDim.x) {
        const int bx = x / kRowBlk;
        int32_t best = row[x];
        for (int q = kRowBlk * bx; q < min(kRowBlk * bx + kRowBlk, W); ++q)
            best = min(best, row[q] + (x - q) * (x - q));
        for (int R = 1;; ++R) {
            const int bl = bx - R, br = bx + R;
            const bool lin = bl >= 0, rin = kRowBlk * br < W;
            if (!lin && !rin) break;
            const int dl = x - (kRowBlk * bl + kRowBlk - 1);     // >= 1 when lin
            const int dr = kRowBlk * br - x;                    // >= 1 when rin
            const int dn = min(lin ? dl : 0x7fff, rin ? dr : 0x7fff);
            if (dn * dn >= best) break;
            if (lin && bmin[bl] + dl * dl < best) {
#pragma unroll
                for (int u = 0; u < kRowBlk; ++u) {
                    const int q = kRowBlk * bl + u;
                    best = min(best, row[q] + (x - q) * (x - q));
                }
            }
            if (rin && bmin[br] + dr * dr < best) {
#pragma unroll
                for (int u = 0; u < kRowBlk; ++u) {
                    const int q = kRowBlk * br + u;
                    if (q < W) best = min(best, row[q] + (x - q) * (x - q));
                }
            }
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
            const dim3 cgrid((unsigned)ceil_div(maxW, 64), (unsigned)ceil_div(maxH, kSeg), b.n);
            edt_segments<<<cgrid, 64, 0, s>>>(edge_maps, d2_out, b);
            EPO_CHECK_LAUNCH();
            edt_columns<<<cgrid, 64, 0, s>>>(edge_maps, d2_out, colsq, b);
            EPO_CHECK_LAUNCH();
            const size_t lds = (size_t)(maxW + ceil_div(maxW, kRowBlk)) * sizeof(int32_t);
            if (lds > 65536) {
                // rows wider than 15420 pixels: more than the default 64 KB of
                // dynamic LDS (gfx950 has 160 KB per workgroup); an error, never
                // a short allocation, if the device cannot give it
                int dev = 0, max_lds = 0;
                EPO_HIP(hipGetDevice(&dev));
                EPO_HIP(hipDeviceGetAttribute(&max_lds, hipDeviceAttributeMaxSharedMemoryPerBlock,
                                              dev));
                EPO_REQUIRE(lds <= (size_t)max_lds,
                            "rows too wide for the device's LDS per workgroup");
                EPO_HIP(hipFuncSetAttribute(reinterpret_cast<const void*>(edt_rows),
                                            hipFuncAttributeMaxDynamicSharedMemorySize,
                                            (int)lds));
            }
            edt_rows<<<dim3((unsigned)maxH, b.n), 256, lds, s>>>(colsq, d2_out, dtf_out, b);
            EPO_CHECK_LAUNCH();
        }
    });
}
