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
// d2(x) = min over q of f(q) + (x - q)^2 is found by an exact search over a
// three-level hierarchy of minima in LDS: blocks of 16 pixels, groups of 16
// blocks (256 px), supers of 16 groups (4096 px).  A pixel scans its own
// block, then the other blocks of its group, the other groups of its super,
// and the other supers, each level outward from the pixel and nearest first
// inside a region it descends into.  A region (block, group, super) is
// descended into only if its minimum f plus the squared distance from x to
// its nearest pixel is below the best value so far, and a level's outward
// walk ends once its nearer remaining region is at least sqrt(best) away.
// Every pixel that can attain the minimum is scanned, so the result is the
// exact minimum.  Near an edge the search ends inside the own group (about
// D/16 block tests, D the distance to the nearest edge); far from every edge
// the minima skip empty stretches 4096 or 256 pixels at a time, so a pixel
// costs O(W/4096 + 16 + 16 + 16) tests whatever the map (a 16384 x 16384 map
// with one edge pixel: 257 ms with blocks alone).
constexpr int kRowBlk = 16;
constexpr int kRowFan = 16;                 // blocks per group, groups per super
constexpr int kGroupPx = kRowBlk * kRowFan;
constexpr int kSuperPx = kGroupPx * kRowFan;

// LDS per row: f (W), block, group and super minima
__host__ __device__ inline int edt_row_lds_ints(int W) {
    const int nb = (W + kRowBlk - 1) / kRowBlk;
    const int ng = (W + kGroupPx - 1) / kGroupPx;
    const int ns = (W + kSuperPx - 1) / kSuperPx;
    return W + nb + ng + ns;
}

struct RowMinima {
    const int32_t* row;
    const int32_t* bmin;
    const int32_t* gmin;
    const int32_t* smin;
    int W;
};

// squared distance from x to the nearest pixel of [lo, hi] (x outside it)
__device__ __forceinline__ int gap2(int x, int lo, int hi) {
    const int d = x < lo ? lo - x : x - hi;
    return d * d;
}

__device__ __forceinline__ void scan_block(const RowMinima& m, int x, int b, int32_t& best) {
    const int q0 = kRowBlk * b;
    if (q0 + kRowBlk <= m.W) {
#pragma unroll
        for (int u = 0; u < kRowBlk; ++u) best = min(best, m.row[q0 + u] + (x - q0 - u) * (x - q0 - u));
    } else {
        for (int q = q0; q < m.W; ++q) best = min(best, m.row[q] + (x - q) * (x - q));
    }
}

// the blocks of group g, nearest to x first (g lies wholly on one side of x)
__device__ __forceinline__ void scan_group(const RowMinima& m, int x, int g, int32_t& best) {
    const int nb = (m.W + kRowBlk - 1) / kRowBlk;
    const int b0 = kRowFan * g, b1 = min(b0 + kRowFan, nb) - 1;
    const bool right = kRowBlk * b0 > x;
    for (int k = 0; k <= b1 - b0; ++k) {
        const int b = right ? b0 + k : b1 - k;
        const int d2b = gap2(x, kRowBlk * b, kRowBlk * b + kRowBlk - 1);
        if (d2b >= best) break;                  // the rest of the group is farther
        if (m.bmin[b] + d2b < best) scan_block(m, x, b, best);
    }
}

// the groups of super s, nearest to x first (s lies wholly on one side of x)
__device__ __forceinline__ void scan_super(const RowMinima& m, int x, int sp, int32_t& best) {
    const int ng = (m.W + kGroupPx - 1) / kGroupPx;
    const int g0 = kRowFan * sp, g1 = min(g0 + kRowFan, ng) - 1;
    const bool right = kGroupPx * g0 > x;
    for (int k = 0; k <= g1 - g0; ++k) {
        const int g = right ? g0 + k : g1 - k;
        const int d2g = gap2(x, kGroupPx * g, kGroupPx * g + kGroupPx - 1);
        if (d2g >= best) break;
        if (m.gmin[g] + d2g < best) scan_group(m, x, g, best);
    }
}

__global__ __launch_bounds__(256) void edt_rows(const int32_t* __restrict__ colsq,
                                               int32_t* __restrict__ d2, float* __restrict__ dtf,
                                               EdtBatch b) {
    extern __shared__ int32_t lds[];
    const int k = blockIdx.y;
    const int W = b.w[k], H = b.h[k];
    const int y = blockIdx.x;
    if (y >= H) return;                  // whole workgroup
    const int nb = (W + kRowBlk - 1) / kRowBlk;
    const int ng = (W + kGroupPx - 1) / kGroupPx;
    const int ns = (W + kSuperPx - 1) / kSuperPx;
    int32_t* row = lds;
    int32_t* bmin = lds + W;
    int32_t* gmin = bmin + nb;
    int32_t* smin = gmin + ng;
    const int64_t base = b.off[k] + (int64_t)y * W;
    for (int x = threadIdx.x; x < W; x += blockDim.x) row[x] = colsq[base + x];
    __syncthreads();
    // block minima, one block per thread; a group's 16 blocks sit on 16
    // adjacent lanes (256 threads and 16 blocks per group are both multiples
    // of 16), so the group minimum is a 16-lane butterfly
    for (int j0 = 0; j0 < nb; j0 += blockDim.x) {
        const int j = j0 + threadIdx.x;
        int32_t mn = kInf;
        if (j < nb) {
            const int q0 = kRowBlk * j;
            if (q0 + kRowBlk <= W) {
#pragma unroll
                for (int u = 0; u < kRowBlk; ++u) mn = min(mn, row[q0 + u]);
            } else {
                for (int q = q0; q < W; ++q) mn = min(mn, row[q]);
            }
            bmin[j] = mn;
        }
#pragma unroll
        for (int o = kRowFan / 2; o >= 1; o >>= 1) mn = min(mn, __shfl_xor(mn, o, 64));
        if (j < nb && (j % kRowFan) == 0) gmin[j / kRowFan] = mn;
    }
    __syncthreads();
    // super minima: only rows wider than one super have other supers
    if (ns > 1) {
        for (int j = threadIdx.x; j < ns; j += blockDim.x) {
            int32_t mn = gmin[kRowFan * j];
            for (int q = kRowFan * j + 1; q < min(kRowFan * j + kRowFan, ng); ++q) mn = min(mn, gmin[q]);
            smin[j] = mn;
        }
        __syncthreads();
    }
    const RowMinima m{row, bmin, gmin, smin, W};
    // f <= (H - 1)^2 < 2^28 or kInf = 2^30, squared distances < 2^28: no
    // int32 overflow in any sum below
    for (int x = threadIdx.x; x < W; x += blockDim.x) {
        const int bx = x / kRowBlk, gx = x / kGroupPx, sx = x / kSuperPx;
        int32_t best = row[x];
        scan_block(m, x, bx, best);
        // the other blocks of the own group, outward
        {
            const int lo = kRowFan * gx, hi = min(lo + kRowFan, nb) - 1;
            for (int R = 1;; ++R) {
                const int bl = bx - R, br = bx + R;
                const bool lin = bl >= lo, rin = br <= hi;
                if (!lin && !rin) break;
                const int dl = lin ? gap2(x, kRowBlk * bl, kRowBlk * bl + kRowBlk - 1) : 0x7fffffff;
                const int dr = rin ? gap2(x, kRowBlk * br, kRowBlk * br + kRowBlk - 1) : 0x7fffffff;
                if (min(dl, dr) >= best) break;
                if (lin && bmin[bl] + dl < best) scan_block(m, x, bl, best);
                if (rin && bmin[br] + dr < best) scan_block(m, x, br, best);
            }
        }
        // the other groups of the own super, outward
        {
            const int lo = kRowFan * sx, hi = min(lo + kRowFan, ng) - 1;
            for (int R = 1;; ++R) {
                const int gl = gx - R, gr = gx + R;
                const bool lin = gl >= lo, rin = gr <= hi;
                if (!lin && !rin) break;
                const int dl = lin ? gap2(x, kGroupPx * gl, kGroupPx * gl + kGroupPx - 1) : 0x7fffffff;
                const int dr = rin ? gap2(x, kGroupPx * gr, kGroupPx * gr + kGroupPx - 1) : 0x7fffffff;
                if (min(dl, dr) >= best) break;
                if (lin && gmin[gl] + dl < best) scan_group(m, x, gl, best);
                if (rin && gmin[gr] + dr < best) scan_group(m, x, gr, best);
            }
        }
        // the other supers, outward
        for (int R = 1; ns > 1; ++R) {
            const int sl = sx - R, sr = sx + R;
            const bool lin = sl >= 0, rin = sr < ns;
            if (!lin && !rin) break;
            const int dl = lin ? gap2(x, kSuperPx * sl, kSuperPx * sl + kSuperPx - 1) : 0x7fffffff;
            const int dr = rin ? gap2(x, kSuperPx * sr, kSuperPx * sr + kSuperPx - 1) : 0x7fffffff;
            if (min(dl, dr) >= best) break;
            if (lin && smin[sl] + dl < best) scan_super(m, x, sl, best);
            if (rin && smin[sr] + dr < best) scan_super(m, x, sr, best);
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
            const size_t lds = (size_t)edt_row_lds_ints(maxW) * sizeof(int32_t);
            if (lds > 65536) {
                // rows wider than 15360 pixels: more than the default 64 KB of
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
