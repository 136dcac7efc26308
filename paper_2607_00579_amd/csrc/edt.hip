// Exact squared Euclidean distance transform on gfx950 (two separable 1-D
// passes, the structure of Felzenszwalb-Huttenlocher), the distance transform
// field of the paper's Sec. 3 and supplementary Sec. A1.2 "Construction
// kernels".
//
//   column pass  g(x, y) = distance to the nearest edge pixel of column x,
//                f = g^2 (EPO_D2_EMPTY if the column has none), stored as
//                uint16 at the start of row y's DTF slots.  One thread
//                per (column, 64-row segment), in two kernels: the first
//                records each segment's first and last edge row (in d2, not
//                yet written); the second takes the nearest edge above and
//                below its segment from those records, then sweeps the
//                segment down and up, holding it in registers in between.  The 64 threads of a wave take 64
//                adjacent columns, so every step is one coalesced access, and
//                the segments give every view H/64 times the waves of a
//                thread-per-column pass.
//   row pass     d2(x, y) = min over q of f(q, y) + (x - q)^2.  One workgroup
//                per row stages f of the row and its minima per 16, 256 and
//                4096 pixels in LDS.  The minimizing q is monotone in x, so
//                the pass first finds a minimizer at every 16th pixel (an
//                exact search pruned by the minima), and every other pixel
//                then only scans the q between the minimizers of the block
//                starts on either side of it (or, when that range is wide,
//                searches from the bound the two give).  Integer arithmetic
//                throughout: the exact minimum.  The same kernel writes
//                DTF = sqrt(d2) in float32.

// Views are processed in batches whose descriptors travel as a kernel
// argument, so the call needs no device allocation.
#include <algorithm>
#include <numeric>
#include <vector>

#include "epo_internal.h"

namespace epo {
namespace {

// views per launch: their descriptors (16 B each) fill most of the 4 KB of
// kernel arguments
constexpr int kEdtBatch = 240;
constexpr int32_t kInf = EPO_D2_EMPTY;
constexpr int kSeg = 64;                 // rows per column-pass thread
constexpr uint16_t kNoEdge = 0xFFFF;     // column distance of a column without edge pixels

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
// the segment is swept down and up.  The column
// distances go out as uint16 at the start of each row's own DTF slots,
// where the row pass reads them before it writes that row's DTF.
__global__ __launch_bounds__(64) void edt_columns(const uint8_t* __restrict__ edge,
                                                  const int32_t* __restrict__ seg,
                                                  float* __restrict__ dtf, EdtBatch b) {
    const int k = blockIdx.z;
    const int W = b.w[k], H = b.h[k];
    const int x = blockIdx.x * blockDim.x + threadIdx.x;
    const int s0 = blockIdx.y, y0 = s0 * kSeg;
    if (x >= W || y0 >= H) return;
    const int y1 = min(y0 + kSeg, H);
    const int n_seg = (H + kSeg - 1) / kSeg;
    const uint8_t* e = edge + b.off[k] + x;
    const int32_t* sm = seg + b.off[k] + x;
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
            reinterpret_cast<uint16_t*>(dtf + b.off[k] + (int64_t)y * W)[x] =
                best >= 0 ? (uint16_t)best : kNoEdge;
        }
    }
}

// One workgroup per row.  The row's column distances live at the start of its
// DTF slots; the row's threads read all of them into LDS (as f = g^2) before
// any of them writes the row's DTF, and no other row touches them.
//
// Minimizers are monotone: with p_q(x) = f(q) + (x - q)^2 and q < q',
// p_q(x) - p_q'(x) = f(q) - f(q') + (q' - q)(2x - q - q') grows with x, so
// once q' is a minimizer at x, no q < q' is one at any x' > x (and no
// q > q' at any x' < x).  Hence for X0 < x < X1 every minimizer of x lies in
// [a minimizer of X0, a minimizer of X1].  Phase 1 finds d2 and a minimizer
// at every block start X0 = 16 b by the exact search below; phase 2 takes
// every other pixel's minimum over the q between the minimizers of its own
// and the next block start (the last block's right end is the row's end):
// by scanning the whole 4-pixel chunks that hold them when there are at
// most kScanMax, else by the same search started from the better of the two
// end values.
//
// The search: a three-level hierarchy of minima in LDS: blocks of 16 pixels,
// groups of 16 blocks (256 px), supers of 16 groups (4096 px).  A pixel scans
// its own block, then the other blocks of its group, the other groups of its
// super, and the other supers, each level outward from the pixel and nearest
// first inside a region it descends into.  A region is descended into only
// if its minimum f plus the squared distance from x to its nearest pixel is
// below the best value so far, and a level's outward walk ends once its
// nearer remaining region is at least sqrt(best) away.  Every pixel that can
// attain the minimum is scanned, so the result is the exact minimum, and the
// recorded q (the first to reach the final value) is a minimizer.  Near an
// edge the search ends inside the own group; far from every edge the minima
// skip empty stretches 4096 or 256 pixels at a time, so a search costs
// O(W/4096 + 16 + 16 + 16) tests whatever the map.
constexpr int kRowBlk = 16;
constexpr int kRowFan = 16;                 // blocks per group, groups per super
constexpr int kGroupPx = kRowBlk * kRowFan;
constexpr int kSuperPx = kGroupPx * kRowFan;
constexpr int kScanMax = 48;                // widest range phase 2 scans blockwise
constexpr int kBlkStride = kRowBlk + 1;     // LDS ints per block of the row

// The row sits in LDS with one padding int after every 16 pixels: pixel q at
// q + q / 16, so block b starts at 17 b and the blocks that different lanes
// scan at once start on different banks (with 16 ints per block they would
// all fall on two).  The padding of the last block (pixels W .. 16 nb - 1)
// holds kInf, so every block is scanned whole.
__device__ __forceinline__ int rix(int q) { return q + (q >> 4); }

// LDS per row: f (17 per block), block, group and super minima, block-start
// minimizers
__host__ __device__ inline int edt_row_lds_ints(int W) {
    const int nb = (W + kRowBlk - 1) / kRowBlk;
    const int ng = (W + kGroupPx - 1) / kGroupPx;
    const int ns = (W + kSuperPx - 1) / kSuperPx;
    return kBlkStride * nb + nb + ng + ns + nb + 1;
}

struct RowMinima {
    const int32_t* row;                     // padded: pixel q at rix(q)
    const int32_t* bmin;
    const int32_t* gmin;
    const int32_t* smin;
    int W;
};

// the best value found so far and the first q that reached it
struct Best {
    int32_t v;
    int32_t q;
};

// squared distance from x to the nearest pixel of [lo, hi] (x outside it)
__device__ __forceinline__ int gap2(int x, int lo, int hi) {
    const int d = x < lo ? lo - x : x - hi;
    return d * d;
}

// block blk (its padding pixels hold kInf), minimizer recorded
__device__ __forceinline__ void scan_block(const RowMinima& m, int x, int blk, Best& b) {
    const int32_t* f = m.row + kBlkStride * blk;
    const int d0 = x - kRowBlk * blk;
#pragma unroll
    for (int u = 0; u < kRowBlk; ++u) {
        const int32_t v = f[u] + (d0 - u) * (d0 - u);
        if (v < b.v) {
            b.v = v;
            b.q = kRowBlk * blk + u;
        }
    }
}

// the value alone over the kChunk pixels kChunk c .. kChunk (c + 1) - 1
// (within one block; phase 2 needs no minimizer)
constexpr int kChunk = 4;
__device__ __forceinline__ int32_t scan_chunk_v(const RowMinima& m, int x, int c, int32_t v) {
    const int q0 = kChunk * c;
    const int32_t* f = m.row + rix(q0);
    const int d0 = x - q0;
#pragma unroll
    for (int u = 0; u < kChunk; ++u) v = min(v, f[u] + (d0 - u) * (d0 - u));
    return v;
}

// the blocks of group g, nearest to x first (g lies wholly on one side of x)
__device__ __forceinline__ void scan_group(const RowMinima& m, int x, int g, Best& b) {
    const int nb = (m.W + kRowBlk - 1) / kRowBlk;
    const int b0 = kRowFan * g, b1 = min(b0 + kRowFan, nb) - 1;
    const bool right = kRowBlk * b0 > x;
    for (int k = 0; k <= b1 - b0; ++k) {
        const int blk = right ? b0 + k : b1 - k;
        const int d2b = gap2(x, kRowBlk * blk, kRowBlk * blk + kRowBlk - 1);
        if (d2b >= b.v) break;                   // the rest of the group is farther
        if (m.bmin[blk] + d2b < b.v) scan_block(m, x, blk, b);
    }
}

// the groups of super s, nearest to x first (s lies wholly on one side of x)
__device__ __forceinline__ void scan_super(const RowMinima& m, int x, int sp, Best& b) {
    const int ng = (m.W + kGroupPx - 1) / kGroupPx;
    const int g0 = kRowFan * sp, g1 = min(g0 + kRowFan, ng) - 1;
    const bool right = kGroupPx * g0 > x;
    for (int k = 0; k <= g1 - g0; ++k) {
        const int g = right ? g0 + k : g1 - k;
        const int d2g = gap2(x, kGroupPx * g, kGroupPx * g + kGroupPx - 1);
        if (d2g >= b.v) break;
        if (m.gmin[g] + d2g < b.v) scan_group(m, x, g, b);
    }
}

// the exact minimum over the row for pixel x, from the bound b (a value some
// q attains, with that q)
__device__ Best search(const RowMinima& m, int x, Best b) {
    const int nb = (m.W + kRowBlk - 1) / kRowBlk;
    const int ng = (m.W + kGroupPx - 1) / kGroupPx;
    const int ns = (m.W + kSuperPx - 1) / kSuperPx;
    const int bx = x / kRowBlk, gx = x / kGroupPx, sx = x / kSuperPx;
    if (m.bmin[bx] < b.v) scan_block(m, x, bx, b);
    // the other blocks of the own group, outward
    {
        const int lo = kRowFan * gx, hi = min(lo + kRowFan, nb) - 1;
        for (int R = 1;; ++R) {
            const int bl = bx - R, br = bx + R;
            const bool lin = bl >= lo, rin = br <= hi;
            if (!lin && !rin) break;
            const int dl = lin ? gap2(x, kRowBlk * bl, kRowBlk * bl + kRowBlk - 1) : 0x7fffffff;
            const int dr = rin ? gap2(x, kRowBlk * br, kRowBlk * br + kRowBlk - 1) : 0x7fffffff;
            if (min(dl, dr) >= b.v) break;
            if (lin && m.bmin[bl] + dl < b.v) scan_block(m, x, bl, b);
            if (rin && m.bmin[br] + dr < b.v) scan_block(m, x, br, b);
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
            if (min(dl, dr) >= b.v) break;
            if (lin && m.gmin[gl] + dl < b.v) scan_group(m, x, gl, b);
            if (rin && m.gmin[gr] + dr < b.v) scan_group(m, x, gr, b);
        }
    }
    // the other supers, outward
    for (int R = 1; ns > 1; ++R) {
        const int sl = sx - R, sr = sx + R;
        const bool lin = sl >= 0, rin = sr < ns;
        if (!lin && !rin) break;
        const int dl = lin ? gap2(x, kSuperPx * sl, kSuperPx * sl + kSuperPx - 1) : 0x7fffffff;
        const int dr = rin ? gap2(x, kSuperPx * sr, kSuperPx * sr + kSuperPx - 1) : 0x7fffffff;
        if (min(dl, dr) >= b.v) break;
        if (lin && m.smin[sl] + dl < b.v) scan_super(m, x, sl, b);
        if (rin && m.smin[sr] + dr < b.v) scan_super(m, x, sr, b);
    }
    return b;
}

// Threads per row: T = 64 (one wave per row, four rows per workgroup, the
// rows independent of each other) for rows of up to 2048 pixels, T = 256 (the
// workgroup) for wider ones.  A batch's rows are many and short: a wave per
// row puts phase 1's W / 16 block starts on the whole wave, and four rows per
// workgroup keep eight waves per SIMD in flight (a CU holds at most 16
// workgroups, so one-wave workgroups would cap it at four).
constexpr int kRowThreadsMax = 256;
inline int edt_row_threads(int max_w) { return max_w <= 2048 ? 64 : kRowThreadsMax; }

// the ordering point between the phases of one row: the workgroup's barrier,
// or, for a row that one wave owns, a wave-level fence (a wave's LDS accesses
// complete in order)
template <int T>
__device__ __forceinline__ void row_sync() {
    if constexpr (T == 64) {
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    } else {
        __syncthreads();
    }
}

template <int T>
__global__ __launch_bounds__(kRowThreadsMax) void edt_rows(int32_t* __restrict__ d2,
                                                          float* __restrict__ dtf, EdtBatch bt,
                                                          int row_ints) {
    extern __shared__ int32_t lds[];
    constexpr int kRowsPerGroup = kRowThreadsMax / T;
    const int k = blockIdx.y;
    const int W = bt.w[k], H = bt.h[k];
    const int sub = (int)threadIdx.x / T;        // the row within the workgroup
    const int t = (int)threadIdx.x % T;          // the thread within the row
    const int y = (int)blockIdx.x * kRowsPerGroup + sub;
    if (y >= H) return;                          // the row's threads together
    const int nb = (W + kRowBlk - 1) / kRowBlk;
    const int ng = (W + kGroupPx - 1) / kGroupPx;
    const int ns = (W + kSuperPx - 1) / kSuperPx;
    int32_t* row = lds + (size_t)sub * row_ints;
    int32_t* bmin = row + kBlkStride * nb;
    int32_t* gmin = bmin + nb;
    int32_t* smin = gmin + ng;
    int32_t* qstart = smin + ns;         // minimizer at each block start, [nb] = W - 1
    const int64_t base = bt.off[k] + (int64_t)y * W;
    const uint16_t* grow = reinterpret_cast<const uint16_t*>(dtf + base);
    for (int x = t; x < W; x += T) {
        const int32_t g = grow[x];
        row[rix(x)] = g == kNoEdge ? kInf : g * g;
    }
    for (int x = W + t; x < kRowBlk * nb; x += T) row[rix(x)] = kInf;
    row_sync<T>();
    // block minima, one block per thread; a group's 16 blocks sit on 16
    // adjacent lanes (T and 16 blocks per group are both multiples of 16),
    // so the group minimum is a 16-lane butterfly
    for (int j0 = 0; j0 < nb; j0 += T) {
        const int j = j0 + t;
        int32_t mn = kInf;
        if (j < nb) {
#pragma unroll
            for (int u = 0; u < kRowBlk; ++u) mn = min(mn, row[kBlkStride * j + u]);
            bmin[j] = mn;
        }
#pragma unroll
        for (int o = kRowFan / 2; o >= 1; o >>= 1) mn = min(mn, __shfl_xor(mn, o, 64));
        if (j < nb && (j % kRowFan) == 0) gmin[j / kRowFan] = mn;
    }
    row_sync<T>();
    // super minima: only rows wider than one super have other supers
    if (ns > 1) {
        for (int j = t; j < ns; j += T) {
            int32_t mn = gmin[kRowFan * j];
            for (int q = kRowFan * j + 1; q < min(kRowFan * j + kRowFan, ng); ++q) mn = min(mn, gmin[q]);
            smin[j] = mn;
        }
        row_sync<T>();
    }
    const RowMinima m{row, bmin, gmin, smin, W};
    // f <= (H - 1)^2 < 2^28 or kInf = 2^30, squared distances < 2^28: no
    // int32 overflow in any sum below
    // phase 1: the block starts (exact search, minimizer recorded)
    for (int j = t; j <= nb; j += T) {
        if (j == nb) {
            qstart[nb] = W - 1;
            continue;
        }
        const int x = kRowBlk * j;
        const Best r = search(m, x, Best{row[rix(x)], x});
        qstart[j] = r.q;
        d2[base + x] = r.v;
        dtf[base + x] = sqrtf((float)r.v);
    }
    row_sync<T>();
    // phase 2: every other pixel, between the minimizers of the block starts
    // on either side of it
    for (int x = t; x < W; x += T) {
        if (x % kRowBlk == 0) continue;
        const int j = x / kRowBlk;
        const int qa = qstart[j], qb = qstart[j + 1];
        int32_t v = row[rix(qa)] + (x - qa) * (x - qa);
        if (qb - qa < kScanMax) {
            // the whole 4-pixel chunks that hold [qa, qb]: the extra pixels
            // only add candidates, and every minimizer of x lies in the range
            for (int c = qa / kChunk; c <= qb / kChunk; ++c) v = scan_chunk_v(m, x, c, v);
        } else {
            Best r{v, qa};
            const int32_t vb = row[rix(qb)] + (x - qb) * (x - qb);
            if (vb < r.v) r = Best{vb, qb};
            v = search(m, x, r).v;
        }
        d2[base + x] = v;
        dtf[base + x] = sqrtf((float)v);
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
        // views batched by size (every view writes at its own offset, so the
        // order changes nothing else): a launch's grid is sized for its
        // largest view, and the others' surplus workgroups exit at once
        std::vector<int32_t> order(n_views);
        std::iota(order.begin(), order.end(), 0);
        std::stable_sort(order.begin(), order.end(), [&](int32_t x, int32_t y) {
            return height[x] != height[y] ? height[x] < height[y] : width[x] < width[y];
        });
        for (int32_t a = 0; a < n_views; a += kEdtBatch) {
            EdtBatch b{};
            b.n = std::min(kEdtBatch, n_views - a);
            int maxW = 1, maxH = 1;
            for (int k = 0; k < b.n; ++k) {
                const int32_t v = order[a + k];
                b.w[k] = width[v];
                b.h[k] = height[v];
                b.off[k] = view_offset[v];
                maxW = std::max(maxW, b.w[k]);
                maxH = std::max(maxH, b.h[k]);
            }
            const dim3 cgrid((unsigned)ceil_div(maxW, 64), (unsigned)ceil_div(maxH, kSeg), b.n);
            edt_segments<<<cgrid, 64, 0, s>>>(edge_maps, d2_out, b);
            EPO_CHECK_LAUNCH();
            edt_columns<<<cgrid, 64, 0, s>>>(edge_maps, d2_out, dtf_out, b);
            EPO_CHECK_LAUNCH();
            const int T = edt_row_threads(maxW);
            const int rows_per_group = kRowThreadsMax / T;
            const int row_ints = edt_row_lds_ints(maxW);
            const size_t lds = (size_t)rows_per_group * row_ints * sizeof(int32_t);
            auto kernel = T == 64 ? edt_rows<64> : edt_rows<kRowThreadsMax>;
            if (lds > 65536) {
                // rows wider than 14508 pixels: more than the default 64 KB of
                // dynamic LDS (gfx950 has 160 KB per workgroup); an error, never
                // a short allocation, if the device cannot give it
                int dev = 0, max_lds = 0;
                EPO_HIP(hipGetDevice(&dev));
                EPO_HIP(hipDeviceGetAttribute(&max_lds, hipDeviceAttributeMaxSharedMemoryPerBlock,
                                              dev));
                EPO_REQUIRE(lds <= (size_t)max_lds,
                            "rows too wide for the device's LDS per workgroup");
                EPO_HIP(hipFuncSetAttribute(reinterpret_cast<const void*>(kernel),
                                            hipFuncAttributeMaxDynamicSharedMemorySize,
                                            (int)lds));
            }
            kernel<<<dim3((unsigned)ceil_div(maxH, rows_per_group), b.n), kRowThreadsMax, lds,
                     s>>>(d2_out, dtf_out, b, row_ints);
            EPO_CHECK_LAUNCH();
        }
    });
}
