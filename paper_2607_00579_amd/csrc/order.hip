// Per-pair copies of the edge records, ordered by the target pixel block they
// project to (a schedule choice of the fused kernel, supplementary Sec. A1.2
// "Per-iteration kernels": the distance-field gather dominates, so the
// gathers of one wave should share cache lines).
//
// The fused kernel reads, for every residual, its 8-byte source record and one
// texel of the target's distance field.  In source order the 64 residuals of a
// wave land on about 27 different 128-byte texture lines (8 x 4 pixel blocks);
// ordered by target block within chunks of 8192 records, on about 8.  The order
// depends on the poses, so it is re-sorted on the device as they move: chunk c
// at the steps s with s mod k == c mod k (k = resort_interval), inside the
// captured iteration.  Any order gives the same residuals; only the float64
// summation order of the sums changes, and the sort is a stable function of
// the poses, so results stay bitwise reproducible.
//
// One workgroup (512 threads) per chunk of <= 8192 records of one pair:
//   1. load the chunk's records (coalesced; 16 per thread, kept in registers),
//      project each at the current poses (float64, as the fused kernel) and
//      take its 8 x 4 target block (bx, by), or "invalid";
//   2. bucket = block relative to the chunk's bounding box of valid blocks,
//      row-major, both axes shifted right until the box has < 4096 buckets;
//      invalid residuals go to the last bucket (4095);
//   3. stable LSD radix sort of (bucket << 13 | index) in LDS, two passes of
//      six bits; each pass ranks the 64 elements of a wave with ballots (the
//      lanes holding the same digit) and offsets the waves' groups by an
//      exclusive scan over (digit, round, wave), so equal buckets keep their
//      source order;
//   4. route every record to its sorted position through LDS and store the
//      chunk coalesced.
#include "epo_internal.h"

namespace epo {
namespace {

constexpr int kSortThreads = 512;
constexpr int kSortWaves = kSortThreads / 64;
constexpr int kSortPer = 16;                               // records per thread
constexpr int kSortChunk = kSortThreads * kSortPer;        // 8192
constexpr int kIdxBits = 13;                               // index within a chunk
static_assert((1 << kIdxBits) == kSortChunk, "index bits cover a chunk");
constexpr int kDigitBits = 6;
constexpr int kDigits = 1 << kDigitBits;
constexpr int kBucketBits = 2 * kDigitBits;                // two passes
constexpr uint32_t kInvalidBucket = (1u << kBucketBits) - 1;
// dynamic LDS: two value buffers (u32, 64 KB), per (round, wave, digit) group
// counts and offsets (u16, 16 KB)
constexpr size_t kSortLds = 2 * kSortChunk * sizeof(uint32_t) +
                            (size_t)kSortPer * kSortWaves * kDigits * sizeof(uint16_t);

__device__ inline int wave_min(int x) {
#pragma unroll
    for (int m = 32; m >= 1; m >>= 1) x = min(x, __shfl_xor(x, m, 64));
    return x;
}
__device__ inline int wave_max(int x) {
#pragma unroll
    for (int m = 32; m >= 1; m >>= 1) x = max(x, __shfl_xor(x, m, 64));
    return x;
}

// lanes of this wave (within `active`) whose value has the same low
// kDigitBits bits of (x >> sh)
__device__ inline uint64_t same_digit(uint32_t x, int sh, uint64_t active) {
    uint64_t peers = active;
#pragma unroll
    for (int b = 0; b < kDigitBits; ++b) {
        const bool bit = (x >> (sh + b)) & 1u;
        const uint64_t on = __ballot(bit);
        peers &= bit ? on : ~on;
    }
    return peers;
}

__global__ __launch_bounds__(kSortThreads) void resort_kernel(
    const uint2* __restrict__ records, uint2* __restrict__ sorted, const Tile* __restrict__ chunks,
    int64_t n_chunks, const int64_t* __restrict__ pair_shift, const PairStatic* __restrict__ ps,
    const double* __restrict__ poses, const float* __restrict__ K,
    const int32_t* __restrict__ wh, const int32_t* __restrict__ step, int32_t every,
    double zmin) {
    extern __shared__ uint32_t lds[];
    uint32_t* buf0 = lds;
    uint32_t* buf1 = lds + kSortChunk;
    uint16_t* grp = reinterpret_cast<uint16_t*>(lds + 2 * kSortChunk);   // [round][wave][digit]
    __shared__ double xf[16];
    __shared__ int bb[4][kSortWaves];
    __shared__ uint32_t wtot[kSortWaves];
    __shared__ int box[5];

    const int64_t phase = step ? (int64_t)((uint32_t)*step % (uint32_t)every) : 0;
    const int64_t c = (int64_t)blockIdx.x * every + phase;
    if (c >= n_chunks) return;
    const Tile ch = chunks[c];
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int n = ch.count;
    if (tid == 0) {
        const PairStatic st = ps[ch.pair];
        double R[9], t[3], M[9];
        relative_pose(poses, K, st.src, st.tgt, R, t, M);
        for (int k = 0; k < 9; ++k) xf[k] = M[k];
        for (int k = 0; k < 3; ++k) xf[9 + k] = t[k];
        xf[12] = K[4 * st.tgt + 0];
        xf[13] = K[4 * st.tgt + 1];
        xf[14] = K[4 * st.tgt + 2];
        xf[15] = K[4 * st.tgt + 3];
        box[0] = wh[2 * st.tgt] - 1;       // cells per row / column
        box[1] = wh[2 * st.tgt + 1] - 1;
    }
    __syncthreads();
    const int wcells = box[0], hcells = box[1];

    // 1. records (element e = k * 512 + tid) and their target blocks
    uint2 rec[kSortPer];
    uint32_t blk[kSortPer];                  // bx | by << 12, or ~0u if invalid
    int bx0 = INT32_MAX, by0 = INT32_MAX, bx1 = -1, by1 = -1;
#pragma unroll
    for (int k = 0; k < kSortPer; ++k) {
        const int e = k * kSortThreads + tid;
        blk[k] = ~0u;
        rec[k] = make_uint2(0u, 0u);
        if (e < n) {
            rec[k] = records[ch.rec + e];
            const double u = (double)(rec[k].x & 0xffffu), v = (double)(rec[k].x >> 16);
            const double Z = (double)__uint_as_float(rec[k].y);
            const double Xx = fma(Z, fma(xf[0], u, fma(xf[1], v, xf[2])), xf[9]);
            const double Xy = fma(Z, fma(xf[3], u, fma(xf[4], v, xf[5])), xf[10]);
            const double Xz = fma(Z, fma(xf[6], u, fma(xf[7], v, xf[8])), xf[11]);
            if (Xz > zmin) {
                const double rz = 1.0 / Xz;
                const double up = fma(xf[12], Xx * rz, xf[14]);
                const double vp = fma(xf[13], Xy * rz, xf[15]);
                if (up >= 0.0 && vp >= 0.0 && up < (double)wcells && vp < (double)hcells) {
                    const int bx = (int)up >> 3, by = (int)vp >> 2;
                    blk[k] = (uint32_t)bx | ((uint32_t)by << 12);
                    bx0 = min(bx0, bx);
                    bx1 = max(bx1, bx);
                    by0 = min(by0, by);
                    by1 = max(by1, by);
                }
            }
        }
    }
    // 2. bounding box of the valid blocks, bucket grid
    bx0 = wave_min(bx0);
    by0 = wave_min(by0);
    bx1 = wave_max(bx1);
    by1 = wave_max(by1);
    if (lane == 0) {
        bb[0][wave] = bx0;
        bb[1][wave] = by0;
        bb[2][wave] = bx1;
        bb[3][wave] = by1;
    }
    __syncthreads();
    if (tid == 0) {
        int a0 = INT32_MAX, b0 = INT32_MAX, a1 = -1, b1 = -1;
        for (int w = 0; w < kSortWaves; ++w) {
            a0 = min(a0, bb[0][w]);
            b0 = min(b0, bb[1][w]);
            a1 = max(a1, bb[2][w]);
            b1 = max(b1, bb[3][w]);
        }
        int sh = 0;
        if (a1 >= 0) {
            while ((int64_t)(((a1 - a0) >> sh) + 1) * (int64_t)(((b1 - b0) >> sh) + 1) >=
                   (int64_t)kInvalidBucket)
                ++sh;
        }
        box[0] = a0;
        box[1] = b0;
        box[2] = sh;
        box[3] = a1 >= 0 ? ((a1 - a0) >> sh) + 1 : 1;   // buckets per row
    }
    __syncthreads();
    {
        const int a0 = box[0], b0 = box[1], sh = box[2], nbw = box[3];
#pragma unroll
        for (int k = 0; k < kSortPer; ++k) {
            const int e = k * kSortThreads + tid;
            if (e < n) {
                uint32_t b = kInvalidBucket;
                if (blk[k] != ~0u) {
                    const int bx = (int)(blk[k] & 0xfffu), by = (int)(blk[k] >> 12);
                    b = (uint32_t)(((by - b0) >> sh) * nbw + ((bx - a0) >> sh));
                }
                buf0[e] = (b << kIdxBits) | (uint32_t)e;
            }
        }
    }
    __syncthreads();

    // 3. two stable passes; element q of a pass (round q / 512, wave, lane)
    // is src[q]; its rank goes to the other buffer
    const int rounds = (n + kSortThreads - 1) / kSortThreads;
    uint32_t* src = buf0;
    uint32_t* dst = buf1;
    for (int pass = 0; pass < 2; ++pass) {
        const int sh = kIdxBits + pass * kDigitBits;
        // group counts of every (round, wave, digit) start at zero
#pragma unroll
        for (int k = 0; k < kSortPer; ++k) grp[k * kSortThreads + tid] = 0;
        __syncthreads();
        uint32_t val[kSortPer], rank[kSortPer];
#pragma unroll
        for (int r = 0; r < kSortPer; ++r) {
            val[r] = 0u;
            rank[r] = 0u;
            if (r < rounds) {
                const int q = r * kSortThreads + tid;
                const bool in = q < n;
                const uint64_t active = __ballot(in);
                if (in) val[r] = src[q];
                const uint64_t peers = same_digit(val[r], sh, active);
                rank[r] = (uint32_t)__popcll(peers & ((1ull << lane) - 1ull));
                // the lowest lane of each digit group records the group's size
                if (in && rank[r] == 0)
                    grp[(r * kSortWaves + wave) * kDigits + ((val[r] >> sh) & (kDigits - 1))] =
                        (uint16_t)__popcll(peers);
            }
        }
        __syncthreads();
        // exclusive scan of the group counts in (digit, round, wave) order:
        // thread t takes digit t / 8 and the 16 (round, wave) slots
        // 16 (t % 8) .. 16 (t % 8) + 15
        {
            const int dgt = tid >> 3, j0 = (tid & 7) * 16;
            uint32_t sum = 0;
#pragma unroll
            for (int j = 0; j < 16; ++j) sum += grp[(j0 + j) * kDigits + dgt];
            // block exclusive scan of the per-thread sums
            uint32_t incl = sum;
#pragma unroll
            for (int m = 1; m < 64; m <<= 1) {
                const uint32_t y = __shfl_up(incl, m, 64);
                if (lane >= m) incl += y;
            }
            if (lane == 63) wtot[wave] = incl;
            __syncthreads();
            uint32_t run = incl - sum;
            for (int w = 0; w < wave; ++w) run += wtot[w];
#pragma unroll
            for (int j = 0; j < 16; ++j) {
                const int a = (j0 + j) * kDigits + dgt;
                const uint32_t x = grp[a];
                grp[a] = (uint16_t)run;
                run += x;
            }
        }
        __syncthreads();
#pragma unroll
        for (int r = 0; r < kSortPer; ++r) {
            const int q = r * kSortThreads + tid;
            if (r < rounds && q < n) {
                const uint32_t d = (val[r] >> sh) & (kDigits - 1);
                dst[grp[(r * kSortWaves + wave) * kDigits + d] + rank[r]] = val[r];
            }
        }
        __syncthreads();
        uint32_t* t = src;
        src = dst;
        dst = t;
    }

    // 4. position of every element in the sorted chunk, records staged in
    // that order, stored coalesced
    uint16_t* dest = grp;
    for (int q = tid; q < n; q += kSortThreads) dest[src[q] & ((1u << kIdxBits) - 1)] = (uint16_t)q;
    __syncthreads();
    uint2* stage = reinterpret_cast<uint2*>(lds);
#pragma unroll
    for (int k = 0; k < kSortPer; ++k) {
        const int e = k * kSortThreads + tid;
        if (e < n) stage[dest[e]] = rec[k];
    }
    __syncthreads();
    uint2* out = sorted + ch.rec + pair_shift[ch.pair];
    for (int q = tid; q < n; q += kSortThreads) out[q] = stage[q];
}

// a copy of the records in source order (before the first sort)
__global__ __launch_bounds__(256) void copy_records_kernel(const uint2* __restrict__ records,
                                                           uint2* __restrict__ sorted,
                                                           const Tile* __restrict__ chunks,
                                                           const int64_t* __restrict__ pair_shift) {
    const Tile ch = chunks[blockIdx.x];
    uint2* out = sorted + ch.rec + pair_shift[ch.pair];
    for (int q = threadIdx.x; q < ch.count; q += 256) out[q] = records[ch.rec + q];
}

void set_sort_lds() {
    static bool done = false;
    if (done) return;
    int dev = 0, max_lds = 0;
    EPO_HIP(hipGetDevice(&dev));
    EPO_HIP(hipDeviceGetAttribute(&max_lds, hipDeviceAttributeMaxSharedMemoryPerBlock, dev));
    EPO_REQUIRE(kSortLds + 1024 <= (size_t)max_lds,
                "the device has too little LDS per workgroup for the record sort");
    EPO_HIP(hipFuncSetAttribute(reinterpret_cast<const void*>(resort_kernel),
                                hipFuncAttributeMaxDynamicSharedMemorySize, (int)kSortLds));
    done = true;
}

}  // namespace

void ensure_sorted_records(Plan& p, hipStream_t s) {
    if (p.sorted_records.p || p.D == 0) return;
    std::vector<int64_t> shift(p.D);
    std::vector<Tile> chunks;
    int64_t off = 0;
    for (int d = 0; d < p.D; ++d) {
        const int i = p.pairs[2 * d];
        const int64_t a = p.rec_off[i], n = p.rec_off[i + 1] - a;
        shift[d] = off - a;
        for (int64_t c = 0; c < n; c += kSortChunk)
            chunks.push_back(Tile{d, (int32_t)std::min<int64_t>(kSortChunk, n - c), a + c});
        off += n;
    }
    EPO_REQUIRE(off == p.n_residuals, "record copies do not cover the residuals");
    p.sorted_records.alloc((size_t)(off + kRecordPad));
    EPO_HIP(hipMemsetAsync(p.sorted_records.p + off, 0, sizeof(uint64_t) * kRecordPad, s));
    EPO_HIP(hipStreamSynchronize(s));      // host vectors below must outlive the copies
    p.pair_shift.alloc(shift.size());
    EPO_HIP(hipMemcpyAsync(p.pair_shift.p, shift.data(), shift.size() * sizeof(int64_t),
                           hipMemcpyHostToDevice, s));
    p.sort_chunks.alloc(std::max<size_t>(chunks.size(), 1));
    if (!chunks.empty())
        EPO_HIP(hipMemcpyAsync(p.sort_chunks.p, chunks.data(), chunks.size() * sizeof(Tile),
                               hipMemcpyHostToDevice, s));
    p.n_sort_chunks = (int64_t)chunks.size();
    if (p.n_sort_chunks > 0) {
        EPO_REQUIRE(p.n_sort_chunks < (int64_t)INT32_MAX, "too many record chunks");
        copy_records_kernel<<<(unsigned)p.n_sort_chunks, 256, 0, s>>>(
            reinterpret_cast<const uint2*>(p.records.p),
            reinterpret_cast<uint2*>(p.sorted_records.p), p.sort_chunks.p, p.pair_shift.p);
        EPO_CHECK_LAUNCH();
    }
    EPO_HIP(hipStreamSynchronize(s));
}

void launch_resort(Plan& p, const double* poses, const int32_t* step, int32_t every,
                   hipStream_t s) {
    if (p.opt.record_order != 2 || p.n_sort_chunks == 0) return;
    EPO_REQUIRE(p.sorted_records.p, "record copies not allocated");
    set_sort_lds();
    if (!step) every = 1;
    const int64_t grid = ceil_div(p.n_sort_chunks, every);
    resort_kernel<<<(unsigned)grid, kSortThreads, kSortLds, s>>>(
        reinterpret_cast<const uint2*>(p.records.p), reinterpret_cast<uint2*>(p.sorted_records.p),
        p.sort_chunks.p, p.n_sort_chunks, p.pair_shift.p, p.pair_static.p, poses, p.K_d.p,
        p.wh_d.p, step, every, (double)p.params.z_min);
    EPO_CHECK_LAUNCH();
}

}  // namespace epo

using namespace epo;

extern "C" epo_status epo_plan_resort(epo_plan plan, const double* poses, const int32_t* step,
                                      int32_t every, void* stream) {
    return guarded([&] {
        EPO_REQUIRE(plan && poses, "null argument");
        EPO_REQUIRE(!step || every >= 1, "every must be >= 1");
        Plan& p = *reinterpret_cast<Plan*>(plan);
        EPO_HIP(hipSetDevice(p.device));
        launch_resort(p, poses, step, every, as_stream(stream));
    });
}

extern "C" epo_status epo_plan_pair_records(epo_plan plan, int32_t d, uint64_t* records_out,
                                            int64_t capacity, int64_t* count) {
    return guarded([&] {
        EPO_REQUIRE(plan && count, "null argument");
        const Plan& p = *reinterpret_cast<Plan*>(plan);
        EPO_REQUIRE(d >= 0 && d < p.D, "pair index out of range");
        const int i = p.pairs[2 * d];
        const int64_t a = p.rec_off[i], n = p.rec_off[i + 1] - a;
        *count = n;
        if (!records_out || n == 0) return;
        EPO_REQUIRE(capacity >= n, "records_out too small");
        EPO_HIP(hipSetDevice(p.device));
        EPO_HIP(hipDeviceSynchronize());
        const uint64_t* src = p.records.p + a;
        if (p.opt.record_order == 2 && p.sorted_records.p) {
            int64_t shift = 0;
            EPO_HIP(hipMemcpy(&shift, p.pair_shift.p + d, sizeof(int64_t), hipMemcpyDeviceToHost));
            src = p.sorted_records.p + a + shift;
        }
        EPO_HIP(hipMemcpy(records_out, src, n * sizeof(uint64_t), hipMemcpyDeviceToHost));
    });
}
