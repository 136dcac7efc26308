// Stochastic viewgraph sub-sampling on the device (paper supplementary Sec.
// "Stochastic viewgraph sub-sampling"; the pair budget M of Alg. EPO.Forward):
// at every step each scene evaluates a fresh uniform random subset of its
// image pairs of size min(|E_scene|, M); the directions of a selected pair are
// evaluated together and the scene's loss is the mean over the selected
// directions, so the pair scale becomes 2 / |D_S| (0 for skipped pairs).
//
// The draw: image pair g (numbered in order of first appearance in the pair
// list) gets the key k = h(h(seed + step) + g), with h the SplitMix64 output
// function (Steele, Lea and Flood, OOPSLA 2014); the selected pairs are the M
// with the smallest (key, g).  The step is read from the device step counter,
// so a captured iteration draws a new subset at every replay.
//
// One workgroup per scene finds the M-th smallest key by an MSB-first radix
// select (eight 8-bit digits, a 256-bin LDS histogram per pass, keys
// recomputed from the hash), so any number of pairs per scene is handled
// without sorting.
#include "epo_internal.h"

namespace epo {
namespace {

__device__ __forceinline__ uint64_t splitmix64(uint64_t x) {
    uint64_t z = x + 0x9E3779B97F4A7C15ull;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

__global__ __launch_bounds__(256) void select_pairs_kernel(
    const int32_t* __restrict__ scene_group_ptr, const int32_t* __restrict__ group_id,
    const int32_t* __restrict__ group_npairs, const int32_t* __restrict__ scene_ptr,
    const int32_t* __restrict__ scene_pairs, const int32_t* __restrict__ group_of_pair,
    const int32_t* __restrict__ step, uint64_t seed, int32_t budget,
    const int32_t* __restrict__ phase, uint8_t* __restrict__ group_sel,
    double* __restrict__ pair_scale) {
    __shared__ uint32_t hist[256];
    __shared__ uint64_t prefix_s;
    __shared__ int rank_s, equal_s;
    __shared__ int dir_part[4];
    __shared__ int wave_tot[4];
    const int s = blockIdx.x;
    const int tid = threadIdx.x;
    if (phase && phase[s] == 2) {
        // a stopped scene evaluates nothing (the whole workgroup leaves here)
        for (int k = scene_ptr[s] + tid; k < scene_ptr[s + 1]; k += 256)
            pair_scale[scene_pairs[k]] = 0.0;
        return;
    }
    const int a = scene_group_ptr[s], n = scene_group_ptr[s + 1] - a;
    const uint64_t base = splitmix64(seed + (uint64_t)(uint32_t)step[0]);
    uint64_t T = ~0ull;             // key of rank budget - 1 (all selected if n <= budget)
    int tie_rank = n;               // keys equal to T that are taken, minus one
    int n_equal = 1;                // keys equal to T
    if (n > budget) {
        uint64_t prefix = 0, mask = 0;
        int rank = budget - 1;
        const int lane = tid & 63, wave = tid >> 6;
        for (int pass = 0; pass < 8; ++pass) {
            const int shift = 56 - 8 * pass;
            hist[tid] = 0u;
            __syncthreads();
            for (int k = tid; k < n; k += 256) {
                const uint64_t key = splitmix64(base + (uint64_t)(uint32_t)group_id[a + k]);
                if ((key & mask) == prefix) atomicAdd(&hist[(key >> shift) & 255u], 1u);
            }
            __syncthreads();
            // bucket b holding the rank: inclusive prefix over the 256 bins
            const int h = (int)hist[tid];
            int x = h;
#pragma unroll
            for (int m = 1; m < 64; m <<= 1) {
                const int y = __shfl_up(x, m, 64);
                if (lane >= m) x += y;
            }
            if (lane == 63) wave_tot[wave] = x;
            __syncthreads();
            for (int w = 0; w < wave; ++w) x += wave_tot[w];
            if (x - h <= rank && rank < x) {         // exactly one bin
                rank_s = rank - (x - h);
                prefix_s = prefix | ((uint64_t)tid << shift);
                equal_s = h;
            }
            __syncthreads();
            rank = rank_s;
            prefix = prefix_s;
            mask |= 255ull << shift;
        }
        T = prefix;
        tie_rank = rank;
        n_equal = equal_s;          // after the last digit: keys equal to T
    }
    // selection and the directions it covers
    int dirs = 0;
    for (int k = tid; k < n; k += 256) {
        const int32_t g = group_id[a + k];
        bool sel = true;
        if (n > budget) {
            const uint64_t key = splitmix64(base + (uint64_t)(uint32_t)g);
            sel = key <= T;
            if (key == T && n_equal > 1) {
                // equal keys are taken in group order
                int before = 0;
                for (int q = 0; q < n; ++q) {
                    const int32_t h = group_id[a + q];
                    before += (h < g && splitmix64(base + (uint64_t)(uint32_t)h) == T) ? 1 : 0;
                }
                sel = before <= tie_rank;
            }
        }
        group_sel[a + k] = sel ? 1 : 0;
        dirs += sel ? group_npairs[a + k] : 0;
    }
#pragma unroll
    for (int m = 32; m >= 1; m >>= 1) dirs += __shfl_xor(dirs, m, 64);
    if ((tid & 63) == 0) dir_part[tid >> 6] = dirs;
    __syncthreads();
    const int n_dir = dir_part[0] + dir_part[1] + dir_part[2] + dir_part[3];
    const double scale = n_dir > 0 ? 2.0 / (double)n_dir : 0.0;
    for (int k = scene_ptr[s] + tid; k < scene_ptr[s + 1]; k += 256) {
        const int d = scene_pairs[k];
        pair_scale[d] = group_sel[group_of_pair[d]] ? scale : 0.0;
    }
}

// Without sub-sampling: every pair at its full scale, or 0 for the pairs of
// a scene the convergence test has stopped (phase 2), when phase is given.
__global__ __launch_bounds__(256) void gate_pairs_kernel(const int32_t* __restrict__ scene_ptr,
                                                         const int32_t* __restrict__ scene_pairs,
                                                         const int32_t* __restrict__ phase,
                                                         const double* __restrict__ scale_all,
                                                         double* __restrict__ pair_scale) {
    const int s = blockIdx.x;
    const bool stopped = phase && phase[s] == 2;
    for (int k = scene_ptr[s] + threadIdx.x; k < scene_ptr[s + 1]; k += 256) {
        const int d = scene_pairs[k];
        pair_scale[d] = stopped ? 0.0 : scale_all[d];
    }
}

// Compacted tile list of the selected pairs, in tile (XCD queue) order, so
// the fused kernel visits only their tiles.  Blocks of 1024 tiles: count,
// one-workgroup scan of the block counts (and the queue split), scatter.
constexpr int kCompact = 1024;

__device__ __forceinline__ bool tile_selected(const Tile* __restrict__ tiles,
                                              const double* __restrict__ pair_scale, int64_t t,
                                              int64_t T) {
    return t < T && pair_scale[tiles[t].pair] != 0.0;
}

__global__ __launch_bounds__(256) void tile_count_kernel(const Tile* __restrict__ tiles,
                                                         const double* __restrict__ pair_scale,
                                                         int64_t T, int32_t* __restrict__ blk) {
    __shared__ int part[4];
    const int64_t base = (int64_t)blockIdx.x * kCompact;
    int c = 0;
    for (int r = 0; r < kCompact / 256; ++r)
        c += tile_selected(tiles, pair_scale, base + r * 256 + threadIdx.x, T) ? 1 : 0;
#pragma unroll
    for (int m = 32; m >= 1; m >>= 1) c += __shfl_xor(c, m, 64);
    if ((threadIdx.x & 63) == 0) part[threadIdx.x >> 6] = c;
    __syncthreads();
    if (threadIdx.x == 0) blk[blockIdx.x] = part[0] + part[1] + part[2] + part[3];
}

// one workgroup: block counts -> exclusive offsets (in place); queue starts
__global__ __launch_bounds__(256) void tile_scan_kernel(int32_t* __restrict__ blk, int32_t B,
                                                        int32_t nq, int64_t* __restrict__ qbegin) {
    __shared__ int wsum[4];
    __shared__ int carry;
    if (threadIdx.x == 0) carry = 0;
    __syncthreads();
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    for (int b0 = 0; b0 < B; b0 += 256) {
        const int b = b0 + (int)threadIdx.x;
        const int v = b < B ? blk[b] : 0;
        int x = v;                                   // inclusive scan within the wave
#pragma unroll
        for (int m = 1; m < 64; m <<= 1) {
            const int y = __shfl_up(x, m, 64);
            if (lane >= m) x += y;
        }
        if (lane == 63) wsum[wave] = x;
        __syncthreads();
        int before = carry;
        for (int w = 0; w < wave; ++w) before += wsum[w];
        if (b < B) blk[b] = before + x - v;          // exclusive offset
        __syncthreads();
        if (threadIdx.x == 255) carry = before + x;
        __syncthreads();
    }
    // the compacted list is split into nq equal contiguous queues (balanced
    // across the XCDs; contiguous, so a target's tiles still share one L2)
    if ((int)threadIdx.x <= nq) qbegin[threadIdx.x] = (int64_t)carry * threadIdx.x / nq;
}

__global__ __launch_bounds__(256) void tile_scatter_kernel(const Tile* __restrict__ tiles,
                                                           const double* __restrict__ pair_scale,
                                                           int64_t T,
                                                           const int32_t* __restrict__ blk,
                                                           int32_t* __restrict__ list) {
    __shared__ int wcnt[kCompact / 64];
    const int64_t base = (int64_t)blockIdx.x * kCompact;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    bool sel[kCompact / 256];
    for (int r = 0; r < kCompact / 256; ++r) {
        sel[r] = tile_selected(tiles, pair_scale, base + r * 256 + threadIdx.x, T);
        const uint64_t m = __ballot(sel[r]);
        if (lane == 0) wcnt[r * 4 + wave] = __popcll(m);
    }
    __syncthreads();
    int off = blk[blockIdx.x];
    // entries are ordered (r, wave, lane) = tile index order
    for (int r = 0; r < kCompact / 256; ++r) {
        const uint64_t m = __ballot(sel[r]);
        int before = off;
        for (int w = 0; w < wave; ++w) before += wcnt[r * 4 + w];
        if (sel[r])
            list[before + __popcll(m & ((1ull << lane) - 1ull))] =
                (int32_t)(base + r * 256 + threadIdx.x);
        for (int w = 0; w < 4; ++w) off += wcnt[r * 4 + w];
    }
}

__global__ __launch_bounds__(256) void sampled_pairs_kernel(const double* __restrict__ pair_scale,
                                                            uint8_t* __restrict__ out, int32_t D) {
    const int d = blockIdx.x * blockDim.x + threadIdx.x;
    if (d < D) out[d] = pair_scale[d] != 0.0 ? 1 : 0;
}

}  // namespace

void launch_pair_selection(Plan& p, const int32_t* step, hipStream_t s) {
    if (p.D == 0) return;
    if (p.sample_budget > 0) {
        select_pairs_kernel<<<(unsigned)p.S, 256, 0, s>>>(
            p.scene_group_ptr.p, p.group_id_sorted.p, p.group_npairs.p, p.scene_ptr.p,
            p.scene_pairs.p, p.group_of_pair.p, step, p.sample_seed, p.sample_budget,
            p.gate_phase, p.group_sel.p, p.pair_scale.p);
        EPO_CHECK_LAUNCH();
    } else if (p.gate_phase || p.scale_gated) {
        // stopped scenes skipped (captured iteration), or the full scales
        // restored after such an iteration ran
        gate_pairs_kernel<<<(unsigned)p.S, 256, 0, s>>>(p.scene_ptr.p, p.scene_pairs.p,
                                                         p.gate_phase, p.pair_scale_all.p,
                                                         p.pair_scale.p);
        EPO_CHECK_LAUNCH();
    }
    if (!compacted_launch(p)) return;
    const int64_t T = p.n_tiles;
    const int32_t B = (int32_t)std::max<int64_t>(ceil_div(T, kCompact), 1);
    tile_count_kernel<<<(unsigned)B, 256, 0, s>>>(p.tiles.p, p.pair_scale.p, T, p.tile_blk.p);
    EPO_CHECK_LAUNCH();
    tile_scan_kernel<<<1, 256, 0, s>>>(p.tile_blk.p, B, p.n_xcd_queues, p.qbegin_d.p);
    EPO_CHECK_LAUNCH();
    tile_scatter_kernel<<<(unsigned)B, 256, 0, s>>>(p.tiles.p, p.pair_scale.p, T, p.tile_blk.p,
                                                    p.tile_list.p);
    EPO_CHECK_LAUNCH();
}

}  // namespace epo

using namespace epo;

extern "C" epo_status epo_plan_set_pair_sampling(epo_plan plan, int32_t budget, uint64_t seed,
                                                 const int32_t* step, void* stream) {
    return guarded([&] {
        EPO_REQUIRE(plan, "null plan");
        EPO_REQUIRE(budget >= 0, "budget must be >= 0 (0 = every pair)");
        EPO_REQUIRE(budget == 0 || step, "a device step counter is required");
        Plan& p = *reinterpret_cast<Plan*>(plan);
        EPO_HIP(hipSetDevice(p.device));
        hipStream_t s = as_stream(stream);
        EPO_HIP(hipStreamSynchronize(s));
        release_graph(p);                   // a captured iteration would keep the old setting
        p.sample_budget = budget;
        p.sample_seed = seed;
        p.sample_step = budget > 0 ? step : nullptr;
        if (budget == 0 && p.D > 0)
            EPO_HIP(hipMemcpyAsync(p.pair_scale.p, p.pair_scale_all.p, sizeof(double) * p.D,
                                   hipMemcpyDeviceToDevice, s));
    });
}

extern "C" epo_status epo_plan_sampled_pairs(epo_plan plan, uint8_t* selected, void* stream) {
    return guarded([&] {
        EPO_REQUIRE(plan && selected, "null argument");
        Plan& p = *reinterpret_cast<Plan*>(plan);
        EPO_HIP(hipSetDevice(p.device));
        if (p.D == 0) return;
        sampled_pairs_kernel<<<(unsigned)ceil_div(p.D, 256), 256, 0, as_stream(stream)>>>(
            p.pair_scale.p, selected, p.D);
        EPO_CHECK_LAUNCH();
    });
}
