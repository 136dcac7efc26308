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
    uint8_t* __restrict__ group_sel, double* __restrict__ pair_scale) {
    __shared__ uint32_t hist[256];
    __shared__ uint64_t prefix_s;
    __shared__ int rank_s;
    __shared__ int dir_part[4];
    const int s = blockIdx.x;
    const int tid = threadIdx.x;
    const int a = scene_group_ptr[s], n = scene_group_ptr[s + 1] - a;
    const uint64_t base = splitmix64(seed + (uint64_t)(uint32_t)step[0]);
    uint64_t T = ~0ull;             // key of rank budget - 1 (all selected if n <= budget)
    int tie_rank = n;               // keys equal to T that are taken, minus one
    if (n > budget) {
        uint64_t prefix = 0, mask = 0;
        int rank = budget - 1;
        for (int pass = 0; pass < 8; ++pass) {
            const int shift = 56 - 8 * pass;
            hist[tid] = 0u;
            __syncthreads();
            for (int k = tid; k < n; k += 256) {
                const uint64_t key = splitmix64(base + (uint64_t)(uint32_t)group_id[a + k]);
                if ((key & mask) == prefix) atomicAdd(&hist[(key >> shift) & 255u], 1u);
            }
            __syncthreads();
            if (tid == 0) {
                int acc = 0, b = 0;
                for (; b < 255; ++b) {
                    if (acc + (int)hist[b] > rank) break;
                    acc += (int)hist[b];
                }
                rank_s = rank - acc;
                prefix_s = prefix | ((uint64_t)b << shift);
            }
            __syncthreads();
            rank = rank_s;
            prefix = prefix_s;
            mask |= 255ull << shift;
        }
        T = prefix;
        tie_rank = rank;
    }
    // selection and the directions it covers
    int dirs = 0;
    for (int k = tid; k < n; k += 256) {
        const int32_t g = group_id[a + k];
        bool sel = true;
        if (n > budget) {
            const uint64_t key = splitmix64(base + (uint64_t)(uint32_t)g);
            sel = key < T;
            if (key == T) {
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

__global__ __launch_bounds__(256) void sampled_pairs_kernel(const double* __restrict__ pair_scale,
                                                            uint8_t* __restrict__ out, int32_t D) {
    const int d = blockIdx.x * blockDim.x + threadIdx.x;
    if (d < D) out[d] = pair_scale[d] != 0.0 ? 1 : 0;
}

}  // namespace

void launch_pair_selection(Plan& p, const int32_t* step, hipStream_t s) {
    if (p.sample_budget <= 0 || p.D == 0) return;
    select_pairs_kernel<<<(unsigned)p.S, 256, 0, s>>>(
        p.scene_group_ptr.p, p.group_id_sorted.p, p.group_npairs.p, p.scene_ptr.p,
        p.scene_pairs.p, p.group_of_pair.p, step, p.sample_seed, p.sample_budget, p.group_sel.p,
        p.pair_scale.p);
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
