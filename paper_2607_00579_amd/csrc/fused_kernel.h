// Device code of the fused residual + adjoint kernel and its per-tile
// reduction (paper Eqs. pi, d_ij, L_ij; supplementary Alg. 3 and Sec. A1.2
// "Per-iteration kernels"): per residual, residual.h; per thread, float64
// sums; per workgroup, wave64 butterflies and an LDS step to one float64
// partial per tile.  Included by edge_cost.hip, which holds the host-side
// launches.  The measured counters of this kernel are keyed to the text of
// this file, residual.h and the data layout section of epo_internal.h.
#pragma once

#include "residual.h"

namespace epo {
namespace fused {

constexpr int kBlock = 256;

// ---------------------------------------------------------------------------
// fused residual + adjoint + tile reduction
// ---------------------------------------------------------------------------

// per-thread sums: the float32 terms of the U residuals a thread has in flight
// are added in float32 (one more rounding, of the size of each term's own
// product rounding), then into float64 (the pose-gradient sums cancel
// strongly, up to a few hundred in sum |term| / |sum|); the valid count in
// integers; ft, fs are the focal-scale sums of the refinement variant
struct Acc {
    double S, g0, g1, g2, g3, g4, g5;
    double ft, fs;
};

// the float32 terms of one residual
struct Terms {
    float S, g0, g1, g2, g3, g4, g5, ft, fs, dz;
    bool valid;
};

// refinement variant (EXT): besides the pose terms, per pair
//   F_t = sum of f_j dH/df_j = sum of (A_u x_n + A_v y_n) = sum of -w
//         (u', v' scale with the target focal length),
//   F_s = sum of f_i dH/df_i = sum of Z (dH/dX') . (c - m)
//         (X_c = Z ((u - cx)/fx, (v - cy)/fy, 1) and fx, fy scale together, so
//         dX'/dlog f_i = Z R_ji (-(u - cx)/fx, -(v - cy)/fy, 0) = Z (c - m) with
//         c = R_ji e_z the third column of R_ji),
//   and the residual's depth derivative dH/dZ (stored for the source-major
//   depth pass)
template <bool EXT>
__device__ __forceinline__ Terms residual_terms(const Residual& r, const uint2 rec,
                                                const double* c3) {
    Terms t;
    t.S = r.rho;
    t.valid = r.valid;
    t.g0 = r.Au * r.rz;
    t.g1 = r.Av * r.rz;
    t.g2 = r.w * r.rz;
    t.g3 = fmaf(r.yn, r.w, -r.Av);
    t.g4 = fmaf(-r.xn, r.w, r.Au);
    t.g5 = fmaf(r.xn, r.Av, -r.yn * r.Au);
    t.ft = t.fs = t.dz = 0.0f;
    if constexpr (EXT) {
        t.ft = -r.w;
        const float cx = (float)(c3[0] - r.mx), cy = (float)(c3[1] - r.my),
                    cz = (float)(c3[2] - r.mz);
        const float zr = __uint_as_float(rec.y) * r.rz;
        t.fs = zr * fmaf(r.Au, cx, fmaf(r.Av, cy, r.w * cz));
        t.dz = depth_derivative(r);
    }
    return t;
}

__device__ inline double wave_sum(double x) {
#pragma unroll
    for (int m = 32; m >= 1; m >>= 1) x += __shfl_xor(x, m, 64);
    return x;
}

// per-tile sums: S, n, G[6] into partials[t]; the refinement variant adds
// F_t, F_s into ext_partials[2 t ..] and, if dz is given, stores every
// residual's depth derivative in the source-major layout of dz_index
template <int FMT, int P, bool EXT>
__device__ __forceinline__ void do_tile(int64_t t, const uint2* __restrict__ records,
                                        const uint32_t* __restrict__ tex,
                                        const Tile* __restrict__ tiles,
                                        const PairDesc* __restrict__ desc,
                                        const double* __restrict__ rel,
                                        Partial* __restrict__ partials,
                                        double* __restrict__ ext_partials,
                                        const int64_t* __restrict__ dz_index,
                                        float* __restrict__ dz,
                                        const double* __restrict__ pair_scale,
                                        const int64_t* __restrict__ pair_shift, const float* lut,
                                        double (*red)[10], float delta, double zmin) {
    const int tid = threadIdx.x;
    const Tile tl = tiles[t];
    // a pair skipped by this step's sub-sampling (or of a stopped scene): no
    // work, no partials (the pair reduction reads none for it)
    if (pair_scale[tl.pair] == 0.0) return;
    const PairDesc pd = desc[tl.pair];
    const uint32_t* texj = view_texture<FMT>(tex, pd.tex_off);
    // the pair's own record order (per-pair copies), or the source view's
    const uint2* rec = records + tl.rec + (pair_shift ? pair_shift[tl.pair] : 0);
    double c3[3] = {0.0, 0.0, 0.0};
    float* dzt = nullptr;
    int64_t dzn = 0;
    if constexpr (EXT) {
        const double* R = rel + 12 * (int64_t)tl.pair;
        c3[0] = R[2];
        c3[1] = R[5];
        c3[2] = R[8];
        if (dz) {
            // source-major derivative layout: the tile starts a 256-record
            // block of its source, and every further row is the next block
            dzn = dz_index[2 * tl.pair + 1];
            dzt = dz + dz_index[2 * tl.pair] + tl.rec * dzn;
        }
    }
    Acc a{0, 0, 0, 0, 0, 0, 0, 0, 0};
    int n = 0;                                  // valid residuals of this thread
    // two residuals in flight per thread (59 VGPRs, so the SIMD keeps eight
    // waves to hide the record load and the dependent tap gather); unrolling
    // all P would multiply the float64 live ranges (the refinement variant
    // keeps one: its focal sums and ray components would push two past 64
    // VGPRs, below eight waves per SIMD)
    constexpr int U = (P < 2 || EXT) ? 1 : 2;
    // the trip count follows the tile's own size (uniform over the
    // workgroup), so a pair's short last tile costs only its residuals
    const int rows = (tl.count + kBlock - 1) / kBlock;
#pragma unroll 1
    for (int k0 = 0; k0 < rows; k0 += U) {
        uint2 r[U];
        // rows past the tile's end read the records that follow it (the
        // record array carries kRecordPad zero records past its end, more
        // than the at most U * kBlock - 1 rows a tile's last iteration
        // overshoots) and are masked, so both loads issue back to back
        // without a branch; the row base is wave-uniform and each lane adds
        // its own fixed byte offset
        const char* rowb = reinterpret_cast<const char*>(rec) + (size_t)k0 * kBlock * 8;
#pragma unroll
        for (int k = 0; k < U; ++k)
            r[k] = *reinterpret_cast<const uint2*>(rowb + ((uint32_t)tid << 3) + k * kBlock * 8);
        Terms tt[U];
#pragma unroll
        for (int k = 0; k < U; ++k) {
            // row (k0 + k) kBlock + tid is inside the tile: compared against a
            // wave-uniform limit, so no per-lane index arithmetic
            const bool in = tid < tl.count - (k0 + k) * kBlock;
            const Residual rs = eval_residual<FMT>(r[k], in, pd, texj, lut, delta, zmin);
            tt[k] = residual_terms<EXT>(rs, r[k], c3);
            if (EXT && dzt && in) dzt[(int64_t)(k0 + k) * kBlock * dzn + tid] = tt[k].dz;
            n += tt[k].valid ? 1 : 0;
        }
#pragma unroll
        for (int k = 1; k < U; ++k) {
            tt[0].S += tt[k].S;
            tt[0].g0 += tt[k].g0;
            tt[0].g1 += tt[k].g1;
            tt[0].g2 += tt[k].g2;
            tt[0].g3 += tt[k].g3;
            tt[0].g4 += tt[k].g4;
            tt[0].g5 += tt[k].g5;
            tt[0].ft += tt[k].ft;
            tt[0].fs += tt[k].fs;
        }
        a.S += (double)tt[0].S;
        a.g0 += (double)tt[0].g0;
        a.g1 += (double)tt[0].g1;
        a.g2 += (double)tt[0].g2;
        a.g3 += (double)tt[0].g3;
        a.g4 += (double)tt[0].g4;
        a.g5 += (double)tt[0].g5;
        if constexpr (EXT) {
            a.ft += (double)tt[0].ft;
            a.fs += (double)tt[0].fs;
        }
    }
    constexpr int NS = EXT ? 10 : 8;
    double s[NS];
    const int wave = tid >> 6, lane = tid & 63;
    s[0] = a.S;
    s[1] = (double)n;
    s[2] = a.g0;
    s[3] = a.g1;
    s[4] = a.g2;
    s[5] = a.g3;
    s[6] = a.g4;
    s[7] = a.g5;
    if constexpr (EXT) {
        s[8] = a.ft;
        s[9] = a.fs;
    }
#pragma unroll
    for (int k = 0; k < NS; ++k) s[k] = wave_sum(s[k]);
    if (lane == 0) {
#pragma unroll
        for (int k = 0; k < NS; ++k) red[wave][k] = s[k];
    }
    __syncthreads();
    if (tid < NS) {
        const double x = (red[0][tid] + red[1][tid]) + (red[2][tid] + red[3][tid]);
        if (tid < 8)
            partials[t].v[tid] = x;
        else
            ext_partials[2 * t + (tid - 8)] = x;
    }
}

// PERS: persistent work-queue launch (a separate instantiation, so the
// one-workgroup-per-tile form carries none of the claim loop's registers)
template <int FMT, int P, bool EXT, bool PERS>
__global__ __launch_bounds__(kBlock) void edge_cost_kernel(
    const uint2* __restrict__ records, const uint32_t* __restrict__ tex,
    const Tile* __restrict__ tiles, const PairDesc* __restrict__ desc,
    const double* __restrict__ rel, Partial* __restrict__ partials,
    double* __restrict__ ext_partials, const int64_t* __restrict__ dz_index,
    float* __restrict__ dz, const double* __restrict__ pair_scale,
    const int64_t* __restrict__ pair_shift, const int64_t* __restrict__ xcd_begin, const int32_t* __restrict__ tile_list,
    int32_t n_queues, int32_t* __restrict__ counters, int32_t chunk, float delta, double zmin) {
    // queue q holds entries [xcd_begin[q], xcd_begin[q + 1]) of the tile list:
    // every tile in XCD order, or (with pair sub-sampling) the step's compacted
    // list of the selected pairs' tiles, in the same order
    __shared__ float lut[256];
    __shared__ double red[4][10];
    __shared__ int64_t claim;
    const int q0 = (int)(blockIdx.x % (unsigned)n_queues);
    if constexpr (!PERS) {
        // one workgroup per tile; workgroup b runs on XCD b mod 8, so the
        // tiles of queue q (consecutive target views) stay on one XCD's L2
        const int64_t e = xcd_begin[q0] + blockIdx.x / (unsigned)n_queues;
        if (e >= xcd_begin[q0 + 1]) return;
        if (FMT == 2) lut[threadIdx.x] = sqrtf((float)threadIdx.x);
        __syncthreads();
        const int64_t t = tile_list ? (int64_t)tile_list[e] : e;
        do_tile<FMT, P, EXT>(t, records, tex, tiles, desc, rel, partials, ext_partials, dz_index,
                             dz, pair_scale, pair_shift, lut, red, delta, zmin);
        return;
    }
    if (FMT == 2) lut[threadIdx.x] = sqrtf((float)threadIdx.x);
    __syncthreads();
    // persistent: claim runs of consecutive tiles from the own queue, then
    // from the others.  One atomic per run: a queue's counter is one hot L2
    // line, so a claim per tile would serialise on it.  The run length shrinks
    // with the work left in the queue (as last seen by this workgroup), from
    // `chunk` down to one tile, so the queues still drain evenly.
    const int64_t per_queue = gridDim.x / (unsigned)n_queues;
    for (int qi = 0; qi < n_queues; ++qi) {
        const int q = (q0 + qi) % n_queues;
        const int64_t begin = xcd_begin[q], end = xcd_begin[q + 1];
        int64_t seen = 0;                       // counter value at this workgroup's last claim
        for (;;) {
            const int64_t left = end - begin - seen;
            const int run = (int)max((int64_t)1, min((int64_t)chunk, left / (8 * per_queue)));
            if (threadIdx.x == 0) claim = atomicAdd(&counters[q], run);
            __syncthreads();
            seen = claim;
            const int64_t e0 = begin + seen;
            __syncthreads();
            if (e0 >= end) break;
            const int64_t e1 = e0 + run < end ? e0 + run : end;
            for (int64_t e = e0; e < e1; ++e) {
                const int64_t t = tile_list ? (int64_t)tile_list[e] : e;
                do_tile<FMT, P, EXT>(t, records, tex, tiles, desc, rel, partials, ext_partials,
                                     dz_index, dz, pair_scale, pair_shift, lut, red, delta,
                                     zmin);
                __syncthreads();
            }
        }
    }
}


}  // namespace fused
}  // namespace epo
