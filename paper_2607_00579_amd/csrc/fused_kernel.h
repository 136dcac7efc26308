// Device code of the fused residual + adjoint kernel and its per-tile
// reduction (paper Eqs. pi, d_ij, L_ij; supplementary Alg. 3 and Sec. A1.2
// "Per-iteration kernels"): per residual, residual.h; per thread, float64
// sums; per wave, lane-swap folds and row rotations (no LDS); per workgroup,
// an LDS step to one float64 partial per tile.  Included by edge_cost.hip, which holds the host-side
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

// per-thread sums in float64: from the float32 adjoint factors A_u, A_v of
// each residual (rounded once), the pose-gradient terms are formed and added
// in float64 with fused multiply-adds (the sums cancel strongly, up to a few
// hundred in sum |term| / |sum|); ft, fs are the focal-scale sums of the
// refinement variant
struct Acc {
    double S, g0, g1, g2, g3, g4, g5;
    double ft, fs;
};

// refinement variant (EXT): besides the pose terms, per pair
//   F_t = sum of f_j dH/df_j = sum of (A_u x_n + A_v y_n) = sum of -w
//         (u', v' scale with the target focal length),
//   F_s = sum of f_i dH/df_i = sum of Z (dH/dX') . (c - m)
//         (X_c = Z ((u - cx)/fx, (v - cy)/fy, 1) and fx, fy scale together, so
//         dX'/dlog f_i = Z R_ji (-(u - cx)/fx, -(v - cy)/fy, 0) = Z (c - m) with
//         c = R_ji e_z the third column of R_ji)
// The pose terms (dH/dX' = (A_u, A_v, w) / z, then dH/dxi = (dH/dX', X' x
// dH/dX') in the target frame, written with X' = z (x_n, y_n, 1)):
//   g0..g2 = (A_u, A_v, w) / z,
//   g3 = y_n w - A_v, g4 = A_u - x_n w, g5 = x_n A_v - y_n A_u.
// An invalid residual has A_u = A_v = rho = 0 and finite coordinates, so it
// adds exact zeros.
template <bool EXT>
__device__ __forceinline__ void accumulate(Acc& a, const Residual& r, const uint2 rec,
                                           const double* c3) {
    const double Au = (double)r.Au, Av = (double)r.Av;
    const double w = -fma(Au, r.xd, Av * r.yd);
    a.S += (double)r.rho;
    a.g0 = fma(Au, r.rd, a.g0);
    a.g1 = fma(Av, r.rd, a.g1);
    a.g2 = fma(w, r.rd, a.g2);
    a.g3 = fma(r.yd, w, a.g3) - Av;
    a.g4 = fma(-r.xd, w, a.g4) + Au;
    a.g5 = fma(-r.yd, Au, fma(r.xd, Av, a.g5));
    if constexpr (EXT) {
        a.ft -= w;
        const double zr = (double)__uint_as_float(rec.y) * r.rd;
        a.fs = fma(zr, fma(Au, c3[0] - r.mx, fma(Av, c3[1] - r.my, w * (c3[2] - r.mz))), a.fs);
    }
}

// U consecutive rows of a tile (U kBlock residuals, one per thread and row)
// into the thread's sums; n counts the thread's valid residuals
template <int FMT, int U, bool EXT>
__device__ __forceinline__ void tile_rows(Acc& a, uint32_t& n, const uint2* __restrict__ rec,
                                          int k0, int count, const PairDesc& pd,
                                          const uint32_t* __restrict__ texj, const float* lut,
                                          float delta, double zmin, const double* c3, float* dzt,
                                          int64_t dzn) {
    const int tid = threadIdx.x;
    uint2 r[U];
    // lanes past the tile's end read the records that follow it (the record
    // array carries kRecordPad zero records past its end, more than the at
    // most kBlock - 1 records a tile's last row overshoots) and are masked,
    // so the loads issue back to back without a branch; the row base is
    // wave-uniform and each lane adds its own fixed byte offset
    const char* rowb = reinterpret_cast<const char*>(rec) + (size_t)k0 * kBlock * 8;
#pragma unroll
    for (int k = 0; k < U; ++k)
        r[k] = *reinterpret_cast<const uint2*>(rowb + ((uint32_t)tid << 3) + k * kBlock * 8);
#pragma unroll
    for (int k = 0; k < U; ++k) {
        // row (k0 + k) kBlock + tid is inside the tile: compared against a
        // wave-uniform limit, so no per-lane index arithmetic
        const bool in = tid < count - (k0 + k) * kBlock;
        const Residual rs = eval_residual<FMT>(r[k], in, pd, texj, lut, delta, zmin);
        accumulate<EXT>(a, rs, r[k], c3);
        // the depth derivative dH/dZ for the source-major depth pass
        if (EXT && dzt && in) dzt[(int64_t)(k0 + k) * kBlock * dzn + tid] = depth_derivative(rs);
        n += rs.valid ? 1u : 0u;
    }
}

// Wave reduction of several float64 sums at once.  Each fold halves the
// lanes a sum spans and pairs two sums in one register: fold32 trades lanes
// 32..63 of x with lanes 0..31 of y (v_permlane32_swap) and adds, so lanes
// 0..31 then hold x summed over lanes l and l + 32, lanes 32..63 y's;
// fold16 does the same between the odd 16-lane rows of x and the even rows
// of y (v_permlane16_swap), leaving x's sums in rows 0 and 2 and y's in rows
// 1 and 3.  row_sum finishes within each 16-lane row by rotations (DPP
// row_ror), after which every lane of a row holds the row's total.  No LDS
// traffic and half the additions of one butterfly per sum.
__device__ __forceinline__ double join(uint32_t lo, uint32_t hi) {
    return __longlong_as_double((long long)(((uint64_t)hi << 32) | lo));
}

__device__ __forceinline__ double fold32(double x, double y) {
    const uint64_t xb = (uint64_t)__double_as_longlong(x), yb = (uint64_t)__double_as_longlong(y);
    const auto lo = __builtin_amdgcn_permlane32_swap((uint32_t)xb, (uint32_t)yb, false, false);
    const auto hi = __builtin_amdgcn_permlane32_swap((uint32_t)(xb >> 32), (uint32_t)(yb >> 32),
                                                     false, false);
    return join(lo[0], hi[0]) + join(lo[1], hi[1]);
}

__device__ __forceinline__ double fold16(double x, double y) {
    const uint64_t xb = (uint64_t)__double_as_longlong(x), yb = (uint64_t)__double_as_longlong(y);
    const auto lo = __builtin_amdgcn_permlane16_swap((uint32_t)xb, (uint32_t)yb, false, false);
    const auto hi = __builtin_amdgcn_permlane16_swap((uint32_t)(xb >> 32), (uint32_t)(yb >> 32),
                                                     false, false);
    return join(lo[0], hi[0]) + join(lo[1], hi[1]);
}

template <int N>
__device__ __forceinline__ double row_ror(double x) {
    const uint64_t b = (uint64_t)__double_as_longlong(x);
    const uint32_t lo = (uint32_t)__builtin_amdgcn_mov_dpp((int)(uint32_t)b, 0x120 + N, 0xf, 0xf, false);
    const uint32_t hi =
        (uint32_t)__builtin_amdgcn_mov_dpp((int)(uint32_t)(b >> 32), 0x120 + N, 0xf, 0xf, false);
    return join(lo, hi);
}

__device__ __forceinline__ double row_sum(double x) {
    x += row_ror<8>(x);
    x += row_ror<4>(x);
    x += row_ror<2>(x);
    x += row_ror<1>(x);
    return x;
}

// the wave totals of v[0..NV) (NV = 8 or 10) into red[0..NV)
template <int NV>
__device__ __forceinline__ void wave_sums(const double (&v)[NV], double* red) {
    static_assert(NV == 8 || NV == 10, "");
    constexpr int NA = (NV + 1) / 2, NB = (NA + 1) / 2;
    double A[NA], B[NB];
#pragma unroll
    for (int k = 0; k < NA; ++k) A[k] = fold32(v[2 * k], v[2 * k + 1 < NV ? 2 * k + 1 : 2 * k]);
#pragma unroll
    for (int k = 0; k < NB; ++k) B[k] = fold16(A[2 * k], A[2 * k + 1 < NA ? 2 * k + 1 : 2 * k]);
#pragma unroll
    for (int k = 0; k < NB; ++k) B[k] = row_sum(B[k]);
    // row r of B[k] holds A[a], a = 2 k + (r & 1), and of that its lower
    // (r < 2) or upper half: v[2 a + (r >> 1)]; a row that holds a sum paired
    // with itself (odd counts) is a duplicate and not written
    const int lane = threadIdx.x & 63;
    if ((lane & 15) == 0) {
        const int r = lane >> 4;
#pragma unroll
        for (int k = 0; k < NB; ++k) {
            const int a = 2 * k + (r & 1);
            const int src = 2 * a + (r >> 1);
            if (a < NA && src < NV) red[src] = B[k];
        }
    }
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
    uint32_t n = 0;                             // valid residuals of this thread
    // two residuals in flight per thread (the SIMD keeps eight waves to hide
    // the record load and the dependent tap gather); unrolling all P would
    // multiply the float64 live ranges (the refinement variant keeps one: its
    // focal sums and ray components would push two past 64 VGPRs, below
    // eight waves per SIMD)
    constexpr int U = (P < 2 || EXT) ? 1 : 2;
    // the trip count follows the tile's own size (uniform over the
    // workgroup), so a pair's short last tile costs only its rows; an odd
    // last row runs alone
    const int rows = (tl.count + kBlock - 1) / kBlock;
    int k0 = 0;
#pragma unroll 1
    for (; k0 + U <= rows; k0 += U)
        tile_rows<FMT, U, EXT>(a, n, rec, k0, tl.count, pd, texj, lut, delta, zmin, c3, dzt, dzn);
    if (U > 1 && k0 < rows)
        tile_rows<FMT, 1, EXT>(a, n, rec, k0, tl.count, pd, texj, lut, delta, zmin, c3, dzt, dzn);
    // per wave: S, n, G[6] (and F_t, F_s) into red[wave][0..NS)
    constexpr int NS = EXT ? 10 : 8;
    const int wave = tid >> 6;
    if constexpr (EXT) {
        const double v[10] = {a.S, (double)n, a.g0, a.g1, a.g2, a.g3, a.g4, a.g5, a.ft, a.fs};
        wave_sums<10>(v, red[wave]);
    } else {
        const double v[8] = {a.S, (double)n, a.g0, a.g1, a.g2, a.g3, a.g4, a.g5};
        wave_sums<8>(v, red[wave]);
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
