// Per-iteration hot path on gfx950: relative poses and the fused residual +
// adjoint kernel (paper Eqs. pi, L, L_ij, d_ij; supplementary Alg. 3 and
// Sec. A1.2 "Per-iteration kernels").  The float64 reductions above the tile
// partials are in reduce.hip.
//
// Fused kernel, per residual (source edge pixel p = (u, v) with depth Z of
// view i, directed pair i -> j):
//   lift + warp in one step: X' = Z M (u, v, 1)^T + t_ji with M = R_ji K_i^-1
//     (the paper lifts to the world once per image and projects per pair;
//     folding the pose-free lift into one 3x3 per pair gives the same point
//     with fewer operations), z = X'_z, x_n = X'_x / z, y_n = X'_y / z,
//     u' = fx_j x_n + cx_j, v' = fy_j y_n + cy_j; this coordinate, the
//     validity test and the cell split are float64, the rest of the residual
//     and its adjoint float32;
//   valid iff z > z_min and 0 <= u' < W_j - 1 and 0 <= v' < H_j - 1;
//   bilinear D from the cell floor(u'), floor(v'); d^ = min(D, lambda);
//   rho = Huber(d^); rho' = dHuber/dd^ if D < lambda else 0;
//   adjoint: with A_u = rho' dD/du' fx_j, A_v = rho' dD/dv' fy_j, the
//   normalised target coordinates x_n, y_n and
//   w = -(A_u x_n + A_v y_n), the left-twist gradient of the target pose is
//     (A_u, A_v, w) / z   and   (y_n w - A_v, A_u - x_n w, x_n A_v - y_n A_u)
//   (the translation block is dH/dX', the rotation block X' x dH/dX', in
//   which the depth cancels).
// A refinement variant of the same kernel also sums the focal-scale terms of
// both views (Sec. 3 Camera Refinement); the per-pixel depth gradient comes
// from a second, source-major pass in refine.hip.
// Each thread adds its float32 residual terms in float64; each workgroup
// reduces its tile to eight float64 partial sums (S, n, G[6]) with wave64
// butterflies and an LDS step across its four waves.  Everything above the
// tile is float64 in a fixed order too: per pair (tiles in order), per
// pose (g_j += w_d G_d, g_i += -w_d Ad(T_ji)^T G_d), per scene.
#include "residual.h"

namespace epo {
namespace {

constexpr int kBlock = 256;

// ---------------------------------------------------------------------------
// relative poses and pair descriptors (one thread per directed pair)
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void pair_setup_kernel(
    const double* __restrict__ poses, const float* __restrict__ K, const int32_t* __restrict__ wh,
    const int64_t* __restrict__ view_off, const int64_t* __restrict__ blk_off,
    const PairStatic* __restrict__ ps,
    const float* __restrict__ lambda, float lambda_max, PairDesc* __restrict__ desc,
    double* __restrict__ rel, int32_t D, int32_t* __restrict__ counters, int32_t n_counters,
    int32_t* __restrict__ status) {
    const int d = blockIdx.x * blockDim.x + threadIdx.x;
    if (d < n_counters) counters[d] = 0;      // work queues of the next cost launch
    if (d >= D) return;
    const PairStatic st = ps[d];
    const int i = st.src, j = st.tgt;
    double Ri[9], ti[3], Rj[9], tj[3];
    for (int r = 0; r < 3; ++r) {
        for (int c = 0; c < 3; ++c) {
            Ri[3 * r + c] = poses[12 * i + 4 * r + c];
            Rj[3 * r + c] = poses[12 * j + 4 * r + c];
        }
        ti[r] = poses[12 * i + 4 * r + 3];
        tj[r] = poses[12 * j + 4 * r + 3];
    }
    // R_ji = R_j R_i^T, t_ji = t_j - R_ji t_i
    double R[9], t[3];
    for (int r = 0; r < 3; ++r)
        for (int c = 0; c < 3; ++c)
            R[3 * r + c] = Rj[3 * r + 0] * Ri[3 * c + 0] + Rj[3 * r + 1] * Ri[3 * c + 1] +
                           Rj[3 * r + 2] * Ri[3 * c + 2];
    for (int r = 0; r < 3; ++r)
        t[r] = tj[r] - (R[3 * r + 0] * ti[0] + R[3 * r + 1] * ti[1] + R[3 * r + 2] * ti[2]);
    const double fxi = K[4 * i + 0], fyi = K[4 * i + 1], cxi = K[4 * i + 2], cyi = K[4 * i + 3];
    const double fxj = K[4 * j + 0], fyj = K[4 * j + 1], cxj = K[4 * j + 2], cyj = K[4 * j + 3];
    // M = R_ji K_i^-1
    double M[9];
    for (int r = 0; r < 3; ++r) {
        M[3 * r + 0] = R[3 * r + 0] / fxi;
        M[3 * r + 1] = R[3 * r + 1] / fyi;
        M[3 * r + 2] = R[3 * r + 2] - R[3 * r + 0] * (cxi / fxi) - R[3 * r + 1] * (cyi / fyi);
    }
    PairDesc o;
    for (int k = 0; k < 9; ++k) o.M[k] = M[k];
    for (int k = 0; k < 3; ++k) o.t[k] = t[k];
    o.fxd = fxj;
    o.fyd = fyj;
    o.cxd = cxj;
    o.cyd = cyj;
    o.fx = (float)fxj;
    o.fy = (float)fyj;
    o.wcells = wh[2 * j + 0] - 1;
    o.hcells = wh[2 * j + 1] - 1;
    const float lam = lambda[st.scene];
    if (!(lam <= lambda_max)) atomicOr(status, 2);
    o.lambda = lam;
    // texture addressing of the format in use: blocked u8 quads (blk_off
    // given: width = 128 (blocks per row - 1), the row-of-blocks stride less
    // the part that 32 y0 covers) or row-major per-pixel texels
    o.width = blk_off ? 128 * ((wh[2 * j + 0] + kQuadBlockW - 1) / kQuadBlockW - 1)
                      : wh[2 * j + 0];
    o.tex_off = blk_off ? blk_off[j] : view_off[j];
    desc[d] = o;
    for (int k = 0; k < 9; ++k) rel[12 * d + k] = R[k];
    for (int k = 0; k < 3; ++k) rel[12 * d + 9 + k] = t[k];
}

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
template <int FMT, bool EXT>
__device__ __forceinline__ Terms residual(const uint2 rec, bool active, const PairDesc& pd,
                                          const uint32_t* __restrict__ texj, const float* lut,
                                          float delta, double zmin, const double* c3) {
    const Residual r = eval_residual<FMT>(rec, active, pd, texj, lut, delta, zmin);
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
                                        const double* __restrict__ pair_scale, const float* lut,
                                        double (*red)[10], float delta, double zmin) {
    const int tid = threadIdx.x;
    const Tile tl = tiles[t];
    // a pair skipped by this step's sub-sampling (or of a stopped scene): no
    // work, no partials (the pair reduction reads none for it)
    if (pair_scale[tl.pair] == 0.0) return;
    const PairDesc pd = desc[tl.pair];
    const uint32_t* texj = view_texture<FMT>(tex, pd.tex_off);
    const uint2* rec = records + tl.rec;
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
            const int left = tl.count - (k0 + k) * kBlock;
            const bool in = tid < left;
            tt[k] = residual<FMT, EXT>(r[k], in, pd, texj, lut, delta, zmin, c3);
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
    const int64_t* __restrict__ xcd_begin, const int32_t* __restrict__ tile_list,
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
                             dz, pair_scale, lut, red, delta, zmin);
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
                                     dz_index, dz, pair_scale, lut, red, delta, zmin);
                __syncthreads();
            }
        }
    }
}

template <int FMT, int P, bool EXT>
void launch_cost_kernel(Plan& p, float* dz, hipStream_t s) {
    const uint32_t* tex = FMT == 2   ? p.tex.p
                          : FMT == 3 ? reinterpret_cast<const uint32_t*>(p.tex_q32.p)
                                     : reinterpret_cast<const uint32_t*>(p.tex_f32.p);
    const int nq = p.n_xcd_queues;
    const bool persistent = p.opt.persistent == 1;
    unsigned grid;
    if (persistent) {
        int64_t want = (int64_t)p.n_cu * 8;
        want = std::min<int64_t>(want, ceil_div(p.n_tiles, 1) + nq);
        grid = (unsigned)(ceil_div(want, nq) * nq);
    } else if (compacted_launch(p)) {
        // with pair sub-sampling (or stopped scenes skipped) the step's tile
        // count is known only on the device: enough workgroups for every
        // tile, split as the compacted list is (nq equal queues); those past
        // a queue's end exit at once
        grid = (unsigned)(ceil_div(p.n_tiles, nq) * nq);
    } else {
        int64_t per_q = 0;
        for (int q = 0; q < nq; ++q)
            per_q = std::max<int64_t>(per_q, p.xcd_begin[q + 1] - p.xcd_begin[q]);
        grid = (unsigned)(per_q * nq);
    }
    if (grid == 0) return;
    auto kernel = persistent ? edge_cost_kernel<FMT, P, EXT, true>
                             : edge_cost_kernel<FMT, P, EXT, false>;
    kernel<<<grid, kBlock, 0, s>>>(
        reinterpret_cast<const uint2*>(p.records.p), tex, p.tiles.p, p.pair_desc.p, p.pair_rel.p,
        p.partials.p, EXT ? p.ext_partials.p : nullptr, p.dz_index.p, dz, p.pair_scale.p,
        compacted_launch(p) ? p.qbegin_d.p : p.xcd_begin_d.p,
        compacted_launch(p) ? p.tile_list.p : nullptr, nq, p.counters.p,
        std::max(1, 16384 / p.tile_size), p.params.huber_delta, p.params.z_min);
    EPO_CHECK_LAUNCH();
}

template <int FMT, bool EXT>
void launch_cost_fmt(Plan& p, float* dz, hipStream_t s) {
    switch (p.opt.points_per_thread) {
        case 1: launch_cost_kernel<FMT, 1, EXT>(p, dz, s); break;
        case 2: launch_cost_kernel<FMT, 2, EXT>(p, dz, s); break;
        case 4: launch_cost_kernel<FMT, 4, EXT>(p, dz, s); break;
        case 8: launch_cost_kernel<FMT, 8, EXT>(p, dz, s); break;
        case 16: launch_cost_kernel<FMT, 16, EXT>(p, dz, s); break;
        default: throw Failure{EPO_ERR_UNSUPPORTED, "points_per_thread must be 1, 2, 4, 8 or 16"};
    }
}

template <bool EXT>
void launch_cost_variant(Plan& p, float* dz, hipStream_t s) {
    if (p.opt.texture_format == 2)
        launch_cost_fmt<2, EXT>(p, dz, s);
    else if (p.opt.texture_format == 3)
        launch_cost_fmt<3, EXT>(p, dz, s);
    else
        launch_cost_fmt<1, EXT>(p, dz, s);
}

}  // namespace

void launch_cost(Plan& p, const double* poses, const float* lambda, double* loss,
                 double* pair_cost, int32_t* pair_valid, double* pair_grad, double* grad,
                 const double* upstream, hipStream_t s, const RefineOut* ext) {
    if (p.D > 0) {
        // this step's pair subset (stochastic sub-sampling, stopped scenes
        // skipped), if enabled, and the compacted list of its tiles
        launch_pair_selection(p, p.capture_step ? p.capture_step : p.sample_step, s);
        pair_setup_kernel<<<(unsigned)ceil_div(std::max(p.D, 16), 256), 256, 0, s>>>(
            poses, p.K_d.p, p.wh_d.p, p.view_offset_d.p,
            p.opt.texture_format == 2 ? p.blk_off_d.p : nullptr, p.pair_static.p, lambda,
            p.params.lambda_max, p.pair_desc.p, p.pair_rel.p, p.D, p.counters.p, 8, p.status.p);
        EPO_CHECK_LAUNCH();
        const bool timed = p.timing;
        if (timed) EPO_HIP(hipEventRecord(p.ev0, s));
        // the refinement variant runs for focal gradients, and for depth
        // gradients when the per-residual derivatives can be stored
        const bool depth = ext && (ext->grad_alpha || ext->grad_beta);
        float* dz = depth && p.dz.p ? p.dz.p : nullptr;
        if (ext && (ext->grad_gamma || dz))
            launch_cost_variant<true>(p, dz, s);
        else
            launch_cost_variant<false>(p, nullptr, s);
        if (timed) {
            EPO_HIP(hipEventRecord(p.ev1, s));
            p.timed_once = true;
        }
    }
    launch_reductions(p, loss, pair_cost, pair_valid, pair_grad, grad, upstream, s,
                      ext ? ext->grad_gamma : nullptr);
    if (ext && (ext->grad_alpha || ext->grad_beta))
        launch_depth_grad(p, upstream, ext->grad_alpha, ext->grad_beta, p.D > 0 && p.dz.p, s);
}

}  // namespace epo

extern "C" epo_status epo_edge_cost_fwd(epo_plan plan, const double* poses, const float* lambda,
                                        double* loss, double* pair_cost, int32_t* pair_valid,
                                        double* pair_grad, double* grad, void* stream) {
    using namespace epo;
    return guarded([&] {
        EPO_REQUIRE(plan, "null plan");
        EPO_REQUIRE(poses && lambda && loss, "poses, lambda and loss are required");
        Plan& p = *reinterpret_cast<Plan*>(plan);
        EPO_HIP(hipSetDevice(p.device));
        launch_cost(p, poses, lambda, loss, pair_cost, pair_valid, pair_grad, grad, nullptr,
                    as_stream(stream));
    });
}

extern "C" epo_status epo_edge_cost_bwd(epo_plan plan, const double* poses, const float* lambda,
                                        const double* upstream, double* grad, void* stream) {
    using namespace epo;
    return guarded([&] {
        EPO_REQUIRE(plan, "null plan");
        EPO_REQUIRE(poses && lambda && grad, "poses, lambda and grad are required");
        Plan& p = *reinterpret_cast<Plan*>(plan);
        EPO_HIP(hipSetDevice(p.device));
        launch_cost(p, poses, lambda, nullptr, nullptr, nullptr, nullptr, grad, upstream,
                    as_stream(stream));
    });
}
