// One edge-alignment residual and its adjoint terms (paper Eqs. pi, d_ij,
// Sec. A1.2 "Per-iteration kernels"), shared by the pair-major fused kernel
// and the source-major depth-gradient kernel.
//
// For a source edge record (u, v, Z) of view i and the descriptor of pair
// i -> j:
//   m  = M (u, v, 1)^T with M = R_ji K_i^-1 (the unit-depth ray in the target
//        frame), X' = Z m + t_ji (float64);
//   z  = X'_z; x_n = X'_x / z, y_n = X'_y / z; u' = fx_j x_n + cx_j, v' likewise;
//   valid iff z > z_min and 0 <= u' < W_j - 1 and 0 <= v' < H_j - 1;
//   D  = bilinear sample of DTF_j in the cell floor(u'), floor(v');
//   rho = Huber(min(D, lambda)), rho' its derivative (0 where D >= lambda);
//   A_u = rho' dD/du' fx_j, A_v = rho' dD/dv' fy_j, w = -(A_u x_n + A_v y_n),
//   so that dH/dX' = (A_u, A_v, w) / z.
#pragma once

#include "epo_internal.h"

namespace epo {

// The tap loads address the view's texture with a 32-bit byte offset from a
// wave-uniform base.  A view has at most 16384^2 pixels, so a 4-byte texel
// offset fits in 32 bits; the 16-byte texels of format 3 do not, and use a
// 64-bit index.  (Raw buffer loads with the same offsets, which would spare
// the 64-bit address add, measured 2 % slower on the fused kernel.)
__device__ __forceinline__ uint32_t texel32(const uint32_t* __restrict__ tex, uint32_t byte_off) {
    return *reinterpret_cast<const uint32_t*>(reinterpret_cast<const char*>(tex) + byte_off);
}

// An invalid residual reads texel 0 of the view (a mask
// rather than a select keeps the compiler from branching around the index
// arithmetic).
__device__ __forceinline__ uint32_t mask_texel(uint32_t idx, bool valid) {
    return idx & (valid ? ~0u : 0u);
}

template <int FMT>
struct Taps;

// first texel of view j: the descriptor's tex_off counts texels of the
// format (4 bytes for formats 1 and 2, 16 bytes for format 3)
template <int FMT>
__device__ __forceinline__ const uint32_t* view_texture(const uint32_t* __restrict__ tex,
                                                        int64_t tex_off) {
    if constexpr (FMT == 3)
        return reinterpret_cast<const uint32_t*>(reinterpret_cast<const float4*>(tex) + tex_off);
    else
        return tex + tex_off;
}

// texel of cell (x0, y0) in a row-major per-pixel texture of row stride W
__device__ __forceinline__ uint32_t row_major_texel(int x0, int y0, int W) {
    return (uint32_t)(__umul24(y0, W) + x0);
}

// Each format's texels come in two steps, so that a caller can issue the
// gathers of several residuals (and further loads) before it waits for any:
// fetch() issues the gather(s) of the cell, decode() turns the raw texel into
// the four taps d00, d10, d01, d11.

// float32 texture: four gathers
template <>
struct Taps<1> {
    using Raw = float4;
    __device__ static inline uint32_t index(int x0, int y0, int W) {
        return row_major_texel(x0, y0, W);
    }
    __device__ static inline Raw fetch(const uint32_t* __restrict__ tex, uint32_t idx, int W) {
        const uint32_t o = idx << 2, row = (uint32_t)W << 2;
        return make_float4(__uint_as_float(texel32(tex, o)), __uint_as_float(texel32(tex, o + 4u)),
                           __uint_as_float(texel32(tex, o + row)),
                           __uint_as_float(texel32(tex, o + row + 4u)));
    }
    __device__ static inline void decode(const Raw& q, const float* /*lut*/, float& d00,
                                         float& d10, float& d01, float& d11) {
        d00 = q.x;
        d10 = q.y;
        d01 = q.z;
        d11 = q.w;
    }
};

// saturated u8 quads: one gather, four LDS look-ups of sqrt(k); texels in
// 8 x 4 pixel blocks (one 128-byte line each), blocks row-major.  index()
// returns the byte offset of the texel of cell (x0, y0):
//   4 (32 (a nbx + x0 / 8) + 8 (y0 % 4) + x0 % 8),  a = y0 / 4,
// written as a k + 32 y0 + 4 (x0 + 3 (x0 & ~7)) with k = 128 (nbx - 1) (the
// descriptor's width field for this format): two 24-bit multiply-adds, shifts
template <>
struct Taps<2> {
    using Raw = uint32_t;
    __device__ static inline uint32_t index(int x0, int y0, int k) {
        const uint32_t x = (uint32_t)x0, y = (uint32_t)y0;
        return __umul24(y >> 2, (uint32_t)k) + (y << 5) + ((__umul24(x & ~7u, 3u) + x) << 2);
    }
    __device__ static inline Raw fetch(const uint32_t* __restrict__ tex, uint32_t off,
                                       int /*W*/) {
        return texel32(tex, off);
    }
    __device__ static inline void decode(const Raw& q, const float* lut, float& d00, float& d10,
                                         float& d01, float& d11) {
        d00 = lut[q & 0xffu];
        d10 = lut[(q >> 8) & 0xffu];
        d01 = lut[(q >> 16) & 0xffu];
        d11 = lut[q >> 24];
    }
};

// float32 quads: the four float32 taps of the cell in one 16-byte gather
template <>
struct Taps<3> {
    using Raw = float4;
    __device__ static inline uint32_t index(int x0, int y0, int W) {
        return row_major_texel(x0, y0, W);
    }
    __device__ static inline Raw fetch(const uint32_t* __restrict__ tex, uint32_t idx,
                                       int /*W*/) {
        return reinterpret_cast<const float4*>(tex)[idx];
    }
    __device__ static inline void decode(const Raw& q, const float* /*lut*/, float& d00,
                                         float& d10, float& d01, float& d11) {
        d00 = q.x;
        d10 = q.y;
        d01 = q.z;
        d11 = q.w;
    }
};

struct Residual {
    float rho;              // Huber value (0 if invalid)
    float Au, Av, w;        // adjoint terms (0 if invalid)
    float xn, yn, rz;       // normalised target coordinates, 1 / z
    bool valid;
    double mx, my, mz;      // unit-depth ray m = M (u, v, 1)^T in the target frame
    double xd, yd, rd;      // x_n, y_n, 1 / z in float64
};

// first step: the projected coordinate, the validity test, the cell split and
// the texel to gather
struct Projected {
    float al, be;           // position inside the cell
    float xn, yn, rz;       // normalised target coordinates, 1 / z
    bool valid;
    uint32_t idx;           // the format's texel index (0 if invalid)
    double mx, my, mz;      // unit-depth ray m = M (u, v, 1)^T in the target frame
    double xd, yd, rd;      // x_n, y_n, 1 / z in float64
};

template <int FMT>
__device__ __forceinline__ Projected project_residual(const uint2 rec, bool active,
                                                      const PairDesc& pd, double zmin) {
    Projected r;
    // projected coordinate in float64 (full rate on CDNA4 with packed FP32
    // off): it decides the bilinear cell, an integer, exactly as the oracle
    const double u = (double)(rec.x & 0xffffu);
    const double v = (double)(rec.x >> 16);
    const double Z = (double)__uint_as_float(rec.y);
    r.mx = fma(pd.M[0], u, fma(pd.M[1], v, pd.M[2]));
    r.my = fma(pd.M[3], u, fma(pd.M[4], v, pd.M[5]));
    r.mz = fma(pd.M[6], u, fma(pd.M[7], v, pd.M[8]));
    const double Xx = fma(Z, r.mx, pd.t[0]);
    const double Xy = fma(Z, r.my, pd.t[1]);
    const double Xz = fma(Z, r.mz, pd.t[2]);
    // 1 / z: hardware reciprocal refined by one Newton step, which squares its
    // relative error (exact when z is a power of two; the parity tests hold
    // the valid counts and cells to the float64 oracle).  It is taken of
    // max(z, z_min), so every coordinate below stays finite for invalid
    // residuals too (z <= z_min fails the validity test on z itself) and only
    // the tap index needs masking
    const double zc = fmax(Xz, zmin);
    double rzd = __builtin_amdgcn_rcp(zc);
    rzd = fma(rzd, fma(-zc, rzd, 1.0), rzd);
    const double xnd = Xx * rzd, ynd = Xy * rzd;          // normalised target coordinates
    const double upd = fma(pd.fxd, xnd, pd.cxd);
    const double vpd = fma(pd.fyd, ynd, pd.cyd);
    // 0 <= u' < W - 1 holds exactly when the cell column floor(u') lies in
    // [0, W - 2]: one unsigned compare of the (saturating) integer cell index.
    // Depths and focal lengths are finite (checked when the plan is built and
    // flagged by the refinement update), so u' is finite; should a non-finite
    // value get through anyway, NaN converts to cell 0, so every read stays
    // inside the texture.
    const double fx0 = floor(upd), fy0 = floor(vpd);
    const int x0 = (int)fx0, y0 = (int)fy0;
    r.valid = active && (Xz > zmin) && ((unsigned)x0 < (unsigned)pd.wcells) &&
              ((unsigned)y0 < (unsigned)pd.hcells);
    // an invalid residual reads the taps of cell (0, 0) and gets zero weight
    // (rho = rho' = 0) below; its coordinates are finite, so every product
    // with that zero weight is zero
    r.al = (float)(upd - fx0);
    r.be = (float)(vpd - fy0);
    // y0 < H and W are below 2^24 whenever the residual is valid; idx is
    // the format's texel index (byte offset for format 2)
    r.idx = mask_texel(Taps<FMT>::index(x0, y0, pd.width), r.valid);
    r.xd = xnd;
    r.yd = ynd;
    r.rd = rzd;
    r.xn = (float)xnd;
    r.yn = (float)ynd;
    r.rz = (float)rzd;
    return r;
}

// second step: bilinear sample, clamp, Huber and the adjoint terms from the
// cell's four taps
__device__ __forceinline__ Residual finish_residual(const Projected& p, float d00, float d10,
                                                    float d01, float d11, const PairDesc& pd,
                                                    float delta) {
    Residual r;
    r.mx = p.mx;
    r.my = p.my;
    r.mz = p.mz;
    r.xn = p.xn;
    r.yn = p.yn;
    r.rz = p.rz;
    r.xd = p.xd;
    r.yd = p.yd;
    r.rd = p.rd;
    const bool valid = p.valid;
    // bilinear sample and its gradient; the cell's cross term
    // d11 - d10 - d01 + d00 is formed once and serves both directions
    const float e0 = d10 - d00, f0 = d01 - d00;
    const float c = (d11 - d01) - e0;
    const float gu = fmaf(p.be, c, e0);
    const float gv = fmaf(p.al, c, f0);
    const float D = fmaf(p.be, gv, fmaf(p.al, e0, d00));
    // Huber of the clamped distance: with m = min(d, delta),
    // m (d - m / 2) is d^2 / 2 below delta and delta (d - delta / 2) above
    // (the same float32 roundings as either branch), and m is the derivative,
    // 0 where the distance is clamped (d >= lambda).  An invalid residual
    // takes d = 0: value and derivative 0
    const float Dv = valid ? D : 0.0f;              // D is finite
    const float dh = fminf(Dv, pd.lambda);
    const float m = fminf(dh, delta);
    r.rho = m * fmaf(-0.5f, m, dh);
    const float drho = Dv < pd.lambda ? m : 0.0f;
    r.Au = drho * gu * pd.fx;
    r.Av = drho * gv * pd.fy;
    r.w = -fmaf(r.Au, r.xn, r.Av * r.yn);
    r.valid = valid;
    return r;
}

template <int FMT>
__device__ __forceinline__ Residual eval_residual(const uint2 rec, bool active,
                                                  const PairDesc& pd,
                                                  const uint32_t* __restrict__ texj,
                                                  const float* lut, float delta, double zmin) {
    const Projected p = project_residual<FMT>(rec, active, pd, zmin);
    const typename Taps<FMT>::Raw q = Taps<FMT>::fetch(texj, p.idx, pd.width);
    float d00, d10, d01, d11;
    Taps<FMT>::decode(q, lut, d00, d10, d01, d11);
    return finish_residual(p, d00, d10, d01, d11, pd, delta);
}

// dH/dZ of the source pixel's depth: X' = Z m + t, so dH/dZ = (dH/dX') . m
// with dH/dX' = (A_u, A_v, w) / z.  Since w = -(A_u x_n + A_v y_n), the
// vector (A_u, A_v, w) is orthogonal to X', and its dot with m = (X' - t) / Z
// is small next to its terms when the baseline t is small next to Z m: in
// float32 the roundings of A_u, A_v and w would be amplified by about
// |Z m| / |t|.  So w and the dot are formed in float64 from the float64
// coordinates (the cancellation then leaves float64 rounding) and the result
// is rounded to float32 once.  One expression shared by the kernel that
// stores it and the one that recomputes it, so both give the same value.
__device__ __forceinline__ float depth_derivative(const Residual& r) {
    const double Au = (double)r.Au, Av = (double)r.Av;
    const double w = -fma(Au, r.xd, Av * r.yd);
    return (float)(r.rd * fma(Au, r.mx, fma(Av, r.my, w * r.mz)));
}

}  // namespace epo
