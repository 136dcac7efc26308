// The paper's pose parameterization on the device (Sec. 3 "Pose Refinement",
// Sec. 4 "Implementation Details"): per scene, every pose comes from its
// initial pose P0 through a refiner MLP, the 6D rotation representation with
// Gram-Schmidt, and a translation offset,
//     P = phi(P0 + MLP(P0)) + [0 | delta],
// trained with AdamW.  MLP: 12 -> 128 -> 128 -> 128 -> 128 -> 128 -> 12,
// ReLU after the first five layers, the first layer's output added to the
// third's (the skip connection), BF16 matrix products with float32
// accumulation (v_mfma_f32_32x32x16_bf16): every product takes bf16 operands
// (weights rounded from their float32 values, activations and activation
// gradients stored in bf16); bias, ReLU, skip sums and masks act on the
// float32 accumulators, rounded once to bf16 where stored; weight and bias
// gradients and the MLP output stay float32.  The pose algebra is float64.
//
// One workgroup (four wave64) per scene, its views in chunks of 64 rows: the
// chunk's activations live in LDS, each layer is a handful of 32 x 32 MFMA
// tiles (two per wave); the forward also stores the activations the backward
// needs.  Weight gradients add up over the chunks in a fixed order, so
// results are bitwise reproducible.
#include "epo_internal.h"

namespace epo {
namespace {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x16 __attribute__((ext_vector_type(16)));

constexpr int kH = 128;           // hidden width
constexpr int kIn = 12;           // pose entries in and out
constexpr int kInPad = 16;        // input width padded to the MFMA k step
constexpr int kRows = 64;         // rows per chunk
constexpr int kLd = kH + 8;       // LDS row stride (bf16) of a forward activation
constexpr int kLdB = kH;          // LDS row stride of a backward gradient (fits 64 KB)

// Packed bf16 weights, per scene (written by mlp_pack_kernel from the float32
// parameters before every forward): the B operand of each product, row j of
// a block holding the eight-element fragments of output column j, so a lane
// reads one fragment with one 16-byte load.
//   forward, layer L:  Wf_L[j][k] = W_L[j][k], rows padded to 32 for the last
//                      layer (12 outputs), columns to 16 for the first (12 inputs)
//   backward, dh_L = dY_{L+1} W_{L+1}:  Wt_L[j][k] = W_{L+1}[k][j], columns
//                      padded to 16 for the last layer (12 outputs)
constexpr int kFwdOff[6] = {0, 2048, 18432, 34816, 51200, 67584};
constexpr int kFwdLd[6] = {16, 128, 128, 128, 128, 128};
constexpr int kBwdOff[6] = {0, 71680, 88064, 104448, 120832, 137216};   // index L = 1..5
constexpr int kBwdLd[6] = {0, 128, 128, 128, 128, 16};
constexpr int kPacked = 139264;
static_assert(kFwdOff[5] + 32 * 128 == kBwdOff[1], "packed forward block");
static_assert(kBwdOff[5] + 128 * 16 == kPacked, "packed backward block");
static_assert(kPacked == kMlpPacked, "packed size");

// parameter offsets (W1, b1, ..., W6, b6), one scene's flat float32 vector
constexpr int kOffW[6] = {0, 1664, 18176, 34688, 51200, 67712};
constexpr int kOffB[6] = {1536, 18048, 34560, 51072, 67584, 69248};
constexpr int kLayerIn[6] = {kIn, kH, kH, kH, kH, kH};
constexpr int kLayerOut[6] = {kH, kH, kH, kH, kH, kIn};
static_assert(kOffB[5] + kIn == EPO_MLP_PARAMS, "parameter layout");

// one 32 x 32 tile of sum_k A(i, k) B(k, j) over k in [0, K), K a multiple of
// 16.  Lane l holds A(l % 32, k0 + 8 (l / 32) + q) and B(k0 + 8 (l / 32) + q,
// l % 32), q = 0..7; accumulator r is element (8 (r / 4) + 4 (l / 32) + r % 4,
// l % 32) of the tile.
template <class FA, class FB>
__device__ __forceinline__ f32x16 mfma_tile(FA A, FB B, int K) {
    const int l = threadIdx.x & 63;
    f32x16 c = {};
    for (int k0 = 0; k0 < K; k0 += 16) {
        bf16x8 a, b;
#pragma unroll
        for (int q = 0; q < 8; ++q) {
            const int k = k0 + 8 * (l >> 5) + q;
            a[q] = A(l & 31, k);
            b[q] = B(k, l & 31);
        }
        c = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a, b, c, 0, 0, 0);
    }
    return c;
}

// the same tile with both operands read as 16-byte fragments: A(i, k) at
// A[(i0 + i) lda + k] (LDS), B(k, j) at B[(j0 + j) ldb + k] (packed weights)
template <int K>
__device__ __forceinline__ f32x16 mfma_tile_vec(const __bf16* A, int lda, int i0,
                                                const __bf16* __restrict__ B, int ldb, int j0) {
    static_assert(K % 16 == 0, "K is a multiple of the MFMA k step");
    constexpr int S = K / 16;
    const int l = threadIdx.x & 63;
    const __bf16* pa = A + (i0 + (l & 31)) * lda + 8 * (l >> 5);
    const __bf16* pb = B + (j0 + (l & 31)) * ldb + 8 * (l >> 5);
    bf16x8 a[S], b[S];
#pragma unroll
    for (int st = 0; st < S; ++st) {
        a[st] = *reinterpret_cast<const bf16x8*>(pa + 16 * st);
        b[st] = *reinterpret_cast<const bf16x8*>(pb + 16 * st);
    }
    f32x16 c = {};
#pragma unroll
    for (int st = 0; st < S; ++st)
        c = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a[st], b[st], c, 0, 0, 0);
    return c;
}

__device__ __forceinline__ int tile_row(int r) { return 8 * (r >> 2) + 4 * ((threadIdx.x & 63) >> 5) + (r & 3); }
__device__ __forceinline__ int tile_col() { return threadIdx.x & 31; }

__device__ __forceinline__ __bf16 to_bf16(float x) { return (__bf16)x; }
__device__ __forceinline__ float to_f32(__bf16 x) { return (float)x; }

// Gram-Schmidt of the first two columns of A (row-major 3 x 3) -> R
__device__ inline void gram_schmidt(const double* A, double* R) {
    double a1[3] = {A[0], A[3], A[6]}, a2[3] = {A[1], A[4], A[7]};
    const double n1 = sqrt(a1[0] * a1[0] + a1[1] * a1[1] + a1[2] * a1[2]);
    double b1[3] = {a1[0] / n1, a1[1] / n1, a1[2] / n1};
    const double c = b1[0] * a2[0] + b1[1] * a2[1] + b1[2] * a2[2];
    double u2[3] = {a2[0] - c * b1[0], a2[1] - c * b1[1], a2[2] - c * b1[2]};
    const double n2 = sqrt(u2[0] * u2[0] + u2[1] * u2[1] + u2[2] * u2[2]);
    double b2[3] = {u2[0] / n2, u2[1] / n2, u2[2] / n2};
    double b3[3] = {b1[1] * b2[2] - b1[2] * b2[1], b1[2] * b2[0] - b1[0] * b2[2],
                    b1[0] * b2[1] - b1[1] * b2[0]};
    for (int r = 0; r < 3; ++r) {
        R[3 * r + 0] = b1[r];
        R[3 * r + 1] = b2[r];
        R[3 * r + 2] = b3[r];
    }
}

__device__ inline void cross3(const double* a, const double* b, double* o) {
    o[0] = a[1] * b[2] - a[2] * b[1];
    o[1] = a[2] * b[0] - a[0] * b[2];
    o[2] = a[0] * b[1] - a[1] * b[0];
}
__device__ inline double dot3(const double* a, const double* b) {
    return a[0] * b[0] + a[1] * b[1] + a[2] * b[2];
}

// dL/dA (row-major 3 x 3, third column 0) from dL/dR = G (row-major)
__device__ inline void gram_schmidt_backward(const double* A, const double* G, double* dA) {
    double a1[3] = {A[0], A[3], A[6]}, a2[3] = {A[1], A[4], A[7]};
    const double n1 = sqrt(dot3(a1, a1));
    double b1[3] = {a1[0] / n1, a1[1] / n1, a1[2] / n1};
    const double c = dot3(b1, a2);
    double u2[3] = {a2[0] - c * b1[0], a2[1] - c * b1[1], a2[2] - c * b1[2]};
    const double n2 = sqrt(dot3(u2, u2));
    double b2[3] = {u2[0] / n2, u2[1] / n2, u2[2] / n2};
    double g1[3] = {G[0], G[3], G[6]}, g2[3] = {G[1], G[4], G[7]}, g3[3] = {G[2], G[5], G[8]};
    double t[3], gb1[3], gb2[3];
    cross3(b2, g3, t);                                   // b3 = b1 x b2
    for (int k = 0; k < 3; ++k) gb1[k] = g1[k] + t[k];
    cross3(g3, b1, t);
    for (int k = 0; k < 3; ++k) gb2[k] = g2[k] + t[k];
    const double p2 = dot3(b2, gb2);                     // b2 = u2 / |u2|
    double gu2[3];
    for (int k = 0; k < 3; ++k) gu2[k] = (gb2[k] - b2[k] * p2) / n2;
    const double p1 = dot3(b1, gu2);                     // u2 = a2 - (b1.a2) b1
    double ga2[3];
    for (int k = 0; k < 3; ++k) {
        ga2[k] = gu2[k] - b1[k] * p1;
        gb1[k] -= c * gu2[k] + p1 * a2[k];
    }
    const double q1 = dot3(b1, gb1);                     // b1 = a1 / |a1|
    for (int r = 0; r < 3; ++r) {
        dA[3 * r + 0] = (gb1[r] - b1[r] * q1) / n1;
        dA[3 * r + 1] = ga2[r];
        dA[3 * r + 2] = 0.0;
    }
}

struct Scratch {
    __bf16* h0;      // [rows][16]
    __bf16* h;       // [5][rows / 64][128][64]: h1 .. h5, each 64-row chunk
                     // column-major (a column's rows contiguous for the
                     // weight-gradient fragments)
    __bf16* r3;      // [rows][128]: relu of the third layer (its mask)
    float* o;        // [rows][12]: MLP outputs
    int64_t rows;    // total rows (the stride of h's layers)
};

// float32 parameters -> packed bf16 operands, one grid row per scene: the
// first kPackFwdBlocks workgroups copy the forward blocks (rows padded,
// coalesced), the others transpose one 32 x 32 tile of a weight matrix each
// through LDS (both the read and the write coalesced)
constexpr int kPackFwdBlocks = 35;                 // x 2048 >= forward block size
constexpr int kPackTiles[6] = {0, 16, 16, 16, 16, 4};   // 32 x 32 tiles of W_1 .. W_5
constexpr int kPackBlocks = kPackFwdBlocks + 68;
static_assert(kPackFwdBlocks * 2048 >= kBwdOff[1], "forward pack coverage");

__global__ __launch_bounds__(256) void mlp_pack_kernel(const float* __restrict__ params,
                                                       __bf16* __restrict__ packed) {
    __shared__ float tile[32][33];
    const int s = blockIdx.y;
    const float* __restrict__ W = params + (int64_t)s * EPO_MLP_PARAMS;
    __bf16* __restrict__ P = packed + (int64_t)s * kPacked;
    if ((int)blockIdx.x < kPackFwdBlocks) {
        for (int u = 0; u < 8; ++u) {
            const int e = (int)blockIdx.x * 2048 + u * 256 + (int)threadIdx.x;
            if (e >= kBwdOff[1]) break;
            int L = 0;
            while (L < 5 && e >= kFwdOff[L + 1]) ++L;
            const int j = (e - kFwdOff[L]) / kFwdLd[L], k = (e - kFwdOff[L]) % kFwdLd[L];
            const float v =
                (j < kLayerOut[L] && k < kLayerIn[L]) ? W[kOffW[L] + j * kLayerIn[L] + k] : 0.0f;
            P[e] = to_bf16(v);
        }
        return;
    }
    // transposed blocks: Wt_L[j][k] = W_L[k][j] (k < out of layer L, else 0)
    int t = (int)blockIdx.x - kPackFwdBlocks, L = 1;
    while (L < 5 && t >= kPackTiles[L]) t -= kPackTiles[L++];
    const int out = kLayerOut[L], in = kLayerIn[L], ld = kBwdLd[L];
    const int nkb = (ld + 31) / 32;                 // tiles along k (the out index)
    const int kb = t % nkb, jb = t / nkb;
    const int c = (int)threadIdx.x & 31, r0 = (int)threadIdx.x >> 5;
    for (int r = r0; r < 32; r += 8) {              // read rows k = kb * 32 + r of W_L
        const int k = kb * 32 + r, j = jb * 32 + c;
        tile[r][c] = (k < out) ? W[kOffW[L] + k * in + j] : 0.0f;
    }
    __syncthreads();
    for (int r = r0; r < 32; r += 8) {              // write rows j = jb * 32 + r of Wt_L
        const int j = jb * 32 + r, k = kb * 32 + c;
        if (k < ld) P[kBwdOff[L] + j * ld + k] = to_bf16(tile[c][r]);
    }
}

__global__ __launch_bounds__(256) void mlp_forward_kernel(
    const float* __restrict__ params, const double* __restrict__ poses0,
    const double* __restrict__ delta, const int32_t* __restrict__ view_ptr,
    const int32_t* __restrict__ view_idx, const int64_t* __restrict__ row_off, Scratch sc,
    const __bf16* __restrict__ packed, double* __restrict__ poses) {
    // 16-byte aligned: the MFMA operands are read as 16-byte fragments
    __shared__ __attribute__((aligned(16))) __bf16 hA[kRows * kLd], hB[kRows * kLd], h1s[kRows * kLd];
    __shared__ float os[kRows * kIn];
    const int s = blockIdx.x;
    const int v0 = view_ptr[s], n = view_ptr[s + 1] - v0;
    const float* __restrict__ W = params + (int64_t)s * EPO_MLP_PARAMS;
    const __bf16* __restrict__ Pk = packed + (int64_t)s * kPacked;
    const int wave = threadIdx.x >> 6;
    for (int c0 = 0; c0 < n; c0 += kRows) {
        const int64_t g0 = row_off[s] + c0;               // first global row of the chunk
        // input: P0 flattened (bf16), zero padding
        for (int k = threadIdx.x; k < kRows * kInPad; k += 256) {
            const int r = k / kInPad, c = k % kInPad;
            const int row = c0 + r;
            const float x = (row < n && c < kIn) ? (float)poses0[12 * view_idx[v0 + row] + c] : 0.0f;
            const __bf16 xb = to_bf16(x);
            hA[r * kLd + c] = xb;
            sc.h0[(g0 + r) * kInPad + c] = xb;
        }
        __syncthreads();
        // layers 1..5 (ping-pong between hA and hB; h1 kept for the skip)
        __bf16* in = hA;
        __bf16* out = hB;
        for (int L = 0; L < 5; ++L) {
            const float* __restrict__ bl = W + kOffB[L];
            __bf16* dst = L == 0 ? h1s : out;
            for (int t = wave; t < (kRows / 32) * (kH / 32); t += 4) {
                const int i0 = 32 * (t / (kH / 32)), j0 = 32 * (t % (kH / 32));
                const f32x16 acc =
                    L == 0 ? mfma_tile_vec<kInPad>(in, kLd, i0, Pk + kFwdOff[0], kFwdLd[0], j0)
                           : mfma_tile_vec<kH>(in, kLd, i0, Pk + kFwdOff[L], kFwdLd[L], j0);
#pragma unroll
                for (int r = 0; r < 16; ++r) {
                    const int i = i0 + tile_row(r), j = j0 + tile_col();
                    const float y = fmaxf(acc[r] + bl[j], 0.0f);
                    __bf16 hv;
                    if (L == 2) {
                        sc.r3[(g0 + i) * kH + j] = to_bf16(y);
                        hv = to_bf16(y + to_f32(h1s[i * kLd + j]));
                    } else {
                        hv = to_bf16(y);
                    }
                    dst[i * kLd + j] = hv;
                }
            }
            __syncthreads();
            {
                // the layer's activations to the store, column-major per chunk
                // (coalesced: consecutive threads take consecutive rows); the
                // next layer only reads dst, so no barrier is needed after
                __bf16* __restrict__ gh = sc.h + (int64_t)L * sc.rows * kH + g0 * kH;
                for (int e = threadIdx.x; e < kRows * kH; e += 256)
                    gh[e] = dst[(e % kRows) * kLd + e / kRows];
            }
            if (L == 0) {
                in = h1s;                                  // layer 2 reads h1
            } else {
                __bf16* t = in == h1s ? hA : in;           // never overwrite h1
                in = out;
                out = t;
            }
        }
        // layer 6: o = h5 W6^T + b6 (float32, 12 outputs)
        {
            const float* __restrict__ bl = W + kOffB[5];
            for (int t = wave; t < kRows / 32; t += 4) {
                const int i0 = 32 * t;
                const f32x16 acc = mfma_tile_vec<kH>(in, kLd, i0, Pk + kFwdOff[5], kFwdLd[5], 0);
#pragma unroll
                for (int r = 0; r < 16; ++r) {
                    const int i = i0 + tile_row(r), j = tile_col();
                    if (j < kIn) {
                        const float y = acc[r] + bl[j];
                        os[i * kIn + j] = y;
                        sc.o[(g0 + i) * kIn + j] = y;
                    }
                }
            }
        }
        __syncthreads();
        // poses: phi(P0 + o) + [0 | delta], float64
        for (int r = threadIdx.x; r < kRows && c0 + r < n; r += 256) {
            const int v = view_idx[v0 + c0 + r];
            double M[12];
            for (int k = 0; k < 12; ++k) M[k] = poses0[12 * v + k] + (double)os[r * kIn + k];
            double A[9] = {M[0], M[1], M[2], M[4], M[5], M[6], M[8], M[9], M[10]}, R[9];
            gram_schmidt(A, R);
            for (int a = 0; a < 3; ++a) {
                for (int b = 0; b < 3; ++b) poses[12 * v + 4 * a + b] = R[3 * a + b];
                poses[12 * v + 4 * a + 3] = M[4 * a + 3] + delta[3 * v + a];
            }
        }
        __syncthreads();
    }
}

// dW (out x in) [+]= dY^T h over the chunk's 64 rows; db [+]= column sums
template <class FD, class FH>
__device__ inline void weight_grad(FD dY, FH h, int out, int in, float* __restrict__ gW,
                                   float* __restrict__ gb, bool first) {
    const int wave = threadIdx.x >> 6;
    const int tm = (out + 31) / 32, tn = (in + 31) / 32;
    for (int t = wave; t < tm * tn; t += 4) {
        const int i0 = 32 * (t / tn), j0 = 32 * (t % tn);
        const f32x16 acc = mfma_tile(
            [&](int i, int k) { return i0 + i < out ? dY(k, i0 + i) : to_bf16(0.0f); },
            [&](int k, int j) { return j0 + j < in ? h(k, j0 + j) : to_bf16(0.0f); }, kRows);
#pragma unroll
        for (int r = 0; r < 16; ++r) {
            const int i = i0 + tile_row(r), j = j0 + tile_col();
            if (i < out && j < in) {
                float* p = gW + i * in + j;
                *p = first ? acc[r] : *p + acc[r];
            }
        }
    }
    for (int j = threadIdx.x; j < out; j += 256) {
        float sum = 0.0f;
        for (int k = 0; k < kRows; ++k) sum += to_f32(dY(k, j));
        gb[j] = first ? sum : gb[j] + sum;
    }
}

// A read element-wise through FA, B as 16-byte fragments: B(k, j) at
// B[(j0 + j) ldb + k]
template <int K, class FA>
__device__ __forceinline__ f32x16 mfma_tile_bvec(FA A, const __bf16* __restrict__ B, int ldb,
                                                 int j0) {
    constexpr int S = K / 16;
    const int l = threadIdx.x & 63;
    const __bf16* pb = B + (j0 + (l & 31)) * ldb + 8 * (l >> 5);
    bf16x8 a[S], b[S];
#pragma unroll
    for (int st = 0; st < S; ++st) {
#pragma unroll
        for (int q = 0; q < 8; ++q) a[st][q] = A(l & 31, 16 * st + 8 * (l >> 5) + q);
        b[st] = *reinterpret_cast<const bf16x8*>(pb + 16 * st);
    }
    f32x16 c = {};
#pragma unroll
    for (int st = 0; st < S; ++st)
        c = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a[st], b[st], c, 0, 0, 0);
    return c;
}

// weight_grad for a 128-wide input whose stored activations are transposed
// per chunk (hT[j kRows + k]: column j of the chunk contiguous over its rows)
template <class FD>
__device__ inline void weight_grad_t(FD dY, const __bf16* __restrict__ hT, int out,
                                     float* __restrict__ gW, float* __restrict__ gb, bool first) {
    const int wave = threadIdx.x >> 6;
    const int tm = (out + 31) / 32, tn = kH / 32;
    for (int t = wave; t < tm * tn; t += 4) {
        const int i0 = 32 * (t / tn), j0 = 32 * (t % tn);
        const f32x16 acc = mfma_tile_bvec<kRows>(
            [&](int i, int k) { return i0 + i < out ? dY(k, i0 + i) : to_bf16(0.0f); }, hT, kRows,
            j0);
#pragma unroll
        for (int r = 0; r < 16; ++r) {
            const int i = i0 + tile_row(r), j = j0 + tile_col();
            if (i < out) {
                float* p = gW + i * kH + j;
                *p = first ? acc[r] : *p + acc[r];
            }
        }
    }
    for (int j = threadIdx.x; j < out; j += 256) {
        float sum = 0.0f;
        for (int k = 0; k < kRows; ++k) sum += to_f32(dY(k, j));
        gb[j] = first ? sum : gb[j] + sum;
    }
}

__global__ __launch_bounds__(256) void mlp_backward_kernel(
    const float* __restrict__ params, const double* __restrict__ poses0,
    const double* __restrict__ poses, const double* __restrict__ grad,
    const int32_t* __restrict__ view_ptr, const int32_t* __restrict__ view_idx,
    const int64_t* __restrict__ row_off, Scratch sc, const __bf16* __restrict__ packed,
    float* __restrict__ param_grad, double* __restrict__ delta_grad) {
    __shared__ __attribute__((aligned(16))) __bf16 dA_[kRows * kLdB], dB_[kRows * kLdB];
    __shared__ float dh3[kRows * kH];
    const int s = blockIdx.x;
    const int v0 = view_ptr[s], n = view_ptr[s + 1] - v0;
    // the weights as the last forward packed them (params holds the same values)
    const __bf16* __restrict__ Pk = packed + (int64_t)s * kPacked;
    float* __restrict__ G = param_grad + (int64_t)s * EPO_MLP_PARAMS;
    const int wave = threadIdx.x >> 6;
    if (n == 0) {
        for (int k = threadIdx.x; k < EPO_MLP_PARAMS; k += 256) G[k] = 0.0f;
        return;
    }
    for (int c0 = 0; c0 < n; c0 += kRows) {
        const bool first = c0 == 0;
        const int64_t g0 = row_off[s] + c0;
        auto hT = [&](int L) {                             // stored h_L (L = 1..5)
            return sc.h + (int64_t)(L - 1) * sc.rows * kH + g0 * kH;
        };
        auto H = [&](int L, int k, int j) { return hT(L)[j * kRows + k]; };
        // dL/do per row from the pose chain (float64), as bf16 operand dY6
        for (int k = threadIdx.x; k < kRows * kInPad; k += 256)
            dA_[(k / kInPad) * kLdB + k % kInPad] = to_bf16(0.0f);
        __syncthreads();
        for (int r = threadIdx.x; r < kRows && c0 + r < n; r += 256) {
            const int v = view_idx[v0 + c0 + r];
            double M[12];
            for (int k = 0; k < 12; ++k) M[k] = poses0[12 * v + k] + (double)sc.o[(g0 + r) * kIn + k];
            const double A[9] = {M[0], M[1], M[2], M[4], M[5], M[6], M[8], M[9], M[10]};
            const double* P = poses + 12 * v;
            const double t[3] = {P[3], P[7], P[11]};
            const double* g = grad + 6 * v;
            double tg[3], w[3];
            cross3(t, g, tg);
            for (int k = 0; k < 3; ++k) w[k] = 0.5 * (g[3 + k] - tg[k]);
            // dL/dR = hat(w) R  (tangent part of the left-twist gradient)
            double GR[9];
            for (int a = 0; a < 3; ++a)
                for (int b = 0; b < 3; ++b) {
                    const double Ra0 = P[4 * 0 + b], Ra1 = P[4 * 1 + b], Ra2 = P[4 * 2 + b];
                    const double h0 = a == 0 ? 0.0 : (a == 1 ? w[2] : -w[1]);
                    const double h1 = a == 0 ? -w[2] : (a == 1 ? 0.0 : w[0]);
                    const double h2 = a == 0 ? w[1] : (a == 1 ? -w[0] : 0.0);
                    GR[3 * a + b] = h0 * Ra0 + h1 * Ra1 + h2 * Ra2;
                }
            double dAm[9];
            gram_schmidt_backward(A, GR, dAm);
            float d_o[12];
            for (int a = 0; a < 3; ++a) {
                for (int b = 0; b < 3; ++b) d_o[4 * a + b] = (float)dAm[3 * a + b];
                d_o[4 * a + 3] = (float)g[a];
                delta_grad[3 * v + a] = g[a];
            }
            for (int k = 0; k < kIn; ++k) dA_[r * kLdB + k] = to_bf16(d_o[k]);
        }
        __syncthreads();
        // layer 6: dW6 = dY6^T h5, db6; dh5 = dY6 W6 -> dY5 = bf16(dh5 [h5 > 0])
        weight_grad_t([&](int k, int i) { return dA_[k * kLdB + i]; }, hT(5), kIn,
                      G + kOffW[5], G + kOffB[5], first);
        __bf16* dYc = dA_;                                   // current layer's dY
        __bf16* dYn = dB_;                                   // next (lower) layer's dY
        for (int L = 5; L >= 1; --L) {
            // dh_L = dY_{L+1} W_{L+1}  (rows x 128), K = out of layer L+1
            const __bf16* __restrict__ Wt = Pk + kBwdOff[L];
            for (int t = wave; t < (kRows / 32) * (kH / 32); t += 4) {
                const int i0 = 32 * (t / (kH / 32)), j0 = 32 * (t % (kH / 32));
                const f32x16 acc = L == 5 ? mfma_tile_vec<kInPad>(dYc, kLdB, i0, Wt, kBwdLd[5], j0)
                                          : mfma_tile_vec<kH>(dYc, kLdB, i0, Wt, kBwdLd[L], j0);
#pragma unroll
                for (int r = 0; r < 16; ++r) {
                    const int i = i0 + tile_row(r), j = j0 + tile_col();
                    float d = acc[r];
                    float mask;
                    if (L == 3) {                            // h3 = relu(y3) + h1
                        dh3[i * kH + j] = d;
                        mask = to_f32(sc.r3[(g0 + i) * kH + j]) > 0.0f ? 1.0f : 0.0f;
                    } else {
                        if (L == 1) d += dh3[i * kH + j];    // the skip's share of dh1
                        mask = to_f32(H(L, i, j)) > 0.0f ? 1.0f : 0.0f;
                    }
                    dYn[i * kLdB + j] = to_bf16(d * mask);
                }
            }
            __syncthreads();
            // dW_L = dY_L^T h_{L-1}, db_L
            if (L >= 2) {
                weight_grad_t([&](int k, int i) { return dYn[k * kLdB + i]; }, hT(L - 1), kH,
                              G + kOffW[L - 1], G + kOffB[L - 1], first);
            } else {
                weight_grad([&](int k, int i) { return dYn[k * kLdB + i]; },
                            [&](int k, int j) { return sc.h0[(g0 + k) * kInPad + j]; }, kH, kIn,
                            G + kOffW[0], G + kOffB[0], first);
            }
            __syncthreads();
            __bf16* t = dYc;
            dYc = dYn;
            dYn = t;
        }
    }
}

// AdamW (decoupled weight decay, then Adam) on every scene's MLP parameters
// (float32) and every view's translation offset (float64), learning rate per
// scene; the step counter is read here and advanced by step_advance_kernel
__global__ __launch_bounds__(256) void adamw_kernel(
    float* __restrict__ x, float* __restrict__ m, float* __restrict__ v,
    const float* __restrict__ g, int64_t n_params, double* __restrict__ d,
    double* __restrict__ dm, double* __restrict__ dv, const double* __restrict__ dg,
    const int32_t* __restrict__ scene_of_view, int32_t n_views, const double* __restrict__ lr,
    double b1, double b2, double eps, double wd_mlp, double wd_delta,
    const int32_t* __restrict__ step) {
    const double s = (double)(step[0] + 1);
    const double c1 = 1.0 - pow(b1, s), c2 = 1.0 - pow(b2, s);
    const int64_t total = n_params + 3 * (int64_t)n_views;
    // 1 - beta formed in float64 before rounding: (1 - (float)0.999) is off
    // by 1.3e-5 relative
    const float b1f = (float)b1, b2f = (float)b2;
    const float omb1 = (float)(1.0 - b1), omb2 = (float)(1.0 - b2);
    for (int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; k < total;
         k += (int64_t)gridDim.x * blockDim.x) {
        if (k < n_params) {
            const float a = (float)lr[k / EPO_MLP_PARAMS];
            const float gk = g[k];
            float xk = x[k] * (1.0f - a * (float)wd_mlp);
            const float mk = b1f * m[k] + omb1 * gk;
            const float vk = b2f * v[k] + omb2 * gk * gk;
            m[k] = mk;
            v[k] = vk;
            xk -= a * (mk / (float)c1) / (sqrtf(vk / (float)c2) + (float)eps);
            x[k] = xk;
        } else {
            const int64_t q = k - n_params;
            const double a = lr[scene_of_view[q / 3]];
            const double gk = dg[q];
            double xk = d[q] * (1.0 - a * wd_delta);
            const double mk = b1 * dm[q] + (1.0 - b1) * gk;
            const double vk = b2 * dv[q] + (1.0 - b2) * gk * gk;
            dm[q] = mk;
            dv[q] = vk;
            xk -= a * (mk / c1) / (sqrt(vk / c2) + eps);
            d[q] = xk;
        }
    }
}

__global__ void step_advance_kernel(int32_t* step) { step[0] += 1; }

Scratch scratch_of(Plan& p) {
    Scratch sc;
    sc.rows = p.mlp_rows;
    sc.h0 = reinterpret_cast<__bf16*>(p.mlp_act.p);
    sc.h = sc.h0 + sc.rows * kInPad;
    sc.r3 = sc.h + 5 * sc.rows * kH;
    sc.o = p.mlp_out.p;
    return sc;
}

}  // namespace

void mlp_setup(Plan& p, hipStream_t s) {
    if (p.mlp_act.p) return;
    std::vector<int32_t> vp(p.S + 1);
    EPO_HIP(hipMemcpyAsync(vp.data(), p.scene_view_ptr.p, sizeof(int32_t) * (p.S + 1),
                           hipMemcpyDeviceToHost, s));
    EPO_HIP(hipStreamSynchronize(s));
    std::vector<int64_t> off(p.S + 1, 0);
    for (int k = 0; k < p.S; ++k)
        off[k + 1] = off[k] + ceil_div(vp[k + 1] - vp[k], kRows) * kRows;
    p.mlp_rows = std::max<int64_t>(off[p.S], kRows);
    p.mlp_row_off.alloc(p.S + 1);
    EPO_HIP(hipMemcpyAsync(p.mlp_row_off.p, off.data(), sizeof(int64_t) * (p.S + 1),
                           hipMemcpyHostToDevice, s));
    p.mlp_act.alloc((size_t)p.mlp_rows * (kInPad + 6 * kH));
    p.mlp_out.alloc((size_t)p.mlp_rows * kIn);
    p.mlp_packed.alloc((size_t)p.S * kPacked);
    EPO_HIP(hipStreamSynchronize(s));
}

void launch_mlp_forward(Plan& p, const float* params, const double* poses0, const double* delta,
                        double* poses, hipStream_t s) {
    __bf16* packed = reinterpret_cast<__bf16*>(p.mlp_packed.p);
    mlp_pack_kernel<<<dim3(kPackBlocks, (unsigned)p.S), 256, 0, s>>>(params, packed);
    EPO_CHECK_LAUNCH();
    mlp_forward_kernel<<<(unsigned)p.S, 256, 0, s>>>(params, poses0, delta, p.scene_view_ptr.p,
                                                     p.scene_view_idx.p, p.mlp_row_off.p,
                                                     scratch_of(p), packed, poses);
    EPO_CHECK_LAUNCH();
}

void launch_mlp_backward(Plan& p, const float* params, const double* poses0, const double* poses,
                         const double* grad, float* param_grad, double* delta_grad,
                         hipStream_t s) {
    mlp_backward_kernel<<<(unsigned)p.S, 256, 0, s>>>(params, poses0, poses, grad,
                                                      p.scene_view_ptr.p, p.scene_view_idx.p,
                                                      p.mlp_row_off.p, scratch_of(p),
                                                      reinterpret_cast<const __bf16*>(p.mlp_packed.p),
                                                      param_grad, delta_grad);
    EPO_CHECK_LAUNCH();
}

void launch_adamw(Plan& p, float* params, float* m, float* v, const float* g, double* delta,
                  double* dm, double* dv, const double* dg, const double* lr, double b1, double b2,
                  double eps, double wd_mlp, double wd_delta, int32_t* step, hipStream_t s) {
    const int64_t n = (int64_t)p.S * EPO_MLP_PARAMS;
    const int64_t total = n + 3 * (int64_t)p.V;
    const unsigned grid = (unsigned)std::min<int64_t>(ceil_div(total, 256), 4096);
    adamw_kernel<<<grid, 256, 0, s>>>(params, m, v, g, n, delta, dm, dv, dg, p.scene_of_view_d.p,
                                      p.V, lr, b1, b2, eps, wd_mlp, wd_delta, step);
    EPO_CHECK_LAUNCH();
    step_advance_kernel<<<1, 1, 0, s>>>(step);
    EPO_CHECK_LAUNCH();
}

}  // namespace epo

using namespace epo;

extern "C" epo_status epo_mlp_forward(epo_plan plan, const float* params, const double* poses0,
                                      const double* delta, double* poses, void* stream) {
    return guarded([&] {
        EPO_REQUIRE(plan && params && poses0 && delta && poses, "null argument");
        Plan& p = *reinterpret_cast<Plan*>(plan);
        EPO_HIP(hipSetDevice(p.device));
        EPO_REQUIRE(p.mlp_act.p, "call epo_mlp_setup first");
        launch_mlp_forward(p, params, poses0, delta, poses, as_stream(stream));
    });
}

extern "C" epo_status epo_mlp_backward(epo_plan plan, const float* params, const double* poses0,
                                       const double* poses, const double* grad,
                                       float* param_grad, double* delta_grad, void* stream) {
    return guarded([&] {
        EPO_REQUIRE(plan && params && poses0 && poses && grad && param_grad && delta_grad,
                    "null argument");
        Plan& p = *reinterpret_cast<Plan*>(plan);
        EPO_HIP(hipSetDevice(p.device));
        EPO_REQUIRE(p.mlp_act.p, "call epo_mlp_setup first");
        launch_mlp_backward(p, params, poses0, poses, grad, param_grad, delta_grad,
                            as_stream(stream));
    });
}

extern "C" epo_status epo_mlp_setup(epo_plan plan, void* stream) {
    return guarded([&] {
        EPO_REQUIRE(plan, "null plan");
        Plan& p = *reinterpret_cast<Plan*>(plan);
        EPO_HIP(hipSetDevice(p.device));
        mlp_setup(p, as_stream(stream));
    });
}

extern "C" epo_status epo_mlp_step(epo_plan plan, float* params, float* adam_m, float* adam_v,
                                   const float* param_grad, double* delta, double* delta_m,
                                   double* delta_v, const double* delta_grad, const double* lr,
                                   double beta1, double beta2, double eps, double wd_mlp,
                                   double wd_delta, int32_t* step, void* stream) {
    return guarded([&] {
        EPO_REQUIRE(plan && params && adam_m && adam_v && param_grad && delta && delta_m &&
                        delta_v && delta_grad && lr && step,
                    "null argument");
        Plan& p = *reinterpret_cast<Plan*>(plan);
        EPO_HIP(hipSetDevice(p.device));
        launch_adamw(p, params, adam_m, adam_v, param_grad, delta, delta_m, delta_v, delta_grad,
                     lr, beta1, beta2, eps, wd_mlp, wd_delta, step, as_stream(stream));
    });
}
