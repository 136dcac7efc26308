// Plan construction and the host-side runtime around the per-iteration
// kernels: edge compaction, sampling textures, the (pair, chunk) tile
// schedule, CSR lists for the fixed-order float64 reductions, the autotuner,
// the captured iteration and the error/status plumbing.
//
// Edge records: every nonzero pixel of E_i (the paper's edge points, Alg. 1
// ExtractEdges; all of them, no sub-sampling) becomes one 8-byte record
// (u: uint16, v: uint16, Z: float32).  Records are ordered by 16 x 16 pixel
// tile, row-major inside a tile, so that the threads of a wave hold nearby
// source pixels whose projections fall in nearby target pixels.
//
// Sampling textures:
//   format 1  float32 sqrt(d2) per pixel, row-major like the maps
//   format 2  per pixel the four taps of the bilinear cell whose top-left
//             corner is the pixel, as bytes min(d2, 255), stored in blocks of
//             8 x 4 pixels (one 128-byte line each), blocks row-major.  The
//             DTF is 1-Lipschitz, so when
//             any tap of a cell has d2 >= 255 every tap is at least
//             sqrt(255) - sqrt(2) > 14.55; the sample then exceeds any clamp
//             lambda <= 14.5 with both the true and the saturated taps, and is
//             clamped with zero gradient either way.  Below saturation the
//             taps are the same float32 sqrt(d2) as format 1, so both formats
//             give bitwise identical residuals.
//   format 3  per pixel the four float32 taps of the cell (16 bytes),
//             row-major.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstring>
#include <memory>
#include <numeric>
#include <unordered_map>

#include "epo_internal.h"

namespace epo {

static thread_local std::string g_last_error;
void set_error(const std::string& msg) { g_last_error = msg; }
void clear_error() { g_last_error.clear(); }

namespace {

constexpr int kTile = 16;          // edge-record ordering tile (pixels)
constexpr float kQ8LambdaMax = 14.5f;

__device__ inline int view_of(const int64_t* __restrict__ first, int V, int64_t t) {
    int lo = 0, hi = V;            // first[lo] <= t < first[hi]
    while (hi - lo > 1) {
        const int mid = (lo + hi) >> 1;
        if (first[mid] <= t) lo = mid; else hi = mid;
    }
    return lo;
}

// one workgroup per 16 x 16 tile of one view; count edge pixels
__global__ __launch_bounds__(256) void count_tiles_kernel(
    const uint8_t* __restrict__ edge, const int64_t* __restrict__ view_off,
    const int32_t* __restrict__ wh, const int64_t* __restrict__ tile_first, int V,
    int32_t* __restrict__ counts) {
    const int64_t t = blockIdx.x;
    const int v = view_of(tile_first, V, t);
    const int W = wh[2 * v], H = wh[2 * v + 1];
    const int tx_n = (W + kTile - 1) / kTile;
    const int64_t local = t - tile_first[v];
    const int tx = (int)(local % tx_n), ty = (int)(local / tx_n);
    const int x = tx * kTile + (threadIdx.x & 15), y = ty * kTile + (threadIdx.x >> 4);
    const bool e = x < W && y < H && edge[view_off[v] + (int64_t)y * W + x] != 0;
    const int c = __syncthreads_count(e);
    if (threadIdx.x == 0) counts[t] = c;
}

__global__ __launch_bounds__(256) void scatter_records_kernel(
    const uint8_t* __restrict__ edge, const float* __restrict__ depth,
    const int64_t* __restrict__ view_off, const int32_t* __restrict__ wh,
    const int64_t* __restrict__ tile_first, int V, const int64_t* __restrict__ tile_rec,
    uint64_t* __restrict__ records, int32_t* __restrict__ bad_depth) {
    __shared__ int wave_cnt[4];
    const int64_t t = blockIdx.x;
    const int v = view_of(tile_first, V, t);
    const int W = wh[2 * v], H = wh[2 * v + 1];
    const int tx_n = (W + kTile - 1) / kTile;
    const int64_t local = t - tile_first[v];
    const int tx = (int)(local % tx_n), ty = (int)(local / tx_n);
    const int x = tx * kTile + (threadIdx.x & 15), y = ty * kTile + (threadIdx.x >> 4);
    const int64_t pix = view_off[v] + (int64_t)y * W + x;
    const bool e = x < W && y < H && edge[pix] != 0;
    const uint64_t mask = __ballot(e);
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int below = __popcll(mask & ((1ull << lane) - 1ull));
    if (lane == 0) wave_cnt[wave] = __popcll(mask);
    __syncthreads();
    int base = 0;
    for (int k = 0; k < wave; ++k) base += wave_cnt[k];
    if (e) {
        const float zf = depth[pix];
        if (!isfinite(zf)) atomicOr(bad_depth, 1);
        const uint32_t z = __float_as_uint(zf);
        records[tile_rec[t] + base + below] =
            (uint64_t)((uint32_t)x | ((uint32_t)y << 16)) | ((uint64_t)z << 32);
    }
}

// float32 sqrt(d2) per pixel: the texture of format 1, and the source the
// other formats are derived from (d2 is not kept by the plan)
__global__ __launch_bounds__(256) void texture_f32_kernel(const int32_t* __restrict__ d2,
                                                          const int64_t* __restrict__ view_off,
                                                          const int32_t* __restrict__ wh,
                                                          float* __restrict__ f32) {
    const int v = blockIdx.y;
    const int64_t n = (int64_t)wh[2 * v] * wh[2 * v + 1], base = view_off[v];
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x)
        f32[base + i] = sqrtf((float)d2[base + i]);
}

// min(d2, 255) from the float32 texture: for d2 <= 255, f = sqrt(d2) rounded
// to float32 squares back to d2 within 5e-5, and f >= 16 exactly when d2 >= 256
__device__ __forceinline__ uint32_t saturated_d2(float f) {
    return f < 16.0f ? (uint32_t)rintf(f * f) : 255u;
}

// the four taps of the bilinear cell at every pixel, as float32 (format 3) or
// as saturated d2 bytes in 8 x 4 pixel blocks (format 2), from the float32
// texture.  Format 3 repeats a pixel past the right column / bottom row,
// format 2 stores 255 there: no valid sample ever uses those cells
__global__ __launch_bounds__(256) void texture_quads_kernel(const float* __restrict__ f32,
                                                            const int64_t* __restrict__ view_off,
                                                            const int32_t* __restrict__ wh,
                                                            const int64_t* __restrict__ blk_off,
                                                            uint32_t* __restrict__ q8,
                                                            float4* __restrict__ q32) {
    const int v = blockIdx.y;
    const int W = wh[2 * v], H = wh[2 * v + 1];
    const int64_t n = (int64_t)W * H, base = view_off[v];
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x) {
        const int y = (int)(i / W), x = (int)(i - (int64_t)y * W);
        const bool rx = x + 1 < W, dy = y + 1 < H;
        const float a = f32[base + i];
        if (q32) {
            const int64_t ix = rx ? 1 : 0, iy = dy ? W : 0;
            q32[base + i] = make_float4(a, f32[base + i + ix], f32[base + i + iy],
                                        f32[base + i + iy + ix]);
        }
        if (q8) {
            const uint32_t t00 = saturated_d2(a);
            const uint32_t t10 = rx ? saturated_d2(f32[base + i + 1]) : 255u;
            const uint32_t t01 = dy ? saturated_d2(f32[base + i + W]) : 255u;
            const uint32_t t11 = (rx && dy) ? saturated_d2(f32[base + i + W + 1]) : 255u;
            // blocked layout: block (x / 8, y / 4), row-major blocks, the
            // block's 8 x 4 texels row-major inside it
            const int64_t nbx = (W + kQuadBlockW - 1) / kQuadBlockW;
            const int64_t o = blk_off[v] +
                              (((int64_t)(y / kQuadBlockH) * nbx + x / kQuadBlockW) << 5) +
                              ((y % kQuadBlockH) * kQuadBlockW) + (x % kQuadBlockW);
            q8[o] = t00 | (t10 << 8) | (t01 << 16) | (t11 << 24);
        }
    }
}

template <class T>
void upload(DevBuf<T>& b, const std::vector<T>& h, hipStream_t s) {
    b.alloc(h.size());
    if (!h.empty())
        EPO_HIP(hipMemcpyAsync(b.p, h.data(), h.size() * sizeof(T), hipMemcpyHostToDevice, s));
}

constexpr int32_t kMaxGraphSteps = 64;   // iterations one captured graph may hold

void validate_options(const epo_plan_options& o) {
    EPO_REQUIRE(o.texture_format >= 1 && o.texture_format <= 3, "texture_format must be 1, 2 or 3");
    EPO_REQUIRE(o.points_per_thread == 1 || o.points_per_thread == 2 || o.points_per_thread == 4 ||
                    o.points_per_thread == 8 || o.points_per_thread == 16,
                "points_per_thread must be 1, 2, 4, 8 or 16");
    EPO_REQUIRE(o.tile_order == 1 || o.tile_order == 2, "tile_order must be 1 or 2");
    EPO_REQUIRE(o.persistent == 1 || o.persistent == 2, "persistent must be 1 or 2");
    EPO_REQUIRE(o.record_order == 1 || o.record_order == 2, "record_order must be 1 or 2");
    EPO_REQUIRE(o.resort_interval >= 1, "resort_interval must be >= 1");
    EPO_REQUIRE(o.graph_steps >= 1 && o.graph_steps <= kMaxGraphSteps,
                "graph_steps must be in [1, 64]");
}

void fill_default_options(Plan& p, epo_plan_options& o) {
    if (o.texture_format == 0) o.texture_format = p.params.lambda_max <= kQ8LambdaMax ? 2 : 1;
    if (o.points_per_thread == 0) o.points_per_thread = 4;
    if (o.tile_order == 0) o.tile_order = 1;
    if (o.persistent == 0) o.persistent = 2;
    if (o.record_order == 0) o.record_order = 1;
    if (o.resort_interval == 0) o.resort_interval = 8;
    if (o.graph_steps == 0) o.graph_steps = 1;
}

// the per-pair record copies exist exactly while record_order 2 is in use
void apply_record_order(Plan& p, hipStream_t s) {
    if (p.opt.record_order == 2) {
        ensure_sorted_records(p, s);
    } else {
        p.sorted_records.release();
        p.pair_shift.release();
        p.sort_chunks.release();
        p.n_sort_chunks = 0;
    }
}

}  // namespace

void release_graph(Plan& p) {
    if (p.graph_exec) (void)hipGraphExecDestroy(p.graph_exec);
    if (p.graph) (void)hipGraphDestroy(p.graph);
    p.graph_exec = nullptr;
    p.graph = nullptr;
}

Plan::~Plan() {
    release_graph(*this);
    if (ev0) (void)hipEventDestroy(ev0);
    if (ev1) (void)hipEventDestroy(ev1);
}

void build_tiles(Plan& p, hipStream_t s) {
    const int64_t ts = 256 * (int64_t)p.opt.points_per_thread;
    p.tile_size = (int32_t)ts;
    std::vector<int32_t> order(p.D);
    std::iota(order.begin(), order.end(), 0);
    if (p.opt.tile_order == 1) {
        // group by target view (its texture stays hot in one XCD's L2)
        std::stable_sort(order.begin(), order.end(), [&](int a, int b) {
            return p.pairs[2 * a + 1] < p.pairs[2 * b + 1];
        });
    }
    std::vector<Tile> tiles;
    std::vector<PairStatic> ps(p.D);
    std::vector<int32_t> per_scene(p.S, 0);
    for (int d = 0; d < p.D; ++d) per_scene[p.scene_of_view[p.pairs[2 * d]]]++;
    for (int d : order) {
        const int i = p.pairs[2 * d], j = p.pairs[2 * d + 1];
        const int64_t a = p.rec_off[i], n = p.rec_off[i + 1] - p.rec_off[i];
        PairStatic& st = ps[d];
        st.src = i;
        st.tgt = j;
        st.scene = p.scene_of_view[i];
        st.first_tile = (int32_t)tiles.size();
        st.n_src = (int32_t)n;
        st.group = p.group_host[d];
        st.pad = 0;
        for (int64_t c = 0; c < n; c += ts) {
            Tile t;
            t.pair = d;
            t.count = (int32_t)std::min<int64_t>(ts, n - c);
            t.rec = a + c;
            tiles.push_back(t);
        }
        st.n_tiles = (int32_t)tiles.size() - st.first_tile;
    }
    EPO_REQUIRE((int64_t)tiles.size() < (int64_t)INT32_MAX, "too many tiles");
    p.n_tiles = (int64_t)tiles.size();
    // the workgroups of XCD q take the q-th eighth of the tile list
    const int nq = p.n_xcd_queues;
    p.xcd_begin.assign(nq + 1, 0);
    for (int q = 0; q <= nq; ++q) p.xcd_begin[q] = p.n_tiles * q / nq;
    EPO_HIP(hipStreamSynchronize(s));     // host vectors below must outlive the copies
    upload(p.tiles, tiles, s);
    upload(p.pair_static, ps, s);
    upload(p.xcd_begin_d, p.xcd_begin, s);
    p.partials.alloc((size_t)std::max<int64_t>(p.n_tiles, 1));
    p.ext_partials.alloc(2 * (size_t)std::max<int64_t>(p.n_tiles, 1));
    p.tile_list.alloc((size_t)std::max<int64_t>(p.n_tiles, 1));
    p.tile_blk.alloc((size_t)std::max<int64_t>(ceil_div(p.n_tiles, 1024), 1));
    p.qbegin_d.alloc(nq + 1);
    EPO_HIP(hipStreamSynchronize(s));
}

unsigned texture_grid(const Plan& p) {
    int64_t maxWH = 1;
    for (int v = 0; v < p.V; ++v) maxWH = std::max<int64_t>(maxWH, (int64_t)p.width[v] * p.height[v]);
    return (unsigned)std::min<int64_t>(ceil_div(maxWH, 256), 1024);
}

void build_texture(Plan& p, const int32_t* d2, hipStream_t s) {
    p.tex_f32.alloc((size_t)p.total_px);
    texture_f32_kernel<<<dim3(texture_grid(p), p.V), 256, 0, s>>>(d2, p.view_offset_d.p, p.wh_d.p,
                                                                  p.tex_f32.p);
    EPO_CHECK_LAUNCH();
    ensure_texture(p, p.opt.texture_format, s);
}

void ensure_texture(Plan& p, int fmt, hipStream_t s) {
    const bool q8 = fmt == 2 && !p.tex.p, q32 = fmt == 3 && !p.tex_q32.p;
    if (!q8 && !q32) return;
    EPO_REQUIRE(fmt != 2 || p.q8_ok, "texture_format 2 needs lambda_max <= 14.5");
    if (q8) p.tex.alloc((size_t)p.total_blk);
    if (q32) p.tex_q32.alloc((size_t)p.total_px);
    texture_quads_kernel<<<dim3(texture_grid(p), p.V), 256, 0, s>>>(
        p.tex_f32.p, p.view_offset_d.p, p.wh_d.p, p.blk_off_d.p, q8 ? p.tex.p : nullptr,
        q32 ? p.tex_q32.p : nullptr);
    EPO_CHECK_LAUNCH();
}

void release_unused_textures(Plan& p) {
    if (p.opt.texture_format != 2) p.tex.release();
    if (p.opt.texture_format != 3) p.tex_q32.release();
}

}  // namespace epo

using namespace epo;

extern "C" epo_status epo_plan_create(epo_plan* out, int32_t n_views, const int32_t* width,
                                      const int32_t* height, const float* K,
                                      const int32_t* scene_of_view, const int64_t* view_offset,
                                      const uint8_t* edge_maps, const float* depth,
                                      const int32_t* d2, const int32_t* pairs, int32_t n_pairs,
                                      const epo_cost_params* params,
                                      const epo_plan_options* options, void* stream) {
    return guarded([&] {
        EPO_REQUIRE(out, "null output handle");
        *out = nullptr;
        EPO_REQUIRE(n_views >= 1, "n_views must be >= 1");
        EPO_REQUIRE(n_pairs >= 0, "n_pairs must be >= 0");
        EPO_REQUIRE(width && height && K && view_offset && edge_maps && depth && d2,
                    "null pointer argument");
        EPO_REQUIRE(n_pairs == 0 || pairs, "null pair list");
        hipStream_t s = as_stream(stream);
        std::unique_ptr<Plan> p(new Plan());
        p->V = n_views;
        p->D = n_pairs;
        p->params = params ? *params : epo_cost_params{1.0f, 1e-4f, 0, 10.0f};
        EPO_REQUIRE(p->params.huber_delta > 0 && std::isfinite(p->params.huber_delta),
                    "huber_delta must be > 0");
        EPO_REQUIRE(p->params.z_min >= 1e-6f && p->params.z_min <= 1e6f,
                    "z_min must be in [1e-6, 1e6]");
        EPO_REQUIRE(p->params.norm_mode == 0 || p->params.norm_mode == 1, "norm_mode must be 0 or 1");
        EPO_REQUIRE(p->params.lambda_max > 0 && std::isfinite(p->params.lambda_max),
                    "lambda_max must be > 0");
        p->width.assign(width, width + n_views);
        p->height.assign(height, height + n_views);
        p->K.assign(K, K + 4 * (size_t)n_views);
        p->view_offset.assign(view_offset, view_offset + n_views);
        p->scene_of_view.assign(n_views, 0);
        if (scene_of_view) p->scene_of_view.assign(scene_of_view, scene_of_view + n_views);
        int32_t S = 0;
        for (int v = 0; v < n_views; ++v) {
            const std::string tag = "view " + std::to_string(v) + ": ";
            // a bilinear cell needs two rows and two columns; the kernel reads the
            // four taps of cell (0, 0) for residuals that fall outside the image
            EPO_REQUIRE(p->width[v] >= 2 && p->width[v] <= EPO_MAX_SIDE && p->height[v] >= 2 &&
                            p->height[v] <= EPO_MAX_SIDE,
                        tag + "side out of [2, 16384]");
            EPO_REQUIRE(p->view_offset[v] >= 0, tag + "negative offset");
            EPO_REQUIRE(p->K[4 * v] > 0 && p->K[4 * v + 1] > 0 && std::isfinite(p->K[4 * v + 2]) &&
                            std::isfinite(p->K[4 * v + 3]) && std::isfinite(p->K[4 * v]) &&
                            std::isfinite(p->K[4 * v + 1]),
                        tag + "focal lengths must be finite and > 0, principal point finite");
            EPO_REQUIRE(p->scene_of_view[v] >= 0, tag + "negative scene index");
            S = std::max(S, p->scene_of_view[v] + 1);
            p->total_px = std::max<int64_t>(p->total_px, p->view_offset[v] +
                                                             (int64_t)p->width[v] * p->height[v]);
        }
        {
            std::vector<int> seen(S, 0);
            for (int v = 0; v < n_views; ++v) seen[p->scene_of_view[v]] = 1;
            for (int k = 0; k < S; ++k)
                EPO_REQUIRE(seen[k], "scenes must be numbered 0..S-1 without gaps");
        }
        p->S = S;
        p->pairs.assign(pairs, pairs + 2 * (size_t)n_pairs);
        for (int d = 0; d < n_pairs; ++d) {
            const int i = p->pairs[2 * d], j = p->pairs[2 * d + 1];
            EPO_REQUIRE(i >= 0 && i < n_views && j >= 0 && j < n_views,
                        "pair " + std::to_string(d) + ": view index out of range");
            EPO_REQUIRE(p->scene_of_view[i] == p->scene_of_view[j],
                        "pair " + std::to_string(d) + ": views of different scenes");
        }
        {
            // image pairs {i, j}: ids in order of first appearance
            p->group_host.assign(n_pairs, 0);
            std::unordered_map<uint64_t, int32_t> ids;
            ids.reserve((size_t)n_pairs);
            for (int d = 0; d < n_pairs; ++d) {
                const uint64_t a = (uint64_t)std::min(p->pairs[2 * d], p->pairs[2 * d + 1]);
                const uint64_t b = (uint64_t)std::max(p->pairs[2 * d], p->pairs[2 * d + 1]);
                const auto it = ids.emplace((a << 32) | b, p->n_groups);
                if (it.second) p->n_groups++;
                p->group_host[d] = it.first->second;
            }
        }
        if (options) {
            p->opt = *options;
        } else {
            p->opt = epo_plan_options{0, 0, 0, 0, 0, 0};
        }
        p->q8_ok = p->params.lambda_max <= kQ8LambdaMax;
        fill_default_options(*p, p->opt);
        validate_options(p->opt);
        if (p->opt.texture_format == 2 && !p->q8_ok)
            throw Failure{EPO_ERR_UNSUPPORTED,
                          "texture_format 2 needs lambda_max <= 14.5 (saturated taps)"};

        // every host-side check is done: from here on the device is used
        EPO_HIP(hipGetDevice(&p->device));
        EPO_HIP(hipDeviceGetAttribute(&p->n_cu, hipDeviceAttributeMultiprocessorCount, p->device));

        // ---- static device data
        std::vector<int32_t> wh(2 * (size_t)n_views);
        for (int v = 0; v < n_views; ++v) {
            wh[2 * v] = p->width[v];
            wh[2 * v + 1] = p->height[v];
        }
        upload(p->wh_d, wh, s);
        upload(p->K_d, p->K, s);
        upload(p->K0_d, p->K, s);
        p->gamma_d.alloc(n_views);
        EPO_HIP(hipMemsetAsync(p->gamma_d.p, 0, sizeof(double) * n_views, s));
        upload(p->view_offset_d, p->view_offset, s);
        p->blk_off.assign(n_views, 0);
        for (int v = 0; v < n_views; ++v) {
            p->blk_off[v] = p->total_blk;
            p->total_blk += (int64_t)ceil_div(p->width[v], kQuadBlockW) *
                            ceil_div(p->height[v], kQuadBlockH) * (kQuadBlockW * kQuadBlockH);
        }
        upload(p->blk_off_d, p->blk_off, s);
        upload(p->scene_of_view_d, p->scene_of_view, s);

        // ---- edge compaction: counts per 16x16 tile, host prefix, scatter
        std::vector<int64_t> tile_first(n_views + 1, 0);
        for (int v = 0; v < n_views; ++v)
            tile_first[v + 1] = tile_first[v] + ceil_div(p->width[v], kTile) *
                                                    ceil_div(p->height[v], kTile);
        const int64_t n_ptiles = tile_first[n_views];
        EPO_REQUIRE(n_ptiles < (int64_t)INT32_MAX, "too many pixel tiles");
        DevBuf<int64_t> tile_first_d;
        upload(tile_first_d, tile_first, s);
        DevBuf<int32_t> counts_d;
        counts_d.alloc((size_t)n_ptiles);
        count_tiles_kernel<<<(unsigned)n_ptiles, 256, 0, s>>>(edge_maps, p->view_offset_d.p,
                                                              p->wh_d.p, tile_first_d.p, n_views,
                                                              counts_d.p);
        EPO_CHECK_LAUNCH();
        std::vector<int32_t> counts((size_t)n_ptiles);
        EPO_HIP(hipMemcpyAsync(counts.data(), counts_d.p, counts.size() * sizeof(int32_t),
                               hipMemcpyDeviceToHost, s));
        EPO_HIP(hipStreamSynchronize(s));
        std::vector<int64_t> tile_rec((size_t)n_ptiles);
        int64_t acc = 0;
        for (int64_t t = 0; t < n_ptiles; ++t) {
            tile_rec[t] = acc;
            acc += counts[t];
        }
        p->rec_off.assign(n_views + 1, 0);
        for (int v = 0; v < n_views; ++v) p->rec_off[v] = tile_rec.empty() ? 0 : tile_rec[tile_first[v]];
        p->rec_off[n_views] = acc;
        {
            // 256-record blocks of each view for the source-major depth pass
            std::vector<Tile> vb;
            for (int v = 0; v < n_views; ++v)
                for (int64_t c = p->rec_off[v]; c < p->rec_off[v + 1]; c += 256)
                    vb.push_back(Tile{v, (int32_t)std::min<int64_t>(256, p->rec_off[v + 1] - c), c});
            EPO_REQUIRE((int64_t)vb.size() < (int64_t)INT32_MAX, "too many record blocks");
            p->n_vblocks = (int64_t)vb.size();
            upload(p->vblocks, vb, s);
            EPO_HIP(hipStreamSynchronize(s));
        }
        DevBuf<int64_t> tile_rec_d;
        upload(tile_rec_d, tile_rec, s);
        p->records.alloc((size_t)(acc + kRecordPad));
        EPO_HIP(hipMemsetAsync(p->records.p + acc, 0, sizeof(uint64_t) * kRecordPad, s));
        DevBuf<int32_t> bad_d;
        bad_d.alloc(1);
        EPO_HIP(hipMemsetAsync(bad_d.p, 0, sizeof(int32_t), s));
        scatter_records_kernel<<<(unsigned)n_ptiles, 256, 0, s>>>(
            edge_maps, depth, p->view_offset_d.p, p->wh_d.p, tile_first_d.p, n_views,
            tile_rec_d.p, p->records.p, bad_d.p);
        EPO_CHECK_LAUNCH();
        int32_t bad = 0;
        EPO_HIP(hipMemcpyAsync(&bad, bad_d.p, sizeof(int32_t), hipMemcpyDeviceToHost, s));
        EPO_HIP(hipStreamSynchronize(s));
        EPO_REQUIRE(bad == 0, "depth is not finite at an edge pixel");

        // ---- textures
        build_texture(*p, d2, s);

        // ---- residual count, CSR lists
        p->n_residuals = 0;
        std::vector<std::vector<int32_t>> in(n_views), outl(n_views), sc(S);
        for (int d = 0; d < n_pairs; ++d) {
            const int i = p->pairs[2 * d], j = p->pairs[2 * d + 1];
            p->n_residuals += p->rec_off[i + 1] - p->rec_off[i];
            in[j].push_back(d);
            outl[i].push_back(d);
            sc[p->scene_of_view[i]].push_back(d);
        }
        auto csr = [&](const std::vector<std::vector<int32_t>>& lists, DevBuf<int32_t>& ptr,
                       DevBuf<int32_t>& idx) {
            std::vector<int32_t> hp(lists.size() + 1, 0), hi;
            for (size_t k = 0; k < lists.size(); ++k) {
                hp[k + 1] = hp[k] + (int32_t)lists[k].size();
                hi.insert(hi.end(), lists[k].begin(), lists[k].end());
            }
            upload(ptr, hp, s);
            upload(idx, hi, s);
            EPO_HIP(hipStreamSynchronize(s));
        };
        {
            // source-major layout of the per-residual depth derivatives
            std::vector<int64_t> dzi(2 * (size_t)std::max(n_pairs, 1), 0);
            int64_t base = 0;
            for (int i = 0; i < n_views; ++i) {
                const int64_t r0 = p->rec_off[i], nrec = p->rec_off[i + 1] - r0;
                const int64_t nout = (int64_t)outl[i].size();
                for (int64_t slot = 0; slot < nout; ++slot) {
                    const int d = outl[i][slot];
                    dzi[2 * d] = base + slot * 256 - r0 * nout;
                    dzi[2 * d + 1] = nout;
                }
                base += ceil_div(nrec, 256) * 256 * nout;
            }
            p->dz_size = base;
            upload(p->dz_index, dzi, s);
            EPO_HIP(hipStreamSynchronize(s));
        }
        csr(in, p->view_in_ptr, p->view_in_idx);
        csr(outl, p->view_out_ptr, p->view_out_idx);
        csr(sc, p->scene_ptr, p->scene_pairs);
        {
            std::vector<std::vector<int32_t>> sv(S);
            for (int v = 0; v < n_views; ++v) sv[p->scene_of_view[v]].push_back(v);
            p->max_views_per_scene = 0;
            for (const auto& l : sv)
                p->max_views_per_scene = std::max<int32_t>(p->max_views_per_scene, (int32_t)l.size());
            csr(sv, p->scene_view_ptr, p->scene_view_idx);
        }
        {
            // groups per scene (group ids increase with first appearance, and
            // a scene's groups are listed in id order), directions per group,
            // and the every-pair scales 2 / |D_scene|
            std::vector<int32_t> g_np(std::max(p->n_groups, 1), 0), g_scene(std::max(p->n_groups, 1), 0);
            for (int d = 0; d < n_pairs; ++d) {
                g_np[p->group_host[d]] += 1;
                g_scene[p->group_host[d]] = p->scene_of_view[p->pairs[2 * d]];
            }
            std::vector<std::vector<int32_t>> sg(S);
            for (int g = 0; g < p->n_groups; ++g) sg[g_scene[g]].push_back(g);
            std::vector<int32_t> gptr(S + 1, 0), gidx;
            for (int k = 0; k < S; ++k) {
                gptr[k + 1] = gptr[k] + (int32_t)sg[k].size();
                gidx.insert(gidx.end(), sg[k].begin(), sg[k].end());
            }
            // the selection kernel walks a scene's groups as the id range
            // [gptr[s], gptr[s+1]) of a scene-major renumbering
            std::vector<int32_t> renum(std::max(p->n_groups, 1), 0);
            for (int k = 0; k < (int)gidx.size(); ++k) renum[gidx[k]] = k;
            std::vector<int32_t> gop(std::max(n_pairs, 1), 0), np_sorted(std::max(p->n_groups, 1), 0);
            std::vector<int32_t> gid_sorted(std::max(p->n_groups, 1), 0);
            for (int d = 0; d < n_pairs; ++d) gop[d] = renum[p->group_host[d]];
            for (int g = 0; g < p->n_groups; ++g) {
                np_sorted[renum[g]] = g_np[g];
                gid_sorted[renum[g]] = g;
            }
            p->group_id_sorted_h = gid_sorted;
            std::vector<int32_t> per_scene(S, 0);
            for (int d = 0; d < n_pairs; ++d) per_scene[p->scene_of_view[p->pairs[2 * d]]]++;
            std::vector<double> scale(std::max(n_pairs, 1), 0.0);
            for (int d = 0; d < n_pairs; ++d)
                scale[d] = 2.0 / (double)per_scene[p->scene_of_view[p->pairs[2 * d]]];
            upload(p->group_of_pair, gop, s);
            upload(p->group_npairs, np_sorted, s);
            upload(p->group_id_sorted, gid_sorted, s);
            upload(p->scene_group_ptr, gptr, s);
            upload(p->pair_scale_all, scale, s);
            upload(p->pair_scale, scale, s);
            p->group_sel.alloc(std::max(p->n_groups, 1));
            EPO_HIP(hipMemsetAsync(p->group_sel.p, 1, p->group_sel.n, s));
            EPO_HIP(hipStreamSynchronize(s));
        }
        p->conv_prev.alloc(12 * (size_t)n_views);
        p->conv_state.alloc(S);
        p->conv_phase.alloc(S);
        EPO_HIP(hipMemsetAsync(p->conv_state.p, 0, sizeof(ConvState) * S, s));
        EPO_HIP(hipMemsetAsync(p->conv_phase.p, 0, sizeof(int32_t) * S, s));

        // ---- per-iteration buffers
        p->pair_desc.alloc(std::max(n_pairs, 1));
        p->pair_rel.alloc(12 * (size_t)std::max(n_pairs, 1));
        p->pair_sum.alloc(8 * (size_t)std::max(n_pairs, 1));
        p->pair_w.alloc(std::max(n_pairs, 1));
        p->pair_ext.alloc(2 * (size_t)std::max(n_pairs, 1));
        p->counters.alloc(16);
        p->status.alloc(1);
        p->pose_done.alloc(1);
        EPO_HIP(hipMemsetAsync(p->counters.p, 0, 16 * sizeof(int32_t), s));
        EPO_HIP(hipMemsetAsync(p->status.p, 0, sizeof(int32_t), s));
        EPO_HIP(hipMemsetAsync(p->pose_done.p, 0, sizeof(int32_t), s));
        EPO_HIP(hipMemsetAsync(p->pair_sum.p, 0, p->pair_sum.n * sizeof(double), s));
        EPO_HIP(hipMemsetAsync(p->pair_w.p, 0, p->pair_w.n * sizeof(double), s));
        p->grad_scratch.alloc(6 * (size_t)n_views);
        p->lambda_buf.alloc(S);
        p->lr_buf.alloc(S);
        build_tiles(*p, s);
        apply_record_order(*p, s);
        EPO_HIP(hipStreamSynchronize(s));
        *out = reinterpret_cast<epo_plan>(p.release());
    });
}

extern "C" epo_status epo_plan_destroy(epo_plan plan) {
    return guarded([&] {
        if (!plan) return;
        Plan* p = reinterpret_cast<Plan*>(plan);
        (void)hipSetDevice(p->device);
        (void)hipDeviceSynchronize();
        delete p;
    });
}

extern "C" epo_status epo_plan_info(epo_plan plan, int32_t* n_scenes, int64_t* n_records,
                                    int64_t* n_residuals, int64_t* n_tiles,
                                    epo_plan_options* options) {
    return guarded([&] {
        EPO_REQUIRE(plan, "null plan");
        const Plan& p = *reinterpret_cast<Plan*>(plan);
        if (n_scenes) *n_scenes = p.S;
        if (n_records) *n_records = p.rec_off.back();
        if (n_residuals) *n_residuals = p.n_residuals;
        if (n_tiles) *n_tiles = p.n_tiles;
        if (options) *options = p.opt;
    });
}

extern "C" epo_status epo_plan_view_records(epo_plan plan, int32_t v, uint64_t* records_out,
                                            int64_t capacity, int64_t* count) {
    return guarded([&] {
        EPO_REQUIRE(plan && count, "null argument");
        const Plan& p = *reinterpret_cast<Plan*>(plan);
        EPO_REQUIRE(v >= 0 && v < p.V, "view index out of range");
        const int64_t n = p.rec_off[v + 1] - p.rec_off[v];
        *count = n;
        if (!records_out) return;
        EPO_REQUIRE(capacity >= n, "records_out too small");
        EPO_HIP(hipSetDevice(p.device));
        EPO_HIP(hipDeviceSynchronize());
        if (n > 0)
            EPO_HIP(hipMemcpy(records_out, p.records.p + p.rec_off[v], n * sizeof(uint64_t),
                              hipMemcpyDeviceToHost));
    });
}

extern "C" epo_status epo_plan_set_options(epo_plan plan, const epo_plan_options* options,
                                           void* stream) {
    return guarded([&] {
        EPO_REQUIRE(plan && options, "null argument");
        Plan& p = *reinterpret_cast<Plan*>(plan);
        EPO_HIP(hipSetDevice(p.device));
        epo_plan_options o = *options;
        fill_default_options(p, o);
        validate_options(o);
        if (o.texture_format == 2 && !p.q8_ok)
            throw Failure{EPO_ERR_UNSUPPORTED,
                          "texture_format 2 needs lambda_max <= 14.5 (saturated taps)"};
        hipStream_t s = as_stream(stream);
        EPO_HIP(hipStreamSynchronize(s));
        release_graph(p);
        const bool rebuild = o.points_per_thread != p.opt.points_per_thread ||
                             o.tile_order != p.opt.tile_order;
        p.opt = o;
        if (rebuild) build_tiles(p, s);
        ensure_texture(p, p.opt.texture_format, s);
        release_unused_textures(p);
        apply_record_order(p, s);
    });
}

extern "C" epo_status epo_plan_autotune(epo_plan plan, const double* poses, const float* lambda,
                                        int32_t iters, epo_plan_options* chosen, void* stream) {
    return guarded([&] {
        EPO_REQUIRE(plan && poses && lambda, "null argument");
        EPO_REQUIRE(iters >= 1, "iters must be >= 1");
        Plan& p = *reinterpret_cast<Plan*>(plan);
        EPO_HIP(hipSetDevice(p.device));
        hipStream_t s = as_stream(stream);
        EPO_HIP(hipStreamSynchronize(s));
        release_graph(p);
        DevBuf<double> loss, grad;
        loss.alloc(p.S);
        grad.alloc(6 * (size_t)p.V);
        hipEvent_t a, b;
        EPO_HIP(hipEventCreate(&a));
        EPO_HIP(hipEventCreate(&b));
        float best = 1e30f;
        epo_plan_options best_o = p.opt;
        const int fmts[3] = {1, 2, 3};
        const int ppts[4] = {2, 4, 8, 16};
        const int orders[2] = {1, 2};
        const int pers[2] = {1, 2};
        const int rorders[2] = {1, 2};
        const int interval = p.opt.resort_interval;
        // record order 2 is charged its re-sort too (1 / interval of the
        // chunks every step) and must beat the best source-order schedule by
        // a clear margin: the copies cost 8 bytes per residual
        float sort_share = 0.0f, best1 = 1e30f;
        constexpr float kOrderMargin = 0.97f;
        try {
            for (int ro : rorders) {
            if (ro == 2) {
                // copies sorted at these poses (the state right after a
                // captured iteration's full sort)
                p.opt.record_order = 2;
                ensure_sorted_records(p, s);
                launch_resort(p, poses, nullptr, 1, s);         // warm-up
                EPO_HIP(hipEventRecord(a, s));
                launch_resort(p, poses, nullptr, 1, s);
                EPO_HIP(hipEventRecord(b, s));
                EPO_HIP(hipEventSynchronize(b));
                float full = 0;
                EPO_HIP(hipEventElapsedTime(&full, a, b));
                sort_share = full / (float)interval * (float)iters;
                best1 = best;
            }
            for (int f : fmts) {
                if (f == 2 && !p.q8_ok) continue;
                ensure_texture(p, f, s);
                for (int pp : ppts)
                    for (int o : orders)
                        for (int pe : pers) {
                            const bool rebuild = pp != p.opt.points_per_thread ||
                                                 o != p.opt.tile_order;
                            p.opt = epo_plan_options{f, pp, o, pe, ro, interval,
                                                     p.opt.graph_steps};
                            if (rebuild) build_tiles(p, s);
                            launch_cost(p, poses, lambda, loss.p, nullptr, nullptr, nullptr, grad.p,
                                        nullptr, s);      // warm-up
                            EPO_HIP(hipEventRecord(a, s));
                            for (int k = 0; k < iters; ++k)
                                launch_cost(p, poses, lambda, loss.p, nullptr, nullptr, nullptr,
                                            grad.p, nullptr, s);
                            EPO_HIP(hipEventRecord(b, s));
                            EPO_HIP(hipEventSynchronize(b));
                            float ms = 0;
                            EPO_HIP(hipEventElapsedTime(&ms, a, b));
                            if (ro == 2) {
                                ms += sort_share;
                                if (ms >= kOrderMargin * best1) continue;
                            }
                            if (ms < best) {
                                best = ms;
                                best_o = p.opt;
                            }
                        }
            }
            }
        } catch (...) {
            (void)hipEventDestroy(a);
            (void)hipEventDestroy(b);
            throw;
        }
        (void)hipEventDestroy(a);
        (void)hipEventDestroy(b);
        const bool rebuild = best_o.points_per_thread != p.opt.points_per_thread ||
                             best_o.tile_order != p.opt.tile_order;
        p.opt = best_o;
        if (rebuild) build_tiles(p, s);
        release_unused_textures(p);
        apply_record_order(p, s);
        if (chosen) *chosen = best_o;
    });
}

namespace {

// Captures the launches `body` makes on a fresh stream, graph_steps times in
// a row, as the plan's iteration graph: `step` is the device counter the pair
// selection reads during capture, with_convergence 2 leaves stopped scenes'
// tiles out of the fused launch, and no timing events are recorded inside
// the graph.
template <class F>
void capture_iteration(Plan& p, const int32_t* step, int32_t with_convergence, hipStream_t user,
                       F&& body) {
    EPO_HIP(hipStreamSynchronize(user));
    release_graph(p);
    hipStream_t cs;
    EPO_HIP(hipStreamCreateWithFlags(&cs, hipStreamNonBlocking));
    const bool timing = p.timing;
    p.timing = false;
    hipError_t cap = hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal);
    if (cap != hipSuccess) {
        p.timing = timing;
        (void)hipStreamDestroy(cs);
        throw Failure{EPO_ERR_HIP, std::string("hipStreamBeginCapture: ") +
                                       hipGetErrorString(cap)};
    }
    p.capture_step = step;
    p.gate_phase = with_convergence == 2 ? p.conv_phase.p : nullptr;
    try {
        for (int k = 0; k < p.opt.graph_steps; ++k) body(cs);
    } catch (...) {
        hipGraph_t junk = nullptr;
        (void)hipStreamEndCapture(cs, &junk);
        if (junk) (void)hipGraphDestroy(junk);
        (void)hipStreamDestroy(cs);
        p.timing = timing;
        p.capture_step = nullptr;
        p.gate_phase = nullptr;
        throw;
    }
    p.timing = timing;
    p.capture_step = nullptr;
    if (p.gate_phase) p.scale_gated = true;
    p.gate_phase = nullptr;
    hipError_t e = hipStreamEndCapture(cs, &p.graph);
    (void)hipStreamDestroy(cs);
    if (e != hipSuccess)
        throw Failure{EPO_ERR_HIP, std::string("hipStreamEndCapture: ") + hipGetErrorString(e)};
    EPO_HIP(hipGraphInstantiate(&p.graph_exec, p.graph, nullptr, nullptr, 0));
}

void check_schedule(const Plan& p, float lambda0, float lambda1, int32_t anneal_steps,
                    int32_t warmup, int32_t total, int32_t with_convergence) {
    EPO_REQUIRE(warmup >= 1 && total > warmup && anneal_steps >= 0, "schedule out of range");
    EPO_REQUIRE(lambda0 <= p.params.lambda_max && lambda1 <= p.params.lambda_max,
                "schedule clamp above the plan's lambda_max");
    EPO_REQUIRE(with_convergence >= 0 && with_convergence <= 2,
                "with_convergence must be 0, 1 or 2");
    EPO_REQUIRE(!with_convergence || p.max_views_per_scene <= kConvMaxViews,
                "a scene has more views than the convergence kernel supports");
}

}  // namespace

extern "C" epo_status epo_iteration_capture(epo_plan plan, double* poses, double* adam_m,
                                            double* adam_v, int32_t* step, double* loss,
                                            double* grad, const uint8_t* fixed_mask,
                                            float lambda0, float lambda1, int32_t anneal_steps,
                                            double peak_lr, int32_t warmup, int32_t total,
                                            double beta1, double beta2, double eps,
                                            int32_t with_convergence, void* stream) {
    return guarded([&] {
        EPO_REQUIRE(plan && poses && adam_m && adam_v && step && loss, "null argument");
        Plan& p = *reinterpret_cast<Plan*>(plan);
        EPO_HIP(hipSetDevice(p.device));
        check_schedule(p, lambda0, lambda1, anneal_steps, warmup, total, with_convergence);
        double* g = grad ? grad : p.grad_scratch.p;
        // record order 2: every copy sorted at the poses the first replay
        // starts from; each replay then re-sorts 1 / resort_interval of them
        launch_resort(p, poses, nullptr, 1, as_stream(stream));
        capture_iteration(p, step, with_convergence, as_stream(stream), [&](hipStream_t cs) {
            // the schedule is evaluated by the pair set-up (one launch fewer);
            // a plan without pairs runs the schedule kernel
            const ScheduleArgs sched{step, lambda0, lambda1, anneal_steps, peak_lr, warmup,
                                     total, p.lambda_buf.p, p.lr_buf.p,
                                     with_convergence ? p.conv_phase.p : nullptr, p.S};
            if (p.D == 0)
                launch_schedule(step, p.S, lambda0, lambda1, anneal_steps, peak_lr, warmup, total,
                                p.lambda_buf.p, p.lr_buf.p, sched.phase, cs);
            launch_resort(p, poses, step, p.opt.resort_interval, cs);
            // a small plan's reductions, pose step and step count go in one
            // launch (the same bits as the separate ones)
            launch_tiles(p, poses, p.lambda_buf.p, cs, nullptr, &sched);
            if (!launch_step_epilogue(p, loss, g, poses, adam_m, adam_v, fixed_mask, p.lr_buf.p,
                                      beta1, beta2, eps, step, cs)) {
                launch_reductions(p, loss, nullptr, nullptr, nullptr, g, nullptr, cs);
                launch_pose_step(poses, adam_m, adam_v, g, p.V, p.scene_of_view_d.p, fixed_mask,
                                 p.lr_buf.p, beta1, beta2, eps, step, cs, p.pose_done.p);
            }
            if (with_convergence) launch_convergence(p, poses, nullptr, cs);
        });
    });
}

extern "C" epo_status epo_mlp_iteration_capture(
    epo_plan plan, float* params, float* adam_m, float* adam_v, float* param_grad, double* delta,
    double* delta_m, double* delta_v, double* delta_grad, const double* poses0, double* poses,
    int32_t* step, double* loss, double* grad, float lambda0, float lambda1,
    int32_t anneal_steps, double peak_lr, int32_t warmup, int32_t total, double beta1,
    double beta2, double eps, double wd_mlp, double wd_delta, int32_t with_convergence,
    void* stream) {
    return guarded([&] {
        EPO_REQUIRE(plan && params && adam_m && adam_v && param_grad && delta && delta_m &&
                        delta_v && delta_grad && poses0 && poses && step && loss,
                    "null argument");
        Plan& p = *reinterpret_cast<Plan*>(plan);
        EPO_HIP(hipSetDevice(p.device));
        EPO_REQUIRE(p.mlp_act.p, "call epo_mlp_setup first");
        check_schedule(p, lambda0, lambda1, anneal_steps, warmup, total, with_convergence);
        double* g = grad ? grad : p.grad_scratch.p;
        launch_resort(p, poses, nullptr, 1, as_stream(stream));
        capture_iteration(p, step, with_convergence, as_stream(stream), [&](hipStream_t cs) {
            // schedule -> (record re-sort) -> cost and adjoint at the current poses -> refiner
            // backward (activations of the forward that made them) -> AdamW
            // (advances the step) -> poses of the new parameters ->
            // (pose-change test)
            // the schedule evaluated by the pair set-up, as in the pose loop
            const ScheduleArgs sched{step, lambda0, lambda1, anneal_steps, peak_lr, warmup,
                                     total, p.lambda_buf.p, p.lr_buf.p,
                                     with_convergence ? p.conv_phase.p : nullptr, p.S};
            if (p.D == 0)
                launch_schedule(step, p.S, lambda0, lambda1, anneal_steps, peak_lr, warmup, total,
                                p.lambda_buf.p, p.lr_buf.p, sched.phase, cs);
            launch_resort(p, poses, step, p.opt.resort_interval, cs);
            launch_tiles(p, poses, p.lambda_buf.p, cs, nullptr, &sched);
            launch_reductions(p, loss, nullptr, nullptr, nullptr, g, nullptr, cs);
            launch_mlp_backward(p, params, poses0, poses, g, param_grad, delta_grad, cs);
            launch_adamw(p, params, adam_m, adam_v, param_grad, delta, delta_m, delta_v,
                         delta_grad, p.lr_buf.p, beta1, beta2, eps, wd_mlp, wd_delta, step, cs);
            launch_mlp_forward(p, params, poses0, delta, poses, cs);
            if (with_convergence) launch_convergence(p, poses, nullptr, cs);
        });
    });
}

extern "C" epo_status epo_joint_iteration_capture(epo_plan plan, double* poses, double* adam_m,
                                                  double* adam_v, int32_t* step, double* loss,
                                                  double* grad, const epo_joint_state* joint,
                                                  float lambda0, float lambda1,
                                                  int32_t anneal_steps, double peak_lr,
                                                  int32_t warmup, int32_t total, double beta1,
                                                  double beta2, double eps,
                                                  int32_t with_convergence, void* stream) {
    return guarded([&] {
        EPO_REQUIRE(plan && poses && adam_m && adam_v && step && loss && joint, "null argument");
        const epo_joint_state j = *joint;
        EPO_REQUIRE(j.gamma && j.alpha && j.beta && j.m_gamma && j.v_gamma && j.m_depth &&
                        j.v_depth && j.steps && j.grad_gamma && j.grad_alpha && j.grad_beta,
                    "null pointer in the joint state");
        EPO_REQUIRE(beta1 >= 0.0 && beta1 < 1.0 && beta2 >= 0.0 && beta2 < 1.0 && eps > 0.0,
                    "beta1, beta2 must be in [0, 1) and eps > 0");
        Plan& p = *reinterpret_cast<Plan*>(plan);
        EPO_HIP(hipSetDevice(p.device));
        check_schedule(p, lambda0, lambda1, anneal_steps, warmup, total, with_convergence);
        hipStream_t user = as_stream(stream);
        // set-up outside the graph: the state's refinement in the plan (the
        // first depth update allocates), the record offsets on the device
        ensure_record_offsets(p, user);
        install_refinement(p, j.gamma, j.alpha, j.beta, user);
        double* g = grad ? grad : p.grad_scratch.p;
        const RefineOut out{j.grad_gamma, j.grad_alpha, j.grad_beta};
        const int32_t* phase = with_convergence ? p.conv_phase.p : nullptr;
        capture_iteration(p, step, with_convergence, user, [&](hipStream_t cs) {
            // schedule -> cost, pose, focal and depth gradients at the current
            // refinement -> joint AdamW gated by the phase (installs the new
            // refinement) -> pose step (advances the step) -> (pose-change
            // test, phase switches)
            // the schedule evaluated by the pair set-up, as in the pose loop
            const ScheduleArgs sched{step, lambda0, lambda1, anneal_steps, peak_lr, warmup,
                                     total, p.lambda_buf.p, p.lr_buf.p, phase, p.S};
            if (p.D == 0)
                launch_schedule(step, p.S, lambda0, lambda1, anneal_steps, peak_lr, warmup, total,
                                p.lambda_buf.p, p.lr_buf.p, phase, cs);
            launch_cost(p, poses, p.lambda_buf.p, loss, nullptr, nullptr, nullptr, g, nullptr, cs,
                        &out, &sched);
            launch_joint_step(p, j, p.lr_buf.p, phase, beta1, beta2, eps, cs);
            launch_pose_step(poses, adam_m, adam_v, g, p.V, p.scene_of_view_d.p, nullptr,
                             p.lr_buf.p, beta1, beta2, eps, step, cs, p.pose_done.p);
            if (with_convergence) launch_convergence(p, poses, nullptr, cs);
        });
    });
}

extern "C" epo_status epo_iteration_launch(epo_plan plan, void* stream) {
    return guarded([&] {
        EPO_REQUIRE(plan, "null plan");
        Plan& p = *reinterpret_cast<Plan*>(plan);
        EPO_REQUIRE(p.graph_exec, "no captured iteration (call epo_iteration_capture)");
        EPO_HIP(hipGraphLaunch(p.graph_exec, as_stream(stream)));
    });
}

extern "C" epo_status epo_get_device_status(epo_plan plan, int32_t* flags, void* stream) {
    return guarded([&] {
        EPO_REQUIRE(plan && flags, "null argument");
        Plan& p = *reinterpret_cast<Plan*>(plan);
        EPO_HIP(hipSetDevice(p.device));
        hipStream_t s = as_stream(stream);
        EPO_HIP(hipMemcpyAsync(flags, p.status.p, sizeof(int32_t), hipMemcpyDeviceToHost, s));
        EPO_HIP(hipStreamSynchronize(s));
        EPO_HIP(hipMemsetAsync(p.status.p, 0, sizeof(int32_t), s));
        EPO_HIP(hipStreamSynchronize(s));
    });
}

extern "C" epo_status epo_plan_enable_timing(epo_plan plan, int32_t enable) {
    return guarded([&] {
        EPO_REQUIRE(plan, "null plan");
        Plan& p = *reinterpret_cast<Plan*>(plan);
        EPO_HIP(hipSetDevice(p.device));
        if (enable && !p.ev0) {
            EPO_HIP(hipEventCreate(&p.ev0));
            EPO_HIP(hipEventCreate(&p.ev1));
        }
        p.timing = enable != 0;
        p.timed_once = false;
    });
}

extern "C" epo_status epo_plan_last_kernel_ms(epo_plan plan, float* ms) {
    return guarded([&] {
        EPO_REQUIRE(plan && ms, "null argument");
        Plan& p = *reinterpret_cast<Plan*>(plan);
        EPO_REQUIRE(p.timing && p.timed_once, "timing not enabled or no timed launch yet");
        EPO_HIP(hipEventSynchronize(p.ev1));
        EPO_HIP(hipEventElapsedTime(ms, p.ev0, p.ev1));
    });
}

extern "C" const char* epo_last_error(void) { return g_last_error.c_str(); }

extern "C" const char* epo_version(void) { return "epo-mi355x 0.1.0 (gfx950)"; }
