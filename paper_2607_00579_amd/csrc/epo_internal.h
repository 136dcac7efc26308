// Internal declarations shared by the translation units of libepo.so.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <string>
#include <vector>

#include "../../include/epo.h"

namespace epo {

// ---------------------------------------------------------------------------
// error handling: thread-local message + status, no exception crosses the ABI
// ---------------------------------------------------------------------------
void set_error(const std::string& msg);
void clear_error();

struct Failure {
    epo_status status;
    std::string msg;
};

#define EPO_REQUIRE(cond, msg)                                                  \
    do {                                                                        \
        if (!(cond)) throw ::epo::Failure{EPO_ERR_INVALID_ARG, (msg)};          \
    } while (0)

#define EPO_HIP(call)                                                           \
    do {                                                                        \
        hipError_t e_ = (call);                                                 \
        if (e_ != hipSuccess)                                                   \
            throw ::epo::Failure{EPO_ERR_HIP, std::string(#call) + ": " +       \
                                                  hipGetErrorString(e_)};       \
    } while (0)

#define EPO_CHECK_LAUNCH()                                                      \
    do {                                                                        \
        hipError_t e_ = hipGetLastError();                                      \
        if (e_ != hipSuccess)                                                   \
            throw ::epo::Failure{EPO_ERR_HIP, std::string("kernel launch: ") +  \
                                                  hipGetErrorString(e_)};       \
    } while (0)

template <class F>
epo_status guarded(F&& f) {
    try {
        clear_error();
        f();
        return EPO_OK;
    } catch (const Failure& e) {
        set_error(e.msg);
        return e.status;
    } catch (const std::exception& e) {
        set_error(std::string("internal error: ") + e.what());
        return EPO_ERR_HIP;
    } catch (...) {
        set_error("internal error");
        return EPO_ERR_HIP;
    }
}

inline hipStream_t as_stream(void* s) { return reinterpret_cast<hipStream_t>(s); }

// ==== data layout read by the fused kernel: begin (the fused kernel's
// measured counters are keyed to this section's text)
// pixel blocks of the u8 quad texture (8 x 4 texels of 4 bytes = 128 bytes)
constexpr int kQuadBlockW = 8;
constexpr int kQuadBlockH = 4;
static_assert(kQuadBlockW * kQuadBlockH == 32, "a quad block is 32 texels (shift by 5)");

// bf16 weights of one scene's refiner MLP packed in MFMA operand order
constexpr int kMlpPacked = 139264;

// zero records allocated past the last edge record: the fused kernel's last
// iteration over a tile reads up to two 256-record rows past the tile's end
// (masked) instead of clamping every row index
constexpr int64_t kRecordPad = 512;

// device buffer owned by a plan
template <class T>
struct DevBuf {
    T* p = nullptr;
    size_t n = 0;
    void alloc(size_t count) {
        release();
        if (count == 0) count = 1;
        EPO_HIP(hipMalloc(&p, count * sizeof(T)));
        n = count;
    }
    void release() {
        if (p) (void)hipFree(p);
        p = nullptr;
        n = 0;
    }
    ~DevBuf() { release(); }
    DevBuf() = default;
    DevBuf(const DevBuf&) = delete;
    DevBuf& operator=(const DevBuf&) = delete;
};

// ---------------------------------------------------------------------------
// per-iteration pair descriptor consumed by the fused kernel
//   X' = Z M (u, v, 1)^T + t  (target camera frame),  M = R_ji K_i^-1, t = t_ji
//   u' = fx_j X'_x / X'_z + cx_j,  v' = fy_j X'_y / X'_z + cy_j
// (float64: the projected coordinate decides the bilinear cell, and float32
// coordinates of a 500-1000 px image flip cells often enough to move pose
// gradients by a few 1e-4)
// ---------------------------------------------------------------------------
struct alignas(16) PairDesc {
    double M[9];
    double t[3];
    double fxd, fyd, cxd, cyd;   // target intrinsics
    float fx, fy;                // target focal lengths (chain rule, float32)
    float lambda;                // clamp of the pair's scene
    int32_t width;               // W_j (texture row stride)
    int32_t wcells, hcells;      // W_j - 1, H_j - 1: bilinear cells per row / column
    int64_t tex_off;             // pixel offset of view j in the texture
};
static_assert(sizeof(PairDesc) == 160, "PairDesc layout");

// static per-pair data (plan lifetime)
struct PairStatic {
    int32_t src, tgt, scene;
    int32_t first_tile, n_tiles;
    int32_t n_src;          // source edge count |E_i|
    int32_t group;          // image pair {i, j} the direction belongs to
    int32_t pad;
};

// one tile = up to tile_size consecutive records of the source view of a pair
struct Tile {
    int32_t pair;
    int32_t count;
    int64_t rec;            // first record
};

// per-tile partial sums: S, n, G[6] (float64)
struct alignas(64) Partial {
    double v[8];
};
// ==== data layout read by the fused kernel: end

// relative pose of the directed pair i -> j (world -> camera poses [V][3][4],
// float64): R_ji = R_j R_i^T, t_ji = t_j - R_ji t_i, and the unit-depth ray map
// M = R_ji K_i^-1 (K as fx, fy, cx, cy per view), so that a source pixel
// (u, v) at depth Z lands at X' = Z M (u, v, 1)^T + t_ji in the target frame
__device__ inline void relative_pose(const double* __restrict__ poses,
                                     const float* __restrict__ K, int i, int j, double R[9],
                                     double t[3], double M[9]) {
    double Ri[9], ti[3], Rj[9], tj[3];
    for (int r = 0; r < 3; ++r) {
        for (int c = 0; c < 3; ++c) {
            Ri[3 * r + c] = poses[12 * i + 4 * r + c];
            Rj[3 * r + c] = poses[12 * j + 4 * r + c];
        }
        ti[r] = poses[12 * i + 4 * r + 3];
        tj[r] = poses[12 * j + 4 * r + 3];
    }
    for (int r = 0; r < 3; ++r)
        for (int c = 0; c < 3; ++c)
            R[3 * r + c] = Rj[3 * r + 0] * Ri[3 * c + 0] + Rj[3 * r + 1] * Ri[3 * c + 1] +
                           Rj[3 * r + 2] * Ri[3 * c + 2];
    for (int r = 0; r < 3; ++r)
        t[r] = tj[r] - (R[3 * r + 0] * ti[0] + R[3 * r + 1] * ti[1] + R[3 * r + 2] * ti[2]);
    const double fxi = K[4 * i + 0], fyi = K[4 * i + 1], cxi = K[4 * i + 2], cyi = K[4 * i + 3];
    for (int r = 0; r < 3; ++r) {
        M[3 * r + 0] = R[3 * r + 0] / fxi;
        M[3 * r + 1] = R[3 * r + 1] / fyi;
        M[3 * r + 2] = R[3 * r + 2] - R[3 * r + 0] * (cxi / fxi) - R[3 * r + 1] * (cyi / fyi);
    }
}

// per-scene convergence state (pose-change signal history and phase)
constexpr int kConvRing = 128;          // >= 2 w - 1 for windows up to 64
constexpr int kConvMaxViews = 4096;     // two doubles per view in LDS (64 KB)
struct ConvState {
    int32_t phase;                      // 0 poses, 1 joint phase, 2 stopped
    int32_t count;                      // signals recorded
    int32_t switch_step[2];             // steps of the 0->1 and 1->2 switches (-1)
    double theta[kConvRing];            // theta_95 history (ring)
};

// ---------------------------------------------------------------------------
// plan
// ---------------------------------------------------------------------------
struct Plan {
    int device = 0;
    int n_cu = 256;
    int32_t V = 0, S = 0, D = 0;
    epo_cost_params params{};
    epo_plan_options opt{};
    std::vector<int32_t> width, height, scene_of_view;
    std::vector<float> K;                 // V x 4
    std::vector<int64_t> view_offset;     // V
    std::vector<int64_t> rec_off;         // V + 1 record offsets
    std::vector<int32_t> pairs;           // D x 2
    std::vector<int32_t> group_host;      // D: image pair of each direction
    int64_t total_px = 0;
    int64_t n_residuals = 0;

    // device, plan lifetime
    DevBuf<uint64_t> records;             // (u | v << 16) | (Z bits << 32)
    // u8 quad texture (format 2) in blocks of kQuadBlockW x kQuadBlockH
    // pixels, one 128-byte cache line each, blocks row-major per view:
    // a wave's projected edge points touch about a fifth fewer lines than
    // with whole image rows
    DevBuf<uint32_t> tex;                 // total_blk texels (format 2 only while in use)
    std::vector<int64_t> blk_off;         // V: first texel of each view's blocks
    DevBuf<int64_t> blk_off_d;
    int64_t total_blk = 0;
    DevBuf<float> tex_f32;                // float32 sqrt(d2) per pixel (always kept: the
                                          // other formats are derived from it)
    DevBuf<float4> tex_q32;               // float32 taps of the cell at each pixel (format 3
                                          // only while it is in use)
    bool q8_ok = false;                   // lambda_max allows the saturated u8 taps
    DevBuf<int32_t> scene_of_view_d;
    DevBuf<float> K_d;                    // V x 4
    DevBuf<int32_t> wh_d;                 // V x 2
    DevBuf<int64_t> view_offset_d;        // V
    DevBuf<PairStatic> pair_static;       // D
    DevBuf<PairDesc> pair_desc;           // D (rewritten every iteration)
    DevBuf<double> pair_rel;              // D x 12: R_ji, t_ji (float64)
    DevBuf<Tile> tiles;                   // T
    // record_order 2: per-pair copies of the records, ordered by the target
    // block each projects to (re-sorted on the device); pair d's copy of its
    // source record r (absolute index) is sorted_records[r + pair_shift[d]]
    DevBuf<uint64_t> sorted_records;      // n_residuals + kRecordPad
    DevBuf<int64_t> pair_shift;           // D
    DevBuf<Tile> sort_chunks;             // sort units: <= 8192 records of one pair
    int64_t n_sort_chunks = 0;
    DevBuf<Partial> partials;             // T
    DevBuf<double> pair_sum;              // D x 8: S, n, G[6] (float64)
    DevBuf<double> pair_w;                // D: weight w_d
    DevBuf<double> pair_scale;            // D: 2 / (pairs of the scene in this step), 0 = skipped
    DevBuf<double> pair_scale_all;        // D: 2 / (pairs of the scene): every pair evaluated
    DevBuf<double> ext_partials;          // T x 2: focal-scale sums F_t, F_s per tile
    DevBuf<double> pair_ext;              // D x 2: F_t, F_s per pair
    DevBuf<int32_t> view_in_idx, view_in_ptr;     // CSR: pairs with tgt == v
    DevBuf<int32_t> view_out_idx, view_out_ptr;   // CSR: pairs with src == v
    DevBuf<int32_t> scene_ptr;            // CSR: pairs of scene s are [scene_ptr[s], scene_ptr[s+1]) of scene_pairs
    DevBuf<int32_t> scene_pairs;
    DevBuf<int32_t> counters;             // work counters of the 8 XCD queues
    DevBuf<int64_t> xcd_begin_d;          // 9 entries: tile range of each queue
    DevBuf<int32_t> tile_list;            // T: the step's selected tiles (pair sub-sampling)
    DevBuf<int32_t> tile_blk;             // per 1024 tiles: selected count, then offset
    DevBuf<int64_t> qbegin_d;             // 9 entries: queue ranges in tile_list
    DevBuf<int32_t> status;               // device status word
    DevBuf<int32_t> pose_done;            // pose-step workgroups finished (the last advances the step)
    DevBuf<int32_t> scene_view_ptr, scene_view_idx;   // CSR: views of each scene
    // stochastic pair sub-sampling: image pairs (groups of one or two
    // directions) numbered in order of first appearance in the pair list
    int32_t n_groups = 0;
    DevBuf<int32_t> group_of_pair;        // D: scene-major group slot of each direction
    DevBuf<int32_t> group_npairs;         // G slots: directions held (1 or 2)
    DevBuf<int32_t> group_id_sorted;      // G slots: group id (first-appearance order)
    std::vector<int32_t> group_id_sorted_h;
    DevBuf<int32_t> scene_group_ptr;      // S + 1: groups of scene s are [ptr[s], ptr[s+1])
    DevBuf<uint8_t> group_sel;            // G slots: selected in the last launch
    int32_t sample_budget = 0;            // M image pairs per scene per step; 0 = all
    uint64_t sample_seed = 0;
    const int32_t* sample_step = nullptr;   // device step counter read by the selection
    const int32_t* capture_step = nullptr;  // the captured iteration's counter (during capture)
    // early exit of stopped scenes (during the capture of an iteration that
    // skips them): the convergence phases the launches read; pair_scale then
    // holds 0 for every pair of a stopped scene, so an eager call without
    // sub-sampling first restores it from pair_scale_all
    const int32_t* gate_phase = nullptr;
    bool scale_gated = false;
    int32_t max_views_per_scene = 0;
    DevBuf<double> conv_prev;             // V x 12 poses of the previous step
    DevBuf<ConvState> conv_state;         // S
    DevBuf<int32_t> conv_phase;           // S (read by the schedule kernel)
    epo_convergence_params conv{25, 0.5f, 50, 0.1f};
    DevBuf<double> grad_scratch;          // V x 6 (graph iteration)
    // pose refiner MLP (allocated by its set-up call): per-scene rows padded
    // to 64, bf16 activations (h0: 16 wide; h1..h5, relu of layer 3: 128 wide)
    int64_t mlp_rows = 0;
    DevBuf<int64_t> mlp_row_off;          // S + 1
    DevBuf<uint16_t> mlp_act;             // mlp_rows x (16 + 6 x 128) bf16
    DevBuf<float> mlp_out;                // mlp_rows x 12 MLP outputs
    DevBuf<uint16_t> mlp_packed;          // S x kMlpPacked bf16 weights in MFMA operand order
    // focal and depth refinement: f = f0 (1 + gamma_v), Z = Z0 alpha + beta
    DevBuf<float> K0_d;                   // V x 4 intrinsics as given (K_d holds the refined ones)
    DevBuf<double> gamma_d;               // V: current focal scales gamma
    DevBuf<float> z0;                     // n_records depths as given (allocated on first update)
    DevBuf<int64_t> rec_off_d;            // V + 1 record offsets (allocated by the first joint step)
    // per-residual depth derivatives, source-major: source view i's records
    // in blocks of 256 (counted from its first record), each block holding
    // one 256-entry chunk per pair out of i, in CSR order, so the depth pass
    // reads one contiguous run per block.  Residual (d, record r) sits at
    // dz_index[2 d] + b n + (r - b), with b the first record of r's block and
    // n = dz_index[2 d + 1] the number of pairs out of the source
    DevBuf<int64_t> dz_index;             // D x 2
    int64_t dz_size = 0;
    DevBuf<float> dz;                     // dz_size dH/dZ per residual (allocated on first
                                          // update when it fits; else the depth pass recomputes)
    bool dz_declined = false;             // no room for dz: recompute form only
    DevBuf<Tile> vblocks;                 // 256-record blocks of each view (pair = view)
    int64_t n_vblocks = 0;
    DevBuf<float> lambda_buf;             // S (graph iteration)
    DevBuf<double> lr_buf;                // S (graph iteration)
    int64_t n_tiles = 0;
    int32_t tile_size = 0;
    int32_t n_xcd_queues = 8;
    std::vector<int64_t> xcd_begin;       // tile range of each XCD queue

    // timing
    bool timing = false;
    hipEvent_t ev0 = nullptr, ev1 = nullptr;
    bool timed_once = false;

    // captured iteration
    hipGraph_t graph = nullptr;
    hipGraphExec_t graph_exec = nullptr;

    ~Plan();
};

// schedule (tile list) construction; (re)allocates tiles and partials
void build_tiles(Plan& p, hipStream_t stream);
// drops a captured iteration (after any change of what it would launch)
void release_graph(Plan& p);

// outputs of the refinement variant (each may be null)
struct RefineOut {
    double* grad_gamma;     // V: dL/dgamma_v
    double* grad_alpha;     // n_records: dL/dalpha = Z0 dL/dZ
    double* grad_beta;      // n_records: dL/dbeta = dL/dZ
};

// the fused kernel runs over a compacted list of this step's tiles (pair
// sub-sampling, or stopped scenes skipped) instead of every tile
inline bool compacted_launch(const Plan& p) { return p.sample_budget > 0 || p.gate_phase; }

// The paper's schedules at step s (Sec. 4 "Implementation Details"): the
// clamp lambda falls linearly from l0 to l1 over `anneal` steps (the same for
// every scene); the learning rate rises linearly over `warmup` steps, then
// follows a cosine to 0 at `total`; a stopped scene (phase 2) gets rate 0.
// One function for the schedule kernel and the pair set-up kernel that takes
// its place in the captured pose iteration.
struct ScheduleArgs {
    const int32_t* step;        // null: no schedule in this launch
    float l0, l1;
    int32_t anneal;
    double peak;
    int32_t warmup, total;
    float* lam;                 // per scene (may be null)
    double* lr;                 // per scene (may be null)
    const int32_t* phase;       // per scene (may be null)
    int32_t S;
};
__device__ inline void schedule_at(const ScheduleArgs& a, int s, float& lv, double& r) {
    const double frac = a.anneal > 0 ? (double)min(s, a.anneal) / (double)a.anneal : 1.0;
    lv = (float)((double)a.l0 - ((double)a.l0 - (double)a.l1) * frac);
    if (s < a.warmup)
        r = a.peak * (double)(s + 1) / (double)a.warmup;
    else
        r = a.peak * 0.5 * (1.0 + cos(M_PI * (double)(s - a.warmup) / (double)(a.total - a.warmup)));
}

// launches of the per-iteration pipeline (no allocation, no sync)
void launch_cost(Plan& p, const double* poses, const float* lambda, double* loss,
                 double* pair_cost, int32_t* pair_valid, double* pair_grad, double* grad,
                 const double* upstream, hipStream_t stream, const RefineOut* ext = nullptr,
                 const ScheduleArgs* sched = nullptr);
void launch_reductions(Plan& p, double* loss, double* pair_cost, int32_t* pair_valid,
                       double* pair_grad, double* grad, const double* upstream,
                       hipStream_t stream, double* grad_gamma = nullptr);
// pair set-up and the fused kernel alone (launch_cost without the reductions);
// with `sched`, the pair set-up also evaluates the schedule (lambda from the
// step instead of `lambda`, and the per-scene lambda and rate written out)
void launch_tiles(Plan& p, const double* poses, const float* lambda, hipStream_t stream,
                  const RefineOut* ext = nullptr, const ScheduleArgs* sched = nullptr);
// reductions + pose step + step count in one launch for small plans (false:
// the plan is too large, nothing launched)
bool launch_step_epilogue(Plan& p, double* loss, double* grad, double* poses, double* m,
                          double* v, const uint8_t* fixed, const double* lr, double b1,
                          double b2, double eps, int32_t* step, hipStream_t stream);
void launch_depth_grad(Plan& p, const double* upstream, double* grad_alpha, double* grad_beta,
                       bool stored, hipStream_t stream);
// with `done` (a device counter at 0), the pose-step kernel's last workgroup
// advances the step itself and rearms the counter; without, a second launch
void launch_pose_step(double* poses, double* m, double* v, const double* grad, int32_t n_views,
                      const int32_t* scene_of_view, const uint8_t* fixed, const double* lr,
                      double b1, double b2, double eps, int32_t* step, hipStream_t stream,
                      int32_t* done = nullptr);
void launch_schedule(const int32_t* step, int32_t n_scenes, float lambda0, float lambda1,
                     int32_t anneal_steps, double peak_lr, int32_t warmup, int32_t total,
                     float* lambda_out, double* lr_out, const int32_t* phase,
                     hipStream_t stream);
void launch_convergence(Plan& p, const double* poses, double* theta_out, hipStream_t stream);
void launch_pair_selection(Plan& p, const int32_t* step, hipStream_t stream);
void launch_convergence_reset(Plan& p, const double* poses, hipStream_t stream);
// textures: float32 sqrt(d2) from d2 (kept), the format in use derived from
// it; a format's texture is built when selected and freed when another is
void build_texture(Plan& p, const int32_t* d2, hipStream_t stream);
void ensure_texture(Plan& p, int fmt, hipStream_t stream);
void release_unused_textures(Plan& p);
// record_order 2: allocate the per-pair record copies (source order until
// the first sort); re-sort them at the given poses: every chunk (step null), or
// the chunks c with c mod every == *step mod every
void ensure_sorted_records(Plan& p, hipStream_t stream);
void launch_resort(Plan& p, const double* poses, const int32_t* step, int32_t every,
                   hipStream_t stream);
// refinement of the joint phase: install (gamma, alpha, beta) in the plan
// (allocates on the first depth update), the joint AdamW step (needs the
// record offsets on the device), and the device copy of the record offsets
void install_refinement(Plan& p, const double* gamma, const float* alpha, const float* beta,
                        hipStream_t stream);
void launch_joint_step(Plan& p, const epo_joint_state& j, const double* lr, const int32_t* phase,
                       double b1, double b2, double eps, hipStream_t stream);
void ensure_record_offsets(Plan& p, hipStream_t stream);
void mlp_setup(Plan& p, hipStream_t stream);
void launch_mlp_forward(Plan& p, const float* params, const double* poses0, const double* delta,
                        double* poses, hipStream_t stream);
void launch_mlp_backward(Plan& p, const float* params, const double* poses0, const double* poses,
                         const double* grad, float* param_grad, double* delta_grad,
                         hipStream_t stream);
void launch_adamw(Plan& p, float* params, float* m, float* v, const float* g, double* delta,
                  double* dm, double* dv, const double* dg, const double* lr, double b1, double b2,
                  double eps, double wd_mlp, double wd_delta, int32_t* step, hipStream_t stream);

inline int64_t ceil_div(int64_t a, int64_t b) { return (a + b - 1) / b; }

}  // namespace epo
