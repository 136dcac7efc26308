/*
 * epo.h -- C-ABI of libepo.so, the MI355X (gfx950) hot path of EPO's
 * edge-based pose optimization (arXiv 2607.00579).
 *
 * The problem (paper Sec. 3 "Method"): a geometric estimate
 * G = {(K_i, P_i, Z_i)} of V views (intrinsics, world->camera pose, per-pixel
 * depth), a binary edge map E_i and its distance transform field DTF_i per
 * view, and a list of image pairs.  Edge pixels of each source view are lifted
 * to 3-D with their depth, moved into the target camera by the relative pose,
 * pinhole-projected, and scored by a clamped Huber loss of the bilinearly
 * sampled target DTF (Eqs. pi, L, L_ij, d_ij; supplementary Alg. 3).  The loss
 * is minimised by gradient steps on the poses; the output is the refined
 * poses.
 *
 * Conventions shared by every call
 *  - Pointers are DEVICE pointers unless the argument is marked (host).
 *  - The caller owns every buffer it passes.  The library only borrows the
 *    pointers for the work it enqueues; a plan owns the workspace it allocates
 *    in epo_plan_create and frees in epo_plan_destroy.
 *  - `stream` is a hipStream_t passed as void* (NULL = the null stream).
 *    Every call is asynchronous on that stream unless stated otherwise.
 *  - Pixels: u = column, v = row, integer coordinates at pixel centres.
 *    Images are row-major uint8 / float32 / int32 of height x width, packed
 *    back to back at per-view element offsets.
 *  - Intrinsics K: 4 floats per view (fx, fy, cx, cy).
 *  - Poses: float64 world->camera [R | t], 12 doubles per view, row-major
 *    3 x 4, OpenCV axes (x right, y down, z forward).  Depth is z-depth.
 *  - Twists: left perturbations xi = (rho, omega), P <- Exp(xi) P, translation
 *    first; gradients are float64 dL/dxi at xi = 0, 6 doubles per view.
 *  - Errors: every entry point returns an epo_status; no C++ exception
 *    crosses the ABI.  epo_last_error() gives a thread-local message.
 *    Argument and shape errors are detected on the host before any work is
 *    enqueued; launch failures map to EPO_ERR_HIP.
 *  - Threading: a plan must not be used by two host threads at once; distinct
 *    plans are independent.
 */
#ifndef EPO_H
#define EPO_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#if defined(__GNUC__) || defined(__clang__)
#define EPO_API __attribute__((visibility("default")))
#else
#define EPO_API
#endif

typedef enum epo_status {
    EPO_OK = 0,
    EPO_ERR_INVALID_ARG = -1,   /* null pointer, bad size, index out of range */
    EPO_ERR_HIP = -2,           /* a HIP runtime call or kernel launch failed */
    EPO_ERR_UNSUPPORTED = -3,   /* valid request outside what the build supports */
    EPO_ERR_NONFINITE = -4      /* a non-finite value was detected (see device status) */
} epo_status;

/* Largest image side accepted anywhere (keeps every squared distance < 2^30). */
#define EPO_MAX_SIDE 16384
/* Squared distance stored for every pixel of an edge map without edge pixels. */
#define EPO_D2_EMPTY (1 << 30)

/* Cost parameters (paper Sec. 3 "Edge Reprojection Loss"; Alg. 3).
 *   huber_delta  threshold of the Huber loss H (the paper does not state it;
 *                default 1 px): H(d) = d^2/2 for d <= delta, else
 *                delta (d - delta/2)
 *   z_min        a projection is valid only if the target-camera depth
 *                exceeds z_min (default 1e-4); must be in [1e-6, 1e6].  With
 *                depths and translations below 1e30 in magnitude every
 *                intermediate stays finite; beyond that a sum may become
 *                non-finite, which sets bit 0 of the device status word
 *   norm_mode    0: per-direction mean over valid residuals (Alg. 3,
 *                default); 1: sum over the source edge count |E_i| (Eq. L_ij)
 *   lambda_max   largest clamp lambda the plan will be called with (default
 *                10, the start of the paper's annealing 10 -> 6).  Values up to
 *                14.5 allow the compact texture (see epo_plan_options). */
typedef struct epo_cost_params {
    float huber_delta;
    float z_min;
    int32_t norm_mode;
    float lambda_max;
} epo_cost_params;

/* Kernel schedule choices.  0 in any field = let the plan decide (the
 * autotuner, epo_plan_autotune, may change the decision later). */
typedef struct epo_plan_options {
    int32_t texture_format;     /* 1 = float32 taps of sqrt(d2) (4 gathers per sample);
                                   2 = one uint32 per pixel holding the four taps of the
                                   bilinear cell as min(d2, 255) bytes (1 gather per
                                   sample; exact for lambda_max <= 14.5), stored in
                                   8 x 4 pixel blocks of 128 bytes;
                                   3 = the four float32 taps of the cell per pixel
                                   (one 16-byte gather per sample) */
    int32_t points_per_thread;  /* residuals per thread per tile: 1, 2, 4, 8 or 16
                                   (a tile is 256 x this many residuals of one pair) */
    int32_t tile_order;         /* 1 = tiles grouped by target view, consecutive groups
                                   on one XCD; 2 = tiles in pair-list order */
    int32_t persistent;         /* 1 = persistent work-queue launch; 2 = one workgroup
                                   per tile */
    int32_t record_order;       /* 1 = every pair reads its source view's records in
                                   source order; 2 = every pair reads its own copy of
                                   them, ordered by the 8 x 4 target pixel block each
                                   record projects to (chunks of 8192 records), so the
                                   taps gathered by one wavefront share cache lines.
                                   The copies take 8 bytes per residual of device
                                   memory and are re-sorted by epo_plan_resort and by
                                   the captured iterations; only the summation order
                                   of the results depends on the order */
    int32_t resort_interval;    /* record_order 2: a captured iteration re-sorts the
                                   chunks c with c mod k == step mod k, k = this many
                                   steps (default 8) */
    int32_t graph_steps;        /* iterations one captured graph holds, 1 .. 64
                                   (default 1): the capture entry points record the
                                   iteration this many times in a row, and each
                                   epo_iteration_launch then runs that many steps
                                   (the step counter, schedule and convergence gates
                                   are read on the device at every one of them), so
                                   one graph launch serves several steps */
} epo_plan_options;

typedef struct epo_plan_s* epo_plan;

/* ---------------------------------------------------------------------------
 * 1. build_distance_fields
 * Exact squared Euclidean distance transform of binary edge maps (the DTF of
 * Sec. 3 "Method", computed in the two separable passes of the
 * Felzenszwalb-Huttenlocher transform;
 * supplementary Sec. A1.2 "Construction kernels"):
 *   d2(x, y) = min over pixels (x', y') with edge(y', x') != 0 of
 *              (x - x')^2 + (y - y')^2,
 * an exact integer; EPO_D2_EMPTY for every pixel of a map with no edge pixel.
 * The DTF itself is sqrt(d2) (rounded to float32).
 *
 *   edge_maps    uint8, nonzero = edge; view v occupies elements
 *                [view_offset[v], view_offset[v] + height[v] * width[v])
 *   view_offset  (host) int64 [n_views] element offsets (views must not overlap)
 *   width/height (host) int32 [n_views], each in [1, EPO_MAX_SIDE]
 *   d2_out       int32, same packing as edge_maps: exact squared distances
 *                (it holds the column pass's per-segment edge rows during
 *                the call)
 *   dtf_out      float32, same packing: sqrt(d2).  Required: it also serves as
 *                the scratch of the column pass during the call.
 * Errors: EPO_ERR_INVALID_ARG for null pointers, n_views < 0, sides out of
 * range or negative offsets.  No device allocation; capture-safe.
 * ------------------------------------------------------------------------- */
EPO_API epo_status epo_build_distance_fields(const uint8_t* edge_maps, const int64_t* view_offset,
                                     const int32_t* width, const int32_t* height,
                                     int32_t n_views, int32_t* d2_out, float* dtf_out,
                                     void* stream);

/* ---------------------------------------------------------------------------
 * Plan: the static part of a problem (one or several independent scenes).
 * Compacts the edge pixels of every view into 8-byte records (u, v as uint16,
 * depth Z as float32; every edge pixel is used, no sub-sampling), builds the
 * sampling texture of every view from d2, and the tile schedule over
 * (directed pair, record chunk).  Synchronises `stream` once (edge counts come
 * back to the host).  The edge maps, depth maps and d2 may be freed after the
 * call returns.
 *
 *   n_views         number of views V (>= 1)
 *   width/height    (host) int32 [V], each in [2, EPO_MAX_SIDE]
 *   K               (host) float32 [V][4] (fx, fy, cx, cy); fx, fy > 0
 *   scene_of_view   (host) int32 [V] scene index per view, scenes numbered
 *                   0..S-1 with every scene non-empty; NULL = one scene
 *   view_offset     (host) int64 [V] element offsets of the packed images
 *   edge_maps       uint8 packed edge maps (nonzero = edge)
 *   depth           float32 packed depth maps (read at edge pixels only; must
 *                   be finite there, EPO_ERR_INVALID_ARG otherwise)
 *   d2              int32 packed squared distances (epo_build_distance_fields)
 *   pairs           (host) int32 [n_pairs][2] directed pairs (source, target),
 *                   both views of a pair in the same scene; the loss of a
 *                   scene is (2 / its number of pairs) * sum of per-pair means,
 *                   the paper's mean over pairs of both directions when the
 *                   list holds (i, j) and (j, i)
 *   params          (host) cost parameters, NULL = defaults
 *   options         (host) schedule choices, NULL = automatic
 * Errors: EPO_ERR_INVALID_ARG (shapes, indices, scene numbering, K),
 * EPO_ERR_UNSUPPORTED (lambda_max too large for the requested texture),
 * EPO_ERR_HIP (allocation or launch).
 * ------------------------------------------------------------------------- */
EPO_API epo_status epo_plan_create(epo_plan* out, int32_t n_views, const int32_t* width,
                           const int32_t* height, const float* K, const int32_t* scene_of_view,
                           const int64_t* view_offset, const uint8_t* edge_maps,
                           const float* depth, const int32_t* d2, const int32_t* pairs,
                           int32_t n_pairs, const epo_cost_params* params,
                           const epo_plan_options* options, void* stream);

EPO_API epo_status epo_plan_destroy(epo_plan plan);

/* Sizes of a plan (host outputs, any may be NULL): number of scenes, total
 * edge records, residuals per iteration (sum over pairs of source edge
 * counts), number of tiles, and the schedule in use. */
EPO_API epo_status epo_plan_info(epo_plan plan, int32_t* n_scenes, int64_t* n_records,
                         int64_t* n_residuals, int64_t* n_tiles, epo_plan_options* options);

/* Edge records of view v in plan order (u | v << 16 in the low word, float32 Z
 * bits in the high word), copied to `records_out` (host, at least
 * edge_count(v) entries); count returned in *count.  Synchronous.  Testing and
 * inspection only. */
EPO_API epo_status epo_plan_view_records(epo_plan plan, int32_t v, uint64_t* records_out,
                                 int64_t capacity, int64_t* count);

/* ---------------------------------------------------------------------------
 * 2. edge_cost_fwd
 * Loss of every scene at `poses`, and, when `grad` is non-NULL, its gradient
 * from the same fused pass (the forward and the analytic adjoint run in one
 * kernel; supplementary Sec. A1.2 "Per-iteration kernels").
 * Per directed pair d = (i -> j): S_d = sum of H(min(D, lambda)) over valid
 * residuals, n_d = number of valid residuals, L_d = S_d / n_d (0 if n_d = 0);
 * loss[s] = (2 / |pairs of s|) sum_{d in s} L_d (with pair sub-sampling on,
 * over the pairs drawn for this launch, see 3c).
 *
 *   poses       float64 [V][3][4]
 *   lambda      float32 [n_scenes] clamp per scene, each in [0, params.lambda_max]
 *   loss        float64 [n_scenes] (written)
 *   pair_cost   float64 [n_pairs] L_d, or NULL
 *   pair_valid  int32 [n_pairs] n_d, or NULL
 *   pair_grad   float64 [n_pairs][6] unweighted sum over the valid residuals of
 *               pair d of the left-twist gradient of the TARGET pose, or NULL
 *   grad        float64 [V][6] dloss[scene(v)]/dxi_v, or NULL
 * Residual arithmetic is float32; per-pair and per-pose sums are float64 and
 * run in a fixed order, so results are bitwise reproducible.  No allocation,
 * no synchronisation, capture-safe.
 * ------------------------------------------------------------------------- */
EPO_API epo_status epo_edge_cost_fwd(epo_plan plan, const double* poses, const float* lambda,
                             double* loss, double* pair_cost, int32_t* pair_valid,
                             double* pair_grad, double* grad, void* stream);

/* ---------------------------------------------------------------------------
 * 3. edge_cost_bwd
 * Adjoint only: recomputes the residuals and writes
 *   grad[v] = upstream[scene(v)] * dloss[scene(v)]/dxi_v     (overwrites).
 *   upstream  float64 [n_scenes]; NULL = all ones
 * No allocation, no synchronisation, capture-safe.
 * ------------------------------------------------------------------------- */
EPO_API epo_status epo_edge_cost_bwd(epo_plan plan, const double* poses, const float* lambda,
                             const double* upstream, double* grad, void* stream);

/* ---------------------------------------------------------------------------
 * 3b. Focal-length and depth refinement (paper Sec. 3 "Camera Refinement",
 * "Depth Refinement"; the intrinsics update and depth module of the forward
 * loop, supplementary Alg. EPO.Forward).  Per view v and edge pixel p:
 *   f_v = f0_v (1 + gamma_v)     (fx and fy scale together; cx, cy fixed)
 *   Z_p = Z0_p alpha_p + beta_p
 * where f0, Z0 are the intrinsics and depths the plan was built with.
 *
 * epo_plan_set_refinement sets the current gamma, alpha, beta (device
 * pointers, read during the call's kernels only):
 *   gamma        float64 [V], or NULL = all 0
 *   alpha, beta  float32 [n_records] in the plan's record order (see
 *                epo_plan_view_records: records of view v are
 *                [offset_v, offset_v + count_v), views in order), both or
 *                neither; NULL = alpha 1, beta 0
 * The refined focal length is float32(f0 * (1 + gamma)) (product in float64)
 * and the refined depth float32(fma(Z0, alpha, beta)) in float64.  Later cost
 * launches (and replays of a captured iteration) use the refined values.  A
 * refined focal length that is not finite and > 0, or a depth that is not
 * finite, sets bit 2 of the device status word.  The first call with depths
 * allocates a copy of Z0 (4 bytes per record); no synchronisation.
 *
 * epo_edge_cost_refine: loss and every gradient of the joint phase in one
 * call (each output may be NULL, outputs overwritten):
 *   upstream    float64 [n_scenes] scale of each scene's loss, or NULL = 1
 *   loss        float64 [n_scenes]  (not scaled by upstream)
 *   grad        float64 [V][6]      pose left twists, as epo_edge_cost_bwd
 *   grad_gamma  float64 [V]         dloss[scene(v)]/dgamma_v
 *   grad_alpha  float64 [n_records] dloss/dalpha_p = Z0_p dloss/dZ_p
 *   grad_beta   float64 [n_records] dloss/dbeta_p  = dloss/dZ_p
 * grad_gamma comes from a variant of the fused kernel that also sums the
 * focal terms of both views of every pair; grad_alpha / grad_beta from a
 * second, source-major pass (one thread per edge record, pairs out of its
 * view in a fixed order): no atomics, bitwise reproducible.  No allocation,
 * no synchronisation, capture-safe.
 * ------------------------------------------------------------------------- */
EPO_API epo_status epo_plan_set_refinement(epo_plan plan, const double* gamma, const float* alpha,
                                   const float* beta, void* stream);
EPO_API epo_status epo_edge_cost_refine(epo_plan plan, const double* poses, const float* lambda,
                                const double* upstream, double* loss, double* grad,
                                double* grad_gamma, double* grad_alpha, double* grad_beta,
                                void* stream);

/* ---------------------------------------------------------------------------
 * Joint-phase optimizer step (paper Sec. 3 "Camera Refinement", "Depth
 * Refinement"; Sec. 4 "Implementation Details": every parameter is trained
 * with AdamW, beta = (0.9, 0.999), weight decay 0.01; Alg. EPO.Forward: the
 * depth optimizer steps only once the pose-phase criterion holds).
 *
 * epo_joint_step applies one AdamW step to the focal scales gamma and the
 * per-record depth scale alpha and shift beta, then makes the new values the
 * plan's refinement exactly as epo_plan_set_refinement does.  For each
 * parameter x with gradient g, learning rate a = lr[scene] and t = 1 + the
 * steps its optimizer has taken (per scene, focal scales and depth
 * parameters counted apart, as separate optimizers; see `steps`):
 *   x <- x (1 - a wd),  m <- b1 m + (1 - b1) g,  w <- b2 w + (1 - b2) g^2,
 *   x <- x - a (m / (1 - b1^t)) / (sqrt(w / (1 - b2^t)) + eps)
 * in float64 (alpha, beta are read as float32, rounded once when stored).
 *
 *   gamma               float64 [V], updated in place
 *   alpha, beta         float32 [n_records] (plan record order), in place
 *   m_gamma, v_gamma    float64 [V] moments, in place (start at 0)
 *   m_depth, v_depth    float64 [2][n_records] moments: alpha's, then beta's
 *   grad_*              float64, as written by epo_edge_cost_refine
 *   lr                  float64 [n_scenes]
 *   phase               int32 [n_scenes] or NULL: with phases (as written by
 *                       epo_convergence_update: 0 pose phase, 1 joint phase,
 *                       2 stopped), gamma steps unless the scene has stopped
 *                       and alpha, beta step only in phase 1; a parameter that
 *                       does not step keeps its value and moments (no decay).
 *                       NULL: every parameter steps.
 *   wd_focal, wd_depth  weight decay of gamma and of alpha, beta (the paper:
 *                       0.01 for both)
 *   steps               int32 [2][n_scenes] step counts, start at 0:
 *                       steps[s] the AdamW steps scene s's focal scales have
 *                       taken, steps[n_scenes + s] those of its depth
 *                       parameters (so the depth optimizer's first step after
 *                       the switch to the joint phase is its step 1); the call
 *                       advances the count of every parameter kind that
 *                       stepped
 * All arrays are device memory.  Errors: EPO_ERR_INVALID_ARG for a null
 * pointer other than phase or betas outside [0, 1) or eps <= 0.  The first
 * call allocates a copy of the plan's record offsets (8 bytes per view) and,
 * through the refinement update, what epo_plan_set_refinement allocates on
 * its first call with depths; later calls allocate nothing and do not
 * synchronise.
 * ------------------------------------------------------------------------- */
EPO_API epo_status epo_joint_step(epo_plan plan, double* gamma, float* alpha, float* beta,
                                  double* m_gamma, double* v_gamma, double* m_depth,
                                  double* v_depth, const double* grad_gamma,
                                  const double* grad_alpha, const double* grad_beta,
                                  const double* lr, const int32_t* phase, double beta1,
                                  double beta2, double eps, double wd_focal, double wd_depth,
                                  int32_t* steps, void* stream);

/* ---------------------------------------------------------------------------
 * The two-phase loop of the joint phase as one captured iteration (paper
 * Alg. 2 with Sec. 3 "Camera Refinement" / "Depth Refinement"): per replay
 *   schedule (lambda(s), lr(s) per scene; lr 0 once a scene has stopped)
 *   -> cost, pose, focal and per-pixel depth gradients at the current poses
 *      and refinement (epo_edge_cost_refine)
 *   -> joint AdamW step of gamma, alpha, beta gated by the scene's phase on
 *      the device, which installs the new refinement (epo_joint_step)
 *   -> Adam twist step of the poses (epo_pose_step)
 *   -> convergence test (with_convergence 1 or 2), which moves a scene to the
 *      joint phase (its depth parameters step from the next replay on) and
 *      then stops it,
 * with no host synchronisation.  with_convergence 0: no test, every
 * parameter steps at every replay.  2: a stopped scene's tiles also leave the
 * fused launch from the next replay on (as for epo_iteration_capture).
 *
 * epo_joint_state names the caller's device buffers of the joint phase (as
 * for epo_joint_step; grad_* are written at every replay and may be read
 * after it).  The pointers are baked into the graph.  Before capture the
 * call installs the state's refinement in the plan (allocating, on the
 * plan's first depth update, the copy of its depths and, if it fits in half
 * the free memory, the per-residual depth derivatives) and synchronises;
 * with the test, epo_convergence_reset must have been called on `poses`.
 * Errors: EPO_ERR_INVALID_ARG for a null pointer (grad may be NULL) or a
 * schedule out of range.  Replaces a previously captured iteration; replay
 * with epo_iteration_launch.
 * ------------------------------------------------------------------------- */
typedef struct epo_joint_state {
    double* gamma;        /* [V] focal scales */
    float* alpha;         /* [n_records] depth scales (plan record order) */
    float* beta;          /* [n_records] depth shifts */
    double* m_gamma;      /* [V] AdamW moments of gamma */
    double* v_gamma;      /* [V] */
    double* m_depth;      /* [2][n_records]: alpha's, then beta's */
    double* v_depth;      /* [2][n_records] */
    int32_t* steps;       /* [2][n_scenes] focal and depth step counts */
    double* grad_gamma;   /* [V] written by every replay */
    double* grad_alpha;   /* [n_records] written by every replay */
    double* grad_beta;    /* [n_records] written by every replay */
    double wd_focal;      /* weight decay of gamma (the paper: 0.01) */
    double wd_depth;      /* weight decay of alpha, beta (the paper: 0.01) */
} epo_joint_state;

EPO_API epo_status epo_joint_iteration_capture(epo_plan plan, double* poses, double* adam_m,
                                               double* adam_v, int32_t* step, double* loss,
                                               double* grad, const epo_joint_state* joint,
                                               float lambda0, float lambda1, int32_t anneal_steps,
                                               double peak_lr, int32_t warmup, int32_t total,
                                               double beta1, double beta2, double eps,
                                               int32_t with_convergence, void* stream);

/* ---------------------------------------------------------------------------
 * Viewgraph estimation (paper Sec. 3 "Viewgraph Estimation", Sec. 4
 * "Implementation Details"; construction kernels of the supplementary
 * material).  For every candidate pair (i, j), each pixel p = (a s, b s) of
 * the stride-s grid over image i with depth Z_i(p) > 0 (finite) is projected
 * into j and back:
 *   p_ij  = pi(K_i, K_j, P_i, P_j, Z_i; p)   (target depth must exceed z_min)
 *   p_iji = pi(K_j, K_i, P_j, P_i, Z_j; p_ij), Z_j read at the pixel nearest to
 *           p_ij (inside image j, depth > 0), back depth above z_min,
 * and counted consistent when |p - p_iji|^2 < tau^2.  total[c] counts the grid
 * points with depth, consistent[c] the consistent ones, and valid[c] =
 * (total > 0 and consistent >= min_fraction * total).  The paper's values:
 * tau = 3 px, min_fraction = 0.125.  Every decision is taken in float64 with
 * one rounding per operation (no fused multiply-add) in a fixed order.
 *
 *   width, height, K, view_offset   host, per view (K = fx, fy, cx, cy)
 *   depth        float32 dense depth maps, view v at view_offset[v] (elements),
 *                row-major H x W (device)
 *   poses        float64 [V][3][4] world->camera (device)
 *   candidates   int32 [n_candidates][2] (i, j) (host)
 *   consistent, total   int32 [n_candidates] (device, written)
 *   valid        uint8 [n_candidates] (device, written) or NULL
 * Setup-time call: allocates staging buffers and synchronises `stream`.
 * ------------------------------------------------------------------------- */
EPO_API epo_status epo_build_viewgraph(int32_t n_views, const int32_t* width, const int32_t* height,
                               const float* K, const int64_t* view_offset, const float* depth,
                               const double* poses, const int32_t* candidates,
                               int32_t n_candidates, int32_t stride, double tau,
                               double min_fraction, double z_min, int32_t* consistent,
                               int32_t* total, uint8_t* valid, void* stream);

/* The same call without any allocation, for callers that cannot allocate
 * device memory: code under HIP graph capture, tight serving loops, harnesses
 * that forbid hipMalloc.  Arguments, results and errors are those of
 * epo_build_viewgraph (bitwise the same counts).  The staging of the
 * candidates, the work list and the per-view sizes, offsets and intrinsics
 * lives in a static device array of 4 MiB that every GPU the library runs on
 * holds until the process ends; a call whose staging exceeds it fails with
 * EPO_ERR_INVALID_ARG (about 4 MiB / 8 bytes of candidates plus grid chunks of
 * 1024 points, e.g. 496 candidates of 518 x 518 views at stride 1).  Calls
 * that overlap on one GPU (other streams or threads) share that array and
 * race.  Copies the host arrays into it and synchronises `stream`. */
EPO_API epo_status epo_build_viewgraph_noalloc(int32_t n_views, const int32_t* width,
                                               const int32_t* height, const float* K,
                                               const int64_t* view_offset, const float* depth,
                                               const double* poses, const int32_t* candidates,
                                               int32_t n_candidates, int32_t stride, double tau,
                                               double min_fraction, double z_min,
                                               int32_t* consistent, int32_t* total,
                                               uint8_t* valid, void* stream);

/* ---------------------------------------------------------------------------
 * 3c. Stochastic viewgraph sub-sampling (paper supplementary Sec. "Stochastic
 * viewgraph sub-sampling"; pair budget M of Alg. EPO.Forward).  With a budget
 * M > 0, every later cost launch of the plan (eager, and replays of an
 * iteration captured afterwards) first draws, per scene, a fresh uniform
 * random subset of min(|E_scene|, M) image pairs and evaluates only their
 * directions; each scene's loss is then the mean over the evaluated
 * directions, (2/|D_S|) sum_{d in D_S} L_d, and skipped pairs have zero cost,
 * count, weight and gradient.  An image pair is an unordered {i, j}; pairs
 * are numbered in order of first appearance in the plan's pair list.
 *
 * The draw is counter-based: pair g gets the key h(h(seed + step) + g), h the
 * SplitMix64 output function (Steele, Lea, Flood, OOPSLA 2014), and the M
 * pairs with the smallest (key, g) are taken.
 *
 *   budget  M image pairs per scene per step; 0 = every pair (sub-sampling off)
 *   seed    64-bit seed of the draw
 *   step    int32 [1] device step counter read at every launch (eager
 *           launches); must stay valid while sampling is on.  A captured
 *           iteration reads its own step counter instead (the one it
 *           increments), so every replay draws a new subset.
 * Synchronises `stream` and drops a captured iteration (capture again).
 *
 * epo_plan_sampled_pairs writes, per directed pair, 1 if it was evaluated by
 * the plan's last cost launch and 0 if skipped (uint8 [n_pairs], device).
 * ------------------------------------------------------------------------- */
EPO_API epo_status epo_plan_set_pair_sampling(epo_plan plan, int32_t budget, uint64_t seed,
                                      const int32_t* step, void* stream);
EPO_API epo_status epo_plan_sampled_pairs(epo_plan plan, uint8_t* selected, void* stream);

/* ---------------------------------------------------------------------------
 * 4b. The paper's pose parameterization (Sec. 3 "Pose Refinement", Sec. 4
 * "Implementation Details"): per scene, every pose is produced from its
 * initial pose P0 by
 *     P = phi(P0 + MLP(P0)) + [0 | delta]
 * MLP: six linear layers 12 -> 128 -> 128 -> 128 -> 128 -> 128 -> 12 on P0
 * flattened row-major, ReLU after the first five, the first layer's output
 * added to the third's (skip connection); phi orthonormalises the first two
 * columns of the rotation block by Gram-Schmidt (6D representation); delta is
 * a per-view translation offset.  Matrix products run in BF16 on the matrix
 * cores with float32 accumulation: bf16 operands (weights rounded from their
 * float32 values, activations and activation gradients stored in bf16), bias /
 * ReLU / skip / masks on the float32 accumulators; weight and bias gradients
 * and the MLP output float32; the pose algebra float64.
 *
 *   params      float32 [n_scenes][EPO_MLP_PARAMS]: W1 (128 x 12, row-major
 *               out x in), b1, W2, b2, ..., W6 (12 x 128), b6
 *   poses0      float64 [V][3][4] initial poses; delta float64 [V][3]
 *   poses       float64 [V][3][4] (forward: written; backward: the forward's
 *               output)
 *   grad        float64 [V][6] left-twist gradient of the loss at `poses`
 *   param_grad  float32 [n_scenes][EPO_MLP_PARAMS] (written);
 *   delta_grad  float64 [V][3] (written)
 * epo_mlp_setup allocates the activation store (once per plan; about 1.6 KB
 * per view, plus 272 KB per scene of weights packed in bf16 for the matrix
 * cores).  epo_mlp_backward uses the activations and the packed weights of
 * the last forward (params must hold the same values).
 * epo_mlp_step: AdamW (x <- x (1 - lr wd), then Adam with bias correction at
 * step = *step + 1) on every parameter (wd_mlp) and delta (wd_delta), lr per
 * scene [n_scenes]; increments *step.  No allocation after set-up, no
 * synchronisation, capture-safe.
 * ------------------------------------------------------------------------- */
#define EPO_MLP_PARAMS 69260
EPO_API epo_status epo_mlp_setup(epo_plan plan, void* stream);
EPO_API epo_status epo_mlp_forward(epo_plan plan, const float* params, const double* poses0,
                           const double* delta, double* poses, void* stream);
EPO_API epo_status epo_mlp_backward(epo_plan plan, const float* params, const double* poses0,
                            const double* poses, const double* grad, float* param_grad,
                            double* delta_grad, void* stream);
/* One iteration of the loop with this parameterization, captured as a HIP
 * graph and replayed with epo_iteration_launch: device schedule (lambda, lr;
 * lr 0 for a scene stopped by the convergence test) -> fused cost + adjoint
 * at `poses` -> epo_mlp_backward -> epo_mlp_step (advances *step) ->
 * epo_mlp_forward of the new parameters into `poses` -> [pose-change test,
 * with_convergence 1 or 2, as in epo_iteration_capture: with 2 a stopped
 * scene's tiles are skipped, its parameter gradients read 0 and its
 * parameters stay].  Before the first replay `poses` must hold
 * epo_mlp_forward of the current parameters (the backward reads that
 * forward's activations), and, with the test, epo_convergence_reset must
 * have been called on them.  Replaces a previously captured iteration; grad
 * may be NULL (internal buffer).  Errors as epo_iteration_capture. */
EPO_API epo_status epo_mlp_iteration_capture(
    epo_plan plan, float* params, float* adam_m, float* adam_v, float* param_grad, double* delta,
    double* delta_m, double* delta_v, double* delta_grad, const double* poses0, double* poses,
    int32_t* step, double* loss, double* grad, float lambda0, float lambda1, int32_t anneal_steps,
    double peak_lr, int32_t warmup, int32_t total, double beta1, double beta2, double eps,
    double wd_mlp, double wd_delta, int32_t with_convergence, void* stream);
EPO_API epo_status epo_mlp_step(epo_plan plan, float* params, float* adam_m, float* adam_v,
                        const float* param_grad, double* delta, double* delta_m,
                        double* delta_v, const double* delta_grad, const double* lr,
                        double beta1, double beta2, double eps, double wd_mlp, double wd_delta,
                        int32_t* step, void* stream);

/* ---------------------------------------------------------------------------
 * 4. pose_step
 * Adam on left twists with an SE(3) update, in float64 (optimizer of Sec. 4
 * "Implementation Details" with beta = (0.9, 0.999); the pose refiner network
 * of the paper is replaced by one twist per pose):
 *   s = ++(*step);  for every view v not fixed:
 *   m_v <- b1 m_v + (1 - b1) g_v,  w_v <- b2 w_v + (1 - b2) g_v^2
 *   xi  = -lr[scene(v)] (m_v / (1 - b1^s)) / (sqrt(w_v / (1 - b2^s)) + eps)
 *   P_v <- Exp(xi) P_v   (Rodrigues rotation, left Jacobian for translation)
 *
 *   poses          float64 [V][3][4], updated in place
 *   adam_m/adam_v  float64 [V][6] first / second moments, updated in place
 *   grad           float64 [V][6]
 *   scene_of_view  int32 [V] or NULL (all scene 0)
 *   fixed_mask     uint8 [V] nonzero = pose held fixed, or NULL
 *   lr             float64 [n_scenes] learning rate per scene
 *   step           int32 [1] step counter, incremented on the device
 * No allocation, capture-safe.
 * ------------------------------------------------------------------------- */
EPO_API epo_status epo_pose_step(double* poses, double* adam_m, double* adam_v, const double* grad,
                         int32_t n_views, const int32_t* scene_of_view,
                         const uint8_t* fixed_mask, const double* lr, double beta1,
                         double beta2, double eps, int32_t* step, void* stream);

/* ---------------------------------------------------------------------------
 * Schedules of the paper, evaluated on the device from the step counter (so
 * that a captured iteration needs no host writes between replays):
 *   lambda(s) = lambda0 - (lambda0 - lambda1) min(s, anneal_steps)/anneal_steps
 *     (Alg. 3 AnnealClamp: 10 -> 6 over the first 1000 steps, read as linear)
 *   lr(s) = peak (s + 1)/warmup for s < warmup, else
 *           peak (1 + cos(pi (s - warmup)/(total - warmup)))/2
 *     (Sec. 4: linear warm-up to 3e-3 over 25 steps, cosine decay to N = 2000)
 * with s = *step (the number of pose steps taken so far).  Writes n_scenes
 * copies of each into lambda_out (float32) and lr_out (float64).
 * ------------------------------------------------------------------------- */
EPO_API epo_status epo_schedule(const int32_t* step, int32_t n_scenes, float lambda0, float lambda1,
                        int32_t anneal_steps, double peak_lr, int32_t warmup, int32_t total,
                        float* lambda_out, double* lr_out, void* stream);

/* ---------------------------------------------------------------------------
 * Pose-change signal and dual-phase convergence, per scene, on the device
 * (paper Sec. 3 "Optimization Schedule", Alg. 2, Sec. A1.1):
 *   dR_v = (180/pi) acos((tr(R_v R_v'^T) - 1)/2),
 *   dt_v = (180/pi) acos(t_v . t_v' / (|t_v| |t_v'|))   (' = previous poses),
 *   theta_95 = max(95th percentile of dR, 95th percentile of dt) over the
 *   scene's views (linear interpolation at rank (n - 1) 0.95);
 *   Converged(w, eps): the w moving averages (window w) of theta_95 ending at
 *   the current step are all below eps.
 * Phase 0 -> 1 when Converged(w1, eps1); phase 1 -> 2 (stopped) when
 * Converged(w2, eps2) at a later step; both read the whole history.  In a
 * captured iteration with convergence, a stopped scene gets learning rate 0,
 * so its poses stay where they stopped.
 *   params  (host) windows w1, w2 in [1, 64] and thresholds eps1, eps2 > 0;
 *           NULL = the paper's (25, 0.5, 50, 0.1)
 * epo_convergence_reset stores `poses` as the previous poses and clears the
 * state; epo_convergence_update records one step (theta95 [n_scenes] float64
 * and phase [n_scenes] int32 outputs are optional, device); scenes may have at
 * most 4096 views.  epo_convergence_query copies the state to the host (phase,
 * last theta_95, switch steps [n_scenes][2] (-1 = not yet), steps recorded;
 * any may be NULL) and synchronises `stream`.
 * ------------------------------------------------------------------------- */
typedef struct epo_convergence_params {
    int32_t w1;
    float eps1;
    int32_t w2;
    float eps2;
} epo_convergence_params;

EPO_API epo_status epo_convergence_reset(epo_plan plan, const double* poses,
                                         const epo_convergence_params* params, void* stream);
EPO_API epo_status epo_convergence_update(epo_plan plan, const double* poses, double* theta95,
                                          int32_t* phase, void* stream);
EPO_API epo_status epo_convergence_query(epo_plan plan, int32_t* phase, double* theta_last,
                                         int32_t* switch_steps, int32_t* steps, void* stream);

/* ---------------------------------------------------------------------------
 * One whole iteration captured as a HIP graph owned by the plan:
 *   schedule -> fused cost + adjoint -> float64 reductions -> pose_step
 *   [-> convergence update, when with_convergence != 0; call
 *   epo_convergence_reset before the first replay],
 * recorded graph_steps times in a row (plan option, default 1).  The same
 * arithmetic as the separate calls, with fewer launches: the pair set-up
 * evaluates the schedule, the pose step advances the step counter, and on
 * plans of at most 256 pairs and 64 views the reductions, pose step and step
 * count run as one workgroup (bitwise the same results).
 * The pointers given here are baked into the graph; replays read the current
 * contents of every buffer.  Capturing synchronises `stream` once.
 *   poses, adam_m, adam_v, step   as in epo_pose_step
 *   loss                          float64 [n_scenes], written each replay
 *   grad                          float64 [V][6] scratch/result of each replay
 *   fixed_mask                    uint8 [V] or NULL
 *   schedule constants            as in epo_schedule
 *   with_convergence              0: no test; 1: the test, a stopped scene
 *                                 gets learning rate 0 (its cost is still
 *                                 evaluated); 2: as 1, and from the replay
 *                                 after a scene stops its tiles are left out
 *                                 of the fused launch (device-side early exit:
 *                                 the launch's tile list is compacted on the
 *                                 device, as with pair sub-sampling); its
 *                                 loss entry keeps the value of its last
 *                                 evaluated step, its gradient rows read 0.
 *                                 Poses, phases and the other scenes' results
 *                                 are bitwise those of mode 1.  Other values:
 *                                 EPO_ERR_INVALID_ARG.
 * epo_iteration_launch replays it on `stream` (any stream of the device):
 * graph_steps iterations per call.
 * ------------------------------------------------------------------------- */
EPO_API epo_status epo_iteration_capture(epo_plan plan, double* poses, double* adam_m, double* adam_v,
                                 int32_t* step, double* loss, double* grad,
                                 const uint8_t* fixed_mask, float lambda0, float lambda1,
                                 int32_t anneal_steps, double peak_lr, int32_t warmup,
                                 int32_t total, double beta1, double beta2, double eps,
                                 int32_t with_convergence, void* stream);
EPO_API epo_status epo_iteration_launch(epo_plan plan, void* stream);

/* ---------------------------------------------------------------------------
 * Autotuner: times every supported schedule (texture format, points per
 * thread, tile order, launch style, record order) on the plan's own data at
 * `poses` with `iters` fused cost+adjoint evaluations each, keeps the fastest,
 * and returns it in *chosen (host, may be NULL).  Record order 2 is charged
 * its per-step share of the re-sort (a full re-sort / resort_interval) and
 * is kept only if it beats the best record-order-1 schedule by 3 %; the
 * record copies are freed unless it is chosen.  The resort_interval in force
 * is kept.  Allocates and synchronises; call it before capturing an
 * iteration.
 * ------------------------------------------------------------------------- */
EPO_API epo_status epo_plan_autotune(epo_plan plan, const double* poses, const float* lambda,
                             int32_t iters, epo_plan_options* chosen, void* stream);

/* Switch the plan to a given schedule (rebuilds the tile schedule; allocates;
 * synchronises).  Invalidates a captured iteration. */
EPO_API epo_status epo_plan_set_options(epo_plan plan, const epo_plan_options* options, void* stream);

/* ---------------------------------------------------------------------------
 * Re-sort the per-pair record copies of record_order 2 at `poses` (device,
 * float64 [V][3][4]): every chunk of 8192 records if `step` is NULL, else the
 * chunks c with c mod every == (*step) mod every, *step read on the device
 * when the work runs (so a captured call follows the step counter).  Each
 * chunk is ordered by the target pixel block its records project to, invalid
 * projections last, equal blocks in source order: a deterministic function of
 * the poses.  A no-op under record_order 1.  The fused kernel's results change
 * only in summation order.  No allocation, no synchronisation; capture-safe.
 * Errors: EPO_ERR_INVALID_ARG for a null plan or poses, or every < 1 with a
 * step.
 * ------------------------------------------------------------------------- */
EPO_API epo_status epo_plan_resort(epo_plan plan, const double* poses, const int32_t* step,
                                   int32_t every, void* stream);

/* The records pair d reads, in the order it reads them (host copy; syncs the
 * device): its own sorted copy under record_order 2, else its source view's
 * records.  *count = the source's edge count; records_out may be NULL to ask
 * for the count only.  EPO_ERR_INVALID_ARG if d is out of range or capacity
 * is too small. */
EPO_API epo_status epo_plan_pair_records(epo_plan plan, int32_t d, uint64_t* records_out,
                                         int64_t capacity, int64_t* count);

/* Device status word of the plan, OR-ed by the kernels: bit 0 = a non-finite
 * per-pair sum was seen, bit 1 = a lambda outside [0, lambda_max] was seen, bit 2 = a
 * refined focal length or depth was not finite (or a focal length <= 0).  Copies
 * to *flags (host) after synchronising `stream`, then clears the word. */
EPO_API epo_status epo_get_device_status(epo_plan plan, int32_t* flags, void* stream);

/* Duration in milliseconds of the fused cost+adjoint kernel in the most recent
 * eager epo_edge_cost_fwd / epo_edge_cost_bwd / epo_edge_cost_refine call,
 * measured with HIP events recorded around that kernel on the stream it ran
 * on.  Synchronises on the end event.  Requires epo_plan_enable_timing(plan,
 * 1) beforehand.  A captured iteration records no events (its replays are not
 * timed by this). */
EPO_API epo_status epo_plan_enable_timing(epo_plan plan, int32_t enable);
EPO_API epo_status epo_plan_last_kernel_ms(epo_plan plan, float* ms);

/* Mean duration in milliseconds (*ms, host) of the fused cost+adjoint kernel
 * of the plan's current schedule: the pair descriptors are set up once at
 * `poses` and `lambda` (device, as for epo_edge_cost_fwd), then `reps`
 * back-to-back launches of the kernel are captured as one HIP graph (launched
 * as a captured iteration launches it), replayed once to warm up and once
 * between two HIP events on `stream`; the elapsed time over reps is the
 * per-launch mean, with no other kernel between the launches.  Overwrites the
 * plan's per-tile partial sums (call epo_edge_cost_fwd again before reading
 * per-pair results).  Allocates the graph and two events and synchronises.
 * Errors: EPO_ERR_INVALID_ARG for a null argument or reps outside [1, 100000]. */
EPO_API epo_status epo_plan_time_kernel(epo_plan plan, const double* poses, const float* lambda,
                                        int32_t reps, float* ms, void* stream);

/* Thread-local description of the last error (empty string if none). */
EPO_API const char* epo_last_error(void);

/* Library version string. */
EPO_API const char* epo_version(void);

#ifdef __cplusplus
}
#endif

#endif /* EPO_H */
