// Host-side argument validation of libepo's C-ABI, for a build whose host code
// is compiled with AddressSanitizer and UndefinedBehaviorSanitizer (see
// paper_2607_00579_amd/build.py, build_host_check).  Every call below is
// rejected on the host before any device work, so the program needs no GPU;
// it exits 0 when each call returns the expected status and names the
// offending argument in epo_last_error(), and a sanitizer report makes it
// fail.
#include <cmath>
#include <cstdint>
#include <cstdio>
#include <cstring>
#include <string>
#include <vector>

#include "epo.h"

static int g_failures = 0;

static void expect(const char* what, epo_status got, epo_status want, const char* needle) {
    const char* msg = epo_last_error();
    const bool ok = got == want && (!needle || (msg && std::strstr(msg, needle)));
    if (!ok) {
        std::fprintf(stderr, "FAIL %s: status %d (want %d), message \"%s\" (want \"%s\")\n", what,
                     (int)got, (int)want, msg ? msg : "", needle ? needle : "");
        ++g_failures;
    }
}

struct PlanArgs {
    int32_t n_views = 2;
    std::vector<int32_t> width{40, 40}, height{30, 30};
    std::vector<float> K{32, 32, 19.5f, 14.5f, 32, 32, 19.5f, 14.5f};
    std::vector<int32_t> scene{0, 0};
    std::vector<int64_t> offset{0, 1200};
    std::vector<int32_t> pairs{0, 1, 1, 0};
    int32_t n_pairs = 2;
    // placeholders: never dereferenced, every call fails before device work
    const uint8_t* edges = reinterpret_cast<const uint8_t*>(1);
    const float* depth = reinterpret_cast<const float*>(1);
    const int32_t* d2 = reinterpret_cast<const int32_t*>(1);
    epo_cost_params params{1.0f, 1e-4f, 0, 10.0f};
    epo_plan_options options{0, 0, 0, 0, 0, 0};
    bool with_params = false, with_options = false;

    epo_status create() {
        epo_plan plan = nullptr;
        const epo_status s = epo_plan_create(
            &plan, n_views, width.data(), height.data(), K.data(), scene.data(), offset.data(),
            edges, depth, d2, pairs.data(), n_pairs, with_params ? &params : nullptr,
            with_options ? &options : nullptr, nullptr);
        if (plan) epo_plan_destroy(plan);
        return s;
    }
};

int main() {
    // distance transform
    expect("edt null", epo_build_distance_fields(nullptr, nullptr, nullptr, nullptr, 3, nullptr,
                                                 nullptr, nullptr),
           EPO_ERR_INVALID_ARG, "null");
    {
        const int32_t w[1] = {20000}, h[1] = {5};
        const int64_t off[1] = {0};
        expect("edt side", epo_build_distance_fields(reinterpret_cast<const uint8_t*>(1), off, w, h,
                                                     1, reinterpret_cast<int32_t*>(1),
                                                     reinterpret_cast<float*>(1), nullptr),
               EPO_ERR_INVALID_ARG, "side");
    }
    expect("edt empty", epo_build_distance_fields(nullptr, nullptr, nullptr, nullptr, 0, nullptr,
                                                  nullptr, nullptr),
           EPO_OK, nullptr);

    // plan creation: shapes, indices, scenes, intrinsics, offsets, options
    {
        PlanArgs a;
        a.width[1] = 1;
        expect("plan width 1", a.create(), EPO_ERR_INVALID_ARG, "side");
    }
    {
        PlanArgs a;
        a.width[1] = 16385;
        expect("plan width 16385", a.create(), EPO_ERR_INVALID_ARG, "side");
    }
    {
        PlanArgs a;
        a.pairs = {0, 2, 1, 0};
        expect("plan pair index", a.create(), EPO_ERR_INVALID_ARG, "out of range");
    }
    {
        PlanArgs a;
        a.scene = {0, 1};
        expect("plan cross-scene pair", a.create(), EPO_ERR_INVALID_ARG, "different scenes");
    }
    {
        PlanArgs a;
        a.scene = {0, 2};
        a.pairs = {0, 0, 1, 1};
        expect("plan scene gap", a.create(), EPO_ERR_INVALID_ARG, "without gaps");
    }
    {
        PlanArgs a;
        a.K[4] = -1.0f;
        expect("plan focal", a.create(), EPO_ERR_INVALID_ARG, "focal");
    }
    {
        PlanArgs a;
        a.offset[1] = -5;
        expect("plan offset", a.create(), EPO_ERR_INVALID_ARG, "negative offset");
    }
    {
        PlanArgs a;
        a.n_views = 0;
        expect("plan no views", a.create(), EPO_ERR_INVALID_ARG, "n_views");
    }
    {
        PlanArgs a;
        a.edges = nullptr;
        expect("plan null edges", a.create(), EPO_ERR_INVALID_ARG, "null");
    }
    {
        PlanArgs a;
        a.with_params = a.with_options = true;
        a.params.lambda_max = 20.0f;
        a.options = epo_plan_options{2, 4, 1, 2, 0, 0};
        expect("plan u8 taps above 14.5", a.create(), EPO_ERR_UNSUPPORTED, "lambda_max");
    }
    {
        PlanArgs a;
        a.with_options = true;
        a.options = epo_plan_options{4, 4, 1, 2, 0, 0};
        expect("plan format 4", a.create(), EPO_ERR_INVALID_ARG, "texture_format");
        a.options = epo_plan_options{1, 3, 1, 2, 0, 0};
        expect("plan 3 points per thread", a.create(), EPO_ERR_INVALID_ARG, "points_per_thread");
        a.options = epo_plan_options{1, 4, 1, 2, 3, 0};
        expect("plan record order 3", a.create(), EPO_ERR_INVALID_ARG, "record_order");
        a.options = epo_plan_options{1, 4, 1, 2, 2, -1};
        expect("plan resort interval", a.create(), EPO_ERR_INVALID_ARG, "resort_interval");
        a.options = epo_plan_options{1, 4, 1, 2, 1, 8, 65};
        expect("plan graph steps", a.create(), EPO_ERR_INVALID_ARG, "graph_steps");
    }
    for (const float zmin : {0.0f, -1.0f, 1e-9f, 1e7f, std::nanf("")}) {
        PlanArgs a;
        a.with_params = true;
        a.params.z_min = zmin;
        expect("plan z_min", a.create(), EPO_ERR_INVALID_ARG, "z_min");
    }

    // per-iteration calls without a plan
    expect("fwd", epo_edge_cost_fwd(nullptr, nullptr, nullptr, nullptr, nullptr, nullptr, nullptr,
                                    nullptr, nullptr),
           EPO_ERR_INVALID_ARG, "null plan");
    expect("bwd", epo_edge_cost_bwd(nullptr, nullptr, nullptr, nullptr, nullptr, nullptr),
           EPO_ERR_INVALID_ARG, "null plan");
    expect("pose step", epo_pose_step(nullptr, nullptr, nullptr, nullptr, 2, nullptr, nullptr,
                                      nullptr, 0.9, 0.999, 1e-8, nullptr, nullptr),
           EPO_ERR_INVALID_ARG, nullptr);
    expect("refinement", epo_plan_set_refinement(nullptr, nullptr, nullptr, nullptr, nullptr),
           EPO_ERR_INVALID_ARG, "null plan");
    expect("refine", epo_edge_cost_refine(nullptr, nullptr, nullptr, nullptr, nullptr, nullptr,
                                          nullptr, nullptr, nullptr, nullptr),
           EPO_ERR_INVALID_ARG, nullptr);
    expect("joint step", epo_joint_step(nullptr, nullptr, nullptr, nullptr, nullptr, nullptr,
                                        nullptr, nullptr, nullptr, nullptr, nullptr, nullptr,
                                        nullptr, 0.9, 0.999, 1e-8, 0.01, 0.01, nullptr, nullptr),
           EPO_ERR_INVALID_ARG, "null plan");
    expect("resort", epo_plan_resort(nullptr, nullptr, nullptr, 1, nullptr), EPO_ERR_INVALID_ARG,
           "null");
    {
        int64_t n = 0;
        expect("pair records", epo_plan_pair_records(nullptr, 0, nullptr, 0, &n),
               EPO_ERR_INVALID_ARG, "null");
    }
    expect("set options", epo_plan_set_options(nullptr, nullptr, nullptr), EPO_ERR_INVALID_ARG,
           "null");
    expect("autotune", epo_plan_autotune(nullptr, nullptr, nullptr, 1, nullptr, nullptr),
           EPO_ERR_INVALID_ARG, "null");
    expect("launch", epo_iteration_launch(nullptr, nullptr), EPO_ERR_INVALID_ARG, "null plan");

    // viewgraph: a candidate out of range; staging beyond the static array
    {
        const int32_t w[3] = {16384, 16384, 16384};
        const float K[12] = {1000, 1000, 8191.5f, 8191.5f, 1000, 1000, 8191.5f, 8191.5f,
                             1000, 1000, 8191.5f, 8191.5f};
        const int64_t off[3] = {0, int64_t(16384) * 16384, int64_t(2) * 16384 * 16384};
        const int32_t bad[2] = {0, 3};
        const float* depth = reinterpret_cast<const float*>(1);
        const double* poses = reinterpret_cast<const double*>(1);
        int32_t* cnt = reinterpret_cast<int32_t*>(1);
        expect("viewgraph candidate", epo_build_viewgraph(3, w, w, K, off, depth, poses, bad, 1, 4,
                                                          3.0, 0.125, 1e-4, cnt, cnt, nullptr,
                                                          nullptr),
               EPO_ERR_INVALID_ARG, "out of range");
        const int32_t cand[6] = {0, 1, 0, 2, 1, 2};
        expect("viewgraph staging", epo_build_viewgraph_noalloc(3, w, w, K, off, depth, poses, cand,
                                                                3, 1, 3.0, 0.125, 1e-4, cnt, cnt,
                                                                nullptr, nullptr),
               EPO_ERR_INVALID_ARG, "no-allocation");
    }

    if (g_failures) {
        std::fprintf(stderr, "%d check(s) failed\n", g_failures);
        return 1;
    }
    std::printf("abi host checks passed\n");
    return 0;
}
