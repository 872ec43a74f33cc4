// Launch autotuner.
//
// The best launch shape depends on the geometry: pixels per voxel decide
// how many rays share a voxel block, the cube side how long the walks are
// and how far they stray from the caches, the view count how much work one
// owner of a block gets.  The autotuner times the candidates on the caller's
// geometry and data (or, without data, on a cube of ones and its own
// projection, whose zero pattern is the real one: masked pixels and rays
// that miss the box are 0), through the same launch paths the library's
// calls take (scratch from the library's pool included), and files the
// winners under the geometry's size class: the cube side, the pixels per view
// and the view count, each rounded up to a power of two, and whether the
// cube has frames.  Every later launch on a geometry of the same class uses
// that entry (tuning_for); other classes keep the process-wide tuning.
//
// Candidates: P - the four wavefront bundles x XCD remap on/off x the cube
// layouts (x-fastest, bricks of 4, 8 and 16 voxels a side); P^T - the
// owner-computes strategy over block shapes for workgroups of 256, 512 and
// 1024 lanes (larger workgroups own larger blocks, so a ray is set up for
// fewer of them), two owner counts and the XCD remap on/off, the LDS-binned
// strategy over three bundles, and the atomic one.  The blocked candidates
// read a ray table when the tuning asks for one (as the solves do).
//
// Each candidate is screened over `reps` launches; the fastest P and P^T
// candidates are then timed against the process-wide tuning in alternation
// (five rounds, medians), and a candidate is kept only if it beats that
// tuning there by 1%: the tuner never files a pick slower than the default.
#include <math.h>

#include <algorithm>
#include <map>
#include <mutex>
#include <vector>

#include "common.h"

namespace tomo {

namespace {

std::mutex g_class_mu;
std::map<uint64_t, tomo_tuning> g_class_tuning;

uint64_t ceil_log2(uint64_t v)
{
    uint64_t k = 0;
    while (((uint64_t)1 << k) < v && k < 63) ++k;
    return k;
}

struct Timer {
    hipEvent_t a = nullptr, b = nullptr;
    Timer()
    {
        (void)hipEventCreate(&a);
        (void)hipEventCreate(&b);
    }
    ~Timer()
    {
        if (a) (void)hipEventDestroy(a);
        if (b) (void)hipEventDestroy(b);
    }
};

// Block shapes per workgroup size: flat ones suit lines of sight near one
// plane (solar observers near the ecliptic), cubic ones views from all
// directions.  The bins take 8 bytes per voxel of the LDS a workgroup has.
struct Shape {
    int nt, b[3];
};
const Shape kShapes[] = {
    {256, {64, 32, 2}},  {256, {64, 64, 1}},  {256, {64, 16, 4}},  {256, {32, 32, 4}},  {256, {32, 16, 8}},
    {256, {16, 32, 8}},  {256, {16, 16, 16}}, {512, {64, 64, 2}},  {512, {128, 32, 2}}, {512, {64, 32, 4}},
    {512, {32, 32, 8}},  {512, {16, 16, 32}}, {512, {128, 64, 1}}, {1024, {128, 64, 2}}, {1024, {64, 64, 4}},
    {1024, {128, 128, 1}}, {1024, {32, 32, 16}},
};

}  // namespace

uint64_t size_class_of(const tomo_geometry *g, int64_t npix)
{
    const tomo_cube &c = g->cube;
    int32_t nmax = c.nx > c.ny ? c.nx : c.ny;
    nmax = nmax > c.nz ? nmax : c.nz;
    const uint64_t per_view = (uint64_t)(npix / (g->nviews > 0 ? g->nviews : 1));
    return ceil_log2((uint64_t)nmax) | (ceil_log2(per_view ? per_view : 1) << 8) |
           (ceil_log2((uint64_t)g->nviews) << 16) | ((uint64_t)(c.nframes > 1) << 24);
}

tomo_tuning tuning_for(const Plan &p)
{
    {
        std::lock_guard<std::mutex> lock(g_class_mu);
        auto it = g_class_tuning.find(p.size_class);
        if (it != g_class_tuning.end()) return it->second;
    }
    return current_tuning();
}

static int autotune_impl(const tomo_geometry *g, const float *cube_in, const float *img_in, int32_t reps,
                         tomo_tuning *out, hipStream_t s)
{
    if (reps < 1 || reps > 100) return set_error(TOMO_EINVAL, "tomo_autotune: reps must be in [1, 100]");
    int st = TOMO_OK;
    PlanRef plan = get_plan(g, &st);
    if (!plan) return st;
    const Plan &p = *plan;
    const int64_t nvox = p.grid.nvox * p.grid.nframes;
    const bool wide = p.grid.nvox >= ((int64_t)1 << 30);  // the atomic strategies refuse such frames

    // candidates
    const tomo_tuning base = current_tuning();
    std::vector<tomo_tuning> pc, bc;
    for (int lay : {0, 2, 3, 4})
        for (int bun : {0, 2, 3, 4})
            for (int xr : {0, 1, 2}) {
                tomo_tuning t = base;
                t.p_bundle = bun;
                t.p_xcd_remap = xr;
                t.p_layout = lay;
                pc.push_back(t);
            }
    for (const Shape &sh : kShapes)
        for (int sp : {0, 8})
            for (int xr : {0, 1, 2}) {  // (the blocked kernel takes no bundle shape)
                tomo_tuning t = base;
                t.bp_default = TOMO_BP_BLOCKED;
                t.bp_threads = sh.nt;
                t.bp_block[0] = sh.b[0];
                t.bp_block[1] = sh.b[1];
                t.bp_block[2] = sh.b[2];
                t.bp_splits = sp;
                t.bp_xcd_remap = xr;
                const BlockedShape bs = blocked_shape(p, t);
                if (blocked_check_lds(bs, p.bp_rows, nullptr) != TOMO_OK) {
                    (void)set_error(TOMO_OK, "");  // a shape this device cannot hold: not a candidate
                    continue;
                }
                bc.push_back(t);
            }
    if (!wide) {
        for (int bun : {2, 3, 4}) {
            tomo_tuning t = base;
            t.bp_default = TOMO_BP_BINNED;
            t.bp_bundle = bun;
            bc.push_back(t);
        }
        tomo_tuning t = base;
        t.bp_default = TOMO_BP_ATOMIC;
        bc.push_back(t);
    }
    // the process-wide tuning's P^T strategy may refuse this frame: then
    // the first blocked candidate stands in for it
    const tomo_tuning base_b = base.bp_default != TOMO_BP_BLOCKED && wide ? bc.front() : base;

    // operands: the caller's, or a cube of ones and its projection
    float *cube = nullptr, *img = nullptr;
    if (!cube_in || !img_in) {
        if (scratch_alloc((void **)&cube, sizeof(float) * (size_t)nvox, s) != hipSuccess ||
            scratch_alloc((void **)&img, sizeof(float) * (size_t)p.npix, s) != hipSuccess) {
            (void)scratch_free(cube, s);
            return set_error(TOMO_ENOMEM, "tomo_autotune: device allocation failed");
        }
    }
    struct Release {
        hipStream_t s;
        void *a, *b;
        ~Release()
        {
            (void)scratch_free(a, s);
            (void)scratch_free(b, s);
        }
    } release{s, cube, img};
    const float *xc = cube_in ? cube_in : cube;
    const float *yc = img_in ? img_in : img;
    // the work buffers the candidates write into: the image and the cube of
    // the synthetic operands are refilled after the candidates have run
    float *img_w = nullptr, *cube_w = nullptr;
    if (scratch_alloc((void **)&img_w, sizeof(float) * (size_t)p.npix, s) != hipSuccess ||
        scratch_alloc((void **)&cube_w, sizeof(float) * (size_t)nvox, s) != hipSuccess) {
        (void)scratch_free(img_w, s);
        return set_error(TOMO_ENOMEM, "tomo_autotune: device allocation failed");
    }
    Release release_w{s, img_w, cube_w};
    int rc = TOMO_OK;
    if (!cube_in || !img_in) {
        rc = launch_fill(cube, nvox, 1.0f, s);
        if (!rc) rc = launch_project_with(p, g, cube, img, true, s, base);
        if (rc) return rc;
    }

    // the blocked candidates read a ray table, as the solves they serve do
    RayTable tab;
    void *tab_mem = nullptr;
    const size_t tab_bytes = base.bp_ray_table ? ray_table_bytes(p) : 0;
    if (tab_bytes && scratch_alloc(&tab_mem, tab_bytes, s) != hipSuccess)
        return set_error(TOMO_ENOMEM, "tomo_autotune: device allocation failed");
    Release release_t{s, tab_mem, nullptr};
    if (tab_mem) {
        rc = ray_table_build(p, tab_mem, tab, s);
        if (rc) return rc;
    }

    Timer tm;
    if (!tm.a || !tm.b) return set_error(TOMO_EHIP, "tomo_autotune: event creation failed");
    // ms per launch over n launches after one untimed one
    auto time_it = [&](auto &&launch, int n, float &ms) -> int {
        int e = launch();
        if (!e) e = hip_fail(hipEventRecord(tm.a, s), "event record");
        for (int k = 0; k < n && !e; ++k) e = launch();
        if (!e) e = hip_fail(hipEventRecord(tm.b, s), "event record");
        if (!e) e = hip_fail(hipEventSynchronize(tm.b), "event synchronise");
        if (!e) e = hip_fail(hipEventElapsedTime(&ms, tm.a, tm.b), "event time");
        ms /= (float)n;
        return e;
    };
    auto run_p = [&](const tomo_tuning &t) { return launch_project_with(p, g, xc, img_w, true, s, t); };
    auto run_b = [&](const tomo_tuning &t) {
        return launch_backproject_tuned(p, g, yc, cube_w, false, true, t.bp_default, s, nullptr, nullptr, 0, t,
                                        tab_mem && t.bp_ray_table ? &tab : nullptr);
    };
    // bring the clocks up before anything is timed: the process-wide
    // tuning's P and P^T repeated for at least 30 ms
    {
        float warm = 0.f, a = 0.f, b = 0.f;
        for (int k = 0; k < 64 && warm < 30.f; ++k) {
            rc = time_it([&] { return run_p(base); }, 1, a);
            if (!rc) rc = time_it([&] { return run_b(base_b); }, 1, b);
            if (rc) return rc;
            warm += a + b;
        }
    }
    // screening
    auto best_of = [&](const std::vector<tomo_tuning> &cands, auto &&run, tomo_tuning &win) -> int {
        float best = INFINITY;
        for (const auto &t : cands) {
            float ms = 0.f;
            const int e = time_it([&] { return run(t); }, reps, ms);
            if (e) return e;
            if (ms < best) {
                best = ms;
                win = t;
            }
        }
        return TOMO_OK;
    };
    tomo_tuning win_p = base, win_b = base_b;
    rc = best_of(pc, run_p, win_p);
    if (!rc) rc = best_of(bc, run_b, win_b);
    if (rc) return rc;
    // confirmation against the process-wide tuning, in alternation: medians
    // of five rounds each; a winner must beat it by 1%
    auto confirm = [&](auto &&run, const tomo_tuning &cand, const tomo_tuning &ref, bool &keep) -> int {
        std::vector<float> tc, tr;
        for (int round = 0; round < 5; ++round) {
            float a = 0.f, b = 0.f;
            int e = time_it([&] { return run(ref); }, reps, a);
            if (!e) e = time_it([&] { return run(cand); }, reps, b);
            if (e) return e;
            tr.push_back(a);
            tc.push_back(b);
        }
        std::sort(tc.begin(), tc.end());
        std::sort(tr.begin(), tr.end());
        keep = tc[2] < 0.99f * tr[2];
        return TOMO_OK;
    };
    bool keep_p = false, keep_b = false;
    rc = confirm(run_p, win_p, base, keep_p);
    if (!rc) {
        if (base_b.bp_default == base.bp_default) rc = confirm(run_b, win_b, base_b, keep_b);
        else keep_b = true;  // the process-wide strategy cannot run here
    }
    if (rc) return rc;
    tomo_tuning win = base;
    if (keep_p) {
        win.p_bundle = win_p.p_bundle;
        win.p_xcd_remap = win_p.p_xcd_remap;
        win.p_layout = win_p.p_layout;
    }
    const tomo_tuning &bsrc = keep_b ? win_b : base_b;
    win.bp_default = bsrc.bp_default;
    win.bp_bundle = bsrc.bp_bundle;
    win.bp_xcd_remap = bsrc.bp_xcd_remap;
    win.bp_block[0] = bsrc.bp_block[0];
    win.bp_block[1] = bsrc.bp_block[1];
    win.bp_block[2] = bsrc.bp_block[2];
    win.bp_splits = bsrc.bp_splits;
    win.bp_lds_bins = bsrc.bp_lds_bins;
    win.bp_threads = bsrc.bp_threads;
    {
        std::lock_guard<std::mutex> lock(g_class_mu);
        g_class_tuning[p.size_class] = win;
    }
    if (out) *out = win;
    return hip_fail(hipStreamSynchronize(s), "tomo_autotune: synchronise");
}

}  // namespace tomo

using namespace tomo;

extern "C" {

int tomo_autotune(const tomo_geometry *g, int32_t reps, tomo_tuning *out, tomo_stream stream)
{
    return autotune_impl(g, nullptr, nullptr, reps, out, (hipStream_t)stream);
}

int tomo_autotune_data(const tomo_geometry *g, const float *cube_d, const float *images_d, int32_t reps,
                       tomo_tuning *out, tomo_stream stream)
{
    if (!cube_d || !images_d) return set_error(TOMO_EINVAL, "tomo_autotune_data: NULL array");
    return autotune_impl(g, cube_d, images_d, reps, out, (hipStream_t)stream);
}

int tomo_get_class_tuning(const tomo_geometry *g, tomo_tuning *out, int32_t *tuned)
{
    if (!out) return set_error(TOMO_EINVAL, "tomo_get_class_tuning: out is NULL");
    int st = TOMO_OK;
    PlanRef plan = get_plan(g, &st);
    if (!plan) return st;
    bool found = false;
    {
        std::lock_guard<std::mutex> lock(g_class_mu);
        auto it = g_class_tuning.find(plan->size_class);
        if (it != g_class_tuning.end()) {
            *out = it->second;
            found = true;
        }
    }
    if (!found) *out = current_tuning();
    if (tuned) *tuned = found ? 1 : 0;
    return TOMO_OK;
}

void tomo_autotune_clear(void)
{
    std::lock_guard<std::mutex> lock(g_class_mu);
    g_class_tuning.clear();
}

}  // extern "C"
