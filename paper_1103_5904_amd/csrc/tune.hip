// Launch autotuner.
//
// The best launch shape depends on the geometry: pixels per voxel decide
// how many rays share a voxel block, the cube side how long the walks are,
// the view count how much work one owner of a block gets.  The autotuner
// times every candidate on the caller's geometry with synthetic data (all
// ones: the walks are what costs, and zero pixels would be skipped), keeps
// the fastest P shape and the fastest P^T strategy and shape, and files them
// under the geometry's size class: the cube side, the pixels per view and
// the view count, each rounded up to a power of two, and whether the cube has
// frames.  Every later launch on a geometry of the same class uses that
// entry (tuning_for); other classes keep the process-wide tuning.
//
// Candidates: P - the four wavefront bundles x XCD remap on/off; P^T - the
// owner-computes strategy over seven block shapes (flat to cubic), two owner
// counts and the XCD remap on/off, the LDS-binned strategy over three
// bundles, and the atomic one.
// The workgroup size is not searched (every kernel is built for 256 lanes,
// four wavefronts), nor is the cube layout (x fastest is the ABI's).
#include <math.h>

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

}  // namespace tomo

using namespace tomo;

extern "C" {

int tomo_autotune(const tomo_geometry *g, int32_t reps, tomo_tuning *out, tomo_stream stream)
{
    if (reps < 1 || reps > 100) return set_error(TOMO_EINVAL, "tomo_autotune: reps must be in [1, 100]");
    int st = TOMO_OK;
    PlanRef plan = get_plan(g, &st);
    if (!plan) return st;
    const Plan &p = *plan;
    hipStream_t s = (hipStream_t)stream;
    const int64_t nvox = p.grid.nvox * p.grid.nframes;

    // candidates
    const tomo_tuning base = current_tuning();
    std::vector<tomo_tuning> pc, bc;
    for (int bun : {0, 2, 3, 4})
        for (int xr : {0, 1}) {
            tomo_tuning t = base;
            t.p_bundle = bun;
            t.p_xcd_remap = xr;
            pc.push_back(t);
        }
    // flat blocks suit lines of sight near one plane (solar observers near the
    // ecliptic); cubic ones suit views from all directions
    const int blocks[7][3] = {{64, 32, 2}, {64, 64, 1}, {64, 16, 4}, {32, 32, 4},
                              {32, 16, 8}, {16, 32, 8}, {16, 16, 16}};
    for (const auto &b : blocks)
        for (int sp : {0, 8})
            for (int xr : {0, 1}) {  // (the blocked kernel takes no bundle shape)
                tomo_tuning t = base;
                t.bp_default = TOMO_BP_BLOCKED;
                t.bp_block[0] = b[0];
                t.bp_block[1] = b[1];
                t.bp_block[2] = b[2];
                t.bp_splits = sp;
                t.bp_xcd_remap = xr;
                bc.push_back(t);
            }
    if (p.grid.nvox < ((int64_t)1 << 30)) {  // the atomic strategies' frame limit
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

    // synthetic operands and the largest scratch any candidate (or the
    // current tuning) needs
    size_t scratch_bytes = blocked_scratch_bytes(p, blocked_shape(p, base));
    for (const auto &t : bc) {
        const size_t b = blocked_scratch_bytes(p, blocked_shape(p, t));
        scratch_bytes = b > scratch_bytes ? b : scratch_bytes;
    }
    float *cube = nullptr, *img = nullptr;
    void *scratch = nullptr;
    if (hipMallocAsync((void **)&cube, sizeof(float) * (size_t)nvox, s) != hipSuccess ||
        hipMallocAsync((void **)&img, sizeof(float) * (size_t)p.npix, s) != hipSuccess ||
        hipMallocAsync(&scratch, scratch_bytes, s) != hipSuccess) {
        if (cube) (void)hipFreeAsync(cube, s);
        if (img) (void)hipFreeAsync(img, s);
        return set_error(TOMO_ENOMEM, "tomo_autotune: device allocation failed");
    }
    struct Release {
        hipStream_t s;
        void *a, *b, *c;
        ~Release()
        {
            (void)hipFreeAsync(a, s);
            (void)hipFreeAsync(b, s);
            (void)hipFreeAsync(c, s);
        }
    } release{s, cube, img, scratch};
    int rc = launch_fill(cube, nvox, 1.0f, s);
    if (!rc) rc = launch_fill(img, p.npix, 1.0f, s);
    if (rc) return rc;

    Timer tm;
    if (!tm.a || !tm.b) return set_error(TOMO_EHIP, "tomo_autotune: event creation failed");
    auto time_it = [&](auto &&launch, float &ms) -> int {
        int e = launch();  // warm-up
        for (int k = 0; k < reps && !e; ++k) {
            if (k == 0) e = hip_fail(hipEventRecord(tm.a, s), "event record");
            if (!e) e = launch();
        }
        if (!e) e = hip_fail(hipEventRecord(tm.b, s), "event record");
        if (!e) e = hip_fail(hipEventSynchronize(tm.b), "event synchronise");
        if (!e) e = hip_fail(hipEventElapsedTime(&ms, tm.a, tm.b), "event time");
        return e;
    };
    // bring the clocks up before anything is timed: the current tuning's P
    // (and P^T, unless this geometry refuses its strategy) repeated for at
    // least 30 ms; then the current tuning is the one to beat, by at least 2%
    // (differences below that are within the timing noise)
    const tomo_tuning base_b = base.bp_default != TOMO_BP_BLOCKED && p.grid.nvox >= ((int64_t)1 << 30)
                                   ? bc.front()  // a blocked candidate: the atomic strategies refuse this frame
                                   : base;
    float best_p = INFINITY, best_b = INFINITY;
    tomo_tuning win = base;
    {
        float warm = 0.f, a = 0.f, b = 0.f;
        for (int k = 0; k < 64 && warm < 30.f; ++k) {
            rc = time_it([&] { return launch_project_tuned(p, g, cube, img, true, s, nullptr, base); }, a);
            if (!rc)
                rc = time_it([&] {
                    return launch_backproject_tuned(p, g, img, cube, false, true, base_b.bp_default, s, nullptr,
                                                    scratch, scratch_bytes, base_b);
                }, b);
            if (rc) return rc;
            warm += a + b;
        }
        best_p = 0.98f * a;
        if (base_b.bp_default == base.bp_default) best_b = 0.98f * b;  // else a candidate must set it
    }
    for (const auto &t : pc) {
        float ms = 0.f;
        rc = time_it([&] { return launch_project_tuned(p, g, cube, img, true, s, nullptr, t); }, ms);
        if (rc) return rc;
        if (ms < best_p) {
            best_p = ms;
            win.p_bundle = t.p_bundle;
            win.p_xcd_remap = t.p_xcd_remap;
        }
    }
    for (const auto &t : bc) {
        float ms = 0.f;
        rc = time_it([&] {
            return launch_backproject_tuned(p, g, img, cube, false, true, t.bp_default, s, nullptr, scratch,
                                            scratch_bytes, t);
        }, ms);
        if (rc) return rc;
        if (ms < best_b) {
            best_b = ms;
            win.bp_default = t.bp_default;
            win.bp_bundle = t.bp_bundle;
            win.bp_xcd_remap = t.bp_xcd_remap;
            win.bp_block[0] = t.bp_block[0];
            win.bp_block[1] = t.bp_block[1];
            win.bp_block[2] = t.bp_block[2];
            win.bp_splits = t.bp_splits;
            win.bp_lds_bins = t.bp_lds_bins;
        }
    }
    {
        std::lock_guard<std::mutex> lock(g_class_mu);
        g_class_tuning[p.size_class] = win;
    }
    if (out) *out = win;
    return TOMO_OK;
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
