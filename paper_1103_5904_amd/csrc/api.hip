// Host side of libtomo: argument validation, the geometry-keyed cache of
// device view tables, error reporting, WCS pointing, and the projector
// entry points.
#include <math.h>
#include <stdarg.h>
#include <stdio.h>
#include <string.h>

#include <algorithm>
#include <mutex>
#include <string>
#include <unordered_map>
#include <vector>

#include "common.h"

namespace tomo {

static thread_local std::string g_last_error;

// Process-wide launch tuning (see tomo_set_tuning).
static std::mutex g_tuning_mu;
// Defaults measured on MI355X: P with 4x16 bundles and the XCD remap (18%
// faster than without on the EUVI-like 128^3 / 28 x 512^2 problem); P^T
// owner-computes with 512-lane workgroups on 128x32x2 blocks, no remap and
// the automatic owner count.  Solar observers sit near the ecliptic, so
// lines of sight run nearly in the x-y plane and cross few z planes: blocks
// flat in z and long in x are crossed by fewer rays per deposit (per launch:
// 1.27 ms against 1.46 ms for 64x32x2 with 256 lanes on the EUVI-like
// problem, 5.50 against 6.65 ms on a COR1-like frame).  The binned strategy,
// which alone takes the bundle field, prefers 8x8 bundles and 4096 bins.
static tomo_tuning g_tuning = {2, 1, 3, 0, 4096, TOMO_BP_BLOCKED, {128, 32, 2}, 0, 512, 0, 1};

tomo_tuning current_tuning()
{
    std::lock_guard<std::mutex> lock(g_tuning_mu);
    return g_tuning;
}

int set_error(int status, const char *fmt, ...)
{
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_last_error = buf;
    return status;
}

int hip_fail(hipError_t e, const char *what)
{
    if (e == hipSuccess) return TOMO_OK;
    return set_error(TOMO_EHIP, "%s: %s", what, hipGetErrorString(e));
}

static bool finite3(const double *v) { return isfinite(v[0]) && isfinite(v[1]) && isfinite(v[2]); }

static double dot3(const double *a, const double *b) { return a[0] * b[0] + a[1] * b[1] + a[2] * b[2]; }

int validate_cube(const tomo_cube *c)
{
    if (!c) return set_error(TOMO_EINVAL, "cube is NULL");
    if (c->nx < 1 || c->ny < 1 || c->nz < 1)
        return set_error(TOMO_EINVAL, "cube dims must be >= 1 (got %d x %d x %d)", c->nx, c->ny, c->nz);
    if (c->nframes < 1) return set_error(TOMO_EINVAL, "nframes must be >= 1 (got %d)", c->nframes);
    if (c->nx > (1 << 24) || c->ny > (1 << 24) || c->nz > (1 << 24))
        return set_error(TOMO_EINVAL, "cube side exceeds 2^24 voxels (got %d x %d x %d)", c->nx, c->ny, c->nz);
    const int64_t nvox = (int64_t)c->nx * c->ny * c->nz;
    if (nvox > (int64_t)1 << 30)
        return set_error(TOMO_EINVAL, "cube of %lld voxels exceeds the 2^30 limit", (long long)nvox);
    for (int a = 0; a < 3; ++a)
        if (!isfinite(c->box_min[a]) || !isfinite(c->box_max[a]) || !(c->box_max[a] > c->box_min[a]))
            return set_error(TOMO_EINVAL, "box bounds on axis %d are invalid", a);
    return TOMO_OK;
}

static int validate_geometry_impl(const tomo_geometry *g, int64_t *npix_out)
{
    if (!g) return set_error(TOMO_EINVAL, "geometry is NULL");
    int rc = validate_cube(&g->cube);
    if (rc) return rc;
    if (g->nviews < 1) return set_error(TOMO_EINVAL, "nviews must be >= 1 (got %d)", g->nviews);
    if (!g->views) return set_error(TOMO_EINVAL, "views is NULL");
    int64_t npix = 0;
    for (int k = 0; k < g->nviews; ++k) {
        const tomo_view &v = g->views[k];
        if (!finite3(v.obs) || !finite3(v.w) || !finite3(v.u) || !finite3(v.v))
            return set_error(TOMO_EINVAL, "view %d: non-finite vector", k);
        const double tol = 1e-6;
        if (fabs(dot3(v.w, v.w) - 1) > tol || fabs(dot3(v.u, v.u) - 1) > tol ||
            fabs(dot3(v.v, v.v) - 1) > tol)
            return set_error(TOMO_EINVAL, "view %d: w, u, v must be unit vectors", k);
        if (fabs(dot3(v.w, v.u)) > tol || fabs(dot3(v.w, v.v)) > tol || fabs(dot3(v.u, v.v)) > tol)
            return set_error(TOMO_EINVAL, "view %d: w, u, v must be orthogonal", k);
        if (!isfinite(v.cdelt[0]) || !isfinite(v.cdelt[1]) || v.cdelt[0] == 0 || v.cdelt[1] == 0)
            return set_error(TOMO_EINVAL, "view %d: cdelt must be finite and non-zero", k);
        if (!isfinite(v.crpix[0]) || !isfinite(v.crpix[1]))
            return set_error(TOMO_EINVAL, "view %d: crpix must be finite", k);
        if (v.ncol < 1 || v.nrow < 1 || v.ncol > 65535 || v.nrow > 65535)
            return set_error(TOMO_EINVAL, "view %d: image size %d x %d is invalid (1..65535 each)", k, v.ncol,
                             v.nrow);
        if (v.frame < 0 || v.frame >= g->cube.nframes)
            return set_error(TOMO_EINVAL, "view %d: frame %d outside [0, %d)", k, v.frame, g->cube.nframes);
        npix += (int64_t)v.ncol * v.nrow;
    }
    if (npix >= (int64_t)1 << 40) return set_error(TOMO_EINVAL, "too many pixels");
    if (g->obstacle) {
        const tomo_obstacle &ob = *g->obstacle;
        if (!finite3(ob.center) || !isfinite(ob.radius) || !(ob.radius > 0.0))
            return set_error(TOMO_EINVAL, "obstacle: centre must be finite and radius finite and > 0");
    }
    if (g->gains)
        for (int k = 0; k < g->nviews; ++k)
            if (!isfinite(g->gains[k])) return set_error(TOMO_EINVAL, "view %d: gain must be finite", k);
    if (npix_out) *npix_out = npix;
    return TOMO_OK;
}

// ------------------------------------------------------------ plan cache

struct CacheEntry {
    std::vector<unsigned char> key;
    std::shared_ptr<Plan> plan;
};

static std::mutex g_cache_mu;
static std::unordered_map<uint64_t, std::vector<CacheEntry>> g_cache;

static uint64_t fnv1a(const unsigned char *p, size_t n, uint64_t h = 1469598103934665603ull)
{
    for (size_t i = 0; i < n; ++i) {
        h ^= p[i];
        h *= 1099511628211ull;
    }
    return h;
}

static std::vector<unsigned char> geometry_key(const tomo_geometry *g)
{
    const tomo_obstacle none = {{0.0, 0.0, 0.0}, 0.0};
    const tomo_obstacle &ob = g->obstacle ? *g->obstacle : none;
    const size_t ng = g->gains ? sizeof(double) * (size_t)g->nviews : 0;
    std::vector<unsigned char> k(sizeof(tomo_cube) + sizeof(int32_t) + sizeof(tomo_obstacle) +
                                 sizeof(tomo_view) * (size_t)g->nviews + 1 + ng);
    unsigned char *q = k.data();
    memcpy(q, &g->cube, sizeof(tomo_cube));
    q += sizeof(tomo_cube);
    memcpy(q, &g->nviews, sizeof(int32_t));
    q += sizeof(int32_t);
    memcpy(q, &ob, sizeof(tomo_obstacle));
    q += sizeof(tomo_obstacle);
    memcpy(q, g->views, sizeof(tomo_view) * (size_t)g->nviews);
    q += sizeof(tomo_view) * (size_t)g->nviews;
    *q++ = g->gains ? 1 : 0;
    if (ng) memcpy(q, g->gains, ng);
    return k;
}

static int build_plan(const tomo_geometry *g, int64_t npix, Plan &p)
{
    const tomo_cube &c = g->cube;
    GridDev &gd = p.grid;
    gd.n[0] = c.nx;
    gd.n[1] = c.ny;
    gd.n[2] = c.nz;
    gd.nframes = c.nframes;
    for (int a = 0; a < 3; ++a) {
        gd.lo[a] = c.box_min[a];
        gd.hi[a] = c.box_max[a];
        gd.delta[a] = (c.box_max[a] - c.box_min[a]) / (double)gd.n[a];
        gd.inv_delta[a] = 1.0 / gd.delta[a];
    }
    gd.nvox = (int64_t)c.nx * c.ny * c.nz;
    gd.has_sph = g->obstacle != nullptr;
    gd.pad = 0;
    for (int a = 0; a < 3; ++a) gd.sph[a] = g->obstacle ? g->obstacle->center[a] : 0.0;
    gd.sph[3] = g->obstacle ? g->obstacle->radius : 0.0;
    std::vector<ViewDev> hv((size_t)g->nviews);
    int64_t pix = 0, tiles = 0;
    for (int k = 0; k < g->nviews; ++k) {
        const tomo_view &v = g->views[k];
        ViewDev &d = hv[(size_t)k];
        for (int a = 0; a < 3; ++a) {
            d.o[a] = v.obs[a];
            d.w[a] = v.w[a];
            d.u[a] = v.u[a];
            d.v[a] = v.v[a];
        }
        d.cd[0] = v.cdelt[0];
        d.cd[1] = v.cdelt[1];
        d.cp[0] = v.crpix[0];
        d.cp[1] = v.crpix[1];
        d.gain = g->gains ? g->gains[k] : 1.0;
        d.ncol = v.ncol;
        d.nrow = v.nrow;
        d.frame = v.frame;
        d.tiles_x = (v.ncol + kTile - 1) / kTile;
        d.pix_off = pix;
        d.tile_off = tiles;
        pix += (int64_t)v.ncol * v.nrow;
        tiles += (int64_t)d.tiles_x * ((v.nrow + kTile - 1) / kTile);
    }
    if (tiles >= ((int64_t)1 << 31)) return set_error(TOMO_EINVAL, "too many pixel tiles");
    p.nviews = g->nviews;
    p.ntiles = tiles;
    p.npix = npix;
    p.max_steps = c.nx + c.ny + c.nz + 3;
    p.max_nrow = 0;
    for (int k = 0; k < g->nviews; ++k) p.max_nrow = g->views[k].nrow > p.max_nrow ? g->views[k].nrow : p.max_nrow;
    p.size_class = size_class_of(g, npix);
    // The blocked P^T's footprint row intervals pay where footprints span
    // several passes of pixels, i.e. where pixels are finer than voxels at the
    // cube: the median over the views of voxel size / pixel size at the cube's
    // centre (measured: 1.8 and up faster with intervals, 0.94 and below
    // faster with whole rectangles).
    {
        std::vector<double> ratio((size_t)g->nviews);
        const double vox = (gd.delta[0] + gd.delta[1] + gd.delta[2]) / 3.0;
        for (int k = 0; k < g->nviews; ++k) {
            const tomo_view &v = g->views[k];
            double d2 = 0.0;
            for (int a = 0; a < 3; ++a) {
                const double t = 0.5 * (gd.lo[a] + gd.hi[a]) - v.obs[a];
                d2 += t * t;
            }
            const double px = sqrt(fabs(v.cdelt[0] * v.cdelt[1])) * sqrt(d2);
            ratio[(size_t)k] = px > 0.0 ? vox / px : 0.0;
        }
        std::nth_element(ratio.begin(), ratio.begin() + ratio.size() / 2, ratio.end());
        p.bp_rows = ratio[ratio.size() / 2] >= 1.4;
    }
    hipError_t e = hipMalloc((void **)&p.views_d, sizeof(ViewDev) * hv.size());
    if (e != hipSuccess) return set_error(TOMO_ENOMEM, "view table allocation: %s", hipGetErrorString(e));
    e = hipMemcpy(p.views_d, hv.data(), sizeof(ViewDev) * hv.size(), hipMemcpyHostToDevice);
    if (e != hipSuccess) return hip_fail(e, "view table upload");
    // views grouped by frame (for owners of a frame's voxel blocks)
    std::vector<int32_t> fv, foff((size_t)c.nframes + 1, 0);
    for (int f = 0; f < c.nframes; ++f) {
        foff[(size_t)f] = (int32_t)fv.size();
        for (int k = 0; k < g->nviews; ++k)
            if (g->views[k].frame == f) fv.push_back(k);
    }
    foff[(size_t)c.nframes] = (int32_t)fv.size();
    p.min_frame_views = g->nviews;
    for (int f = 0; f < c.nframes; ++f) {
        const int32_t nf = foff[(size_t)f + 1] - foff[(size_t)f];
        p.min_frame_views = nf < p.min_frame_views ? nf : p.min_frame_views;
    }
    if (fv.empty()) fv.push_back(0);
    e = hipMalloc((void **)&p.frame_views_d, sizeof(int32_t) * fv.size());
    if (e == hipSuccess) e = hipMalloc((void **)&p.frame_voff_d, sizeof(int32_t) * foff.size());
    if (e != hipSuccess) return set_error(TOMO_ENOMEM, "frame table allocation: %s", hipGetErrorString(e));
    e = hipMemcpy(p.frame_views_d, fv.data(), sizeof(int32_t) * fv.size(), hipMemcpyHostToDevice);
    if (e == hipSuccess)
        e = hipMemcpy(p.frame_voff_d, foff.data(), sizeof(int32_t) * foff.size(), hipMemcpyHostToDevice);
    if (e != hipSuccess) return hip_fail(e, "frame table upload");
    e = hipMalloc((void **)&p.spill_d, sizeof(unsigned));
    if (e != hipSuccess) return set_error(TOMO_ENOMEM, "counter allocation: %s", hipGetErrorString(e));
    e = hipMemset(p.spill_d, 0, sizeof(unsigned));
    if (e != hipSuccess) return hip_fail(e, "counter init");
    return TOMO_OK;
}

PlanRef get_plan(const tomo_geometry *g, int *status, bool build)
{
    int64_t npix = 0;
    int rc = validate_geometry_impl(g, &npix);
    if (rc) {
        *status = rc;
        return nullptr;
    }
    std::vector<unsigned char> key = geometry_key(g);
    const uint64_t h = fnv1a(key.data(), key.size());
    int dev = 0;
    hipGetDevice(&dev);
    const uint64_t hd = h ^ ((uint64_t)dev * 0x9e3779b97f4a7c15ull);
    std::lock_guard<std::mutex> lock(g_cache_mu);
    auto &bucket = g_cache[hd];
    for (auto &e : bucket)
        if (e.key == key) return e.plan;
    if (!build) {
        *status = set_error(TOMO_EINVAL, "this geometry has no device tables yet: make another call with it "
                                         "first (for instance tomo_count_crossings or tomo_backproject)");
        return nullptr;
    }
    if (g_cache.size() > 256) g_cache.clear();  // bound the cache; plans are rebuilt on demand
    CacheEntry ent;
    ent.key = std::move(key);
    ent.plan = std::make_shared<Plan>();
    rc = build_plan(g, npix, *ent.plan);
    if (rc) {
        *status = rc;
        return nullptr;
    }
    PlanRef out = ent.plan;
    g_cache[hd].push_back(std::move(ent));
    return out;
}

}  // namespace tomo

using namespace tomo;

extern "C" {

int tomo_validate_geometry(const tomo_geometry *g) { return validate_geometry_impl(g, nullptr); }

int64_t tomo_geometry_pixels(const tomo_geometry *g)
{
    int64_t n = 0;
    return validate_geometry_impl(g, &n) ? 0 : n;
}

void tomo_release_cache(void)
{
    std::lock_guard<std::mutex> lock(g_cache_mu);
    g_cache.clear();
}

const char *tomo_status_string(int status)
{
    switch (status) {
    case TOMO_OK: return "ok";
    case TOMO_EINVAL: return "invalid argument";
    case TOMO_EHIP: return "HIP runtime error";
    case TOMO_ENONFINITE: return "non-finite value in the solver";
    case TOMO_ENOCONV: return "not converged within max_iter";
    case TOMO_ENOMEM: return "out of memory";
    case TOMO_EUNSUPPORTED: return "unsupported option";
    default: return "unknown status";
    }
}

const char *tomo_last_error(void) { return g_last_error.c_str(); }

int tomo_get_tuning(tomo_tuning *out)
{
    if (!out) return set_error(TOMO_EINVAL, "tomo_get_tuning: out is NULL");
    *out = current_tuning();
    return TOMO_OK;
}

int tomo_set_tuning(const tomo_tuning *in)
{
    if (!in) return set_error(TOMO_EINVAL, "tomo_set_tuning: in is NULL");
    auto bundle_ok = [](int b) { return b == 0 || b == 2 || b == 3 || b == 4; };
    if (!bundle_ok(in->p_bundle) || !bundle_ok(in->bp_bundle))
        return set_error(TOMO_EINVAL, "tomo_set_tuning: bundle must be 0, 2, 3 or 4");
    if (in->p_xcd_remap < 0 || in->p_xcd_remap > 2 || in->bp_xcd_remap < 0 || in->bp_xcd_remap > 2)
        return set_error(TOMO_EINVAL, "tomo_set_tuning: xcd_remap must be 0, 1 or 2");
    if (in->bp_lds_bins < 512 || in->bp_lds_bins > 8192)
        return set_error(TOMO_EINVAL, "tomo_set_tuning: bp_lds_bins must be in [512, 8192]");
    if (in->bp_default != TOMO_BP_BINNED && in->bp_default != TOMO_BP_ATOMIC &&
        in->bp_default != TOMO_BP_BLOCKED)
        return set_error(TOMO_EINVAL, "tomo_set_tuning: bp_default must be BLOCKED, BINNED or ATOMIC");
    for (int a = 0; a < 3; ++a)
        if (in->bp_block[a] < 1 || in->bp_block[a] > 256)
            return set_error(TOMO_EINVAL, "tomo_set_tuning: bp_block entries must be in [1, 256]");
    if (in->bp_block[0] * in->bp_block[1] * in->bp_block[2] > 16384)
        return set_error(TOMO_EINVAL, "tomo_set_tuning: bp_block holds more than 16384 voxels");
    if (in->bp_splits < 0 || in->bp_splits > 64)
        return set_error(TOMO_EINVAL, "tomo_set_tuning: bp_splits must be in [0, 64]");
    if (in->bp_threads != 256 && in->bp_threads != 512 && in->bp_threads != 1024)
        return set_error(TOMO_EINVAL, "tomo_set_tuning: bp_threads must be 256, 512 or 1024");
    if (in->p_layout != 0 && (in->p_layout < 2 || in->p_layout > 4))
        return set_error(TOMO_EINVAL, "tomo_set_tuning: p_layout must be 0, 2, 3 or 4");
    if (in->bp_ray_table != 0 && in->bp_ray_table != 1)
        return set_error(TOMO_EINVAL, "tomo_set_tuning: bp_ray_table must be 0 or 1");
    std::lock_guard<std::mutex> lock(g_tuning_mu);
    g_tuning = *in;
    return TOMO_OK;
}

int tomo_binning_spills(const tomo_geometry *g, int64_t *count_h)
{
    if (!count_h) return set_error(TOMO_EINVAL, "tomo_binning_spills: count_h is NULL");
    int st = TOMO_OK;
    PlanRef p = get_plan(g, &st);
    if (!p) return st;
    unsigned h = 0;
    int rc = hip_fail(hipDeviceSynchronize(), "synchronise");
    if (!rc) rc = hip_fail(hipMemcpy(&h, p->spill_d, sizeof(h), hipMemcpyDeviceToHost), "copy counter");
    if (!rc) rc = hip_fail(hipMemset(p->spill_d, 0, sizeof(unsigned)), "reset counter");
    if (!rc) *count_h = (int64_t)h;
    return rc;
}

int tomo_project(const tomo_geometry *g, const float *cube_d, float *images_d, tomo_stream stream)
{
    if (!cube_d || !images_d) return set_error(TOMO_EINVAL, "tomo_project: NULL array");
    int st = TOMO_OK;
    PlanRef p = get_plan(g, &st);
    if (!p) return st;
    return launch_project(*p, g, cube_d, images_d, true, (hipStream_t)stream);
}

int tomo_backproject_ex(const tomo_geometry *g, const float *images_d, float *cube_d,
                        int accumulate, int strategy, tomo_stream stream)
{
    if (!cube_d || !images_d) return set_error(TOMO_EINVAL, "tomo_backproject: NULL array");
    if (strategy < TOMO_BP_AUTO || strategy > TOMO_BP_BLOCKED)
        return set_error(TOMO_EINVAL, "tomo_backproject: unknown strategy %d", strategy);
    int st = TOMO_OK;
    PlanRef p = get_plan(g, &st);
    if (!p) return st;
    return launch_backproject(*p, g, images_d, cube_d, accumulate != 0, true, strategy,
                              (hipStream_t)stream);
}

int tomo_backproject(const tomo_geometry *g, const float *images_d, float *cube_d, int accumulate,
                     tomo_stream stream)
{
    return tomo_backproject_ex(g, images_d, cube_d, accumulate, TOMO_BP_AUTO, stream);
}

// Helioprojective TAN pointing.  Cube frame: x toward heliographic
// longitude 0 / latitude 0, z toward solar north.  At the observer, S points
// to Sun centre, N is solar north projected perpendicular to S, and
// W = S x N is solar west.  A helioprojective direction (tx, ty) is
// cos(ty) cos(tx) S + cos(ty) sin(tx) W + sin(ty) N.  The detector frame at
// the reference direction w uses the local unit tangent along +ty for v and
// u = w x v along +tx, turned by the image rotation crota.
int tomo_view_from_wcs(double dsun, double hgln_deg, double hglt_deg, double crval1_as,
                       double crval2_as, double crota_deg, double cdelt1_as, double cdelt2_as,
                       double crpix1, double crpix2, int32_t ncol, int32_t nrow, tomo_view *out)
{
    if (!out) return set_error(TOMO_EINVAL, "tomo_view_from_wcs: out is NULL");
    const double in[] = {dsun, hgln_deg, hglt_deg, crval1_as, crval2_as, crota_deg, cdelt1_as,
                         cdelt2_as, crpix1, crpix2};
    for (double x : in)
        if (!isfinite(x)) return set_error(TOMO_EINVAL, "tomo_view_from_wcs: non-finite keyword");
    if (!(dsun > 0) || cdelt1_as == 0 || cdelt2_as == 0 || ncol < 1 || nrow < 1)
        return set_error(TOMO_EINVAL, "tomo_view_from_wcs: invalid distance, scale or size");
    const double deg = M_PI / 180.0, arcsec = deg / 3600.0;
    const double lon = hgln_deg * deg, lat = hglt_deg * deg;
    const double cl = cos(lat);
    double obs[3] = {dsun * cl * cos(lon), dsun * cl * sin(lon), dsun * sin(lat)};
    double S[3] = {-cl * cos(lon), -cl * sin(lon), -sin(lat)};
    double N[3] = {-S[2] * S[0], -S[2] * S[1], 1.0 - S[2] * S[2]};
    const double nn = sqrt(dot3(N, N));
    for (double &x : N) x /= nn;
    const double W[3] = {S[1] * N[2] - S[2] * N[1], S[2] * N[0] - S[0] * N[2], S[0] * N[1] - S[1] * N[0]};
    const double tx = crval1_as * arcsec, ty = crval2_as * arcsec;
    const double a = cos(ty) * cos(tx), b = cos(ty) * sin(tx), c = sin(ty);
    const double ea = -sin(ty) * cos(tx), eb = -sin(ty) * sin(tx), ec = cos(ty);
    double w[3], ety[3], etx[3];
    for (int k = 0; k < 3; ++k) {
        w[k] = a * S[k] + b * W[k] + c * N[k];
        ety[k] = ea * S[k] + eb * W[k] + ec * N[k];
    }
    etx[0] = w[1] * ety[2] - w[2] * ety[1];
    etx[1] = w[2] * ety[0] - w[0] * ety[2];
    etx[2] = w[0] * ety[1] - w[1] * ety[0];
    const double cr = cos(crota_deg * deg), sr = sin(crota_deg * deg);
    for (int k = 0; k < 3; ++k) {
        out->obs[k] = obs[k];
        out->w[k] = w[k];
        out->u[k] = cr * etx[k] + sr * ety[k];
        out->v[k] = -sr * etx[k] + cr * ety[k];
    }
    out->cdelt[0] = cdelt1_as * arcsec;
    out->cdelt[1] = cdelt2_as * arcsec;
    out->crpix[0] = crpix1 - 1.0;
    out->crpix[1] = crpix2 - 1.0;
    out->ncol = ncol;
    out->nrow = nrow;
    out->frame = 0;
    out->reserved = 0;
    return TOMO_OK;
}

}  // extern "C"

// ------------------------------------------------------------ scratch pool

namespace tomo {

// The library's stream-ordered scratch comes from a private memory pool per
// device whose release threshold keeps up to kPoolKeep bytes of freed
// memory mapped between calls: repeated calls (a back-projection inside a
// caller's loop, the autotuner's candidates) reuse it instead of mapping
// fresh memory at every call.  Without a pool the default one serves.
constexpr uint64_t kPoolKeep = (uint64_t)1 << 30;
constexpr int kPoolDevices = 64;
static std::mutex g_pool_mu;
static hipMemPool_t g_pool[kPoolDevices];
static bool g_pool_tried[kPoolDevices];

static hipMemPool_t scratch_pool()
{
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kPoolDevices) return nullptr;
    std::lock_guard<std::mutex> lock(g_pool_mu);
    if (!g_pool_tried[dev]) {
        g_pool_tried[dev] = true;
        hipMemPoolProps props;
        memset(&props, 0, sizeof(props));
        props.allocType = hipMemAllocationTypePinned;
        props.handleTypes = hipMemHandleTypeNone;
        props.location.type = hipMemLocationTypeDevice;
        props.location.id = dev;
        hipMemPool_t pool = nullptr;
        if (hipMemPoolCreate(&pool, &props) == hipSuccess) {
            uint64_t keep = kPoolKeep;
            (void)hipMemPoolSetAttribute(pool, hipMemPoolAttrReleaseThreshold, &keep);
            g_pool[dev] = pool;
        } else {
            (void)hipGetLastError();
        }
    }
    return g_pool[dev];
}

hipError_t scratch_alloc(void **p, size_t bytes, hipStream_t s)
{
    hipMemPool_t pool = scratch_pool();
    if (pool) return hipMallocFromPoolAsync(p, bytes, pool, s);
    return hipMallocAsync(p, bytes, s);
}

hipError_t scratch_free(void *p, hipStream_t s) { return p ? hipFreeAsync(p, s) : hipSuccess; }

}  // namespace tomo
