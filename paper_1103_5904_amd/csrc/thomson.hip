// White-light Thomson-scattering operators (Sec. "White Light: Thomson
// Scattering"; Eq. 4C, Eq. thomson_lo, Eq. brightness, Eq. thomson_direct):
//   pB = scale O P M n_e,    B = scale (P M' - O P M) n_e,
// O = diag(rho_k^2) over lines of sight (squared impact parameter), M and M'
// diagonal over voxels from Billings' coefficients at sin(Omega) = R_sun / r:
//   m  = ((1 - u) C1 + u C2) / r^4,   m' = 2 ((1 - u) C3 + u C4) / r^2,
// r and rho in solar radii from the Sun's centre, zero for voxel centres on
// or inside the photosphere.  C4 takes +1/8 before its bracket (its small-
// angle limit C4 / C3 -> 2/3, the limb-darkened flux ratio, fixes the sign
// the printed equation garbles).
//
// gfx950 design: the diagonals are recomputed on the fly in FP64 by two
// streaming kernels (one over voxels, folding in the map mask; one over
// pixels), around the projector's own kernels: the unmasked walk for P and
// the deterministic owner-computes kernel for P^T.  B takes two projections
// (and its transpose two back-projections), as the paper notes.
#include <math.h>

#include <vector>

#include "common.h"

namespace tomo {

struct SunDev {
    double c[3];     // centre, box units
    double inv_r;    // 1 / R_sun in box units
    double u;        // limb darkening
    double scale;    // pi sigma I0 / 2
};

__device__ inline void thomson_weights(double r, double u, double &m, double &mp)
{
    if (!(r > 1.0)) {
        m = mp = 0.0;
        return;
    }
    const double s = 1.0 / r, ss = s * s, c = sqrt(1.0 - ss);
    const double lg = log((1.0 + s) / c), ccs = c * c / s;
    const double c1 = c * ss;
    const double c2 = -0.125 * (1.0 - 3.0 * ss - ccs * (1.0 + 3.0 * ss) * lg);
    const double c3 = 4.0 / 3.0 - c - c * c * c / 3.0;
    const double c4 = 0.125 * (5.0 + ss - ccs * (5.0 - ss) * lg);
    const double r2 = r * r;
    m = ((1.0 - u) * c1 + u * c2) / (r2 * r2);
    mp = 2.0 * ((1.0 - u) * c3 + u * c4) / r2;
}

// r (solar radii) of voxel v's centre
__device__ inline double voxel_r(const GridDev &g, const SunDev &sun, int64_t v)
{
    const int i = (int)(v % g.n[0]);
    const int64_t jk = v / g.n[0];
    const int j = (int)(jk % g.n[1]), k = (int)(jk / g.n[1]);
    const int idx[3] = {i, j, k};
    double r2 = 0.0;
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        const double x = g.lo[a] + ((double)idx[a] + 0.5) * g.delta[a] - sun.c[a];
        r2 = fma(x, x, r2);
    }
    return sqrt(r2) * sun.inv_r;
}

// out_m = M M_map x (and out_mp = M' M_map x) over every frame
__global__ __launch_bounds__(kThreads) void k_thomson_weigh(const float *__restrict__ x, GridDev g, SunDev sun,
                                                           const uint8_t *__restrict__ map_mask,
                                                           float *__restrict__ out_m, float *__restrict__ out_mp)
{
    for (int64_t v = (int64_t)blockIdx.x * kThreads + threadIdx.x; v < g.nvox; v += (int64_t)gridDim.x * kThreads) {
        double m, mp;
        thomson_weights(voxel_r(g, sun, v), sun.u, m, mp);
        if (map_mask && !map_mask[v]) m = mp = 0.0;
        for (int32_t f = 0; f < g.nframes; ++f) {
            const int64_t i = (int64_t)f * g.nvox + v;
            const double xv = x[i];
            out_m[i] = (float)(m * xv);
            if (out_mp) out_mp[i] = (float)(mp * xv);
        }
    }
}

// rho^2 (solar radii) of pixel (col, row)'s line of sight
__device__ inline double pixel_rho2(const ViewDev &v, const SunDev &sun, int col, int row)
{
    const double x = ((double)col - v.cp[0]) * v.cd[0], y = ((double)row - v.cp[1]) * v.cd[1];
    double d[3], o[3];
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        d[a] = v.w[a] + x * v.u[a] + y * v.v[a];
        o[a] = v.o[a] - sun.c[a];
    }
    const double cx = o[1] * d[2] - o[2] * d[1], cy = o[2] * d[0] - o[0] * d[2], cz = o[0] * d[1] - o[1] * d[0];
    const double dd = d[0] * d[0] + d[1] * d[1] + d[2] * d[2];
    return (cx * cx + cy * cy + cz * cz) / dd * (sun.inv_r * sun.inv_r);
}

// forward pixel pass, in place: img = scale rho^2 img (pB), or
// img = scale (img_mp - rho^2 img) (B, img_mp != nullptr); grid.y = view
__global__ __launch_bounds__(kThreads) void k_thomson_pixels_fwd(const ViewDev *__restrict__ views, SunDev sun,
                                                                float *__restrict__ img,
                                                                const float *__restrict__ img_mp)
{
    const ViewDev &v = views[blockIdx.y];
    const int64_t np = (int64_t)v.ncol * v.nrow;
    for (int64_t i = (int64_t)blockIdx.x * kThreads + threadIdx.x; i < np; i += (int64_t)gridDim.x * kThreads) {
        const int col = (int)(i % v.ncol), row = (int)(i / v.ncol);
        const double o = pixel_rho2(v, sun, col, row);
        const int64_t k = v.pix_off + i;
        double val = -o * (double)img[k];
        val = img_mp ? val + (double)img_mp[k] : -val;
        img[k] = (float)(sun.scale * val);
    }
}

// transpose pixel pass: y_o = scale rho^2 y; y_s = scale y (if non-null)
__global__ __launch_bounds__(kThreads) void k_thomson_pixels_bwd(const ViewDev *__restrict__ views, SunDev sun,
                                                                const float *__restrict__ y,
                                                                float *__restrict__ y_o, float *__restrict__ y_s)
{
    const ViewDev &v = views[blockIdx.y];
    const int64_t np = (int64_t)v.ncol * v.nrow;
    for (int64_t i = (int64_t)blockIdx.x * kThreads + threadIdx.x; i < np; i += (int64_t)gridDim.x * kThreads) {
        const int col = (int)(i % v.ncol), row = (int)(i / v.ncol);
        const int64_t k = v.pix_off + i;
        const double yv = (double)y[k] * sun.scale;
        y_o[k] = (float)(pixel_rho2(v, sun, col, row) * yv);
        if (y_s) y_s[k] = (float)yv;
    }
}

// transpose voxel pass: x (+)= M_map (M a) (pB), or M_map (M' b - M a) (B)
__global__ __launch_bounds__(kThreads) void k_thomson_combine(const float *__restrict__ a,
                                                             const float *__restrict__ b, GridDev g, SunDev sun,
                                                             const uint8_t *__restrict__ map_mask,
                                                             float *__restrict__ x, int32_t accumulate)
{
    for (int64_t v = (int64_t)blockIdx.x * kThreads + threadIdx.x; v < g.nvox; v += (int64_t)gridDim.x * kThreads) {
        double m, mp;
        thomson_weights(voxel_r(g, sun, v), sun.u, m, mp);
        if (map_mask && !map_mask[v]) m = mp = 0.0;
        for (int32_t f = 0; f < g.nframes; ++f) {
            const int64_t i = (int64_t)f * g.nvox + v;
            double val = -m * (double)a[i];
            val = b ? val + mp * (double)b[i] : -val;
            x[i] = accumulate ? (float)((double)x[i] + val) : (float)val;
        }
    }
}

static unsigned stream_blocks(int64_t n)
{
    const int64_t b = (n + kThreads - 1) / kThreads;
    return (unsigned)(b > 4096 ? 4096 : (b < 1 ? 1 : b));
}

static int check_thomson(const tomo_thomson *t, int32_t kind, SunDev &sun)
{
    if (!t) return set_error(TOMO_EINVAL, "thomson: parameters are NULL");
    if (kind != TOMO_THOMSON_PB && kind != TOMO_THOMSON_B)
        return set_error(TOMO_EINVAL, "thomson: kind must be TOMO_THOMSON_PB or TOMO_THOMSON_B");
    if (!(t->u >= 0.0 && t->u <= 1.0)) return set_error(TOMO_EINVAL, "thomson: u must lie in [0, 1]");
    if (!isfinite(t->scale)) return set_error(TOMO_EINVAL, "thomson: scale must be finite");
    if (!isfinite(t->sun_center[0]) || !isfinite(t->sun_center[1]) || !isfinite(t->sun_center[2]) ||
        !isfinite(t->sun_radius) || !(t->sun_radius > 0.0))
        return set_error(TOMO_EINVAL, "thomson: the Sun's centre must be finite and its radius > 0");
    for (int a = 0; a < 3; ++a) sun.c[a] = t->sun_center[a];
    sun.inv_r = 1.0 / t->sun_radius;
    sun.u = t->u;
    sun.scale = t->scale;
    return TOMO_OK;
}

// Stream-ordered scratch released on every path.
struct Scratch {
    hipStream_t s;
    std::vector<void *> p;
    void *take(size_t bytes)
    {
        void *q = nullptr;
        if (scratch_alloc(&q, bytes, s) != hipSuccess) return nullptr;
        p.push_back(q);
        return q;
    }
    ~Scratch()
    {
        for (void *q : p) (void)scratch_free(q, s);
    }
};

static int max_view_pixels(const tomo_geometry *g)
{
    int64_t m = 1;
    for (int k = 0; k < g->nviews; ++k) {
        const int64_t n = (int64_t)g->views[k].ncol * g->views[k].nrow;
        m = n > m ? n : m;
    }
    return (int)((m + kThreads - 1) / kThreads > 1024 ? 1024 : (m + kThreads - 1) / kThreads);
}

}  // namespace tomo

using namespace tomo;

extern "C" {

int tomo_thomson_project(const tomo_geometry *g, const tomo_thomson *t, int32_t kind, const float *ne_d,
                         float *images_d, tomo_stream stream)
{
    SunDev sun;
    int rc = check_thomson(t, kind, sun);
    if (rc) return rc;
    if (!ne_d || !images_d) return set_error(TOMO_EINVAL, "tomo_thomson_project: NULL array");
    int st = TOMO_OK;
    PlanRef plan = get_plan(g, &st);
    if (!plan) return st;
    const Plan &p = *plan;
    hipStream_t s = (hipStream_t)stream;
    const int64_t total = p.grid.nvox * p.grid.nframes;
    const bool two = kind == TOMO_THOMSON_B;
    Scratch sc{s, {}};
    float *cm = (float *)sc.take(sizeof(float) * (size_t)total);
    float *cmp = two ? (float *)sc.take(sizeof(float) * (size_t)total) : nullptr;
    float *imp = two ? (float *)sc.take(sizeof(float) * (size_t)p.npix) : nullptr;
    if (!cm || (two && (!cmp || !imp))) return set_error(TOMO_ENOMEM, "tomo_thomson_project: scratch allocation");
    hipLaunchKernelGGL(k_thomson_weigh, dim3(stream_blocks(p.grid.nvox)), dim3(kThreads), 0, s, ne_d, p.grid, sun,
                       g->map_mask, cm, cmp);
    rc = hip_fail(hipGetLastError(), "thomson weighting launch");
    if (!rc) rc = launch_project(p, g, cm, images_d, false, s);
    if (!rc && two) rc = launch_project(p, g, cmp, imp, false, s);
    if (rc) return rc;
    hipLaunchKernelGGL(k_thomson_pixels_fwd, dim3((unsigned)max_view_pixels(g), (unsigned)p.nviews), dim3(kThreads),
                       0, s, p.views_d, sun, images_d, imp);
    return hip_fail(hipGetLastError(), "thomson pixel launch");
}

int tomo_thomson_backproject(const tomo_geometry *g, const tomo_thomson *t, int32_t kind, const float *images_d,
                             float *ne_d, int32_t accumulate, tomo_stream stream)
{
    SunDev sun;
    int rc = check_thomson(t, kind, sun);
    if (rc) return rc;
    if (!ne_d || !images_d) return set_error(TOMO_EINVAL, "tomo_thomson_backproject: NULL array");
    int st = TOMO_OK;
    PlanRef plan = get_plan(g, &st);
    if (!plan) return st;
    const Plan &p = *plan;
    hipStream_t s = (hipStream_t)stream;
    const int64_t total = p.grid.nvox * p.grid.nframes;
    const bool two = kind == TOMO_THOMSON_B;
    Scratch sc{s, {}};
    float *yo = (float *)sc.take(sizeof(float) * (size_t)p.npix);
    float *ys = two ? (float *)sc.take(sizeof(float) * (size_t)p.npix) : nullptr;
    float *a = (float *)sc.take(sizeof(float) * (size_t)total);
    float *b = two ? (float *)sc.take(sizeof(float) * (size_t)total) : nullptr;
    if (!yo || !a || (two && (!ys || !b)))
        return set_error(TOMO_ENOMEM, "tomo_thomson_backproject: scratch allocation");
    hipLaunchKernelGGL(k_thomson_pixels_bwd, dim3((unsigned)max_view_pixels(g), (unsigned)p.nviews), dim3(kThreads),
                       0, s, p.views_d, sun, images_d, yo, ys);
    rc = hip_fail(hipGetLastError(), "thomson pixel launch");
    if (!rc) rc = launch_backproject(p, g, yo, a, false, false, TOMO_BP_BLOCKED, s);
    if (!rc && two) rc = launch_backproject(p, g, ys, b, false, false, TOMO_BP_BLOCKED, s);
    if (rc) return rc;
    hipLaunchKernelGGL(k_thomson_combine, dim3(stream_blocks(p.grid.nvox)), dim3(kThreads), 0, s, a, b, p.grid, sun,
                       g->map_mask, ne_d, accumulate ? 1 : 0);
    return hip_fail(hipGetLastError(), "thomson combine launch");
}

}  // extern "C"
