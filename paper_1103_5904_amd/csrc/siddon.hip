// Siddon line-of-sight projector P and its transpose P^T for gfx950.
//
// What is computed (TomograPy, Eq. lo): for every detector pixel, the sum
// over the voxels its line of sight crosses of (length inside the voxel) x
// (voxel value); the transpose scatters the same lengths times the pixel
// value.  Siddon's method finds the lengths from the ray's crossings of the
// x, y and z voxel planes taken in increasing order.
//
// GPU design (not the paper's OpenMP scheme):
// * One ray per lane.  A 256-lane workgroup owns a 16x16 pixel tile of one
//   view and each 64-lane wavefront a compact bundle (8x8 by default), so
//   the lanes of a wave walk neighbouring rays and gather from the same few
//   cache lines at each step.
// * Ray set-up in FP64 (slab clip against the box, entry voxel, first
//   crossing per axis, exit), then an incremental walk that keeps the three
//   "next crossing" parameters relative to the entry point.  The first
//   crossing and the spacing of each axis are rounded to one power-of-two
//   grid sized to the ray's chord, so that every crossing value fits in 51
//   significant bits: the incremental additions are then exact, each
//   crossing equals first + j * spacing exactly, and the exit (the same
//   expression at the box face) is reached exactly, so a ray can never step
//   past the face before it stops.  The rounding moves crossings by < 1e-15
//   of the chord.  FP64 issues at the same VALU rate as unpacked FP32 on
//   CDNA and keeps segment lengths exact to ~1e-15, far inside the required
//   tolerances, and dyadic rays come out bit-exact.
// * Gathers and atomics go through raw buffer resources: 32-bit offsets and
//   a hardware range check (out-of-range loads read 0, atomics are dropped).
// * P^T uses hardware FP32 atomic adds at L2 (buffer_atomic_add_f32).
// * P and P^T share the walk routine, so their matrices are identical.
#include <math.h>
#include <stdio.h>

#include "walk.h"

namespace tomo {

// ------------------------------------------------------------- kernels

template <bool kMapMask, bool kDataMask, bool kObstacle>
__global__ __launch_bounds__(kThreads) void k_project(
    GridDev g, const ViewDev *__restrict__ views, int32_t nviews, Bundle bun, int32_t maxit,
    const float *__restrict__ cube, const uint8_t *__restrict__ map_mask,
    const uint8_t *__restrict__ data_mask, float *__restrict__ images,
    const int *__restrict__ done_flag)
{
    if (done_flag && *done_flag) return;
    project_tile<kMapMask, kDataMask, kObstacle>(g, views, nviews, bun.log2_bw, block_tile(bun), maxit, cube,
                                                 map_mask, data_mask, images);
}

template <bool kMapMask, bool kDataMask>
__global__ __launch_bounds__(kThreads) void k_backproject_atomic(
    GridDev g, const ViewDev *__restrict__ views, int32_t nviews, Bundle bun, int32_t maxit,
    const float *__restrict__ images, const uint8_t *__restrict__ map_mask,
    const uint8_t *__restrict__ data_mask, float *__restrict__ cube,
    const int *__restrict__ done_flag)
{
    if (done_flag && *done_flag) return;
    const LanePixel lp = lane_pixel(views, nviews, block_tile(bun), bun.log2_bw);
    const ViewDev &v = views[lp.view];
    if (lp.col >= v.ncol || lp.row >= v.nrow) return;
    const int64_t pix = v.pix_off + (int64_t)lp.row * v.ncol + lp.col;
    const float yv = images[pix];
    if (!nonzero_bits(yv)) return;
    if (kDataMask && !data_mask[pix]) return;
    RayState r;
    if (!ray_setup(g, v, lp.col, lp.row, r)) return;
    const auto rc = make_rsrc(cube + (int64_t)v.frame * g.nvox, (uint32_t)(g.nvox * 4));
    const double wy = (double)yv * (r.dn * v.gain);
    if constexpr (kMapMask) {
        const auto rm = make_rsrc(map_mask, (uint32_t)g.nvox);
        ray_walk(r, maxit, [&](int32_t off, double dl) {
            if (buf_load_u8(rm, (uint32_t)off)) buf_atomic_add_f32(rc, (uint32_t)off * 4u, (float)(dl * wy));
        });
    } else {
        ray_walk(r, maxit, [&](int32_t off, double dl) {
            buf_atomic_add_f32(rc, (uint32_t)off * 4u, (float)(dl * wy));
        });
    }
}

template <bool kDataMask>
__global__ __launch_bounds__(kThreads) void k_count(GridDev g, const ViewDev *__restrict__ views,
                                                     int32_t nviews, Bundle bun, int32_t maxit,
                                                     const uint8_t *__restrict__ data_mask,
                                                     unsigned long long *__restrict__ total)
{
    __shared__ int64_t lds[4];
    const LanePixel lp = lane_pixel(views, nviews, block_tile(bun), bun.log2_bw);
    const ViewDev &v = views[lp.view];
    int64_t cnt = 0;
    if (lp.col < v.ncol && lp.row < v.nrow) {
        const int64_t pix = v.pix_off + (int64_t)lp.row * v.ncol + lp.col;
        RayState r;
        if ((!kDataMask || data_mask[pix]) && ray_setup(g, v, lp.col, lp.row, r))
            ray_walk(r, maxit, [&](int32_t, double dl) { cnt += dl * r.dn > 0.0; });
    }
    const int64_t s = block_sum_i64(cnt, lds);
    if (threadIdx.x == 0) atomicAdd(total, (unsigned long long)s);
}

__global__ void k_trace(GridDev g, const ViewDev *__restrict__ views, int32_t view, int32_t col,
                        int32_t row, int32_t maxit, int32_t cap, int32_t *__restrict__ idx,
                        double *__restrict__ len, double *__restrict__ dpar,
                        int32_t *__restrict__ n_out)
{
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    RayState r;
    int n = 0;
    if (ray_setup(g, views[view], col, row, r)) {
        ray_walk(r, maxit, [&](int32_t off, double dl) {
            const double l = dl * r.dn;
            if (l > 0.0) {
                if (n < cap) {
                    idx[n] = off;
                    len[n] = l;
                    dpar[n] = dl;
                }
                ++n;
            }
        });
    }
    *n_out = n;
}

__global__ __launch_bounds__(kThreads) void k_fill(float *__restrict__ x, int64_t n, float v)
{
    for (int64_t i = (int64_t)blockIdx.x * kThreads + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * kThreads)
        x[i] = v;
}

// out = M x over every frame: out[f][v] = x[f][v] where map_mask[v], else 0.
// Lets P M x run the unmasked walk, whose one gather per step is the
// projector's bound (a mask byte per step would double the gathers).
__global__ __launch_bounds__(kThreads) void k_mask_copy(const float *__restrict__ x,
                                                        const uint8_t *__restrict__ mask, int64_t nvox,
                                                        int32_t nframes, float *__restrict__ out)
{
    for (int64_t v = (int64_t)blockIdx.x * kThreads + threadIdx.x; v < nvox; v += (int64_t)gridDim.x * kThreads) {
        const bool keep = mask[v] != 0;
        for (int32_t f = 0; f < nframes; ++f) out[(int64_t)f * nvox + v] = keep ? x[(int64_t)f * nvox + v] : 0.0f;
    }
}

// The bricked copy of M x (every frame): one thread per position of a
// bricked frame, in the copy's own order, so that a wavefront writes 256
// contiguous bytes and reads runs of 2^k voxels of x rows (a row's other
// runs are read by the neighbouring bricks' threads soon after, from L2).
// Positions in the padding of partial bricks are left alone: no walk reads
// them.
__global__ __launch_bounds__(kThreads) void k_brick_copy(const float *__restrict__ x,
                                                         const uint8_t *__restrict__ mask, GridDev g, BrickDev bk,
                                                         float *__restrict__ out, const int *__restrict__ done_flag)
{
    if (done_flag && *done_flag) return;
    const int32_t nx = g.n[0], ny = g.n[1], nz = g.n[2];
    const uint32_t k = (uint32_t)bk.k, m = (1u << k) - 1u;
    const uint32_t nb0 = (uint32_t)bk.nb[0], nb01 = (uint32_t)bk.nb[0] * (uint32_t)bk.nb[1];
    for (int64_t o = (int64_t)blockIdx.x * kThreads + threadIdx.x; o < bk.frame_stride;
         o += (int64_t)gridDim.x * kThreads) {
        const uint32_t b = (uint32_t)((uint64_t)o >> (3 * k)), l = (uint32_t)o & ((1u << (3 * k)) - 1u);
        const uint32_t b2 = b / nb01, rb = b - b2 * nb01;
        const uint32_t b1 = rb / nb0, b0 = rb - b1 * nb0;
        const int32_t i0 = (int32_t)((b0 << k) | (l & m));
        const int32_t i1 = (int32_t)((b1 << k) | ((l >> k) & m));
        const int32_t i2 = (int32_t)((b2 << k) | (l >> (2 * k)));
        if (i0 >= nx || i1 >= ny || i2 >= nz) continue;
        const int64_t v = ((int64_t)i2 * ny + i1) * nx + i0;
        const bool keep = !mask || mask[v] != 0;
        for (int32_t f = 0; f < g.nframes; ++f)
            out[(int64_t)f * bk.frame_stride + o] = keep ? x[(int64_t)f * g.nvox + v] : 0.0f;
    }
}

template <bool kDataMask, bool kObstacle, bool kWide>
__global__ __launch_bounds__(kThreads) void k_project_bricked(
    GridDev g, const ViewDev *__restrict__ views, int32_t nviews, Bundle bun, int32_t maxit,
    const float *__restrict__ bricked, BrickDev bk, const uint8_t *__restrict__ data_mask,
    float *__restrict__ images, const int *__restrict__ done_flag)
{
    if (done_flag && *done_flag) return;
    project_tile_bricked<kDataMask, kObstacle, false, kWide>(g, views, nviews, bun.log2_bw, block_tile(bun), maxit,
                                                             bricked, bk, data_mask, images);
}

// The same with the per-axis offset terms in LDS (n0 + n1 + n2 entries of
// dynamic shared memory), filled by the workgroup before its walk.
template <bool kDataMask, bool kObstacle, bool kWide>
__global__ __launch_bounds__(kThreads) void k_project_bricked_lut(
    GridDev g, const ViewDev *__restrict__ views, int32_t nviews, Bundle bun, int32_t maxit,
    const float *__restrict__ bricked, BrickDev bk, const uint8_t *__restrict__ data_mask,
    float *__restrict__ images, const int *__restrict__ done_flag)
{
    extern __shared__ uint32_t lut[];
    if (done_flag && *done_flag) return;
    const int ntab = g.n[0] + g.n[1] + g.n[2];
    for (int e = threadIdx.x; e < ntab; e += kThreads) {
        const int a = e < g.n[0] ? 0 : (e < g.n[0] + g.n[1] ? 1 : 2);
        const int i = a == 0 ? e : (a == 1 ? e - g.n[0] : e - g.n[0] - g.n[1]);
        // byte offsets where a buffer resource spans the frame (one add
        // less per step), element offsets for the clamped global loads
        lut[e] = brick_axis_term(bk, a, i) * (kWide ? 1u : 4u);
    }
    __syncthreads();
    project_tile_bricked<kDataMask, kObstacle, true, kWide>(g, views, nviews, bun.log2_bw, block_tile(bun), maxit,
                                                            bricked, bk, data_mask, images, lut);
}

// ------------------------------------------------------------ launchers

static int64_t grid_blocks(int64_t n) { return (n + kThreads - 1) / kThreads; }

int launch_fill(float *x, int64_t n, float v, hipStream_t s)
{
    if (n <= 0) return TOMO_OK;
    int64_t nb = grid_blocks(n);
    if (nb > 4096) nb = 4096;
    hipLaunchKernelGGL(k_fill, dim3((unsigned)nb), dim3(kThreads), 0, s, x, n, v);
    return hip_fail(hipGetLastError(), "fill kernel launch");
}

int launch_project_tuned(const Plan &p, const tomo_geometry *g, const float *cube, float *images,
                         bool use_map_mask, hipStream_t s, const int *done_flag, const tomo_tuning &tu)
{
    const Bundle b{tu.p_bundle, tu.p_xcd_remap};
    const bool mm = use_map_mask && g->map_mask, dm = g->data_mask != nullptr;
    const dim3 grid((unsigned)p.ntiles), blk(kThreads);
#define TOMO_LAUNCH_P3(M, D, O)                                                                     \
    hipLaunchKernelGGL((k_project<M, D, O>), grid, blk, 0, s, p.grid, p.views_d, p.nviews, b,        \
                       p.max_steps, cube, g->map_mask, g->data_mask, images, done_flag)
#define TOMO_LAUNCH_P(M, D)                                                                         \
    do {                                                                                            \
        if (p.grid.has_sph) TOMO_LAUNCH_P3(M, D, true);                                             \
        else TOMO_LAUNCH_P3(M, D, false);                                                           \
    } while (0)
    if (mm && dm) TOMO_LAUNCH_P(true, true);
    else if (mm) TOMO_LAUNCH_P(true, false);
    else if (dm) TOMO_LAUNCH_P(false, true);
    else TOMO_LAUNCH_P(false, false);
#undef TOMO_LAUNCH_P
#undef TOMO_LAUNCH_P3
    return hip_fail(hipGetLastError(), "projection kernel launch");
}

int launch_project(const Plan &p, const tomo_geometry *g, const float *cube, float *images,
                   bool use_map_mask, hipStream_t s)
{
    return launch_project_with(p, g, cube, images, use_map_mask, s, tuning_for(p));
}

// The bricked layout of a plan's frames for brick side 2^k, or false when a
// padded frame would not be addressable with 32-bit element offsets.
bool brick_layout(const Plan &p, int k, BrickDev &bk)
{
    const int B = 1 << k;
    bk.k = k;
    int64_t stride = (int64_t)B * B * B;
    for (int a = 0; a < 3; ++a) {
        bk.nb[a] = (p.grid.n[a] + B - 1) / B;
        stride *= bk.nb[a];
    }
    bk.frame_stride = stride;
    return stride < ((int64_t)1 << 32);
}

int brick_copy_launch(const Plan &p, const float *cube, const uint8_t *map_mask, const BrickDev &bk, float *out,
                      hipStream_t s, const int *done_flag)
{
    int64_t nb = grid_blocks(bk.frame_stride);
    nb = nb > 8192 ? 8192 : nb;
    hipLaunchKernelGGL(k_brick_copy, dim3((unsigned)nb), dim3(kThreads), 0, s, cube, map_mask, p.grid, bk, out,
                       done_flag);
    return hip_fail(hipGetLastError(), "brick copy launch");
}

int launch_project_from_bricks(const Plan &p, const tomo_geometry *g, const float *br, const BrickDev &bk,
                               float *images, hipStream_t s, const int *done_flag, const tomo_tuning &tu)
{
    const Bundle b{tu.p_bundle, tu.p_xcd_remap};
    const bool dm = g->data_mask != nullptr;
    const dim3 grid((unsigned)p.ntiles), blk(kThreads);
    // the per-axis offset terms in LDS when they fit in 32 KiB
    const size_t lut = sizeof(uint32_t) * ((size_t)p.grid.n[0] + p.grid.n[1] + p.grid.n[2]);
    // a frame a buffer resource cannot span takes plain global loads
    const bool wide = bk.frame_stride >= ((int64_t)1 << 30);
#define TOMO_LAUNCH_PB(K, D, O)                                                                                \
    do {                                                                                                       \
        if (wide)                                                                                              \
            hipLaunchKernelGGL((K<D, O, true>), grid, blk, lut_bytes, s, p.grid, p.views_d, p.nviews, b,       \
                               p.max_steps, br, bk, g->data_mask, images, done_flag);                         \
        else                                                                                                   \
            hipLaunchKernelGGL((K<D, O, false>), grid, blk, lut_bytes, s, p.grid, p.views_d, p.nviews, b,      \
                               p.max_steps, br, bk, g->data_mask, images, done_flag);                         \
    } while (0)
#define TOMO_LAUNCH_PB_ALL(K)                                         \
    do {                                                              \
        if (dm) {                                                     \
            if (p.grid.has_sph) TOMO_LAUNCH_PB(K, true, true);        \
            else TOMO_LAUNCH_PB(K, true, false);                      \
        } else {                                                      \
            if (p.grid.has_sph) TOMO_LAUNCH_PB(K, false, true);       \
            else TOMO_LAUNCH_PB(K, false, false);                     \
        }                                                             \
    } while (0)
    if (lut <= 32768) {
        const size_t lut_bytes = lut;
        TOMO_LAUNCH_PB_ALL(k_project_bricked_lut);
    } else {
        const size_t lut_bytes = 0;
        TOMO_LAUNCH_PB_ALL(k_project_bricked);
    }
#undef TOMO_LAUNCH_PB_ALL
#undef TOMO_LAUNCH_PB
    return hip_fail(hipGetLastError(), "bricked projection kernel launch");
}

int launch_project_bricked(const Plan &p, const tomo_geometry *g, const float *cube, float *images,
                           bool use_map_mask, hipStream_t s, const int *done_flag, const tomo_tuning &tu)
{
    BrickDev bk;
    float *br = nullptr;
    if (!brick_layout(p, tu.p_layout, bk) ||
        scratch_alloc((void **)&br, sizeof(float) * (size_t)(bk.frame_stride * p.grid.nframes), s) != hipSuccess) {
        (void)hipGetLastError();  // no bricked copy: the x-fastest walk gives the same result
        tomo_tuning lin = tu;
        lin.p_layout = 0;
        return launch_project_tuned(p, g, cube, images, use_map_mask, s, done_flag, lin);
    }
    int rc = brick_copy_launch(p, cube, use_map_mask ? g->map_mask : nullptr, bk, br, s, done_flag);
    if (!rc) rc = launch_project_from_bricks(p, g, br, bk, images, s, done_flag, tu);
    (void)scratch_free(br, s);
    return rc;
}

int launch_project_with(const Plan &p, const tomo_geometry *g, const float *cube, float *images,
                        bool use_map_mask, hipStream_t s, const tomo_tuning &tu)
{
    if (tu.p_layout >= 2) return launch_project_bricked(p, g, cube, images, use_map_mask, s, nullptr, tu);
    if (use_map_mask && g->map_mask) {
        // P M x as the unmasked walk over a masked copy (stream-ordered
        // scratch); without the memory, the walk tests the mask itself
        float *tmp = nullptr;
        const int64_t total = p.grid.nvox * p.grid.nframes;
        if (scratch_alloc((void **)&tmp, sizeof(float) * (size_t)total, s) == hipSuccess) {
            int64_t nb = grid_blocks(p.grid.nvox);
            nb = nb > 4096 ? 4096 : nb;
            hipLaunchKernelGGL(k_mask_copy, dim3((unsigned)nb), dim3(kThreads), 0, s, cube, g->map_mask,
                               p.grid.nvox, (int32_t)p.grid.nframes, tmp);
            int rc = hip_fail(hipGetLastError(), "mask copy launch");
            if (!rc) rc = launch_project_tuned(p, g, tmp, images, false, s, nullptr, tu);
            (void)scratch_free(tmp, s);
            return rc;
        }
        (void)hipGetLastError();  // the failed allocation's error is not the caller's
    }
    return launch_project_tuned(p, g, cube, images, use_map_mask, s, nullptr, tu);
}

size_t bricked_copy_bytes(const Plan &p, const tomo_tuning &tu)
{
    BrickDev bk;
    if (tu.p_layout < 2 || !brick_layout(p, tu.p_layout, bk)) return 0;
    return sizeof(float) * (size_t)(bk.frame_stride * p.grid.nframes);
}

int launch_project_flagged(const Plan &p, const tomo_geometry *g, const float *cube,
                           float *images, hipStream_t s, const int *done_flag, float *bricks)
{
    const tomo_tuning tu = tuning_for(p);
    if (tu.p_layout >= 2) {
        BrickDev bk;
        if (bricks && brick_layout(p, tu.p_layout, bk)) {
            int rc = brick_copy_launch(p, cube, nullptr, bk, bricks, s, done_flag);
            if (!rc) rc = launch_project_from_bricks(p, g, bricks, bk, images, s, done_flag, tu);
            return rc;
        }
        return launch_project_bricked(p, g, cube, images, false, s, done_flag, tu);
    }
    return launch_project_tuned(p, g, cube, images, false, s, done_flag, tu);
}

int resolve_bp_strategy(const Plan &p, int strategy)
{
    return strategy == TOMO_BP_AUTO ? tuning_for(p).bp_default : strategy;
}

int launch_backproject(const Plan &p, const tomo_geometry *g, const float *images, float *cube,
                       bool accumulate, bool use_map_mask, int strategy, hipStream_t s,
                       const int *done_flag, void *scratch, size_t scratch_bytes, const RayTable *tab)
{
    return launch_backproject_tuned(p, g, images, cube, accumulate, use_map_mask, strategy, s, done_flag,
                                    scratch, scratch_bytes, tuning_for(p), tab);
}

int launch_backproject_tuned(const Plan &p, const tomo_geometry *g, const float *images, float *cube,
                             bool accumulate, bool use_map_mask, int strategy, hipStream_t s,
                             const int *done_flag, void *scratch, size_t scratch_bytes,
                             const tomo_tuning &tu, const RayTable *tab)
{
    if (strategy == TOMO_BP_AUTO) strategy = tu.bp_default;
    if (strategy == TOMO_BP_BLOCKED) {
        if (scratch)
            return launch_backproject_blocked(p, g, images, cube, accumulate, use_map_mask, s, done_flag,
                                              scratch, scratch_bytes, tu, tab);
        const size_t need = blocked_scratch_bytes(p, blocked_shape(p, tu), g->data_mask != nullptr);
        void *tmp = nullptr;
        if (scratch_alloc(&tmp, need, s) != hipSuccess)
            return set_error(TOMO_ENOMEM, "back-projection scratch of %zu bytes", need);
        const int rc = launch_backproject_blocked(p, g, images, cube, accumulate, use_map_mask, s,
                                                  done_flag, tmp, need, tu, tab);
        (void)scratch_free(tmp, s);
        return rc;
    }
    // the atomic kernels address a frame through a buffer resource, whose
    // byte range is 32-bit
    if (p.grid.nvox >= ((int64_t)1 << 30))
        return set_error(TOMO_EUNSUPPORTED, "binned and atomic back-projection need frames below 2^30 voxels");
    if (!accumulate) {
        int rc = launch_fill(cube, p.grid.nvox * p.grid.nframes, 0.0f, s);
        if (rc) return rc;
    }
    if (strategy == TOMO_BP_BINNED)
        return launch_backproject_binned(p, g, images, cube, use_map_mask, s, done_flag, tu);
    const Bundle b{tu.bp_bundle, tu.bp_xcd_remap};
    const bool mm = use_map_mask && g->map_mask, dm = g->data_mask != nullptr;
    const dim3 grid((unsigned)p.ntiles), blk(kThreads);
#define TOMO_LAUNCH_BP(M, D)                                                                        \
    hipLaunchKernelGGL((k_backproject_atomic<M, D>), grid, blk, 0, s, p.grid, p.views_d, p.nviews,  \
                       b, p.max_steps, images, g->map_mask, g->data_mask, cube, done_flag)
    if (mm && dm) TOMO_LAUNCH_BP(true, true);
    else if (mm) TOMO_LAUNCH_BP(true, false);
    else if (dm) TOMO_LAUNCH_BP(false, true);
    else TOMO_LAUNCH_BP(false, false);
#undef TOMO_LAUNCH_BP
    return hip_fail(hipGetLastError(), "back-projection kernel launch");
}

}  // namespace tomo

using namespace tomo;

extern "C" int tomo_count_crossings(const tomo_geometry *g, int64_t *total_h, tomo_stream stream)
{
    if (!total_h) return set_error(TOMO_EINVAL, "tomo_count_crossings: total_h is NULL");
    int st = TOMO_OK;
    PlanRef p = get_plan(g, &st);
    if (!p) return st;
    hipStream_t s = (hipStream_t)stream;
    unsigned long long *d = nullptr;
    if (scratch_alloc((void **)&d, sizeof(*d), s) != hipSuccess)
        return set_error(TOMO_ENOMEM, "tomo_count_crossings: device allocation failed");
    (void)hipMemsetAsync(d, 0, sizeof(*d), s);
    const tomo_tuning tu = tuning_for(*p);
    const Bundle b{tu.p_bundle, tu.p_xcd_remap};
    if (g->data_mask)
        hipLaunchKernelGGL((k_count<true>), dim3((unsigned)p->ntiles), dim3(kThreads), 0, s, p->grid,
                           p->views_d, p->nviews, b, p->max_steps, g->data_mask, d);
    else
        hipLaunchKernelGGL((k_count<false>), dim3((unsigned)p->ntiles), dim3(kThreads), 0, s,
                           p->grid, p->views_d, p->nviews, b, p->max_steps, g->data_mask, d);
    int rc = hip_fail(hipGetLastError(), "count kernel launch");
    unsigned long long h = 0;
    if (!rc) rc = hip_fail(hipMemcpyAsync(&h, d, sizeof(h), hipMemcpyDeviceToHost, s), "copy count");
    if (!rc) rc = hip_fail(hipStreamSynchronize(s), "count synchronise");
    (void)scratch_free(d, s);
    if (!rc) *total_h = (int64_t)h;
    return rc;
}

extern "C" int tomo_trace_ray(const tomo_geometry *g, int32_t view, int32_t col, int32_t row,
                              int32_t *idx_h, double *len_h, double *dpar_h, int32_t cap,
                              int32_t *n_out)
{
    if (!idx_h || !len_h || !n_out || cap < 0)
        return set_error(TOMO_EINVAL, "tomo_trace_ray: NULL output or negative capacity");
    int st = TOMO_OK;
    PlanRef p = get_plan(g, &st);
    if (!p) return st;
    if (view < 0 || view >= g->nviews || col < 0 || row < 0 || col >= g->views[view].ncol ||
        row >= g->views[view].nrow)
        return set_error(TOMO_EINVAL, "tomo_trace_ray: pixel (%d, %d, %d) out of range", view, col,
                         row);
    const int32_t need = p->max_steps;
    int32_t *di = nullptr, *dn = nullptr;
    double *dl = nullptr, *dp = nullptr;
    int rc = TOMO_OK;
    if (hipMalloc((void **)&di, sizeof(int32_t) * need) != hipSuccess ||
        hipMalloc((void **)&dl, sizeof(double) * need) != hipSuccess ||
        hipMalloc((void **)&dp, sizeof(double) * need) != hipSuccess ||
        hipMalloc((void **)&dn, sizeof(int32_t)) != hipSuccess) {
        rc = set_error(TOMO_ENOMEM, "tomo_trace_ray: device allocation failed");
    } else {
        hipLaunchKernelGGL(k_trace, dim3(1), dim3(64), 0, 0, p->grid, p->views_d, view, col, row,
                           p->max_steps, need, di, dl, dp, dn);
        rc = hip_fail(hipGetLastError(), "trace kernel launch");
        int32_t n = 0;
        if (!rc) rc = hip_fail(hipMemcpy(&n, dn, sizeof(n), hipMemcpyDeviceToHost), "copy count");
        if (!rc) {
            *n_out = n;
            if (n > cap) {
                rc = set_error(TOMO_EINVAL, "tomo_trace_ray: %d segments exceed capacity %d", n, cap);
            } else if (n > 0) {
                rc = hip_fail(hipMemcpy(idx_h, di, sizeof(int32_t) * n, hipMemcpyDeviceToHost), "copy idx");
                if (!rc)
                    rc = hip_fail(hipMemcpy(len_h, dl, sizeof(double) * n, hipMemcpyDeviceToHost), "copy len");
                if (!rc && dpar_h)
                    rc = hip_fail(hipMemcpy(dpar_h, dp, sizeof(double) * n, hipMemcpyDeviceToHost), "copy dpar");
            }
        }
    }
    (void)hipFree(di);
    (void)hipFree(dl);
    (void)hipFree(dp);
    (void)hipFree(dn);
    return rc;
}
