// Owner-computes transpose P^T for gfx950 (TOMO_BP_BLOCKED).
//
// On MI355X a device-scope FP32 atomic to global memory is performed past
// the XCD's L2 and costs a memory transaction of its own, so any P^T that
// adds into the cube with atomics is bound by the number of atomics, not by
// its walk.  Here the cube is cut into blocks of bx x by x bz voxels and each
// workgroup owns one block (optionally one share of the block's views, see
// below):
//
// * For every view, the pixels whose rays can cross the block lie in the
//   bounding rectangle of the block's eight corners projected through the
//   pinhole (plus one pixel of margin); corners behind the observer widen it
//   to the whole detector.  Where pixels are finer than voxels (kRows, set
//   per geometry by the plan), each row of a rectangle of at most 64 rows
//   keeps only the column interval whose rays meet the block's box: the
//   rays of a row fill a plane through the observer, which cuts the box in
//   a convex polygon, and the polygon's corners on the box's edges bound the
//   interval (FP32, on a box padded far beyond that rounding, plus one pixel
//   each side).  A flat block seen edge-on projects to a slanted band that
//   fills about 60% of its rectangle, and every ray dropped saves a set-up.
//   Where footprints are a few pixels, intervals cannot save a pass, and the
//   kernel compiled without them keeps 91 VGPRs against 128.
// * The footprint is walked 256 pixels per pass in row-major order; each
//   lane takes one of those rays, sets it up exactly as P does and walks
//   only its part inside the block.  The walk's crossing parameters
//   live on a power-of-two grid on which every sum the walk forms is exact:
//   the k-th crossing of axis a is s_a + k ds_a whatever the order of
//   additions.  So the parameter interval [E, X) in which the ray is inside
//   the block and the walk state at E (crossings done on each axis, current
//   voxel) follow in closed form from integers, and the in-block walk
//   reproduces P's segments bit for bit: the matrix stays the transpose of
//   P's.
// * Contributions go to 64-bit fixed-point LDS bins (integer LDS atomics;
//   sums are exact and order-independent).  The scale is a power of two from
//   the largest |gain y| of the views involved and the number of their pixels, a
//   bound on the rays that can reach one voxel, so no bin can overflow.
//   Items whose views hold a non-finite value accumulate in FP32 LDS bins
//   instead.
// * At the end the block is written once with plain stores: the cube itself
//   (map mask and accumulate applied) when the block has one owner, else the
//   owner's slice of a partial buffer [splits][frames * nvox] that a second
//   kernel sums in a fixed order.  No global atomics anywhere, and the
//   result is deterministic.
#include <limits.h>

#include "blocked.h"

namespace tomo {

template <bool kDataMask>
__global__ __launch_bounds__(kThreads) void k_view_absmax(const ViewDev *__restrict__ views,
                                                          const float *__restrict__ images,
                                                          const uint8_t *__restrict__ data_mask,
                                                          uint32_t *__restrict__ ymax,
                                                          const int *__restrict__ done_flag)
{
    __shared__ uint32_t red[kThreads / 64];
    if (done_flag && *done_flag) return;
    const int vi = blockIdx.x / kYmaxParts, part = blockIdx.x % kYmaxParts;
    const uint32_t m = view_absmax_part<kDataMask>(views[vi], part, images, data_mask, red);
    if (threadIdx.x == 0) ymax[blockIdx.x] = m;
}

// Kept pixels of every image row (see KeptRows): one wavefront per row, 64
// columns per ballot.
__global__ __launch_bounds__(kThreads) void k_kept_rows(const ViewDev *__restrict__ views, int32_t nviews,
                                                        const uint8_t *__restrict__ data_mask,
                                                        uint16_t *__restrict__ pre, uint16_t *__restrict__ cols,
                                                        const int *__restrict__ done_flag)
{
    if (done_flag && *done_flag) return;
    const int lane = threadIdx.x & 63;
    for (int vi = blockIdx.y; vi < nviews; vi += gridDim.y) {
        const ViewDev &v = views[vi];
        const int row = blockIdx.x * (kThreads / 64) + (threadIdx.x >> 6);
        if (row >= v.nrow) continue;
        const int64_t rb = v.pix_off + (int64_t)row * v.ncol;
        int base = 0;
        for (int c0 = 0; c0 < v.ncol; c0 += 64) {
            const int c = c0 + lane;
            const bool keep = c < v.ncol && data_mask[rb + c] != 0;
            const uint64_t bal = __ballot(keep);
            const int below = __popcll(bal & ((1ull << lane) - 1ull));
            if (c < v.ncol) {
                pre[rb + c] = (uint16_t)(base + below);
                if (keep) cols[rb + base + below] = (uint16_t)c;
            }
            base += __popcll(bal);
        }
    }
}

// The ray table of a geometry (RayTable): one thread per pixel, views along
// the grid's y.
__global__ __launch_bounds__(kThreads) void k_ray_table(GridDev g, const ViewDev *__restrict__ views, int32_t nviews,
                                                        double *__restrict__ d, uint64_t *__restrict__ k, int64_t n)
{
    for (int vi = blockIdx.y; vi < nviews; vi += gridDim.y) {
        const ViewDev &v = views[vi];
        const int64_t np = (int64_t)v.ncol * v.nrow;
        for (int64_t q = (int64_t)blockIdx.x * kThreads + threadIdx.x; q < np; q += (int64_t)gridDim.x * kThreads) {
            const int row = (int)(q / v.ncol), col = (int)(q - (int64_t)row * v.ncol);
            RayState r;
            RayAxes ax;
            const bool ok = ray_setup<true>(g, v, col, row, r, &ax);
            ray_table_put(d, k, n, v.pix_off + q, ok, r, ax);
        }
    }
}

size_t ray_table_bytes(const Plan &p)
{
    for (int a = 0; a < 3; ++a)
        if (p.grid.n[a] > (1 << kRayTableSideBits)) return 0;
    if (p.npix <= 0) return 0;
    const size_t n = (size_t)p.npix;
    return ((sizeof(double) * kRayTableCols * n + 255) & ~(size_t)255) + sizeof(uint64_t) * n;
}

int ray_table_build(const Plan &p, void *mem, RayTable &out, hipStream_t s)
{
    if (!ray_table_bytes(p) || !mem) return set_error(TOMO_EINVAL, "ray table: none for this geometry");
    const size_t n = (size_t)p.npix;
    double *d = (double *)mem;
    uint64_t *k = (uint64_t *)((char *)mem + ((sizeof(double) * kRayTableCols * n + 255) & ~(size_t)255));
    // a view's pixels grid-stride over gx workgroups, sized for the mean view
    const int64_t per_view = (p.npix + p.nviews - 1) / p.nviews;
    int64_t gx = (per_view + kThreads - 1) / kThreads;
    gx = gx < 1 ? 1 : (gx > 1024 ? 1024 : gx);
    const dim3 grid((unsigned)gx, (unsigned)(p.nviews < 65535 ? p.nviews : 65535));
    hipLaunchKernelGGL(k_ray_table, grid, dim3(kThreads), 0, s, p.grid, p.views_d, p.nviews, d, k, p.npix);
    out.d = d;
    out.k = k;
    out.n = p.npix;
    return hip_fail(hipGetLastError(), "ray table kernel launch");
}

template <int NT, bool kMapMask, bool kDataMask, bool kObstacle, bool kRows>
__global__ __launch_bounds__(NT) __attribute__((amdgpu_waves_per_eu(4))) void k_backproject_blocked(
    GridDev g, const ViewDev *__restrict__ views, const int32_t *__restrict__ frame_views,
    const int32_t *__restrict__ frame_voff, BlockDev bd, Bundle bun, const float *__restrict__ images,
    const uint8_t *__restrict__ map_mask, const uint8_t *__restrict__ data_mask, KeptRows kept,
    const uint32_t *__restrict__ ymax_parts, float *__restrict__ out, int32_t accumulate,
    const int *__restrict__ done_flag, unsigned *__restrict__ spill, RayTable tab)
{
    extern __shared__ unsigned long long bins[];  // bx*by*bz fixed-point (or FP32) sums
    __shared__ BlockedShared<NT, kRows> sh;
    if (done_flag && *done_flag) return;
    const int64_t nitems = (int64_t)bd.nb[0] * bd.nb[1] * bd.nb[2] * g.nframes * bd.splits;
    const int64_t item = xcd_order(bun.xcd_remap, blockIdx.x, gridDim.x);
    if (item >= nitems) return;
    blocked_item<NT, kMapMask, kDataMask, kObstacle, kRows>(g, views, frame_views, frame_voff, bd, item, images,
                                                            map_mask, data_mask, kept, ymax_parts, out, accumulate,
                                                            spill, tab, bins, sh);
}

// out[i] = M (sum over owners of part[s][i]) (+ out[i]), owners in order.
template <bool kMapMask>
__global__ __launch_bounds__(kThreads) void k_sum_owners(const float *__restrict__ part, int32_t splits,
                                                         int64_t total, int64_t nvox,
                                                         const uint8_t *__restrict__ map_mask,
                                                         float *__restrict__ out, int32_t accumulate,
                                                         const int *__restrict__ done_flag)
{
    if (done_flag && *done_flag) return;
    for (int64_t i = (int64_t)blockIdx.x * kThreads + threadIdx.x; i < total;
         i += (int64_t)gridDim.x * kThreads) {
        float s = 0.0f;
        for (int k = 0; k < splits; ++k) s += part[(int64_t)k * total + i];
        if (kMapMask && !map_mask[i % nvox]) s = 0.0f;
        out[i] = accumulate ? out[i] + s : s;
    }
}

BlockedShape blocked_shape(const Plan &p, const tomo_tuning &tu)
{
    BlockedShape bs;
    bs.b[0] = tu.bp_block[0];
    bs.b[1] = tu.bp_block[1];
    bs.b[2] = tu.bp_block[2];
    bs.nt = tu.bp_threads == 512 || tu.bp_threads == 1024 ? tu.bp_threads : 256;
    int64_t nblk = 1;
    for (int a = 0; a < 3; ++a) {
        bs.nb[a] = (p.grid.n[a] + bs.b[a] - 1) / bs.b[a];
        nblk *= bs.nb[a];
    }
    nblk *= p.grid.nframes;
    int s = tu.bp_splits;
    if (s <= 0) {  // enough owners for about two rounds of the resident workgroups
        const int64_t want = 2048 * 256 / bs.nt;
        s = (int)((want + nblk - 1) / nblk);
        s = s < 1 ? 1 : (s > 8 ? 8 : s);
    }
    if (s > p.min_frame_views && p.min_frame_views >= 1) s = p.min_frame_views;
    bs.splits = s < 1 ? 1 : s;
    bs.items = nblk * bs.splits;
    return bs;
}

static size_t align256(size_t b) { return (b + 255) & ~(size_t)255; }

// Scratch layout: per-view partial maxima; the owners' partial sums (when
// blocks have several owners); the kept-pixel rows (row intervals over a
// data mask).
struct BlockedScratch {
    uint32_t *ymax;
    float *part;
    KeptRows kept;
};

static size_t blocked_layout(const Plan &p, const BlockedShape &bs, bool data_mask, char *base, BlockedScratch *out)
{
    size_t off = 0;
    auto take = [&](size_t bytes) {
        char *q = base ? base + off : nullptr;
        off += align256(bytes);
        return q;
    };
    BlockedScratch sc;
    sc.ymax = (uint32_t *)take(sizeof(uint32_t) * (size_t)p.nviews * kYmaxParts);
    sc.part = bs.splits > 1 ? (float *)take(sizeof(float) * (size_t)bs.splits * (size_t)(p.grid.nvox * p.grid.nframes))
                            : nullptr;
    sc.kept.pre = sc.kept.cols = nullptr;
    if (p.bp_rows && data_mask) {
        sc.kept.pre = (const uint16_t *)take(sizeof(uint16_t) * (size_t)p.npix);
        sc.kept.cols = (const uint16_t *)take(sizeof(uint16_t) * (size_t)p.npix);
    }
    if (out) *out = sc;
    return off;
}

size_t blocked_scratch_bytes(const Plan &p, const BlockedShape &bs, bool data_mask)
{
    return blocked_layout(p, bs, data_mask, nullptr, nullptr);
}

int kept_rows_launch(const Plan &p, const ViewDev *views, int32_t nviews, const uint8_t *data_mask, uint16_t *pre,
                     uint16_t *cols, hipStream_t s, const int *done_flag)
{
    const int32_t max_rows = p.max_nrow > 0 ? p.max_nrow : 1;
    const dim3 grid((unsigned)((max_rows + kThreads / 64 - 1) / (kThreads / 64)),
                    (unsigned)(nviews < 65535 ? nviews : 65535));
    hipLaunchKernelGGL(k_kept_rows, grid, dim3(kThreads), 0, s, views, nviews, data_mask, pre, cols, done_flag);
    return hip_fail(hipGetLastError(), "kept-row kernel launch");
}

int blocked_static_lds(int nt, bool rows)
{
    switch (nt) {
    case 512: return rows ? (int)sizeof(BlockedShared<512, true>) : (int)sizeof(BlockedShared<512, false>);
    case 1024: return rows ? (int)sizeof(BlockedShared<1024, true>) : (int)sizeof(BlockedShared<1024, false>);
    default: return rows ? (int)sizeof(BlockedShared<256, true>) : (int)sizeof(BlockedShared<256, false>);
    }
}

// Largest LDS a workgroup may take on the current device (static + dynamic).
static size_t lds_limit()
{
    static size_t cached = 0;
    if (!cached) {
        int dev = 0, v = 0;
        (void)hipGetDevice(&dev);
        if (hipDeviceGetAttribute(&v, hipDeviceAttributeMaxSharedMemoryPerBlock, dev) != hipSuccess || v <= 0)
            v = 65536;
        cached = (size_t)v;
    }
    return cached;
}

int blocked_check_lds(const BlockedShape &bs, bool rows, size_t *dyn_out)
{
    const size_t dyn = sizeof(unsigned long long) * ((size_t)bs.b[0] * bs.b[1] * bs.b[2] + 1);  // + dummy bin
    if (dyn_out) *dyn_out = dyn;
    if (dyn + (size_t)blocked_static_lds(bs.nt, rows) > lds_limit())
        return set_error(TOMO_EINVAL, "blocked back-projection: a %dx%dx%d block with %d lanes needs %zu bytes of "
                                      "LDS, above the %zu a workgroup may take",
                         bs.b[0], bs.b[1], bs.b[2], bs.nt, dyn + (size_t)blocked_static_lds(bs.nt, rows),
                         lds_limit());
    return TOMO_OK;
}

// Raises a kernel's dynamic-LDS limit when a launch needs more than the
// default 64 KiB.
template <class K>
static int allow_lds(K kernel, size_t dyn)
{
    if (dyn <= 65536) return TOMO_OK;
    return hip_fail(hipFuncSetAttribute(reinterpret_cast<const void *>(kernel),
                                        hipFuncAttributeMaxDynamicSharedMemorySize, (int)dyn),
                    "dynamic LDS attribute");
}

template <int NT>
static int launch_blocked_nt(const Plan &p, const tomo_geometry *g, const BlockDev &bd, const Bundle &bun,
                             const BlockedShape &bs, size_t lds, const float *images, const KeptRows &kept,
                             const uint32_t *ymax, float *dst, int acc, bool mm, bool dm, hipStream_t s,
                             const int *done_flag, const RayTable &tab)
{
    int rc = TOMO_OK;
#define TOMO_LAUNCH_BK4(M, D, O, R)                                                                             \
    do {                                                                                                        \
        rc = allow_lds(k_backproject_blocked<NT, M, D, O, R>, lds);                                             \
        if (!rc)                                                                                                \
            hipLaunchKernelGGL((k_backproject_blocked<NT, M, D, O, R>), dim3((unsigned)bs.items), dim3(NT), lds, \
                               s, p.grid, p.views_d, p.frame_views_d, p.frame_voff_d, bd, bun, images,          \
                               g->map_mask, g->data_mask, kept, ymax, dst, acc, done_flag, p.spill_d, tab);    \
    } while (0)
#define TOMO_LAUNCH_BK3(M, D, O)                       \
    do {                                               \
        if (p.bp_rows) TOMO_LAUNCH_BK4(M, D, O, true); \
        else TOMO_LAUNCH_BK4(M, D, O, false);          \
    } while (0)
#define TOMO_LAUNCH_BK(M, D)                             \
    do {                                                 \
        if (p.grid.has_sph) TOMO_LAUNCH_BK3(M, D, true); \
        else TOMO_LAUNCH_BK3(M, D, false);               \
    } while (0)
    if (mm && dm) TOMO_LAUNCH_BK(true, true);
    else if (mm) TOMO_LAUNCH_BK(true, false);
    else if (dm) TOMO_LAUNCH_BK(false, true);
    else TOMO_LAUNCH_BK(false, false);
#undef TOMO_LAUNCH_BK
#undef TOMO_LAUNCH_BK3
#undef TOMO_LAUNCH_BK4
    return rc ? rc : hip_fail(hipGetLastError(), "blocked back-projection kernel launch");
}

int launch_backproject_blocked(const Plan &p, const tomo_geometry *g, const float *images, float *cube,
                               bool accumulate, bool use_map_mask, hipStream_t s, const int *done_flag,
                               void *scratch, size_t scratch_bytes, const tomo_tuning &tu, const RayTable *tab)
{
    const BlockedShape bs = blocked_shape(p, tu);
    const RayTable rt = tab ? *tab : RayTable{};
    if (rt.d && rt.n != p.npix)
        return set_error(TOMO_EINVAL, "blocked back-projection: ray table of another geometry");
    const bool mm = use_map_mask && g->map_mask, dm = g->data_mask != nullptr;
    const size_t need = blocked_scratch_bytes(p, bs, dm);
    if (!scratch || scratch_bytes < need)
        return set_error(TOMO_EINVAL, "blocked back-projection: scratch of %zu bytes needed", need);
    if (bs.items >= ((int64_t)1 << 31)) return set_error(TOMO_EINVAL, "blocked back-projection: too many blocks");
    size_t lds = 0;
    int rc = blocked_check_lds(bs, p.bp_rows, &lds);
    if (rc) return rc;
    BlockedScratch sc;
    blocked_layout(p, bs, dm, (char *)scratch, &sc);
    if (dm)
        hipLaunchKernelGGL(k_view_absmax<true>, dim3((unsigned)(p.nviews * kYmaxParts)), dim3(kThreads), 0, s,
                           p.views_d, images, g->data_mask, sc.ymax, done_flag);
    else
        hipLaunchKernelGGL(k_view_absmax<false>, dim3((unsigned)(p.nviews * kYmaxParts)), dim3(kThreads), 0, s,
                           p.views_d, images, g->data_mask, sc.ymax, done_flag);
    if (sc.kept.cols) {
        rc = kept_rows_launch(p, p.views_d, p.nviews, g->data_mask, const_cast<uint16_t *>(sc.kept.pre),
                              const_cast<uint16_t *>(sc.kept.cols), s, done_flag);
        if (rc) return rc;
    }
    BlockDev bd;
    for (int a = 0; a < 3; ++a) {
        bd.b[a] = bs.b[a];
        bd.nb[a] = bs.nb[a];
    }
    bd.splits = bs.splits;
    bd.maxit = bs.b[0] + bs.b[1] + bs.b[2] + 3;
    const Bundle bun{tu.bp_bundle, tu.bp_xcd_remap};
    float *dst = bs.splits == 1 ? cube : sc.part;
    const int acc = accumulate ? 1 : 0;
    switch (bs.nt) {
    case 512:
        rc = launch_blocked_nt<512>(p, g, bd, bun, bs, lds, images, sc.kept, sc.ymax, dst, acc, mm, dm, s, done_flag,
                                    rt);
        break;
    case 1024:
        rc = launch_blocked_nt<1024>(p, g, bd, bun, bs, lds, images, sc.kept, sc.ymax, dst, acc, mm, dm, s,
                                     done_flag, rt);
        break;
    default:
        rc = launch_blocked_nt<256>(p, g, bd, bun, bs, lds, images, sc.kept, sc.ymax, dst, acc, mm, dm, s, done_flag,
                                    rt);
    }
    if (rc || bs.splits == 1) return rc;
    const int64_t total = p.grid.nvox * p.grid.nframes;
    int64_t nb = (total + kThreads - 1) / kThreads;
    nb = nb > 4096 ? 4096 : nb;
    if (mm)
        hipLaunchKernelGGL(k_sum_owners<true>, dim3((unsigned)nb), dim3(kThreads), 0, s, sc.part, bs.splits, total,
                           p.grid.nvox, g->map_mask, cube, acc, done_flag);
    else
        hipLaunchKernelGGL(k_sum_owners<false>, dim3((unsigned)nb), dim3(kThreads), 0, s, sc.part, bs.splits, total,
                           p.grid.nvox, g->map_mask, cube, acc, done_flag);
    return hip_fail(hipGetLastError(), "owner sum kernel launch");
}

}  // namespace tomo

// ---------------------------------------------------------------------------
// The allocation-free transpose.  Its scratch (the per-view maxima, the
// owners' partial sums when blocks have several owners, the kept-pixel row
// tables under a data mask) lives in a static device array instead of
// stream-ordered memory; every byte of it that a launch reads, the same
// launch writes first, so nothing needs clearing between calls.  In host code the array's
// name stands for a host-side shadow, not for device memory: the array's
// device address is taken once per GPU with hipGetSymbolAddress and only
// that address is handed to kernels.

#include <mutex>

namespace tomo {

constexpr size_t kNoAllocScratch = TOMO_NOALLOC_SCRATCH_BYTES;
constexpr int kMaxDevices = 64;

__device__ __align__(256) unsigned char scratch[kNoAllocScratch];

static std::mutex g_scratch_mu;
static void *g_scratch_ptr[kMaxDevices];

// Device address of this GPU's copy of `scratch` (looked up on the first
// call on each device, with that device current).
static int noalloc_scratch(void **out)
{
    int dev = 0;
    int rc = hip_fail(hipGetDevice(&dev), "tomo_backproject_noalloc: current device");
    if (rc) return rc;
    if (dev < 0 || dev >= kMaxDevices)
        return set_error(TOMO_EUNSUPPORTED, "tomo_backproject_noalloc: device %d beyond %d", dev, kMaxDevices);
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void *p = nullptr;
        rc = hip_fail(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)), "tomo_backproject_noalloc: scratch address");
        if (rc) return rc;
        if (!p) return set_error(TOMO_EHIP, "tomo_backproject_noalloc: scratch address is NULL");
        g_scratch_ptr[dev] = p;
    }
    *out = g_scratch_ptr[dev];
    return TOMO_OK;
}

}  // namespace tomo

extern "C" int tomo_backproject_noalloc(const tomo_geometry *g, const float *images_d, float *cube_d,
                                        int accumulate, tomo_stream stream)
{
    using namespace tomo;
    if (!cube_d || !images_d) return set_error(TOMO_EINVAL, "tomo_backproject_noalloc: NULL array");
    int st = TOMO_OK;
    PlanRef p = get_plan(g, &st, false);
    if (!p) return st;
    const tomo_tuning tu = tuning_for(*p);
    const BlockedShape bs = blocked_shape(*p, tu);
    const size_t need = blocked_scratch_bytes(*p, bs, g->data_mask != nullptr);
    if (need > kNoAllocScratch)
        return set_error(TOMO_EINVAL,
                         "tomo_backproject_noalloc: %zu bytes of scratch needed (%d owners per block over %lld "
                         "voxels), above the %zu-byte static array",
                         need, bs.splits, (long long)(p->grid.nvox * p->grid.nframes), kNoAllocScratch);
    void *sp = nullptr;
    const int rc = noalloc_scratch(&sp);
    if (rc) return rc;
    return launch_backproject_blocked(*p, g, images_d, cube_d, accumulate != 0, true, (hipStream_t)stream,
                                      nullptr, sp, kNoAllocScratch, tu);
}
