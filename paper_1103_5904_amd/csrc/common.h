// Internal definitions shared by the libtomo HIP sources (gfx950 only).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <memory>

#include "../../include/tomo.h"

namespace tomo {

constexpr int kThreads = 256;  // every kernel uses 256-lane workgroups
constexpr int kTile = 16;      // a projector workgroup covers 16x16 pixels
constexpr double kFar = 1.0e300;  // "never crossed" (finite: keeps fmin cheap)

// Per-view constants, built in FP64 on the host from a tomo_view.
struct ViewDev {
    double o[3];        // observer
    double w[3];        // tangent point direction
    double u[3];        // +column direction
    double v[3];        // +row direction
    double cd[2];       // cdelt (radians per pixel)
    double cp[2];       // crpix (0-based)
    double gain;        // instrument gain: the view's rows of P are scaled by it
    int64_t pix_off;    // first pixel of the view in the image vector
    int64_t tile_off;   // first 16x16 tile of the view in a launch
    int32_t ncol, nrow;
    int32_t tiles_x;    // tiles per image row
    int32_t frame;
};

// Voxel grid, passed to kernels by value.
struct GridDev {
    int32_t n[3];
    int32_t nframes;
    double lo[3];
    double hi[3];
    double delta[3];
    double inv_delta[3];  // 1 / delta
    int64_t nvox;       // voxels per frame
    double sph[4];      // opaque sphere: centre, radius (valid when has_sph)
    int32_t has_sph;
    int32_t pad;
};

// Wave-level ray bundle inside a 16x16 tile: each 64-lane wavefront takes a
// bw x bh block of pixels (bw * bh == 64), and the four wavefronts tile the
// 16x16 workgroup tile; or (log2_bw == 0) each wavefront takes every other
// pixel of the tile in both directions, offset by its index.
struct Bundle {
    int32_t log2_bw;    // 3 -> 8x8, 4 -> 16x4, 2 -> 4x16, 0 -> interleaved
    int32_t xcd_remap;  // tile order (xcd_order): 0 launch order, 1 a run per XCD, 2 runs per XCD in step
};

// Owner-computes P^T launch shape (device copy).
struct BlockDev {
    int32_t b[3];     // block dimensions (voxels)
    int32_t nb[3];    // blocks per axis
    int32_t splits;   // owners per block (views dealt round-robin)
    int32_t maxit;    // bound on in-block segments per ray
};

// Raw buffer resource over [base, base + bytes): loads outside the range
// return 0 and stores/atomics outside it are dropped by the hardware.
__device__ inline __amdgpu_buffer_rsrc_t make_rsrc(const void *base, uint32_t bytes)
{
    return __builtin_amdgcn_make_buffer_rsrc(const_cast<void *>(base), (short)0, (int)bytes,
                                             0x00020000);
}

__device__ inline float buf_load_f32(__amdgpu_buffer_rsrc_t r, uint32_t byte_off)
{
    return __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(r, (int)byte_off, 0, 0));
}

__device__ inline uint32_t buf_load_u8(__amdgpu_buffer_rsrc_t r, uint32_t byte_off)
{
    return (uint32_t)__builtin_amdgcn_raw_buffer_load_b8(r, (int)byte_off, 0, 0);
}

// "v is not +-0", decided on the bit pattern: true for NaN even in code
// built without NaN semantics, so NaN data keeps propagating.
__device__ inline bool nonzero_bits(float v) { return (__builtin_bit_cast(uint32_t, v) << 1) != 0u; }

__device__ inline void buf_atomic_add_f32(__amdgpu_buffer_rsrc_t r, uint32_t byte_off, float v)
{
    __builtin_amdgcn_raw_ptr_buffer_atomic_fadd_f32(v, r, (int)byte_off, 0, 0);
}

// MI355X hands consecutive workgroups to its 8 XCDs in turn.  Remapping the
// block index gives each XCD (and its L2) one contiguous run of tiles, so
// the blocks resident on an XCD walk neighbouring rays through the same part
// of the cube.  Bijective on [0, nb).
__device__ inline int64_t xcd_remap(int64_t b, int64_t nb)
{
    const int64_t q = nb >> 3, r = nb & 7;
    const int64_t x = b & 7, i = b >> 3;
    return x * q + (x < r ? x : r) + i;
}

// The same with runs of kXcdChunk: each group of 8 kXcdChunk consecutive
// workgroup ids covers 8 kXcdChunk consecutive tiles, kXcdChunk of them
// (contiguous) per XCD.  All XCDs then advance through the tile list
// together, so the data they touch at one time stays a window of it (one
// frame of a multi-frame cube, not eight), while each XCD's L2 still sees
// neighbouring tiles.  The ragged last group keeps the identity.  Bijective
// on [0, nb).
constexpr int64_t kXcdChunk = 64;
__device__ inline int64_t xcd_remap_chunked(int64_t b, int64_t nb)
{
    const int64_t g = b / (8 * kXcdChunk);
    if ((g + 1) * 8 * kXcdChunk > nb) return b;
    const int64_t w = b - g * 8 * kXcdChunk;
    return g * 8 * kXcdChunk + (w & 7) * kXcdChunk + (w >> 3);
}

// Tile order of a launch: 0 = launch order, 1 = one contiguous run per
// XCD, 2 = runs of kXcdChunk per XCD advancing together.
__device__ inline int64_t xcd_order(int32_t mode, int64_t b, int64_t nb)
{
    return mode == 1 ? xcd_remap(b, nb) : (mode == 2 ? xcd_remap_chunked(b, nb) : b);
}

// Sum of one double per thread over a 256-thread block; the result is valid
// in thread 0.  Fixed order, so deterministic.
__device__ inline double block_sum(double v, double *lds /* >= 4 */)
{
    for (int o = 32; o > 0; o >>= 1) v += __shfl_down(v, o, 64);
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    if (lane == 0) lds[wid] = v;
    __syncthreads();
    double s = 0.0;
    if (threadIdx.x == 0) s = (lds[0] + lds[1]) + (lds[2] + lds[3]);
    __syncthreads();
    return s;
}

__device__ inline int64_t block_sum_i64(int64_t v, int64_t *lds /* >= 4 */)
{
    for (int o = 32; o > 0; o >>= 1) v += __shfl_down(v, o, 64);
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    if (lane == 0) lds[wid] = v;
    __syncthreads();
    int64_t s = 0;
    if (threadIdx.x == 0) s = (lds[0] + lds[1]) + (lds[2] + lds[3]);
    __syncthreads();
    return s;
}

// ------------------------------------------------------------ host side

// Device copy of a geometry's view table plus launch constants.
struct Plan {
    GridDev grid;
    ViewDev *views_d = nullptr;  // device [nviews], freed with the plan
    int32_t nviews = 0;
    int64_t ntiles = 0;          // 16x16 tiles over all views
    int64_t npix = 0;            // total pixels
    int32_t max_steps = 0;       // bound on segments per ray
    int32_t max_nrow = 0;        // most image rows of any view
    unsigned *spill_d = nullptr; // device counter: binned writes that missed their LDS box
    int32_t *frame_views_d = nullptr;  // device [nviews]: view indices grouped by frame
    int32_t *frame_voff_d = nullptr;   // device [nframes + 1]: offsets into frame_views_d
    int32_t min_frame_views = 0;       // fewest views any frame has
    bool bp_rows = false;              // blocked P^T walks footprint row intervals (pixels finer than voxels)
    uint64_t size_class = 0;           // key of the autotuner's cache (size_class_of)
    Plan() = default;
    Plan(const Plan &) = delete;
    Plan &operator=(const Plan &) = delete;
    ~Plan()
    {
        if (views_d) (void)hipFree(views_d);
        if (spill_d) (void)hipFree(spill_d);
        if (frame_views_d) (void)hipFree(frame_views_d);
        if (frame_voff_d) (void)hipFree(frame_voff_d);
    }
};

using PlanRef = std::shared_ptr<const Plan>;

// Returns the cached plan for g (building it on first use unless build is
// false), or null with the error recorded.  Thread-safe; a plan stays valid
// while referenced even if the cache is released.
PlanRef get_plan(const tomo_geometry *g, int *status, bool build = true);

int set_error(int status, const char *fmt, ...);
int hip_fail(hipError_t e, const char *what);
// Stream-ordered scratch from the library's memory pool (freed memory stays
// mapped for later calls, up to a bound).
hipError_t scratch_alloc(void **p, size_t bytes, hipStream_t s);
hipError_t scratch_free(void *p, hipStream_t s);
int validate_cube(const tomo_cube *c);
tomo_tuning current_tuning();
uint64_t size_class_of(const tomo_geometry *g, int64_t npix);
// The tuning launches on this plan use: its size class's autotuned entry if
// there is one, else the process-wide tuning.
tomo_tuning tuning_for(const Plan &p);

// Per-ray results of the ray set-up over a whole geometry, for launches
// that would otherwise redo the set-up of one ray many times (the blocked
// P^T sets a ray up once per block it crosses).  Built once for a geometry
// that several P^T applications share (a CG solve, a batch); the walk state
// read back is bit for bit the set-up's, so results do not change.
// Structure of arrays over the geometry's n pixels (image-vector order):
//   d[c n + i], c = 0..10: next crossing s0 s1 s2, spacing ds0 ds1 ds2, exit
//                          parameter send (0: the ray misses), |d|, and
//                          ~1 / spacing rds0 rds1 rds2 (0: axis not crossed)
//   k[i]:                  entry voxel index per axis, 20 bits each from
//                          bit 0, 20, 40; bit 60 + a set: the ray moves up axis a
struct RayTable {
    const double *d = nullptr;
    const uint64_t *k = nullptr;
    int64_t n = 0;
};
constexpr int kRayTableCols = 11;
constexpr int kRayTableSideBits = 20;  // largest cube side a table holds: 2^20 voxels
// Bytes of a plan's table (0: its cube is too large for one).
size_t ray_table_bytes(const Plan &p);
// Lays the table out over `mem` (ray_table_bytes of device memory) and
// launches its build on s.
int ray_table_build(const Plan &p, void *mem, RayTable &out, hipStream_t s);

// Launchers (siddon.hip)
int launch_project(const Plan &p, const tomo_geometry *g, const float *cube, float *images,
                   bool use_map_mask, hipStream_t s);
// The same path with an explicit tuning (the autotuner's candidates).
// A bricked copy of the cube: bricks of B = 2^k voxels a side in x-fastest
// order, x fastest inside each brick, every frame padded to whole bricks.
struct BrickDev {
    int32_t k;            // log2 of the brick side
    int32_t nb[3];        // bricks per axis
    int64_t frame_stride; // floats per padded frame
};
// The bricked layout of a plan's cube with bricks of 2^k (false: a frame
// would pass 2^32 floats), and the copy of M x into it (map_mask may be
// null; frames past the done flag's raise are skipped like any launch).
bool brick_layout(const Plan &p, int k, BrickDev &bk);
int brick_copy_launch(const Plan &p, const float *cube, const uint8_t *map_mask, const BrickDev &bk, float *out,
                      hipStream_t s, const int *done_flag);
// P from a bricked copy made by brick_copy_launch (the map mask is in it).
int launch_project_from_bricks(const Plan &p, const tomo_geometry *g, const float *br, const BrickDev &bk,
                               float *images, hipStream_t s, const int *done_flag, const tomo_tuning &tu);
int launch_project_with(const Plan &p, const tomo_geometry *g, const float *cube, float *images,
                        bool use_map_mask, hipStream_t s, const tomo_tuning &tu);
// scratch: blocked strategy only; when null the launcher takes stream-ordered
// scratch from the pool for this launch.
// tab: a built ray table of the plan, read by the blocked strategy instead
// of setting rays up (null: set up in the launch).
int launch_backproject(const Plan &p, const tomo_geometry *g, const float *images, float *cube,
                       bool accumulate, bool use_map_mask, int strategy, hipStream_t s,
                       const int *done_flag = nullptr, void *scratch = nullptr,
                       size_t scratch_bytes = 0, const RayTable *tab = nullptr);
// P of the plan's tuning without a map mask; a tuning that walks bricks
// copies the cube into `bricks` (bricked_copy_bytes of them) when given,
// else into stream-ordered scratch for this launch.
int launch_project_flagged(const Plan &p, const tomo_geometry *g, const float *cube,
                           float *images, hipStream_t s, const int *done_flag, float *bricks = nullptr);
// Bytes of the bricked copy P takes with tuning tu on this plan (0: none).
size_t bricked_copy_bytes(const Plan &p, const tomo_tuning &tu);
int launch_project_tuned(const Plan &p, const tomo_geometry *g, const float *cube, float *images,
                         bool use_map_mask, hipStream_t s, const int *done_flag, const tomo_tuning &tu);
int launch_backproject_tuned(const Plan &p, const tomo_geometry *g, const float *images, float *cube,
                             bool accumulate, bool use_map_mask, int strategy, hipStream_t s,
                             const int *done_flag, void *scratch, size_t scratch_bytes,
                             const tomo_tuning &tu, const RayTable *tab = nullptr);
int launch_fill(float *x, int64_t n, float v, hipStream_t s);
int launch_backproject_binned(const Plan &p, const tomo_geometry *g, const float *images,
                              float *cube, bool use_map_mask, hipStream_t s, const int *done_flag,
                              const tomo_tuning &tu);

// Owner-computes back-projection (blocked.hip)
struct BlockedShape {
    int32_t b[3];    // block dimensions
    int32_t nb[3];   // blocks per axis
    int32_t splits;  // owners per block
    int32_t nt;      // lanes per workgroup
    int64_t items;   // workgroups of one launch
};
BlockedShape blocked_shape(const Plan &p, const tomo_tuning &tu);
// Scratch of one blocked launch; data_mask: the geometry has a data mask.
size_t blocked_scratch_bytes(const Plan &p, const BlockedShape &bs, bool data_mask);
// Static LDS of the blocked kernel for nt lanes (with or without row
// intervals), and the check that a shape's bins fit beside it (TOMO_EINVAL
// if not; *dyn_out receives the dynamic LDS bytes).
int blocked_static_lds(int nt, bool rows);
int blocked_check_lds(const BlockedShape &bs, bool rows, size_t *dyn_out);
// Kept-pixel rows of a data mask (one wavefront per image row).
int kept_rows_launch(const Plan &p, const ViewDev *views, int32_t nviews, const uint8_t *data_mask, uint16_t *pre,
                     uint16_t *cols, hipStream_t s, const int *done_flag);
int launch_backproject_blocked(const Plan &p, const tomo_geometry *g, const float *images, float *cube,
                               bool accumulate, bool use_map_mask, hipStream_t s, const int *done_flag,
                               void *scratch, size_t scratch_bytes, const tomo_tuning &tu,
                               const RayTable *tab = nullptr);
// Strategy a TOMO_BP_* request resolves to under the plan's tuning.
int resolve_bp_strategy(const Plan &p, int strategy);

// Learned preconditioner network (convnet.hip)
size_t convnet_forward_ws_bytes(int64_t nvox);
int convnet_forward_dev(const tomo_cube &c, const float *P, const float *x, float *out,
                        const double *norm2, const uint8_t *map_mask, void *ws, hipStream_t s,
                        bool prep_frags, const int *skip);

}  // namespace tomo
