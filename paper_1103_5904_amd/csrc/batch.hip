// Batched persistent launches over several independent systems (time-frame
// cubes and independent reconstructions of uneven sizes).
//
// * One persistent P^T launch covers every system, so that systems of very
//   different sizes share the machine without one launch per system and
//   without tail effects between them.  P, whose tiles need no owner and
//   no queue, runs each system's own tuned single-geometry launch (tile
//   shape, XCD order, cube layout; the bricked copies live in the batch);
//   a persistent P over all systems measured slower per tile than those
//   launches, whatever its register budget.  The P^T grid holds
//   as many workgroups as the chip keeps resident; each pulls (system,
//   frame, voxel block, owner) items from eight device work queues, one per
//   XCD, draining its own XCD's queue first.  The blocks are dealt to the
//   queues in runs of 4, so that the queues advance through the list
//   together and the XCDs work on one frame of a multi-frame cube at a
//   time: the images and voxels of that frame stay in the Infinity Cache
//   (eight 64 MiB frames at once do not fit).  The last workgroup to leave
//   resets the queues, so a launch needs no host-side clearing and can be
//   captured in a graph.
// * A P^T item runs the same device code as the single-geometry launch
//   (blocked_item) with the system's own owners per block; the workgroup
//   size and the largest block follow the dominant system (most rays),
//   which changes no bit of the result.  A batched result equals the
//   per-system one bit for bit.
// * The batched CG keeps one state (scalars, done flag) per system on the
//   device.  An iteration is the systems' P launches, one batched P^T and
//   three vector kernels per system; a system that has converged is skipped by every
//   kernel through its done flag.  With use_graph, the iterations of one
//   check interval are captured once as a HIP graph and replayed.
#include <math.h>
#include <stddef.h>
#include <stdint.h>
#include <string.h>

#include <vector>

#include "batch.h"
#include "blocked.h"

namespace tomo {

// Next item for this workgroup (thread 0), or -1 when every queue is empty.
// The items are dealt to the queues in runs of `chunk`: queue x holds runs
// x, x + 8, x + 16, ...  All XCDs then advance through the item list
// together (the systems and frames one at a time, so that what they read
// stays in the caches), while each drains runs of neighbouring items.
__device__ inline int64_t next_item(unsigned long long *q, int64_t total, int64_t chunk, int &visited)
{
    const int home = (int)(blockIdx.x % kQueues);
    while (visited < kQueues) {
        const int qx = (home + visited) % kQueues;
        const int64_t k = (int64_t)atomicAdd(&q[qx], 1ull);
        const int64_t i = ((k / chunk) * kQueues + qx) * chunk + k % chunk;
        if (i < total) return i;
        ++visited;
    }
    return -1;
}

// A value the whole workgroup holds alike (read from LDS after a barrier),
// declared uniform so that what is indexed by it - the system's table
// entry, its pointers and shapes - lives in scalar registers.
__device__ inline int64_t uniform(int64_t v)
{
    const uint64_t u = (uint64_t)v;
    const uint32_t lo = (uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)u);
    const uint32_t hi = (uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)(u >> 32));
    return (int64_t)(((uint64_t)hi << 32) | lo);
}

// The last workgroup out clears the queues for the next launch.
__device__ inline void leave_queues(unsigned long long *q)
{
    if (threadIdx.x == 0) {
        __threadfence();
        const unsigned long long prev = atomicAdd(&q[kQueues], 1ull);
        if (prev == gridDim.x - 1) {
            for (int k = 0; k <= kQueues; ++k) atomicExch(&q[k], 0ull);
            __threadfence();
        }
    }
}

// Largest k with begin(k) <= t (begin ascending, begin(0) == 0).
template <class F>
__device__ inline int find_system(int nsys, int64_t t, F begin)
{
    int lo = 0, hi = nsys - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (begin(mid) <= t) lo = mid;
        else hi = mid - 1;
    }
    return lo;
}

// max |y| per view share for every view of every system.
__global__ __launch_bounds__(kThreads) void k_batch_absmax(const SysDev *__restrict__ sys, int32_t nsys,
                                                           Operands ops, uint32_t *__restrict__ ymax)
{
    __shared__ uint32_t red[kThreads / 64];
    const int gv = blockIdx.x / kYmaxParts, part = blockIdx.x % kYmaxParts;
    const int k = find_system(nsys, gv, [&](int i) { return (int64_t)sys[i].view_begin; });
    if (ops.done[k] && *ops.done[k]) return;
    const SysDev &sd = sys[k];
    const ViewDev &v = sd.views[gv - sd.view_begin];
    const uint32_t m = sd.data_mask ? view_absmax_part<true>(v, part, ops.src[k], sd.data_mask, red)
                                    : view_absmax_part<false>(v, part, ops.src[k], sd.data_mask, red);
    if (threadIdx.x == 0) ymax[blockIdx.x] = m;
}

template <int NT, bool kRows>
__global__ __launch_bounds__(NT) __attribute__((amdgpu_waves_per_eu(4))) void k_batch_backproject(
    const SysDev *__restrict__ sys, int32_t nsys, Operands ops, int64_t nitems, const uint32_t *__restrict__ ymax,
    unsigned long long *q, unsigned *__restrict__ spill)
{
    extern __shared__ unsigned long long bins[];
    __shared__ BlockedShared<NT, kRows> sh;
    __shared__ int64_t s_item;
    int visited = 0;
    for (;;) {
        if (threadIdx.x == 0) s_item = next_item(q, nitems, 4, visited);
        __syncthreads();
        const int64_t t = uniform(s_item);
        __syncthreads();
        if (t < 0) break;
        const int k = find_system(nsys, t, [&](int i) { return sys[i].item_begin; });
        if (ops.done[k] && *ops.done[k]) continue;
        const SysDev &sd = sys[k];
        const int64_t li = t - sd.item_begin;
        float *out = sd.bd.splits == 1 ? ops.dst[k] : sd.part;
        const uint32_t *ym = ymax + (int64_t)sd.view_begin * kYmaxParts;
        const bool mm = ops.map && sd.map_mask, dm = sd.data_mask != nullptr;
        const KeptRows kept{sd.kept_pre, sd.kept_cols};
#define TOMO_ITEM(M, D, O)                                                                                      \
    blocked_item<NT, M, D, O, kRows>(sd.grid, sd.views, sd.frame_views, sd.frame_voff, sd.bd, li, ops.src[k],  \
                                     sd.map_mask, sd.data_mask, kept, ym, out, ops.acc, spill, sd.tab, bins, sh)
        if (sd.grid.has_sph) {  // the obstacle's variant: one code path for every mask combination
            if (mm && dm) TOMO_ITEM(true, true, true);
            else if (mm) TOMO_ITEM(true, false, true);
            else if (dm) TOMO_ITEM(false, true, true);
            else TOMO_ITEM(false, false, true);
        } else if (mm && dm) {
            TOMO_ITEM(true, true, false);
        } else if (mm) {
            TOMO_ITEM(true, false, false);
        } else if (dm) {
            TOMO_ITEM(false, true, false);
        } else {
            TOMO_ITEM(false, false, false);
        }
#undef TOMO_ITEM
    }
    leave_queues(q);
}

// Systems whose blocks have several owners: dst = M (sum of the owners'
// partials, in owner order) (+ dst).
__global__ __launch_bounds__(kThreads) void k_batch_sum_owners(const SysDev *__restrict__ sys, int32_t nsys,
                                                               Operands ops)
{
    for (int k = 0; k < nsys; ++k) {
        const SysDev &sd = sys[k];
        if (sd.bd.splits <= 1 || (ops.done[k] && *ops.done[k])) continue;
        float *dst = ops.dst[k];
        const bool mm = ops.map && sd.map_mask;
        for (int64_t i = (int64_t)blockIdx.x * kThreads + threadIdx.x; i < sd.ntot;
             i += (int64_t)gridDim.x * kThreads) {
            float s = 0.0f;
            for (int o = 0; o < sd.bd.splits; ++o) s += sd.part[(int64_t)o * sd.ntot + i];
            if (mm && !sd.map_mask[i % sd.grid.nvox]) s = 0.0f;
            dst[i] = ops.acc ? dst[i] + s : s;
        }
    }
}

}  // namespace tomo

using namespace tomo;


tomo_batch_s::~tomo_batch_s()
{
    int cur = 0;
    (void)hipGetDevice(&cur);
    (void)hipSetDevice(device);
    (void)hipDeviceSynchronize();
    if (sys_d) (void)hipFree(sys_d);
    if (q) (void)hipFree(q);
    if (ymax) (void)hipFree(ymax);
    if (part) (void)hipFree(part);
    if (kept) (void)hipFree(kept);
    if (bricks) (void)hipFree(bricks);
    if (tables) (void)hipFree(tables);
    if (spill) (void)hipFree(spill);
    (void)hipSetDevice(cur);
}

namespace tomo {

int batch_project_ops(tomo_batch b, const Operands &h, hipStream_t s)
{
    // each system's own tuned P (tile shape, XCD order, cube layout), the
    // bricked copies in the batch's buffers
    for (int k = 0; k < b->nsys; ++k) {
        const SysDev &sd = b->sys_h[(size_t)k];
        const Plan &p = *b->plans[(size_t)k];
        const tomo_geometry *g = &b->geoms[(size_t)k];
        const tomo_tuning &tu = b->tunings[(size_t)k];
        int rc;
        if (sd.bricked) {
            rc = brick_copy_launch(p, h.src[k], h.map ? sd.map_mask : nullptr, sd.bk, sd.bricked, s, h.done[k]);
            if (!rc) rc = launch_project_from_bricks(p, g, sd.bricked, sd.bk, h.dst[k], s, h.done[k], tu);
        } else {
            rc = launch_project_tuned(p, g, h.src[k], h.dst[k], h.map != 0, s, h.done[k], tu);
        }
        if (rc) return rc;
    }
    return TOMO_OK;
}

// The persistent P^T kernel for a batch's workgroup size and row mode.
template <int NT, bool kRows>
static const void *batch_bp_kernel()
{
    return reinterpret_cast<const void *>(k_batch_backproject<NT, kRows>);
}

static const void *batch_bp_kernel_for(int nt, bool rows)
{
    switch (nt) {
    case 512: return rows ? batch_bp_kernel<512, true>() : batch_bp_kernel<512, false>();
    case 1024: return rows ? batch_bp_kernel<1024, true>() : batch_bp_kernel<1024, false>();
    default: return rows ? batch_bp_kernel<256, true>() : batch_bp_kernel<256, false>();
    }
}

int batch_backproject_ops(tomo_batch b, const Operands &ops, hipStream_t s)
{
    hipLaunchKernelGGL(k_batch_absmax, dim3((unsigned)(b->nviews * kYmaxParts)), dim3(kThreads), 0, s,
                       b->sys_d, b->nsys, ops, b->ymax);
    for (int k = 0; k < b->nsys; ++k) {  // the kept pixels of data masks, for row intervals
        const SysDev &sd = b->sys_h[(size_t)k];
        if (!sd.kept_cols) continue;
        const int rc = kept_rows_launch(*b->plans[(size_t)k], sd.views, sd.nviews, sd.data_mask, sd.kept_pre,
                                        sd.kept_cols, s, ops.done[k]);
        if (rc) return rc;
    }
#define TOMO_BATCH_BP(NT, R)                                                                                     \
    hipLaunchKernelGGL((k_batch_backproject<NT, R>), dim3(b->grid_b), dim3(NT), b->lds_bytes, s, b->sys_d, b->nsys, \
                       ops, b->nitems, b->ymax, b->q, b->spill)
    if (b->nt == 512) {
        if (b->rows) TOMO_BATCH_BP(512, true);
        else TOMO_BATCH_BP(512, false);
    } else if (b->nt == 1024) {
        if (b->rows) TOMO_BATCH_BP(1024, true);
        else TOMO_BATCH_BP(1024, false);
    } else {
        if (b->rows) TOMO_BATCH_BP(256, true);
        else TOMO_BATCH_BP(256, false);
    }
#undef TOMO_BATCH_BP
    bool owners = false;
    for (const auto &sd : b->sys_h) owners = owners || sd.bd.splits > 1;
    if (owners) {
        int64_t most = 0;
        for (const auto &sd : b->sys_h) most = sd.ntot > most ? sd.ntot : most;
        int64_t nb = (most + kThreads - 1) / kThreads;
        nb = nb > 2048 ? 2048 : (nb < 1 ? 1 : nb);
        hipLaunchKernelGGL(k_batch_sum_owners, dim3((unsigned)nb), dim3(kThreads), 0, s, b->sys_d, b->nsys, ops);
    }
    return hip_fail(hipGetLastError(), "batched back-projection launch");
}

}  // namespace tomo

extern "C" {

int tomo_batch_create(const tomo_geometry *systems, int32_t nsystems, tomo_batch *out)
{
    if (!out) return set_error(TOMO_EINVAL, "tomo_batch_create: out is NULL");
    *out = nullptr;
    if (!systems || nsystems < 1 || nsystems > kMaxSys)
        return set_error(TOMO_EINVAL, "tomo_batch_create: 1 to %d systems", kMaxSys);
    auto b = new (std::nothrow) tomo_batch_s;
    if (!b) return set_error(TOMO_ENOMEM, "tomo_batch_create: host allocation failed");
    (void)hipGetDevice(&b->device);
    b->nsys = nsystems;
    int64_t part_floats = 0, kept_pix = 0, brick_floats = 0;
    size_t table_bytes = 0;
    std::vector<size_t> table_at;  // offset of each system's ray table (SIZE_MAX: none)
    int nrows = 0;  // systems whose plans ask for footprint row intervals
    std::vector<PlanRef> plans;
    std::vector<tomo_tuning> tunings;
    for (int k = 0; k < nsystems; ++k) {
        int st = TOMO_OK;
        PlanRef p = get_plan(&systems[k], &st);
        if (!p) {
            delete b;
            return st;
        }
        plans.push_back(p);
        tunings.push_back(tuning_for(*p));
    }
    // One workgroup size and LDS size serve every item of the persistent
    // P^T: the dominant system's (most rays).  The others keep their tuned
    // blocks when those fit its LDS, else take its block shape, and keep
    // their tuned number of owners per block: with the same owners (the same
    // views summed in each owner's exact bins) the result does not depend
    // on the block shape or the workgroup size, bit for bit.
    int dom = 0;
    for (int k = 1; k < nsystems; ++k)
        if (plans[(size_t)k]->npix > plans[(size_t)dom]->npix) dom = k;
    const BlockedShape dom_bs = blocked_shape(*plans[(size_t)dom], tunings[(size_t)dom]);
    const int64_t dom_bins = (int64_t)dom_bs.b[0] * dom_bs.b[1] * dom_bs.b[2];
    std::vector<bool> bricked(nsystems, false);
    for (int k = 0; k < nsystems; ++k) {
        const PlanRef &p = plans[(size_t)k];
        tomo_tuning tu = tunings[(size_t)k];
        tu.bp_splits = blocked_shape(*p, tu).splits;
        tu.bp_threads = dom_bs.nt;
        if ((int64_t)tu.bp_block[0] * tu.bp_block[1] * tu.bp_block[2] > dom_bins)
            for (int a = 0; a < 3; ++a) tu.bp_block[a] = dom_bs.b[a];
        const BlockedShape bs = blocked_shape(*p, tu);
        SysDev sd;
        memset(&sd, 0, sizeof(sd));
        sd.grid = p->grid;
        sd.views = p->views_d;
        sd.frame_views = p->frame_views_d;
        sd.frame_voff = p->frame_voff_d;
        sd.map_mask = systems[k].map_mask;
        sd.data_mask = systems[k].data_mask;
        for (int a = 0; a < 3; ++a) {
            sd.bd.b[a] = bs.b[a];
            sd.bd.nb[a] = bs.nb[a];
        }
        sd.bd.splits = bs.splits;
        sd.bd.maxit = bs.b[0] + bs.b[1] + bs.b[2] + 3;
        sd.nviews = p->nviews;
        sd.p_log2_bw = tu.p_bundle;
        if (tu.p_layout >= 2 && brick_layout(*p, tu.p_layout, sd.bk)) {
            bricked[(size_t)k] = true;
            brick_floats += sd.bk.frame_stride * p->grid.nframes;
        }
        const size_t tb = tu.bp_ray_table ? ray_table_bytes(*p) : 0;
        table_at.push_back(tb ? table_bytes : SIZE_MAX);
        table_bytes += (tb + 255) & ~(size_t)255;
        sd.maxit = p->max_steps;
        sd.view_begin = b->nviews;
        sd.tile_begin = b->ntiles;
        sd.item_begin = b->nitems;
        sd.ntot = p->grid.nvox * p->grid.nframes;
        b->ntiles += p->ntiles;
        b->nitems += bs.items;
        b->nviews += p->nviews;
        if (bs.splits > 1) part_floats += (int64_t)bs.splits * sd.ntot;
        const size_t lds = sizeof(unsigned long long) * ((size_t)bs.b[0] * bs.b[1] * bs.b[2] + 1);  // + dummy bin
        b->lds_bytes = lds > b->lds_bytes ? lds : b->lds_bytes;
        b->nt = bs.nt;
        nrows += p->bp_rows ? 1 : 0;
        if (systems[k].data_mask) kept_pix += p->npix;
        b->plans.push_back(p);
        b->tunings.push_back(tunings[(size_t)k]);
        b->geoms.push_back(systems[k]);
        b->geoms.back().obstacle = nullptr;  // captured in the plan's grid
        b->geoms.back().gains = nullptr;     // captured in the plan's view table
        b->sys_h.push_back(sd);
    }
    if (b->ntiles >= ((int64_t)1 << 31) || b->nitems >= ((int64_t)1 << 40)) {
        delete b;
        return set_error(TOMO_EINVAL, "tomo_batch_create: too much work for one batch");
    }
    hipError_t e = hipMalloc((void **)&b->q, sizeof(unsigned long long) * (kQueues + 1));
    if (e == hipSuccess) e = hipMemset(b->q, 0, sizeof(unsigned long long) * (kQueues + 1));
    if (e == hipSuccess) e = hipMalloc((void **)&b->ymax, sizeof(uint32_t) * (size_t)b->nviews * kYmaxParts);
    if (e == hipSuccess) e = hipMalloc((void **)&b->spill, sizeof(unsigned));
    if (e == hipSuccess) e = hipMemset(b->spill, 0, sizeof(unsigned));
    if (e == hipSuccess && part_floats > 0) e = hipMalloc((void **)&b->part, sizeof(float) * (size_t)part_floats);
    b->rows = 2 * nrows > (int)b->sys_h.size();
    if (e == hipSuccess && b->rows && kept_pix > 0)
        e = hipMalloc((void **)&b->kept, 2 * sizeof(uint16_t) * (size_t)kept_pix);
    if (e == hipSuccess && brick_floats > 0) e = hipMalloc((void **)&b->bricks, sizeof(float) * (size_t)brick_floats);
    if (e == hipSuccess && table_bytes > 0) e = hipMalloc((void **)&b->tables, table_bytes);
    if (e != hipSuccess) {
        delete b;
        return set_error(TOMO_ENOMEM, "tomo_batch_create: device allocation failed (%s)", hipGetErrorString(e));
    }
    int64_t off = 0, koff = 0, boff = 0;
    for (size_t k = 0; k < b->sys_h.size(); ++k) {
        SysDev &sd = b->sys_h[k];
        if (bricked[k]) {
            sd.bricked = b->bricks + boff;
            boff += sd.bk.frame_stride * sd.grid.nframes;
        }
        if (sd.bd.splits > 1) {
            sd.part = b->part + off;
            off += (int64_t)sd.bd.splits * sd.ntot;
        }
        if (b->kept && sd.data_mask) {
            const int64_t np = b->plans[k]->npix;
            sd.kept_pre = b->kept + koff;
            sd.kept_cols = b->kept + koff + np;
            koff += 2 * np;
        }
        if (table_at[k] != SIZE_MAX) {  // the system's rays, set up once for the batch's life
            RayTable t;
            const int rc = ray_table_build(*b->plans[k], b->tables + table_at[k], t, nullptr);
            if (rc) {
                delete b;
                return rc;
            }
            sd.tab = t;
        }
    }
    if (table_bytes > 0 && (e = hipStreamSynchronize(nullptr)) != hipSuccess) {
        delete b;
        return set_error(TOMO_ENOMEM, "tomo_batch_create: ray table build failed (%s)", hipGetErrorString(e));
    }
    e = hipMalloc((void **)&b->sys_d, sizeof(SysDev) * b->sys_h.size());
    if (e == hipSuccess) e = hipMemcpy(b->sys_d, b->sys_h.data(), sizeof(SysDev) * b->sys_h.size(), hipMemcpyHostToDevice);
    if (e != hipSuccess) {
        delete b;
        return set_error(TOMO_ENOMEM, "tomo_batch_create: system table upload failed (%s)", hipGetErrorString(e));
    }
    // persistent grids: as many workgroups as stay resident, at most one per item
    int cus = 0, per_b = 0;
    (void)hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, b->device);
    {
        BlockedShape probe;
        probe.b[0] = 1;
        probe.b[1] = 1;
        probe.b[2] = (int32_t)(b->lds_bytes / sizeof(unsigned long long)) - 1;
        probe.nt = b->nt;
        const int lrc = blocked_check_lds(probe, b->rows, nullptr);
        if (lrc) {
            delete b;
            return lrc;
        }
        const void *kern = batch_bp_kernel_for(b->nt, b->rows);
        if (b->lds_bytes > 65536 &&
            hipFuncSetAttribute(kern, hipFuncAttributeMaxDynamicSharedMemorySize, (int)b->lds_bytes) != hipSuccess) {
            delete b;
            return set_error(TOMO_EHIP, "tomo_batch_create: dynamic LDS attribute");
        }
        (void)hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_b, kern, b->nt, b->lds_bytes);
    }
    cus = cus > 0 ? cus : 256;
    per_b = per_b > 0 ? per_b : 1;
    const int64_t gb = (int64_t)cus * per_b;
    b->grid_p = (unsigned)(b->ntiles > 0 ? b->ntiles : 1);  // one workgroup per tile
    b->grid_b = (unsigned)(gb < b->nitems ? gb : (b->nitems > 0 ? b->nitems : 1));
    *out = b;
    return TOMO_OK;
}

void tomo_batch_destroy(tomo_batch b) { delete b; }

int tomo_batch_project(tomo_batch b, const float *const *cubes_d, float *const *images_d, tomo_stream stream)
{
    if (!b || !cubes_d || !images_d) return set_error(TOMO_EINVAL, "tomo_batch_project: NULL argument");
    Operands ops;
    memset(&ops, 0, sizeof(ops));
    for (int k = 0; k < b->nsys; ++k) {
        if (!cubes_d[k] || !images_d[k]) return set_error(TOMO_EINVAL, "tomo_batch_project: NULL array");
        ops.src[k] = cubes_d[k];
        ops.dst[k] = images_d[k];
    }
    ops.map = 1;
    return batch_project_ops(b, ops, (hipStream_t)stream);
}

int tomo_batch_backproject(tomo_batch b, const float *const *images_d, float *const *cubes_d, int accumulate,
                           tomo_stream stream)
{
    if (!b || !cubes_d || !images_d) return set_error(TOMO_EINVAL, "tomo_batch_backproject: NULL argument");
    Operands ops;
    memset(&ops, 0, sizeof(ops));
    for (int k = 0; k < b->nsys; ++k) {
        if (!cubes_d[k] || !images_d[k]) return set_error(TOMO_EINVAL, "tomo_batch_backproject: NULL array");
        ops.src[k] = images_d[k];
        ops.dst[k] = cubes_d[k];
    }
    ops.map = 1;
    ops.acc = accumulate ? 1 : 0;
    return batch_backproject_ops(b, ops, (hipStream_t)stream);
}

int tomo_batch_binning_spills(tomo_batch b, int64_t *count_h)
{
    if (!b || !count_h) return set_error(TOMO_EINVAL, "tomo_batch_binning_spills: NULL argument");
    unsigned h = 0;
    int rc = hip_fail(hipDeviceSynchronize(), "synchronise");
    if (!rc) rc = hip_fail(hipMemcpy(&h, b->spill, sizeof(h), hipMemcpyDeviceToHost), "copy counter");
    if (!rc) rc = hip_fail(hipMemset(b->spill, 0, sizeof(unsigned)), "reset counter");
    if (!rc) *count_h = (int64_t)h;
    return rc;
}

int64_t tomo_batch_items(tomo_batch b, int32_t which)
{
    if (!b) return -1;
    return which == 0 ? b->ntiles : (which == 1 ? b->nitems : (which == 2 ? b->grid_p : b->grid_b));
}

}  // extern "C"
