// LDS-binned transpose P^T for gfx950.
//
// The atomic P^T (one FP32 atomic per ray/voxel segment) is limited by the
// L2 serialising same-address atomics: the 64 neighbouring rays of a
// wavefront cross the same few voxels at every step.  Here a workgroup
// keeps its partial sums in LDS instead:
//
// * The workgroup's 16x16 rays (one view) are nearly parallel and form a
//   thin pencil through the cube.  Let D be the axis the tile's central ray
//   crosses most often.  The pencil is processed in chunks of consecutive
//   D-slabs, in the direction of travel.
// * For a chunk of slabs [clo, chi], the voxels the bundle can touch lie in
//   an axis-aligned box: the rays' positions on any D-plane lie in the
//   convex hull of the four corner rays' positions (a pinhole maps the pixel
//   rectangle to a convex set on a plane), and positions are linear in the
//   D coordinate, so the extremes over the chunk are at its two end planes.
//   One voxel of margin on each side absorbs rounding and the step taken
//   when a ray leaves the chunk.  The chunk length is the largest that keeps
//   the box within the LDS budget.
// * Each ray walks exactly as in P (same set-up and walk arithmetic, so the
//   matrix is the transpose of P's), but tracks its voxel as an offset in the
//   LDS box and adds length * value there.  At the chunk's far D-plane it
//   stops, converts its LDS offset back to voxel coordinates and waits for
//   the next chunk.
// * The LDS bins hold 64-bit fixed-point sums, added with integer LDS
//   atomics: on gfx950 an LDS FP32 atomic add costs ~3 cycles per lane
//   whatever the addresses, an integer one a few cycles per wavefront.  The
//   tile's scale is a power of two chosen from its largest |y| so that no bin
//   can exceed 2^61 (at most 256 rays x voxel diagonal x max |y| per bin);
//   the rounding of one contribution is then below 2^-53 of the largest
//   possible one.  Integer sums are exact, so the LDS stage does not depend
//   on the order of additions.
// * Between chunks the workgroup flushes the box: one global FP32 atomic per
//   non-zero bin (the map mask is applied here), then clears it.
// * Tiles whose corner rays do not all travel the same way along D, or whose
//   box would not fit the LDS budget even for one slab (very wide pixels,
//   observers next to the box), fall back to one global atomic per segment.
#include <limits.h>

#include "walk.h"

namespace tomo {

constexpr int kMaxChunk = 256;   // slabs per chunk at most

// Corner ray of the tile, in voxel units, parametrised by the D coordinate:
// position on axis a at D = c is q[a] + (c - q[D]) * rat[a].
struct Corner {
    double q[3];
    double rat[3];
};

// The box bounds carry a voxel of margin, so reciprocals stand in for
// divisions here.
__device__ inline void corner_ray(const GridDev &g, const ViewDev &v, int col, int row, int D,
                                  const double *inv_delta, Corner &c, double &gD)
{
    const double x = ((double)col - v.cp[0]) * v.cd[0];
    const double y = ((double)row - v.cp[1]) * v.cd[1];
    double G[3];
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        G[a] = (v.w[a] + x * v.u[a] + y * v.v[a]) * inv_delta[a];
        c.q[a] = (v.o[a] - g.lo[a]) * inv_delta[a];
    }
    gD = G[D];
    const double r = 1.0 / G[D];
#pragma unroll
    for (int a = 0; a < 3; ++a) c.rat[a] = G[a] * r;
}

// Voxel-index range [lo, hi] on axis a touched between the D-planes c0 and
// c1, with one voxel of margin, clamped to the grid.
__device__ inline void axis_range(const Corner *cr, int a, int D, double c0, double c1, int n,
                                  int &lo, int &hi)
{
    double mn = 1e300, mx = -1e300;
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        const double p0 = cr[k].q[a] + (c0 - cr[k].q[D]) * cr[k].rat[a];
        const double p1 = cr[k].q[a] + (c1 - cr[k].q[D]) * cr[k].rat[a];
        mn = fmin(mn, fmin(p0, p1));
        mx = fmax(mx, fmax(p0, p1));
    }
    lo = clampi((int)floor(mn) - 1, 0, n - 1);
    hi = clampi((int)floor(mx) + 1, 0, n - 1);
}

template <bool kMapMask, bool kDataMask>
__global__ __launch_bounds__(kThreads) void k_backproject_binned(
    GridDev g, const ViewDev *__restrict__ views, int32_t nviews, Bundle bun, int32_t maxit,
    const float *__restrict__ images, const uint8_t *__restrict__ map_mask,
    const uint8_t *__restrict__ data_mask, float *__restrict__ cube,
    const int *__restrict__ done_flag, unsigned *__restrict__ spill, int32_t kBinCap)
{
    extern __shared__ unsigned long long bins[];  // kBinCap 64-bit fixed-point sums
    __shared__ int range[2];
    __shared__ unsigned ymax_bits;
    __shared__ Corner s_cr[4];
    __shared__ double s_gd[4];
    if (done_flag && *done_flag) return;

    const int64_t tile = block_tile(bun);
    const LanePixel lp = lane_pixel(views, nviews, tile, bun.log2_bw);
    const ViewDev &v = views[lp.view];
    const auto rc = make_rsrc(cube + (int64_t)v.frame * g.nvox, (uint32_t)(g.nvox * 4));
    const int32_t gstride[3] = {1, g.n[0], g.n[0] * g.n[1]};

    // ---- this lane's ray
    RayState r;
    RayAxes ax;
    bool active = false;
    double wy = 0.0;
    float yv = 0.0f;
    if (lp.col < v.ncol && lp.row < v.nrow) {
        const int64_t pix = v.pix_off + (int64_t)lp.row * v.ncol + lp.col;
        yv = images[pix];
        if (nonzero_bits(yv) && (!kDataMask || data_mask[pix]) && ray_setup(g, v, lp.col, lp.row, r, &ax)) {
            active = true;
            wy = (double)yv * (r.dn * v.gain);
        }
    }

    // ---- tile geometry (uniform across the workgroup, corners kept in LDS)
    const int64_t t = tile - v.tile_off;
    const int c0 = (int)(t % v.tiles_x) * kTile, r0 = (int)(t / v.tiles_x) * kTile;
    const int c1 = min(c0 + kTile - 1, v.ncol - 1), r1 = min(r0 + kTile - 1, v.nrow - 1);
    const double inv_delta[3] = {1.0 / g.delta[0], 1.0 / g.delta[1], 1.0 / g.delta[2]};
    int D = 0;
    {
        const double x = (0.5 * (c0 + c1) - v.cp[0]) * v.cd[0];
        const double y = (0.5 * (r0 + r1) - v.cp[1]) * v.cd[1];
        double best = -1.0;
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            const double ga = fabs((v.w[a] + x * v.u[a] + y * v.v[a]) * inv_delta[a]);
            if (ga > best) {
                best = ga;
                D = a;
            }
        }
    }
    const int A1 = D == 0 ? 1 : 0, A2 = D == 2 ? 1 : 2;
    if (threadIdx.x < 4) {
        const int k = threadIdx.x;
        corner_ray(g, v, (k & 1) ? c1 : c0, (k & 2) ? r1 : r0, D, inv_delta, s_cr[k], s_gd[k]);
    }
    if (threadIdx.x == 0) ymax_bits = 0u;
    // D-range of the bundle: entry and exit slabs of every active ray
    if (threadIdx.x == 0) {
        range[0] = INT_MAX;
        range[1] = INT_MIN;
    }
    for (int i = threadIdx.x; i < kBinCap; i += kThreads) bins[i] = 0ull;
    __syncthreads();
    const int sD = s_gd[0] > 0.0 ? 1 : -1;
    bool binned = true;
#pragma unroll
    for (int k = 0; k < 4; ++k) binned = binned && (s_gd[k] * sD > 0.0);
    const Corner *cr = s_cr;
    if (active) {
        atomicMax(&ymax_bits, __builtin_bit_cast(uint32_t, fabsf(yv)));
        const double qx = (v.o[D] - g.lo[D]) * inv_delta[D];
        const double xe = ((double)lp.col - v.cp[0]) * v.cd[0];
        const double ye = ((double)lp.row - v.cp[1]) * v.cd[1];
        const double dD = v.w[D] + xe * v.u[D] + ye * v.v[D];
        // exit slab, widened by one toward the direction of travel
        const double qexit = qx + (ax.tin + r.send) * dD * inv_delta[D];
        int ex = sD > 0 ? (int)ceil(qexit) : (int)floor(qexit) - 1;
        ex = clampi(ex, 0, g.n[D] - 1);
        const int en = ax.idx[D];
        atomicMin(&range[0], min(en, ex));
        atomicMax(&range[1], max(en, ex));
    }
    __syncthreads();
    const int dlo = range[0], dhi = range[1];
    if (dlo > dhi) return;  // no active ray (uniform)
    // non-finite data cannot be held in fixed point: such tiles take the
    // FP32-atomic path
    binned = binned && ymax_bits < 0x7f800000u;

    // fixed-point scale: every bin stays below 2^61
    const double ymax = (double)__builtin_bit_cast(float, ymax_bits) * fabs(v.gain);
    const double vdiag = sqrt(g.delta[0] * g.delta[0] + g.delta[1] * g.delta[1] + g.delta[2] * g.delta[2]);
    int eb = 0;
    (void)frexp((double)kThreads * vdiag * ymax * 1.0000001, &eb);  // bound < 2^eb
    const double fx_scale = ldexp(1.0, 61 - eb), fx_inv = ldexp(1.0, eb - 61);
    const double wys = wy * fx_scale;

    // One slab must fit everywhere in the range.  The continuous width of
    // a one-slab box is convex in its position, so its maximum is at an end
    // of the range; rounding to voxels can add one more row and column.
    if (binned) {
        int l1, h1, l2, h2;
#pragma unroll
        for (int e = 0; e < 2; ++e) {
            const double cpl = e == 0 ? dlo : dhi;
            axis_range(cr, A1, D, cpl, cpl + 1.0, g.n[A1], l1, h1);
            axis_range(cr, A2, D, cpl, cpl + 1.0, g.n[A2], l2, h2);
            binned = binned && (h1 - l1 + 2) * (h2 - l2 + 2) <= kBinCap;
        }
    }

    if (!binned) {  // uniform fall-back: one global atomic per segment
        if (active) {
            const auto rm = make_rsrc(map_mask, kMapMask ? (uint32_t)g.nvox : 0u);
            ray_walk(r, maxit, [&](int32_t off, double dl) {
                if (!kMapMask || buf_load_u8(rm, (uint32_t)off))
                    buf_atomic_add_f32(rc, (uint32_t)off * 4u, (float)(dl * wy));
            });
        }
        return;
    }

    // ---- chunked walk
    int myD = ax.idx[D], my1 = ax.idx[A1], my2 = ax.idx[A2];
    double scur = 0.0;
    int cur = sD > 0 ? dlo : dhi;
    while (sD > 0 ? cur <= dhi : cur >= dlo) {
        // largest chunk whose box fits the LDS budget
        const int remain = sD > 0 ? dhi - cur + 1 : cur - dlo + 1;
        int K = min(remain, kMaxChunk);
        int clo = 0, chi = 0, lo1 = 0, hi1 = 0, lo2 = 0, hi2 = 0, T1 = 1, T2 = 1;
        for (;;) {
            clo = sD > 0 ? cur : cur - K + 1;
            chi = sD > 0 ? cur + K - 1 : cur;
            axis_range(cr, A1, D, (double)clo, (double)(chi + 1), g.n[A1], lo1, hi1);
            axis_range(cr, A2, D, (double)clo, (double)(chi + 1), g.n[A2], lo2, hi2);
            T1 = hi1 - lo1 + 1;
            T2 = hi2 - lo2 + 1;
            if (K * T1 * T2 <= kBinCap || K == 1) break;
            K = max(1, min(K - 1, (K * 3) / 4));
        }
        const int plane = T1 * T2, tsize = min(K * plane, kBinCap);

        if (active && myD >= clo && myD <= chi) {
            int32_t loff = ((myD - clo) * T2 + (my2 - lo2)) * T1 + (my1 - lo1);
            r.st[D] = sD * plane;
            r.st[A1] = r.st[A1] > 0 ? 1 : (r.st[A1] < 0 ? -1 : 0);
            r.st[A2] = r.st[A2] > 0 ? T1 : (r.st[A2] < 0 ? -T1 : 0);
            // parameter of the chunk's far D-plane (exact on the ray's grid)
            const double sfar = r.s[D] + (double)(sD > 0 ? chi - myD : myD - clo) * r.ds[D];
            r.off = loff;
            int left = 0;  // 1: ray finished, 2: ray moved on to the next chunk
            for (int it = 0; it < maxit && !left; ++it) {
                const double m = fmin(fmin(r.s[0], r.s[1]), fmin(r.s[2], r.send));
                const long long fx = (long long)rint((m - scur) * wys);
                if ((uint32_t)r.off < (uint32_t)tsize) atomicAdd(&bins[r.off], (unsigned long long)fx);
                else atomicAdd(spill, 1u);
                if (m >= r.send) {
                    left = 1;
                    break;
                }
#pragma unroll
                for (int a = 0; a < 3; ++a) {
                    const bool tie = (r.s[a] == m);
                    r.s[a] += tie ? r.ds[a] : 0.0;
                    r.off += tie ? r.st[a] : 0;
                }
                scur = m;
                if (m >= sfar) left = 2;
            }
            if (left == 2) {  // back to voxel coordinates in the next slab
                const int lD = sD > 0 ? K : -1;
                const int rem = r.off - lD * plane;
                my1 = lo1 + rem % T1;
                my2 = lo2 + rem / T1;
                myD = sD > 0 ? chi + 1 : clo - 1;
            } else {
                active = false;
            }
        }
        __syncthreads();
        // flush the box: one global atomic per touched voxel
        for (int e = threadIdx.x; e < tsize; e += kThreads) {
            const long long acc = (long long)bins[e];
            if (acc != 0) {
                bins[e] = 0ull;
                const float val = (float)((double)acc * fx_inv);
                const int l1 = e % T1, q = e / T1;
                const int l2 = q % T2, lD = q / T2;
                const int32_t off = (clo + lD) * gstride[D] + (lo1 + l1) * gstride[A1] +
                                    (lo2 + l2) * gstride[A2];
                if (!kMapMask || map_mask[off]) buf_atomic_add_f32(rc, (uint32_t)off * 4u, val);
            }
        }
        __syncthreads();
        cur = sD > 0 ? chi + 1 : clo - 1;
    }
}

int launch_backproject_binned(const Plan &p, const tomo_geometry *g, const float *images,
                              float *cube, bool use_map_mask, hipStream_t s, const int *done_flag,
                              const tomo_tuning &tu)
{
    const Bundle b{tu.bp_bundle, tu.bp_xcd_remap};
    const int cap = tu.bp_lds_bins;
    const bool mm = use_map_mask && g->map_mask, dm = g->data_mask != nullptr;
    const dim3 grid((unsigned)p.ntiles), blk(kThreads);
    const size_t lds = sizeof(unsigned long long) * (size_t)cap;
#define TOMO_LAUNCH_BB(M, D)                                                                          \
    hipLaunchKernelGGL((k_backproject_binned<M, D>), grid, blk, lds, s, p.grid, p.views_d, p.nviews,  \
                       b, p.max_steps, images, g->map_mask, g->data_mask, cube, done_flag, p.spill_d, \
                       cap)
    if (mm && dm) TOMO_LAUNCH_BB(true, true);
    else if (mm) TOMO_LAUNCH_BB(true, false);
    else if (dm) TOMO_LAUNCH_BB(false, true);
    else TOMO_LAUNCH_BB(false, false);
#undef TOMO_LAUNCH_BB
    return hip_fail(hipGetLastError(), "binned back-projection kernel launch");
}

}  // namespace tomo
