// Device-side ray set-up and Siddon walk shared by every projector kernel
// (P, the two P^T strategies, the crossing counter and the trace export), so
// that all of them produce bit-identical segments.  See siddon.hip for the
// design notes.
#pragma once

#include <math.h>

#include "common.h"

namespace tomo {

struct RayState {
    double s[3];   // next crossing on each axis (ray parameter from the entry)
    double ds[3];  // parameter spacing of consecutive planes on each axis
    double send;   // exit parameter
    double dn;     // |d|: converts parameter differences to lengths
    int32_t off;   // flat offset of the current voxel within its frame
    int32_t st[3]; // signed flat stride of a step on each axis
};

__device__ inline int clampi(int v, int lo, int hi) { return v < lo ? lo : (v > hi ? hi : v); }

// n / d from a reciprocal inv ~ 1/d and one residual correction: the
// residual n - q d is exact in FP64 (fma), and q + r inv lands on the exactly
// rounded quotient whenever that quotient is representable, and within an
// ulp otherwise.  So equal quotients from equal data stay equal (ties
// between axes, entries exactly on a plane) at a fraction of a division.
__device__ inline double qdiv(double n, double d, double inv)
{
    const double q = n * inv;
    return fma(fma(-q, d, n), inv, q);
}

// 1 / d from v_rcp_f64 and two Newton steps (five instructions against the
// IEEE division's eleven); measured equal to the correctly rounded
// reciprocal on 2^22 random normal inputs.  qdiv only needs it within an ulp.
// Magnitudes near the ends of the exponent range take the IEEE division.
__device__ inline double recip(double d)
{
    const double a = fabs(d);
    if (a > 0x1p-1000 && a < 0x1p1000) {
        double r = __builtin_amdgcn_rcp(d);
        r = fma(r, fma(-d, r, 1.0), r);
        return fma(r, fma(-d, r, 1.0), r);
    }
    return 1.0 / d;
}

// Line of sight through pixel (col, row): gnomonic pinhole d = w + x u + y v.
// Returns false if the half-line misses the (half-open) box.
// Per-axis entry state, for kernels that need voxel coordinates.
struct RayAxes {
    int idx[3];     // entry voxel index on each axis
    int k0[3];      // index of the first plane crossed on each axis (after the entry)
    double tin;     // ray parameter of the entry point
    double rds[3];  // ~1 / (spacing) before its rounding to the grid (0: axis not crossed)
};

// kObstacle = false leaves out the obstacle's code (only for grids without
// one); true cuts the ray at the obstacle when the grid has one.  V is any
// view record with the pointing fields of ViewDev (o, w, u, v, cd, cp).
template <bool kObstacle = true, class V>
__device__ inline bool ray_setup(const GridDev &g, const V &v, int col, int row,
                                 RayState &r, RayAxes *ax = nullptr)
{
    const double x = ((double)col - v.cp[0]) * v.cd[0];
    const double y = ((double)row - v.cp[1]) * v.cd[1];
    double d[3];
#pragma unroll
    for (int a = 0; a < 3; ++a) d[a] = v.w[a] + x * v.u[a] + y * v.v[a];
    r.dn = sqrt(d[0] * d[0] + d[1] * d[1] + d[2] * d[2]);

    // slab clip of t >= 0 against the box (one division per axis, the
    // other quotients from its reciprocal)
    double inv[3];
#pragma unroll
    for (int a = 0; a < 3; ++a) inv[a] = d[a] != 0.0 ? recip(d[a]) : 0.0;
    double tin = 0.0, tout = kFar;
    bool inside = true;
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        if (d[a] != 0.0) {
            const double t1 = qdiv(g.lo[a] - v.o[a], d[a], inv[a]);
            const double t2 = qdiv(g.hi[a] - v.o[a], d[a], inv[a]);
            tin = fmax(tin, fmin(t1, t2));
            tout = fmin(tout, fmax(t1, t2));
        } else {
            inside = inside && (g.lo[a] <= v.o[a]) && (v.o[a] < g.hi[a]);
        }
    }
    if (!inside || !(tout > tin)) return false;

    int idx[3];
    double sf[3], ds[3], jface[3];
    const int32_t stride[3] = {1, g.n[0], g.n[0] * g.n[1]};
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        const int N = g.n[a];
        if (d[a] != 0.0) {
            // voxel entered first: half-open voxels, so a ray starting on a
            // plane belongs to the voxel on the side it moves into
            const double p = qdiv(v.o[a] + tin * d[a] - g.lo[a], g.delta[a], g.inv_delta[a]);
            const bool up = d[a] > 0.0;
            int i = up ? clampi((int)floor(p), 0, N - 1) : clampi((int)ceil(p) - 1, 0, N - 1);
            const double k0 = up ? (double)(i + 1) : (double)i;  // first plane ahead
            sf[a] = qdiv(g.lo[a] + k0 * g.delta[a] - v.o[a], d[a], inv[a]) - tin;
            ds[a] = qdiv(g.delta[a], fabs(d[a]), fabs(inv[a]));
            jface[a] = up ? (double)N - k0 : k0;  // crossings to reach the far face
            int kplane = (int)k0;
            if (sf[a] <= 0.0) {  // rounding put the entry just before plane k0
                i = clampi(i + (up ? 1 : -1), 0, N - 1);
                sf[a] += ds[a];
                jface[a] -= 1.0;
                kplane += up ? 1 : -1;
            }
            idx[a] = i;
            if (ax) {
                ax->k0[a] = kplane;
                ax->rds[a] = fabs(d[a]) * g.inv_delta[a];
            }
            r.st[a] = up ? stride[a] : -stride[a];
        } else {
            // an observer exactly on a plane (k delta from the face) gives k,
            // the voxel above it
            idx[a] = clampi((int)floor(qdiv(v.o[a] - g.lo[a], g.delta[a], g.inv_delta[a])), 0, N - 1);
            if (ax) {
                ax->k0[a] = 0;
                ax->rds[a] = 0.0;
            }
            sf[a] = kFar;
            ds[a] = 0.0;
            jface[a] = 0.0;
            r.st[a] = 0;
        }
    }
    // Only values up to ~3 chords are ever compared: an axis whose first
    // crossing lies beyond 2 chords is never crossed, and a spacing above
    // 2 chords means at most one crossing, so both are capped.  Then every
    // value the walk forms is below span = 4 chords, and a power-of-two grid
    // q with span < 2^51 q makes all the additions exact.
    const double chord = tout - tin, lim = 2.0 * chord;
    int ex = 0;
    (void)frexp(4.0 * chord, &ex);  // 4 chord < 2^ex
    double send = kFar;
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        if (d[a] != 0.0 && sf[a] <= lim) {
            ds[a] = ldexp(rint(ldexp(fmin(ds[a], lim), 51 - ex)), ex - 51);
            sf[a] = ldexp(rint(ldexp(sf[a], 51 - ex)), ex - 51);
            send = fmin(send, sf[a] + jface[a] * ds[a]);
        } else {
            sf[a] = kFar;
            ds[a] = 0.0;
        }
        r.s[a] = sf[a];
        r.ds[a] = ds[a];
    }
    if (kObstacle && g.has_sph) {
        // the obstacle: the line of sight ends where it enters the sphere's
        // interior, found from the closest approach t* of the line to the
        // centre (at distance h): t* - sqrt((R^2 - h^2) / d.d); the end is
        // put on the ray's grid, so that every walk stops at the same value
        double oc[3], dd = 0.0, od = 0.0, oo = 0.0;
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            oc[a] = v.o[a] - g.sph[a];
            dd = fma(d[a], d[a], dd);
            od = fma(oc[a], d[a], od);
            oo = fma(oc[a], oc[a], oo);
        }
        const double r2 = g.sph[3] * g.sph[3];
        if (oo <= r2) return false;  // observer on or inside the sphere
        if (od < 0.0) {
            const double ts = -od / dd;
            double h2 = 0.0;
#pragma unroll
            for (int a = 0; a < 3; ++a) {
                const double p = fma(ts, d[a], oc[a]);
                h2 = fma(p, p, h2);
            }
            if (h2 < r2) {
                const double tc = ts - sqrt((r2 - h2) / dd) - tin;  // from the entry
                send = fmin(send, ldexp(rint(ldexp(tc, 51 - ex)), ex - 51));
            }
        }
    }
    if (!(send > 0.0) || !(send < kFar)) return false;
    r.send = send;
    r.off = (idx[2] * g.n[1] + idx[1]) * g.n[0] + idx[0];
    if (ax) {
        for (int a = 0; a < 3; ++a) ax->idx[a] = idx[a];
        ax->tin = tin;
    }
    return true;
}

// Stores the set-up of pixel i (ok: ray_setup's result) into a ray table's
// columns d and index words k, n rows each.  Every field is written, also
// for a ray that misses (send = 0), so the table's contents depend on the
// geometry alone.
__device__ inline void ray_table_put(double *__restrict__ d, uint64_t *__restrict__ k, int64_t n, int64_t i,
                                     bool ok, const RayState &r, const RayAxes &ax)
{
    uint64_t w = 0;
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        d[a * n + i] = ok ? r.s[a] : 0.0;
        d[(3 + a) * n + i] = ok ? r.ds[a] : 0.0;
        d[(8 + a) * n + i] = ok ? ax.rds[a] : 0.0;
        if (ok) {
            w |= (uint64_t)(uint32_t)ax.idx[a] << (kRayTableSideBits * a);
            if (r.st[a] > 0) w |= 1ull << (60 + a);
        }
    }
    d[6 * n + i] = ok ? r.send : 0.0;
    d[7 * n + i] = ok ? r.dn : 0.0;
    k[i] = w;
}

// The set-up of pixel i read back from a ray table: the fields of r and ax
// that the blocked P^T uses (r.s, r.ds, r.send, r.dn, the signs of r.st;
// ax.idx, ax.rds), bit for bit as ray_setup left them.  False: the ray
// misses the box.
__device__ inline bool ray_table_get(const RayTable &t, int64_t i, RayState &r, RayAxes &ax)
{
    const double *__restrict__ d = t.d;
    const int64_t n = t.n;
    const uint64_t w = t.k[i];
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        r.s[a] = d[a * n + i];
        r.ds[a] = d[(3 + a) * n + i];
        ax.rds[a] = d[(8 + a) * n + i];
        ax.idx[a] = (int)((w >> (kRayTableSideBits * a)) & ((1u << kRayTableSideBits) - 1u));
        r.st[a] = r.ds[a] == 0.0 ? 0 : (((w >> (60 + a)) & 1u) ? 1 : -1);
    }
    r.send = d[6 * n + i];
    r.dn = d[7 * n + i];
    return r.send > 0.0;
}

// 1.0 if t else 0.0: only the high word differs, so one select; fma(ds, f,
// s) then equals s + ds or s exactly.
__device__ inline double tie_factor(bool t)
{
    return __builtin_bit_cast(double, (uint64_t)(t ? 0x3FF00000u : 0u) << 32);
}

// Walk the ray voxel by voxel.  visit(off, dl) receives the flat voxel
// offset and the parameter length of the segment (length = dl * |d|).
// Simultaneous crossings advance every tied axis in one step.  maxit bounds
// the loop whatever the arithmetic does; the loop body holds four steps, so
// the bound is tested once per four (it may run up to three steps past it).
template <class Visit>
__device__ inline void ray_walk(RayState &r, int maxit, Visit &&visit)
{
    double scur = 0.0;
    // The state advances before the segment is visited, so that a gather
    // of the segment's voxel (issued from its offset at the top of the
    // step) has the tie updates to arrive in; after the last segment the
    // advanced state is not used.
    auto step = [&]() {  // true once the ray has ended
        const double m = fmin(fmin(r.s[0], r.s[1]), fmin(r.s[2], r.send));
        const int32_t off = r.off;
        const double dl = m - scur;
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            const bool t = (r.s[a] == m);
            r.s[a] = fma(r.ds[a], tie_factor(t), r.s[a]);  // s + ds or s, exact on the common grid
            r.off += t ? r.st[a] : 0;
        }
        scur = m;
        visit(off, dl);
        return m >= r.send;
    };
    for (int it = 0; it < maxit; it += 4) {
        if (step() || step() || step() || step()) break;
    }
}

// Tile -> (view, pixel of this lane).  Views are sorted by tile_off.
struct LanePixel {
    int view;
    int col, row;
};

__device__ inline LanePixel lane_pixel(const ViewDev *__restrict__ views, int nviews, int64_t tile,
                                       int log2_bw)
{
    int lo = 0, hi = nviews - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (views[mid].tile_off <= tile) lo = mid;
        else hi = mid - 1;
    }
    const int64_t t = tile - views[lo].tile_off;
    const int tpr = views[lo].tiles_x;
    const int tx = (int)(t % tpr), ty = (int)(t / tpr);
    const int w = threadIdx.x >> 6, l = threadIdx.x & 63;
    LanePixel lp;
    lp.view = lo;
    if (log2_bw == 0) {  // 8x8 lanes at a 2-pixel pitch, wavefront w offset by (w&1, w>>1)
        lp.col = tx * kTile + (l & 7) * 2 + (w & 1);
        lp.row = ty * kTile + (l >> 3) * 2 + (w >> 1);
        return lp;
    }
    const int bw = 1 << log2_bw, bh = 64 >> log2_bw;
    const int wpr = kTile >> log2_bw;  // wave bundles per tile row
    lp.col = tx * kTile + (w % wpr) * bw + (l & (bw - 1));
    lp.row = ty * kTile + (w / wpr) * bh + (l >> log2_bw);
    return lp;
}

__device__ inline int64_t block_tile(const Bundle &b)
{
    return xcd_order(b.xcd_remap, blockIdx.x, gridDim.x);
}

// P for one 16x16 tile (all threads of the workgroup): each lane's pixel =
// sum over its ray's segments of length x voxel value, written to images.
template <bool kMapMask, bool kDataMask, bool kObstacle>
__device__ inline void project_tile(const GridDev &g, const ViewDev *__restrict__ views, int32_t nviews,
                                    int log2_bw, int64_t tile, int32_t maxit,
                                    const float *__restrict__ cube, const uint8_t *__restrict__ map_mask,
                                    const uint8_t *__restrict__ data_mask, float *__restrict__ images)
{
    const LanePixel lp = lane_pixel(views, nviews, tile, log2_bw);
    const ViewDev &v = views[lp.view];
    if (lp.col >= v.ncol || lp.row >= v.nrow) return;
    const int64_t pix = v.pix_off + (int64_t)lp.row * v.ncol + lp.col;
    float out = 0.0f;
    RayState r;
    if ((!kDataMask || data_mask[pix]) && ray_setup<kObstacle>(g, v, lp.col, lp.row, r)) {
        const float *__restrict__ base = cube + (int64_t)v.frame * g.nvox;
        // a buffer resource spans below 2^32 bytes: a frame of 2^30 voxels
        // takes plain global loads, their offsets clamped into the frame as
        // the buffer's range check would
        const bool wide = g.nvox >= ((int64_t)1 << 30);
        const uint32_t last = (uint32_t)(g.nvox - 1);
        const auto rc = make_rsrc(base, wide ? 0u : (uint32_t)(g.nvox * 4));
        // software-pipelined by one segment: a step issues its voxel's gather
        // before it adds the previous segment, so each load has a whole step
        // to land
        double acc = 0.0, dl_prev = 0.0;
        float x_prev = 0.0f;
        if constexpr (kMapMask) {
            const auto rm = make_rsrc(map_mask, (uint32_t)g.nvox);
            uint32_t m_prev = 0u;
            auto walk_masked = [&](auto load) {
                ray_walk(r, maxit, [&](int32_t off, double dl) {
                    const float x = load((uint32_t)off);
                    const uint32_t mk = buf_load_u8(rm, (uint32_t)off);
                    acc = fma(dl_prev, m_prev ? (double)x_prev : 0.0, acc);
                    x_prev = x;
                    m_prev = mk;
                    dl_prev = dl;
                });
            };
            if (wide)
                walk_masked([&](uint32_t o) { return base[min(o, last)]; });
            else
                walk_masked([&](uint32_t o) { return buf_load_f32(rc, o * 4u); });
            if (!m_prev) x_prev = 0.0f;
        } else if (wide) {
            ray_walk(r, maxit, [&](int32_t off, double dl) {
                const float x = base[min((uint32_t)off, last)];
                acc = fma(dl_prev, (double)x_prev, acc);
                x_prev = x;
                dl_prev = dl;
            });
        } else if (g.nvox < ((int64_t)1 << 29)) {
            // offsets in bytes from here on (below 2^31, so int32 holds them)
            r.off *= 4;
#pragma unroll
            for (int a = 0; a < 3; ++a) r.st[a] *= 4;
            ray_walk(r, maxit, [&](int32_t off, double dl) {
                const float x = buf_load_f32(rc, (uint32_t)off);
                acc = fma(dl_prev, (double)x_prev, acc);
                x_prev = x;
                dl_prev = dl;
            });
        } else {
            ray_walk(r, maxit, [&](int32_t off, double dl) {
                const float x = buf_load_f32(rc, (uint32_t)off * 4u);
                acc = fma(dl_prev, (double)x_prev, acc);
                x_prev = x;
                dl_prev = dl;
            });
        }
        acc = fma(dl_prev, (double)x_prev, acc);
        out = (float)(acc * (r.dn * v.gain));
    }
    images[pix] = out;
}

// Offset of voxel (i0, i1, i2) in its frame of the bricked copy.
__device__ inline uint32_t brick_offset(const BrickDev &bk, int i0, int i1, int i2)
{
    const uint32_t m = (1u << bk.k) - 1u;
    const uint32_t brick = ((uint32_t)(i2 >> bk.k) * (uint32_t)bk.nb[1] + (uint32_t)(i1 >> bk.k)) * (uint32_t)bk.nb[0] +
                           (uint32_t)(i0 >> bk.k);
    return (brick << (3 * bk.k)) | (((uint32_t)i2 & m) << (2 * bk.k)) | (((uint32_t)i1 & m) << bk.k) |
           ((uint32_t)i0 & m);
}

// The bricked offset is a sum of one term per axis: brick_offset(i0, i1,
// i2) = f0(i0) + f1(i1) + f2(i2) with f_a(i) = (i >> k) S_a 2^3k + (i & m)
// 2^(k a), S = (1, nb0, nb0 nb1), since the brick index is linear in the
// per-axis brick coordinates and the in-brick bits do not overlap it.
__device__ inline uint32_t brick_axis_term(const BrickDev &bk, int a, int i)
{
    const uint32_t m = (1u << bk.k) - 1u;
    const uint32_t s = a == 0 ? 1u : (a == 1 ? (uint32_t)bk.nb[0] : (uint32_t)bk.nb[0] * (uint32_t)bk.nb[1]);
    return ((((uint32_t)i >> bk.k) * s) << (3 * bk.k)) + (((uint32_t)i & m) << (bk.k * a));
}

// P for one 16x16 tile from a bricked copy of M x (the map mask applied by
// the copy): the same walk as project_tile, the voxel indices carried per
// axis and the offset formed from them; the same segments summed in the
// same order, so the same bits.  With kLut the offset is the sum of three
// per-axis terms read from LDS (lut: f0 over the n0 x indices, then f1,
// then f2; in bytes unless kWide), one add and three LDS reads per step
// instead of the shifts, masks and multiplies of brick_offset.
template <bool kDataMask, bool kObstacle, bool kLut, bool kWide>
__device__ inline void project_tile_bricked(const GridDev &g, const ViewDev *__restrict__ views, int32_t nviews,
                                            int log2_bw, int64_t tile, int32_t maxit, const float *__restrict__ bricked,
                                            const BrickDev &bk, const uint8_t *__restrict__ data_mask,
                                            float *__restrict__ images, const uint32_t *lut = nullptr)
{
    const LanePixel lp = lane_pixel(views, nviews, tile, log2_bw);
    const ViewDev &v = views[lp.view];
    if (lp.col >= v.ncol || lp.row >= v.nrow) return;
    const int64_t pix = v.pix_off + (int64_t)lp.row * v.ncol + lp.col;
    float out = 0.0f;
    RayState r;
    RayAxes ax;
    if ((!kDataMask || data_mask[pix]) && ray_setup<kObstacle>(g, v, lp.col, lp.row, r, &ax)) {
        const float *__restrict__ base = bricked + (int64_t)v.frame * bk.frame_stride;
        const uint32_t last = (uint32_t)(bk.frame_stride - 1);
        const auto rc = make_rsrc(base, kWide ? 0u : (uint32_t)(bk.frame_stride * 4));
        int i[3] = {ax.idx[0], ax.idx[1], ax.idx[2]};
        int dir[3];
#pragma unroll
        for (int a = 0; a < 3; ++a) dir[a] = r.st[a] > 0 ? 1 : (r.st[a] < 0 ? -1 : 0);
        // the kind of load is fixed per kernel (kWide: frames of 2^30 floats
        // and more, which a buffer resource cannot span).  Pipelined by one
        // segment: a step issues its voxel's gather before it adds the
        // previous segment, so two gathers are in flight and each has a
        // whole step to land
        double acc = 0.0, dl_prev = 0.0, scur = 0.0;
        float x_prev = 0.0f;
        auto step = [&]() {
            const double m = fmin(fmin(r.s[0], r.s[1]), fmin(r.s[2], r.send));
            const uint32_t off = kLut ? lut[i[0]] + lut[g.n[0] + i[1]] + lut[g.n[0] + g.n[1] + i[2]]
                                      : brick_offset(bk, i[0], i[1], i[2]);
            const float x = kWide ? base[min(off, last)] : buf_load_f32(rc, kLut ? off : off * 4u);
            const double dl = m - scur;
#pragma unroll
            for (int a = 0; a < 3; ++a) {
                const bool t = (r.s[a] == m);
                r.s[a] = fma(r.ds[a], tie_factor(t), r.s[a]);
                i[a] += t ? dir[a] : 0;
            }
            scur = m;
            acc = fma(dl_prev, (double)x_prev, acc);
            x_prev = x;
            dl_prev = dl;
            return m >= r.send;
        };
        for (int it = 0; it < maxit; it += 4) {
            if (step() || step() || step() || step()) break;
        }
        acc = fma(dl_prev, (double)x_prev, acc);
        out = (float)(acc * (r.dn * v.gain));
    }
    images[pix] = out;
}

}  // namespace tomo
