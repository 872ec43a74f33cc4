// Device code of the owner-computes P^T shared by its single-geometry
// launch (blocked.hip) and the batched persistent launch (batch.hip).
#pragma once

#include "walk.h"

namespace tomo {

constexpr int kYmaxParts = 64;  // partial maxima per view (64 workgroups per view keep the pass short)

// LDS byte address of a pointer into shared memory, and atomic adds at such
// an address: a walk that carries its bin as an address needs no shift or
// base add per step (the clamp's result is the instruction's address).
__device__ inline uint32_t lds_address(const void *p)
{
    return (uint32_t)(uintptr_t)(__attribute__((address_space(3))) const char *)p;
}
__device__ inline void lds_add_u64(uint32_t a, unsigned long long v)
{
    __hip_atomic_fetch_add((__attribute__((address_space(3))) unsigned long long *)(uintptr_t)a, v,
                           __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
}
__device__ inline void lds_add_f32(uint32_t a, float v)
{
    __hip_atomic_fetch_add((__attribute__((address_space(3))) float *)(uintptr_t)a, v, __ATOMIC_RELAXED,
                           __HIP_MEMORY_SCOPE_WORKGROUP);
}

// max |gain y| over the share `part` of view v's unmasked pixels, as an
// FP32 bit pattern (bit patterns of magnitudes order like the magnitudes;
// anything >= 0x7f800000 is non-finite).  The product is rounded to FP32,
// which the scale's margin of 1e-7 covers.  Valid in thread 0.
template <bool kDataMask>
__device__ inline uint32_t view_absmax_part(const ViewDev &v, int part, const float *__restrict__ images,
                                            const uint8_t *__restrict__ data_mask, uint32_t *red /* LDS [4] */)
{
    const int64_t np = (int64_t)v.ncol * v.nrow;
    uint32_t m = 0u;
    for (int64_t i = (int64_t)part * kThreads + threadIdx.x; i < np; i += (int64_t)kYmaxParts * kThreads) {
        const int64_t pix = v.pix_off + i;
        const uint32_t b = __builtin_bit_cast(uint32_t, images[pix]) & 0x7fffffffu;
        if (!kDataMask || data_mask[pix]) m = b > m ? b : m;
    }
    for (int o = 32; o > 0; o >>= 1) {
        const uint32_t t = (uint32_t)__shfl_down((int)m, o, 64);
        m = t > m ? t : m;
    }
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = m;
    __syncthreads();
    uint32_t r = 0u;
    if (threadIdx.x == 0) {
        r = red[0];
        for (int k = 1; k < kThreads / 64; ++k) r = red[k] > r ? red[k] : r;
        if (r < 0x7f800000u)  // a product that overflows FP32 reads as non-finite
            r = __builtin_bit_cast(uint32_t, (float)((double)__builtin_bit_cast(float, r) * fabs(v.gain)));
    }
    __syncthreads();
    return r;
}

// Kept pixels of a data-masked image, row by row: for pixel (row, col),
// pre[pix] = kept pixels before col in its row, and the first pre[row end]
// entries of the row in cols hold the kept columns in order.  With them a
// footprint row's column interval maps to a run of kept pixels, so masked
// pixels never take a lane of the blocked P^T's passes.
struct KeptRows {
    const uint16_t *pre;
    const uint16_t *cols;
};

// One view of a chunk staged in LDS: the pointing fields ray_setup reads,
// plus what the passes need to address the view's pixels and weigh them.
struct StagedView {
    double o[3], w[3], u[3], v[3];
    double cd[2], cp[2];
    double vscale;    // gain times the fixed-point scale of the owner's bins
    int64_t pix_off;  // first pixel of the view in the image vector
    int32_t ncol, nrow;
};

// Shared-memory scratch of one item besides the bins: up to C views of the
// owner, staged with their footprints, so that the passes then run over the
// footprint pixels of all of them without workgroup barriers.  A footprint is
// the bounding rectangle of the block's projection and, when the rectangle
// has at most kRowsMax rows, one column interval per row (the projection of a
// box is convex, so the pixels of one row whose rays meet it form an
// interval) with the running pixel count.  vpre holds the pixels of the
// chunk's views before each view: the passes take the concatenated list 256
// (or NT) pixels at a time, so a pass is ragged only at the chunk's end.
constexpr int kRowsMax = 64;
template <int NT, bool kRows>
struct BlockedShared {
    static constexpr int C = kRows ? (NT >= 512 ? 16 : 8) : 32;  // views per chunk
    StagedView view[C];
    int rect[C][4];                      // c0, c1, r0, r1 (c0 > c1: the block is not seen)
    int rows[C];                         // 1: walk the row intervals, 0: the whole rectangle
    int64_t vpre[C + 1];                 // pixels of the chunk's views before view j
    uint16_t cs[kRows ? C : 1][kRowsMax];      // first column (or kept-pixel index) of each row's run
    int32_t pre[kRows ? C : 1][kRowsMax + 1];  // pixels in the rows before (pre[H]: all)
};

// Column interval [cs, ce] of image row `row` of view v whose rays can meet
// the box [o + lo, o + hi].  The rays of the row, d = e + x u with
// e = w + y v, fill the plane through the observer with normal n = e x u,
// and the box meets that plane in a convex polygon whose corners lie on the
// box's edges; a point p of the plane lies on the ray of
// x = -(p . (e x n)) / (p . (u x n)) (any basis, orthonormal or not), so the
// polygon's corners bound the row's columns.  FP32: the caller pads the box
// by far more than its rounding, and the interval is widened by one pixel
// each side and clipped to [c0, c1]; ce < cs: none.  Returns false if a
// corner is not in front of the observer (the caller then keeps the whole
// row).
template <class V>
__device__ inline bool row_interval(const V &v, int row, const float (&lo)[3], const float (&hi)[3], int c0,
                                    int c1, int &cs, int &ce)
{
    const float y = (float)(((double)row - v.cp[1]) * v.cd[1]);
    const float w[3] = {(float)v.w[0], (float)v.w[1], (float)v.w[2]};
    const float u[3] = {(float)v.u[0], (float)v.u[1], (float)v.u[2]};
    const float vv[3] = {(float)v.v[0], (float)v.v[1], (float)v.v[2]};
    const float e[3] = {w[0] + y * vv[0], w[1] + y * vv[1], w[2] + y * vv[2]};
    const float n[3] = {e[1] * u[2] - e[2] * u[1], e[2] * u[0] - e[0] * u[2], e[0] * u[1] - e[1] * u[0]};
    const float an[3] = {u[1] * n[2] - u[2] * n[1], u[2] * n[0] - u[0] * n[2], u[0] * n[1] - u[1] * n[0]};
    const float bn[3] = {e[1] * n[2] - e[2] * n[1], e[2] * n[0] - e[0] * n[2], e[0] * n[1] - e[1] * n[0]};
    // a corner's S = p.n, W = p.(u x n), U = -p.(e x n) as sums of one
    // low-or-high term per axis
    float ts[2][3], tw[2][3], tu[2][3];
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        ts[0][a] = lo[a] * n[a];
        ts[1][a] = hi[a] * n[a];
        tw[0][a] = lo[a] * an[a];
        tw[1][a] = hi[a] * an[a];
        tu[0][a] = -(lo[a] * bn[a]);
        tu[1][a] = -(hi[a] * bn[a]);
    }
    auto corner = [&](int k, float (&t)[2][3]) { return t[k & 1][0] + t[(k >> 1) & 1][1] + t[k >> 2][2]; };
#pragma unroll
    for (int k = 0; k < 8; ++k)
        if (!(corner(k, tw) > 0.0f)) return false;
    float xmin = 3.0e38f, xmax = -3.0e38f;
    // the 12 edges: corner k without bit b to corner k | b
#pragma unroll
    for (int ed = 0; ed < 12; ++ed) {
        const int b = 1 << (ed >> 2), q = ed & 3;
        const int k = b == 1 ? q << 1 : (b == 2 ? (q & 1) | ((q & 2) << 1) : q), l = k | b;
        const float sk = corner(k, ts), sl = corner(l, ts);
        if (sk > 0.0f ? sl > 0.0f : (sk < 0.0f && sl < 0.0f)) continue;  // no crossing
        const float uk = corner(k, tu), ul = corner(l, tu), wk = corner(k, tw), wl = corner(l, tw);
        if (sk == sl) {  // both zero: the edge lies in the plane
            const float xa = uk / wk, xb = ul / wl;
            xmin = fminf(xmin, fminf(xa, xb));
            xmax = fmaxf(xmax, fmaxf(xa, xb));
        } else {  // the crossing at t = sk / (sk - sl) along the edge
            const float x = (sk * ul - sl * uk) / (sk * wl - sl * wk);
            xmin = fminf(xmin, x);
            xmax = fmaxf(xmax, x);
        }
    }
    if (!(xmin <= xmax)) {
        cs = c0;
        ce = c0 - 1;
        return true;
    }
    const double ca = v.cp[0] + (double)xmin / v.cd[0], cb = v.cp[0] + (double)xmax / v.cd[0];
    cs = (int)fmax(floor(fmin(ca, cb)) - 1.0, (double)c0);
    ce = (int)fmin(ceil(fmax(ca, cb)) + 1.0, (double)c1);
    return true;
}

// One owner item of the blocked P^T: (frame, block, split) from the item
// index, every ray of the owner's views that can cross the block walked
// inside it, and the block written once.  bins: nbins 64-bit LDS words plus
// a dummy.  Called by all NT threads of the workgroup.  kept.cols != null
// (with kDataMask) takes the passes over kept pixels only, in row-interval
// footprints.  tab.d != null: each ray's set-up is read from the geometry's
// ray table instead of computed.
template <int NT, bool kMapMask, bool kDataMask, bool kObstacle, bool kRows>
__device__ inline void blocked_item(const GridDev &g, const ViewDev *__restrict__ views,
                                    const int32_t *__restrict__ frame_views,
                                    const int32_t *__restrict__ frame_voff, const BlockDev &bd,
                                    int64_t item, const float *__restrict__ images,
                                    const uint8_t *__restrict__ map_mask,
                                    const uint8_t *__restrict__ data_mask, KeptRows kept,
                                    const uint32_t *__restrict__ ymax_parts, float *__restrict__ out,
                                    int32_t accumulate, unsigned *__restrict__ spill, const RayTable &tab,
                                    unsigned long long *bins, BlockedShared<NT, kRows> &sh)
{
    using Sh = BlockedShared<NT, kRows>;
    constexpr int C = Sh::C;
    static_assert(8 * C <= NT, "eight lanes per staged view");
    const int tid = threadIdx.x;
    // ---- item -> (frame, block, split)
    const int64_t nblk = (int64_t)bd.nb[0] * bd.nb[1] * bd.nb[2];
    const int split = (int)(item % bd.splits);
    const int64_t fb = item / bd.splits;
    const int frame = (int)(fb / nblk);
    const int64_t blk = fb % nblk;
    const int bi = (int)(blk % bd.nb[0]), bj = (int)((blk / bd.nb[0]) % bd.nb[1]),
              bk = (int)(blk / ((int64_t)bd.nb[0] * bd.nb[1]));
    const int blo[3] = {bi * bd.b[0], bj * bd.b[1], bk * bd.b[2]};
    const int bhi[3] = {min(blo[0] + bd.b[0], g.n[0]), min(blo[1] + bd.b[1], g.n[1]),
                        min(blo[2] + bd.b[2], g.n[2])};
    const int nbins = bd.b[0] * bd.b[1] * bd.b[2];
    const int32_t lstride[3] = {1, bd.b[0], bd.b[0] * bd.b[1]};

    const int v0 = frame_voff[frame], v1 = frame_voff[frame + 1];

    // ---- fixed-point scale from the views this owner handles (uniform):
    // the largest |gain y| among them
    uint32_t ybits = 0u;
    double rays = 0.0;
    for (int k = v0 + split; k < v1; k += bd.splits) {
        const int vi = frame_views[k];
        for (int p = 0; p < kYmaxParts; ++p) {
            const uint32_t b = ymax_parts[vi * kYmaxParts + p];
            ybits = b > ybits ? b : ybits;
        }
        rays += (double)views[vi].ncol * (double)views[vi].nrow;
    }
    const bool finite = ybits < 0x7f800000u;
    const double ymax = (double)__builtin_bit_cast(float, ybits);
    const double vdiag = sqrt(g.delta[0] * g.delta[0] + g.delta[1] * g.delta[1] + g.delta[2] * g.delta[2]);
    // scale 2^(61 - eb): every bin below 2^61 (at most `rays` contributions
    // of at most vdiag max|y| each) and every single contribution below 2^50,
    // so that adding 1.5 * 2^52 rounds it to an integer held in the low
    // mantissa bits
    int eb = 0, e1 = 0;
    (void)frexp(fmax(rays, 1.0) * vdiag * ymax * 1.0000001, &eb);
    (void)frexp(vdiag * ymax * 1.0000001, &e1);
    eb = eb > e1 + 11 ? eb : e1 + 11;
    const double fx_scale = ldexp(1.0, 61 - eb), fx_inv = ldexp(1.0, eb - 61);
    // bins as LDS byte addresses: bin l at bbase + 8 l (the FP32 bins of
    // non-finite data in the low half of the same word); blim is the dummy bin
    const uint32_t bbase = lds_address(bins), blim = bbase + 8u * (uint32_t)nbins;

    __syncthreads();  // the previous item of this workgroup is done with the bins
    for (int i = tid; i <= nbins; i += NT) bins[i] = 0ull;  // + the dummy bin
    unsigned spills = 0u;
    const bool compact = kRows && kDataMask && kept.cols != nullptr;

    const int nvi = v1 - v0 > split ? (v1 - v0 - split + bd.splits - 1) / bd.splits : 0;  // owner's views
    for (int cs0 = 0; cs0 < nvi; cs0 += C) {
        const int nch = min(C, nvi - cs0);
        // ---- footprints: thread 8 j + c projects corner c of the chunk's
        // view j; the 8 lanes of a view reduce with shuffles
        __syncthreads();  // the previous chunk's staging is no longer in use
        if (tid < 8 * C) {
            const int j = tid >> 3, c = tid & 7;
            const bool live = j < nch;
            const ViewDev &v = views[frame_views[v0 + split + (cs0 + (live ? j : 0)) * bd.splits]];
            double cc = 0.0, cr = 0.0;
            int bad = 0;
            if (live) {
                const int ci[3] = {(c & 1) ? bhi[0] : blo[0], (c & 2) ? bhi[1] : blo[1],
                                   (c & 4) ? bhi[2] : blo[2]};
                double d[3];
#pragma unroll
                for (int a = 0; a < 3; ++a) d[a] = g.lo[a] + (double)ci[a] * g.delta[a] - v.o[a];
                const double dep = d[0] * v.w[0] + d[1] * v.w[1] + d[2] * v.w[2];
                const double nd = sqrt(d[0] * d[0] + d[1] * d[1] + d[2] * d[2]);
                if (!(dep > 1e-6 * nd)) {
                    bad = 1;  // behind the observer: the whole detector
                } else {
                    const double x = (d[0] * v.u[0] + d[1] * v.u[1] + d[2] * v.u[2]) / dep;
                    const double y = (d[0] * v.v[0] + d[1] * v.v[1] + d[2] * v.v[2]) / dep;
                    cc = v.cp[0] + x / v.cd[0];
                    cr = v.cp[1] + y / v.cd[1];
                }
            }
            double cmn = cc, cmx = cc, rmn = cr, rmx = cr;
#pragma unroll
            for (int o = 1; o < 8; o <<= 1) {
                cmn = fmin(cmn, __shfl_xor(cmn, o));
                cmx = fmax(cmx, __shfl_xor(cmx, o));
                rmn = fmin(rmn, __shfl_xor(rmn, o));
                rmx = fmax(rmx, __shfl_xor(rmx, o));
                bad |= __shfl_xor(bad, o);
            }
            if (live) {
                StagedView &sv = sh.view[j];
                // the eight lanes of the view copy its pointing fields
#pragma unroll
                for (int a = 0; a < 3; ++a) {
                    if (c == 0) sv.o[a] = v.o[a];
                    if (c == 1) sv.w[a] = v.w[a];
                    if (c == 2) sv.u[a] = v.u[a];
                    if (c == 3) sv.v[a] = v.v[a];
                }
                if (c == 4) {
                    sv.cd[0] = v.cd[0];
                    sv.cd[1] = v.cd[1];
                    sv.cp[0] = v.cp[0];
                    sv.cp[1] = v.cp[1];
                }
                if (c == 5) {
                    // the view's gain times the bin scale (a power of two: exact)
                    sv.vscale = v.gain * (finite ? fx_scale : 1.0);
                    sv.pix_off = v.pix_off;
                    sv.ncol = v.ncol;
                    sv.nrow = v.nrow;
                }
                if (c == 0) {
                    int c0 = 0, c1 = v.ncol - 1, r0 = 0, r1 = v.nrow - 1;
                    if (!bad) {  // clamp in double before converting: far-off corners stay finite
                        c0 = (int)fmax(floor(cmn) - 1.0, 0.0);
                        c1 = (int)fmin(ceil(cmx) + 1.0, (double)(v.ncol - 1));
                        r0 = (int)fmax(floor(rmn) - 1.0, 0.0);
                        r1 = (int)fmin(ceil(rmx) + 1.0, (double)(v.nrow - 1));
                    }
                    sh.rect[j][0] = c0;
                    sh.rect[j][1] = c1;
                    sh.rect[j][2] = r0;
                    sh.rect[j][3] = r1;
                    sh.rows[j] = kRows && !bad && c0 <= c1 && r1 - r0 < kRowsMax;
                }
            }
        }
        __syncthreads();

        if constexpr (kRows) {
            // ---- row intervals: one row per thread, widths first (in pre[row + 1])
            for (int t = tid; t < nch * kRowsMax; t += NT) {
                const int j = t / kRowsMax, rr = t % kRowsMax;
                const int c0 = sh.rect[j][0], c1 = sh.rect[j][1], r0 = sh.rect[j][2], r1 = sh.rect[j][3];
                if (!sh.rows[j] || rr > r1 - r0) continue;
                const StagedView &v = sh.view[j];
                // the block's box less the observer, padded by 1e-3 of a voxel
                // plus 1e-5 of the largest coordinate in play: far above the FP32
                // rounding of the interval (relative 1e-7 of these magnitudes) and
                // the rays' FP64 set-up, so that every ray the exact set-up finds
                // inside the block is kept
                float lo[3], hi[3];
#pragma unroll
                for (int a = 0; a < 3; ++a) {
                    const double big = fmax(fmax(fabs(g.lo[a]), fabs(g.hi[a])), fabs(v.o[a]));
                    const double pad = 1e-3 * g.delta[a] + 1e-5 * big;
                    lo[a] = (float)((g.lo[a] + (double)blo[a] * g.delta[a] - pad) - v.o[a]);
                    hi[a] = (float)((g.lo[a] + (double)bhi[a] * g.delta[a] + pad) - v.o[a]);
                }
                int a0 = c0, a1 = c1;
                if (!row_interval(v, r0 + rr, lo, hi, c0, c1, a0, a1)) {
                    a0 = c0;
                    a1 = c1;
                }
                int start = a0, width = a1 >= a0 ? a1 - a0 + 1 : 0;
                if (compact && width > 0) {  // the run of kept pixels in [a0, a1]
                    const int64_t rb = v.pix_off + (int64_t)(r0 + rr) * v.ncol;
                    start = kept.pre[rb + a0];
                    width = (int)kept.pre[rb + a1] + (data_mask[rb + a1] ? 1 : 0) - start;
                }
                sh.cs[j][rr] = (uint16_t)start;
                sh.pre[j][rr + 1] = width;
            }
            __syncthreads();
            if (tid < nch && sh.rows[tid]) {  // running counts
                const int j = tid, h = sh.rect[j][3] - sh.rect[j][2] + 1;
                sh.pre[j][0] = 0;
                for (int rr = 1; rr <= h; ++rr) sh.pre[j][rr] += sh.pre[j][rr - 1];
            }
            __syncthreads();
        }
        if (tid == 0) {  // the chunk's views back to back
            int64_t acc = 0;
            for (int j = 0; j < nch; ++j) {
                sh.vpre[j] = acc;
                const int c0 = sh.rect[j][0], c1 = sh.rect[j][1], r0 = sh.rect[j][2], r1 = sh.rect[j][3];
                if (c0 <= c1 && r0 <= r1)
                    acc += (kRows && sh.rows[j]) ? (int64_t)sh.pre[j][r1 - r0 + 1]
                                                 : (int64_t)(c1 - c0 + 1) * (r1 - r0 + 1);
            }
            sh.vpre[nch] = acc;
        }
        __syncthreads();
        const int64_t total = sh.vpre[nch];

        // ---- the footprint pixels of all the chunk's views, NT per pass: thread
        // i takes pixel i of each pass, so a wavefront walks a run of 64
        // neighbouring pixels; each pass loads the next pass's pixel value so
        // that its latency is hidden by the walk.  A lane's pixel index only
        // grows, so its view j and row rr are found by scanning forward.
        int j = 0, rr = 0;
        // returns true when the pixel comes from a row's run of kept pixels
        // (its data mask need not be read)
        auto locate = [&](int64_t L, int &col, int &row) -> bool {
            while (j < nch - 1 && L >= sh.vpre[j + 1]) {
                ++j;
                rr = 0;
            }
            const int64_t lin = L - sh.vpre[j];
            const int c0 = sh.rect[j][0], r0 = sh.rect[j][2];
            if (kRows && sh.rows[j]) {
                const int H = sh.rect[j][3] - r0 + 1;
                while (rr < H - 1 && lin >= sh.pre[j][rr + 1]) ++rr;
                const int k = (int)sh.cs[j][rr] + ((int)lin - sh.pre[j][rr]);
                row = r0 + rr;
                col = compact ? (int)kept.cols[sh.view[j].pix_off + (int64_t)row * sh.view[j].ncol + k] : k;
                return compact;
            }
            {
                const int W = sh.rect[j][1] - c0 + 1;
                int q, r;
                if (lin < (1 << 22)) {  // FP32 holds lin exactly; q is then within one of lin / W
                    q = (int)((float)lin * (1.0f / (float)W));
                    r = (int)lin - q * W;
                    if (r < 0) {
                        --q;
                        r += W;
                    } else if (r >= W) {
                        ++q;
                        r -= W;
                    }
                } else {
                    q = (int)(lin / W);
                    r = (int)(lin - (int64_t)q * W);
                }
                row = r0 + q;
                col = c0 + r;
            }
            return false;
        };
        int64_t L = tid;
        int col = 0, row = 0;
        bool ok = L < total;
        int jn = 0;
        int64_t pixn = 0;
        float ynext = 0.0f;
        bool mnext = true;
        if (ok) {
            const bool known = locate(L, col, row);
            jn = j;
            pixn = sh.view[j].pix_off + (int64_t)row * sh.view[j].ncol + col;
            ynext = images[pixn];
            if (kDataMask && !known) mnext = data_mask[pixn] != 0;
        }
        for (int64_t base = 0; base < total; base += NT) {
            const int pcol = col, prow = row, pj = jn;
            const int64_t ppix = pixn;
            const bool pok = ok, pm = mnext;
            const float yv = ynext;
            L += NT;
            ok = L < total;
            if (ok) {
                const bool known = locate(L, col, row);
                jn = j;
                pixn = sh.view[j].pix_off + (int64_t)row * sh.view[j].ncol + col;
                ynext = images[pixn];
                mnext = true;
                if (kDataMask && !known) mnext = data_mask[pixn] != 0;
            }
            if (!pok || !nonzero_bits(yv) || (kDataMask && !pm)) continue;
            const StagedView &v = sh.view[pj];
            RayState r;
            RayAxes ax;
            if (tab.d) {
                if (!ray_table_get(tab, ppix, r, ax)) continue;
            } else if (!ray_setup<kObstacle>(g, v, pcol, prow, r, &ax)) {
                continue;
            }
            // parameter interval [E, X) inside the block, exact on the ray's grid
            double E = 0.0, X = r.send;
            bool hit = true;
#pragma unroll
            for (int a = 0; a < 3; ++a) {
                if (r.ds[a] == 0.0) {  // index constant along the ray
                    hit = hit && ax.idx[a] >= blo[a] && ax.idx[a] < bhi[a];
                    continue;
                }
                const bool up = r.st[a] > 0;
                const int J = up ? blo[a] - ax.idx[a] : ax.idx[a] - (bhi[a] - 1);  // crossings to enter
                const int K = up ? bhi[a] - ax.idx[a] : ax.idx[a] - blo[a] + 1;    // crossings to leave
                hit = hit && K > 0;
                if (J > 0) E = fmax(E, r.s[a] + (double)(J - 1) * r.ds[a]);
                X = fmin(X, r.s[a] + (double)(K - 1) * r.ds[a]);
            }
            if (!hit || !(X > E)) continue;
            // walk state at E: crossings with parameter <= E are done
            int32_t loc = 0;
            int32_t lst[3];  // bin steps in bytes
            bool inblk = true;
#pragma unroll
            for (int a = 0; a < 3; ++a) {
                int idx = ax.idx[a];
                if (r.ds[a] != 0.0) {
                    int jj = 0;
                    if (E >= r.s[a]) {
                        // the estimate from the unrounded spacing is within
                        // one of the count: the grid moves a spacing by at
                        // most 2^-49 crossings-per-chord of itself, so C
                        // crossings shift by at most 2^-49 C^2 < 1/2 on a
                        // cube side of at most 2^24 voxels (a capped
                        // spacing only makes it smaller, where the count
                        // is 1); one exact comparison each way settles it
                        jj = max((int)floor((E - r.s[a]) * ax.rds[a]) + 1, 1);
                        jj -= (jj > 1 && r.s[a] + (double)(jj - 1) * r.ds[a] > E) ? 1 : 0;
                        jj += (r.s[a] + (double)jj * r.ds[a] <= E) ? 1 : 0;
                    }
                    r.s[a] += (double)jj * r.ds[a];
                    idx += r.st[a] > 0 ? jj : -jj;
                    lst[a] = 8 * (r.st[a] > 0 ? lstride[a] : -lstride[a]);
                } else {
                    lst[a] = 0;
                }
                inblk = inblk && idx >= blo[a] && idx < bhi[a];
                loc += (idx - blo[a]) * lstride[a];
            }
            // On the exact grid a walk that starts inside the block stays
            // inside until X (each axis takes fewer crossings than it needs
            // to leave), so a start outside it is the only possible spill:
            // counted, and the ray skipped.
            if (!inblk) {
                ++spills;
                continue;
            }
            const double wys = (double)yv * r.dn * v.vscale;
            uint32_t la = bbase + 8u * (uint32_t)loc;  // the bin's LDS address
            // four steps per loop body, as in ray_walk; the clamp to the
            // dummy bin only guards the LDS range (an address below the bins,
            // which an exact walk never reaches, would stay inside the
            // workgroup's LDS)
            auto walk = [&](auto deposit) {
                double scur = E;
                auto step = [&]() {
                    const double m = fmin(fmin(r.s[0], r.s[1]), fmin(r.s[2], r.send));
                    deposit(min(la, blim), (m - scur) * wys);
                    if (m >= X) return true;
#pragma unroll
                    for (int a = 0; a < 3; ++a) {
                        const bool tie = (r.s[a] == m);
                        r.s[a] = fma(r.ds[a], tie_factor(tie), r.s[a]);
                        la += tie ? (uint32_t)lst[a] : 0u;
                    }
                    scur = m;
                    return false;
                };
                for (int it = 0; it < bd.maxit; it += 4) {
                    if (step() || step() || step() || step()) break;
                }
            };
            if (finite) {
                walk([&](uint32_t l, double val) {
                    // val + 1.5 * 2^52 rounds val to an integer (|val| < 2^50) in the low bits
                    const double t = val + 6755399441055744.0;
                    const long long q = (long long)__builtin_bit_cast(uint64_t, t) - 0x4338000000000000ll;
                    lds_add_u64(l, (unsigned long long)q);
                });
            } else {
                walk([&](uint32_t l, double val) { lds_add_f32(l, (float)val); });
            }
        }
    }
    if (spills) atomicAdd(spill, spills);
    __syncthreads();

    // ---- write the block once
    const int ex = bhi[0] - blo[0], ey = bhi[1] - blo[1], ez = bhi[2] - blo[2];
    const int nin = ex * ey * ez;
    const int64_t fbase = (int64_t)frame * g.nvox;
    const int64_t total = g.nvox * g.nframes;
    for (int e = tid; e < nin; e += NT) {
        const int lx = e % ex, ly = (e / ex) % ey, lz = e / (ex * ey);
        const int l = (lz * bd.b[1] + ly) * bd.b[0] + lx;
        const float val = finite ? (float)((double)(long long)bins[l] * fx_inv)
                                 : *reinterpret_cast<const float *>(bins + l);
        const int64_t off = ((int64_t)(blo[2] + lz) * g.n[1] + (blo[1] + ly)) * g.n[0] + (blo[0] + lx);
        if (bd.splits == 1) {
            float o = (!kMapMask || map_mask[off]) ? val : 0.0f;
            if (accumulate) o += out[fbase + off];
            out[fbase + off] = o;
        } else {
            out[(int64_t)split * total + fbase + off] = val;
        }
    }
}

}  // namespace tomo
