// Regularised inversion: the prior D^T D (+ D_t^T D_t) and conjugate
// gradient on the normal equations of TomograPy's criterion (Eq. criterion,
// Eq. stsrt):  A x = b,  A = M (P^T P + lambda_r D^T D + lambda_t D_t^T D_t) M,
// b = M P^T y.
//
// GPU design: FP32 vectors, FP64 dot products and scalars.  Every scalar of
// the recurrence (alpha, beta, residual norms) lives in device memory and is
// summed in a fixed order (deterministic).  In the plain CG iteration each
// workgroup leaves its partial of p.q or r.r, and every workgroup of the
// next kernel sums them itself; elsewhere the last workgroup to finish sums
// them (a counter and a device-scope fence per workgroup, which costs a
// write-back of the XCD's L2 each).  A device "done" flag, raised when the residual
// target or the iteration limit is reached, makes every later kernel of the
// iteration return at once, so the host enqueues iterations in chunks and
// synchronises only between chunks.  The vector updates are fused into
// three streaming passes per iteration around one P and one P^T.
#include <math.h>
#include <stddef.h>
#include <string.h>

#include <vector>

#include "batch.h"
#include "common.h"

namespace tomo {

constexpr int kRedBlocks = 1024;  // workgroups of every reducing vector kernel (at most)
constexpr int kIterBlocks = 2048; // workgroups of the fence-free CG passes (at most): their latency-bound
                                  // loops want more waves, and their partials cost no fences

struct CgState {
    double rr;        // r.r (plain CG) or z.r (flexible CG) of the current iterate
    double pq;        // p.A p
    double alpha, beta;
    double bb;        // b.b
    double thresh2;   // (rtol ||b||)^2, or -1 when no residual target
    double res2;      // r.r of the current iterate
    double aux;       // scratch result of the last reduction
    double res_prev;  // flexible CG: r.r of the previous iterate (stall test)
    double rr_prev;   // rr as the x/r update read it (beta's denominator)
    double drop2;     // flexible CG: (1 - min_drop)^2
    int32_t iter;     // iterations completed
    int32_t max_iter; // iteration limit
    int32_t done;     // 1: stop (converged, limit reached or non-finite)
    int32_t nonfinite;
    int32_t window;   // flexible CG: stalled iterations before the fall-back
    int32_t stall;    // consecutive iterations without a residual decrease
    int32_t fellback; // 1 once the solver has switched to plain CG
    int32_t fb_iter;  // iteration of the switch
    int32_t restart;  // 1: the next direction restarts (beta = 0)
    int32_t fb_snap;  // fellback and restart as the dot-product pass found them
    int32_t rs_snap;  //   (read by the direction update while it rewrites them)
    int32_t net_off;  // 1: skip the network (done, or fallen back)
};

struct Workspace {
    double *partials;   // [kRedBlocks][4]
    unsigned *counter;  // last-block detection
    double *cpart;      // [4][kIterBlocks]: per-workgroup partials summed by the next kernel
    int32_t nq;         // workgroups of k_cg_q (the partials of p.q)
    CgState *st;
    double *hist;       // [max_iter + 1]
};

// ------------------------------------------------------------ stencils

struct Dims {
    int32_t nx, ny, nz, nf;
    int64_t nvox;   // per frame
    int64_t total;  // nvox * nf
};

// Voxel coordinates of a flat index: frame f, in-frame offset rem and
// (i, j, k).  32-bit arithmetic when the whole vector has < 2^31 entries
// (64-bit divisions are long instruction sequences on the GPU).
struct VoxIdx {
    int64_t f, rem;
    int32_t i, j, k;
};

__device__ inline VoxIdx vox_index(const Dims &d, int64_t idx)
{
    VoxIdx o;
    if (d.total < ((int64_t)1 << 31)) {
        const uint32_t u = (uint32_t)idx, nv = (uint32_t)d.nvox;
        const uint32_t f = u / nv, rem = u - f * nv;
        const uint32_t jk = rem / (uint32_t)d.nx;
        o.f = f;
        o.rem = rem;
        o.i = (int32_t)(rem - jk * (uint32_t)d.nx);
        o.k = (int32_t)(jk / (uint32_t)d.ny);
        o.j = (int32_t)(jk - (uint32_t)o.k * (uint32_t)d.ny);
    } else {
        o.f = idx / d.nvox;
        o.rem = idx - o.f * d.nvox;
        o.i = (int32_t)(o.rem % d.nx);
        const int64_t jk = o.rem / d.nx;
        o.j = (int32_t)(jk % d.ny);
        o.k = (int32_t)(jk / d.ny);
    }
    return o;
}

// Voxel heights of the weighted prior (Eq. srt_inversion): the height of
// voxel (i, j, k) is |c0 + (i, j, k) * step| + offset, c0 the first voxel's
// centre relative to the height origin.  FP32, recomputed where needed (no
// height array in memory).
struct HeightDev {
    float c0[3];
    float step[3];
    float offset;
    int32_t pad;
};

__device__ inline float height_of(float dx, float dy, float dz, float off)
{
    return sqrtf(fmaf(dx, dx, fmaf(dy, dy, dz * dz))) + off;
}

// lambda_r (D^T D x)_v + lambda_t (D_t^T D_t x)_v, or with kHeight
// lambda_r (R D^T D R x)_v + lambda_t (D_t^T D_t x)_v: forward differences
// between in-range neighbours only (free ends).
// c = x[idx]; xm, xp: x one frame before and after (read only where those
// frames exist and lambda_t != 0).
template <bool kHeight = false>
__device__ inline float prior_core(const float *__restrict__ x, const Dims &d, int64_t idx, const VoxIdx &c_,
                                   float lr, float lt, const HeightDev &hd, float c, float xm, float xp)
{
    const int32_t i = c_.i, j = c_.j, k = c_.k;
    const int64_t f = c_.f;
    const int64_t pl = (int64_t)d.nx * d.ny;
    float s = 0.0f, w = 1.0f;
    if constexpr (!kHeight) {
        if (i > 0) s += c - x[idx - 1];
        if (i < d.nx - 1) s += c - x[idx + 1];
        if (j > 0) s += c - x[idx - d.nx];
        if (j < d.ny - 1) s += c - x[idx + d.nx];
        if (k > 0) s += c - x[idx - pl];
        if (k < d.nz - 1) s += c - x[idx + pl];
    } else {
        // (R D^T D R x)_v = h_v sum over neighbours n of (h_v x_v - h_n x_n)
        const float dx = fmaf((float)i, hd.step[0], hd.c0[0]);
        const float dy = fmaf((float)j, hd.step[1], hd.c0[1]);
        const float dz = fmaf((float)k, hd.step[2], hd.c0[2]);
        w = height_of(dx, dy, dz, hd.offset);
        const float hc = w * c;
        if (i > 0) s += hc - height_of(dx - hd.step[0], dy, dz, hd.offset) * x[idx - 1];
        if (i < d.nx - 1) s += hc - height_of(dx + hd.step[0], dy, dz, hd.offset) * x[idx + 1];
        if (j > 0) s += hc - height_of(dx, dy - hd.step[1], dz, hd.offset) * x[idx - d.nx];
        if (j < d.ny - 1) s += hc - height_of(dx, dy + hd.step[1], dz, hd.offset) * x[idx + d.nx];
        if (k > 0) s += hc - height_of(dx, dy, dz - hd.step[2], hd.offset) * x[idx - pl];
        if (k < d.nz - 1) s += hc - height_of(dx, dy, dz + hd.step[2], hd.offset) * x[idx + pl];
    }
    float out = lr * (w * s);
    if (lt != 0.0f) {
        float t = 0.0f;
        if (f > 0) t += c - xm;
        if (f < d.nf - 1) t += c - xp;
        out += lt * t;
    }
    return out;
}

template <bool kHeight = false>
__device__ inline float prior_at(const float *__restrict__ x, const Dims &d, int64_t idx, const VoxIdx &c,
                                 float lr, float lt, const HeightDev &hd = HeightDev{})
{
    const bool tm = lt != 0.0f;
    const float xm = tm && c.f > 0 ? x[idx - d.nvox] : 0.0f;
    const float xp = tm && c.f < d.nf - 1 ? x[idx + d.nvox] : 0.0f;
    return prior_core<kHeight>(x, d, idx, c, lr, lt, hd, x[idx], xm, xp);
}

template <bool kHeight>
__global__ __launch_bounds__(kThreads) void k_prior(const float *__restrict__ x,
                                                    float *__restrict__ out, Dims d, float lr,
                                                    float lt, int accumulate, HeightDev hd)
{
    for (int64_t i = (int64_t)blockIdx.x * kThreads + threadIdx.x; i < d.total;
         i += (int64_t)gridDim.x * kThreads) {
        const float v = prior_at<kHeight>(x, d, i, vox_index(d, i), lr, lt, hd);
        out[i] = accumulate ? out[i] + v : v;
    }
}

// --------------------------------------------------------- reductions

// Reduce NV doubles per thread over the whole grid.  Returns true in the
// last workgroup to finish, whose thread 0 then holds the grid totals in t.
// The partials are summed in block order: deterministic.
template <int NV>
__device__ inline bool grid_reduce(const double (&a)[NV], const Workspace &ws, double (&t)[NV])
{
    __shared__ double lds[4];
    __shared__ int last;
    double sa[NV];
#pragma unroll
    for (int k = 0; k < NV; ++k) sa[k] = block_sum(a[k], lds);
    if (threadIdx.x == 0) {
#pragma unroll
        for (int k = 0; k < NV; ++k) ws.partials[4 * blockIdx.x + k] = sa[k];
        __threadfence();
        const unsigned prev = atomicAdd(ws.counter, 1u);
        last = (prev == gridDim.x - 1);
    }
    __syncthreads();
    if (!last) return false;
    __threadfence();
    // every load of this thread issued before any is summed (one memory
    // latency instead of one per partial); partials in a fixed order
    double pa[NV];
#pragma unroll
    for (int k = 0; k < NV; ++k) pa[k] = 0.0;
    constexpr int kPer = kRedBlocks / kThreads;
    double v[kPer][NV];
#pragma unroll
    for (int u = 0; u < kPer; ++u) {
        const int i = threadIdx.x + u * kThreads;
#pragma unroll
        for (int k = 0; k < NV; ++k)
            v[u][k] = i < (int)gridDim.x ? __builtin_nontemporal_load(&ws.partials[4 * i + k]) : 0.0;
    }
#pragma unroll
    for (int u = 0; u < kPer; ++u)
#pragma unroll
        for (int k = 0; k < NV; ++k) pa[k] += v[u][k];
#pragma unroll
    for (int k = 0; k < NV; ++k) t[k] = block_sum(pa[k], lds);
    if (threadIdx.x == 0) *ws.counter = 0u;
    return true;
}

__device__ inline bool grid_reduce2(double a, double b, const Workspace &ws, double &t0, double &t1)
{
    const double in[2] = {a, b};
    double out[2];
    const bool last = grid_reduce<2>(in, ws, out);
    t0 = out[0];
    t1 = out[1];
    return last;
}

// Total of the per-workgroup partials that the previous kernel left in
// part[0 .. nb), summed in the same fixed order as grid_reduce
// (deterministic) by every workgroup that needs it: the launch boundary has
// made them visible, so their producer needs no fence and no counter (a
// device-scope release per workgroup writes back the XCD's L2).  Valid in
// every thread.
__device__ inline double sum_partials(const double *__restrict__ part, int nb)
{
    __shared__ double lds[4];
    __shared__ double tot;
    constexpr int kPer = kIterBlocks / kThreads;
    double v[kPer];
#pragma unroll
    for (int u = 0; u < kPer; ++u) {
        const int i = threadIdx.x + u * kThreads;
        v[u] = i < nb ? part[i] : 0.0;
    }
    double pa = 0.0;
#pragma unroll
    for (int u = 0; u < kPer; ++u) pa += v[u];
    const double t = block_sum(pa, lds);
    if (threadIdx.x == 0) tot = t;
    __syncthreads();
    return tot;
}

// This workgroup's share of a sum, for sum_partials in the next kernel.
__device__ inline void put_partial(double a, double *part)
{
    __shared__ double lds[4];
    const double t = block_sum(a, lds);
    if (threadIdx.x == 0) part[blockIdx.x] = t;
}

__device__ inline bool bad(double v) { return !isfinite(v); }

// The stop flag as this workgroup's thread 0 reads it, the same in all of
// its threads: workgroup 0 of the running kernel may raise it while the
// others start, and their threads must agree before a workgroup barrier.
__device__ inline bool stopped(const CgState *st)
{
    __shared__ int f;
    if (threadIdx.x == 0) f = st->done;
    __syncthreads();
    return f != 0;
}

// alpha = rr / p.q from k_cg_q's partials, the same in every workgroup;
// workgroup 0 records it.  Returns false (every workgroup alike) when the
// step is not usable, and then raises the stop flag.
__device__ inline bool take_alpha(const Workspace &ws, double &alpha)
{
    CgState &s = *ws.st;
    const double tpq = sum_partials(ws.cpart, ws.nq);
    const double rr = s.rr;
    alpha = rr / tpq;
    const bool ok = !bad(alpha) && tpq > 0.0;
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        s.pq = tpq;
        s.alpha = alpha;
        s.rr_prev = rr;
        if (!ok) {
            s.nonfinite = 1;
            s.done = 1;
        }
    }
    return ok;
}

// r = b - q (or r = b), p = r, q = 0; state from r.r and b.b.
__global__ __launch_bounds__(kThreads) void k_cg_start(const float *__restrict__ b,
                                                       float *__restrict__ r, float *__restrict__ p,
                                                       float *__restrict__ q, int64_t n,
                                                       int subtract_q, Workspace ws, double rtol,
                                                       int32_t max_iter, int32_t iter0)
{
    double rr = 0.0, bb = 0.0;
    for (int64_t i = (int64_t)blockIdx.x * kThreads + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * kThreads) {
        const float bv = b[i];
        const float rv = subtract_q ? (float)((double)bv - (double)q[i]) : bv;
        r[i] = rv;
        p[i] = rv;
        q[i] = 0.0f;
        rr += (double)rv * rv;
        bb += (double)bv * bv;
    }
    double trr, tbb;
    if (grid_reduce2(rr, bb, ws, trr, tbb) && threadIdx.x == 0) {
        CgState &s = *ws.st;
        s.rr = trr;
        s.res2 = trr;
        s.bb = tbb;
        s.thresh2 = rtol > 0.0 ? rtol * rtol * tbb : -1.0;
        s.iter = iter0;
        s.max_iter = max_iter;
        s.nonfinite = bad(trr) || bad(tbb);
        s.done = s.nonfinite || tbb == 0.0 || trr <= s.thresh2 || iter0 >= max_iter;
        ws.hist[iter0] = tbb > 0.0 ? sqrt(trr / tbb) : 0.0;
    }
}

// q = M (q + prior(p)); per-workgroup partials of p.q.  Each workgroup
// takes one contiguous span of the vector, and the spans of one XCD are
// adjacent (MI355X deals consecutive workgroups to its 8 XCDs in turn), so
// the stencil's neighbours a row and a plane away were read into the same
// XCD's L2 by its own workgroups; with one frame per XCD, the temporal
// neighbours are the lines that the neighbouring XCDs are reading at the
// same time.
template <bool kHeight>
__global__ __launch_bounds__(kThreads) void k_cg_q(const float *__restrict__ p,
                                                   float *__restrict__ q,
                                                   const uint8_t *__restrict__ map_mask, Dims d,
                                                   float lr, float lt, Workspace ws, HeightDev hd)
{
    if (ws.st->done) return;
    const int64_t span = ((d.total + gridDim.x - 1) / gridDim.x + kThreads - 1) / kThreads * kThreads;
    const int64_t beg = xcd_remap(blockIdx.x, gridDim.x) * span;
    const int64_t end = beg + span < d.total ? beg + span : d.total;
    double pq = 0.0;
    for (int64_t i = beg + threadIdx.x; i < end; i += kThreads) {
        const VoxIdx c = vox_index(d, i);
        float v = q[i] + prior_at<kHeight>(p, d, i, c, lr, lt, hd);
        if (map_mask && !map_mask[c.rem]) v = 0.0f;
        q[i] = v;
        pq += (double)p[i] * v;
    }
    put_partial(pq, ws.cpart);
}

// k_cg_q for the plain prior on rows of a multiple of four voxels (and a
// map mask, if any, on a 4-byte boundary): each thread takes four
// consecutive voxels of one row, so the centre values, the row and plane
// neighbours, the temporal neighbours, q and the mask are 16-byte (4-byte)
// loads, and the voxel coordinates are derived once per four.  Per voxel
// the sum runs in prior_core's order, so q is the same, bit for bit; the
// p.q partial sums the same products in another order.
__device__ inline float4 ld4(const float *__restrict__ a, int64_t i)
{
    return *reinterpret_cast<const float4 *>(a + i);
}

__global__ __launch_bounds__(kThreads) void k_cg_q4(const float *__restrict__ p, float *__restrict__ q,
                                                    const uint8_t *__restrict__ map_mask, Dims d, float lr,
                                                    float lt, Workspace ws)
{
    if (ws.st->done) return;
    const int64_t n4 = d.total >> 2;
    const int64_t span = ((n4 + gridDim.x - 1) / gridDim.x + kThreads - 1) / kThreads * kThreads;
    const int64_t beg = xcd_remap(blockIdx.x, gridDim.x) * span;
    const int64_t end = beg + span < n4 ? beg + span : n4;
    const int64_t pl = (int64_t)d.nx * d.ny;
    const float4 zero4 = make_float4(0.f, 0.f, 0.f, 0.f);
    double pq = 0.0;
    for (int64_t g = beg + threadIdx.x; g < end; g += kThreads) {
        const int64_t idx = g << 2;
        const VoxIdx c = vox_index(d, idx);
        const float4 c4 = ld4(p, idx);
        const float xl = c.i > 0 ? p[idx - 1] : 0.0f;
        const float xr = c.i + 4 < d.nx ? p[idx + 4] : 0.0f;
        const float4 ym = c.j > 0 ? ld4(p, idx - d.nx) : zero4;
        const float4 yp = c.j < d.ny - 1 ? ld4(p, idx + d.nx) : zero4;
        const float4 zm = c.k > 0 ? ld4(p, idx - pl) : zero4;
        const float4 zp = c.k < d.nz - 1 ? ld4(p, idx + pl) : zero4;
        const bool tm = lt != 0.0f && c.f > 0, tp = lt != 0.0f && c.f < d.nf - 1;
        const float4 fm = tm ? ld4(p, idx - d.nvox) : zero4;
        const float4 fp = tp ? ld4(p, idx + d.nvox) : zero4;
        float4 q4 = ld4(q, idx);
        uint32_t m4 = 0xffffffffu;
        if (map_mask) m4 = *reinterpret_cast<const uint32_t *>(map_mask + c.rem);
        const float cv[4] = {c4.x, c4.y, c4.z, c4.w};
        const float ymv[4] = {ym.x, ym.y, ym.z, ym.w}, ypv[4] = {yp.x, yp.y, yp.z, yp.w};
        const float zmv[4] = {zm.x, zm.y, zm.z, zm.w}, zpv[4] = {zp.x, zp.y, zp.z, zp.w};
        const float fmv[4] = {fm.x, fm.y, fm.z, fm.w}, fpv[4] = {fp.x, fp.y, fp.z, fp.w};
        float qv[4] = {q4.x, q4.y, q4.z, q4.w};
#pragma unroll
        for (int e = 0; e < 4; ++e) {
            const float cc = cv[e];
            const float left = e > 0 ? cv[e - 1] : xl, right = e < 3 ? cv[e + 1] : xr;
            float sum = 0.0f;
            if (c.i + e > 0) sum += cc - left;
            if (c.i + e < d.nx - 1) sum += cc - right;
            if (c.j > 0) sum += cc - ymv[e];
            if (c.j < d.ny - 1) sum += cc - ypv[e];
            if (c.k > 0) sum += cc - zmv[e];
            if (c.k < d.nz - 1) sum += cc - zpv[e];
            float out = lr * sum;
            if (lt != 0.0f) {
                float t = 0.0f;
                if (c.f > 0) t += cc - fmv[e];
                if (c.f < d.nf - 1) t += cc - fpv[e];
                out += lt * t;
            }
            float v = qv[e] + out;
            if (!((m4 >> (8 * e)) & 0xffu)) v = 0.0f;
            qv[e] = v;
            pq += (double)cc * v;
        }
        *reinterpret_cast<float4 *>(q + idx) = make_float4(qv[0], qv[1], qv[2], qv[3]);
    }
    put_partial(pq, ws.cpart);
}

// alpha = rr / p.q; x += alpha p; r -= alpha q; q = 0 when the next P^T
// adds into q (zero_q; the blocked P^T writes q outright); per-workgroup
// partials of the new r.r.
__global__ __launch_bounds__(kThreads) void k_cg_xr(float *__restrict__ x, float *__restrict__ r,
                                                    const float *__restrict__ p,
                                                    float *__restrict__ q, int64_t n, Workspace ws,
                                                    int32_t zero_q)
{
    if (stopped(ws.st)) return;
    double alpha;
    if (!take_alpha(ws, alpha)) return;
    double rr = 0.0;
    for (int64_t i = (int64_t)blockIdx.x * kThreads + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * kThreads) {
        const float pv = p[i];
        x[i] = (float)((double)x[i] + alpha * pv);
        const float rv = (float)((double)r[i] - alpha * q[i]);
        r[i] = rv;
        if (zero_q) q[i] = 0.0f;
        rr += (double)rv * rv;
    }
    put_partial(rr, ws.cpart + kIterBlocks);
}

// rr_new = r.r from k_cg_xr's partials; beta = rr_new / rr; p = r + beta p.
// Workgroup 0 commits the iteration (rr, history, stop test).  rr itself is
// not read here (beta takes rr_prev), so that commit races with no reader;
// a workgroup that already sees the stop flag leaves p alone, which no later
// step reads (a restart rebuilds p from r).
__global__ __launch_bounds__(kThreads) void k_cg_p(const float *__restrict__ r,
                                                   float *__restrict__ p, int64_t n, Workspace ws)
{
    if (stopped(ws.st)) return;
    CgState &s = *ws.st;
    const double trr = sum_partials(ws.cpart + kIterBlocks, gridDim.x);
    const double beta = trr / s.rr_prev;
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        s.beta = beta;
        s.rr = trr;
        s.res2 = trr;
        s.iter += 1;
        ws.hist[s.iter] = sqrt(trr / s.bb);
        if (bad(trr) || bad(beta)) s.nonfinite = 1;
        s.done = s.nonfinite || trr <= s.thresh2 || s.iter >= s.max_iter;
    }
    for (int64_t i = (int64_t)blockIdx.x * kThreads + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * kThreads)
        p[i] = (float)((double)r[i] + beta * p[i]);
}

// ---- flexible CG (preconditioner network z = ||r|| N(r / ||r||))

// Set-up after k_cg_start: the first direction will be p = z (beta = 0).
__global__ void k_fcg_init(Workspace ws, int32_t window, double min_drop)
{
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    CgState &s = *ws.st;
    s.alpha = 0.0;
    s.rr_prev = s.rr;
    s.window = window;
    s.drop2 = (1.0 - min_drop) * (1.0 - min_drop);
    s.res_prev = s.res2;
    s.stall = 0;
    s.restart = 0;
    s.net_off = s.done || s.fellback;
}

// x += alpha p; r -= alpha q (q is kept for beta); per-workgroup partials
// of the new r.r, which k_fcg_commit sums.
__global__ __launch_bounds__(kThreads) void k_fcg_xr(float *__restrict__ x, float *__restrict__ r,
                                                     const float *__restrict__ p,
                                                     const float *__restrict__ q, int64_t n,
                                                     Workspace ws)
{
    if (stopped(ws.st)) return;
    double alpha;
    if (!take_alpha(ws, alpha)) return;
    double rr = 0.0;
    for (int64_t i = (int64_t)blockIdx.x * kThreads + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * kThreads) {
        x[i] = (float)((double)x[i] + alpha * p[i]);
        const float rv = (float)((double)r[i] - alpha * q[i]);
        r[i] = rv;
        rr += (double)rv * rv;
    }
    put_partial(rr, ws.cpart + kIterBlocks);
}

// One workgroup: res2 = r.r from k_fcg_xr's `nparts` partials, then the
// iteration's commit (history, stall test, fall-back, stop test) before the
// network reads ||r|| and its skip flag.  A single small workgroup after the
// vector pass costs less than a last-workgroup reduction inside it (one
// device-scope fence per workgroup).
__global__ __launch_bounds__(kThreads) void k_fcg_commit(Workspace ws, int32_t nparts)
{
    if (stopped(ws.st)) return;
    const double trr = sum_partials(ws.cpart + kIterBlocks, nparts);
    if (threadIdx.x != 0) return;
    CgState &s = *ws.st;
    s.res_prev = s.res2;
    s.res2 = trr;
    s.iter += 1;
    ws.hist[s.iter] = sqrt(trr / s.bb);
    if (bad(trr)) s.nonfinite = 1;
    s.stall = trr > s.drop2 * s.res_prev ? s.stall + 1 : 0;
    if (!s.fellback && s.stall >= s.window) {
        s.fellback = 1;
        s.fb_iter = s.iter;
        s.restart = 1;
        s.stall = 0;
    }
    s.done = s.nonfinite || trr <= s.thresh2 || s.iter >= s.max_iter;
    s.net_off = s.done || s.fellback;
}

// z.r, z.q, r.r, r.q per workgroup (for k_fcg_p); q = 0 when the next P^T
// adds into q (zero_q).  Workgroup 0 snapshots the fall-back state that
// k_fcg_p reads while it rewrites it.
__global__ __launch_bounds__(kThreads) void k_fcg_dots(const float *__restrict__ z,
                                                       const float *__restrict__ r,
                                                       float *__restrict__ q, int64_t n,
                                                       Workspace ws, int32_t zero_q)
{
    if (stopped(ws.st)) return;
    const bool usez = !ws.st->fellback;
    double a[4] = {0.0, 0.0, 0.0, 0.0};
    for (int64_t i = (int64_t)blockIdx.x * kThreads + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * kThreads) {
        const double rv = r[i], qv = q[i];
        const double zv = usez ? (double)z[i] : 0.0;
        a[0] += zv * rv;
        a[1] += zv * qv;
        a[2] += rv * rv;
        a[3] += rv * qv;
        if (zero_q) q[i] = 0.0f;
    }
#pragma unroll
    for (int k = 0; k < 4; ++k) put_partial(a[k], ws.cpart + k * kIterBlocks);
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        ws.st->fb_snap = ws.st->fellback;
        ws.st->rs_snap = ws.st->restart;
    }
}

// beta from k_fcg_dots' totals: Polak-Ribiere -alpha z.q / (z.r)_old, or
// plain CG after the fall-back (and 0 on a restart); a direction with
// z.r <= 0 (or non-finite) triggers the fall-back.  Every workgroup takes
// the same decisions from the same totals and the snapshot; workgroup 0
// commits them.  Then p = z + beta p (or r + beta p after the fall-back).
__global__ __launch_bounds__(kThreads) void k_fcg_p(const float *__restrict__ z,
                                                    const float *__restrict__ r,
                                                    float *__restrict__ p, int64_t n, Workspace ws)
{
    if (stopped(ws.st)) return;
    CgState &s = *ws.st;
    double t[4];
#pragma unroll
    for (int k = 0; k < 4; ++k) t[k] = sum_partials(ws.cpart + k * kIterBlocks, gridDim.x);
    const bool fb0 = s.fb_snap != 0;
    const bool fb = fb0 || !(t[0] > 0.0 && !bad(t[0]));
    const bool rs = s.rs_snap != 0 || fb != fb0;
    double num, beta;
    if (fb) {
        num = t[2];
        beta = rs ? 0.0 : num / s.rr_prev;
    } else {
        num = t[0];
        beta = -s.alpha * t[1] / s.rr_prev;
    }
    const bool stop = bad(beta) || bad(num);
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        if (fb && !fb0) {
            s.fellback = 1;
            s.fb_iter = s.iter;
        }
        if (stop) {
            s.nonfinite = 1;
            s.done = 1;
        }
        s.beta = beta;
        s.rr = num;
        s.restart = 0;
        s.net_off = s.done || s.fellback;
    }
    if (stop) return;
    const float *src = fb ? r : z;
    for (int64_t i = (int64_t)blockIdx.x * kThreads + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * kThreads)
        p[i] = (float)((double)src[i] + beta * p[i]);
}

// q = M (q + prior(x)); aux = |b - q|^2 (true residual of x).
template <bool kHeight>
__global__ __launch_bounds__(kThreads) void k_true_res(const float *__restrict__ x,
                                                       float *__restrict__ q,
                                                       const float *__restrict__ b,
                                                       const uint8_t *__restrict__ map_mask,
                                                       Dims d, float lr, float lt, Workspace ws, HeightDev hd)
{
    double rr = 0.0;
    for (int64_t i = (int64_t)blockIdx.x * kThreads + threadIdx.x; i < d.total;
         i += (int64_t)gridDim.x * kThreads) {
        const VoxIdx c = vox_index(d, i);
        float v = q[i] + prior_at<kHeight>(x, d, i, c, lr, lt, hd);
        if (map_mask && !map_mask[c.rem]) v = 0.0f;
        q[i] = v;
        const double e = (double)b[i] - v;
        rr += e * e;
    }
    double t, unused;
    if (grid_reduce2(rr, 0.0, ws, t, unused) && threadIdx.x == 0) ws.st->aux = t;
}

// aux = number of non-finite values among the unmasked pixels of y.
__global__ __launch_bounds__(kThreads) void k_count_nonfinite(const float *__restrict__ y, int64_t n,
                                                              const uint8_t *__restrict__ data_mask,
                                                              Workspace ws)
{
    double bad_count = 0.0;
    for (int64_t i = (int64_t)blockIdx.x * kThreads + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * kThreads)
        if ((!data_mask || data_mask[i]) && !isfinite(y[i])) bad_count += 1.0;
    double t, unused;
    if (grid_reduce2(bad_count, 0.0, ws, t, unused) && threadIdx.x == 0) ws.st->aux = t;
}

// x = M x (masked start point).
__global__ __launch_bounds__(kThreads) void k_mask(float *__restrict__ x,
                                                   const uint8_t *__restrict__ map_mask, Dims d)
{
    for (int64_t i = (int64_t)blockIdx.x * kThreads + threadIdx.x; i < d.total;
         i += (int64_t)gridDim.x * kThreads)
        if (!map_mask[vox_index(d, i).rem]) x[i] = 0.0f;
}

// ------------------------------------------------------------ host side

static Dims dims_of(const tomo_cube &c)
{
    Dims d;
    d.nx = c.nx;
    d.ny = c.ny;
    d.nz = c.nz;
    d.nf = c.nframes;
    d.nvox = (int64_t)c.nx * c.ny * c.nz;
    d.total = d.nvox * c.nframes;
    return d;
}

static unsigned elem_blocks(int64_t n)
{
    int64_t nb = (n + kThreads - 1) / kThreads;
    return (unsigned)(nb > kRedBlocks ? kRedBlocks : (nb < 1 ? 1 : nb));
}

static unsigned iter_blocks(int64_t n)
{
    int64_t nb = (n + kThreads - 1) / kThreads;
    return (unsigned)(nb > kIterBlocks ? kIterBlocks : (nb < 1 ? 1 : nb));
}

// Height parameters of the weighted prior for this cube (h == NULL: none).
static int height_dev(const tomo_cube &c, const tomo_height *h, HeightDev &hd, const char *who)
{
    memset(&hd, 0, sizeof(hd));
    if (!h) return TOMO_OK;
    if (!isfinite(h->center[0]) || !isfinite(h->center[1]) || !isfinite(h->center[2]) || !isfinite(h->offset))
        return set_error(TOMO_EINVAL, "%s: height centre and offset must be finite", who);
    const int32_t n[3] = {c.nx, c.ny, c.nz};
    for (int a = 0; a < 3; ++a) {
        const double step = (c.box_max[a] - c.box_min[a]) / (double)n[a];
        hd.step[a] = (float)step;
        hd.c0[a] = (float)(c.box_min[a] + 0.5 * step - h->center[a]);
    }
    hd.offset = (float)h->offset;
    return TOMO_OK;
}

// The fused q pass of every CG: the four-voxel kernel where the rows allow
// it (plain prior, rows of a multiple of four voxels, map mask on a 4-byte
// boundary), else the one-voxel kernel.
static void launch_cg_q(bool hw, unsigned blocks, hipStream_t s, const float *p, float *q, const uint8_t *mm,
                        const Dims &d, float lr, float lt, const Workspace &ws, const HeightDev &hd)
{
    if (hw) {
        hipLaunchKernelGGL(k_cg_q<true>, dim3(blocks), dim3(kThreads), 0, s, p, q, mm, d, lr, lt, ws, hd);
    } else if (d.nx % 4 == 0 && ((uintptr_t)mm & 3u) == 0) {
        hipLaunchKernelGGL(k_cg_q4, dim3(blocks), dim3(kThreads), 0, s, p, q, mm, d, lr, lt, ws);
    } else {
        hipLaunchKernelGGL(k_cg_q<false>, dim3(blocks), dim3(kThreads), 0, s, p, q, mm, d, lr, lt, ws, hd);
    }
}

template <typename... Args>
static void launch_true_res(bool hw, unsigned blocks, hipStream_t s, Args... a)
{
    if (hw) hipLaunchKernelGGL(k_true_res<true>, dim3(blocks), dim3(kThreads), 0, s, a...);
    else hipLaunchKernelGGL(k_true_res<false>, dim3(blocks), dim3(kThreads), 0, s, a...);
}

// Device allocations of one solve, released on every exit path: stream-
// ordered scratch; or consecutive 256-byte aligned pieces of a caller's
// workspace or of one stream-ordered block (arena; `owned` is that block,
// freed with the buffers); or, to size such a workspace (measure), no
// memory at all: every piece is a non-null placeholder that nothing
// dereferences.
struct SolveBuffers {
    hipStream_t s = nullptr;
    std::vector<void *> ptrs;
    void *owned = nullptr;
    char *arena = nullptr;
    size_t arena_bytes = 0;
    bool measure = false;
    size_t used = 0;  // arena or measure: bytes taken so far
    void *alloc(size_t bytes)
    {
        if (arena || measure) {
            const size_t at = (used + 255) & ~(size_t)255;
            if (measure) {
                used = at + bytes;
                return reinterpret_cast<void *>((uintptr_t)256);
            }
            if (at + bytes > arena_bytes) return nullptr;
            used = at + bytes;
            return arena + at;
        }
        void *p = nullptr;
        if (scratch_alloc(&p, bytes, s) != hipSuccess) return nullptr;
        ptrs.push_back(p);
        return p;
    }
    ~SolveBuffers()
    {
        for (void *p : ptrs) (void)scratch_free(p, s);
        if (owned) (void)scratch_free(owned, s);
    }
};

// The device buffers of tomo_cg_solve on one geometry: the vectors, the
// reduction workspace, the blocked P^T's scratch and ray table (when the
// tuning asks for one), P's bricked copy (when the tuning walks bricks) and
// the network's activations (flexible CG).  One sequence of allocations
// serves the solve and the workspace size query.
struct CgBufs {
    float *b = nullptr, *r = nullptr, *p = nullptr, *q = nullptr, *img = nullptr, *z = nullptr;
    float *bricks = nullptr;
    Workspace ws;
    int bps = TOMO_BP_BLOCKED;
    void *bscr = nullptr;
    size_t bscr_bytes = 0;
    void *table = nullptr;  // ray table memory (null: none)
    void *netws = nullptr;
};

static bool cg_buffers(SolveBuffers &buf, const Plan &plan, const tomo_geometry *g, const tomo_cg_params *prm,
                       CgBufs &o)
{
    const Dims d = dims_of(g->cube);
    const int64_t n = d.total;
    const tomo_tuning tu = tuning_for(plan);
    o.b = (float *)buf.alloc(sizeof(float) * n);
    o.r = (float *)buf.alloc(sizeof(float) * n);
    o.p = (float *)buf.alloc(sizeof(float) * n);
    o.q = (float *)buf.alloc(sizeof(float) * n);
    o.img = (float *)buf.alloc(sizeof(float) * plan.npix);
    o.ws.partials = (double *)buf.alloc(sizeof(double) * 4 * kRedBlocks);
    o.ws.counter = (unsigned *)buf.alloc(sizeof(unsigned));
    o.ws.cpart = (double *)buf.alloc(sizeof(double) * 4 * kIterBlocks);
    o.ws.nq = (int32_t)iter_blocks(n);
    o.ws.st = (CgState *)buf.alloc(sizeof(CgState));
    o.ws.hist = (double *)buf.alloc(sizeof(double) * ((size_t)prm->max_iter + 1));
    bool ok = o.b && o.r && o.p && o.q && o.img && o.ws.partials && o.ws.counter && o.ws.cpart && o.ws.st &&
              o.ws.hist;
    // back-projection strategy and its scratch, fixed for the whole solve
    o.bps = resolve_bp_strategy(plan, prm->bp_strategy);
    if (o.bps == TOMO_BP_BLOCKED) {
        o.bscr_bytes = blocked_scratch_bytes(plan, blocked_shape(plan, tu), g->data_mask != nullptr);
        o.bscr = buf.alloc(o.bscr_bytes);
        ok = ok && o.bscr;
        const size_t nt = tu.bp_ray_table ? ray_table_bytes(plan) : 0;
        if (nt) {
            o.table = buf.alloc(nt);
            ok = ok && o.table;
        }
    }
    const size_t nbr = bricked_copy_bytes(plan, tu);
    if (nbr) {
        o.bricks = (float *)buf.alloc(nbr);
        ok = ok && o.bricks;
    }
    if (prm->precond) {
        o.z = (float *)buf.alloc(sizeof(float) * n);
        o.netws = buf.alloc(convnet_forward_ws_bytes(d.nvox));
        ok = ok && o.z && o.netws;
    }
    return ok;
}

struct EventPool {
    std::vector<hipEvent_t> ev;
    hipEvent_t get()
    {
        hipEvent_t e = nullptr;
        if (hipEventCreate(&e) != hipSuccess) return nullptr;
        ev.push_back(e);
        return e;
    }
    ~EventPool()
    {
        for (hipEvent_t e : ev) (void)hipEventDestroy(e);
    }
};

}  // namespace tomo

using namespace tomo;

extern "C" {

void tomo_cg_default_params(tomo_cg_params *p)
{
    if (!p) return;
    memset(p, 0, sizeof(*p));
    p->lambda_r = 1e-2;
    p->max_iter = 50;
    p->check_every = 10;
    p->fallback_window = 3;
    p->min_drop = 1e-6;
}

int tomo_apply_height_prior(const tomo_cube *cube, const tomo_height *h, double lambda_r, double lambda_t,
                            const float *x_d, float *out_d, int accumulate, tomo_stream stream)
{
    int rc = validate_cube(cube);
    if (rc) return rc;
    if (!x_d || !out_d) return set_error(TOMO_EINVAL, "tomo_apply_prior: NULL array");
    if (!(lambda_r >= 0) || !(lambda_t >= 0) || !isfinite(lambda_r) || !isfinite(lambda_t))
        return set_error(TOMO_EINVAL, "tomo_apply_prior: weights must be finite and >= 0");
    if (x_d == out_d) return set_error(TOMO_EINVAL, "tomo_apply_prior: x and out must differ");
    HeightDev hd;
    rc = height_dev(*cube, h, hd, "tomo_apply_height_prior");
    if (rc) return rc;
    const Dims d = dims_of(*cube);
    const dim3 grid(elem_blocks(d.total));
    if (h)
        hipLaunchKernelGGL(k_prior<true>, grid, dim3(kThreads), 0, (hipStream_t)stream, x_d, out_d, d,
                           (float)lambda_r, (float)lambda_t, accumulate, hd);
    else
        hipLaunchKernelGGL(k_prior<false>, grid, dim3(kThreads), 0, (hipStream_t)stream, x_d, out_d, d,
                           (float)lambda_r, (float)lambda_t, accumulate, hd);
    return hip_fail(hipGetLastError(), "prior kernel launch");
}

int tomo_apply_prior(const tomo_cube *cube, double lambda_r, double lambda_t, const float *x_d,
                     float *out_d, int accumulate, tomo_stream stream)
{
    return tomo_apply_height_prior(cube, nullptr, lambda_r, lambda_t, x_d, out_d, accumulate, stream);
}

size_t tomo_cg_workspace_bytes(const tomo_geometry *g, const tomo_cg_params *prm)
{
    if (!g || !prm || prm->max_iter < 0 || prm->use_graph || prm->bp_strategy < TOMO_BP_AUTO ||
        prm->bp_strategy > TOMO_BP_BLOCKED)
        return 0;
    int st = TOMO_OK;
    PlanRef plan = get_plan(g, &st);
    if (!plan) return 0;
    SolveBuffers m;
    m.measure = true;
    CgBufs sized;
    (void)cg_buffers(m, *plan, g, prm, sized);
    return m.used;
}

int tomo_cg_solve(const tomo_geometry *g, const float *y_d, float *x_d, const tomo_cg_params *prm,
                  tomo_cg_report *rep, tomo_stream stream)
{
    if (!y_d || !x_d || !prm || !rep) return set_error(TOMO_EINVAL, "tomo_cg_solve: NULL argument");
    if (!(prm->lambda_r >= 0) || !(prm->lambda_t >= 0) || !isfinite(prm->lambda_r) ||
        !isfinite(prm->lambda_t) || prm->max_iter < 0 || !(prm->rtol >= 0) ||
        !isfinite(prm->rtol) || prm->check_every < 1 || prm->record_count < 0 ||
        (prm->record_count > 0 && !prm->record_x && !prm->record_r))
        return set_error(TOMO_EINVAL, "tomo_cg_solve: invalid parameters");
    if (prm->bp_strategy < TOMO_BP_AUTO || prm->bp_strategy > TOMO_BP_BLOCKED)
        return set_error(TOMO_EINVAL, "tomo_cg_solve: unknown bp_strategy %d", prm->bp_strategy);
    if (prm->precond && (prm->fallback_window < 1 || !(prm->min_drop >= 0) || !(prm->min_drop < 1)))
        return set_error(TOMO_EINVAL, "tomo_cg_solve: fallback_window must be >= 1 and min_drop in [0, 1)");
    int st = TOMO_OK;
    PlanRef plan = get_plan(g, &st);
    if (!plan) return st;
    if (prm->lambda_t > 0 && g->cube.nframes < 2)
        return set_error(TOMO_EINVAL, "tomo_cg_solve: lambda_t needs nframes >= 2");
    if (prm->precond && g->cube.nframes != 1)
        return set_error(TOMO_EUNSUPPORTED, "tomo_cg_solve: the preconditioner needs nframes == 1");
    if (prm->use_graph) {  // graph-captured iterations: a batch of one
        if (prm->workspace)
            return set_error(TOMO_EUNSUPPORTED, "tomo_cg_solve: use_graph takes no caller workspace");
        if (prm->precond || prm->record_count > 0)
            return set_error(TOMO_EUNSUPPORTED, "tomo_cg_solve: use_graph without preconditioner or recording");
        tomo_batch bt = nullptr;
        int e = tomo_batch_create(g, 1, &bt);
        if (e) return e;
        e = tomo_batch_cg_solve(bt, &y_d, &x_d, prm, rep, stream);
        tomo_batch_destroy(bt);
        return e;
    }
    const bool fcg = prm->precond != nullptr;
    hipStream_t s = (hipStream_t)stream;
    const Dims d = dims_of(g->cube);
    const int64_t n = d.total;
    const float lr = (float)prm->lambda_r, lt = (float)prm->lambda_t;
    const int maxit = prm->max_iter;
    const bool hw = prm->height != nullptr;
    HeightDev hd;
    int hrc = height_dev(g->cube, prm->height, hd, "tomo_cg_solve");
    if (hrc) return hrc;

    SolveBuffers buf;
    buf.s = s;
    {
        SolveBuffers m;
        m.measure = true;
        CgBufs sized;
        (void)cg_buffers(m, *plan, g, prm, sized);
        if (prm->workspace) {
            if ((uintptr_t)prm->workspace & 255u)
                return set_error(TOMO_EINVAL, "tomo_cg_solve: the workspace must be 256-byte aligned");
            if (prm->workspace_bytes < m.used)
                return set_error(TOMO_EINVAL, "tomo_cg_solve: workspace of %zu bytes, %zu needed",
                                 prm->workspace_bytes, m.used);
            buf.arena = (char *)prm->workspace;
            buf.arena_bytes = prm->workspace_bytes;
        } else {
            // one block from the pool for all of the solve's buffers: the
            // pool then reuses the same block solve after solve (separate
            // pieces of a few hundred MB were measured to cost ~1 ms a solve)
            if (scratch_alloc(&buf.owned, m.used, s) != hipSuccess)
                return set_error(TOMO_ENOMEM, "tomo_cg_solve: device allocation of %zu bytes failed", m.used);
            buf.arena = (char *)buf.owned;
            buf.arena_bytes = m.used;
        }
    }
    CgBufs cb;
    if (!cg_buffers(buf, *plan, g, prm, cb)) return set_error(TOMO_ENOMEM, "tomo_cg_solve: device allocation failed");
    float *b = cb.b, *r = cb.r, *p = cb.p, *q = cb.q, *img = cb.img, *z = cb.z;
    Workspace ws = cb.ws;
    const int bps = cb.bps;
    // the blocked P^T writes every voxel of q; the atomic ones add into a
    // q that the x/r update has cleared
    const int bp_acc = bps == TOMO_BP_BLOCKED ? 0 : 1;
    void *bscr = cb.bscr;
    const size_t bscr_bytes = cb.bscr_bytes;
    void *netws = cb.netws;
    int rc = hip_fail(hipMemsetAsync(ws.counter, 0, sizeof(unsigned), s), "counter init");
    if (!rc) rc = hip_fail(hipMemsetAsync(ws.st, 0, sizeof(CgState), s), "state init");
    if (rc) return rc;
    // pinned host copy of the device state, one per calling thread, kept
    // until the process ends (a pinned allocation per call costs more than a
    // short solve's iterations)
    thread_local CgState *hst = nullptr;
    if (!hst && hipHostMalloc((void **)&hst, sizeof(CgState)) != hipSuccess) {
        hst = nullptr;
        return set_error(TOMO_ENOMEM, "tomo_cg_solve: pinned allocation failed");
    }

    const unsigned eb = elem_blocks(n);
    int n_proj = 0, n_bp = 0;
    const bool timed = rep->time_kernels != 0;
    EventPool evp;
    std::vector<hipEvent_t> evP, evB;  // start/stop pairs

    // non-finite data: report, do not iterate
    hipLaunchKernelGGL(k_count_nonfinite, dim3(elem_blocks(plan->npix)), dim3(kThreads), 0, s, y_d,
                       plan->npix, g->data_mask, ws);
    rc = hip_fail(hipMemcpyAsync(hst, ws.st, sizeof(CgState), hipMemcpyDeviceToHost, s), "state copy");
    if (!rc) rc = hip_fail(hipStreamSynchronize(s), "cg synchronise");
    if (rc) return rc;
    if (hst->aux > 0.0) {
        if (!prm->x0_given) {
            rc = launch_fill(x_d, n, 0.0f, s);
            if (!rc) rc = hip_fail(hipStreamSynchronize(s), "cg synchronise");
            if (rc) return rc;
        }
        memset(rep, 0, offsetof(tomo_cg_report, history));
        rep->status = TOMO_ENONFINITE;
        rep->fell_back = -1;
        rep->rel_res = rep->true_rel_res = NAN;
        rep->history_len = 0;
        return TOMO_OK;
    }

    // the rays' set-ups, once for all the solve's P^T
    RayTable tab_v;
    const RayTable *tab = nullptr;
    if (cb.table) {
        rc = ray_table_build(*plan, cb.table, tab_v, s);
        if (rc) return rc;
        tab = &tab_v;
    }
    // b = M P^T y
    rc = launch_backproject(*plan, g, y_d, b, false, true, bps, s, nullptr, bscr, bscr_bytes, tab);
    if (rc) return rc;
    ++n_bp;
    if (g->map_mask && prm->x0_given) {
        hipLaunchKernelGGL(k_mask, dim3(eb), dim3(kThreads), 0, s, x_d, g->map_mask, d);
    }
    auto apply_A_to = [&](const float *v) -> int {  // q = M (P^T P + prior) v, excluding the prior
        int e = launch_project_flagged(*plan, g, v, img, s, nullptr, cb.bricks);
        if (!e) e = launch_backproject(*plan, g, img, q, false, false, bps, s, nullptr, bscr, bscr_bytes, tab);
        n_proj++;
        n_bp++;
        return e;
    };
    if (prm->x0_given) {
        rc = apply_A_to(x_d);
        if (rc) return rc;
        launch_true_res(hw, eb, s, x_d, q, b, g->map_mask, d, lr, lt, ws, hd);
    } else {
        rc = launch_fill(x_d, n, 0.0f, s);
        if (rc) return rc;
    }
    hipLaunchKernelGGL(k_cg_start, dim3(eb), dim3(kThreads), 0, s, b, r, p, q, n,
                       prm->x0_given ? 1 : 0, ws, prm->rtol, maxit, 0);
    rc = hip_fail(hipGetLastError(), "cg start");
    if (rc) return rc;
    bool frags_ready = false;
    // flexible CG: first direction p = z = N(r) (or r if z.r <= 0)
    auto fcg_start = [&]() -> int {
        hipLaunchKernelGGL(k_fcg_init, dim3(1), dim3(64), 0, s, ws, prm->fallback_window, prm->min_drop);
        int e = convnet_forward_dev(g->cube, prm->precond, r, z, &ws.st->res2, g->map_mask, netws, s,
                                    !frags_ready, &ws.st->net_off);
        frags_ready = true;
        if (e) return e;
        hipLaunchKernelGGL(k_fcg_dots, dim3(eb), dim3(kThreads), 0, s, z, r, q, n, ws, bp_acc);
        hipLaunchKernelGGL(k_fcg_p, dim3(eb), dim3(kThreads), 0, s, z, r, p, n, ws);
        return hip_fail(hipGetLastError(), "fcg start");
    };
    if (fcg) {
        rc = fcg_start();
        if (rc) return rc;
    }
    int enqueued = 0;  // iterations enqueued so far (recording index)
    auto record = [&](int k) -> int {
        if (k >= prm->record_count) return TOMO_OK;
        int e = TOMO_OK;
        if (prm->record_x)
            e = hip_fail(hipMemcpyAsync(prm->record_x + (int64_t)k * n, x_d, sizeof(float) * n,
                                        hipMemcpyDeviceToDevice, s), "record x");
        if (!e && prm->record_r)
            e = hip_fail(hipMemcpyAsync(prm->record_r + (int64_t)k * n, r, sizeof(float) * n,
                                        hipMemcpyDeviceToDevice, s), "record r");
        return e;
    };
    rc = record(0);
    if (rc) return rc;

    auto enqueue_iteration = [&]() -> int {
        hipEvent_t e0 = nullptr, e1 = nullptr, e2 = nullptr;
        if (timed) {
            e0 = evp.get();
            e1 = evp.get();
            e2 = evp.get();
            (void)hipEventRecord(e0, s);
        }
        int e = launch_project_flagged(*plan, g, p, img, s, &ws.st->done, cb.bricks);
        if (timed) (void)hipEventRecord(e1, s);
        if (!e)
            e = launch_backproject(*plan, g, img, q, bp_acc != 0, false, bps, s, &ws.st->done, bscr, bscr_bytes,
                                   tab);
        if (timed) {
            (void)hipEventRecord(e2, s);
            evP.push_back(e0);
            evP.push_back(e1);
            evB.push_back(e1);
            evB.push_back(e2);
        }
        if (e) return e;
        launch_cg_q(hw, (unsigned)ws.nq, s, p, q, g->map_mask, d, lr, lt, ws, hd);
        if (!fcg) {
            hipLaunchKernelGGL(k_cg_xr, dim3(ws.nq), dim3(kThreads), 0, s, x_d, r, p, q, n, ws, bp_acc);
            hipLaunchKernelGGL(k_cg_p, dim3(ws.nq), dim3(kThreads), 0, s, r, p, n, ws);
        } else {
            hipLaunchKernelGGL(k_fcg_xr, dim3(ws.nq), dim3(kThreads), 0, s, x_d, r, p, q, n, ws);
            hipLaunchKernelGGL(k_fcg_commit, dim3(1), dim3(kThreads), 0, s, ws, ws.nq);
            e = convnet_forward_dev(g->cube, prm->precond, r, z, &ws.st->res2, g->map_mask, netws, s,
                                    false, &ws.st->net_off);
            if (e) return e;
            hipLaunchKernelGGL(k_fcg_dots, dim3(eb), dim3(kThreads), 0, s, z, r, q, n, ws, bp_acc);
            hipLaunchKernelGGL(k_fcg_p, dim3(eb), dim3(kThreads), 0, s, z, r, p, n, ws);
        }
        return hip_fail(hipGetLastError(), "cg iteration launch");
    };

    int done_iters = 0;
    double true_rel = -1.0;
    int restarts = 0;
    for (;;) {
        // run chunks until the device says stop.  Iterations enqueued past
        // convergence return at once but still cost their launches, so once
        // the residual's decay rate over the last chunk predicts the target
        // within check_every iterations, the next chunk stops there.
        int enq = 0;
        int chunk = prm->rtol > 0 ? prm->check_every : maxit;
        double ref_res2 = -1.0;
        int ref_iter = 0;
        while (done_iters + enq < maxit) {
            const int todo = chunk < maxit - done_iters - enq ? chunk : maxit - done_iters - enq;
            for (int k = 0; k < todo; ++k) {
                rc = enqueue_iteration();
                if (!rc) rc = record(++enqueued);
                if (rc) return rc;
            }
            enq += todo;
            rc = hip_fail(hipMemcpyAsync(hst, ws.st, sizeof(CgState), hipMemcpyDeviceToHost, s), "state copy");
            if (!rc) rc = hip_fail(hipStreamSynchronize(s), "cg synchronise");
            if (rc) return rc;
            if (hst->done) break;
            if (prm->rtol > 0) {
                chunk = prm->check_every;
                if (ref_res2 > 0.0 && hst->res2 > 0.0 && hst->thresh2 > 0.0 && hst->iter > ref_iter) {
                    const double rate = log(hst->res2 / ref_res2) / (double)(hst->iter - ref_iter);
                    if (rate < 0.0) {
                        const double need = log(hst->thresh2 / hst->res2) / rate;
                        if (need < (double)chunk) chunk = need < 1.0 ? 1 : (int)ceil(need);
                    }
                }
                ref_res2 = hst->res2;
                ref_iter = hst->iter;
            }
        }
        rc = hip_fail(hipMemcpyAsync(hst, ws.st, sizeof(CgState), hipMemcpyDeviceToHost, s), "state copy");
        if (!rc) rc = hip_fail(hipStreamSynchronize(s), "cg synchronise");
        if (rc) return rc;
        const int it_now = hst->iter;
        n_proj += it_now - done_iters;
        n_bp += it_now - done_iters;
        done_iters = it_now;
        if (hst->nonfinite) break;
        // true residual of x
        rc = apply_A_to(x_d);
        if (rc) return rc;
        launch_true_res(hw, eb, s, x_d, q, b, g->map_mask, d, lr, lt, ws, hd);
        rc = hip_fail(hipMemcpyAsync(hst, ws.st, sizeof(CgState), hipMemcpyDeviceToHost, s), "state copy");
        if (!rc) rc = hip_fail(hipStreamSynchronize(s), "cg synchronise");
        if (rc) return rc;
        true_rel = hst->bb > 0 ? sqrt(hst->aux / hst->bb) : 0.0;
        const bool unconfirmed = prm->rtol > 0 && true_rel > prm->rtol;
        if (!unconfirmed || done_iters >= maxit || restarts >= 8) break;
        // restart from the true residual
        ++restarts;
        hipLaunchKernelGGL(k_cg_start, dim3(eb), dim3(kThreads), 0, s, b, r, p, q, n, 1, ws,
                           prm->rtol, maxit, done_iters);
        rc = hip_fail(hipGetLastError(), "cg restart");
        if (rc) return rc;
        if (fcg) {
            rc = fcg_start();
            if (rc) return rc;
        }
    }

    // report
    rc = hip_fail(hipMemcpyAsync(hst, ws.st, sizeof(CgState), hipMemcpyDeviceToHost, s), "state copy");
    if (!rc) rc = hip_fail(hipStreamSynchronize(s), "cg synchronise");
    if (rc) return rc;
    rep->iters = hst->iter;
    rep->fell_back = hst->fellback ? hst->fb_iter : -1;
    rep->n_project = n_proj;
    rep->n_backproject = n_bp;
    rep->bnorm = sqrt(hst->bb);
    rep->rel_res = hst->bb > 0 ? sqrt(hst->res2 / hst->bb) : 0.0;
    rep->true_rel_res = true_rel;
    if (hst->nonfinite) rep->status = TOMO_ENONFINITE;
    else if (prm->rtol > 0 && !(true_rel <= prm->rtol)) rep->status = TOMO_ENOCONV;
    else rep->status = TOMO_OK;
    rep->history_len = 0;
    if (rep->history && rep->history_cap > 0) {
        const int nh = hst->iter + 1 < rep->history_cap ? hst->iter + 1 : rep->history_cap;
        rc = hip_fail(hipMemcpy(rep->history, ws.hist, sizeof(double) * nh, hipMemcpyDeviceToHost),
                      "history copy");
        if (rc) return rc;
        rep->history_len = nh;
    }
    rep->ms_project = rep->ms_backproject = 0.0;
    if (timed) {
        const size_t np = evP.size() / 2;
        const size_t use = (size_t)hst->iter < np ? (size_t)hst->iter : np;
        for (size_t k = 0; k < use; ++k) {
            float a = 0.f, bms = 0.f;
            (void)hipEventElapsedTime(&a, evP[2 * k], evP[2 * k + 1]);
            (void)hipEventElapsedTime(&bms, evB[2 * k], evB[2 * k + 1]);
            rep->ms_project += a;
            rep->ms_backproject += bms;
        }
    }
    return TOMO_OK;
}

// ------------------------------------------------------------ batched CG

int tomo_batch_cg_solve(tomo_batch bt, const float *const *y_d, float *const *x_d, const tomo_cg_params *prm,
                        tomo_cg_report *rep, tomo_stream stream)
{
    if (!bt || !y_d || !x_d || !prm || !rep) return set_error(TOMO_EINVAL, "tomo_batch_cg_solve: NULL argument");
    const int ns = bt->nsys;
    for (int k = 0; k < ns; ++k) {
        const tomo_cg_params &q = prm[k];
        if (!y_d[k] || !x_d[k]) return set_error(TOMO_EINVAL, "tomo_batch_cg_solve: NULL array (system %d)", k);
        if (!(q.lambda_r >= 0) || !(q.lambda_t >= 0) || !isfinite(q.lambda_r) || !isfinite(q.lambda_t) ||
            q.max_iter < 0 || !(q.rtol >= 0) || !isfinite(q.rtol))
            return set_error(TOMO_EINVAL, "tomo_batch_cg_solve: invalid parameters (system %d)", k);
        if (q.precond || q.record_count > 0 || q.record_x || q.record_r)
            return set_error(TOMO_EUNSUPPORTED, "tomo_batch_cg_solve: no preconditioner or recording");
        if (q.lambda_t > 0 && bt->geoms[(size_t)k].cube.nframes < 2)
            return set_error(TOMO_EINVAL, "tomo_batch_cg_solve: lambda_t needs nframes >= 2 (system %d)", k);
    }
    if (prm[0].check_every < 1) return set_error(TOMO_EINVAL, "tomo_batch_cg_solve: check_every must be >= 1");
    const int chunk = prm[0].check_every;
    const bool use_graph = prm[0].use_graph != 0;
    hipStream_t s = (hipStream_t)stream;

    struct Sys {
        Dims d;
        int64_t n, npix;
        float *b, *r, *p, *q, *img;
        Workspace ws;
        float lr, lt;
        bool hw;       // height-weighted spatial prior
        HeightDev hd;
        const uint8_t *mm, *dm;
        int maxit;
        double rtol;
        bool x0, skip;
        double true_rel;
        int restarts, n_proj, n_bp;
    };
    std::vector<Sys> sy((size_t)ns);
    SolveBuffers buf;
    buf.s = s;
    CgState *states = (CgState *)buf.alloc(sizeof(CgState) * (size_t)ns);
    if (!states) return set_error(TOMO_ENOMEM, "tomo_batch_cg_solve: device allocation failed");
    for (int k = 0; k < ns; ++k) {
        Sys &c = sy[(size_t)k];
        const tomo_geometry &g = bt->geoms[(size_t)k];
        c.d = dims_of(g.cube);
        c.n = c.d.total;
        c.npix = bt->plans[(size_t)k]->npix;
        c.lr = (float)prm[k].lambda_r;
        c.lt = (float)prm[k].lambda_t;
        c.hw = prm[k].height != nullptr;
        int hrc = height_dev(g.cube, prm[k].height, c.hd, "tomo_batch_cg_solve");
        if (hrc) return hrc;
        c.mm = g.map_mask;
        c.dm = g.data_mask;
        c.maxit = prm[k].max_iter;
        c.rtol = prm[k].rtol;
        c.x0 = prm[k].x0_given != 0;
        c.skip = false;
        c.true_rel = -1.0;
        c.restarts = 0;
        c.n_proj = c.n_bp = 0;
        c.b = (float *)buf.alloc(sizeof(float) * c.n);
        c.r = (float *)buf.alloc(sizeof(float) * c.n);
        c.p = (float *)buf.alloc(sizeof(float) * c.n);
        c.q = (float *)buf.alloc(sizeof(float) * c.n);
        c.img = (float *)buf.alloc(sizeof(float) * c.npix);
        c.ws.partials = (double *)buf.alloc(sizeof(double) * 4 * kRedBlocks);
        c.ws.counter = (unsigned *)buf.alloc(sizeof(unsigned));
        c.ws.cpart = (double *)buf.alloc(sizeof(double) * 4 * kIterBlocks);
        c.ws.nq = (int32_t)iter_blocks(c.n);
        c.ws.st = states + k;
        c.ws.hist = (double *)buf.alloc(sizeof(double) * ((size_t)c.maxit + 1));
        if (!c.b || !c.r || !c.p || !c.q || !c.img || !c.ws.partials || !c.ws.counter || !c.ws.cpart || !c.ws.hist)
            return set_error(TOMO_ENOMEM, "tomo_batch_cg_solve: device allocation failed");
        int rc = hip_fail(hipMemsetAsync(c.ws.counter, 0, sizeof(unsigned), s), "counter init");
        if (rc) return rc;
    }
    int rc = hip_fail(hipMemsetAsync(states, 0, sizeof(CgState) * (size_t)ns, s), "state init");
    if (rc) return rc;
    thread_local CgState *hst = nullptr;  // pinned, kept until the process ends
    if (!hst && hipHostMalloc((void **)&hst, sizeof(CgState) * kMaxSys) != hipSuccess) {
        hst = nullptr;
        return set_error(TOMO_ENOMEM, "tomo_batch_cg_solve: pinned allocation failed");
    }
    auto pull_states = [&]() -> int {
        int e = hip_fail(hipMemcpyAsync(hst, states, sizeof(CgState) * (size_t)ns, hipMemcpyDeviceToHost, s),
                         "state copy");
        if (!e) e = hip_fail(hipStreamSynchronize(s), "cg synchronise");
        return e;
    };

    // non-finite data: such systems are reported and take no further part
    for (auto &c : sy)
        hipLaunchKernelGGL(k_count_nonfinite, dim3(elem_blocks(c.npix)), dim3(kThreads), 0, s, y_d[&c - &sy[0]],
                           c.npix, c.dm, c.ws);
    rc = pull_states();
    if (rc) return rc;
    static const int one = 1;
    for (int k = 0; k < ns; ++k) {
        Sys &c = sy[(size_t)k];
        if (hst[k].aux > 0.0) {
            c.skip = true;
            rc = hip_fail(hipMemcpyAsync(&states[k].done, &one, sizeof(int), hipMemcpyHostToDevice, s), "flag");
            if (!rc && !c.x0) rc = launch_fill(x_d[k], c.n, 0.0f, s);
            if (rc) return rc;
        }
    }

    auto ops_of = [&](bool all_flags) {
        Operands o;
        memset(&o, 0, sizeof(o));
        for (int k = 0; k < ns; ++k)
            o.done[k] = (all_flags || sy[(size_t)k].skip) ? &states[k].done : nullptr;
        return o;
    };
    // The operand sets of the solve: the right-hand side, the true
    // residual's P and P^T, an iteration's P and P^T.
    enum { kRhs, kAxP, kAxPT, kItP, kItPT, kSets };
    Operands oset[kSets];
    for (int i = 0; i < kSets; ++i) oset[i] = ops_of(i != kAxP && i != kAxPT);
    for (int k = 0; k < ns; ++k) {
        const Sys &c = sy[(size_t)k];
        oset[kRhs].src[k] = y_d[k];
        oset[kRhs].dst[k] = c.b;
        oset[kAxP].src[k] = x_d[k];
        oset[kAxP].dst[k] = c.img;
        oset[kAxPT].src[k] = c.img;
        oset[kAxPT].dst[k] = c.q;
        oset[kItP].src[k] = c.p;
        oset[kItP].dst[k] = c.img;
        oset[kItPT].src[k] = c.img;
        oset[kItPT].dst[k] = c.q;  // every voxel of q written: the x/r update need not clear it
    }
    oset[kRhs].map = 1;
    // b = M P^T y
    rc = batch_backproject_ops(bt, oset[kRhs], s);
    if (rc) return rc;
    auto apply_A_x = [&]() -> int {  // q = (P^T P) x for every active system (prior added by k_true_res)
        int e = batch_project_ops(bt, oset[kAxP], s);
        if (!e) e = batch_backproject_ops(bt, oset[kAxPT], s);
        for (auto &c : sy)
            if (!c.skip) {
                c.n_proj++;
                c.n_bp++;
            }
        return e;
    };
    bool any_x0 = false;
    for (int k = 0; k < ns; ++k) {
        Sys &c = sy[(size_t)k];
        c.n_bp++;
        if (c.skip) continue;
        if (c.x0) {
            any_x0 = true;
            if (c.mm) hipLaunchKernelGGL(k_mask, dim3(elem_blocks(c.n)), dim3(kThreads), 0, s, x_d[k], c.mm, c.d);
        } else {
            rc = launch_fill(x_d[k], c.n, 0.0f, s);
            if (rc) return rc;
        }
    }
    if (any_x0) {
        rc = apply_A_x();
        if (rc) return rc;
        for (int k = 0; k < ns; ++k) {
            Sys &c = sy[(size_t)k];
            if (c.skip) continue;
            if (!c.x0) {  // that product was not needed for this system
                c.n_proj--;
                c.n_bp--;
                continue;
            }
            launch_true_res(c.hw, elem_blocks(c.n), s, x_d[k], c.q, c.b, c.mm, c.d, c.lr, c.lt, c.ws, c.hd);
        }
    }
    for (int k = 0; k < ns; ++k) {
        Sys &c = sy[(size_t)k];
        if (c.skip) continue;
        hipLaunchKernelGGL(k_cg_start, dim3(elem_blocks(c.n)), dim3(kThreads), 0, s, c.b, c.r, c.p, c.q, c.n,
                           c.x0 ? 1 : 0, c.ws, c.rtol, c.maxit, 0);
    }
    rc = hip_fail(hipGetLastError(), "batched cg start");
    if (rc) return rc;

    // Kernel timing: three events per iteration slot of a check interval
    // (before the batched P, between it and the batched P^T, after it),
    // read after every interval.  In a graph they are event-record nodes,
    // recorded again at every replay.
    bool timed = rep[0].time_kernels != 0;
    EventPool evp;
    std::vector<hipEvent_t> slot_ev;
    if (timed) {
        for (int i = 0; i < 3 * chunk; ++i) {
            hipEvent_t e = evp.get();
            if (!e) return set_error(TOMO_EHIP, "tomo_batch_cg_solve: event creation failed");
            slot_ev.push_back(e);
        }
    }
    double ms_p = 0.0, ms_b = 0.0;
    int slots_used = 0;  // slots recorded since the last read
    auto read_slots = [&]() -> int {  // after a synchronisation
        for (int i = 0; i < slots_used; ++i) {
            float a = 0.f, b2 = 0.f;
            int e = hip_fail(hipEventElapsedTime(&a, slot_ev[(size_t)(3 * i)], slot_ev[(size_t)(3 * i + 1)]),
                             "timing event read");
            if (!e)
                e = hip_fail(hipEventElapsedTime(&b2, slot_ev[(size_t)(3 * i + 1)], slot_ev[(size_t)(3 * i + 2)]),
                             "timing event read");
            if (e) return e;
            ms_p += a;
            ms_b += b2;
        }
        slots_used = 0;
        return TOMO_OK;
    };

    // the three parts of one iteration of every system
    auto part_p = [&](hipStream_t st) -> int { return batch_project_ops(bt, oset[kItP], st); };
    auto part_bp = [&](hipStream_t st) -> int { return batch_backproject_ops(bt, oset[kItPT], st); };
    auto part_vec = [&](hipStream_t st) -> int {
        for (int k = 0; k < ns; ++k) {
            Sys &c = sy[(size_t)k];
            if (c.skip) continue;
            const unsigned eb = (unsigned)c.ws.nq;
            launch_cg_q(c.hw, eb, st, c.p, c.q, c.mm, c.d, c.lr, c.lt, c.ws, c.hd);
            hipLaunchKernelGGL(k_cg_xr, dim3(eb), dim3(kThreads), 0, st, x_d[k], c.r, c.p, c.q, c.n, c.ws, 0);
            hipLaunchKernelGGL(k_cg_p, dim3(eb), dim3(kThreads), 0, st, c.r, c.p, c.n, c.ws);
        }
        return hip_fail(hipGetLastError(), "batched cg iteration launch");
    };
    auto enqueue_iteration = [&](hipStream_t st, int slot) -> int {  // direct launches
        auto mark = [&](int j) {
            return timed ? hip_fail(hipEventRecord(slot_ev[(size_t)(3 * slot + j)], st), "timing event record")
                         : TOMO_OK;
        };
        int e = mark(0);
        if (!e) e = part_p(st);
        if (!e) e = mark(1);
        if (!e) e = part_bp(st);
        if (!e) e = mark(2);
        if (!e) e = part_vec(st);
        return e;
    };

    // The check interval as a graph, built node by node: each part is
    // captured on a private stream (the caller's may be the null stream) as
    // a child graph, chained behind the previous node, with the timing
    // events as event-record nodes between the parts.  Replayed on the
    // caller's stream.
    struct GraphGuard {
        hipStream_t cs = nullptr;
        hipGraph_t graph = nullptr;
        std::vector<hipGraph_t> children;
        hipGraphExec_t exec = nullptr;
        void clear()
        {
            if (exec) (void)hipGraphExecDestroy(exec);
            if (graph) (void)hipGraphDestroy(graph);
            for (hipGraph_t c : children) (void)hipGraphDestroy(c);
            exec = nullptr;
            graph = nullptr;
            children.clear();
        }
        ~GraphGuard()
        {
            clear();
            if (cs) (void)hipStreamDestroy(cs);
        }
    } gg;
    auto build_graph = [&](bool with_events) -> int {
        gg.clear();
        int e = hip_fail(hipGraphCreate(&gg.graph, 0), "graph create");
        hipGraphNode_t prev = nullptr;
        auto add_part = [&](auto &&part) -> int {
            hipGraph_t child = nullptr;
            int r = hip_fail(hipStreamBeginCapture(gg.cs, hipStreamCaptureModeThreadLocal), "begin capture");
            if (r) return r;
            const int cap = part(gg.cs);
            r = hip_fail(hipStreamEndCapture(gg.cs, &child), "end capture");
            if (child) gg.children.push_back(child);
            if (!r && cap) r = cap;
            hipGraphNode_t node = nullptr;
            if (!r)
                r = hip_fail(hipGraphAddChildGraphNode(&node, gg.graph, prev ? &prev : nullptr, prev ? 1 : 0, child),
                             "child graph node");
            if (!r) prev = node;
            return r;
        };
        auto add_event = [&](int slot, int j) -> int {
            if (!with_events) return TOMO_OK;
            hipGraphNode_t node = nullptr;
            const int r = hip_fail(hipGraphAddEventRecordNode(&node, gg.graph, prev ? &prev : nullptr, prev ? 1 : 0,
                                                              slot_ev[(size_t)(3 * slot + j)]),
                                   "event record node");
            if (!r) prev = node;
            return r;
        };
        for (int i = 0; i < chunk && !e; ++i) {
            e = add_event(i, 0);
            if (!e) e = add_part(part_p);
            if (!e) e = add_event(i, 1);
            if (!e) e = add_part(part_bp);
            if (!e) e = add_event(i, 2);
            if (!e) e = add_part(part_vec);
        }
        if (!e) e = hip_fail(hipGraphInstantiate(&gg.exec, gg.graph, nullptr, nullptr, 0), "graph instantiate");
        return e;
    };
    bool timing_lost = false;  // the graph could not hold the timing events
    if (use_graph) {
        rc = hip_fail(hipStreamCreateWithFlags(&gg.cs, hipStreamNonBlocking), "capture stream");
        if (rc) return rc;
        rc = build_graph(timed);
        if (rc && timed) {  // without the events, the iterations are still timed as a whole by the caller
            (void)hipGetLastError();
            timed = false;
            timing_lost = true;
            rc = build_graph(false);
        }
        if (rc) return rc;
    }

    for (;;) {
        for (;;) {
            if (gg.exec) {
                rc = hip_fail(hipGraphLaunch(gg.exec, s), "graph launch");
            } else {
                for (int i = 0; i < chunk && !rc; ++i) rc = enqueue_iteration(s, i);
            }
            if (timed) slots_used = chunk;
            if (!rc) rc = pull_states();
            if (!rc && timed) rc = read_slots();
            if (rc) return rc;
            bool all = true;
            for (int k = 0; k < ns; ++k) all = all && (sy[(size_t)k].skip || hst[k].done);
            if (all) break;
        }
        // true residuals
        rc = apply_A_x();
        if (rc) return rc;
        for (int k = 0; k < ns; ++k) {
            Sys &c = sy[(size_t)k];
            if (c.skip) continue;
            launch_true_res(c.hw, elem_blocks(c.n), s, x_d[k], c.q, c.b, c.mm, c.d, c.lr, c.lt, c.ws, c.hd);
        }
        rc = pull_states();
        if (rc) return rc;
        bool restarted = false;
        for (int k = 0; k < ns; ++k) {
            Sys &c = sy[(size_t)k];
            if (c.skip || hst[k].nonfinite) continue;
            c.true_rel = hst[k].bb > 0 ? sqrt(hst[k].aux / hst[k].bb) : 0.0;
            const bool unconfirmed = c.rtol > 0 && c.true_rel > c.rtol;
            if (unconfirmed && hst[k].iter < c.maxit && c.restarts < 8) {
                ++c.restarts;
                restarted = true;
                hipLaunchKernelGGL(k_cg_start, dim3(elem_blocks(c.n)), dim3(kThreads), 0, s, c.b, c.r, c.p, c.q,
                                   c.n, 1, c.ws, c.rtol, c.maxit, hst[k].iter);
            }
        }
        if (!restarted) break;
        rc = hip_fail(hipGetLastError(), "batched cg restart");
        if (rc) return rc;
    }

    // reports
    for (int k = 0; k < ns; ++k) {
        Sys &c = sy[(size_t)k];
        tomo_cg_report &r = rep[k];
        double *hist_h = r.history;
        const int32_t cap = r.history_cap;
        memset(&r, 0, offsetof(tomo_cg_report, history));
        r.fell_back = -1;
        if (c.skip) {
            r.status = TOMO_ENONFINITE;
            r.rel_res = r.true_rel_res = NAN;
            r.history_len = 0;
            continue;
        }
        const CgState &h = hst[k];
        r.iters = h.iter;
        r.n_project = c.n_proj + h.iter;
        r.n_backproject = c.n_bp + h.iter;
        r.bnorm = sqrt(h.bb);
        r.rel_res = h.bb > 0 ? sqrt(h.res2 / h.bb) : 0.0;
        r.true_rel_res = c.true_rel;
        if (h.nonfinite) r.status = TOMO_ENONFINITE;
        else if (c.rtol > 0 && !(c.true_rel <= c.rtol)) r.status = TOMO_ENOCONV;
        else r.status = TOMO_OK;
        r.history_len = 0;
        if (hist_h && cap > 0) {
            const int nh = h.iter + 1 < cap ? h.iter + 1 : cap;
            rc = hip_fail(hipMemcpy(hist_h, c.ws.hist, sizeof(double) * nh, hipMemcpyDeviceToHost), "history copy");
            if (rc) return rc;
            r.history_len = nh;
        }
        r.ms_project = timing_lost ? NAN : ms_p;
        r.ms_backproject = timing_lost ? NAN : ms_b;
        r.time_kernels = rep[0].time_kernels;
    }
    return TOMO_OK;
}

}  // extern "C"
