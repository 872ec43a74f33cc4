// The learned preconditioner network N for flexible CG: three 3x3x3
// convolutions (1 -> 16 -> 16 -> 1 channels, zero padding 1, ReLU between
// layers), its MSE training gradient, and Adam.  The paper names
// preconditioning as the untried remedy for slow CG convergence (Sec.
// "Smooth Temporal Evolution"); the network approximates the inverse of the
// normal operator on residuals.
//
// gfx950 design:
// * Hidden activations are BF16, channels-last ([voxel][16], 32 B per voxel),
//   so one voxel's 16 channels are one contiguous 32-byte run.
// * The 16 -> 16 layer is a real contraction (6912 MACs per voxel) and runs
//   on MFMA: for each tap, D[cout][voxel] += W_tap[cout][cin] x X_tap[cin][voxel]
//   with v_mfma_f32_16x16x16_bf16 over a row tile of 16 voxels.  Lane l
//   holds A = W_tap[l%16][4(l/16)..+3] (weights, kept in registers for all 27
//   taps), B = X[voxel l%16][4(l/16)..+3] (one 8-byte load, the 64 lanes
//   covering 512 contiguous bytes) and D = out[voxel l%16][4(l/16)..+3]
//   (one 8-byte store).  The same kernel computes the data gradient with
//   flipped, transposed weights.
// * The 1 -> 16 and 16 -> 1 layers (432 MACs per voxel) are bandwidth-bound
//   and run on VALU, weights read as uniform (scalar) loads.
// * Weight gradients are reductions over all voxels: per-block FP64 partial
//   sums, reduced in a fixed order (deterministic).
#include <math.h>

#include "common.h"

namespace tomo {

typedef short bf16x4 __attribute__((ext_vector_type(4)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

constexpr int kC = 16;
constexpr int kTaps = 27;
constexpr int OW1 = 0, OB1 = 432, OW2 = 448, OB2 = 7360, OW3 = 7376, OB3 = 7808;
static_assert(OB3 + 1 == TOMO_CONVNET_NPARAMS, "parameter layout");
constexpr int kWgBlocks = 512;  // blocks of the weight-gradient reductions

__device__ inline uint16_t f2bf(float f)
{
    uint32_t u = __builtin_bit_cast(uint32_t, f);
    u += 0x7fffu + ((u >> 16) & 1u);  // round to nearest even
    return (uint16_t)(u >> 16);
}

__device__ inline float bf2f(uint16_t h) { return __builtin_bit_cast(float, (uint32_t)h << 16); }

struct Vol {
    int32_t nx, ny, nz;
    int64_t n;
};

__device__ inline void vox_ijk(const Vol &d, int64_t v, int &i, int &j, int &k)
{
    i = (int)(v % d.nx);
    const int64_t r = v / d.nx;
    j = (int)(r % d.ny);
    k = (int)(r / d.ny);
}

// optional device scale sqrt(*norm2) (norm2 == nullptr: 1)
__device__ inline float read_scale(const double *norm2)
{
    return norm2 ? (float)sqrt(*norm2) : 1.0f;
}

// ------------------------------------------------------------- forward

// Forward kernels work on output tiles of 16 x 4 x 4 voxels (one per
// workgroup, on a 3-D grid: no index division).  The tile's input region
// with its one-voxel halo (18 x 6 x 6) is staged in LDS once, zero outside
// the volume, and every tap reads LDS instead of re-gathering from L2.
constexpr int kTX = 16, kTY = 4, kTZ = 4;
constexpr int kRX = kTX + 2, kRY = kTY + 2, kRZ = kTZ + 2, kRegion = kRX * kRY * kRZ;

__device__ inline int region_index(int lx, int ly, int lz, int t)
{
    return ((lz + t / 9) * kRY + (ly + (t / 3) % 3)) * kRX + lx + t % 3;
}

// Stages the [voxel][16] BF16 region of the tile at (x0, y0, z0) into
// lds[kRegion * 2] (two 16-byte halves per voxel).
__device__ inline void stage_channels(const uint16_t *__restrict__ src, const Vol &d, int x0, int y0, int z0,
                                      uint4 *lds)
{
    for (int e = threadIdx.x; e < kRegion * 2; e += kThreads) {
        const int rv = e >> 1;
        const int ex = rv % kRX, ey = (rv / kRX) % kRY, ez = rv / (kRX * kRY);
        const int gx = x0 + ex - 1, gy = y0 + ey - 1, gz = z0 + ez - 1;
        uint4 v = make_uint4(0u, 0u, 0u, 0u);
        if (gx >= 0 && gx < d.nx && gy >= 0 && gy < d.ny && gz >= 0 && gz < d.nz)
            v = reinterpret_cast<const uint4 *>(src + (((int64_t)gz * d.ny + gy) * d.nx + gx) * kC)[e & 1];
        lds[e] = v;
    }
}

// layer 1: a1[v][c] = relu(b1[c] + sum_t w1[c][t] x[v + t - 1] / s)
__global__ __launch_bounds__(kThreads) void k_conv1(const float *__restrict__ P,
                                                    const float *__restrict__ x, Vol d,
                                                    const double *__restrict__ norm2,
                                                    uint16_t *__restrict__ a1,
                                                    const int *__restrict__ skip)
{
    __shared__ float xs[kRegion];
    __shared__ float wsh[kC * kTaps + kC];  // w1 then b1 (contiguous in P)
    if (skip && *skip) return;
    const float s = read_scale(norm2);
    const float inv = s > 0.0f ? 1.0f / s : 0.0f;
    const int x0 = blockIdx.x * kTX, y0 = blockIdx.y * kTY, z0 = blockIdx.z * kTZ;
    for (int e = threadIdx.x; e < kRegion; e += kThreads) {
        const int ex = e % kRX, ey = (e / kRX) % kRY, ez = e / (kRX * kRY);
        const int gx = x0 + ex - 1, gy = y0 + ey - 1, gz = z0 + ez - 1;
        float v = 0.0f;
        if (gx >= 0 && gx < d.nx && gy >= 0 && gy < d.ny && gz >= 0 && gz < d.nz)
            v = x[((int64_t)gz * d.ny + gy) * d.nx + gx] * inv;
        xs[e] = v;
    }
    for (int e = threadIdx.x; e < kC * kTaps + kC; e += kThreads) wsh[e] = P[OW1 + e];
    __syncthreads();
    const int lx = threadIdx.x % kTX, ly = (threadIdx.x / kTX) % kTY, lz = threadIdx.x / (kTX * kTY);
    const int gx = x0 + lx, gy = y0 + ly, gz = z0 + lz;
    if (gx >= d.nx || gy >= d.ny || gz >= d.nz) return;
    float in[kTaps];
#pragma unroll
    for (int t = 0; t < kTaps; ++t) in[t] = xs[region_index(lx, ly, lz, t)];
    uint32_t packed[8];
#pragma unroll
    for (int c = 0; c < kC; c += 2) {
        float a0 = wsh[kC * kTaps + c], a1v = wsh[kC * kTaps + c + 1];
#pragma unroll
        for (int t = 0; t < kTaps; ++t) {
            a0 = fmaf(wsh[c * kTaps + t], in[t], a0);
            a1v = fmaf(wsh[(c + 1) * kTaps + t], in[t], a1v);
        }
        packed[c / 2] = (uint32_t)f2bf(fmaxf(a0, 0.0f)) | ((uint32_t)f2bf(fmaxf(a1v, 0.0f)) << 16);
    }
    const int64_t v = ((int64_t)gz * d.ny + gy) * d.nx + gx;
    uint4 *dst = reinterpret_cast<uint4 *>(a1 + v * kC);
    dst[0] = make_uint4(packed[0], packed[1], packed[2], packed[3]);
    dst[1] = make_uint4(packed[4], packed[5], packed[6], packed[7]);
}

// Weight fragments of the 16 -> 16 layer for MFMA: frag[t][lane] holds
// W[cout = lane%16][cin = 4(lane/16)..+3] at tap t.  With transpose = 1 the
// fragments are those of the data-gradient convolution:
// W'[cin][cout][t'] = W[cout][cin][26 - t'] (taps flipped).
__global__ void k_conv16_frags(const float *__restrict__ P, int transpose, bf16x4 *__restrict__ frag)
{
    const int idx = blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= kTaps * 64) return;
    const int t = idx / 64, lane = idx % 64;
    const int row = lane % 16, k0 = 4 * (lane / 16);
    bf16x4 f;
#pragma unroll
    for (int e = 0; e < 4; ++e) {
        const int col = k0 + e;
        const float w = transpose ? P[OW2 + (col * kC + row) * kTaps + (kTaps - 1 - t)]
                                  : P[OW2 + (row * kC + col) * kTaps + t];
        f[e] = (short)f2bf(w);
    }
    frag[idx] = f;
}

// 16 -> 16 convolution on MFMA.  Each wavefront takes four 16-voxel rows of
// the tile; per row and tap one v_mfma_f32_16x16x16_bf16 with the weights
// in registers and the inputs read from the LDS region.  out = act(bias +
// conv) where act is ReLU (relu = 1), or multiplication by [mask > 0] (mask
// != nullptr, the ReLU derivative of the layer below), or nothing.
__global__ __launch_bounds__(kThreads) void k_conv16(const uint16_t *__restrict__ in,
                                                     const bf16x4 *__restrict__ frag,
                                                     const float *__restrict__ bias, Vol d,
                                                     int relu, const uint16_t *__restrict__ mask,
                                                     uint16_t *__restrict__ out,
                                                     const int *__restrict__ skip)
{
    __shared__ uint4 region[kRegion * 2];
    if (skip && *skip) return;
    const int x0 = blockIdx.x * kTX, y0 = blockIdx.y * kTY, z0 = blockIdx.z * kTZ;
    stage_channels(in, d, x0, y0, z0, region);
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    bf16x4 w[kTaps];
#pragma unroll
    for (int t = 0; t < kTaps; ++t) w[t] = frag[t * 64 + lane];
    const int vl = lane % 16, cg = 4 * (lane / 16);
    float b[4] = {0.f, 0.f, 0.f, 0.f};
    if (bias)
#pragma unroll
        for (int r = 0; r < 4; ++r) b[r] = bias[cg + r];
    __syncthreads();
    const char *rbytes = reinterpret_cast<const char *>(region);
    const int xo = x0 + vl;
    for (int rr = 0; rr < 4; ++rr) {
        const int ri = wave * 4 + rr;
        const int ly = ri % kTY, lz = ri / kTY;
        f32x4 acc = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
        for (int t = 0; t < kTaps; ++t) {
            const bf16x4 bv =
                *reinterpret_cast<const bf16x4 *>(rbytes + region_index(vl, ly, lz, t) * 32 + cg * 2);
            acc = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(w[t], bv, acc, 0, 0, 0);
        }
        const int yo = y0 + ly, zo = z0 + lz;
        if (xo < d.nx && yo < d.ny && zo < d.nz) {
            const int64_t vo = ((int64_t)zo * d.ny + yo) * d.nx + xo;
            bf16x4 m = {1, 1, 1, 1};
            if (mask) m = *reinterpret_cast<const bf16x4 *>(mask + vo * kC + cg);
            bf16x4 o;
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                float val = acc[r] + b[r];
                if (relu) val = fmaxf(val, 0.0f);
                if (mask && !(bf2f((uint16_t)m[r]) > 0.0f)) val = 0.0f;
                o[r] = (short)f2bf(val);
            }
            *reinterpret_cast<bf16x4 *>(out + vo * kC + cg) = o;
        }
    }
}

// layer 3: out[v] = s * (b3 + sum_{c,t} w3[c][t] a2[v + t - 1][c]), zero
// where the map mask is 0.
__global__ __launch_bounds__(kThreads) void k_conv3(const float *__restrict__ P,
                                                    const uint16_t *__restrict__ a2, Vol d,
                                                    const double *__restrict__ norm2,
                                                    const uint8_t *__restrict__ map_mask,
                                                    float *__restrict__ out,
                                                    const int *__restrict__ skip)
{
    __shared__ uint4 region[kRegion * 2];
    __shared__ float wsh[kC * kTaps + 1];  // w3 then b3 (contiguous in P)
    if (skip && *skip) return;
    const float s = read_scale(norm2);
    const int x0 = blockIdx.x * kTX, y0 = blockIdx.y * kTY, z0 = blockIdx.z * kTZ;
    stage_channels(a2, d, x0, y0, z0, region);
    for (int e = threadIdx.x; e < kC * kTaps + 1; e += kThreads) wsh[e] = P[OW3 + e];
    __syncthreads();
    const int lx = threadIdx.x % kTX, ly = (threadIdx.x / kTX) % kTY, lz = threadIdx.x / (kTX * kTY);
    const int gx = x0 + lx, gy = y0 + ly, gz = z0 + lz;
    if (gx >= d.nx || gy >= d.ny || gz >= d.nz) return;
    float acc = wsh[kC * kTaps];
#pragma unroll 3
    for (int t = 0; t < kTaps; ++t) {
        const int rv = region_index(lx, ly, lz, t);
        const uint4 lo = region[2 * rv], hi = region[2 * rv + 1];
        const uint32_t wds[8] = {lo.x, lo.y, lo.z, lo.w, hi.x, hi.y, hi.z, hi.w};
#pragma unroll
        for (int c = 0; c < kC; c += 2) {
            acc = fmaf(wsh[c * kTaps + t], bf2f((uint16_t)(wds[c / 2] & 0xffffu)), acc);
            acc = fmaf(wsh[(c + 1) * kTaps + t], bf2f((uint16_t)(wds[c / 2] >> 16)), acc);
        }
    }
    const int64_t v = ((int64_t)gz * d.ny + gy) * d.nx + gx;
    float o = s * acc;
    if (map_mask && !map_mask[v]) o = 0.0f;
    out[v] = o;
}

// ------------------------------------------------------------ training

// g[v] = 2 (out[v] - target[v]) / n; loss = mean((out - target)^2) (FP64).
__global__ __launch_bounds__(kThreads) void k_mse(const float *__restrict__ out,
                                                  const float *__restrict__ target, int64_t n,
                                                  float *__restrict__ g, double *__restrict__ partial)
{
    __shared__ double lds[4];
    double acc = 0.0;
    const float sc = 2.0f / (float)n;
    for (int64_t v = (int64_t)blockIdx.x * kThreads + threadIdx.x; v < n;
         v += (int64_t)gridDim.x * kThreads) {
        const float e = out[v] - target[v];
        g[v] = sc * e;
        acc += (double)e * e;
    }
    const double s = block_sum(acc, lds);
    if (threadIdx.x == 0) partial[blockIdx.x] = s;
}

// g_h2[v][c] = [a2[v][c] > 0] * sum_t w3[c][t] g[v - t + 1]  (data gradient of layer 3)
__global__ __launch_bounds__(kThreads) void k_conv3_bwd(const float *__restrict__ P,
                                                        const float *__restrict__ g,
                                                        const uint16_t *__restrict__ a2, Vol d,
                                                        uint16_t *__restrict__ gh2)
{
    for (int64_t v = (int64_t)blockIdx.x * kThreads + threadIdx.x; v < d.n;
         v += (int64_t)gridDim.x * kThreads) {
        int i, j, k;
        vox_ijk(d, v, i, j, k);
        float gin[kTaps];
#pragma unroll
        for (int t = 0; t < kTaps; ++t) {  // output voxel v - (t - 1) used input v at tap t
            const int ii = i - (t % 3 - 1), jj = j - ((t / 3) % 3 - 1), kk = k - (t / 9 - 1);
            const bool ok = ii >= 0 && ii < d.nx && jj >= 0 && jj < d.ny && kk >= 0 && kk < d.nz;
            gin[t] = ok ? g[((int64_t)kk * d.ny + jj) * d.nx + ii] : 0.0f;
        }
        const uint4 *ms = reinterpret_cast<const uint4 *>(a2 + v * kC);
        const uint4 lo = ms[0], hi = ms[1];
        const uint32_t mw[8] = {lo.x, lo.y, lo.z, lo.w, hi.x, hi.y, hi.z, hi.w};
        uint32_t packed[8];
#pragma unroll
        for (int c = 0; c < kC; c += 2) {
            float s0 = 0.f, s1 = 0.f;
#pragma unroll
            for (int t = 0; t < kTaps; ++t) {
                s0 = fmaf(P[OW3 + c * kTaps + t], gin[t], s0);
                s1 = fmaf(P[OW3 + (c + 1) * kTaps + t], gin[t], s1);
            }
            if (!(bf2f((uint16_t)(mw[c / 2] & 0xffffu)) > 0.f)) s0 = 0.f;
            if (!(bf2f((uint16_t)(mw[c / 2] >> 16)) > 0.f)) s1 = 0.f;
            packed[c / 2] = (uint32_t)f2bf(s0) | ((uint32_t)f2bf(s1) << 16);
        }
        uint4 *dst = reinterpret_cast<uint4 *>(gh2 + v * kC);
        dst[0] = make_uint4(packed[0], packed[1], packed[2], packed[3]);
        dst[1] = make_uint4(packed[4], packed[5], packed[6], packed[7]);
    }
}

// Per-block partial sums of the 16 -> 1 weight gradient and bias gradient:
// gw3[c][t] = sum_v g[v] a2[v + t - 1][c]; gb3 = sum_v g[v].
// Thread c*27 + t (of the first 432) owns one weight; thread 432 the bias.
__global__ __launch_bounds__(448) void k_wgrad3(const float *__restrict__ g,
                                                const uint16_t *__restrict__ a2, Vol d,
                                                double *__restrict__ part /* [blocks][433] */)
{
    const int o = threadIdx.x;
    const int c = o / kTaps, t = o % kTaps;
    const int ox = t % 3 - 1, oy = (t / 3) % 3 - 1, oz = t / 9 - 1;
    double acc = 0.0;
    for (int64_t v = blockIdx.x; v < d.n; v += gridDim.x) {
        const float gv = g[v];
        if (o == 432) {
            acc += gv;
        } else if (o < 432) {
            int i, j, k;
            vox_ijk(d, v, i, j, k);
            const int ii = i + ox, jj = j + oy, kk = k + oz;
            if (ii >= 0 && ii < d.nx && jj >= 0 && jj < d.ny && kk >= 0 && kk < d.nz)
                acc += (double)gv * bf2f(a2[(((int64_t)kk * d.ny + jj) * d.nx + ii) * kC + c]);
        }
    }
    if (o < 433) part[(int64_t)blockIdx.x * 433 + o] = acc;
}

// Per-block partial sums of the 1 -> 16 weight gradient:
// gw1[c][t] = sum_v gh1[v][c] x[v + t - 1] / s; gb1[c] = sum_v gh1[v][c].
__global__ __launch_bounds__(448) void k_wgrad1(const uint16_t *__restrict__ gh1,
                                                const float *__restrict__ x, Vol d,
                                                double *__restrict__ part /* [blocks][448] */)
{
    const int o = threadIdx.x;
    double acc = 0.0;
    if (o < 432) {
        const int c = o / kTaps, t = o % kTaps;
        const int ox = t % 3 - 1, oy = (t / 3) % 3 - 1, oz = t / 9 - 1;
        for (int64_t v = blockIdx.x; v < d.n; v += gridDim.x) {
            int i, j, k;
            vox_ijk(d, v, i, j, k);
            const int ii = i + ox, jj = j + oy, kk = k + oz;
            if (ii >= 0 && ii < d.nx && jj >= 0 && jj < d.ny && kk >= 0 && kk < d.nz)
                acc += (double)bf2f(gh1[v * kC + c]) * x[((int64_t)kk * d.ny + jj) * d.nx + ii];
        }
    } else {
        const int c = o - 432;
        for (int64_t v = blockIdx.x; v < d.n; v += gridDim.x) acc += bf2f(gh1[v * kC + c]);
    }
    part[(int64_t)blockIdx.x * 448 + o] = acc;
}

// Per-block partial sums of the 16 -> 16 weight gradient:
// gw2[co][ci][t] = sum_v gh2[v][co] a1[v + t - 1][ci]; gb2[co] = sum_v gh2[v][co].
// Thread (co, ci) = (tid / 16, tid % 16) owns the 27 taps of one pair.
__global__ __launch_bounds__(kThreads) void k_wgrad2(const uint16_t *__restrict__ gh2,
                                                     const uint16_t *__restrict__ a1, Vol d,
                                                     double *__restrict__ part /* [blocks][6928] */)
{
    const int co = threadIdx.x / 16, ci = threadIdx.x % 16;
    float acc[kTaps];
#pragma unroll
    for (int t = 0; t < kTaps; ++t) acc[t] = 0.f;
    double bacc = 0.0;
    double dacc[kTaps];
#pragma unroll
    for (int t = 0; t < kTaps; ++t) dacc[t] = 0.0;
    int cnt = 0;
    const int64_t nrows = (int64_t)d.ny * d.nz;
    for (int64_t row = blockIdx.x; row < nrows; row += gridDim.x) {
        const int j = (int)(row % d.ny), k = (int)(row / d.ny);
        for (int i = 0; i < d.nx; ++i) {
            const int64_t v = (row * d.nx) + i;
            const float gv = bf2f(gh2[v * kC + co]);
            if (ci == 0) bacc += gv;
            if (gv == 0.0f) continue;  // ReLU zeros: common, and they add nothing
#pragma unroll
            for (int t = 0; t < kTaps; ++t) {
                const int ii = i + t % 3 - 1, jj = j + (t / 3) % 3 - 1, kk = k + t / 9 - 1;
                if (ii >= 0 && ii < d.nx && jj >= 0 && jj < d.ny && kk >= 0 && kk < d.nz)
                    acc[t] = fmaf(gv, bf2f(a1[(((int64_t)kk * d.ny + jj) * d.nx + ii) * kC + ci]), acc[t]);
            }
            if (++cnt == 64) {  // fold the FP32 partials into FP64 regularly
#pragma unroll
                for (int t = 0; t < kTaps; ++t) {
                    dacc[t] += acc[t];
                    acc[t] = 0.f;
                }
                cnt = 0;
            }
        }
    }
    double *dst = part + (int64_t)blockIdx.x * 6928;
#pragma unroll
    for (int t = 0; t < kTaps; ++t) dst[(co * kC + ci) * kTaps + t] = dacc[t] + acc[t];
    if (ci == 0) dst[6912 + co] = bacc;
}

// grad[off + o] = sum over blocks of part[b][o] (fixed order).
__global__ void k_reduce_parts(const double *__restrict__ part, int nblocks, int width,
                               float *__restrict__ grad, int off)
{
    const int o = blockIdx.x * blockDim.x + threadIdx.x;
    if (o >= width) return;
    double s = 0.0;
    for (int b = 0; b < nblocks; ++b) s += part[(int64_t)b * width + o];
    grad[off + o] = (float)s;
}

__global__ void k_adam(float *__restrict__ p, const float *__restrict__ g, float *__restrict__ m,
                       float *__restrict__ v, int n, double lr, double b1, double b2, double eps,
                       double c1, double c2)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const double gi = g[i];
    const double mi = b1 * m[i] + (1.0 - b1) * gi;
    const double vi = b2 * v[i] + (1.0 - b2) * gi * gi;
    m[i] = (float)mi;
    v[i] = (float)vi;
    p[i] = (float)((double)p[i] - lr * (mi / c1) / (sqrt(vi / c2) + eps));
}

// ------------------------------------------------------------ host side

struct NetWs {
    uint16_t *a1, *a2, *gh;  // [n][16] each
    float *out, *g;          // [n]
    bf16x4 *frag, *fragT;    // [27][64]
    double *part;            // weight-gradient partials
    double *loss_part;       // [kRedLossBlocks]
};
constexpr int kLossBlocks = 1024;

static size_t align256(size_t b) { return (b + 255) & ~(size_t)255; }

static size_t ws_layout(int64_t n, NetWs *w, char *base)
{
    size_t off = 0;
    auto take = [&](size_t bytes) {
        char *p = base ? base + off : nullptr;
        off += align256(bytes);
        return p;
    };
    NetWs t;
    t.a1 = (uint16_t *)take(sizeof(uint16_t) * kC * n);
    t.a2 = (uint16_t *)take(sizeof(uint16_t) * kC * n);
    t.gh = (uint16_t *)take(sizeof(uint16_t) * kC * n);
    t.out = (float *)take(sizeof(float) * n);
    t.g = (float *)take(sizeof(float) * n);
    t.frag = (bf16x4 *)take(sizeof(bf16x4) * kTaps * 64);
    t.fragT = (bf16x4 *)take(sizeof(bf16x4) * kTaps * 64);
    t.part = (double *)take(sizeof(double) * kWgBlocks * 6928);
    t.loss_part = (double *)take(sizeof(double) * kLossBlocks);
    if (w) *w = t;
    return off;
}

// Forward-only workspace (activations and fragments) for flexible CG.
size_t convnet_forward_ws_bytes(int64_t n)
{
    return align256(sizeof(uint16_t) * kC * n) * 2 + align256(sizeof(bf16x4) * kTaps * 64);
}

static dim3 tile_grid(const Vol &d)
{
    return dim3((unsigned)((d.nx + kTX - 1) / kTX), (unsigned)((d.ny + kTY - 1) / kTY),
                (unsigned)((d.nz + kTZ - 1) / kTZ));
}

static unsigned vox_blocks(int64_t n)
{
    int64_t b = (n + kThreads - 1) / kThreads;
    return (unsigned)(b > 8192 ? 8192 : (b < 1 ? 1 : b));
}

// z = s N(x / s) on the device (s = sqrt(*norm2), or 1), zero where the map
// mask is 0; nothing happens while *skip != 0.  ws: convnet_forward_ws_bytes(n)
// bytes; prep_frags = false reuses the weight fragments of an earlier call.
int convnet_forward_dev(const tomo_cube &c, const float *P, const float *x, float *out,
                        const double *norm2, const uint8_t *map_mask, void *ws, hipStream_t s,
                        bool prep_frags, const int *skip)
{
    const Vol d{c.nx, c.ny, c.nz, (int64_t)c.nx * c.ny * c.nz};
    char *base = (char *)ws;
    uint16_t *a1 = (uint16_t *)base;
    uint16_t *a2 = (uint16_t *)(base + align256(sizeof(uint16_t) * kC * d.n));
    bf16x4 *frag = (bf16x4 *)(base + 2 * align256(sizeof(uint16_t) * kC * d.n));
    if (prep_frags)
        hipLaunchKernelGGL(k_conv16_frags, dim3((kTaps * 64 + 255) / 256), dim3(256), 0, s, P, 0, frag);
    hipLaunchKernelGGL(k_conv1, tile_grid(d), dim3(kThreads), 0, s, P, x, d, norm2, a1, skip);
    hipLaunchKernelGGL(k_conv16, tile_grid(d), dim3(kThreads), 0, s, a1, frag, P + OB2, d, 1,
                       (const uint16_t *)nullptr, a2, skip);
    hipLaunchKernelGGL(k_conv3, tile_grid(d), dim3(kThreads), 0, s, P, a2, d, norm2, map_mask, out, skip);
    return hip_fail(hipGetLastError(), "convnet forward launch");
}

}  // namespace tomo

using namespace tomo;

static int check_net_cube(const tomo_cube *c)
{
    int rc = validate_cube(c);
    if (rc) return rc;
    if (c->nframes != 1) return set_error(TOMO_EINVAL, "convnet: the cube must hold one frame");
    return TOMO_OK;
}

extern "C" {

size_t tomo_convnet_workspace_bytes(const tomo_cube *cube)
{
    if (!cube || validate_cube(cube)) return 0;
    return ws_layout((int64_t)cube->nx * cube->ny * cube->nz, nullptr, nullptr);
}

int tomo_convnet_forward(const tomo_cube *cube, const float *params_d, const float *x_d,
                         float *out_d, void *ws_d, size_t ws_bytes, tomo_stream stream)
{
    int rc = check_net_cube(cube);
    if (rc) return rc;
    if (!params_d || !x_d || !out_d || !ws_d)
        return set_error(TOMO_EINVAL, "tomo_convnet_forward: NULL argument");
    const int64_t n = (int64_t)cube->nx * cube->ny * cube->nz;
    if (ws_bytes < ws_layout(n, nullptr, nullptr))
        return set_error(TOMO_EINVAL, "tomo_convnet_forward: workspace too small");
    return convnet_forward_dev(*cube, params_d, x_d, out_d, nullptr, nullptr, ws_d,
                               (hipStream_t)stream, true, nullptr);
}

// Forward pass that keeps the activations, then back-propagation of the
// output gradient g_d (d loss / d out, one value per voxel) into grad_d.  With
// target_d set, g_d is ignored and replaced by the MSE gradient
// 2 (out - target) / n, whose per-block loss partials land in w.loss_part.
static int convnet_train_pass(const tomo_cube *cube, const float *params_d, const float *x_d,
                              const float *target_d, const float *g_d, float *grad_d, void *ws_d,
                              hipStream_t s)
{
    const int64_t n = (int64_t)cube->nx * cube->ny * cube->nz;
    NetWs w;
    ws_layout(n, &w, (char *)ws_d);
    const Vol d{cube->nx, cube->ny, cube->nz, n};
    const dim3 rowgrid = tile_grid(d);
    // forward, keeping activations
    hipLaunchKernelGGL(k_conv16_frags, dim3((kTaps * 64 + 255) / 256), dim3(256), 0, s, params_d, 0, w.frag);
    hipLaunchKernelGGL(k_conv16_frags, dim3((kTaps * 64 + 255) / 256), dim3(256), 0, s, params_d, 1, w.fragT);
    const int *noskip = nullptr;
    hipLaunchKernelGGL(k_conv1, rowgrid, dim3(kThreads), 0, s, params_d, x_d, d,
                       (const double *)nullptr, w.a1, noskip);
    hipLaunchKernelGGL(k_conv16, rowgrid, dim3(kThreads), 0, s, w.a1, w.frag, params_d + OB2, d, 1,
                       (const uint16_t *)nullptr, w.a2, noskip);
    if (target_d) {
        hipLaunchKernelGGL(k_conv3, rowgrid, dim3(kThreads), 0, s, params_d, w.a2, d,
                           (const double *)nullptr, (const uint8_t *)nullptr, w.out, noskip);
        // loss and d loss / d out
        hipLaunchKernelGGL(k_mse, dim3(kLossBlocks), dim3(kThreads), 0, s, w.out, target_d, n, w.g,
                           w.loss_part);
        g_d = w.g;
    }
    // layer 3
    hipLaunchKernelGGL(k_wgrad3, dim3(kWgBlocks), dim3(448), 0, s, g_d, w.a2, d, w.part);
    hipLaunchKernelGGL(k_reduce_parts, dim3(2), dim3(256), 0, s, w.part, kWgBlocks, 433, grad_d, OW3);
    hipLaunchKernelGGL(k_conv3_bwd, dim3(vox_blocks(n)), dim3(kThreads), 0, s, params_d, g_d, w.a2, d, w.gh);
    // layer 2 (gh = d loss / d h2)
    hipLaunchKernelGGL(k_wgrad2, dim3(kWgBlocks), dim3(kThreads), 0, s, w.gh, w.a1, d, w.part);
    hipLaunchKernelGGL(k_reduce_parts, dim3((6928 + 255) / 256), dim3(256), 0, s, w.part, kWgBlocks, 6928,
                       grad_d, OW2);
    // d loss / d h1 = [a1 > 0] conv^T(gh); written over a2 (no longer needed)
    hipLaunchKernelGGL(k_conv16, rowgrid, dim3(kThreads), 0, s, w.gh, w.fragT, (const float *)nullptr, d,
                       0, w.a1, w.a2, noskip);
    // layer 1
    hipLaunchKernelGGL(k_wgrad1, dim3(kWgBlocks), dim3(448), 0, s, w.a2, x_d, d, w.part);
    hipLaunchKernelGGL(k_reduce_parts, dim3(2), dim3(256), 0, s, w.part, kWgBlocks, 448, grad_d, OW1);
    return hip_fail(hipGetLastError(), "convnet backward launch");
}

int tomo_convnet_loss_grad(const tomo_cube *cube, const float *params_d, const float *x_d,
                           const float *target_d, float *grad_d, double *loss_h, void *ws_d,
                           size_t ws_bytes, tomo_stream stream)
{
    int rc = check_net_cube(cube);
    if (rc) return rc;
    if (!params_d || !x_d || !target_d || !grad_d || !ws_d)
        return set_error(TOMO_EINVAL, "tomo_convnet_loss_grad: NULL argument");
    const int64_t n = (int64_t)cube->nx * cube->ny * cube->nz;
    if (ws_bytes < ws_layout(n, nullptr, nullptr))
        return set_error(TOMO_EINVAL, "tomo_convnet_loss_grad: workspace too small");
    hipStream_t s = (hipStream_t)stream;
    rc = convnet_train_pass(cube, params_d, x_d, target_d, nullptr, grad_d, ws_d, s);
    if (rc) return rc;
    if (loss_h) {
        NetWs w;
        ws_layout(n, &w, (char *)ws_d);
        double parts[kLossBlocks];
        rc = hip_fail(hipMemcpyAsync(parts, w.loss_part, sizeof(parts), hipMemcpyDeviceToHost, s), "loss copy");
        if (!rc) rc = hip_fail(hipStreamSynchronize(s), "loss synchronise");
        if (rc) return rc;
        double acc = 0.0;
        for (int b = 0; b < kLossBlocks; ++b) acc += parts[b];
        *loss_h = acc / (double)n;
    }
    return TOMO_OK;
}

int tomo_convnet_backward(const tomo_cube *cube, const float *params_d, const float *x_d,
                          const float *dout_d, float *grad_d, void *ws_d, size_t ws_bytes,
                          tomo_stream stream)
{
    int rc = check_net_cube(cube);
    if (rc) return rc;
    if (!params_d || !x_d || !dout_d || !grad_d || !ws_d)
        return set_error(TOMO_EINVAL, "tomo_convnet_backward: NULL argument");
    const int64_t n = (int64_t)cube->nx * cube->ny * cube->nz;
    if (ws_bytes < ws_layout(n, nullptr, nullptr))
        return set_error(TOMO_EINVAL, "tomo_convnet_backward: workspace too small");
    return convnet_train_pass(cube, params_d, x_d, nullptr, dout_d, grad_d, ws_d, (hipStream_t)stream);
}

int tomo_adam_step(float *params_d, const float *grad_d, float *m_d, float *v_d, int32_t n,
                   int32_t step, double lr, double beta1, double beta2, double eps,
                   tomo_stream stream)
{
    if (!params_d || !grad_d || !m_d || !v_d || n < 1 || step < 1 || !(lr > 0) || !(beta1 >= 0) ||
        !(beta1 < 1) || !(beta2 >= 0) || !(beta2 < 1) || !(eps > 0))
        return set_error(TOMO_EINVAL, "tomo_adam_step: invalid argument");
    const double c1 = 1.0 - pow(beta1, step), c2 = 1.0 - pow(beta2, step);
    hipLaunchKernelGGL(k_adam, dim3((n + 255) / 256), dim3(256), 0, (hipStream_t)stream, params_d, grad_d,
                       m_d, v_d, n, lr, beta1, beta2, eps, c1, c2);
    return hip_fail(hipGetLastError(), "adam launch");
}

}  // extern "C"
