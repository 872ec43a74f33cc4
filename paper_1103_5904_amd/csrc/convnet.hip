// The learned preconditioner network N for flexible CG: three 3x3x3
// convolutions (1 -> 16 -> 16 -> 1 channels, zero padding 1, ReLU between
// layers), its parameter gradients (for an MSE loss, or for any loss given
// its output gradient: the energy-norm error the preconditioner is trained
// on), and Adam.  The paper names
// preconditioning as the untried remedy for slow CG convergence (Sec.
// "Smooth Temporal Evolution"); the network approximates the inverse of the
// normal operator on residuals.
//
// gfx950 design:
// * Hidden activations are BF16, channels-last ([voxel][16], 32 B per voxel),
//   so one voxel's 16 channels are one contiguous 32-byte run.
// * Every layer is a contraction over (tap, input channel) and runs on MFMA
//   over row tiles of 16 voxels: D[cout][voxel] += A[cout][k] B[k][voxel],
//   with the weights held in registers and the inputs read from an LDS copy
//   of the tile's region.  For a 16-channel input the taps (dz, dy, dx) go
//   in nine x-triples: v_mfma_f32_16x16x32_bf16 takes dx = 0 and 1 (two
//   taps of 16 channels), v_mfma_f32_16x16x16_bf16 takes dx = 2.  The B
//   operand of an x-triple depends only on the input row (y + dy, z + dz),
//   so each input row read from LDS feeds the up to three output rows that
//   use it (dy = 0, 1, 2): half the LDS reads of pairing the taps in order.
//   D lands as out[voxel l % 16][4 (l / 16) .. +3]: one 8-byte store.  The
//   same kernel computes the 16 -> 16 data gradient with flipped, transposed
//   weights.
// * The 1 -> 16 layer takes its 27 taps as the contraction index; it and the
//   16 -> 1 layer keep ~16 significant bits of their weights by splitting
//   them into a BF16 value and a BF16 remainder (for the last layer the two
//   are rows 0 and 1 of one weight matrix, so the split costs nothing).
// * Weight gradients are reductions over all voxels: per-block FP64 partial
//   sums, reduced in a fixed order (deterministic).
#include <math.h>

#include <map>
#include <mutex>

#include "common.h"

namespace tomo {

typedef short bf16x4 __attribute__((ext_vector_type(4)));
typedef short bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

constexpr int kC = 16;
constexpr int kTaps = 27;
constexpr int OW1 = 0, OB1 = 432, OW2 = 448, OB2 = 7360, OW3 = 7376, OB3 = 7808;
static_assert(OB3 + 1 == TOMO_CONVNET_NPARAMS, "parameter layout");
constexpr int kWgBlocks = 512;  // blocks of the weight-gradient reductions

// round to nearest even (gfx950 converts in one instruction)
__device__ inline uint16_t f2bf(float f) { return __builtin_bit_cast(uint16_t, (__bf16)f); }

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
// Wavefront w takes the four 16-voxel rows (y = 0..3, z = w) of the tile,
// interleaved so that four independent MFMA accumulations are in flight.
constexpr int kTX = 16, kTY = 4, kTZ = 4;
constexpr int kRX = kTX + 2, kRY = kTY + 2, kRZ = kTZ + 2, kRegion = kRX * kRY * kRZ;
static_assert(kTY == 4 && kTZ * 64 == kThreads, "one wavefront per tile z, four rows each");

// region entry of output voxel (lx, ly, lz) of the tile at tap t
__device__ inline int region_index(int lx, int ly, int lz, int t)
{
    return ((lz + t / 9) * kRY + (ly + (t / 3) % 3)) * kRX + lx + t % 3;
}

// Stages the [voxel][16] BF16 region of the tile at (x0, y0, z0) into LDS as
// two planes of kRegion 16-byte entries: plane h holds channels 8h..8h+7.
// Sixteen lanes reading one plane at sixteen consecutive voxels then cover
// 256 contiguous bytes (no bank conflicts).
__device__ inline void stage_channels(const uint16_t *__restrict__ src, const Vol &d, int x0, int y0, int z0,
                                      uint4 *lds)
{
    for (int e = threadIdx.x; e < kRegion * 2; e += kThreads) {
        const int rv = e >> 1, h = e & 1;
        const int ex = rv % kRX, ey = (rv / kRX) % kRY, ez = rv / (kRX * kRY);
        const int gx = x0 + ex - 1, gy = y0 + ey - 1, gz = z0 + ez - 1;
        uint4 v = make_uint4(0u, 0u, 0u, 0u);
        if (gx >= 0 && gx < d.nx && gy >= 0 && gy < d.ny && gz >= 0 && gz < d.nz)
            v = reinterpret_cast<const uint4 *>(src + (((int64_t)gz * d.ny + gy) * d.nx + gx) * kC)[h];
        lds[h * kRegion + rv] = v;
    }
}

// MFMA weight fragments.  v_mfma_f32_16x16x32_bf16 computes D(16x16) +=
// A(16x32) B(32x16) with lane l holding A[l % 16][8 (l / 16) + e] and
// B[8 (l / 16) + e][l % 16] (e = 0..7) and D[4 (l / 16) + r][l % 16] (r =
// 0..3); v_mfma_f32_16x16x16_bf16 has the same D with A[l % 16][4 (l / 16) +
// e], e = 0..3.  A 16 -> C layer contracts over (tap, input channel), the
// taps t = 9 dz + 3 dy + dx taken in x-triples q = 3 dz + dy (t = 3 q + dx):
// the K = 32 instruction of triple q has k = 16 dx + c for dx = 0, 1 (lane
// group g = l / 16 reads dx = g / 2 from LDS plane g % 2), the K = 16
// instruction has k = c for dx = 2 (lane group g reads channels 4g..4g+3).
// Fragment f of a set is the 64 bf16x8 entries [64 f, 64 f + 64): f = q
// for the K = 32 fragment of triple q, f = 9 + q for its K = 16 fragment
// (elements 0..3).
//   forward set, kFragFwd entries:
//   * fragments 0-17: the 16 -> 16 layer, A[cout][k] = W2[cout][c][tap];
//   * fragments 18-35: the 16 -> 1 layer, row 0 = bf16(W3[0][c][tap]), row 1 =
//     its remainder W3 - bf16(W3), rows 2-15 zero: output row 0 + row 1 is
//     the layer with ~16 significant bits of weight at no extra instruction;
//   * fragments 36-37: the 1 -> 16 layer with the 27 taps as k (27-31 zero),
//     A[cout][k] = bf16(W1[cout][k]) and its remainder.
//   transposed set (transpose = 1), kFragConv entries: the 16 -> 16 data
//   gradient, A[cin][k] = W2[c][cin][26 - tap] (taps flipped).
constexpr int kTriples = 9;
constexpr int kConvFrags = 2 * kTriples;
constexpr int kFragConv = kConvFrags * 64;
constexpr int kFrag3 = kFragConv, kFrag1 = 2 * kFragConv;
constexpr int kFragFwd = 2 * kFragConv + 2 * 64;

__global__ void k_conv_frags(const float *__restrict__ P, int transpose, bf16x8 *__restrict__ frag)
{
    const int idx = blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= (transpose ? kFragConv : kFragFwd)) return;
    const int f = idx / 64, lane = idx % 64;
    const int row = lane % 16, g = lane / 16;
    bf16x8 out;
#pragma unroll
    for (int e = 0; e < 8; ++e) {
        float w = 0.0f;
        if (transpose || f < 2 * kConvFrags) {
            const int ff = f % kConvFrags;
            const bool k16 = ff >= kTriples;
            const int q = k16 ? ff - kTriples : ff;
            const int tap = 3 * q + (k16 ? 2 : (g >> 1));
            const int c = k16 ? 4 * g + e : 8 * (g & 1) + e;
            if (k16 && e >= 4) {
                w = 0.0f;
            } else if (transpose) {
                w = P[OW2 + (c * kC + row) * kTaps + (kTaps - 1 - tap)];
            } else if (f < kConvFrags) {
                w = P[OW2 + (row * kC + c) * kTaps + tap];
            } else if (row < 2) {
                w = P[OW3 + c * kTaps + tap];
                if (row == 1) w -= bf2f(f2bf(w));
            }
        } else {
            const int tap = 8 * g + e;
            if (tap < kTaps) {
                w = P[OW1 + row * kTaps + tap];
                if (f == 2 * kConvFrags + 1) w -= bf2f(f2bf(w));
            }
        }
        out[e] = (short)f2bf(w);
    }
    frag[idx] = out;
}

// Per-lane LDS byte offsets of the B operands for output voxel (vl, 0, lz)
// of the tile and input row (y, z) = (0, lz) of the region: k32 for the
// dx = 0, 1 pair, k16 for dx = 2.  Input row (dy', dz') further adds
// (dz' kRY + dy') kRX entries (a compile-time immediate).
struct ConvOffsets {
    uint32_t k32;
    uint32_t k16;
};

__device__ inline ConvOffsets conv_offsets(int vl, int lz, int g)
{
    ConvOffsets o;
    o.k32 = (uint32_t)(((g & 1) * kRegion + region_index(vl, 0, lz, g >> 1)) * 16);
    o.k16 = (uint32_t)(((g >> 1) * kRegion + region_index(vl, 0, lz, 2)) * 16 + (g & 1) * 8);
    return o;
}

// acc[y] += sum over taps and channels of A x region, for the four output
// rows y of the wavefront; w, wt: the K = 32 and K = 16 fragments of the
// nine x-triples of a 16 -> C layer, in registers.  Per input plane dz the
// six input rows (region rows lz + dz, yi) are read once; output row y takes
// row y + dy through triple 3 dz + dy.  The four rows are interleaved, so
// three independent MFMA instructions separate two that update the same
// accumulator: an instruction then never reads as its accumulator input the
// result of one still in flight.
__device__ inline void conv_rows(const char *rbytes, const ConvOffsets &o, const bf16x8 (&w)[kTriples],
                                 const bf16x4 (&wt)[kTriples], f32x4 (&acc)[kTY])
{
#pragma unroll
    for (int dz = 0; dz < 3; ++dz) {
        bf16x8 b32[kRY];
        bf16x4 b16[kRY];
#pragma unroll
        for (int yi = 0; yi < kRY; ++yi) {
            const uint32_t row = (uint32_t)((dz * kRY + yi) * kRX * 16);
            b32[yi] = *reinterpret_cast<const bf16x8 *>(rbytes + o.k32 + row);
            b16[yi] = *reinterpret_cast<const bf16x4 *>(rbytes + o.k16 + row);
        }
#pragma unroll
        for (int dy = 0; dy < 3; ++dy) {
#pragma unroll
            for (int y = 0; y < kTY; ++y)
                acc[y] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(w[3 * dz + dy], b32[y + dy], acc[y], 0, 0, 0);
            __builtin_amdgcn_sched_barrier(0);  // keep the four-row interleave as written
        }
#pragma unroll
        for (int dy = 0; dy < 3; ++dy) {
#pragma unroll
            for (int y = 0; y < kTY; ++y)
                acc[y] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(wt[3 * dz + dy], b16[y + dy], acc[y], 0, 0, 0);
            __builtin_amdgcn_sched_barrier(0);
        }
    }
}

__device__ inline void load_conv_frags(const bf16x8 *__restrict__ frag, int lane, bf16x8 (&w)[kTriples],
                                       bf16x4 (&wt)[kTriples])
{
#pragma unroll
    for (int q = 0; q < kTriples; ++q) {
        w[q] = frag[q * 64 + lane];
        const bf16x8 t = frag[(kTriples + q) * 64 + lane];
        wt[q] = __builtin_shufflevector(t, t, 0, 1, 2, 3);
    }
}

// layer 1: a1[v][c] = relu(b1[c] + sum_t w1[c][t] x[v + t - 1] / s), on
// MFMA with the taps as the contraction index (k = tap, 27-31 with zero
// weight).  Weights and inputs are each split into a BF16 value and a BF16
// remainder, and the three products that matter (hi hi, hi lo, lo hi) keep
// ~16 significant bits: three v_mfma_f32_16x16x32_bf16 per 16-voxel row.
__global__ __launch_bounds__(kThreads) void k_conv1(const bf16x8 *__restrict__ frag1,
                                                    const float *__restrict__ P,
                                                    const float *__restrict__ x, Vol d,
                                                    const double *__restrict__ norm2,
                                                    uint16_t *__restrict__ a1,
                                                    const int *__restrict__ skip)
{
    __shared__ float xs[kRegion];
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
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const bf16x8 wh = frag1[lane], wl = frag1[64 + lane];  // BF16 weights, remainders
    const int vl = lane % 16, g = lane / 16, cg = 4 * g;
    // taps 8g..8g+7 of this lane; taps past 26 read tap 26 (zero weight)
    int off[8];
#pragma unroll
    for (int e = 0; e < 8; ++e) off[e] = region_index(vl, 0, wave, min(8 * g + e, kTaps - 1));
    float b[4];
#pragma unroll
    for (int r = 0; r < 4; ++r) b[r] = P[OB1 + cg + r];
    __syncthreads();
    f32x4 acc[kTY];
#pragma unroll
    for (int y = 0; y < kTY; ++y) {
        // inputs split the same way: x = bf16(x) + bf16(x - bf16(x)) (+ tiny)
        bf16x8 xh, xl;
#pragma unroll
        for (int e = 0; e < 8; ++e) {
            const float v = xs[off[e] + y * kRX];
            const uint16_t h = f2bf(v);
            xh[e] = (short)h;
            xl[e] = (short)f2bf(v - bf2f(h));
        }
        acc[y] = f32x4{0.f, 0.f, 0.f, 0.f};
        acc[y] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(wh, xh, acc[y], 0, 0, 0);
        acc[y] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(wh, xl, acc[y], 0, 0, 0);
        acc[y] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(wl, xh, acc[y], 0, 0, 0);
    }
    const int xo = x0 + vl, zo = z0 + wave;
#pragma unroll
    for (int y = 0; y < kTY; ++y) {
        const int yo = y0 + y;
        if (xo < d.nx && yo < d.ny && zo < d.nz) {
            const int64_t vo = ((int64_t)zo * d.ny + yo) * d.nx + xo;
            bf16x4 o;
#pragma unroll
            for (int r = 0; r < 4; ++r) o[r] = (short)f2bf(fmaxf(acc[y][r] + b[r], 0.0f));
            *reinterpret_cast<bf16x4 *>(a1 + vo * kC + cg) = o;
        }
    }
}

// Epilogue of a 16 -> 16 layer for the tile at (x0, y0, z0): out =
// act(bias + acc) as BF16, act as for conv16_tile.
__device__ inline void conv16_store(const f32x4 (&acc)[kTY], const float (&b)[4], const Vol &d, int x0, int y0,
                                    int z0, int relu, const uint16_t *__restrict__ mask, uint16_t *__restrict__ out)
{
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int vl = lane % 16, cg = 4 * (lane / 16);
    const int xo = x0 + vl, zo = z0 + wave;
#pragma unroll
    for (int y = 0; y < kTY; ++y) {
        const int yo = y0 + y;
        if (xo < d.nx && yo < d.ny && zo < d.nz) {
            const int64_t vo = ((int64_t)zo * d.ny + yo) * d.nx + xo;
            bf16x4 m = {1, 1, 1, 1};
            if (mask) m = *reinterpret_cast<const bf16x4 *>(mask + vo * kC + cg);
            bf16x4 ov;
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                float val = acc[y][r] + b[r];
                if (relu) val = fmaxf(val, 0.0f);
                if (mask && !(bf2f((uint16_t)m[r]) > 0.0f)) val = 0.0f;
                ov[r] = (short)f2bf(val);
            }
            *reinterpret_cast<bf16x4 *>(out + vo * kC + cg) = ov;
        }
    }
}

// Epilogue of the 16 -> 1 layer: out = s (b3 + row 0 + row 1), zero where
// the map mask is 0.
__device__ inline void conv3_store(const f32x4 (&acc)[kTY], float s, float b3, const Vol &d, int x0, int y0, int z0,
                                   const uint8_t *__restrict__ map_mask, float *__restrict__ out)
{
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int xo = x0 + lane % 16, zo = z0 + wave;
#pragma unroll
    for (int y = 0; y < kTY; ++y) {
        const int yo = y0 + y;
        if (lane < 16 && xo < d.nx && yo < d.ny && zo < d.nz) {
            const int64_t vo = ((int64_t)zo * d.ny + yo) * d.nx + xo;
            float ov = s * ((acc[y][0] + acc[y][1]) + b3);
            if (map_mask && !map_mask[vo]) ov = 0.0f;
            out[vo] = ov;
        }
    }
}

// 16 -> 16 convolution of the tile at (x0, y0, z0) from its staged LDS
// region: fourteen MFMA instructions per 16-voxel row with the weights in
// registers.  out = act(bias + conv) where act is ReLU (relu = 1), or
// multiplication by [mask > 0] (mask != nullptr, the ReLU derivative of the
// layer below), or nothing.  Starts with the barrier that publishes the
// region.
__device__ inline void conv16_tile(const uint4 *region, const bf16x8 *__restrict__ frag,
                                   const float *__restrict__ bias, const Vol &d, int x0, int y0, int z0,
                                   int relu, const uint16_t *__restrict__ mask, uint16_t *__restrict__ out)
{
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    bf16x8 w[kTriples];
    bf16x4 wt[kTriples];
    load_conv_frags(frag, lane, w, wt);
    const int vl = lane % 16, g = lane / 16, cg = 4 * g;
    const ConvOffsets o = conv_offsets(vl, wave, g);
    float b[4] = {0.f, 0.f, 0.f, 0.f};
    if (bias)
#pragma unroll
        for (int r = 0; r < 4; ++r) b[r] = bias[cg + r];
    __syncthreads();
    f32x4 acc[kTY];
#pragma unroll
    for (int y = 0; y < kTY; ++y) acc[y] = f32x4{0.f, 0.f, 0.f, 0.f};
    conv_rows(reinterpret_cast<const char *>(region), o, w, wt, acc);
    conv16_store(acc, b, d, x0, y0, z0, relu, mask, out);
}

// 16 -> 16 convolution of a stored activation (training forward, and the
// data gradient with the transposed fragments).
__global__ __launch_bounds__(kThreads) void k_conv16(const uint16_t *__restrict__ in,
                                                     const bf16x8 *__restrict__ frag,
                                                     const float *__restrict__ bias, Vol d,
                                                     int relu, const uint16_t *__restrict__ mask,
                                                     uint16_t *__restrict__ out,
                                                     const int *__restrict__ skip)
{
    __shared__ uint4 region[kRegion * 2];
    if (skip && *skip) return;
    const int x0 = blockIdx.x * kTX, y0 = blockIdx.y * kTY, z0 = blockIdx.z * kTZ;
    stage_channels(in, d, x0, y0, z0, region);
    conv16_tile(region, frag, bias, d, x0, y0, z0, relu, mask, out);
}

// layer 3: out[v] = s * (b3 + sum_{c,t} w3[c][t] a2[v + t - 1][c]), zero
// where the map mask is 0.  On MFMA like the 16 -> 16 layer with the 1 x 16
// weight row as rows 0 (BF16 value) and 1 (BF16 remainder) of a 16 x 16
// matrix: D rows 0 and 1 land in lanes 0-15, elements 0 and 1.
__global__ __launch_bounds__(kThreads) void k_conv3(const bf16x8 *__restrict__ frag3,
                                                    const float *__restrict__ P,
                                                    const uint16_t *__restrict__ a2, Vol d,
                                                    const double *__restrict__ norm2,
                                                    const uint8_t *__restrict__ map_mask,
                                                    float *__restrict__ out,
                                                    const int *__restrict__ skip)
{
    __shared__ uint4 region[kRegion * 2];
    if (skip && *skip) return;
    const float s = read_scale(norm2);
    const int x0 = blockIdx.x * kTX, y0 = blockIdx.y * kTY, z0 = blockIdx.z * kTZ;
    stage_channels(a2, d, x0, y0, z0, region);
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    bf16x8 w[kTriples];
    bf16x4 wt[kTriples];
    load_conv_frags(frag3, lane, w, wt);
    const int vl = lane % 16, g = lane / 16;
    const ConvOffsets o = conv_offsets(vl, wave, g);
    const float b3 = P[OB3];
    __syncthreads();
    f32x4 acc[kTY];
#pragma unroll
    for (int y = 0; y < kTY; ++y) acc[y] = f32x4{0.f, 0.f, 0.f, 0.f};
    conv_rows(reinterpret_cast<const char *>(region), o, w, wt, acc);
    conv3_store(acc, s, b3, d, x0, y0, z0, map_mask, out);
}

// ---- persistent forward kernels (inference): each workgroup takes tiles
// t, t + G, t + 2G, ... (G workgroups) and, while it computes one, the
// region of its next tile arrives in the other of two LDS buffers through
// direct-to-LDS buffer loads (no registers, no staging stores), so the
// staging latency hides behind the MFMA work instead of adding to it.
// Each tile's arithmetic is that of k_conv16 / k_conv3, bit for bit.
constexpr int kChunks = (2 * kRegion + 63) / 64;  // 64-slot wave loads per region
constexpr int kSlots = kChunks * 64;              // region buffer with its padding

// Issues the loads of the region of the tile at (x0, y0, z0) into buf: slot
// s of plane h = s / kRegion holds channels 8h..8h+7 of region voxel
// s % kRegion; voxels outside the volume and the padding get offsets past
// the buffer's range, which the hardware reads as zeros.  Lane l of a wave
// load writes slot 64 c + l.  rs spans the [voxel][16] BF16 activation.
__device__ inline void stage_channels_lds(__amdgpu_buffer_rsrc_t rs, const Vol &d, int x0, int y0, int z0,
                                          uint4 *buf)
{
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    for (int c = wave; c < kChunks; c += kThreads / 64) {
        const int sl = c * 64 + lane;
        uint32_t off = 0xFFFFFFF0u;
        if (sl < 2 * kRegion) {
            const int h = sl >= kRegion ? 1 : 0, rv = sl - h * kRegion;
            const int ex = rv % kRX, ey = (rv / kRX) % kRY, ez = rv / (kRX * kRY);
            const int gx = x0 + ex - 1, gy = y0 + ey - 1, gz = z0 + ez - 1;
            if (gx >= 0 && gx < d.nx && gy >= 0 && gy < d.ny && gz >= 0 && gz < d.nz)
                off = (uint32_t)((((int64_t)gz * d.ny + gy) * d.nx + gx) * (kC * 2) + h * 16);
        }
        __builtin_amdgcn_raw_ptr_buffer_load_lds(rs, (__attribute__((address_space(3))) void *)(buf + c * 64), 16,
                                                 (int)off, 0, 0, 0);
    }
}

// Largest activation the persistent kernels address through one buffer
// resource (offsets below the out-of-range marker).
constexpr int64_t kMaxPipelinedVoxels = ((int64_t)1 << 27) - 1;

// The tile loop of a persistent forward kernel: tile(region, x0, y0, z0)
// computes and stores one tile from a published region.  The two buffers
// alternate at compile time (two tiles per round).
template <class Tile>
__device__ inline void pipelined_tiles(const uint16_t *__restrict__ in, const Vol &d, uint4 *buf0, uint4 *buf1,
                                       Tile &&tile)
{
    const int ntx = (d.nx + kTX - 1) / kTX, nty = (d.ny + kTY - 1) / kTY, ntz = (d.nz + kTZ - 1) / kTZ;
    const int T = ntx * nty * ntz;
    const auto rs = make_rsrc(in, (uint32_t)(d.n * kC * 2));
    auto origin = [&](int t, int &x0, int &y0, int &z0) {
        x0 = (t % ntx) * kTX;
        const int r = t / ntx;
        y0 = (r % nty) * kTY;
        z0 = (r / nty) * kTZ;
    };
    int t = blockIdx.x, x0, y0, z0;
    if (t >= T) return;
    origin(t, x0, y0, z0);
    stage_channels_lds(rs, d, x0, y0, z0, buf0);
    // one step: publish cur (its loads done, every wave past the previous
    // tile, so next is free), prefetch the next tile into next, compute t
    auto step = [&](uint4 *cur, uint4 *next) -> bool {
        asm volatile("s_waitcnt vmcnt(0)" ::: "memory");
        __syncthreads();
        const int tn = t + (int)gridDim.x;
        int nx0 = 0, ny0 = 0, nz0 = 0;
        if (tn < T) {
            origin(tn, nx0, ny0, nz0);
            stage_channels_lds(rs, d, nx0, ny0, nz0, next);
        }
        tile(cur, x0, y0, z0);
        if (tn >= T) return false;
        t = tn;
        x0 = nx0;
        y0 = ny0;
        z0 = nz0;
        return true;
    };
    while (step(buf0, buf1) && step(buf1, buf0)) {
    }
}

// Persistent 16 -> 16 layer with ReLU (the inference forward's layer 2).
__global__ __launch_bounds__(kThreads) void k_conv16p(const uint16_t *__restrict__ in,
                                                      const bf16x8 *__restrict__ frag,
                                                      const float *__restrict__ bias, Vol d,
                                                      uint16_t *__restrict__ out, const int *__restrict__ skip)
{
    __shared__ uint4 buf0[kSlots];
    __shared__ uint4 buf1[kSlots];
    if (skip && *skip) return;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    bf16x8 w[kTriples];
    bf16x4 wt[kTriples];
    load_conv_frags(frag, lane, w, wt);
    const int vl = lane % 16, g = lane / 16, cg = 4 * g;
    const ConvOffsets o = conv_offsets(vl, wave, g);
    float b[4];
#pragma unroll
    for (int r = 0; r < 4; ++r) b[r] = bias[cg + r];
    pipelined_tiles(in, d, buf0, buf1, [&](const uint4 *region, int x0, int y0, int z0) {
        f32x4 acc[kTY];
#pragma unroll
        for (int y = 0; y < kTY; ++y) acc[y] = f32x4{0.f, 0.f, 0.f, 0.f};
        conv_rows(reinterpret_cast<const char *>(region), o, w, wt, acc);
        conv16_store(acc, b, d, x0, y0, z0, 1, nullptr, out);
    });
}

// Persistent 16 -> 1 layer (the inference forward's layer 3).
__global__ __launch_bounds__(kThreads) void k_conv3p(const bf16x8 *__restrict__ frag3,
                                                     const float *__restrict__ P,
                                                     const uint16_t *__restrict__ a2, Vol d,
                                                     const double *__restrict__ norm2,
                                                     const uint8_t *__restrict__ map_mask,
                                                     float *__restrict__ out, const int *__restrict__ skip)
{
    __shared__ uint4 buf0[kSlots];
    __shared__ uint4 buf1[kSlots];
    if (skip && *skip) return;
    const float s = read_scale(norm2);
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    bf16x8 w[kTriples];
    bf16x4 wt[kTriples];
    load_conv_frags(frag3, lane, w, wt);
    const int vl = lane % 16, g = lane / 16;
    const ConvOffsets o = conv_offsets(vl, wave, g);
    const float b3 = P[OB3];
    pipelined_tiles(a2, d, buf0, buf1, [&](const uint4 *region, int x0, int y0, int z0) {
        f32x4 acc[kTY];
#pragma unroll
        for (int y = 0; y < kTY; ++y) acc[y] = f32x4{0.f, 0.f, 0.f, 0.f};
        conv_rows(reinterpret_cast<const char *>(region), o, w, wt, acc);
        conv3_store(acc, s, b3, d, x0, y0, z0, map_mask, out);
    });
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
    bf16x8 *frag, *fragT;    // forward and transposed fragment sets
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
    t.frag = (bf16x8 *)take(sizeof(bf16x8) * kFragFwd);
    t.fragT = (bf16x8 *)take(sizeof(bf16x8) * kFragConv);
    t.part = (double *)take(sizeof(double) * kWgBlocks * 6928);
    t.loss_part = (double *)take(sizeof(double) * kLossBlocks);
    if (w) *w = t;
    return off;
}

// Forward-only workspace (activations and fragments) for flexible CG.
size_t convnet_forward_ws_bytes(int64_t n)
{
    return align256(sizeof(uint16_t) * kC * n) * 2 + align256(sizeof(bf16x8) * kFragFwd);
}

static dim3 tile_grid(const Vol &d)
{
    return dim3((unsigned)((d.nx + kTX - 1) / kTX), (unsigned)((d.ny + kTY - 1) / kTY),
                (unsigned)((d.nz + kTZ - 1) / kTZ));
}

// Workgroups of a persistent forward kernel: as many as stay resident on the
// device (occupancy x compute units, queried once per kernel), at most one
// per tile.
static unsigned persistent_grid(const void *kernel, int64_t tiles)
{
    static std::mutex mu;
    static std::map<const void *, int64_t> resident;
    int64_t r = 0;
    {
        std::lock_guard<std::mutex> lock(mu);
        auto it = resident.find(kernel);
        if (it != resident.end()) {
            r = it->second;
        } else {
            int dev = 0, cus = 0, per = 0;
            (void)hipGetDevice(&dev);
            (void)hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
            (void)hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, kernel, kThreads, 0);
            r = (int64_t)(cus > 0 ? cus : 256) * (per > 0 ? per : 1);
            resident[kernel] = r;
        }
    }
    return (unsigned)(tiles < r ? (tiles > 0 ? tiles : 1) : r);
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
    bf16x8 *frag = (bf16x8 *)(base + 2 * align256(sizeof(uint16_t) * kC * d.n));
    if (prep_frags)
        hipLaunchKernelGGL(k_conv_frags, dim3((kFragFwd + 255) / 256), dim3(256), 0, s, P, 0, frag);
    hipLaunchKernelGGL(k_conv1, tile_grid(d), dim3(kThreads), 0, s, frag + kFrag1, P, x, d, norm2, a1, skip);
    if (d.n <= kMaxPipelinedVoxels) {  // persistent, pipelined layers 2 and 3
        const dim3 tg = tile_grid(d);
        const int64_t tiles = (int64_t)tg.x * tg.y * tg.z;
        const unsigned g16 = persistent_grid(reinterpret_cast<const void *>(k_conv16p), tiles);
        const unsigned g3 = persistent_grid(reinterpret_cast<const void *>(k_conv3p), tiles);
        hipLaunchKernelGGL(k_conv16p, dim3(g16), dim3(kThreads), 0, s, a1, frag, P + OB2, d, a2, skip);
        hipLaunchKernelGGL(k_conv3p, dim3(g3), dim3(kThreads), 0, s, frag + kFrag3, P, a2, d, norm2, map_mask, out,
                           skip);
    } else {
        hipLaunchKernelGGL(k_conv16, tile_grid(d), dim3(kThreads), 0, s, a1, frag, P + OB2, d, 1,
                           (const uint16_t *)nullptr, a2, skip);
        hipLaunchKernelGGL(k_conv3, tile_grid(d), dim3(kThreads), 0, s, frag + kFrag3, P, a2, d, norm2, map_mask,
                           out, skip);
    }
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
    hipLaunchKernelGGL(k_conv_frags, dim3((kFragFwd + 255) / 256), dim3(256), 0, s, params_d, 0, w.frag);
    hipLaunchKernelGGL(k_conv_frags, dim3((kFragConv + 255) / 256), dim3(256), 0, s, params_d, 1, w.fragT);
    const int *noskip = nullptr;
    hipLaunchKernelGGL(k_conv1, rowgrid, dim3(kThreads), 0, s, w.frag + kFrag1, params_d, x_d, d,
                       (const double *)nullptr, w.a1, noskip);
    hipLaunchKernelGGL(k_conv16, rowgrid, dim3(kThreads), 0, s, w.a1, w.frag, params_d + OB2, d, 1,
                       (const uint16_t *)nullptr, w.a2, noskip);
    if (target_d) {
        hipLaunchKernelGGL(k_conv3, rowgrid, dim3(kThreads), 0, s, w.frag + kFrag3, params_d, w.a2, d,
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
