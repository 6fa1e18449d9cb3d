// vo_net.hip -- the learned depth/rigidness proposal: six 3x3 convolutions
// (32 channels, BF16 weights and activations, FP32 accumulation on the matrix
// cores), its loss, backward pass and Adam, on NHWC activations.
//
// A convolution is an implicit GEMM per 16-pixel row segment:
//   out[p][m] = sum over taps and k of Wl[tap][m][k] * in[p + off(tap)][k]
// on v_mfma_f32_16x16x32_bf16.  The weights are the A operand (lane l holds
// Wl[tap][l % 16][8 (l / 16) .. + 7]), the input the B operand (lane l holds the
// eight channels 8 (l / 16) .. + 7 of pixel l % 16: one 16-byte load), and the
// accumulator returns out[pixel l % 16][4 (l / 16) + i], i = 0..3: four
// consecutive channels of one pixel, stored as one 8-byte word.  The same
// kernel runs the backward pass to the input, with the per-tap transposed and
// flipped weights and the next layer's ReLU mask.  The weight gradient stages a
// 32-pixel segment of the output gradient and the three input rows around it in
// LDS, transposed so that a lane's eight pixels are contiguous, and sums
// per-workgroup partials in a fixed order.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "vo_internal.hpp"

namespace vo {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

constexpr int kNetC = 32;     // channels of every activation buffer
constexpr int kNetCo6 = 16;   // outputs of the last layer (1 + T <= 9 used)

__device__ __forceinline__ bf16x8 load8(const __bf16 *p)
{
    const uint4 u = *(const uint4 *)p;
    bf16x8 v;
    __builtin_memcpy(&v, &u, 16);
    return v;
}

__device__ __forceinline__ bf16x8 zero8()
{
    const uint4 u = {0u, 0u, 0u, 0u};
    bf16x8 v;
    __builtin_memcpy(&v, &u, 16);
    return v;
}

__device__ __forceinline__ void store4(__bf16 *p, float a, float b, float c, float d)
{
    __bf16 v[4] = {(__bf16)a, (__bf16)b, (__bf16)c, (__bf16)d};
    uint2 u;
    __builtin_memcpy(&u, v, 8);
    *(uint2 *)p = u;
}

// ---------------------------------------------------------------------------
// input: flows [N][T][H][W][2] -> x [N][H][W][32], channel 2(t-1) + c = component
// c of X_t / in_scale, non-finite as 0, channels 2T.. zero
__global__ void __launch_bounds__(256) k_net_input(const float2 *__restrict__ flows, __bf16 *__restrict__ x,
                                                   int N, int T, int H, int W, float inv_scale)
{
    const int64_t HW = (int64_t)H * W;
    const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= (int64_t)N * HW) return;
    const int64_t n = p / HW, j = p - n * HW;
    float v[kNetC];
#pragma unroll
    for (int c = 0; c < kNetC; ++c) v[c] = 0.0f;
#pragma unroll
    for (int t = 0; t < kTMax; ++t) {
        if (t < T) {
            const float2 f = flows[(n * T + t) * HW + j];
            v[2 * t] = isfinite(f.x) ? f.x * inv_scale : 0.0f;
            v[2 * t + 1] = isfinite(f.y) ? f.y * inv_scale : 0.0f;
        }
    }
    __bf16 *o = x + p * kNetC;
#pragma unroll
    for (int c = 0; c < kNetC; c += 4) store4(o + c, v[c], v[c + 1], v[c + 2], v[c + 3]);
}

// ---------------------------------------------------------------------------
enum ConvMode { kConvRelu = 0, kConvLinearF32 = 1, kConvMasked = 2 };

struct ConvArgs {
    const __bf16 *in;    // [N][H][W][32]
    const __bf16 *w;     // [9][16 MT][32]: tap, output channel m, input channel k
    const float *bias;   // [16 MT] (modes 0, 1)
    const __bf16 *mask;  // [N][H][W][32] (mode 2): out *= (mask > 0)
    void *out;           // bf16 [N][H][W][32] (modes 0, 2) or float [N][H][W][16] (mode 1)
    int N, H, W;
    int tiles;           // N * H * ceil(W / 16)
};

template <int MODE, int MT>
__global__ void __launch_bounds__(256) k_conv(ConvArgs a)
{
    const int lane = threadIdx.x & 63;
    const int wave = blockIdx.x * 4 + (threadIdx.x >> 6), nwave = gridDim.x * 4;
    const int r = lane & 15, q = lane >> 4;
    // this lane's weights for every tap and output tile
    bf16x8 wr[9][MT];
#pragma unroll
    for (int tap = 0; tap < 9; ++tap)
#pragma unroll
        for (int mt = 0; mt < MT; ++mt) wr[tap][mt] = load8(a.w + ((tap * 16 * MT) + 16 * mt + r) * kNetC + 8 * q);
    const int tpr = (a.W + 15) >> 4;
    for (int g = wave; g < a.tiles; g += nwave) {
        const int row = g / tpr, x0 = (g - row * tpr) * 16;
        const int n = row / a.H, y = row - n * a.H;
        const int xp = x0 + r;
        f32x4 acc[MT];
#pragma unroll
        for (int mt = 0; mt < MT; ++mt) acc[mt] = (f32x4){0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll
        for (int tap = 0; tap < 9; ++tap) {
            const int yy = y + tap / 3 - 1, xx = xp + tap % 3 - 1;
            const bool in = yy >= 0 && yy < a.H && xx >= 0 && xx < a.W;
            const bf16x8 b = in ? load8(a.in + (((int64_t)n * a.H + yy) * a.W + xx) * kNetC + 8 * q) : zero8();
#pragma unroll
            for (int mt = 0; mt < MT; ++mt)
                acc[mt] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(wr[tap][mt], b, acc[mt], 0, 0, 0);
        }
        if (xp < a.W) {
            const int64_t p = ((int64_t)n * a.H + y) * a.W + xp;
#pragma unroll
            for (int mt = 0; mt < MT; ++mt) {
                const int m = 16 * mt + 4 * q;
                float v[4] = {acc[mt][0], acc[mt][1], acc[mt][2], acc[mt][3]};
                if (MODE != kConvMasked) {
#pragma unroll
                    for (int i = 0; i < 4; ++i) v[i] += a.bias[m + i];
                }
                if (MODE == kConvRelu) {
#pragma unroll
                    for (int i = 0; i < 4; ++i) v[i] = fmaxf(v[i], 0.0f);
                }
                if (MODE == kConvMasked) {
                    const uint2 mu = *(const uint2 *)(a.mask + p * kNetC + m);
                    __bf16 mk[4];
                    __builtin_memcpy(mk, &mu, 8);
#pragma unroll
                    for (int i = 0; i < 4; ++i) v[i] = (float)mk[i] > 0.0f ? v[i] : 0.0f;
                }
                if (MODE == kConvLinearF32) {
                    *(float4 *)((float *)a.out + p * kNetCo6 + m) = make_float4(v[0], v[1], v[2], v[3]);
                } else {
                    store4((__bf16 *)a.out + p * kNetC + m, v[0], v[1], v[2], v[3]);
                }
            }
        }
    }
}

// ---------------------------------------------------------------------------
// The whole forward pass on one output tile of kFuseTH x kFuseTW pixels, every
// intermediate activation in LDS: the tile's input region (6 pixels of halo,
// one per layer) is staged once, and each layer reads one LDS buffer and
// writes the other, its output region one pixel smaller on every side.
// Output pixels of a region are taken 16 at a time in row-major order (a group
// may span two rows), so no MFMA lane idles at row ends.  Positions outside
// the image hold 0 in every buffer (the zero padding of each layer).  Every
// output is computed as k_conv computes it (the same taps in the same order,
// the same bias, ReLU and BF16 rounding), so the result equals the per-layer
// pass bit for bit.
constexpr int kFuseTW = 32, kFuseTH = 16, kFuseHalo = 6;
constexpr int kFuseInW = kFuseTW + 2 * kFuseHalo, kFuseInH = kFuseTH + 2 * kFuseHalo;
constexpr int kFuseBufA = kFuseInW * kFuseInH * kNetC;                   // BF16 elements
constexpr int kFuseBufB = (kFuseInW - 2) * (kFuseInH - 2) * kNetC;
constexpr int kFuseThreads = 512;

struct FusedArgs {
    const __bf16 *x;      // [N][H][W][32] network input
    const __bf16 *w[6];   // [9][16 MT][32] per layer
    const float *b[6];    // [16 MT] per layer
    float *z;             // [N][H][W][16]
    int N, H, W;
    int tiles_x, tiles_y;
};

template <int MT, bool LAST>
__device__ __forceinline__ void fused_layer(const FusedArgs &a, int k, const __bf16 *in, __bf16 *out, int win,
                                            int hin, int oy, int ox, int n, int lane, int wave)
{
    const int r = lane & 15, q = lane >> 4;
    const int wout = win - 2, hout = hin - 2, npx = wout * hout;
    bf16x8 wr[9][MT];
#pragma unroll
    for (int tap = 0; tap < 9; ++tap)
#pragma unroll
        for (int mt = 0; mt < MT; ++mt) wr[tap][mt] = load8(a.w[k] + ((tap * 16 * MT) + 16 * mt + r) * kNetC + 8 * q);
    // two groups of 16 pixels per step: their accumulation chains interleave
    // on the matrix core (each chain's nine taps depend on one another)
    constexpr int G = 2;
    for (int g0 = G * wave; g0 * 16 < npx; g0 += G * (kFuseThreads / 64)) {
        int pix[G], prow[G], pcol[G];
#pragma unroll
        for (int j = 0; j < G; ++j) {
            pix[j] = (g0 + j) * 16 + r;
            const int pc = pix[j] < npx ? pix[j] : npx - 1;   // idle lanes read a valid pixel
            prow[j] = pc / wout;
            pcol[j] = pc - prow[j] * wout;
        }
        f32x4 acc[G][MT];
#pragma unroll
        for (int j = 0; j < G; ++j)
#pragma unroll
            for (int mt = 0; mt < MT; ++mt) acc[j][mt] = (f32x4){0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll
        for (int tap = 0; tap < 9; ++tap) {
#pragma unroll
            for (int j = 0; j < G; ++j) {
                const bf16x8 bv = load8(in + ((prow[j] + tap / 3) * win + pcol[j] + tap % 3) * kNetC + 8 * q);
#pragma unroll
                for (int mt = 0; mt < MT; ++mt)
                    acc[j][mt] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(wr[tap][mt], bv, acc[j][mt], 0, 0, 0);
            }
        }
#pragma unroll
        for (int j = 0; j < G; ++j) {
            if (pix[j] >= npx) continue;
            const int gy = oy + prow[j], gx = ox + pcol[j];   // the output pixel in the image
            const bool inside = gy >= 0 && gy < a.H && gx >= 0 && gx < a.W;
#pragma unroll
            for (int mt = 0; mt < MT; ++mt) {
                const int m = 16 * mt + 4 * q;
                float v[4] = {acc[j][mt][0], acc[j][mt][1], acc[j][mt][2], acc[j][mt][3]};
#pragma unroll
                for (int i = 0; i < 4; ++i) v[i] += a.b[k][m + i];
                if constexpr (LAST) {
                    if (inside)
                        *(float4 *)(a.z + (((int64_t)n * a.H + gy) * a.W + gx) * kNetCo6 + m) =
                            make_float4(v[0], v[1], v[2], v[3]);
                } else {
#pragma unroll
                    for (int i = 0; i < 4; ++i) v[i] = inside ? fmaxf(v[i], 0.0f) : 0.0f;
                    store4(out + pix[j] * kNetC + m, v[0], v[1], v[2], v[3]);
                }
            }
        }
    }
}

__global__ void __launch_bounds__(kFuseThreads) k_net_fused(FusedArgs a)
{
    extern __shared__ __bf16 fl[];
    __bf16 *bufA = fl, *bufB = fl + kFuseBufA;
    const int per = a.tiles_x * a.tiles_y;
    const int n = blockIdx.x / per, t = blockIdx.x - n * per;
    const int ty = t / a.tiles_x, tx = t - ty * a.tiles_x;
    const int y0 = ty * kFuseTH - kFuseHalo, x0 = tx * kFuseTW - kFuseHalo;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    // the input region, 16 bytes (eight channels) per item, zero outside the image
    for (int i = threadIdx.x; i < kFuseInW * kFuseInH * 4; i += kFuseThreads) {
        const int pix = i >> 2, c = i & 3;
        const int row = pix / kFuseInW, col = pix - row * kFuseInW;
        const int gy = y0 + row, gx = x0 + col;
        uint4 u = {0u, 0u, 0u, 0u};
        if (gy >= 0 && gy < a.H && gx >= 0 && gx < a.W)
            u = *(const uint4 *)(a.x + (((int64_t)n * a.H + gy) * a.W + gx) * kNetC + 8 * c);
        *(uint4 *)(bufA + pix * kNetC + 8 * c) = u;
    }
    __syncthreads();
    int win = kFuseInW, hin = kFuseInH;
    for (int k = 0; k < 5; ++k) {
        const __bf16 *in = (k & 1) ? bufB : bufA;
        __bf16 *out = (k & 1) ? bufA : bufB;
        fused_layer<2, false>(a, k, in, out, win, hin, y0 + k + 1, x0 + k + 1, n, lane, wave);
        __syncthreads();
        win -= 2;
        hin -= 2;
    }
    fused_layer<1, true>(a, 5, bufB, nullptr, win, hin, y0 + 6, x0 + 6, n, lane, wave);
}

// ---------------------------------------------------------------------------
// weight gradient of one layer: partial[blk][tap][m][k] = sum over the block's
// pixels of dy[p][m] x[p + off(tap)][k], partial bias sums pb[blk][m]
struct WgradArgs {
    const __bf16 *x;     // layer input [N][H][W][32]
    const __bf16 *dy;    // output gradient [N][H][W][32] (channels >= CO are 0)
    float *part;         // [blocks][9][32][32]
    float *pbias;        // [blocks][32]
    int N, H, W;
    int segs;            // N * H * ceil(W / 32)
};

__global__ void __launch_bounds__(256) k_conv_wgrad(WgradArgs a)
{
    // dyT[m][p] and three shifted copies xT[dx][row][k][p] of the input rows
    __shared__ __attribute__((aligned(16))) __bf16 dyT[kNetC][32];
    __shared__ __attribute__((aligned(16))) __bf16 xT[3][3][kNetC][32];
    const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
    const int r = lane & 15, q = lane >> 4;
    // wave wv owns the (tap, m-tile, k-tile) combinations 9 wv .. 9 wv + 8
    f32x4 acc[9];
#pragma unroll
    for (int i = 0; i < 9; ++i) acc[i] = (f32x4){0.0f, 0.0f, 0.0f, 0.0f};
    float bsum = 0.0f;   // thread tid < 32: bias gradient of channel tid
    const int spr = (a.W + 31) >> 5;
    for (int s = blockIdx.x; s < a.segs; s += gridDim.x) {
        const int row = s / spr, x0 = (s - row * spr) * 32;
        const int n = row / a.H, y = row - n * a.H;
        __syncthreads();   // the previous segment's reads are done
        // dy: 32 pixels x 32 channels, 16 bytes per thread (threads 0..127)
        if (tid < 128) {
            const int p = tid >> 2, c8 = (tid & 3) * 8;
            const int xx = x0 + p;
            bf16x8 v = zero8();
            if (xx < a.W) v = load8(a.dy + (((int64_t)n * a.H + y) * a.W + xx) * kNetC + c8);
#pragma unroll
            for (int j = 0; j < 8; ++j) dyT[c8 + j][p] = v[j];
        }
        // input rows y-1, y, y+1 at columns x0-1 .. x0+32, stored for each dx as
        // xT[dx][row][k][p] = x[row][x0 + p + dx - 1][k]
        for (int i = tid; i < 3 * 34 * 4; i += 256) {
            const int rr = i / (34 * 4), rem = i - rr * 34 * 4, col = rem >> 2, c8 = (rem & 3) * 8;
            const int yy = y + rr - 1, xx = x0 + col - 1;
            bf16x8 v = zero8();
            if (yy >= 0 && yy < a.H && xx >= 0 && xx < a.W)
                v = load8(a.x + (((int64_t)n * a.H + yy) * a.W + xx) * kNetC + c8);
#pragma unroll
            for (int dx = 0; dx < 3; ++dx) {
                const int p = col - dx;   // xT[dx][.][.][p] holds column x0 + p + dx - 1
                if (p >= 0 && p < 32) {
#pragma unroll
                    for (int j = 0; j < 8; ++j) xT[dx][rr][c8 + j][p] = v[j];
                }
            }
        }
        __syncthreads();
        if (tid < kNetC) {
#pragma unroll 8
            for (int p = 0; p < 32; ++p) bsum += (float)dyT[tid][p];
        }
#pragma unroll
        for (int i = 0; i < 9; ++i) {
            const int combo = 9 * wv + i;   // tap * 4 + mt * 2 + kt
            const int tap = combo >> 2, mt = (combo >> 1) & 1, kt = combo & 1;
            const int dyy = tap / 3, dxx = tap % 3;
            // A[m][pixel]: lane l: m = 16 mt + l % 16, pixels 8 (l / 16) .. + 7
            const bf16x8 av = *(const bf16x8 *)&dyT[16 * mt + r][8 * q];
            // B[pixel][k]: lane l: k = 16 kt + l % 16, pixels 8 (l / 16) .. + 7
            const bf16x8 bv = *(const bf16x8 *)&xT[dxx][dyy][16 * kt + r][8 * q];
            acc[i] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(av, bv, acc[i], 0, 0, 0);
        }
    }
    // D[m][k]: lane l holds m = 16 mt + 4 (l / 16) + i, k = 16 kt + l % 16
    float *dst = a.part + (size_t)blockIdx.x * 9 * kNetC * kNetC;
#pragma unroll
    for (int i = 0; i < 9; ++i) {
        const int combo = 9 * wv + i;
        const int tap = combo >> 2, mt = (combo >> 1) & 1, kt = combo & 1;
#pragma unroll
        for (int e = 0; e < 4; ++e)
            dst[(tap * kNetC + 16 * mt + 4 * q + e) * kNetC + 16 * kt + r] = acc[i][e];
    }
    if (tid < kNetC) a.pbias[(size_t)blockIdx.x * kNetC + tid] = bsum;
}

// fixed-order sum of the partials into the layer's gradient in the packed
// parameter layout w[dy][dx][ci][co], b[co] (co < CO used)
__global__ void __launch_bounds__(256) k_wgrad_reduce(const float *__restrict__ part, const float *__restrict__ pbias,
                                                      int blocks, int CO, float *__restrict__ g)
{
    const int e = blockIdx.x * blockDim.x + threadIdx.x;   // packed index
    const int nw = 9 * kNetC * CO;
    if (e < nw) {
        const int tap = e / (kNetC * CO), rem = e - tap * kNetC * CO, ci = rem / CO, co = rem - ci * CO;
        const int src = (tap * kNetC + co) * kNetC + ci;   // partial layout [tap][m = co][k = ci]
        double s = 0.0;
        for (int b = 0; b < blocks; ++b) s += part[(size_t)b * 9 * kNetC * kNetC + src];
        g[e] = (float)s;
    } else if (e < nw + CO) {
        const int co = e - nw;
        double s = 0.0;
        for (int b = 0; b < blocks; ++b) s += pbias[(size_t)b * kNetC + co];
        g[e] = (float)s;
    }
}

// ---------------------------------------------------------------------------
// loss of z [N][H][W][16] against log theta* and W*; writes dloss/dz as bf16
// [N][H][W][32] (channels > T zero) and per-block partial sums of the loss
struct LossArgs {
    const float *z;
    const float *depth;   // theta* [N][H][W] (> 0)
    const float *rig;     // W* [N][T][H][W]
    __bf16 *dz;
    double *part;         // [blocks]
    int N, T, H, W;
};

__global__ void __launch_bounds__(256) k_net_loss(LossArgs a)
{
    __shared__ double red[256];
    const int64_t HW = (int64_t)a.H * a.W, npx = (int64_t)a.N * HW;
    const double inv_px = 1.0 / (double)npx, inv_pt = 1.0 / ((double)npx * a.T);
    double acc = 0.0;
    for (int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; p < npx; p += (int64_t)gridDim.x * blockDim.x) {
        const int64_t n = p / HW, j = p - n * HW;
        const float *zp = a.z + p * kNetCo6;
        float g[kNetC];
#pragma unroll
        for (int c = 0; c < kNetC; ++c) g[c] = 0.0f;
        const float d = zp[0] - logf(a.depth[p]);
        acc += (double)d * d * inv_px;
        g[0] = (float)(2.0 * d * inv_px);
#pragma unroll
        for (int t = 0; t < kTMax; ++t) {
            if (t < a.T) {
                const float s = zp[1 + t], w = a.rig[(n * a.T + t) * HW + j];
                const float sp = fmaxf(s, 0.0f) + log1pf(expf(-fabsf(s)));
                acc += (double)(sp - w * s) * inv_pt;
                g[1 + t] = (float)((1.0 / (1.0 + exp(-(double)s)) - w) * inv_pt);
            }
        }
        __bf16 *o = a.dz + p * kNetC;
#pragma unroll
        for (int c = 0; c < kNetC; c += 4) store4(o + c, g[c], g[c + 1], g[c + 2], g[c + 3]);
    }
    red[threadIdx.x] = acc;
    __syncthreads();
    for (int s = 128; s > 0; s >>= 1) {
        if ((int)threadIdx.x < s) red[threadIdx.x] += red[threadIdx.x + s];
        __syncthreads();
    }
    if (threadIdx.x == 0) a.part[blockIdx.x] = red[0];
}

__global__ void k_net_loss_reduce(const double *part, int n, double *out)
{
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    double s = 0.0;
    for (int i = 0; i < n; ++i) s += part[i];
    *out = s;
}

// ---------------------------------------------------------------------------
// proposal outputs: theta = exp(z_0), W_t = sigmoid(z_t)
__global__ void __launch_bounds__(256) k_net_outputs(const float *__restrict__ z, float *__restrict__ depth,
                                                     float *__restrict__ rig, int N, int T, int H, int W)
{
    const int64_t HW = (int64_t)H * W;
    const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= (int64_t)N * HW) return;
    const int64_t n = p / HW, j = p - n * HW;
    const float *zp = z + p * kNetCo6;
    if (depth) depth[p] = expf(zp[0]);
    if (rig)
        for (int t = 0; t < T; ++t) rig[(n * T + t) * HW + j] = 1.0f / (1.0f + expf(-zp[1 + t]));
}

// ---------------------------------------------------------------------------
// Adam on the packed FP32 parameters, then the BF16 copies: forward
// wf[tap][m = co][k = ci] (16 MT rows, zero beyond CO) and, for the input
// gradient, wb[tap'][m = ci][k = co] with tap' = 8 - tap (zero beyond CO)
struct AdamArgs {
    float *p, *m, *v;
    const float *g;
    int n;
    float lr, b1, b2, eps;
    float o1, o2, c1, c2;            // 1 - b1, 1 - b2, 1 - b1^t, 1 - b2^t (rounded once from FP64)
    int update;                      // 0: layouts only
};

struct LayerMap {
    int off, CO, MT;     // packed offset, real output channels, output tiles
    __bf16 *wf, *wb;     // wb may be NULL (first layer)
};

struct NetLayers {
    LayerMap L[6];
};

__global__ void __launch_bounds__(256) k_net_adam(AdamArgs a, NetLayers nl)
{
    const int e = blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= a.n) return;
    float p = a.p[e];
    if (a.update) {
        const float g = a.g[e];
        const float m = a.b1 * a.m[e] + a.o1 * g;
        const float v = a.b2 * a.v[e] + a.o2 * g * g;
        a.m[e] = m;
        a.v[e] = v;
        p -= a.lr * (m / a.c1) / (sqrtf(v / a.c2) + a.eps);
        a.p[e] = p;
    }
    int k = 0;
    while (k < 5 && e >= nl.L[k + 1].off) ++k;
    const LayerMap &L = nl.L[k];
    const int le = e - L.off, nw = 9 * kNetC * L.CO;
    if (le >= nw) return;   // bias: used in FP32 directly
    const int tap = le / (kNetC * L.CO), rem = le - tap * kNetC * L.CO, ci = rem / L.CO, co = rem - ci * L.CO;
    L.wf[(tap * 16 * L.MT + co) * kNetC + ci] = (__bf16)p;
    if (L.wb) L.wb[((8 - tap) * kNetC + ci) * kNetC + co] = (__bf16)p;
}

}  // namespace vo

// ===========================================================================
// host side
// ===========================================================================
using namespace vo;

struct voldor_net {
    int T, N_max, H_max, W_max;
    int n_params;
    int off[7];
    int CO[6];
    float *p, *m, *v, *g;          // packed FP32 parameters, Adam moments, gradient
    __bf16 *wf[6], *wb[6];
    __bf16 *act[6];                // layer inputs, [N][H][W][32]
    float *z;                      // [N][H][W][16]
    __bf16 *gbuf[2];               // gradients, [N][H][W][32]
    float *part, *pbias;           // weight-gradient partials
    double *lpart;                 // loss partials
    int step;
};

namespace {

constexpr int kWgradBlocks = 512;
constexpr int kLossBlocks = 512;

template <typename T>
hipError_t nalloc(T **p, size_t n)
{
    return hipMalloc((void **)p, n * sizeof(T) + 16);
}

NetLayers layer_map(voldor_net *nt)
{
    NetLayers nl;
    for (int k = 0; k < 6; ++k) {
        nl.L[k].off = nt->off[k];
        nl.L[k].CO = nt->CO[k];
        nl.L[k].MT = nt->CO[k] / 16;
        nl.L[k].wf = nt->wf[k];
        nl.L[k].wb = k > 0 ? nt->wb[k] : nullptr;
    }
    return nl;
}

int adam_launch(voldor_net *nt, int update, float lr, hipStream_t s)
{
    AdamArgs a;
    a.p = nt->p;
    a.m = nt->m;
    a.v = nt->v;
    a.g = nt->g;
    a.n = nt->n_params;
    a.lr = lr;
    a.b1 = 0.9f;
    a.b2 = 0.999f;
    a.eps = 1e-8f;
    a.o1 = (float)(1.0 - 0.9);
    a.o2 = (float)(1.0 - 0.999);
    a.c1 = (float)(1.0 - pow(0.9, nt->step));
    a.c2 = (float)(1.0 - pow(0.999, nt->step));
    a.update = update;
    hipLaunchKernelGGL(k_net_adam, dim3((nt->n_params + 255) / 256), dim3(256), 0, s, a, layer_map(nt));
    return hipGetLastError() == hipSuccess ? 0 : VOLDOR_EDEVICE;
}

bool net_dims_ok(const voldor_net *nt, int N, int H, int W)
{
    return nt && N >= 1 && N <= nt->N_max && H >= 3 && W >= 3 && H <= nt->H_max && W <= nt->W_max;
}

int conv_launch(int mode, int MT, const __bf16 *in, const __bf16 *w, const float *bias, const __bf16 *mask,
                void *out, int N, int H, int W, hipStream_t s)
{
    ConvArgs a;
    a.in = in;
    a.w = w;
    a.bias = bias;
    a.mask = mask;
    a.out = out;
    a.N = N;
    a.H = H;
    a.W = W;
    a.tiles = N * H * ((W + 15) / 16);
    int blocks = (a.tiles + 3) / 4;
    if (blocks > 2048) blocks = 2048;   // each wave keeps its weights over several tiles
    if (mode == kConvRelu && MT == 2) hipLaunchKernelGGL((k_conv<kConvRelu, 2>), dim3(blocks), dim3(256), 0, s, a);
    else if (mode == kConvLinearF32 && MT == 1)
        hipLaunchKernelGGL((k_conv<kConvLinearF32, 1>), dim3(blocks), dim3(256), 0, s, a);
    else if (mode == kConvMasked && MT == 2)
        hipLaunchKernelGGL((k_conv<kConvMasked, 2>), dim3(blocks), dim3(256), 0, s, a);
    else
        return VOLDOR_EINVAL;
    return hipGetLastError() == hipSuccess ? 0 : VOLDOR_EDEVICE;
}

// the forward pass for inference: the input channels, then all six layers in
// one launch with the activations in LDS (k_net_fused)
int forward_fused_launch(voldor_net *nt, const float *flows, int N, int H, int W, hipStream_t s)
{
    const int64_t npx = (int64_t)N * H * W;
    hipLaunchKernelGGL(k_net_input, dim3((unsigned)((npx + 255) / 256)), dim3(256), 0, s, (const float2 *)flows,
                       nt->act[0], N, nt->T, H, W, 1.0f / 16.0f);
    FusedArgs a;
    a.x = nt->act[0];
    for (int k = 0; k < 6; ++k) {
        a.w[k] = nt->wf[k];
        a.b[k] = nt->p + nt->off[k] + 9 * kNetC * nt->CO[k];
    }
    a.z = nt->z;
    a.N = N;
    a.H = H;
    a.W = W;
    a.tiles_x = (W + kFuseTW - 1) / kFuseTW;
    a.tiles_y = (H + kFuseTH - 1) / kFuseTH;
    const size_t lds = sizeof(__bf16) * (size_t)(kFuseBufA + kFuseBufB);
    if (hipFuncSetAttribute((const void *)k_net_fused, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds) !=
        hipSuccess)
        return VOLDOR_EDEVICE;
    hipLaunchKernelGGL(k_net_fused, dim3((unsigned)(N * a.tiles_x * a.tiles_y)), dim3(kFuseThreads), lds, s, a);
    return hipGetLastError() == hipSuccess ? 0 : VOLDOR_EDEVICE;
}

int forward_launch(voldor_net *nt, const float *flows, int N, int H, int W, hipStream_t s)
{
    const int64_t npx = (int64_t)N * H * W;
    hipLaunchKernelGGL(k_net_input, dim3((unsigned)((npx + 255) / 256)), dim3(256), 0, s, (const float2 *)flows,
                       nt->act[0], N, nt->T, H, W, 1.0f / 16.0f);
    int rc = hipGetLastError() == hipSuccess ? 0 : VOLDOR_EDEVICE;
    for (int k = 0; k < 5 && rc == 0; ++k)
        rc = conv_launch(kConvRelu, 2, nt->act[k], nt->wf[k], nt->p + nt->off[k] + 9 * kNetC * nt->CO[k], nullptr,
                         nt->act[k + 1], N, H, W, s);
    if (rc == 0)
        rc = conv_launch(kConvLinearF32, 1, nt->act[5], nt->wf[5], nt->p + nt->off[5] + 9 * kNetC * nt->CO[5],
                         nullptr, nt->z, N, H, W, s);
    return rc;
}

int wgrad_launch(voldor_net *nt, int k, const __bf16 *dy, int N, int H, int W, hipStream_t s)
{
    WgradArgs a;
    a.x = nt->act[k];
    a.dy = dy;
    a.part = nt->part;
    a.pbias = nt->pbias;
    a.N = N;
    a.H = H;
    a.W = W;
    a.segs = N * H * ((W + 31) / 32);
    const int blocks = a.segs < kWgradBlocks ? a.segs : kWgradBlocks;
    hipLaunchKernelGGL(k_conv_wgrad, dim3(blocks), dim3(256), 0, s, a);
    const int ne = 9 * kNetC * nt->CO[k] + nt->CO[k];
    hipLaunchKernelGGL(k_wgrad_reduce, dim3((ne + 255) / 256), dim3(256), 0, s, nt->part, nt->pbias, blocks,
                       nt->CO[k], nt->g + nt->off[k]);
    return hipGetLastError() == hipSuccess ? 0 : VOLDOR_EDEVICE;
}

// forward, loss and backward: nt->g holds the gradient, *loss_out the loss
int grad_launch(voldor_net *nt, const float *flows, int N, int H, int W, const float *depth, const float *rig,
                double *loss_out, hipStream_t s)
{
    int rc = forward_launch(nt, flows, N, H, W, s);
    if (rc) return rc;
    LossArgs la;
    la.z = nt->z;
    la.depth = depth;
    la.rig = rig;
    la.dz = nt->gbuf[0];
    la.part = nt->lpart;
    la.N = N;
    la.T = nt->T;
    la.H = H;
    la.W = W;
    hipLaunchKernelGGL(k_net_loss, dim3(kLossBlocks), dim3(256), 0, s, la);
    if (loss_out) hipLaunchKernelGGL(k_net_loss_reduce, dim3(1), dim3(64), 0, s, nt->lpart, kLossBlocks, loss_out);
    if (hipGetLastError() != hipSuccess) return VOLDOR_EDEVICE;
    int cur = 0;
    for (int k = 5; k >= 0 && rc == 0; --k) {
        rc = wgrad_launch(nt, k, nt->gbuf[cur], N, H, W, s);
        if (rc == 0 && k > 0) {
            rc = conv_launch(kConvMasked, 2, nt->gbuf[cur], nt->wb[k], nullptr, nt->act[k], nt->gbuf[cur ^ 1], N, H,
                             W, s);
            cur ^= 1;
        }
    }
    return rc;
}

}  // namespace

extern "C" {

int voldor_net_create(voldor_net **out, int T, int N_max, int H_max, int W_max)
{
    if (!out) return VOLDOR_EINVAL;
    *out = nullptr;
    if (T < 1 || T > 8 || N_max < 1 || H_max < 3 || W_max < 3 || H_max > 4096 || W_max > 4096 ||
        (int64_t)N_max * H_max * W_max > (1ll << 26))
        return VOLDOR_EINVAL;
    voldor_net *nt = (voldor_net *)calloc(1, sizeof(voldor_net));
    if (!nt) return VOLDOR_ENOMEM;
    nt->T = T;
    nt->N_max = N_max;
    nt->H_max = H_max;
    nt->W_max = W_max;
    int off = 0;
    for (int k = 0; k < 6; ++k) {
        nt->off[k] = off;
        nt->CO[k] = k == 5 ? kNetCo6 : kNetC;
        off += 9 * kNetC * nt->CO[k] + nt->CO[k];
    }
    nt->off[6] = off;
    nt->n_params = off;
    const size_t npx = (size_t)N_max * H_max * W_max;
    bool ok = nalloc(&nt->p, off) == hipSuccess && nalloc(&nt->m, off) == hipSuccess &&
              nalloc(&nt->v, off) == hipSuccess && nalloc(&nt->g, off) == hipSuccess;
    for (int k = 0; k < 6 && ok; ++k) {
        ok = nalloc(&nt->wf[k], (size_t)9 * 32 * kNetC) == hipSuccess &&
             nalloc(&nt->wb[k], (size_t)9 * kNetC * kNetC) == hipSuccess &&
             nalloc(&nt->act[k], npx * kNetC) == hipSuccess;
    }
    ok = ok && nalloc(&nt->z, npx * kNetCo6) == hipSuccess;
    ok = ok && nalloc(&nt->gbuf[0], npx * kNetC) == hipSuccess && nalloc(&nt->gbuf[1], npx * kNetC) == hipSuccess;
    ok = ok && nalloc(&nt->part, (size_t)kWgradBlocks * 9 * kNetC * kNetC) == hipSuccess;
    ok = ok && nalloc(&nt->pbias, (size_t)kWgradBlocks * kNetC) == hipSuccess;
    ok = ok && nalloc(&nt->lpart, kLossBlocks) == hipSuccess;
    if (!ok) {
        voldor_net_destroy(nt);
        return VOLDOR_ENOMEM;
    }
    // zero everything that is read before written: padded weight rows, moments
    bool z = hipMemset(nt->m, 0, sizeof(float) * off) == hipSuccess &&
             hipMemset(nt->v, 0, sizeof(float) * off) == hipSuccess &&
             hipMemset(nt->p, 0, sizeof(float) * off) == hipSuccess;
    for (int k = 0; k < 6 && z; ++k)
        z = hipMemset(nt->wf[k], 0, sizeof(__bf16) * 9 * 32 * kNetC) == hipSuccess &&
            hipMemset(nt->wb[k], 0, sizeof(__bf16) * 9 * kNetC * kNetC) == hipSuccess;
    if (!z || hipDeviceSynchronize() != hipSuccess) {
        voldor_net_destroy(nt);
        return VOLDOR_EDEVICE;
    }
    *out = nt;
    return VOLDOR_OK;
}

void voldor_net_destroy(voldor_net *nt)
{
    if (!nt) return;
    void *bufs[] = {nt->p, nt->m, nt->v, nt->g, nt->z, nt->gbuf[0], nt->gbuf[1], nt->part, nt->pbias, nt->lpart};
    for (void *b : bufs)
        if (b) (void)hipFree(b);
    for (int k = 0; k < 6; ++k) {
        if (nt->wf[k]) (void)hipFree(nt->wf[k]);
        if (nt->wb[k]) (void)hipFree(nt->wb[k]);
        if (nt->act[k]) (void)hipFree(nt->act[k]);
    }
    free(nt);
}

int voldor_net_param_count(const voldor_net *nt)
{
    return nt ? nt->n_params : VOLDOR_EINVAL;
}

int voldor_net_set_params(voldor_net *nt, const float *host_params)
{
    if (!nt || !host_params) return VOLDOR_EINVAL;
    if (hipMemcpy(nt->p, host_params, sizeof(float) * nt->n_params, hipMemcpyHostToDevice) != hipSuccess ||
        hipMemset(nt->m, 0, sizeof(float) * nt->n_params) != hipSuccess ||
        hipMemset(nt->v, 0, sizeof(float) * nt->n_params) != hipSuccess)
        return VOLDOR_EDEVICE;
    nt->step = 0;
    if (adam_launch(nt, 0, 0.0f, nullptr) != 0) return VOLDOR_EDEVICE;
    return hipDeviceSynchronize() == hipSuccess ? VOLDOR_OK : VOLDOR_EDEVICE;
}

int voldor_net_get_params(voldor_net *nt, float *host_params)
{
    if (!nt || !host_params) return VOLDOR_EINVAL;
    if (hipDeviceSynchronize() != hipSuccess) return VOLDOR_EDEVICE;
    return hipMemcpy(host_params, nt->p, sizeof(float) * nt->n_params, hipMemcpyDeviceToHost) == hipSuccess
               ? VOLDOR_OK
               : VOLDOR_EDEVICE;
}

int voldor_net_forward(voldor_net *nt, const float *flows, int N, int H, int W, float *depth, float *rig,
                       float *z_out, void *stream)
{
    if (!flows || !net_dims_ok(nt, N, H, W) || ((uintptr_t)flows & 7) != 0) return VOLDOR_EINVAL;
    hipStream_t s = (hipStream_t)stream;
    int rc = forward_fused_launch(nt, flows, N, H, W, s);
    const int64_t npx = (int64_t)N * H * W;
    if (rc == 0 && (depth || rig)) {
        hipLaunchKernelGGL(k_net_outputs, dim3((unsigned)((npx + 255) / 256)), dim3(256), 0, s, nt->z, depth, rig, N,
                           nt->T, H, W);
        rc = hipGetLastError() == hipSuccess ? 0 : VOLDOR_EDEVICE;
    }
    if (rc == 0 && z_out &&
        hipMemcpyAsync(z_out, nt->z, sizeof(float) * npx * kNetCo6, hipMemcpyDeviceToDevice, s) != hipSuccess)
        rc = VOLDOR_EDEVICE;
    return rc;
}

int voldor_net_gradient(voldor_net *nt, const float *flows, int N, int H, int W, const float *depth, const float *rig,
                        double *loss_out, float *grad_out, void *stream)
{
    if (!flows || !depth || !rig || !net_dims_ok(nt, N, H, W) || ((uintptr_t)flows & 7) != 0) return VOLDOR_EINVAL;
    hipStream_t s = (hipStream_t)stream;
    int rc = grad_launch(nt, flows, N, H, W, depth, rig, loss_out, s);
    if (rc == 0 && grad_out &&
        hipMemcpyAsync(grad_out, nt->g, sizeof(float) * nt->n_params, hipMemcpyDeviceToDevice, s) != hipSuccess)
        rc = VOLDOR_EDEVICE;
    return rc;
}

int voldor_net_train_step(voldor_net *nt, const float *flows, int N, int H, int W, const float *depth,
                          const float *rig, float lr, double *loss_out, void *stream)
{
    if (!flows || !depth || !rig || !net_dims_ok(nt, N, H, W) || ((uintptr_t)flows & 7) != 0 || !(lr > 0.0f))
        return VOLDOR_EINVAL;
    hipStream_t s = (hipStream_t)stream;
    int rc = grad_launch(nt, flows, N, H, W, depth, rig, loss_out, s);
    if (rc == 0) {
        ++nt->step;
        rc = adam_launch(nt, 1, lr, s);
    }
    return rc;
}

int voldor_net_layer(voldor_net *nt, int k, int backward, const void *in, const void *mask, void *out, int N, int H,
                     int W, void *stream)
{
    if (!net_dims_ok(nt, N, H, W) || k < 0 || k > 5 || !in || !out) return VOLDOR_EINVAL;
    hipStream_t s = (hipStream_t)stream;
    if (!backward) {
        const float *bias = nt->p + nt->off[k] + 9 * kNetC * nt->CO[k];
        return k < 5 ? conv_launch(kConvRelu, 2, (const __bf16 *)in, nt->wf[k], bias, nullptr, out, N, H, W, s)
                     : conv_launch(kConvLinearF32, 1, (const __bf16 *)in, nt->wf[k], bias, nullptr, out, N, H, W, s);
    }
    if (k == 0 || !mask) return VOLDOR_EINVAL;
    return conv_launch(kConvMasked, 2, (const __bf16 *)in, nt->wb[k], nullptr, (const __bf16 *)mask, out, N, H, W, s);
}

}  // extern "C"
