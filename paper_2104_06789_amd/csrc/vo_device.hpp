// vo_device.hpp -- device-side building blocks of the gfx950 window solver.
//
// Philox4x64-10 counters, the FP32 emission of Eq. 1-8 (projection, bilinear
// flow lookup, Fisk log-densities in log form), FP64 3x3 algebra, SE(3)
// exp/log and the P3P solver used by the pose step.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace vo {

constexpr int kTMax = 16;          // frames per window

enum : uint64_t { kDepthStream = 1, kPoseStream = 2, kBootStream = 3 };

// ---------------------------------------------------------------------------
// Philox4x64-10 (Salmon, Moraes, Dror, Shaw, SC'11): 10 rounds of two
// 64x64->128 multiplies with a Weyl-sequence key schedule.
// ---------------------------------------------------------------------------
__device__ __forceinline__ void philox4x64_10(uint64_t c[4], uint64_t k0, uint64_t k1)
{
    const uint64_t m0 = 0xD2E7470EE14C6C93ull, m1 = 0xCA5A826395121157ull;
    const uint64_t w0 = 0x9E3779B97F4A7C15ull, w1 = 0xBB67AE8584CAA73Bull;
#pragma unroll
    for (int r = 0; r < 10; ++r) {
        const uint64_t h0 = __umul64hi(m0, c[0]), l0 = m0 * c[0];
        const uint64_t h1 = __umul64hi(m1, c[2]), l1 = m1 * c[2];
        const uint64_t n0 = h1 ^ c[1] ^ k0;
        const uint64_t n2 = h0 ^ c[3] ^ k1;
        c[0] = n0;
        c[1] = l1;
        c[2] = n2;
        c[3] = l0;
        k0 += w0;
        k1 += w1;
    }
}

// index in [0, n) from a 32-bit uniform word
__device__ __forceinline__ int64_t u32_to_index(uint32_t u, int64_t n)
{
    return (int64_t)(((uint64_t)u * (uint64_t)n) >> 32);
}

// ---------------------------------------------------------------------------
// FP32 frame data: cumulative pose M_t = (R, t) stored as D = R - I and t so
// that pixel displacements avoid the cancellation of pi_t - pixel.
// ---------------------------------------------------------------------------
struct FrameF {
    float D[9];
    float t[3];
};

struct EmisParams {
    float fx, fy, cx, cy;
    float log_a1, a2, b1, b2;
    float lam2, beta_min, x_floor;
    int model;                    // residual model: 0 Fisk (Eq. 5), 1 Gaussian flow error
    float ifx, ify;               // 1/fx, 1/fy
    float l2a1, a2l;              // log2 a1, a2 / ln 2: log2 alpha = a2l |v| + l2a1
};

// A pointer that a kernel reads from device memory (the argument arrays of the
// batched launches) is generic to the compiler, which then accesses memory
// through it with flat instructions.  Those count on the LDS wait counter as
// well, so every wait for an LDS result also waits for the loads from memory
// in flight.  Passing it through the global address space lets the compiler
// use global instructions.  Only for pointers into device memory, with one
// value across the workgroup (they sit in scalar registers).
template <class T>
__device__ __forceinline__ T *global_ptr(T *p)
{
    __attribute__((address_space(1))) T *g = (__attribute__((address_space(1))) T *)p;
    asm("" : "+s"(g));   // keeps the two casts from folding into none
    return (T *)g;
}

// hardware reciprocal (v_rcp_f32, about 1 ulp) instead of an IEEE division
__device__ __forceinline__ float frcp(float x) { return __builtin_amdgcn_rcpf(x); }

// The depth-independent part of the displacement of a frame-0 pixel with
// normalised coordinates (xh, yh) in frame f: with P = M (th r),
// pi(th) - (x, y) = (fx (th ax + bx), fy (th ay + by)) / (th az + tz).
struct Geo {
    float ax, ay, az, bx, by, tz;
};

__device__ __forceinline__ Geo pixel_geometry(const FrameF &f, float xh, float yh)
{
    const float e0 = fmaf(f.D[0], xh, fmaf(f.D[1], yh, f.D[2]));
    const float e1 = fmaf(f.D[3], xh, fmaf(f.D[4], yh, f.D[5]));
    const float e2 = fmaf(f.D[6], xh, fmaf(f.D[7], yh, f.D[8]));
    Geo g;
    g.ax = fmaf(-xh, e2, e0);
    g.ay = fmaf(-yh, e2, e1);
    g.az = 1.0f + e2;
    g.bx = fmaf(-xh, f.t[2], f.t[0]);
    g.by = fmaf(-yh, f.t[2], f.t[1]);
    g.tz = f.t[2];
    return g;
}

// the displacement at depth th; false if the point is not in front
__device__ __forceinline__ bool displacement_at(const Geo &g, float th, float fx, float fy, float &dx, float &dy)
{
    const float pz = fmaf(th, g.az, g.tz);
    if (!(pz > 0.0f)) return false;
    const float inv = frcp(pz);
    dx = fx * fmaf(th, g.ax, g.bx) * inv;
    dy = fy * fmaf(th, g.ay, g.by) * inv;
    return true;
}

// The same without a branch: dx, dy are written whatever pz is (not finite
// or meaningless behind the camera) and the result says whether the point is
// in front.  For callers that mask the values they use; with the same
// arithmetic, the in-front values equal displacement_at's bit for bit.
__device__ __forceinline__ bool displacement_any(const Geo &g, float th, float fx, float fy, float &dx, float &dy)
{
    const float pz = fmaf(th, g.az, g.tz);
    const float inv = frcp(pz);
    dx = fx * fmaf(th, g.ax, g.bx) * inv;
    dy = fy * fmaf(th, g.ay, g.by) * inv;
    return pz > 0.0f;
}

// a + b and a - b never fused with a product that feeds them.  Which product
// the compiler would fuse depends on the code around the expression, so the
// kernels that evaluate the same emission (the sweep's passes, the rigidness
// pass, the pose step) would round it differently; these sums keep every
// kernel on one FP32 function of its inputs.
__device__ __forceinline__ float add_nc(float a, float b)
{
#pragma clang fp contract(off)
    return a + b;
}

__device__ __forceinline__ float sub_nc(float a, float b)
{
#pragma clang fp contract(off)
    return a - b;
}

// Displacement pi_t(theta) - (x, y) of the frame-0 pixel with normalised
// coordinates (xh, yh) at depth th.  False if the point is not in front.
__device__ __forceinline__ bool displacement(const FrameF &f, float xh, float yh, float th,
                                             float fx, float fy, float &dx, float &dy)
{
    return displacement_at(pixel_geometry(f, xh, yh), th, fx, fy, dx, dy);
}

// Natural log / exp on the hardware base-2 units (v_log_f32, v_exp_f32):
// arguments here are normal positive numbers (logs) or bounded (exps), so no
// denormal fix-ups are needed; results within a few ulp.
__device__ __forceinline__ float fast_log(float x) { return __builtin_amdgcn_logf(x) * 0.69314718055994531f; }
__device__ __forceinline__ float fast_exp(float x) { return __builtin_amdgcn_exp2f(x * 1.4426950408889634f); }

// log(1 + e) for e in [0, 1] on the hardware log2 unit, to an absolute error of
// half an ulp of 1 (6e-8): the rounding of u = 1 + e.  Enough inside the
// log-odds d, whose other terms carry errors of that size.
__device__ __forceinline__ float log1p_unit(float e) { return fast_log(1.0f + e); }

// The same to a relative error of a few ulp, given u = 1 + e rounded and its
// reciprocal: log(1 + e) = log u - log(u / (1 + e)), and u / (1 + e) = 1 + dl / u
// with dl = (u - 1) - e exact in FP32 (|dl| <= 2^-24), so the correction is
// dl / u to first order.  For well-fitting candidates ell = -log(1 + e^d) is
// tiny, and the M-step ranks them by it: there its absolute error must scale
// with its size.
__device__ __forceinline__ float log1p_rel(float e, float u, float inv_u)
{
    return fmaf(-((u - 1.0f) - e), inv_u, fast_log(u));
}

__device__ __forceinline__ float softplus(float z)
{
    return add_nc(fmaxf(z, 0.0f), log1p_unit(fast_exp(-fabsf(z))));
}

// taps_finite: all four taps of a bilinear lookup are finite iff the
// interpolated u + v is.  Each tap component enters u (or v) through
// w a + (1 - w) b forms evaluated as fma(w, b - a, a) and sums: a NaN tap
// propagates, and an infinite one gives +-inf where its weight is nonzero and
// inf - inf or 0 * inf = NaN where it is zero, whatever the weights; finite
// taps (flows far below 1e38) give finite u and v.  So the kernels test the
// interpolated values instead of the eight taps.

// Bilinear interpolation of taps a (x0, y0), b (x0 + 1, y0), c (x0, y0 + 1),
// d (x0 + 1, y0 + 1) at fractions (ax, ay).  The fused multiply-adds are
// written out, so that no kernel is left a choice of which product to fuse:
// every kernel evaluates the same FP32 function.
__device__ __forceinline__ float bilerp(float a, float b, float c, float d, float ax, float ay)
{
    const float top = fmaf(ax, b - a, a), bot = fmaf(ax, d - c, c);
    return fmaf(ay, bot, (1.0f - ay) * top);
}

// Bilinear sample of flow X (one frame, float2 [H][W]) at (px, py).
// Domain [0, W-1] x [0, H-1]; all four taps must be finite.
__device__ __forceinline__ bool sample_flow(const float2 *__restrict__ X, int H, int W, float px,
                                            float py, float &u, float &v)
{
    if (!(px >= 0.0f && px <= (float)(W - 1) && py >= 0.0f && py <= (float)(H - 1))) return false;
    int x0 = (int)floorf(px), y0 = (int)floorf(py);
    x0 = min(x0, W - 2);
    y0 = min(y0, H - 2);
    const float ax = px - (float)x0, ay = py - (float)y0;
    const float2 *row0 = X + (size_t)y0 * W + x0;
    const float2 *row1 = row0 + W;
    const float2 a = row0[0], b = row0[1], c = row1[0], d = row1[1];
    u = bilerp(a.x, b.x, c.x, d.x, ax, ay);
    v = bilerp(a.y, b.y, c.y, d.y, ax, ay);
    return isfinite(a.x + a.y + b.x + b.y + c.x + c.y + d.x + d.y);
}

struct Emis {
    float ell;  // log r
    float r;    // rho / (rho + mu)
};

// Emission given the residual (rx, ry) = xi - v and the observed flow v:
// d = log(mu / rho) with the densities of Eq. 4 and Eq. 8 sharing
// log(alpha) = log a1 + a2 |v|.
// MODEL 0, Fisk (Eq. 5) with beta = max(b1 |v| + b2, beta_min): the common
// log(beta) - log(alpha) term cancels in the ratio.
// MODEL 1, Gaussian flow error: the squared EPE is exponential with mean
// s = alpha / ln 2 (the Fisk's median alpha), so d = (x - m) / s for the
// squared residual x and the Eq. 8 argument m = lambda^2 |v|^2.
constexpr float kLn2F = 0.69314718055994531f;
constexpr float kLogLn2F = -0.36651292058166432f;   // log(ln 2)

// The sweep and the rigidness pass take the log-odds in base 2,
// D = d / ln 2 = log2(mu / rho): the hardware units are log2 and exp2, so
// neither scales between the two bases inside the emission (with alpha in
// base 2, la = log2 alpha = a2 |v| / ln 2 + log2 a1).
// softplus2(z) = log2(1 + 2^z), the base-2 form of softplus.
__device__ __forceinline__ float softplus2(float z)
{
    return add_nc(fmaxf(z, 0.0f), __builtin_amdgcn_logf(1.0f + __builtin_amdgcn_exp2f(-fabsf(z))));
}

template <int MODEL = 0>
__device__ __forceinline__ float log2_odds(float rx, float ry, float vx, float vy, const EmisParams &e)
{
    // squared residual clamped to [x_floor, 1e30] so every exponent below stays finite
    const float x2 = fminf(fmaxf(fmaf(rx, rx, ry * ry), e.x_floor), 1e30f);
    const float vn2 = fmaf(vx, vx, vy * vy);
    const float vn = __builtin_amdgcn_sqrtf(vn2);
    const float la = fmaf(e.a2l, vn, e.l2a1);
    if constexpr (MODEL == 1) {
        // d = (x - m) ln 2 / alpha, so D = (x - m) / alpha
        const float m = fmaxf(e.lam2 * vn2, e.x_floor);
        return (x2 - m) * __builtin_amdgcn_exp2f(-la);
    } else {
        const float beta = fmaxf(fmaf(e.b1, vn, e.b2), e.beta_min);
        const float lx = __builtin_amdgcn_logf(x2);
        const float lm = __builtin_amdgcn_logf(fmaxf(e.lam2 * vn2, e.x_floor));
        const float z1 = beta * sub_nc(lx, la), z2 = beta * sub_nc(lm, la);
        return fmaf(beta - 1.0f, sub_nc(lm, lx), -2.0f * (softplus2(z2) - softplus2(z1)));
    }
}

// The same D, and log mu itself (natural log; Eq. 8: the model's density at
// squared EPE lambda^2 |v|^2, normalisation included), for the
// maximum-likelihood depth criterion (Eq. 9), whose per-frame term is
// q log rho + (1 - q) log mu = log mu - q d.
template <int MODEL = 0>
__device__ __forceinline__ float log2_odds_mu(float rx, float ry, float vx, float vy, const EmisParams &e,
                                              float &lmu)
{
    const float x2 = fminf(fmaxf(fmaf(rx, rx, ry * ry), e.x_floor), 1e30f);
    const float vn2 = fmaf(vx, vx, vy * vy);
    const float vn = __builtin_amdgcn_sqrtf(vn2);
    const float la = fmaf(e.a2l, vn, e.l2a1);
    if constexpr (MODEL == 1) {
        const float m = fmaxf(e.lam2 * vn2, e.x_floor);
        const float ia = __builtin_amdgcn_exp2f(-la);   // 1 / alpha = (1 / s) / ln 2
        lmu = fmaf(kLn2F, fmaf(-m, ia, -la), kLogLn2F);   // -m / s - log s
        return (x2 - m) * ia;
    } else {
        const float beta = fmaxf(fmaf(e.b1, vn, e.b2), e.beta_min);
        const float lx = __builtin_amdgcn_logf(x2);
        const float lm = __builtin_amdgcn_logf(fmaxf(e.lam2 * vn2, e.x_floor));
        const float z1 = beta * sub_nc(lx, la), z2 = beta * sub_nc(lm, la);
        lmu = kLn2F * (fmaf(beta - 1.0f, sub_nc(lm, la), sub_nc(__builtin_amdgcn_logf(beta), la)) - 2.0f * softplus2(z2));
        return fmaf(beta - 1.0f, sub_nc(lm, lx), -2.0f * (softplus2(z2) - softplus2(z1)));
    }
}

// r = 1 / (1 + e^d), 0 below the smallest normal FP32 number (whatever the
// denormal mode of the exponential: d > 87.3), and
// ell = log r = -(max(d, 0) + log(1 + e^-|d|))
constexpr float kFltMin = 1.17549435e-38f;
__device__ __forceinline__ float posterior_from(float d, float e, float inv)
{
    const float r = d < 0.0f ? inv : e * inv;
    return r >= kFltMin ? r : 0.0f;
}

__device__ __forceinline__ Emis emis_from_d(float d)
{
    const float e = fast_exp(-fabsf(d));
    const float u = 1.0f + e;
    const float inv = frcp(u);
    Emis o;
    o.ell = -(fmaxf(d, 0.0f) + log1p_rel(e, u, inv));
    o.r = posterior_from(d, e, inv);
    return o;
}

// The same from the base-2 log-odds D: e = 2^-|D| = e^-|d|, and
// log(1 + e) = ln 2 log2 u - ((u - 1) - e) / u with u = 1 + e rounded, so
// ell = ((u - 1) - e) / u - ln 2 (max(D, 0) + log2 u).
__device__ __forceinline__ Emis emis_from_D(float D)
{
    const float e = __builtin_amdgcn_exp2f(-fabsf(D));
    const float u = 1.0f + e;
    const float inv = frcp(u);
    Emis o;
    o.ell = fmaf((u - 1.0f) - e, inv, -kLn2F * (fmaxf(D, 0.0f) + __builtin_amdgcn_logf(u)));
    o.r = posterior_from(D, e, inv);
    return o;
}

// log(-ell) = log(log(1 + e^d)) from D, the log of the negated per-frame MIE
// term, for the scores kept in log form (below).  For d < -8, log(1 + e^d) =
// e^d (1 - e^d / 2 + ...), so log(-ell) = d - e^d / 2 to within 2e-8; above,
// the log of -ell itself (then at least 3e-4, so relative accuracy holds).
// Also returns r = 1 / (1 + e^d).
constexpr float kLog2Minus8F = -11.541560327111707f;   // -8 / ln 2
__device__ __forceinline__ float neg_ell_log2(float D, float &r)
{
    const float e = __builtin_amdgcn_exp2f(-fabsf(D));
    const float u = 1.0f + e;
    const float inv = frcp(u);
    r = posterior_from(D, e, inv);
    const float nl = fmaf(-((u - 1.0f) - e), inv, kLn2F * (fmaxf(D, 0.0f) + __builtin_amdgcn_logf(u)));
    return D < kLog2Minus8F ? fmaf(-0.5f, e, D * kLn2F) : fast_log(nl);
}

// A maximum-inlier score S = sum_t q_t ell_t (Eq. 10) kept as
// -log(-S) = -log(sum_t e^{v_t}), v_t = log q_t + log(-ell_t), by a running
// log-sum-exp: (m, a) with sum = e^m a, m the largest v_t so far.  The map
// S -> -log(-S) is increasing, so scores compare as before, but the terms of
// well-fitting candidates do not underflow: with the Gaussian residual model
// ell = -e^d reaches e^-100, below the FP32 range, where a linear FP32 sum
// would make every such candidate tie at 0.  Terms with q_t = 0 add nothing;
// all q_t = 0 gives +inf (S = 0, the maximum).  Terms with q_t below the
// smallest normal FP32 number are dropped as 0.
struct LogScore {
    float m, a;
};

__device__ __forceinline__ LogScore logscore_init()
{
    LogScore s;
    s.m = -INFINITY;
    s.a = 0.0f;
    return s;
}

__device__ __forceinline__ void logscore_add(LogScore &s, float q, float lam)
{
    if (!(q >= kFltMin)) return;   // (a subnormal q's log could be -inf)
    const float v = lam + fast_log(q);
    const float dd = v - s.m;
    const float e = fast_exp(-fabsf(dd));
    if (dd > 0.0f) {
        s.a = fmaf(s.a, e, 1.0f);
        s.m = v;
    } else {
        s.a += e;
    }
}

__device__ __forceinline__ float logscore_value(const LogScore &s) { return -(s.m + fast_log(s.a)); }

// ---------------------------------------------------------------------------
// FP64 helpers
// ---------------------------------------------------------------------------

// e^x for x <= 0 (Gaussian kernel weights).  Range reduction x = n ln2 + r
// with ln2 split into a 31-bit head (n * head exact for |n| <= 1022) and a
// tail, |r| <= ln2/2; e^r by its Taylor series to degree 11 (truncation
// error below 7e-15 relative); 2^n assembled from the exponent bits.
__device__ __forceinline__ double exp_nonpos(double x)
{
    if (!(x > -708.0)) return 0.0;
    const double n = rint(x * 1.4426950408889634);
    const double r = fma(-n, 1.9082149292705877e-10, fma(-n, 0.6931471803691238, x));
    double p = 1.0 / 39916800.0;
    p = fma(p, r, 1.0 / 3628800.0);
    p = fma(p, r, 1.0 / 362880.0);
    p = fma(p, r, 1.0 / 40320.0);
    p = fma(p, r, 1.0 / 5040.0);
    p = fma(p, r, 1.0 / 720.0);
    p = fma(p, r, 1.0 / 120.0);
    p = fma(p, r, 1.0 / 24.0);
    p = fma(p, r, 1.0 / 6.0);
    p = fma(p, r, 0.5);
    p = fma(p, r, 1.0);
    p = fma(p, r, 1.0);
    return p * __longlong_as_double((long long)((int)n + 1023) << 52);
}
struct M3 {
    double a[9];
};

__device__ __forceinline__ void mv3(const double *A, const double *x, double *y)
{
    y[0] = A[0] * x[0] + A[1] * x[1] + A[2] * x[2];
    y[1] = A[3] * x[0] + A[4] * x[1] + A[5] * x[2];
    y[2] = A[6] * x[0] + A[7] * x[1] + A[8] * x[2];
}

__device__ __forceinline__ void mm3(const double *A, const double *B, double *C)
{
    double T[9];
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
        for (int j = 0; j < 3; ++j)
            T[3 * i + j] = A[3 * i] * B[j] + A[3 * i + 1] * B[3 + j] + A[3 * i + 2] * B[6 + j];
#pragma unroll
    for (int i = 0; i < 9; ++i) C[i] = T[i];
}

__device__ __forceinline__ double dot3d(const double *a, const double *b)
{
    return a[0] * b[0] + a[1] * b[1] + a[2] * b[2];
}

__device__ __forceinline__ void cross3d(const double *a, const double *b, double *c)
{
    const double c0 = a[1] * b[2] - a[2] * b[1];
    const double c1 = a[2] * b[0] - a[0] * b[2];
    const double c2 = a[0] * b[1] - a[1] * b[0];
    c[0] = c0;
    c[1] = c1;
    c[2] = c2;
}

// compose C = A o B for 12-double poses (R row-major, t)
__device__ __forceinline__ void pose_mul(const double *A, const double *B, double *C)
{
    double R[9], t[3];
    mm3(A, B, R);
    mv3(A, B + 9, t);
    for (int k = 0; k < 3; ++k) t[k] += A[9 + k];
    for (int k = 0; k < 9; ++k) C[k] = R[k];
    for (int k = 0; k < 3; ++k) C[9 + k] = t[k];
}

// rotation angle in [0, pi]
__device__ __forceinline__ double rot_angle(const double *R)
{
    const double wx = R[7] - R[5], wy = R[2] - R[6], wz = R[3] - R[1];
    return atan2(0.5 * sqrt(wx * wx + wy * wy + wz * wz), 0.5 * (R[0] + R[4] + R[8] - 1.0));
}

// se(3) exp: p = (rho, phi) -> R, t = V rho
__device__ inline void se3_exp(const double *p, double *R, double *t)
{
    const double *w = p + 3;
    const double th2 = w[0] * w[0] + w[1] * w[1] + w[2] * w[2];
    const double th = sqrt(th2);
    double A, B, C;
    if (th < 1e-5) {
        A = 1.0 - th2 * (1.0 / 6.0) + th2 * th2 * (1.0 / 120.0);
        B = 0.5 - th2 * (1.0 / 24.0) + th2 * th2 * (1.0 / 720.0);
        C = 1.0 / 6.0 - th2 * (1.0 / 120.0) + th2 * th2 * (1.0 / 5040.0);
    } else {
        const double s = sin(th), c = cos(th);
        A = s / th;
        B = (1.0 - c) / th2;
        C = (th - s) / (th2 * th);
    }
    // W = [w]x, W^2 = w w^T - th2 I
    const double W[9] = {0, -w[2], w[1], w[2], 0, -w[0], -w[1], w[0], 0};
    double W2[9];
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) W2[3 * i + j] = w[i] * w[j] - (i == j ? th2 : 0.0);
    double V[9];
    for (int i = 0; i < 9; ++i) {
        const double I = (i == 0 || i == 4 || i == 8) ? 1.0 : 0.0;
        R[i] = I + A * W[i] + B * W2[i];
        V[i] = I + B * W[i] + C * W2[i];
    }
    mv3(V, p, t);
}

// se(3) log: R, t -> p = (V^-1 t, phi), |phi| in [0, pi]; *angle (optional)
// receives |phi|, the same number rot_angle(R) gives
__device__ inline void se3_log(const double *R, const double *t, double *p, double *angle = nullptr)
{
    const double wx = R[7] - R[5], wy = R[2] - R[6], wz = R[3] - R[1];
    const double s = 0.5 * sqrt(wx * wx + wy * wy + wz * wz);
    const double c = 0.5 * (R[0] + R[4] + R[8] - 1.0);
    const double th = atan2(s, c);
    if (angle) *angle = th;
    double phi[3];
    if (th < 1e-5) {
        const double f = 0.5 + th * th * (1.0 / 12.0);
        phi[0] = f * wx;
        phi[1] = f * wy;
        phi[2] = f * wz;
    } else if (th < 3.1405926535897931) {
        const double f = th / (2.0 * sin(th));
        phi[0] = f * wx;
        phi[1] = f * wy;
        phi[2] = f * wz;
    } else {
        // near pi: the symmetric part (R + R^T)/2 = c I + (1 - c) n n^T; the
        // largest diagonal entry gives the best-conditioned component of n
        const double oc = 1.0 - c;
        const int m = R[8] > (R[4] > R[0] ? R[4] : R[0]) ? 2 : (R[4] > R[0] ? 1 : 0);
        double n[3];
        if (m == 0) {
            n[0] = sqrt(fmax(0.0, (R[0] - c) / oc));
            n[1] = (R[1] + R[3]) / (2.0 * oc * n[0]);
            n[2] = (R[2] + R[6]) / (2.0 * oc * n[0]);
        } else if (m == 1) {
            n[1] = sqrt(fmax(0.0, (R[4] - c) / oc));
            n[0] = (R[3] + R[1]) / (2.0 * oc * n[1]);
            n[2] = (R[5] + R[7]) / (2.0 * oc * n[1]);
        } else {
            n[2] = sqrt(fmax(0.0, (R[8] - c) / oc));
            n[0] = (R[6] + R[2]) / (2.0 * oc * n[2]);
            n[1] = (R[7] + R[5]) / (2.0 * oc * n[2]);
        }
        const double nn = sqrt(n[0] * n[0] + n[1] * n[1] + n[2] * n[2]);
        double sg = (n[0] * wx + n[1] * wy + n[2] * wz) < 0 ? -1.0 : 1.0;
        for (int k = 0; k < 3; ++k) phi[k] = sg * th * n[k] / nn;
    }
    // V^-1 = I - 1/2 [phi]x + D [phi]x^2
    double Dc;
    if (th < 1e-5) {
        Dc = 1.0 / 12.0 + th * th * (1.0 / 720.0);
    } else {
        Dc = (1.0 - th * sin(th) / (2.0 * (1.0 - cos(th)))) / (th * th);
    }
    const double W[9] = {0, -phi[2], phi[1], phi[2], 0, -phi[0], -phi[1], phi[0], 0};
    const double th2 = phi[0] * phi[0] + phi[1] * phi[1] + phi[2] * phi[2];
    double Vi[9];
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) {
            const double W2 = phi[i] * phi[j] - (i == j ? th2 : 0.0);
            Vi[3 * i + j] = (i == j ? 1.0 : 0.0) - 0.5 * W[3 * i + j] + Dc * W2;
        }
    mv3(Vi, t, p);
    p[3] = phi[0];
    p[4] = phi[1];
    p[5] = phi[2];
}

// ---------------------------------------------------------------------------
// P3P.  With unknown distances s_i along unit bearings f_i and the side
// lengths of the 3-D triangle, the law of cosines gives three quadrics.  With
// u = s2/s1 and v = s3/s1, subtracting two of them yields u as a rational
// function N(v)/D(v); substituting into the third gives a quartic in v
// (Grunert's route).  The quartic factors into two quadratics (Ferrari, via
// the largest root of the resolvent cubic); root slots 0, 1 belong to the
// first factor and 2, 3 to the second, so that one lane can solve one slot.
// Each real root is polished by Newton steps, and the camera-frame triangle
// s_i f_i is aligned rigidly onto the 3-D triangle.  Everything is indexed
// statically: no private-memory arrays.
// ---------------------------------------------------------------------------
// largest real root of x^3 + a2 x^2 + a1 x + a0
__device__ inline double cubic_largest_root(double a2, double a1, double a0)
{
    const double q = (3.0 * a1 - a2 * a2) / 9.0;
    const double r = (9.0 * a2 * a1 - 27.0 * a0 - 2.0 * a2 * a2 * a2) / 54.0;
    const double disc = q * q * q + r * r;
    const double sh = a2 / 3.0;
    if (disc > 0) {
        const double sd = sqrt(disc);
        return cbrt(r + sd) + cbrt(r - sd) - sh;
    }
    if (q == 0) return -sh;
    const double mq = sqrt(-q);
    const double th = acos(fmin(1.0, fmax(-1.0, r / (mq * mq * mq))));
    // of the three trigonometric roots 2 mq cos((th + 2 pi k) / 3) - sh,
    // k = 0 is the largest for th in [0, pi]
    return 2.0 * mq * cos(th / 3.0) - sh;
}

__device__ inline double quartic_eval(const double *c, double v)
{
    return (((c[4] * v + c[3]) * v + c[2]) * v + c[1]) * v + c[0];
}

// Real root in `slot` (0..3) of c4 v^4 + ... + c0 (c4 != 0); false if that
// root of the factorisation is complex.
__device__ inline bool quartic_root_slot(const double *c, int slot, double &out)
{
    const double b = c[3] / c[4], cc = c[2] / c[4], d = c[1] / c[4], e = c[0] / c[4];
    const double b2 = b * b;
    const double p = cc - 0.375 * b2;
    const double q = d - 0.5 * b * cc + 0.125 * b2 * b;
    const double r = e - 0.25 * b * d + 0.0625 * b2 * cc - 3.0 / 256.0 * b2 * b2;
    const double sgn = (slot & 1) ? -1.0 : 1.0;
    double y = 0.0;
    bool ok = false;
    const double scale = fmax(1.0, fmax(fabs(p), sqrt(fabs(r))));
    if (fabs(q) < 1e-14 * scale * sqrt(scale)) {
        // biquadratic y^4 + p y^2 + r: y^2 = z1 (slots 0, 1) or z2 (slots 2, 3)
        const double dd = p * p - 4.0 * r;
        if (dd >= 0) {
            const double sd = sqrt(dd);
            const double z = slot < 2 ? 0.5 * (-p + sd) : 0.5 * (-p - sd);
            if (z >= 0) {
                y = sgn * sqrt(z);
                ok = true;
            }
        }
    } else {
        // resolvent m^3 + p m^2 + (p^2/4 - r) m - q^2/8 = 0, largest root (> 0)
        double m = cubic_largest_root(p, 0.25 * p * p - r, -0.125 * q * q);
        for (int it = 0; it < 2; ++it) {
            const double f = ((m + p) * m + (0.25 * p * p - r)) * m - 0.125 * q * q;
            const double df = (3.0 * m + 2.0 * p) * m + (0.25 * p * p - r);
            if (df != 0) m -= f / df;
        }
        if (m > 0) {
            const double s = sqrt(2.0 * m);
            const double k = q / (2.0 * s);
            // y^2 - s y + (p/2 + m + k) = 0 and y^2 + s y + (p/2 + m - k) = 0
            const double c1 = 0.5 * p + m + k, c2 = 0.5 * p + m - k;
            const double d1 = s * s - 4.0 * c1, d2 = s * s - 4.0 * c2;
            const double tol = -1e-12 * (s * s + 4.0 * fabs(c1) + 4.0 * fabs(c2));
            const double dq = slot < 2 ? d1 : d2;
            if (dq >= tol) {
                const double sq = sqrt(fmax(dq, 0.0));
                y = 0.5 * ((slot < 2 ? s : -s) + sgn * sq);
                ok = true;
            }
        }
    }
    if (!ok) return false;
    double v = y - 0.25 * b;
    for (int it = 0; it < 3; ++it) {  // Newton polish on the original quartic
        const double f = quartic_eval(c, v);
        const double df = ((4.0 * c[4] * v + 3.0 * c[3]) * v + 2.0 * c[2]) * v + c[1];
        if (df == 0) break;
        const double dv = f / df;
        v -= dv;
        if (fabs(dv) <= 1e-16 * fabs(v)) break;
    }
    out = v;
    return true;
}

// Newton steps on the three law-of-cosines equations in the distances
//   s2^2 + s3^2 - 2 ca s2 s3 = A2,  s1^2 + s3^2 - 2 cb s1 s3 = B2,
//   s1^2 + s2^2 - 2 cg s1 s2 = C2.
// Where two solutions give (nearly) the same v, the quartic's root carries only
// about half of the FP64 digits; the distances are refined on the equations
// themselves.  The 3x3 Newton system is solved by cofactors (Cramer), and a
// step is taken only while it lowers the residual.
__device__ inline double lc_residual(double s1, double s2, double s3, double A2, double B2, double C2,
                                     double ca, double cb, double cg, double &F0, double &F1, double &F2)
{
    F0 = fma(s2, s2, fma(s3, s3, -A2)) - 2.0 * ca * s2 * s3;
    F1 = fma(s1, s1, fma(s3, s3, -B2)) - 2.0 * cb * s1 * s3;
    F2 = fma(s1, s1, fma(s2, s2, -C2)) - 2.0 * cg * s1 * s2;
    return fabs(F0) + fabs(F1) + fabs(F2);
}

__device__ inline void refine_distances(double &s1, double &s2, double &s3, double A2, double B2, double C2,
                                        double ca, double cb, double cg)
{
    double F0, F1, F2;
    double res = lc_residual(s1, s2, s3, A2, B2, C2, ca, cb, cg, F0, F1, F2);
    for (int it = 0; it < 4 && res > 0.0; ++it) {
        // Jacobian rows: (0, j01, j02), (j10, 0, j12), (j20, j21, 0)
        const double j01 = 2.0 * (s2 - ca * s3), j02 = 2.0 * (s3 - ca * s2);
        const double j10 = 2.0 * (s1 - cb * s3), j12 = 2.0 * (s3 - cb * s1);
        const double j20 = 2.0 * (s1 - cg * s2), j21 = 2.0 * (s2 - cg * s1);
        // cofactors of the rows: c0 = r1 x r2, c1 = r2 x r0, c2 = r0 x r1
        const double c0x = -j12 * j21, c0y = j12 * j20, c0z = j10 * j21;
        const double c1x = j21 * j02, c1y = -j20 * j02, c1z = j20 * j01;
        const double c2x = j01 * j12, c2y = j02 * j10, c2z = -j01 * j10;
        const double det = j01 * c0y + j02 * c0z;   // r0 . c0
        if (!(fabs(det) > 0.0)) break;
        const double id = 1.0 / det;
        const double n1 = s1 - (F0 * c0x + F1 * c1x + F2 * c2x) * id;
        const double n2 = s2 - (F0 * c0y + F1 * c1y + F2 * c2y) * id;
        const double n3 = s3 - (F0 * c0z + F1 * c1z + F2 * c2z) * id;
        double G0, G1, G2;
        const double rn = lc_residual(n1, n2, n3, A2, B2, C2, ca, cb, cg, G0, G1, G2);
        if (!(rn < res) || !(n1 > 0.0 && n2 > 0.0 && n3 > 0.0)) break;
        s1 = n1;
        s2 = n2;
        s3 = n3;
        res = rn;
        F0 = G0;
        F1 = G1;
        F2 = G2;
    }
}

// Orthonormal frame of a triangle: columns e1 along X1->X2, e3 normal, e2 = e3 x e1.
__device__ inline void triangle_frame(const double *X1, const double *X2, const double *X3, double *F)
{
    double e1[3] = {X2[0] - X1[0], X2[1] - X1[1], X2[2] - X1[2]};
    const double d[3] = {X3[0] - X1[0], X3[1] - X1[1], X3[2] - X1[2]};
    const double n1 = sqrt(dot3d(e1, e1));
    for (int k = 0; k < 3; ++k) e1[k] /= n1;
    double e3[3];
    cross3d(e1, d, e3);
    const double n3 = sqrt(dot3d(e3, e3));
    for (int k = 0; k < 3; ++k) e3[k] /= n3;
    double e2[3];
    cross3d(e3, e1, e2);
    for (int k = 0; k < 3; ++k) {
        F[3 * k] = e1[k];
        F[3 * k + 1] = e2[k];
        F[3 * k + 2] = e3[k];
    }
}

// P: 3 points (rows) in the source frame; f: 3 unit bearings (rows) in the
// target camera.  The pose (R, t) with f_i ~ R P_i + t of quartic root slot
// `slot`; false if that root is complex, not admissible or not finite.
__device__ inline bool p3p_root(const double *P, const double *f, int slot, double *R, double *t)
{
    double s23[3], s13[3], s12[3];
    for (int k = 0; k < 3; ++k) {
        s23[k] = P[3 + k] - P[6 + k];
        s13[k] = P[k] - P[6 + k];
        s12[k] = P[k] - P[3 + k];
    }
    const double A2 = dot3d(s23, s23), B2 = dot3d(s13, s13), C2 = dot3d(s12, s12);
    if (!(A2 > 0) || !(B2 > 0) || !(C2 > 0)) return false;
    const double ca = dot3d(f + 3, f + 6), cb = dot3d(f, f + 6), cg = dot3d(f, f + 3);
    // N(v) = n2 v^2 + n1 v + n0 ; D(v) = e1 v + e0 ; Q(v) = v^2 - 2 cb v + 1
    const double K = C2 - A2;
    const double n2 = B2 + K, n1 = -2.0 * K * cb, n0 = K - B2;
    const double e1 = 2.0 * B2 * ca, e0 = -2.0 * B2 * cg;
    // quartic: B2 N^2 - 2 B2 cg N D + (B2 - C2 Q) D^2
    const double g2 = -C2, g1 = 2.0 * C2 * cb, g0 = B2 - C2;  // B2 - C2 Q
    double c[5];
    // N D is cubic; N^2 and (B2 - C2 Q) D^2 are quartic
    c[4] = B2 * n2 * n2 + g2 * e1 * e1;
    c[3] = B2 * 2.0 * n2 * n1 - 2.0 * B2 * cg * (n2 * e1) + (g1 * e1 * e1 + 2.0 * g2 * e1 * e0);
    c[2] = B2 * (n1 * n1 + 2.0 * n2 * n0) - 2.0 * B2 * cg * (n2 * e0 + n1 * e1) +
           (g0 * e1 * e1 + 2.0 * g1 * e1 * e0 + g2 * e0 * e0);
    c[1] = B2 * 2.0 * n1 * n0 - 2.0 * B2 * cg * (n1 * e0 + n0 * e1) + (2.0 * g0 * e1 * e0 + g1 * e0 * e0);
    c[0] = B2 * n0 * n0 - 2.0 * B2 * cg * (n0 * e0) + g0 * e0 * e0;
    if (c[4] == 0) return false;
    double v;
    if (!quartic_root_slot(c, slot, v)) return false;
    const double D = e1 * v + e0, Q = (v - 2.0 * cb) * v + 1.0;
    if (!(v > 0) || fabs(D) < 1e-14 * B2 || !(Q > 0)) return false;
    const double u = ((n2 * v + n1) * v + n0) / D;
    if (!(u > 0)) return false;
    double s1 = sqrt(B2 / Q), s2 = u * s1, s3 = v * s1;
    refine_distances(s1, s2, s3, A2, B2, C2, ca, cb, cg);
    double X[9];
    for (int k = 0; k < 3; ++k) {
        X[k] = s1 * f[k];
        X[3 + k] = s2 * f[3 + k];
        X[6 + k] = s3 * f[6 + k];
    }
    double FP[9], FX[9];
    triangle_frame(P, P + 3, P + 6, FP);
    triangle_frame(X, X + 3, X + 6, FX);
    for (int a = 0; a < 3; ++a)  // R = FX FP^T
        for (int bb = 0; bb < 3; ++bb)
            R[3 * a + bb] = FX[3 * a] * FP[3 * bb] + FX[3 * a + 1] * FP[3 * bb + 1] +
                            FX[3 * a + 2] * FP[3 * bb + 2];
    double RP[3];
    mv3(R, P, RP);
    for (int k = 0; k < 3; ++k) t[k] = X[k] - RP[k];
    bool ok = true;
    for (int k = 0; k < 9; ++k) ok = ok && isfinite(R[k]);
    for (int k = 0; k < 3; ++k) ok = ok && isfinite(t[k]);
    return ok;
}

}  // namespace vo
