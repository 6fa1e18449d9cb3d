// vo_sweep.hip -- FP32 directional sweep of the depth/rigidness update
// (E-step forward-backward, Eq. 11-14; M-step maximum-inlier sampling and
// propagation, Eq. 10 and Fig. 5), the unsmoothed rigidness with the
// log-likelihood of Eq. 3, and the Philox test kernel.
//
// One workgroup of kSweepThreads owns one chain (an image row for directions
// 0/2, a column for 1/3) for all T frames; every phase runs out of LDS:
//   A  ell_t and r_t of the previous depth and, for the maximum-inlier
//      criterion, ell_t of the random sample: one item per (position, frame)
//      evaluated at both depths, sharing the frame geometry (MLE: log-odds and
//      log mu of the previous depth; its sample follows phase B);
//   B  forward-backward per frame: one wave per frame, one chain segment per
//      lane, 2x2 transfer matrices combined by wave shuffles (prefix and
//      suffix scans), then each lane replays its segment;
//   S  MIE scores sum_t q_t ell_t of the previous depth and of the random
//      sample, the local best a_k = best(prev, sample) with its score;
//   C  for every origin k, next(k) = first j > k where a_k loses as the
//      propagated neighbour (prev > neighbour > sample on ties), found in
//      rounds over a shrinking list of live origins with a look-ahead that
//      grows as the list shrinks (the whole workgroup evaluates each round);
//   D  the propagation path 0 -> next(0) -> next(next(0)) ... by pointer
//      doubling; each position takes the local best of the last path node at
//      or before it.
// C/D give exactly the result of the serial walk along the chain: each score
// is the same FP32 function of (position, value) in every phase.
#include <algorithm>

#include "vo_internal.hpp"

namespace vo {

constexpr int kSweepThreads = 512;
#ifndef VO_PAIR_ITEMS
#define VO_PAIR_ITEMS 1
#endif
constexpr int kPairItems = VO_PAIR_ITEMS;   // items per thread in flight in the paired pass
constexpr int kMleItems = 2;                // items per thread in flight in the MLE passes
constexpr int kSweepWaves = kSweepThreads / 64;
constexpr float kLogHalf = -0.69314718055994531f;

__device__ __forceinline__ int chain_pixel(int dir, int H, int W, int c, int k)
{
    switch (dir) {
    case 0: return c * W + k;
    case 1: return k * W + c;
    case 2: return c * W + (W - 1 - k);
    default: return (H - 1 - k) * W + c;
    }
}

// FP32 frame t (R - I, t) of the FP64 cumulative pose M_t, built by threads
// 0..T of a workgroup into LDS
__device__ __forceinline__ void load_frames(const double *Mcum, int T, FrameF *fr)
{
    const int t = threadIdx.x;
    if (t <= T) {
        const double *m = Mcum + 12 * t;
        for (int i = 0; i < 9; ++i) fr[t].D[i] = (float)(m[i] - ((i == 0 || i == 4 || i == 8) ? 1.0 : 0.0));
        for (int i = 0; i < 3; ++i) fr[t].t[i] = (float)m[9 + i];
    }
}

// pixel coordinates of chain position k (no integer division)
__device__ __forceinline__ void chain_xy(int dir, int H, int W, int c, int k, int &x, int &y)
{
    x = (dir & 1) ? c : (dir == 0 ? k : W - 1 - k);
    y = (dir & 1) ? (dir == 1 ? k : H - 1 - k) : c;
}

// The four bilinear taps of frame plane f0 at (x0, y0): a (x0, y0), b (x0 + 1,
// y0), c (x0, y0 + 1), d (x0 + 1, y0 + 1).  TR: the plane is stored transposed
// ([W][H], the column sweeps' copy), where (x0, y0) and (x0, y0 + 1) are
// neighbours, so that the lanes of a column chain, consecutive in y, read
// neighbouring words; the values are the same either way.
template <bool TR>
__device__ __forceinline__ void flow_taps(const float2 *__restrict__ flows, int f0, int x0, int y0, int H, int W,
                                          float2 &a, float2 &b, float2 &c, float2 &d)
{
    if constexpr (TR) {
        const float2 *r0 = flows + (f0 + x0 * H + y0);
        a = r0[0];
        c = r0[1];
        b = r0[H];
        d = r0[H + 1];
    } else {
        const float2 *r0 = flows + (f0 + y0 * W + x0);
        a = r0[0];
        b = r0[1];
        c = r0[W];
        d = r0[W + 1];
    }
}

// Depth score at chain position k, frames in chunks (three; two for the
// log-form score) so that the flow gathers of a chunk are in flight together:
// MIE (Eq. 10) sum_t q_t ell_t(th), a missing frame log 1/2; MLE (Eq. 9)
// sum_t log mu_t - q_t d_t, a missing frame 0
template <int CRIT, int MODEL, bool TR>
__device__ __forceinline__ float chain_score(const FrameF *fr, const float2 *__restrict__ flows,
                                             int T, int H, int W, const EmisParams &e, int x, int y,
                                             float xh, float yh, float th, const float *q, int L,
                                             int k)
{
    // MIE with the Gaussian residual model: the score in log form (LogScore)
    constexpr bool LOGS = CRIT == 0 && MODEL == 1;
    float s = 0.0f;
    LogScore ls = logscore_init();
    float pdx = 0.0f, pdy = 0.0f;
    bool pok = th > 0.0f;
    const int HW = H * W;   // T H W < 2^31 (frames <= 16, sides <= 4096)
    // frames per chunk (their gathers in flight together); the log-form
    // score of the Gaussian model holds more state, so two
    constexpr int FC = LOGS ? 2 : 3;
    for (int t0 = 1; t0 <= T; t0 += FC) {
        float dx[FC], dy[FC], qv[FC];
        bool ok[FC];
#pragma unroll
        for (int u = 0; u < FC; ++u) qv[u] = q[(min(t0 + u, T) - 1) * L + k];   // issued with the gathers
#pragma unroll
        for (int u = 0; u < FC; ++u) {
            const int t = t0 + u;
            const bool f = displacement_any(pixel_geometry(fr[t <= T ? t : T], xh, yh), th, e.fx, e.fy, dx[u], dy[u]);
            ok[u] = (t <= T) & (th > 0.0f) & f;
        }
        float2 ta[FC], tb[FC], tc[FC], td[FC];
        float ax[FC], ay[FC], lx[FC], ly[FC];
        bool val[FC];
#pragma unroll
        for (int u = 0; u < FC; ++u) {
            const float bdx = u == 0 ? pdx : dx[u - 1], bdy = u == 0 ? pdy : dy[u - 1];
            const bool bok = u == 0 ? pok : ok[u - 1];
            const float px = add_nc((float)x, bdx), py = add_nc((float)y, bdy);
            val[u] = bok & ok[u] & (px >= 0.0f) & (px <= (float)(W - 1)) & (py >= 0.0f) & (py <= (float)(H - 1));
            lx[u] = bdx;
            ly[u] = bdy;
            const float spx = val[u] ? px : 0.0f, spy = val[u] ? py : 0.0f;
            const float fx0 = fminf(floorf(spx), (float)(W - 2)), fy0 = fminf(floorf(spy), (float)(H - 2));
            const int x0 = (int)fx0, y0 = (int)fy0;
            ax[u] = spx - fx0;
            ay[u] = spy - fy0;
            const int tf = val[u] ? t0 + u - 1 : 0;
            flow_taps<TR>(flows, tf * HW, x0, y0, H, W, ta[u], tb[u], tc[u], td[u]);
        }
#pragma unroll
        for (int u = 0; u < FC; ++u) {
            const int t = t0 + u;
            if (t > T) break;
            // computed for every frame (branch-free), kept where observed
            const float2 a = ta[u], b = tb[u], c = tc[u], d = td[u];
            const float vu = bilerp(a.x, b.x, c.x, d.x, ax[u], ay[u]);
            const float vv = bilerp(a.y, b.y, c.y, d.y, ax[u], ay[u]);
            const bool obs = val[u] & isfinite(vu + vv);   // every tap finite (see taps_finite)
            if constexpr (LOGS) {
                float lam = kLogLn2F;
                if (obs) {
                    const float dd = log2_odds<MODEL>(sub_nc(sub_nc(dx[u], lx[u]), vu), sub_nc(sub_nc(dy[u], ly[u]), vv), vu, vv, e);
                    float rr;
                    lam = neg_ell_log2(dd, rr);
                }
                logscore_add(ls, qv[u], lam);
            } else if constexpr (CRIT == 0) {
                const float dd = log2_odds<MODEL>(sub_nc(sub_nc(dx[u], lx[u]), vu), sub_nc(sub_nc(dy[u], ly[u]), vv), vu, vv, e);
                const float ell = emis_from_D(dd).ell;
                s = fmaf(qv[u], obs ? ell : kLogHalf, s);
            } else {
                float lmu;
                const float dd = log2_odds_mu<MODEL>(sub_nc(sub_nc(dx[u], lx[u]), vu), sub_nc(sub_nc(dy[u], ly[u]), vv), vu, vv, e, lmu);
                if (obs) s += fmaf(-qv[u], dd * kLn2F, lmu);
            }
        }
        pdx = dx[FC - 1];
        pdy = dy[FC - 1];
        pok = ok[FC - 1];
    }
    if constexpr (LOGS) return logscore_value(ls);
    return s;
}

// D = log2(mu/rho) for a batch of B independent (pixel, frame, depth) items;
// the flow gathers of the whole batch are issued before any of them is used.
// ok[b] false: missing observation (or inactive item).  MU: log mu as well.
template <int B, int MODEL, bool MU, bool TR>
__device__ __forceinline__ void batch_log_odds(const FrameF *fr, const float2 *__restrict__ flows, int H,
                                               int W, const EmisParams &e, const int *x, const int *y,
                                               const float *th, const int *t, const bool *act, float *d,
                                               bool *ok, float *lmu = nullptr)
{
    const int HW = H * W;
    float dx0[B], dy0[B], dx1[B], dy1[B], ax[B], ay[B];
    float2 ta[B], tb[B], tc[B], td[B];
#pragma unroll
    for (int b = 0; b < B; ++b) {
        const float xh = ((float)x[b] - e.cx) * e.ifx, yh = ((float)y[b] - e.cy) * e.ify;
        bool v = act[b] && th[b] > 0.0f;
        const int tt = act[b] ? t[b] : 1;
        dx0[b] = 0.0f;
        dy0[b] = 0.0f;
        if (tt > 1) v = v && displacement(fr[tt - 1], xh, yh, th[b], e.fx, e.fy, dx0[b], dy0[b]);
        v = v && displacement(fr[tt], xh, yh, th[b], e.fx, e.fy, dx1[b], dy1[b]);
        const float px = add_nc((float)x[b], dx0[b]), py = add_nc((float)y[b], dy0[b]);
        v = v && px >= 0.0f && px <= (float)(W - 1) && py >= 0.0f && py <= (float)(H - 1);
        ok[b] = v;
        const float spx = v ? px : 0.0f, spy = v ? py : 0.0f;
        const int x0 = min((int)floorf(spx), W - 2), y0 = min((int)floorf(spy), H - 2);
        ax[b] = spx - (float)x0;
        ay[b] = spy - (float)y0;
        flow_taps<TR>(flows, (v ? tt - 1 : 0) * HW, x0, y0, H, W, ta[b], tb[b], tc[b], td[b]);
    }
#pragma unroll
    for (int b = 0; b < B; ++b) {
        const float2 A = ta[b], Bv = tb[b], Cv = tc[b], Dv = td[b];
        const float vu = bilerp(A.x, Bv.x, Cv.x, Dv.x, ax[b], ay[b]);
        const float vv = bilerp(A.y, Bv.y, Cv.y, Dv.y, ax[b], ay[b]);
        ok[b] = ok[b] && isfinite(vu + vv);   // every tap finite (see taps_finite)
        if constexpr (MU) {
            float lm = 0.0f;
            d[b] = ok[b] ? log2_odds_mu<MODEL>(sub_nc(sub_nc(dx1[b], dx0[b]), vu), sub_nc(sub_nc(dy1[b], dy0[b]), vv), vu, vv, e, lm) : 0.0f;
            lmu[b] = ok[b] ? lm : 0.0f;
        } else {
            d[b] = ok[b] ? log2_odds<MODEL>(sub_nc(sub_nc(dx1[b], dx0[b]), vu), sub_nc(sub_nc(dy1[b], dy0[b]), vv), vu, vv, e) : 0.0f;
        }
    }
}

// The maximum-inlier pass over B (pixel, frame) items, each evaluated at the
// previous depth thp and at the random sample ths: the frame geometry of an
// item is computed once for both depths.  Every log-odds is the same FP32
// function of (pixel, frame, depth) as in batch_log_odds and chain_score.
template <int B, int MODEL, bool TR>
__device__ __forceinline__ void batch_log_odds_pair(const FrameF *fr, const float2 *__restrict__ flows, int H,
                                                    int W, const EmisParams &e, const int *x, const int *y,
                                                    const float *thp, const float *ths, const int *t,
                                                    const bool *act, float *dp, float *ds, bool *okp, bool *oks)
{
    const int HW = H * W;
    float dx0[2 * B], dy0[2 * B], dx1[2 * B], dy1[2 * B], ax[2 * B], ay[2 * B];
    float2 ta[2 * B], tb[2 * B], tc[2 * B], td[2 * B];
    bool v[2 * B];
#pragma unroll
    for (int b = 0; b < B; ++b) {
        const float xh = ((float)x[b] - e.cx) * e.ifx, yh = ((float)y[b] - e.cy) * e.ify;
        const int tt = act[b] ? t[b] : 1;
        const Geo g1 = pixel_geometry(fr[tt], xh, yh);
        const Geo g0 = pixel_geometry(fr[tt > 1 ? tt - 1 : 0], xh, yh);
#pragma unroll
        for (int c = 0; c < 2; ++c) {
            // branch-free: every value is computed and the flags mask them
            const int i = 2 * b + c;
            const float th = c ? ths[b] : thp[b];
            float ex, ey;
            const bool f0 = displacement_any(g0, th, e.fx, e.fy, ex, ey);
            const bool f1 = displacement_any(g1, th, e.fx, e.fy, dx1[i], dy1[i]);
            dx0[i] = tt > 1 ? ex : 0.0f;
            dy0[i] = tt > 1 ? ey : 0.0f;
            const float px = add_nc((float)x[b], dx0[i]), py = add_nc((float)y[b], dy0[i]);
            const bool ok = act[b] & (th > 0.0f) & (f0 | (tt <= 1)) & f1 & (px >= 0.0f) & (px <= (float)(W - 1)) &
                            (py >= 0.0f) & (py <= (float)(H - 1));
            v[i] = ok;
            const float spx = ok ? px : 0.0f, spy = ok ? py : 0.0f;
            const float fx0 = fminf(floorf(spx), (float)(W - 2)), fy0 = fminf(floorf(spy), (float)(H - 2));
            const int x0 = (int)fx0, y0 = (int)fy0;
            ax[i] = spx - fx0;
            ay[i] = spy - fy0;
            flow_taps<TR>(flows, (ok ? tt - 1 : 0) * HW, x0, y0, H, W, ta[i], tb[i], tc[i], td[i]);
        }
    }
#pragma unroll
    for (int i = 0; i < 2 * B; ++i) {
        const float2 A = ta[i], Bv = tb[i], Cv = tc[i], Dv = td[i];
        const float vu = bilerp(A.x, Bv.x, Cv.x, Dv.x, ax[i], ay[i]);
        const float vv = bilerp(A.y, Bv.y, Cv.y, Dv.y, ax[i], ay[i]);
        const bool ok = v[i] & isfinite(vu + vv);   // every tap finite (see taps_finite)
        const float dv = log2_odds<MODEL>(sub_nc(sub_nc(dx1[i], dx0[i]), vu), sub_nc(sub_nc(dy1[i], dy0[i]), vv), vu, vv, e);
        const float d = ok ? dv : 0.0f;
        if (i & 1) {
            ds[i >> 1] = d;
            oks[i >> 1] = ok;
        } else {
            dp[i >> 1] = d;
            okp[i >> 1] = ok;
        }
    }
}

struct SweepArgs {
    const float *theta_in;
    float *theta_out;
    const float2 *flows;
    const float2 *flows_t;   // the same planes transposed, [T][W][H] (column sweeps)
    const double *Mcum;    // cumulative poses M_0..M_T (device)
    const double *range;   // d_lo, d_hi (device)
    float *q_out;
    const int *status;
    int T, H, W, dir;
    EmisParams e;
    float gamma;
    uint64_t seed;
    int64_t gsweep;
    int la_cap;            // look-ahead cap of the propagation rounds (0: none)
};

struct Mat2 {
    float a, b, c, d;  // [[a b] [c d]]
};

__device__ __forceinline__ Mat2 mul_norm(const Mat2 &x, const Mat2 &y)
{
    Mat2 r;
    r.a = x.a * y.a + x.b * y.c;
    r.b = x.a * y.b + x.b * y.d;
    r.c = x.c * y.a + x.d * y.c;
    r.d = x.c * y.b + x.d * y.d;
    const float inv = frcp(r.a + r.b + r.c + r.d);
    r.a *= inv;
    r.b *= inv;
    r.c *= inv;
    r.d *= inv;
    return r;
}

__device__ __forceinline__ Mat2 shfl_up_m(const Mat2 &m, int d)
{
    Mat2 r;
    r.a = __shfl_up(m.a, d, 64);
    r.b = __shfl_up(m.b, d, 64);
    r.c = __shfl_up(m.c, d, 64);
    r.d = __shfl_up(m.d, d, 64);
    return r;
}

__device__ __forceinline__ Mat2 shfl_down_m(const Mat2 &m, int d)
{
    Mat2 r;
    r.a = __shfl_down(m.a, d, 64);
    r.b = __shfl_down(m.b, d, 64);
    r.c = __shfl_down(m.c, d, 64);
    r.d = __shfl_down(m.d, d, 64);
    return r;
}

// Forward-backward over one frame's chain by one wave, one segment [s0, s1)
// of at most SEG positions per lane held in registers: the segment's forward
// and backward transfer products, their prefix and suffix over the lanes by
// shuffles, then the forward and the backward replay, which leave q in rq.
// Every register index is static after unrolling and positions past s1 are
// masked by selects (branches there make the allocator spill).  The products
// with Gamma are formed from the running matrix, so that per position only r
// and the forward message stay live (products of r and gamma shared by the
// two passes would each stay live across both).  r stays in registers from
// its first read, so both replays take the E-step's own r.
template <int SEG>
__device__ __forceinline__ void fb_segment_regs(float *rq, int s0, int s1, float g, float gc, int lane)
{
    const int n = s1 - s0;
    // positions past s1 read whatever follows (the next frame, or the first
    // words of region 2, which holds at least 6 L >= SEG words); unused
    float rr[SEG];
#pragma unroll
    for (int i = 0; i < SEG; ++i) rr[i] = rq[s0 + i];
    // forward A_k = diag(r, 1-r) Gamma, product A_{s1-1}..A_{s0}: Gamma F,
    // rows scaled by r and 1-r
    Mat2 F = {1, 0, 0, 1};
#pragma unroll
    for (int i = 0; i < SEG; ++i) {
        const float r1 = rr[i];
        const float ua = g * F.a + gc * F.c, ub = g * F.b + gc * F.d;
        const float uc = gc * F.a + g * F.c, ud = gc * F.b + g * F.d;
        Mat2 Fn = {r1 * ua, r1 * ub, fmaf(-r1, uc, uc), fmaf(-r1, ud, ud)};
        const float inv = frcp(Fn.a + Fn.b + Fn.c + Fn.d);
        Fn.a *= inv;
        Fn.b *= inv;
        Fn.c *= inv;
        Fn.d *= inv;
        const bool on = i < n;
        F.a = on ? Fn.a : F.a;
        F.b = on ? Fn.b : F.b;
        F.c = on ? Fn.c : F.c;
        F.d = on ? Fn.d : F.d;
    }
    // backward G_k = Gamma diag(r, 1-r), product G_{s0}..G_{s1-1}: rows of B
    // scaled by r and 1-r, then Gamma
    Mat2 B = {1, 0, 0, 1};
#pragma unroll
    for (int i = SEG - 1; i >= 0; --i) {
        const float r1 = rr[i];
        const float va = r1 * B.a, vb = r1 * B.b, vc = fmaf(-r1, B.c, B.c), vd = fmaf(-r1, B.d, B.d);
        Mat2 Bn = {g * va + gc * vc, g * vb + gc * vd, gc * va + g * vc, gc * vb + g * vd};
        const float inv = frcp(Bn.a + Bn.b + Bn.c + Bn.d);
        Bn.a *= inv;
        Bn.b *= inv;
        Bn.c *= inv;
        Bn.d *= inv;
        const bool on = i < n;
        B.a = on ? Bn.a : B.a;
        B.b = on ? Bn.b : B.b;
        B.c = on ? Bn.c : B.c;
        B.d = on ? Bn.d : B.d;
    }
    // inclusive prefix of forward products (later segments on the left),
    // inclusive suffix of backward products (earlier segments on the left)
    Mat2 P = F;
    for (int dd = 1; dd < 64; dd <<= 1) {
        const Mat2 Q = shfl_up_m(P, dd);
        if (lane >= dd) P = mul_norm(P, Q);
    }
    Mat2 Sx = B;
    for (int dd = 1; dd < 64; dd <<= 1) {
        const Mat2 Q = shfl_down_m(Sx, dd);
        if (lane + dd < 64) Sx = mul_norm(Sx, Q);
    }
    const Mat2 Pp = shfl_up_m(P, 1), Sn = shfl_down_m(Sx, 1);
    float f1 = 0.5f, f0 = 0.5f;   // m_f before the segment
    if (lane > 0) {
        const float n1 = 0.5f * (Pp.a + Pp.b), n0 = 0.5f * (Pp.c + Pp.d);
        const float inv = frcp(n1 + n0);
        f1 = n1 * inv;
        f0 = n0 * inv;
    }
    float b1 = 0.5f, b0 = 0.5f;   // m_b at the segment's last position
    if (lane < 63) {
        const float n1 = 0.5f * (Sn.a + Sn.b), n0 = 0.5f * (Sn.c + Sn.d);
        const float inv = frcp(n1 + n0);
        b1 = n1 * inv;
        b0 = n0 * inv;
    }
    float ff[SEG];
#pragma unroll
    for (int i = 0; i < SEG; ++i) {
        const float r1 = rr[i];
        const float p1 = g * f1 + gc * f0, p0 = gc * f1 + g * f0;
        const float n1 = r1 * p1, n0 = fmaf(-r1, p0, p0);
        const float inv = frcp(n1 + n0);
        f1 = n1 * inv;
        f0 = n0 * inv;
        ff[i] = f1;
    }
#pragma unroll
    for (int i = SEG - 1; i >= 0; --i) {
        const float ff1 = ff[i], ff0 = 1.0f - ff1;
        const float n1 = ff1 * b1, n0 = ff0 * b0;
        if (i < n) rq[s0 + i] = n1 * frcp(n1 + n0);
        if (i > 0) {
            const float r1 = rr[i];
            const float e1 = r1 * b1, e0 = fmaf(-r1, b0, b0);
            const float m1 = g * e1 + gc * e0, m0 = gc * e1 + g * e0;
            const float inv = frcp(m1 + m0);
            b1 = i < n ? m1 * inv : b1;
            b0 = i < n ? m0 * inv : b0;
        }
    }
}

// LDS words of region 2 of a chain of length L and T frames: the previous
// depth's ell (MLE: d) in phases A-S, the live lists in C, the jump tables in D
__host__ __device__ inline int sweep_region2_words(int T, int L, int nt = kSweepThreads)
{
    int w = T * L;
    if (w < 6 * L) w = 6 * L;   // the live lists: two of (origin, position) pairs, two of first losses
    if (w < 4 * L + nt) w = 4 * L + nt;
    return w;
}

// CRIT 0: maximum-inlier depth criterion (Eq. 10); 1: maximum likelihood (Eq. 9).
// MODEL 0: Fisk residual model (Eq. 5); 1: Gaussian flow error.
// NT threads per chain (256, 512, 768 or 1024): every item is the same function of
// its inputs whatever NT is, so all widths give the same result bit for bit;
// NT only sets how a chain's work is spread (and how many chains fit a CU)
// XCD-aware item order: workgroups are dealt round-robin to the 8 XCDs, so
// give each XCD a contiguous range of items (neighbouring chains share flow
// cache lines in that XCD's L2)
__device__ __forceinline__ int xcd_item(int block, int nitems)
{
    const int xcd = block & 7, slot = block >> 3;
    const int per = (nitems + 7) >> 3;
    const int full = nitems - (per - 1) * 8;
    return xcd < full ? xcd * per + slot : full * per + (xcd - full) * (per - 1) + slot;
}

// The sweep of one chain by one workgroup; lds is the dynamic area, fr and
// s_cnt the workgroup's frames and list counters.
template <int CRIT, int NT, int MODEL, bool TR>
__device__ __forceinline__ void sweep_chain(const SweepArgs &a, const int chain, float *lds, FrameF *fr,
                                            int *s_cnt)
{
    // column chains (TR) gather from the transposed copy of the flows
    const float2 *__restrict__ fl = TR ? a.flows_t : a.flows;
    if (a.status && *a.status != kStatusOk) return;
    // MIE with the Gaussian residual model keeps lam = log(-ell) per item and
    // the scores in log form (LogScore in vo_device.hpp)
    constexpr bool LOGS = CRIT == 0 && MODEL == 1;

    const int T = a.T, H = a.H, W = a.W, dir = a.dir;
    const int L = (dir & 1) ? H : W;
    const int tid = threadIdx.x;

    float *th = lds;                                   // [L]   previous depth
    float *sm = th + L;                                // [L]   random sample
    float *fq = sm + L;                                // [T][L] r -> forward message -> q
    float *lq = fq + T * L;                            // region 2: ell(prev) (MLE: then the sample's terms), lists, doubling
    // region 3, [max(T, 4)][L]: MIE ell of the random sample; MLE (region 2
    // then holds d = log(mu/rho) of the previous depth) its log mu.  Phase S
    // reads a position's rows and then writes that position's local best,
    // its score, the sample flag and (later) next() over rows 0-3: each
    // thread only over the rows of its own positions, read before written
    float *lmq = lq + sweep_region2_words(T, L, NT);
    float *ls = lmq;
    float *aval = lmq;                                 // [L]   local best value
    float *sa = aval + L;                              // [L]   score: previous, then local best
    int *flg = (int *)(sa + L);                        // [L]   1 if the sample is the local best
    int *nxt = flg + L;                                // [L]   next(k)

    load_frames(a.Mcum, T, fr);
    if (tid == 0) {
        s_cnt[0] = 0;
        s_cnt[1] = 0;
    }
    const float llo = (float)log(a.range[0]);
    const float lrange = (float)(log(a.range[1]) - log(a.range[0]));
    for (int k = tid; k < L; k += NT) th[k] = a.theta_in[chain_pixel(dir, H, W, chain, k)];
    // random depth, log-uniform: the 8 chain positions whose coordinate along
    // the sweep axis is 8g .. 8g + 7 take the 32-bit words of the Philox block
    // with counter (gsweep, chain, g, 0), hi before lo of each 64-bit output
    for (int g = tid; g < (L + 7) / 8; g += NT) {
        uint64_t c[4] = {(uint64_t)a.gsweep, (uint64_t)chain, (uint64_t)g, 0ull};
        philox4x64_10(c, a.seed, kDepthStream);
#pragma unroll
        for (int m = 0; m < 8; ++m) {
            const int ax = 8 * g + m;
            if (ax < L) {
                const uint32_t w = (m & 1) ? (uint32_t)c[m >> 1] : (uint32_t)(c[m >> 1] >> 32);
                const float u = ((float)w + 0.5f) * 2.3283064365386963e-10f;
                sm[dir >= 2 ? L - 1 - ax : ax] = expf(fmaf(u, lrange, llo));
            }
        }
    }
    __syncthreads();

    // ---- A (MIE): ell and r of the previous depth and ell of the random
    // sample, one item per (position, frame) evaluated at both depths,
    // kPairItems items per thread in flight
    if constexpr (CRIT == 0) {
        constexpr int PB = kPairItems;
        // item i = (t - 1) L + k; the thread's items are NT apart, (t, k)
        // carried from one item to the next
        int t = tid / L + 1, k = tid - (t - 1) * L;
        for (int i0 = tid; i0 < T * L; i0 += PB * NT) {
            int xs[PB], ys[PB], ts[PB];
            float thp[PB], ths[PB], dp[PB], ds[PB];
            bool act[PB], okp[PB], oks[PB];
#pragma unroll
            for (int b = 0; b < PB; ++b) {
                act[b] = i0 + b * NT < T * L;
                const int kk = act[b] ? k : 0;
                chain_xy(dir, H, W, chain, kk, xs[b], ys[b]);
                ts[b] = act[b] ? t : 1;
                thp[b] = th[kk];
                ths[b] = sm[kk];
                k += NT;
                while (k >= L) { k -= L; ++t; }
            }
            batch_log_odds_pair<PB, MODEL, TR>(fr, fl, H, W, a.e, xs, ys, thp, ths, ts, act, dp, ds, okp, oks);
#pragma unroll
            for (int b = 0; b < PB; ++b) {
                const int i = i0 + b * NT;
                if (!act[b]) continue;
                // computed for every item, kept where observed
                constexpr float miss = LOGS ? kLogLn2F : kLogHalf;
                float ell, r, els;
                if constexpr (LOGS) {
                    float rp, rs;
                    const float lp = neg_ell_log2(dp[b], rp), lz = neg_ell_log2(ds[b], rs);
                    ell = okp[b] ? lp : miss;
                    r = okp[b] ? rp : 0.5f;
                    els = oks[b] ? lz : miss;
                } else {
                    const Emis mp = emis_from_D(dp[b]), mz = emis_from_D(ds[b]);
                    ell = okp[b] ? mp.ell : miss;
                    r = okp[b] ? mp.r : 0.5f;
                    els = oks[b] ? mz.ell : miss;
                }
                lq[i] = ell;
                fq[i] = r;
                ls[i] = els;
            }
        }
    }
    // ---- A (MLE): log-odds and log mu of the previous depth, two items per
    // thread in flight (the sample follows the E-step: its terms need q)
    if constexpr (CRIT == 1)
    for (int i0 = tid; i0 < T * L; i0 += kMleItems * NT) {
        int xs[kMleItems], ys[kMleItems], ts[kMleItems];
        float ths[kMleItems], dd[kMleItems];
        bool act[kMleItems], ok[kMleItems];
        // item i = (t - 1) L + k; the thread's items are NT apart
        int t = i0 / L + 1, k = i0 - (t - 1) * L;
#pragma unroll
        for (int b = 0; b < kMleItems; ++b) {
            act[b] = i0 + b * NT < T * L;
            const int kk = act[b] ? k : 0;
            chain_xy(dir, H, W, chain, kk, xs[b], ys[b]);
            ts[b] = act[b] ? t : 1;
            ths[b] = th[kk];
            k += NT;
            while (k >= L) { k -= L; ++t; }
        }
        {
            float lm[kMleItems];
            batch_log_odds<kMleItems, MODEL, true, TR>(fr, fl, H, W, a.e, xs, ys, ths, ts, act, dd, ok, lm);
#pragma unroll
            for (int b = 0; b < kMleItems; ++b) {
                const int i = i0 + b * NT;
                if (!act[b]) continue;
                // missing: d = 0 (r = 1/2 in the E-step) and log mu = 0 (term 0)
                lq[i] = dd[b] * kLn2F;   // d = log(mu / rho)
                lmq[i] = lm[b];
                fq[i] = ok[b] ? emis_from_D(dd[b]).r : 0.5f;
            }
        }
    }
    __syncthreads();

    // ---- B: forward-backward, one wave per frame, one segment per lane
    {
        const int lane = tid & 63, wv = tid >> 6;
        // segment length: a function of L alone (the same segments, and so
        // the same rounding, whatever NT is)
        const int seglen = ((L + 63) / 64) | 1;
        const float g = a.gamma, gc = 1.0f - a.gamma;
        const int s0 = min(lane * seglen, L), s1 = min(s0 + seglen, L);
        for (int t = wv; t < T; t += (NT / 64)) {
            float *rq = fq + t * L;
            const float *ll = lq + t * L;
            // segments held in registers up to 11 positions (chains of 704)
            if (seglen <= 5) { fb_segment_regs<5>(rq, s0, s1, g, gc, lane); continue; }
            if (seglen <= 7) { fb_segment_regs<7>(rq, s0, s1, g, gc, lane); continue; }
            if (seglen <= 11) { fb_segment_regs<11>(rq, s0, s1, g, gc, lane); continue; }
            // segment transfer matrices: forward A_k = diag(r,1-r) Gamma,
            // product A_{s1-1}..A_{s0}; backward G_k = Gamma diag(r,1-r),
            // product G_{s0}..G_{s1-1}
            Mat2 F = {1, 0, 0, 1}, B = {1, 0, 0, 1};
            for (int k = s0; k < s1; ++k) {
                const float r1 = rq[k], r0 = 1.0f - r1;
                const Mat2 A = {r1 * g, r1 * gc, r0 * gc, r0 * g};
                F = mul_norm(A, F);
            }
            for (int k = s1 - 1; k >= s0; --k) {
                const float r1 = rq[k], r0 = 1.0f - r1;
                const Mat2 G = {g * r1, gc * r0, gc * r1, g * r0};
                B = mul_norm(G, B);
            }
            // inclusive prefix of forward products (later segments on the left)
            Mat2 P = F;
            for (int dd = 1; dd < 64; dd <<= 1) {
                const Mat2 Q = shfl_up_m(P, dd);
                if (lane >= dd) P = mul_norm(P, Q);
            }
            // inclusive suffix of backward products (earlier segments on the left)
            Mat2 Sx = B;
            for (int dd = 1; dd < 64; dd <<= 1) {
                const Mat2 Q = shfl_down_m(Sx, dd);
                if (lane + dd < 64) Sx = mul_norm(Sx, Q);
            }
            const Mat2 Pp = shfl_up_m(P, 1), Sn = shfl_down_m(Sx, 1);
            float f1 = 0.5f, f0 = 0.5f;   // m_f before the segment
            if (lane > 0) {
                const float n1 = 0.5f * (Pp.a + Pp.b), n0 = 0.5f * (Pp.c + Pp.d);
                const float inv = frcp(n1 + n0);
                f1 = n1 * inv;
                f0 = n0 * inv;
            }
            float b1 = 0.5f, b0 = 0.5f;   // m_b at the segment's last position
            if (lane < 63) {
                const float n1 = 0.5f * (Sn.a + Sn.b), n0 = 0.5f * (Sn.c + Sn.d);
                const float inv = frcp(n1 + n0);
                b1 = n1 * inv;
                b0 = n0 * inv;
            }
            for (int k = s0; k < s1; ++k) {
                const float r1 = rq[k], r0 = 1.0f - r1;
                const float p1 = g * f1 + gc * f0, p0 = gc * f1 + g * f0;
                const float n1 = r1 * p1, n0 = r0 * p0;
                const float inv = frcp(n1 + n0);
                f1 = n1 * inv;
                f0 = n0 * inv;
                rq[k] = f1;
            }
            for (int k = s1 - 1; k >= s0; --k) {
                const float ff1 = rq[k], ff0 = 1.0f - ff1;
                const float n1 = ff1 * b1, n0 = ff0 * b0;
                rq[k] = n1 * frcp(n1 + n0);
                if (k > s0) {
                    float r1 = LOGS        ? fast_exp(-fast_exp(ll[k]))
                               : CRIT == 0 ? fast_exp(ll[k])
                                           : frcp(1.0f + fast_exp(ll[k]));
                    r1 = r1 >= kFltMin ? r1 : 0.0f;   // as in phase A
                    const float r0 = 1.0f - r1;
                    const float e1 = r1 * b1, e0 = r0 * b0;
                    const float m1 = g * e1 + gc * e0, m0 = gc * e1 + g * e0;
                    const float inv = frcp(m1 + m0);
                    b1 = m1 * inv;
                    b0 = m0 * inv;
                }
            }
        }
    }
    __syncthreads();
    if (a.q_out) {
        for (int i = tid; i < T * L; i += NT) {
            const int t = i / L, k = i - t * L;
            a.q_out[(size_t)t * H * W + chain_pixel(dir, H, W, chain, k)] = fq[i];
        }
    }

    // ---- S: scores of the previous depth and of the sample; the local best
    if constexpr (CRIT == 0) {
        for (int k = tid; k < L; k += NT) {
            float sp = 0.0f, ss = 0.0f;
            if constexpr (LOGS) {
                LogScore lp = logscore_init(), lz = logscore_init();
                for (int t = 0; t < T; ++t) {
                    logscore_add(lp, fq[t * L + k], lq[t * L + k]);
                    logscore_add(lz, fq[t * L + k], ls[t * L + k]);
                }
                sp = logscore_value(lp);
                ss = logscore_value(lz);
            } else {
                // frames four at a time: their loads in flight together
                for (int t0 = 0; t0 < T; t0 += 4) {
                    float qv[4], pv[4], sv[4];
#pragma unroll
                    for (int u = 0; u < 4; ++u) {
                        const int i = min(t0 + u, T - 1) * L + k;
                        qv[u] = fq[i];
                        pv[u] = lq[i];
                        sv[u] = ls[i];
                    }
#pragma unroll
                    for (int u = 0; u < 4; ++u) {
                        if (t0 + u < T) {
                            sp = fmaf(qv[u], pv[u], sp);
                            ss = fmaf(qv[u], sv[u], ss);
                        }
                    }
                }
            }
            const bool smp = ss > sp;
            aval[k] = smp ? sm[k] : th[k];
            sa[k] = smp ? ss : sp;
            flg[k] = smp ? 1 : 0;
        }
    } else {
        for (int k = tid; k < L; k += NT) {
            float s = 0.0f;
            for (int t = 0; t < T; ++t) s += fmaf(-fq[t * L + k], lq[t * L + k], lmq[t * L + k]);
            sa[k] = s;
        }
        __syncthreads();
        // the sample's whole term log mu - q d (0 where missing), one item per
        // (position, frame)
        for (int i0 = tid; i0 < T * L; i0 += kMleItems * NT) {
            int xs[kMleItems], ys[kMleItems], ts[kMleItems];
            float ths[kMleItems], dd[kMleItems], lm[kMleItems];
            bool act[kMleItems], ok[kMleItems];
            // item i = (t - 1) L + k; the thread's items are NT apart
            int t = i0 / L + 1, k = i0 - (t - 1) * L;
#pragma unroll
            for (int b = 0; b < kMleItems; ++b) {
                act[b] = i0 + b * NT < T * L;
                const int kk = act[b] ? k : 0;
                chain_xy(dir, H, W, chain, kk, xs[b], ys[b]);
                ts[b] = act[b] ? t : 1;
                ths[b] = sm[kk];
                k += NT;
                while (k >= L) { k -= L; ++t; }
            }
            batch_log_odds<kMleItems, MODEL, true, TR>(fr, fl, H, W, a.e, xs, ys, ths, ts, act, dd, ok, lm);
#pragma unroll
            for (int b = 0; b < kMleItems; ++b) {
                const int i = i0 + b * NT;
                if (act[b]) lq[i] = ok[b] ? fmaf(-fq[i], dd[b] * kLn2F, lm[b]) : 0.0f;
            }
        }
        __syncthreads();
        for (int k = tid; k < L; k += NT) {
            float s = 0.0f;
            for (int t = 0; t < T; ++t) s += lq[t * L + k];
            const bool smp = s > sa[k];
            aval[k] = smp ? sm[k] : th[k];
            if (smp) sa[k] = s;
            flg[k] = smp ? 1 : 0;
        }
    }
    __syncthreads();   // the live lists below reuse region 2
    // live origins (origin, next position to test), starting at k+1; a local
    // best equal to the previous depth at k+1 scores exactly that depth there
    // and loses (the previous depth wins ties), so next(k) = k+1 at once
    int2 *list0 = (int2 *)lq, *list1 = list0 + L;
    // first losing offset of each live origin, INT_MAX until one is seen
    int *first0 = (int *)(list1 + L), *first1 = first0 + L;
    for (int k = tid; k < L; k += NT) {
        if (k == L - 1) {
            nxt[k] = L;
        } else if (aval[k] == th[k + 1]) {
            nxt[k] = k + 1;
        } else {
            const int at = atomicAdd(&s_cnt[0], 1);
            list0[at] = make_int2(k, k + 1);
            first0[at] = INT_MAX;
        }
    }
    __syncthreads();

    // ---- C: survival of every local best as the propagated neighbour
    int cur = 0;
    for (;;) {
        const int n = s_cnt[cur];
        if (n == 0) break;
        int2 *lc = cur ? list1 : list0, *ln = cur ? list0 : list1;
        int *first = cur ? first1 : first0, *firstn = cur ? first0 : first1;
        int la = max(NT / n, 1);   // look-ahead per live origin
        if (a.la_cap > 0 && la > a.la_cap) la = a.la_cap;
        const int items = n * la;
        const float ila = frcp((float)la);
        for (int i = tid; i < items; i += NT) {
            // i / la through FP32: (i + 1/2) / la is at least 1/(2 la) from an integer
            const int sl = (int)(((float)i + 0.5f) * ila), p = i - sl * la;
            const int2 e = lc[sl];
            const int jpos = e.y + p;
            bool w = false;
            if (jpos < L && flg[jpos] && aval[e.x] == sm[jpos]) {
                // the sample of jpos is its local best and has this very value:
                // the same score, and the neighbour wins the tie
                w = true;
            } else if (jpos < L && !(aval[e.x] == th[jpos])) {   // equal to the previous depth: loses
                int x, y;
                chain_xy(dir, H, W, chain, jpos, x, y);
                const float xh = ((float)x - a.e.cx) * a.e.ifx, yh = ((float)y - a.e.cy) * a.e.ify;
                const float s = chain_score<CRIT, MODEL, TR>(fr, fl, T, H, W, a.e, x, y, xh, yh, aval[e.x], fq, L, jpos);
                w = flg[jpos] ? (s >= sa[jpos]) : (s > sa[jpos]);
            }
            if (!w) atomicMin(&first[sl], p);
        }
        if (tid == 0) s_cnt[cur ^ 1] = 0;
        __syncthreads();
        for (int sl = tid; sl < n; sl += NT) {
            const int2 e = lc[sl];
            const int p = first[sl];   // INT_MAX: survived the whole look-ahead
            if (p < la) {
                nxt[e.x] = min(e.y + p, L);
            } else if (e.y + la >= L) {
                nxt[e.x] = L;
            } else {
                const int at = atomicAdd(&s_cnt[cur ^ 1], 1);
                ln[at] = make_int2(e.x, e.y + la);
                firstn[at] = INT_MAX;
            }
        }
        __syncthreads();
        cur ^= 1;
    }

    // ---- D: nodes reachable from 0 through next(), by pointer doubling
    int *J0 = (int *)lq, *J1 = J0 + L, *mark = J1 + L;
    float *thn = (float *)(mark + L);
    for (int k = tid; k < L; k += NT) mark[k] = k == 0;
    __syncthreads();
    // round i follows jumps of 2^i hops (Jc = next^(2^i)): a node h hops from
    // 0 is marked once the rounds of the set bits of h have run.  Marks only
    // grow and only reach nodes reachable from 0, so a mark that another
    // thread sets during the same round changes nothing at the end; the jump
    // table of the next round goes to the other buffer, so one barrier per
    // round suffices.
    const int *Jc = nxt;
    int *Jn = J0;
    for (int span = 1; span < L; span <<= 1) {
        for (int k = tid; k < L; k += NT) {
            const int to = Jc[k];
            if (mark[k] && to < L) mark[to] = 1;
            Jn[k] = to < L ? Jc[to] : L;
        }
        __syncthreads();
        Jc = Jn;
        Jn = Jn == J0 ? J1 : J0;
    }
    for (int k = tid; k < L; k += NT) {
        if (mark[k]) {
            const int e = nxt[k];
            const float v = aval[k];
            for (int j = k; j < e; ++j) thn[j] = v;
        }
    }
    __syncthreads();
    for (int k = tid; k < L; k += NT) a.theta_out[chain_pixel(dir, H, W, chain, k)] = thn[k];
}

template <int CRIT, int NT, int MODEL>
__global__ void __launch_bounds__(NT, 6) k_sweep(SweepArgs a)
{
    extern __shared__ float lds[];
    __shared__ FrameF fr[kTMax + 1];
    __shared__ int s_cnt[2];
    const int chain = xcd_item(blockIdx.x, gridDim.x);
    if (a.dir & 1)
        sweep_chain<CRIT, NT, MODEL, true>(a, chain, lds, fr, s_cnt);
    else
        sweep_chain<CRIT, NT, MODEL, false>(a, chain, lds, fr, s_cnt);
}

// One sweep of the chains of several windows (a lockstep batch lane): item u
// is chain u - first[w] of window w, first[] the windows' chain offsets
// (first[nwin] = gridDim.x); each window's arguments are those of its single
// launch, so every chain gets exactly its single-window result.
// the arguments of a batched launch with their pointers in the global
// address space (global_ptr)
__device__ __forceinline__ SweepArgs to_global(SweepArgs a)
{
    a.theta_in = global_ptr(a.theta_in);
    a.theta_out = global_ptr(a.theta_out);
    a.flows = global_ptr(a.flows);
    a.flows_t = global_ptr(a.flows_t);
    a.Mcum = global_ptr(a.Mcum);
    a.range = global_ptr(a.range);
    a.q_out = global_ptr(a.q_out);
    a.status = global_ptr(a.status);
    return a;
}

template <int CRIT, int NT, int MODEL>
__global__ void __launch_bounds__(NT, 6) k_sweep_multi(const SweepArgs *args, const int *first, int nwin)
{
    extern __shared__ float lds[];
    __shared__ FrameF fr[kTMax + 1];
    __shared__ int s_cnt[2];
    const int u = xcd_item(blockIdx.x, gridDim.x);
    int w = 0;
    while (w + 1 < nwin && u >= first[w + 1]) ++w;
    const SweepArgs a = to_global(args[w]);
    if (a.dir & 1)
        sweep_chain<CRIT, NT, MODEL, true>(a, u - first[w], lds, fr, s_cnt);
    else
        sweep_chain<CRIT, NT, MODEL, false>(a, u - first[w], lds, fr, s_cnt);
}

// ---------------------------------------------------------------------------
// unsmoothed rigidness W_t = r_t(theta) (last row of Table 1), optional dense
// emission maps, optional log-likelihood partial sums of Eq. 3
// ---------------------------------------------------------------------------
struct RigArgs {
    const float *theta;
    float *theta_gauge;     // optional: theta / |t_1| written back in place (scale gauge)
    const double *rel;      // relative poses (t_1 gives the gauge)
    const float2 *flows;
    const double *Mcum;
    const int *status;
    float *r, *ell, *logrho, *logmu;
    double *ll_part;
    int T, H, W;
    int nblk;               // workgroups over the window's pixels
    EmisParams e;
};

__device__ __forceinline__ void rigidness_body(const RigArgs &a)
{
    if (a.status && *a.status != kStatusOk) return;
    __shared__ FrameF fr[kTMax + 1];
    __shared__ double red[2][256];
    load_frames(a.Mcum, a.T, fr);
    __syncthreads();
    const int HW = a.H * a.W;
    double gscale = 1.0;
    if (a.theta_gauge) {
        const double *t1 = a.rel + 9;
        const double g = sqrt(t1[0] * t1[0] + t1[1] * t1[1] + t1[2] * t1[2]);
        gscale = g > 0 ? g : 1.0;
    }
    double acc = 0.0, mass = 0.0;
    for (int j = blockIdx.x * blockDim.x + threadIdx.x; j < HW; j += a.nblk * blockDim.x) {
        const int y = j / a.W, x = j - y * a.W;
        const float xh = ((float)x - a.e.cx) * a.e.ifx, yh = ((float)y - a.e.cy) * a.e.ify;
        const float th = a.theta[j];
        float px0 = 0.0f, py0 = 0.0f;
        bool ok0 = th > 0.0f;
        // frames in chunks of four: the flow gathers of a chunk are in flight together
        for (int t0 = 1; t0 <= a.T; t0 += 4) {
            float dx1[4], dy1[4], bx[4], by[4], ax[4], ay[4];
            bool val[4], ok1[4];
            float2 ta[4], tb[4], tc[4], td[4];
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                const int t = t0 + u;
                dx1[u] = 0.0f;
                dy1[u] = 0.0f;
                ok1[u] = t <= a.T && displacement(fr[t <= a.T ? t : a.T], xh, yh, th, a.e.fx, a.e.fy, dx1[u], dy1[u]);
                bx[u] = u == 0 ? px0 : dx1[u - 1];
                by[u] = u == 0 ? py0 : dy1[u - 1];
                const bool bok = u == 0 ? ok0 : ok1[u - 1];
                const float spx = add_nc((float)x, bx[u]), spy = add_nc((float)y, by[u]);
                val[u] = bok && ok1[u] && spx >= 0.0f && spx <= (float)(a.W - 1) && spy >= 0.0f &&
                         spy <= (float)(a.H - 1);
                const float qx = val[u] ? spx : 0.0f, qy = val[u] ? spy : 0.0f;
                const int x0 = min((int)floorf(qx), a.W - 2), y0 = min((int)floorf(qy), a.H - 2);
                ax[u] = qx - (float)x0;
                ay[u] = qy - (float)y0;
                const float2 *r0 = a.flows + ((val[u] ? t - 1 : 0) * HW + y0 * a.W + x0);
                ta[u] = r0[0];
                tb[u] = r0[1];
                tc[u] = r0[a.W];
                td[u] = r0[a.W + 1];
            }
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                const int t = t0 + u;
                if (t > a.T) break;
                float r = 0.5f, ell = -0.69314718055994531f, lr = 0.0f, lm = 0.0f;
                const float2 A = ta[u], B = tb[u], Cc = tc[u], D = td[u];
                const float vu = bilerp(A.x, B.x, Cc.x, D.x, ax[u], ay[u]);
                const float vv = bilerp(A.y, B.y, Cc.y, D.y, ax[u], ay[u]);
                if (val[u] && isfinite(vu + vv)) {   // every tap finite (see taps_finite)
                    const float rx = sub_nc(sub_nc(dx1[u], bx[u]), vu), ry = sub_nc(sub_nc(dy1[u], by[u]), vv);
                    const float d2 = a.e.model ? log2_odds<1>(rx, ry, vu, vv, a.e) : log2_odds<0>(rx, ry, vu, vv, a.e);
                    const Emis m = emis_from_D(d2);
                    r = m.r;
                    ell = m.ell;
                    if (a.logrho || a.logmu || a.ll_part) {
                        const float vn = __builtin_amdgcn_sqrtf(fmaf(vu, vu, vv * vv));
                        const float la = fmaf(a.e.a2, vn, a.e.log_a1);
                        const float x2 = fminf(fmaxf(fmaf(rx, rx, ry * ry), a.e.x_floor), 1e30f);
                        if (a.e.model) {   // exponential with mean s = alpha / ln 2
                            lr = fmaf(-x2, kLn2F * fast_exp(-la), kLogLn2F - la);
                        } else {           // Fisk (Eq. 5)
                            const float beta = fmaxf(fmaf(a.e.b1, vn, a.e.b2), a.e.beta_min);
                            const float s1 = fast_log(x2) - la;
                            const float lb = fast_log(beta) - la;
                            lr = lb + (beta - 1.0f) * s1 - 2.0f * softplus(beta * s1);
                        }
                        lm = fmaf(d2, kLn2F, lr);
                        const double w = r;
                        const double term = w * (double)lr + (1.0 - w) * (double)lm;
                        acc += term;
                        mass += fabs(term);
                    }
                }
                const int o = (t - 1) * HW + j;
                if (a.r) a.r[o] = r;
                if (a.ell) a.ell[o] = ell;
                if (a.logrho) a.logrho[o] = lr;
                if (a.logmu) a.logmu[o] = lm;
            }
            px0 = dx1[3];
            py0 = dy1[3];
            ok0 = ok1[3];
        }
        if (a.theta_gauge) a.theta_gauge[j] = (float)((double)th / gscale);
    }
    if (a.ll_part) {
        red[0][threadIdx.x] = acc;
        red[1][threadIdx.x] = mass;
        __syncthreads();
        for (int s = 128; s > 0; s >>= 1) {
            if (threadIdx.x < s) {
                red[0][threadIdx.x] += red[0][threadIdx.x + s];
                red[1][threadIdx.x] += red[1][threadIdx.x + s];
            }
            __syncthreads();
        }
        if (threadIdx.x == 0) {
            a.ll_part[2 * blockIdx.x] = red[0][0];
            a.ll_part[2 * blockIdx.x + 1] = red[1][0];
        }
    }
}

__global__ void __launch_bounds__(256) k_rigidness(RigArgs a) { rigidness_body(a); }

// the rigidness pass of several windows (a lockstep batch lane), blockIdx.y
// selecting a window's arguments
__device__ __forceinline__ RigArgs to_global(RigArgs a)
{
    a.theta = global_ptr(a.theta);
    a.theta_gauge = global_ptr(a.theta_gauge);
    a.rel = global_ptr(a.rel);
    a.flows = global_ptr(a.flows);
    a.Mcum = global_ptr(a.Mcum);
    a.status = global_ptr(a.status);
    a.r = global_ptr(a.r);
    a.ell = global_ptr(a.ell);
    a.logrho = global_ptr(a.logrho);
    a.logmu = global_ptr(a.logmu);
    a.ll_part = global_ptr(a.ll_part);
    return a;
}

__global__ void __launch_bounds__(256) k_rigidness_multi(const RigArgs *args)
{
    const RigArgs a = to_global(args[blockIdx.y]);
    if ((int)blockIdx.x >= a.nblk) return;   // past this window's workgroups
    rigidness_body(a);
}

// fixed-order sum of the per-block partial sums
__device__ __forceinline__ void ll_reduce_body(const double *part, int n, const int *status, double *out)
{
    if (status && *status != kStatusOk) return;
    __shared__ double red[2][256];
    double a = 0, m = 0;
    for (int i = threadIdx.x; i < n; i += 256) {
        a += part[2 * i];
        m += part[2 * i + 1];
    }
    red[0][threadIdx.x] = a;
    red[1][threadIdx.x] = m;
    __syncthreads();
    for (int s = 128; s > 0; s >>= 1) {
        if (threadIdx.x < s) {
            red[0][threadIdx.x] += red[0][threadIdx.x + s];
            red[1][threadIdx.x] += red[1][threadIdx.x + s];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        out[0] = red[0][0];
        out[1] = red[1][0];
    }
}

__global__ void k_ll_reduce(const double *part, int n, const int *status, double *out)
{
    ll_reduce_body(part, n, status, out);
}

struct LLArgs {
    const double *part;
    const int *status;
    double *out;
    int n;
};

__global__ void k_ll_reduce_multi(const LLArgs *args)
{
    const LLArgs a = args[blockIdx.y];
    ll_reduce_body(global_ptr(a.part), a.n, global_ptr(a.status), global_ptr(a.out));
}

__global__ void k_philox(const uint64_t *ctr, uint64_t k0, uint64_t k1, uint64_t *out, int n)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    uint64_t c[4] = {ctr[4 * i], ctr[4 * i + 1], ctr[4 * i + 2], ctr[4 * i + 3]};
    philox4x64_10(c, k0, k1);
    for (int k = 0; k < 4; ++k) out[4 * i + k] = c[k];
}

// ---------------------------------------------------------------------------
size_t sweep_lds_bytes(int T, int L, int criterion, int nt)
{
    // th, sm, fq, region 2, region 3 (both criteria hold a third [T][L] array:
    // MIE the sample's ell, MLE log mu; at least 4 rows for the local bests)
    (void)criterion;
    return ((size_t)(2 + T + (T > 4 ? T : 4)) * L + (size_t)sweep_region2_words(T, L, nt)) * sizeof(float);
}

void sweep_cfg_for(const voldor_ctx *c, int axis, int L, int T, int crit, int *nt, int *la)
{
    *nt = c->sweep_nt[axis];
    *la = c->sweep_la[axis];
    for (int i = 0; i < c->n_sweep_tab; ++i) {
        const SweepCfg &e = c->sweep_tab[i];
        if (e.L == L && e.T == T && e.crit == crit) {
            *nt = e.nt;
            *la = e.la;
            return;
        }
    }
}

void sweep_cfg_store(voldor_ctx *c, int L, int T, int crit, int nt, int la)
{
    int slot = -1;
    for (int i = 0; i < c->n_sweep_tab; ++i)
        if (c->sweep_tab[i].L == L && c->sweep_tab[i].T == T && c->sweep_tab[i].crit == crit) slot = i;
    if (slot < 0) {
        if (c->n_sweep_tab < kSweepTab) {
            slot = c->n_sweep_tab++;
        } else {   // full: drop the oldest entry
            for (int i = 1; i < kSweepTab; ++i) c->sweep_tab[i - 1] = c->sweep_tab[i];
            slot = kSweepTab - 1;
        }
    }
    c->sweep_tab[slot] = SweepCfg{L, T, crit, nt, la};
}

template <int CRIT, int NT, int MODEL>
static int launch_sweep_nt(const SweepArgs &a, int nchain, size_t lds, hipStream_t s)
{
    if (lds > 65536 &&
        hipFuncSetAttribute((const void *)k_sweep<CRIT, NT, MODEL>, hipFuncAttributeMaxDynamicSharedMemorySize,
                            (int)lds) != hipSuccess)
        return VOLDOR_EDEVICE;
    hipLaunchKernelGGL((k_sweep<CRIT, NT, MODEL>), dim3(nchain), dim3(NT), lds, s, a);
    return hipGetLastError() == hipSuccess ? 0 : VOLDOR_EDEVICE;
}

// arguments, threads per chain and LDS bytes of one sweep of a window
static void sweep_args(voldor_ctx *c, const float *theta_in, float *theta_out, const float2 *flows,
                       const WinDims &d, const EmisParams &e, float gamma, uint64_t seed, int64_t gsweep,
                       int dir, const double *range_dev, float *q_out, int criterion, SweepArgs &a, int &nt,
                       size_t &lds)
{
    const int L = (dir & 1) ? d.H : d.W;
    int la = 0;
    nt = 512;
    sweep_cfg_for(c, dir & 1, L, d.T, criterion, &nt, &la);
    lds = sweep_lds_bytes(d.T, L, criterion, nt);
    a.theta_in = theta_in;
    a.theta_out = theta_out;
    a.flows = flows;
    a.flows_t = c->flows_t;
    a.Mcum = c->Mcum;
    a.range = range_dev;
    a.q_out = q_out;
    a.status = c->status;
    a.T = d.T;
    a.H = d.H;
    a.W = d.W;
    a.dir = dir;
    a.e = e;
    a.gamma = gamma;
    a.seed = seed;
    a.gsweep = gsweep;
    a.la_cap = la;
}

int launch_sweep(voldor_ctx *c, const float *theta_in, float *theta_out, const float2 *flows,
                 const WinDims &d, const EmisParams &e, float gamma, uint64_t seed, int64_t gsweep,
                 int dir, const double *range_dev, float *q_out, hipStream_t s, int criterion)
{
    const int L = (dir & 1) ? d.H : d.W;
    const int nchain = (dir & 1) ? d.W : d.H;
    if (L < 16) return VOLDOR_EINVAL;
    SweepArgs a;
    int nt = 512;
    size_t lds = 0;
    sweep_args(c, theta_in, theta_out, flows, d, e, gamma, seed, gsweep, dir, range_dev, q_out, criterion, a, nt,
               lds);
    switch ((nt * 2 + (criterion ? 1 : 0)) * 2 + (e.model ? 1 : 0)) {
    case 1024: return launch_sweep_nt<0, 256, 0>(a, nchain, lds, s);
    case 1025: return launch_sweep_nt<0, 256, 1>(a, nchain, lds, s);
    case 1026: return launch_sweep_nt<1, 256, 0>(a, nchain, lds, s);
    case 1027: return launch_sweep_nt<1, 256, 1>(a, nchain, lds, s);
    case 2048: return launch_sweep_nt<0, 512, 0>(a, nchain, lds, s);
    case 2049: return launch_sweep_nt<0, 512, 1>(a, nchain, lds, s);
    case 2050: return launch_sweep_nt<1, 512, 0>(a, nchain, lds, s);
    case 2051: return launch_sweep_nt<1, 512, 1>(a, nchain, lds, s);
    case 3072: return launch_sweep_nt<0, 768, 0>(a, nchain, lds, s);
    case 3073: return launch_sweep_nt<0, 768, 1>(a, nchain, lds, s);
    case 3074: return launch_sweep_nt<1, 768, 0>(a, nchain, lds, s);
    case 3075: return launch_sweep_nt<1, 768, 1>(a, nchain, lds, s);
    case 4096: return launch_sweep_nt<0, 1024, 0>(a, nchain, lds, s);
    case 4097: return launch_sweep_nt<0, 1024, 1>(a, nchain, lds, s);
    case 4098: return launch_sweep_nt<1, 1024, 0>(a, nchain, lds, s);
    case 4099: return launch_sweep_nt<1, 1024, 1>(a, nchain, lds, s);
    default: return VOLDOR_EINVAL;
    }
}

void plan_sweep(Plan &p, std::vector<MultiLaunch> &out, const std::vector<WinRef> &w,
                const std::vector<int> &idx, float gamma, uint64_t seed, int64_t gsweep, int dir,
                int criterion)
{
    const int n = (int)idx.size();
    std::vector<SweepArgs> a(n);
    std::vector<int> nt(n);
    std::vector<size_t> lds(n);
    for (int k = 0; k < n; ++k) {
        const WinRef &r = w[idx[k]];
        sweep_args(r.c, r.depth, r.depth, r.X, r.d, r.e, gamma, seed, gsweep, dir, r.c->range, nullptr, criterion,
                   a[k], nt[k], lds[k]);
    }
    // one launch per (threads per chain, LDS bytes) class: a launch's LDS is
    // that of every chain in it, so no chain holds more than its own
    std::vector<bool> done(n, false);
    for (int k0 = 0; k0 < n; ++k0) {
        if (done[k0]) continue;
        std::vector<SweepArgs> sel;
        std::vector<int> first(1, 0);
        const int cls = nt[k0];
        const size_t lmax = lds[k0];
        for (int k = k0; k < n; ++k) {
            if (done[k] || nt[k] != cls || lds[k] != lmax) continue;
            done[k] = true;
            sel.push_back(a[k]);
            first.push_back(first.back() + ((dir & 1) ? a[k].W : a[k].H));
        }
        MultiLaunch l = {};
        l.kind = kMultiSweep;
        l.variant = (cls * 2 + (criterion ? 1 : 0)) * 2 + (sel[0].e.model ? 1 : 0);
        l.nwin = (int)sel.size();
        l.off = p.put(sel.data(), sel.size());
        l.off2 = p.put(first.data(), first.size());
        l.gx = first.back();
        l.lds = lmax;
        out.push_back(l);
    }
}

template <int CRIT, int NT, int MODEL>
static int launch_sweep_multi_nt(const MultiLaunch &m, const unsigned char *dev, hipStream_t s)
{
    if (m.lds > 65536 &&
        hipFuncSetAttribute((const void *)k_sweep_multi<CRIT, NT, MODEL>, hipFuncAttributeMaxDynamicSharedMemorySize,
                            (int)m.lds) != hipSuccess)
        return VOLDOR_EDEVICE;
    hipLaunchKernelGGL((k_sweep_multi<CRIT, NT, MODEL>), dim3(m.gx), dim3(NT), m.lds, s,
                       (const SweepArgs *)(dev + m.off), (const int *)(dev + m.off2), m.nwin);
    return hipGetLastError() == hipSuccess ? 0 : VOLDOR_EDEVICE;
}

void plan_rigidness(Plan &p, std::vector<MultiLaunch> &out, const std::vector<WinRef> &w,
                    const std::vector<int> &idx, bool gauge, const std::vector<double *> &ll)
{
    const int n = (int)idx.size();
    std::vector<RigArgs> a(n);
    std::vector<LLArgs> r(n);
    int gx = 0;
    for (int k = 0; k < n; ++k) {
        const WinRef &wr = w[idx[k]];
        RigArgs &x = a[k];
        x.theta = wr.depth;
        x.theta_gauge = gauge ? wr.depth : nullptr;
        x.rel = gauge ? wr.poses : nullptr;
        x.flows = wr.X;
        x.Mcum = wr.c->Mcum;
        x.status = wr.c->status;
        x.r = gauge ? wr.rig : nullptr;
        x.ell = nullptr;
        x.logrho = nullptr;
        x.logmu = nullptr;
        x.ll_part = gauge ? nullptr : wr.c->ll_part;
        x.T = wr.d.T;
        x.H = wr.d.H;
        x.W = wr.d.W;
        x.e = wr.e;
        const int HW = wr.d.H * wr.d.W;
        x.nblk = std::min((HW + 255) / 256, kLLBlocks);
        gx = std::max(gx, x.nblk);
        r[k].part = wr.c->ll_part;
        r[k].status = wr.c->status;
        r[k].out = gauge ? nullptr : ll[k];
        r[k].n = x.nblk;
    }
    MultiLaunch l = {};
    l.kind = kMultiRig;
    l.nwin = n;
    l.off = p.put(a.data(), n);
    l.gx = gx;
    out.push_back(l);
    if (!gauge) {
        l.kind = kMultiLL;
        l.off = p.put(r.data(), n);
        l.gx = 1;
        out.push_back(l);
    }
}

int launch_sweep_multi(const MultiLaunch &m, const unsigned char *dev, hipStream_t s)
{
    if (m.nwin < 1) return 0;
    if (m.kind == kMultiRig) {
        hipLaunchKernelGGL(k_rigidness_multi, dim3(m.gx, m.nwin), dim3(256), 0, s, (const RigArgs *)(dev + m.off));
        return hipGetLastError() == hipSuccess ? 0 : VOLDOR_EDEVICE;
    }
    if (m.kind == kMultiLL) {
        hipLaunchKernelGGL(k_ll_reduce_multi, dim3(1, m.nwin), dim3(256), 0, s, (const LLArgs *)(dev + m.off));
        return hipGetLastError() == hipSuccess ? 0 : VOLDOR_EDEVICE;
    }
    if (m.kind != kMultiSweep) return VOLDOR_EINVAL;
    switch (m.variant) {
    case 1024: return launch_sweep_multi_nt<0, 256, 0>(m, dev, s);
    case 1025: return launch_sweep_multi_nt<0, 256, 1>(m, dev, s);
    case 1026: return launch_sweep_multi_nt<1, 256, 0>(m, dev, s);
    case 1027: return launch_sweep_multi_nt<1, 256, 1>(m, dev, s);
    case 2048: return launch_sweep_multi_nt<0, 512, 0>(m, dev, s);
    case 2049: return launch_sweep_multi_nt<0, 512, 1>(m, dev, s);
    case 2050: return launch_sweep_multi_nt<1, 512, 0>(m, dev, s);
    case 2051: return launch_sweep_multi_nt<1, 512, 1>(m, dev, s);
    case 3072: return launch_sweep_multi_nt<0, 768, 0>(m, dev, s);
    case 3073: return launch_sweep_multi_nt<0, 768, 1>(m, dev, s);
    case 3074: return launch_sweep_multi_nt<1, 768, 0>(m, dev, s);
    case 3075: return launch_sweep_multi_nt<1, 768, 1>(m, dev, s);
    case 4096: return launch_sweep_multi_nt<0, 1024, 0>(m, dev, s);
    case 4097: return launch_sweep_multi_nt<0, 1024, 1>(m, dev, s);
    case 4098: return launch_sweep_multi_nt<1, 1024, 0>(m, dev, s);
    case 4099: return launch_sweep_multi_nt<1, 1024, 1>(m, dev, s);
    default: return VOLDOR_EINVAL;
    }
}

int launch_rigidness(voldor_ctx *c, const float *theta, const float2 *flows, const WinDims &d,
                     const EmisParams &e, float *r, float *ell, float *logrho, float *logmu,
                     double *ll_out, hipStream_t s, float *theta_gauge, const double *rel_poses)
{
    RigArgs a;
    a.theta = theta;
    a.theta_gauge = theta_gauge;
    a.rel = rel_poses;
    a.flows = flows;
    a.Mcum = c->Mcum;
    a.status = c->status;
    a.r = r;
    a.ell = ell;
    a.logrho = logrho;
    a.logmu = logmu;
    a.ll_part = ll_out ? c->ll_part : nullptr;
    a.T = d.T;
    a.H = d.H;
    a.W = d.W;
    a.e = e;
    const int HW = d.H * d.W;
    int blocks = (HW + 255) / 256;
    if (blocks > kLLBlocks) blocks = kLLBlocks;
    a.nblk = blocks;
    hipLaunchKernelGGL(k_rigidness, dim3(blocks), dim3(256), 0, s, a);
    if (ll_out) hipLaunchKernelGGL(k_ll_reduce, dim3(1), dim3(256), 0, s, c->ll_part, blocks, c->status, ll_out);
    return hipGetLastError() == hipSuccess ? 0 : VOLDOR_EDEVICE;
}

// The flow planes transposed ([T][H][W] -> [T][W][H]) through 32 x 32 LDS
// tiles, for the column sweeps' gathers; once per window.
__global__ void __launch_bounds__(256) k_transpose_flows(const float2 *__restrict__ X, float2 *__restrict__ Xt,
                                                         int H, int W)
{
    __shared__ float2 tile[32][33];
    const size_t plane = (size_t)H * W * blockIdx.z;
    const int x0 = blockIdx.x * 32, y0 = blockIdx.y * 32;
    for (int j = threadIdx.y; j < 32; j += 8) {
        const int x = x0 + threadIdx.x, y = y0 + j;
        if (x < W && y < H) tile[j][threadIdx.x] = X[plane + (size_t)y * W + x];
    }
    __syncthreads();
    for (int j = threadIdx.y; j < 32; j += 8) {
        const int y = y0 + threadIdx.x, x = x0 + j;
        if (x < W && y < H) Xt[plane + (size_t)x * H + y] = tile[threadIdx.x][j];
    }
}

int launch_transpose_flows(voldor_ctx *c, const float2 *flows, int T, int H, int W, hipStream_t s)
{
    if (T > c->T_max || H > c->H_max || W > c->W_max) return VOLDOR_EINVAL;
    hipLaunchKernelGGL(k_transpose_flows, dim3((W + 31) / 32, (H + 31) / 32, T), dim3(32, 8), 0, s, flows,
                       c->flows_t, H, W);
    return hipGetLastError() == hipSuccess ? 0 : VOLDOR_EDEVICE;
}

int launch_philox(const uint64_t *ctr, uint64_t k0, uint64_t k1, uint64_t *out, int n, hipStream_t s)
{
    if (n <= 0) return 0;
    hipLaunchKernelGGL(k_philox, dim3((n + 255) / 256), dim3(256), 0, s, ctr, k0, k1, out, n);
    return hipGetLastError() == hipSuccess ? 0 : VOLDOR_EDEVICE;
}

}  // namespace vo
