// vo_sweep.hip -- FP32 directional sweep of the depth/rigidness update
// (E-step forward-backward, Eq. 11-14; M-step maximum-inlier sampling and
// propagation, Eq. 10 and Fig. 5), the unsmoothed rigidness with the
// log-likelihood of Eq. 3, and the Philox test kernel.
//
// One workgroup owns one chain (an image row for directions 0/2, a column for
// 1/3) for all T frames, so every phase of a sweep runs out of LDS:
//   A  ell_t(prev) and r_t(prev) for every chain position and frame;
//   B  forward-backward per frame as a segmented scan of 2x2 transfer
//      matrices (one segment per thread, serial over the segments);
//   S  scores of the previous depth and of the random sample under q, the
//      local best a_j = best(prev, sample);
//   C  for every position k, how far its local best would survive as the
//      propagated neighbour: next(k) = first j > k where it loses;
//   D  the propagation path 0 -> next(0) -> next(next(0)) ... found by pointer
//      doubling; every position takes the local best of the last path node
//      at or before it.
// C/D reproduce the serial left-to-right walk exactly (each score is the same
// FP32 function of position and value), without a serial dependency chain.
#include "vo_internal.hpp"

namespace vo {

__device__ __forceinline__ int chain_pixel(int dir, int H, int W, int c, int k)
{
    switch (dir) {
    case 0: return c * W + k;
    case 1: return k * W + c;
    case 2: return c * W + (W - 1 - k);
    default: return (H - 1 - k) * W + c;
    }
}

// Emission terms of depth th at pixel (x, y) for frame t (1..T): returns the
// log-odds d = log(mu/rho), or +nan when the observation is missing.
__device__ __forceinline__ float frame_log_odds(const FrameF *fr, const float2 *__restrict__ flows,
                                                int H, int W, const EmisParams &e, int x, int y,
                                                float xh, float yh, float th, int t, float &px0,
                                                float &py0, bool &ok0)
{
    // px0/py0/ok0 carry pi_{t-1} - pixel between consecutive frames
    float dx1, dy1;
    const bool ok1 = displacement(fr[t], xh, yh, th, e.fx, e.fy, dx1, dy1);
    float d = __int_as_float(0x7fc00000);
    if (ok0 && ok1) {
        float vu, vv;
        const float2 *X = flows + (size_t)(t - 1) * H * W;
        if (sample_flow(X, H, W, (float)x + px0, (float)y + py0, vu, vv)) {
            const float rx = (dx1 - px0) - vu, ry = (dy1 - py0) - vv;
            d = log_mu_over_rho(rx, ry, vu, vv, e);
        }
    }
    px0 = dx1;
    py0 = dy1;
    ok0 = ok1;
    return d;
}

// MIE score sum_t q_t ell_t(th) at chain position k (q in LDS, [T][L]).
__device__ __forceinline__ float mie_score(const FrameF *fr, const float2 *__restrict__ flows,
                                           int T, int H, int W, const EmisParams &e, int x, int y,
                                           float xh, float yh, float th, const float *q, int L,
                                           int k)
{
    float px0 = 0.0f, py0 = 0.0f, s = 0.0f;
    bool ok0 = th > 0.0f;
    for (int t = 1; t <= T; ++t) {
        const float d = frame_log_odds(fr, flows, H, W, e, x, y, xh, yh, th, t, px0, py0, ok0);
        const float ell = isnan(d) ? -0.69314718055994531f : emis_from_d(d).ell;
        s = fmaf(q[(t - 1) * L + k], ell, s);
    }
    return s;
}

struct SweepArgs {
    const float *theta_in;
    float *theta_out;
    const float2 *flows;
    const FrameF *frames;
    const double *range;   // d_lo, d_hi (device)
    float *q_out;
    const int *status;
    int T, H, W, dir;
    EmisParams e;
    float gamma;
    uint64_t seed;
    int64_t gsweep;
};

__global__ void __launch_bounds__(kBlock) k_sweep(SweepArgs a)
{
    if (a.status && *a.status != kStatusOk) return;
    extern __shared__ float lds[];
    __shared__ FrameF fr[kTMax + 1];
    __shared__ float seg_f[kBlock][4], seg_b[kBlock][4];  // per-thread segment matrices
    __shared__ float fin[kBlock][2], bout[kBlock][2];      // segment boundary messages

    const int T = a.T, H = a.H, W = a.W, dir = a.dir;
    const int L = (dir & 1) ? H : W;
    const int tid = threadIdx.x;
    // XCD-aware chain order: consecutive chains on one XCD share its L2
    const int nchain = gridDim.x;
    const int xcd = blockIdx.x & 7, slot = blockIdx.x >> 3;
    const int per = (nchain + 7) >> 3;
    int chain = xcd * per + slot;
    {
        // map the 8 interleaved ranges back onto [0, nchain) without holes
        const int full = nchain - (per - 1) * 8;  // XCDs that get `per` chains
        if (xcd < full) chain = xcd * per + slot;
        else chain = full * per + (xcd - full) * (per - 1) + slot;
    }

    float *th = lds;                       // [L] previous depth
    float *sm = th + L;                    // [L] random sample
    float *lq = sm + L;                    // [T][L] ell(prev); later overlay
    const int over = (T > 8 ? T : 8);
    float *fq = lq + over * L;             // [T][L] r -> forward message -> q

    for (int i = tid; i < (T + 1) * 12; i += kBlock) ((float *)fr)[i] = ((const float *)a.frames)[i];

    const float d_lo = (float)a.range[0];
    const float lrange = (float)(log(a.range[1]) - log(a.range[0]));
    const float llo = logf(d_lo);
    for (int k = tid; k < L; k += kBlock) {
        const int j = chain_pixel(dir, H, W, chain, k);
        th[k] = a.theta_in[j];
        uint64_t c[4] = {(uint64_t)a.gsweep, (uint64_t)j, 0ull, 0ull};
        philox4x64_10(c, a.seed, kDepthStream);
        const float u = ((float)(uint32_t)(c[0] >> 32) + 0.5f) * 2.3283064365386963e-10f;
        sm[k] = expf(fmaf(u, lrange, llo));
    }
    __syncthreads();

    // ---- A: emissions of the previous depth
    for (int k = tid; k < L; k += kBlock) {
        const int j = chain_pixel(dir, H, W, chain, k);
        const int x = j % W, y = j / W;
        const float xh = ((float)x - a.e.cx) / a.e.fx, yh = ((float)y - a.e.cy) / a.e.fy;
        const float t0 = th[k];
        float px0 = 0.0f, py0 = 0.0f;
        bool ok0 = t0 > 0.0f;
        for (int t = 1; t <= T; ++t) {
            const float d = frame_log_odds(fr, a.flows, H, W, a.e, x, y, xh, yh, t0, t, px0, py0, ok0);
            Emis m;
            if (isnan(d)) { m.ell = -0.69314718055994531f; m.r = 0.5f; }
            else m = emis_from_d(d);
            lq[(t - 1) * L + k] = m.ell;
            fq[(t - 1) * L + k] = m.r;
        }
    }
    __syncthreads();

    // ---- B: forward-backward per frame, one segment per thread
    const int nseg = kBlock / T;
    const int seglen = (L + nseg - 1) / nseg;
    const float g = a.gamma, gc = 1.0f - a.gamma;
    const int ft = tid / nseg, fs = tid - ft * nseg;
    const bool fb_thread = ft < T;
    const int s0 = min(fs * seglen, L), s1 = min(s0 + seglen, L);
    if (fb_thread) {
        const float *rr = fq + ft * L;
        // forward: A_k = diag(r, 1-r) Gamma ; product A_{s1-1} ... A_{s0}
        float F00 = 1, F01 = 0, F10 = 0, F11 = 1;
        for (int k = s0; k < s1; ++k) {
            const float r1 = rr[k], r0 = 1.0f - r1;
            const float a00 = r1 * g, a01 = r1 * gc, a10 = r0 * gc, a11 = r0 * g;
            const float n00 = a00 * F00 + a01 * F10, n01 = a00 * F01 + a01 * F11;
            const float n10 = a10 * F00 + a11 * F10, n11 = a10 * F01 + a11 * F11;
            const float inv = 1.0f / (n00 + n01 + n10 + n11);
            F00 = n00 * inv; F01 = n01 * inv; F10 = n10 * inv; F11 = n11 * inv;
        }
        // backward: G_k = Gamma diag(r, 1-r) ; product G_{s0} ... G_{s1-1}
        float B00 = 1, B01 = 0, B10 = 0, B11 = 1;
        for (int k = s1 - 1; k >= s0; --k) {
            const float r1 = rr[k], r0 = 1.0f - r1;
            const float g00 = g * r1, g01 = gc * r0, g10 = gc * r1, g11 = g * r0;
            const float n00 = g00 * B00 + g01 * B10, n01 = g00 * B01 + g01 * B11;
            const float n10 = g10 * B00 + g11 * B10, n11 = g10 * B01 + g11 * B11;
            const float inv = 1.0f / (n00 + n01 + n10 + n11);
            B00 = n00 * inv; B01 = n01 * inv; B10 = n10 * inv; B11 = n11 * inv;
        }
        seg_f[tid][0] = F00; seg_f[tid][1] = F01; seg_f[tid][2] = F10; seg_f[tid][3] = F11;
        seg_b[tid][0] = B00; seg_b[tid][1] = B01; seg_b[tid][2] = B10; seg_b[tid][3] = B11;
    }
    __syncthreads();
    if (tid < T) {
        const int base = tid * nseg;
        float m1 = 0.5f, m0 = 0.5f;  // m_f(-1)
        for (int s = 0; s < nseg; ++s) {
            fin[base + s][0] = m1;
            fin[base + s][1] = m0;
            const float *F = seg_f[base + s];
            const float n1 = F[0] * m1 + F[1] * m0, n0 = F[2] * m1 + F[3] * m0;
            const float inv = 1.0f / (n1 + n0);
            m1 = n1 * inv;
            m0 = n0 * inv;
        }
        float b1 = 0.5f, b0 = 0.5f;  // m_b(L-1)
        for (int s = nseg - 1; s >= 0; --s) {
            bout[base + s][0] = b1;
            bout[base + s][1] = b0;
            const float *B = seg_b[base + s];
            const float n1 = B[0] * b1 + B[1] * b0, n0 = B[2] * b1 + B[3] * b0;
            const float inv = 1.0f / (n1 + n0);
            b1 = n1 * inv;
            b0 = n0 * inv;
        }
    }
    __syncthreads();
    if (fb_thread && s0 < s1) {
        float *qq = fq + ft * L;
        const float *ll = lq + ft * L;
        float f1 = fin[tid][0], f0 = fin[tid][1];
        for (int k = s0; k < s1; ++k) {
            const float r1 = qq[k], r0 = 1.0f - r1;
            const float p1 = g * f1 + gc * f0, p0 = gc * f1 + g * f0;
            const float n1 = r1 * p1, n0 = r0 * p0;
            const float inv = 1.0f / (n1 + n0);
            f1 = n1 * inv;
            f0 = n0 * inv;
            qq[k] = f1;
        }
        float b1 = bout[tid][0], b0 = bout[tid][1];
        for (int k = s1 - 1; k >= s0; --k) {
            const float ff1 = qq[k], ff0 = 1.0f - ff1;
            const float n1 = ff1 * b1, n0 = ff0 * b0;
            qq[k] = n1 / (n1 + n0);
            if (k > s0) {
                const float r1 = __expf(ll[k]), r0 = 1.0f - r1;
                const float e1 = r1 * b1, e0 = r0 * b0;
                const float m1 = g * e1 + gc * e0, m0 = gc * e1 + g * e0;
                const float inv = 1.0f / (m1 + m0);
                b1 = m1 * inv;
                b0 = m0 * inv;
            }
        }
    }
    __syncthreads();
    if (a.q_out) {
        for (int i = tid; i < T * L; i += kBlock) {
            const int t = i / L, k = i - t * L;
            a.q_out[(size_t)t * H * W + chain_pixel(dir, H, W, chain, k)] = fq[i];
        }
    }

    // ---- S: score of the previous depth (ell from A), kept in registers
    float sprev[kMaxPerThread];
#pragma unroll
    for (int i = 0; i < kMaxPerThread; ++i) {
        const int k = tid + i * kBlock;
        float s = 0.0f;
        if (k < L)
            for (int t = 0; t < T; ++t) s = fmaf(fq[t * L + k], lq[t * L + k], s);
        sprev[i] = s;
    }
    __syncthreads();  // lq becomes the overlay below
    float *aval = lq;                      // [L] local best value
    float *sa = aval + L;                  // [L] its score
    int *flg = (int *)(sa + L);            // [L] 1 if the sample is the local best
    int *nxt = flg + L;                    // [L] next(k)
    int *J0 = nxt + L, *J1 = J0 + L;       // [L] doubling pointers
    int *mark = J1 + L;                    // [L] on the propagation path
    float *thn = (float *)(mark + L);      // [L] new depth
#pragma unroll
    for (int i = 0; i < kMaxPerThread; ++i) {
        const int k = tid + i * kBlock;
        if (k < L) {
            const int j = chain_pixel(dir, H, W, chain, k);
            const int x = j % W, y = j / W;
            const float xh = ((float)x - a.e.cx) / a.e.fx, yh = ((float)y - a.e.cy) / a.e.fy;
            const float ss = mie_score(fr, a.flows, T, H, W, a.e, x, y, xh, yh, sm[k], fq, L, k);
            const bool smp = ss > sprev[i];
            aval[k] = smp ? sm[k] : th[k];
            sa[k] = smp ? ss : sprev[i];
            flg[k] = smp ? 1 : 0;
            mark[k] = (k == 0);
        }
    }
    __syncthreads();

    // ---- C: survival of every local best as the propagated neighbour
    for (int k = tid; k < L; k += kBlock) {
        const float v = aval[k];
        int jpos = k + 1;
        for (; jpos < L; ++jpos) {
            const int j = chain_pixel(dir, H, W, chain, jpos);
            const int x = j % W, y = j / W;
            const float xh = ((float)x - a.e.cx) / a.e.fx, yh = ((float)y - a.e.cy) / a.e.fy;
            const float s = mie_score(fr, a.flows, T, H, W, a.e, x, y, xh, yh, v, fq, L, jpos);
            // the neighbour beats the previous depth only strictly, and the
            // sample on ties (previous > neighbour > sample)
            const bool win = flg[jpos] ? (s >= sa[jpos]) : (s > sa[jpos]);
            if (!win) break;
        }
        nxt[k] = jpos;
        J0[k] = jpos;
    }
    __syncthreads();

    // ---- D: nodes reachable from 0 through next(), by pointer doubling
    int *Jc = J0, *Jn = J1;
    for (int span = 1; span < L; span <<= 1) {
        for (int k = tid; k < L; k += kBlock) {
            const int to = Jc[k];
            if (mark[k] && to < L) mark[to] = 1;
        }
        __syncthreads();
        for (int k = tid; k < L; k += kBlock) {
            const int to = Jc[k];
            Jn[k] = to < L ? Jc[to] : L;
        }
        __syncthreads();
        int *tmp = Jc; Jc = Jn; Jn = tmp;
    }
    for (int k = tid; k < L; k += kBlock) {
        const int to = Jc[k];
        if (mark[k] && to < L) mark[to] = 1;
    }
    __syncthreads();
    for (int k = tid; k < L; k += kBlock) {
        if (mark[k]) {
            const int e = nxt[k];
            const float v = aval[k];
            for (int j = k; j < e; ++j) thn[j] = v;
        }
    }
    __syncthreads();
    for (int k = tid; k < L; k += kBlock) a.theta_out[chain_pixel(dir, H, W, chain, k)] = thn[k];
}

// ---------------------------------------------------------------------------
// unsmoothed rigidness W_t = r_t(theta) (last row of Table 1), optional dense
// emission maps, optional log-likelihood partial sums of Eq. 3
// ---------------------------------------------------------------------------
struct RigArgs {
    const float *theta;
    const float2 *flows;
    const FrameF *frames;
    const int *status;
    float *r, *ell, *logrho, *logmu;
    double *ll_part;
    int T, H, W;
    EmisParams e;
};

__global__ void __launch_bounds__(256) k_rigidness(RigArgs a)
{
    if (a.status && *a.status != kStatusOk) return;
    __shared__ FrameF fr[kTMax + 1];
    __shared__ double red[2][256];
    for (int i = threadIdx.x; i < (a.T + 1) * 12; i += blockDim.x)
        ((float *)fr)[i] = ((const float *)a.frames)[i];
    __syncthreads();
    const int HW = a.H * a.W;
    double acc = 0.0, mass = 0.0;
    for (int j = blockIdx.x * blockDim.x + threadIdx.x; j < HW; j += gridDim.x * blockDim.x) {
        const int x = j % a.W, y = j / a.W;
        const float xh = ((float)x - a.e.cx) / a.e.fx, yh = ((float)y - a.e.cy) / a.e.fy;
        const float th = a.theta[j];
        float px0 = 0.0f, py0 = 0.0f;
        bool ok0 = th > 0.0f;
        for (int t = 1; t <= a.T; ++t) {
            // same steps as frame_log_odds, keeping the pieces of log rho / log mu
            float dx1, dy1;
            const bool ok1 = displacement(fr[t], xh, yh, th, a.e.fx, a.e.fy, dx1, dy1);
            float r = 0.5f, ell = -0.69314718055994531f, lr = 0.0f, lm = 0.0f;
            if (ok0 && ok1) {
                float vu, vv;
                const float2 *X = a.flows + (size_t)(t - 1) * HW;
                if (sample_flow(X, a.H, a.W, (float)x + px0, (float)y + py0, vu, vv)) {
                    const float rx = (dx1 - px0) - vu, ry = (dy1 - py0) - vv;
                    const float d = log_mu_over_rho(rx, ry, vu, vv, a.e);
                    const Emis m = emis_from_d(d);
                    r = m.r;
                    ell = m.ell;
                    if (a.logrho || a.logmu || a.ll_part) {
                        const float vn = sqrtf(fmaf(vu, vu, vv * vv));
                        const float la = fmaf(a.e.a2, vn, a.e.log_a1);
                        const float beta = fmaxf(fmaf(a.e.b1, vn, a.e.b2), a.e.beta_min);
                        const float x2 = fmaxf(fmaf(rx, rx, ry * ry), a.e.x_floor);
                        const float s1 = __logf(x2) - la;
                        const float lb = __logf(beta) - la;
                        lr = lb + (beta - 1.0f) * s1 - 2.0f * softplus(beta * s1);
                        lm = lr + d;
                        const double w = r;
                        const double term = w * (double)lr + (1.0 - w) * (double)lm;
                        acc += term;
                        mass += fabs(term);
                    }
                }
            }
            px0 = dx1;
            py0 = dy1;
            ok0 = ok1;
            const size_t o = (size_t)(t - 1) * HW + j;
            if (a.r) a.r[o] = r;
            if (a.ell) a.ell[o] = ell;
            if (a.logrho) a.logrho[o] = lr;
            if (a.logmu) a.logmu[o] = lm;
        }
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

// fixed-order sum of the per-block partial sums
__global__ void k_ll_reduce(const double *part, int n, const int *status, double *out)
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

// FP32 frames (R - I, t) from the FP64 cumulative poses
__global__ void k_frames(const double *M, FrameF *fr, int T)
{
    const int t = threadIdx.x;
    if (t > T) return;
    const double *m = M + 12 * t;
    for (int i = 0; i < 9; ++i) fr[t].D[i] = (float)(m[i] - ((i == 0 || i == 4 || i == 8) ? 1.0 : 0.0));
    for (int i = 0; i < 3; ++i) fr[t].t[i] = (float)m[9 + i];
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
size_t sweep_lds_bytes(int T, int L)
{
    const int over = T > 8 ? T : 8;
    return (size_t)(2 + over + T) * L * sizeof(float);
}

int launch_frames(voldor_ctx *c, int T, hipStream_t s)
{
    hipLaunchKernelGGL(k_frames, dim3(1), dim3(64), 0, s, c->Mcum, c->frames, T);
    return hipGetLastError() == hipSuccess ? 0 : VOLDOR_EDEVICE;
}

int launch_sweep(voldor_ctx *c, const float *theta_in, float *theta_out, const float2 *flows,
                 const WinDims &d, const EmisParams &e, float gamma, uint64_t seed, int64_t gsweep,
                 int dir, const double *range_dev, float *q_out, hipStream_t s)
{
    const int L = (dir & 1) ? d.H : d.W;
    const int nchain = (dir & 1) ? d.W : d.H;
    const size_t lds = sweep_lds_bytes(d.T, L);
    if (L > kBlock * kMaxPerThread) return VOLDOR_EINVAL;
    SweepArgs a;
    a.theta_in = theta_in;
    a.theta_out = theta_out;
    a.flows = flows;
    a.frames = c->frames;
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
    if (lds > 65536 &&
        hipFuncSetAttribute((const void *)k_sweep, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds) != hipSuccess)
        return VOLDOR_EDEVICE;
    hipLaunchKernelGGL(k_sweep, dim3(nchain), dim3(kBlock), lds, s, a);
    return hipGetLastError() == hipSuccess ? 0 : VOLDOR_EDEVICE;
}

int launch_rigidness(voldor_ctx *c, const float *theta, const float2 *flows, const WinDims &d,
                     const EmisParams &e, float *r, float *ell, float *logrho, float *logmu,
                     double *ll_out, hipStream_t s)
{
    RigArgs a;
    a.theta = theta;
    a.flows = flows;
    a.frames = c->frames;
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
    hipLaunchKernelGGL(k_rigidness, dim3(blocks), dim3(256), 0, s, a);
    if (ll_out) hipLaunchKernelGGL(k_ll_reduce, dim3(1), dim3(256), 0, s, c->ll_part, blocks, c->status, ll_out);
    return hipGetLastError() == hipSuccess ? 0 : VOLDOR_EDEVICE;
}

int launch_philox(const uint64_t *ctr, uint64_t k0, uint64_t k1, uint64_t *out, int n, hipStream_t s)
{
    if (n <= 0) return 0;
    hipLaunchKernelGGL(k_philox, dim3((n + 255) / 256), dim3(256), 0, s, ctr, k0, k1, out, n);
    return hipGetLastError() == hipSuccess ? 0 : VOLDOR_EDEVICE;
}

}  // namespace vo
