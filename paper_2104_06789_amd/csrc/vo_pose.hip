// vo_pose.hip -- FP64 pose step of one frame (Sec. 5.2, Eq. 15-19):
//   k_pose_groups  S random pixel triples -> 3-D points in camera t-1 and
//                  bearings in camera t through the flow X_t -> P3P roots in
//                  front of both cameras -> se(3) samples weighted by the
//                  product of the three rigidness values;
//   k_pose_seed    kernel density of each start candidate (previous pose and
//                  the first samples in group order) over all samples;
//   k_pose_ms      densest candidate, Gaussian mean-shift to the mode,
//                  T_t = exp(p*), M_t = T_t o M_{t-1};
// plus the scale gauge |t_1| = 1.
#include "vo_internal.hpp"


namespace vo {

struct GroupArgs {
    const float *theta;
    const float *rig;
    const float2 *flows;
    const double *Mprev;   // M_{t-1}
    double *samples;       // SoA [8][ns]: p (6), weight, valid; slot 4g+r of group g
    int *gcnt;             // [S] valid samples of each group
    const int *status;
    WinDims d;
    int S, t, it, ns;
    uint64_t seed;
};

__device__ __forceinline__ bool flow_bilinear_d(const float2 *X, int H, int W, double px, double py,
                                                double &u, double &v)
{
    if (!(px >= 0.0 && px <= (double)(W - 1) && py >= 0.0 && py <= (double)(H - 1))) return false;
    int x0 = (int)floor(px), y0 = (int)floor(py);
    x0 = min(x0, W - 2);
    y0 = min(y0, H - 2);
    const double ax = px - x0, ay = py - y0;
    const float2 a = X[(size_t)y0 * W + x0], b = X[(size_t)y0 * W + x0 + 1];
    const float2 c = X[(size_t)(y0 + 1) * W + x0], dd = X[(size_t)(y0 + 1) * W + x0 + 1];
    if (!isfinite(a.x + a.y + b.x + b.y + c.x + c.y + dd.x + dd.y)) return false;
    const double w00 = (1 - ax) * (1 - ay), w01 = ax * (1 - ay), w10 = (1 - ax) * ay, w11 = ax * ay;
    u = w00 * a.x + w01 * b.x + w10 * c.x + w11 * dd.x;
    v = w00 * a.y + w01 * b.y + w10 * c.y + w11 * dd.y;
    return true;
}

__global__ void __launch_bounds__(64) k_pose_groups(GroupArgs a)
{
    if (a.status && *a.status != kStatusOk) return;
    const int g = blockIdx.x * blockDim.x + threadIdx.x;
    if (g >= a.S) return;
    double *out = a.samples + (size_t)4 * g;
    for (int c = 0; c < 8; ++c)
        for (int r = 0; r < 4; ++r) out[(size_t)c * a.ns + r] = 0.0;
    a.gcnt[g] = 0;
    const int H = a.d.H, W = a.d.W;
    const int64_t HW = (int64_t)H * W;
    int64_t j[3];
    bool drawn = false;
    for (int att = 0; att < 8 && !drawn; ++att) {
        uint64_t c[4] = {(uint64_t)a.it, (uint64_t)a.t, (uint64_t)g, (uint64_t)att};
        philox4x64_10(c, a.seed, kPoseStream);
        for (int k = 0; k < 3; ++k) j[k] = u32_to_index((uint32_t)(c[k] >> 32), HW);
        drawn = j[0] != j[1] && j[0] != j[2] && j[1] != j[2];
    }
    if (!drawn) return;
    double P[9], f[9], w = 1.0;
    const double *M = a.Mprev;
    const float2 *X = a.flows + (size_t)(a.t - 1) * HW;
    for (int k = 0; k < 3; ++k) {
        const int x = (int)(j[k] % W), y = (int)(j[k] / W);
        const double th = (double)a.theta[j[k]];
        const double r[3] = {(x - a.d.cx) / a.d.fx, (y - a.d.cy) / a.d.fy, 1.0};
        double Q[3];
        mv3(M, r, Q);
        for (int c = 0; c < 3; ++c) Q[c] = th * Q[c] + M[9 + c];
        if (!(Q[2] > 0)) return;
        double u0 = a.d.fx * Q[0] / Q[2] + a.d.cx, v0 = a.d.fy * Q[1] / Q[2] + a.d.cy;
        if (a.t == 1) { u0 = x; v0 = y; }   // pi_0 is the pixel itself
        double fu, fv;
        if (!flow_bilinear_d(X, H, W, u0, v0, fu, fv)) return;
        const double bx = (u0 + fu - a.d.cx) / a.d.fx, by = (v0 + fv - a.d.cy) / a.d.fy;
        const double nb = sqrt(bx * bx + by * by + 1.0);
        P[3 * k] = Q[0];
        P[3 * k + 1] = Q[1];
        P[3 * k + 2] = Q[2];
        f[3 * k] = bx / nb;
        f[3 * k + 1] = by / nb;
        f[3 * k + 2] = 1.0 / nb;
        if (a.rig) w *= (double)a.rig[(size_t)(a.t - 1) * HW + j[k]];
    }
    double Rs[36], ts[12];
    const int nr = p3p_solve(P, f, Rs, ts);
    int keep[4], nk = 0;
    double key[4][4];
    for (int i = 0; i < nr; ++i) {
        bool front = true;
        for (int k = 0; k < 3; ++k) {
            const double z = Rs[9 * i + 6] * P[3 * k] + Rs[9 * i + 7] * P[3 * k + 1] +
                             Rs[9 * i + 8] * P[3 * k + 2] + ts[3 * i + 2];
            front = front && z > 0;
        }
        if (!front) continue;
        key[nk][0] = rot_angle(Rs + 9 * i);
        key[nk][1] = ts[3 * i];
        key[nk][2] = ts[3 * i + 1];
        key[nk][3] = ts[3 * i + 2];
        keep[nk++] = i;
    }
    // canonical order: rotation angle, then t_x, t_y, t_z (insertion sort)
    for (int a1 = 1; a1 < nk; ++a1) {
        for (int b1 = a1; b1 > 0; --b1) {
            bool less = false;
            for (int c = 0; c < 4; ++c) {
                if (key[b1][c] < key[b1 - 1][c]) { less = true; break; }
                if (key[b1][c] > key[b1 - 1][c]) break;
            }
            if (!less) break;
            for (int c = 0; c < 4; ++c) { const double tmp = key[b1][c]; key[b1][c] = key[b1 - 1][c]; key[b1 - 1][c] = tmp; }
            const int tk = keep[b1]; keep[b1] = keep[b1 - 1]; keep[b1 - 1] = tk;
        }
    }
    int nv = 0;
    for (int s = 0; s < nk; ++s) {
        const int i = keep[s];
        double p[6];
        se3_log(Rs + 9 * i, ts + 3 * i, p);
        bool fin = true;
        for (int c = 0; c < 6; ++c) fin = fin && isfinite(p[c]);
        if (!fin) continue;
        double *o = out + nv;   // valid samples fill the group's slots without gaps
        for (int c = 0; c < 6; ++c) o[(size_t)c * a.ns] = p[c];
        o[(size_t)6 * a.ns] = w;
        o[(size_t)7 * a.ns] = 1.0;
        ++nv;
    }
    a.gcnt[g] = nv;
}

__device__ __forceinline__ double mahal2(const double *a, const double *b, double is2t, double is2r)
{
    const double d0 = a[0] - b[0], d1 = a[1] - b[1], d2 = a[2] - b[2];
    const double d3 = a[3] - b[3], d4 = a[4] - b[4], d5 = a[5] - b[5];
    return (d0 * d0 + d1 * d1 + d2 * d2) * is2t + (d3 * d3 + d4 * d4 + d5 * d5) * is2r;
}

template <int NT>
__device__ __forceinline__ double block_sum(double v, double *red)
{
    for (int off = 32; off > 0; off >>= 1) v += __shfl_down(v, off, 64);
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    __syncthreads();
    if (lane == 0) red[wv] = v;
    __syncthreads();
    double s = 0.0;
    if (threadIdx.x == 0) {
        for (int i = 0; i < NT / 64; ++i) s += red[i];
        red[NT / 64] = s;
    }
    __syncthreads();
    return red[NT / 64];
}

// Dense copy of the valid samples in (group, root) order: SoA dense[c][i],
// c = 0..5 the se(3) coordinates, c = 6 the weight; info = (N, sum w, groups).
struct CompactArgs {
    const double *samples;  // SoA [8][ns]
    const int *gcnt;        // [S]
    double *dense;          // [7][stride]
    double *info;           // [4]
    const int *status;
    int S, ns, stride;
};

constexpr int kCompactThreads = 1024;
constexpr int kCompactGroups = kMaxGroups / kCompactThreads;  // groups per thread (max)

__global__ void __launch_bounds__(kCompactThreads) k_pose_compact(CompactArgs a)
{
    if (a.status && *a.status != kStatusOk) return;
    __shared__ int wsum[kCompactThreads / 64];
    __shared__ int goff[kMaxGroups];
    __shared__ unsigned char gcl[kMaxGroups];
    __shared__ double red[3][kCompactThreads / 64];
    const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
    const int chunk = (a.S + kCompactThreads - 1) / kCompactThreads;
    const int g0 = min(tid * chunk, a.S), g1 = min(g0 + chunk, a.S);
    int cn[kCompactGroups];
    int cnt = 0, groups = 0;
#pragma unroll
    for (int u = 0; u < kCompactGroups; ++u) {
        cn[u] = (g0 + u < g1) ? a.gcnt[g0 + u] : 0;
        cnt += cn[u];
        groups += cn[u] > 0;
    }
    // exclusive scan of the counts: first dense index of every group
    int incl = cnt;
    for (int off = 1; off < 64; off <<= 1) {
        const int v = __shfl_up(incl, off, 64);
        if (lane >= off) incl += v;
    }
    if (lane == 63) wsum[wv] = incl;
    __syncthreads();
    int base = 0;
    for (int w = 0; w < wv; ++w) base += wsum[w];
    int off = base + incl - cnt;
#pragma unroll
    for (int u = 0; u < kCompactGroups; ++u)
        if (g0 + u < g1) {
            goff[g0 + u] = off;
            gcl[g0 + u] = (unsigned char)cn[u];
            off += cn[u];
        }
    __syncthreads();
    // coalesced copy, slot by slot: the valid samples of group g fill its
    // slots 4g .. 4g + gcnt[g] - 1
    double wt = 0.0;
    const int nslot = 4 * a.S;
    for (int s0 = tid; s0 < nslot; s0 += 4 * kCompactThreads) {
        double v[4][7];
        int dst[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            const int sl = s0 + u * kCompactThreads;
            const int g = sl >> 2, r = sl & 3;
            dst[u] = (sl < nslot && r < gcl[g]) ? goff[g] + r : -1;
#pragma unroll
            for (int c = 0; c < 7; ++c) v[u][c] = dst[u] >= 0 ? a.samples[(size_t)c * a.ns + sl] : 0.0;
        }
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            if (dst[u] < 0) continue;
#pragma unroll
            for (int c = 0; c < 7; ++c) a.dense[(size_t)c * a.stride + dst[u]] = v[u][c];
            wt += v[u][6];
        }
    }
    double v3[3] = {(double)cnt, wt, (double)groups};
    for (int c = 0; c < 3; ++c) {
        double v = v3[c];
        for (int o = 32; o > 0; o >>= 1) v += __shfl_down(v, o, 64);
        if (lane == 0) red[c][wv] = v;
    }
    __syncthreads();
    if (tid < 3) {
        double sum = 0.0;
        for (int w = 0; w < kCompactThreads / 64; ++w) sum += red[tid][w];
        a.info[tid] = sum;
    }
}

// AoS copy [4S][8] of the sample slots (test hook of the pose step)
__global__ void k_samples_aos(const double *soa, int ns, double *aos)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= ns) return;
    for (int c = 0; c < 8; ++c) aos[(size_t)8 * i + c] = soa[(size_t)c * ns + i];
}

struct SeedArgs {
    const double *dense;
    const double *info;
    double *seed_score;    // [n_seeds + 1][8]: p, density, valid
    const double *prev;    // previous relative pose T_t
    const int *status;
    int stride, have_prev;
    double is2t, is2r;
};

// density of one start candidate (block 0: the previous pose; block b: the
// (b-1)-th sample in group order) over all samples
__global__ void __launch_bounds__(256) k_pose_seed(SeedArgs a)
{
    if (a.status && *a.status != kStatusOk) return;
    __shared__ double red[8];
    __shared__ double seed[6];
    const int b = blockIdx.x, tid = threadIdx.x;
    const int N = (int)a.info[0];
    double *o = a.seed_score + 8 * b;
    if ((b == 0 && !a.have_prev) || (b > 0 && b - 1 >= N)) {
        if (tid == 0) o[7] = 0.0;
        return;
    }
    if (tid == 0) {
        if (b == 0) {
            double p[6];
            se3_log(a.prev, a.prev + 9, p);
            for (int c = 0; c < 6; ++c) seed[c] = p[c];
        } else {
            for (int c = 0; c < 6; ++c) seed[c] = a.dense[(size_t)c * a.stride + (b - 1)];
        }
    }
    __syncthreads();
    double sd[6];
    for (int c = 0; c < 6; ++c) sd[c] = seed[c];
    double s = 0.0;
    for (int i = tid; i < N; i += 256) {
        double q[6];
        for (int c = 0; c < 6; ++c) q[c] = a.dense[(size_t)c * a.stride + i];
        s += a.dense[(size_t)6 * a.stride + i] * exp_nonpos(-0.5 * mahal2(sd, q, a.is2t, a.is2r));
    }
    const double D = block_sum<256>(s, red);
    if (tid == 0) {
        for (int c = 0; c < 6; ++c) o[c] = sd[c];
        o[6] = D;
        o[7] = 1.0;
    }
}

struct MsArgs {
    const double *dense;
    const double *info;
    const double *seed_score;
    double *rel;            // relative poses [T][12]; T_t written at t-1
    double *Mcum;           // cumulative poses [T+1][12]; M_t written
    int *diag;              // [4]
    const int *status;
    int stride, n_seeds, t, max_iters, fallback_prev_frame;
    double is2t, is2r, tol;
};

constexpr int kMsThreads = 512;
constexpr int kMsRegs = 8;   // samples held in registers per thread

// Gaussian mean-shift from the densest start candidate, one workgroup;
// samples beyond kMsThreads * kMsRegs are streamed from memory each iteration.
__global__ void __launch_bounds__(kMsThreads) k_pose_ms(MsArgs a)
{
    if (a.status && *a.status != kStatusOk) return;
    __shared__ double red[kMsThreads / 64][8];
    __shared__ double p[8];
    __shared__ int s_stop;
    const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
    const int N = (int)a.info[0];
    const double WS = a.info[1];
    double *Tt = a.rel + 12 * (a.t - 1);
    if (N == 0 || !(WS > 0.0)) {
        if (tid == 0) {
            if (a.fallback_prev_frame)
                for (int k = 0; k < 12; ++k) Tt[k] = a.rel[12 * (a.t - 2) + k];
            pose_mul(Tt, a.Mcum + 12 * (a.t - 1), a.Mcum + 12 * a.t);
            a.diag[0] = N;
            a.diag[1] = (int)a.info[2];
            a.diag[2] = 0;
            a.diag[3] = 1;
        }
        return;
    }
    double q[kMsRegs][7];
#pragma unroll
    for (int m = 0; m < kMsRegs; ++m) {
        const int i = tid + m * kMsThreads;
#pragma unroll
        for (int c = 0; c < 7; ++c) q[m][c] = i < N ? a.dense[(size_t)c * a.stride + i] : 0.0;
    }
    // densest start candidate, earliest on ties (a workgroup arg-max)
    {
        double sc = -1.0;
        int id = kMsThreads;
        if (tid <= a.n_seeds && a.seed_score[8 * tid + 7] != 0.0) {
            sc = a.seed_score[8 * tid + 6];
            id = tid;
        }
        for (int o = 32; o > 0; o >>= 1) {
            const double so = __shfl_down(sc, o, 64);
            const int io = __shfl_down(id, o, 64);
            if (so > sc || (so == sc && io < id)) { sc = so; id = io; }
        }
        if (lane == 0) { red[wv][0] = sc; red[wv][1] = (double)id; }
        __syncthreads();
        if (tid == 0) {
            for (int w = 1; w < kMsThreads / 64; ++w) {
                const double so = red[w][0];
                const int io = (int)red[w][1];
                if (so > sc || (so == sc && io < id)) { sc = so; id = io; }
            }
            for (int c = 0; c < 6; ++c)
                p[c] = id < kMsThreads ? a.seed_score[8 * id + c] : a.dense[(size_t)c * a.stride];
            s_stop = 0;
        }
    }
    __syncthreads();
    int it = 0;
    for (; it < a.max_iters; ++it) {
        double pc[6];
        for (int c = 0; c < 6; ++c) pc[c] = p[c];
        double acc[7] = {0, 0, 0, 0, 0, 0, 0};
#pragma unroll
        for (int m = 0; m < kMsRegs; ++m) {
            if (tid + m * kMsThreads < N) {
                const double k = q[m][6] * exp_nonpos(-0.5 * mahal2(pc, q[m], a.is2t, a.is2r));
                acc[6] += k;
#pragma unroll
                for (int c = 0; c < 6; ++c) acc[c] += k * q[m][c];
            }
        }
        for (int i = tid + kMsRegs * kMsThreads; i < N; i += kMsThreads) {
            double qq[7];
            for (int c = 0; c < 7; ++c) qq[c] = a.dense[(size_t)c * a.stride + i];
            const double k = qq[6] * exp_nonpos(-0.5 * mahal2(pc, qq, a.is2t, a.is2r));
            acc[6] += k;
            for (int c = 0; c < 6; ++c) acc[c] += k * qq[c];
        }
#pragma unroll
        for (int c = 0; c < 7; ++c)
            for (int off = 32; off > 0; off >>= 1) acc[c] += __shfl_down(acc[c], off, 64);
        if (lane == 0)
            for (int c = 0; c < 7; ++c) red[wv][c] = acc[c];
        __syncthreads();
        if (tid < 7) {
            double s = 0.0;
            for (int w = 0; w < kMsThreads / 64; ++w) s += red[w][tid];
            red[0][tid] = s;   // row 0 is read back only after the next barrier
        }
        __syncthreads();
        if (tid == 0) {
            const double den = red[0][6];
            if (!(den > 0.0)) {
                s_stop = 2;
            } else {
                double np[6];
                for (int c = 0; c < 6; ++c) np[c] = red[0][c] / den;
                const double step = sqrt(mahal2(np, pc, a.is2t, a.is2r));
                for (int c = 0; c < 6; ++c) p[c] = np[c];
                s_stop = step < a.tol ? 1 : 0;
            }
        }
        __syncthreads();
        const int st = s_stop;
        if (st == 2) break;
        if (st == 1) { ++it; break; }
    }
    if (tid == 0) {
        double pp[6], R[9], tv[3];
        for (int c = 0; c < 6; ++c) pp[c] = p[c];
        se3_exp(pp, R, tv);
        for (int k = 0; k < 9; ++k) Tt[k] = R[k];
        for (int k = 0; k < 3; ++k) Tt[9 + k] = tv[k];
        pose_mul(Tt, a.Mcum + 12 * (a.t - 1), a.Mcum + 12 * a.t);
        a.diag[0] = N;
        a.diag[1] = (int)a.info[2];
        a.diag[2] = it;
        a.diag[3] = 0;
    }
}

// scale gauge |t_1| = 1: translations, depth range, cumulative poses
__global__ void k_gauge_poses(double *rel, double *Mcum, double *range, int T, const int *status)
{
    if (status && *status != kStatusOk) return;
    if (threadIdx.x != 0) return;
    const double *t1 = rel + 9;
    const double s = sqrt(t1[0] * t1[0] + t1[1] * t1[1] + t1[2] * t1[2]);
    const double inv = s > 0 ? 1.0 / s : 1.0;
    range[2] = s > 0 ? s : 1.0;
    for (int t = 0; t < T; ++t)
        for (int k = 0; k < 3; ++k) rel[12 * t + 9 + k] *= inv;
    range[0] *= inv;
    range[1] *= inv;
    for (int k = 0; k < 12; ++k) Mcum[k] = (k == 0 || k == 4 || k == 8) ? 1.0 : 0.0;
    for (int t = 1; t <= T; ++t) pose_mul(rel + 12 * (t - 1), Mcum + 12 * (t - 1), Mcum + 12 * t);
}

__global__ void k_gauge_theta(float *theta, int HW, const double *range, const int *status)
{
    if (status && *status != kStatusOk) return;
    const int j = blockIdx.x * blockDim.x + threadIdx.x;
    if (j < HW) theta[j] = (float)((double)theta[j] / range[2]);
}

__global__ void k_cumulative(const double *rel, double *Mcum, int T)
{
    if (threadIdx.x != 0) return;
    for (int k = 0; k < 12; ++k) Mcum[k] = (k == 0 || k == 4 || k == 8) ? 1.0 : 0.0;
    for (int t = 1; t <= T; ++t) pose_mul(rel + 12 * (t - 1), Mcum + 12 * (t - 1), Mcum + 12 * t);
}

// ---------------------------------------------------------------------------
int launch_pose_step(voldor_ctx *c, const float *theta, const float *rig, const float2 *flows,
                     const WinDims &d, const PoseParams &pp, int t, int it, int have_prev,
                     double *rel_poses, hipStream_t s)
{
    GroupArgs g;
    g.theta = theta;
    g.rig = d.use_w ? rig : nullptr;
    g.flows = flows;
    g.Mprev = c->Mcum + 12 * (t - 1);
    g.samples = c->samples;
    g.gcnt = c->gcnt;
    g.status = c->status;
    g.d = d;
    g.S = pp.S;
    g.ns = 4 * pp.S;
    g.t = t;
    g.it = it;
    g.seed = pp.seed;
    hipLaunchKernelGGL(k_pose_groups, dim3((pp.S + 63) / 64), dim3(64), 0, s, g);
    int *diag = c->pose_diag + 4 * (t - 1);
    const int stride = 4 * c->S_max;
    CompactArgs ca{c->samples, c->gcnt, c->dense, c->pose_info, c->status, pp.S, 4 * pp.S, stride};
    hipLaunchKernelGGL(k_pose_compact, dim3(1), dim3(kCompactThreads), 0, s, ca);
    SeedArgs sa;
    sa.dense = c->dense;
    sa.info = c->pose_info;
    sa.seed_score = c->seed_score;
    sa.prev = rel_poses + 12 * (t - 1);
    sa.status = c->status;
    sa.stride = stride;
    sa.have_prev = have_prev;
    sa.is2t = 1.0 / pp.s2t;
    sa.is2r = 1.0 / pp.s2r;
    hipLaunchKernelGGL(k_pose_seed, dim3(pp.n_seeds + 1), dim3(256), 0, s, sa);
    MsArgs m;
    m.dense = c->dense;
    m.info = c->pose_info;
    m.seed_score = c->seed_score;
    m.rel = rel_poses;
    m.Mcum = c->Mcum;
    m.diag = diag;
    m.status = c->status;
    m.stride = stride;
    m.n_seeds = pp.n_seeds;
    m.t = t;
    m.max_iters = pp.ms_max_iters;
    m.fallback_prev_frame = (!have_prev && t >= 2) ? 1 : 0;
    m.is2t = 1.0 / pp.s2t;
    m.is2r = 1.0 / pp.s2r;
    m.tol = pp.ms_tol;
    hipLaunchKernelGGL(k_pose_ms, dim3(1), dim3(kMsThreads), 0, s, m);
    return hipGetLastError() == hipSuccess ? 0 : VOLDOR_EDEVICE;
}

int launch_samples_aos(voldor_ctx *c, int S, double *out, hipStream_t s)
{
    const int ns = 4 * S;
    hipLaunchKernelGGL(k_samples_aos, dim3((ns + 255) / 256), dim3(256), 0, s, c->samples, ns, out);
    return hipGetLastError() == hipSuccess ? 0 : VOLDOR_EDEVICE;
}

int launch_gauge(voldor_ctx *c, double *rel_poses, float *theta, const WinDims &d, hipStream_t s)
{
    hipLaunchKernelGGL(k_gauge_poses, dim3(1), dim3(64), 0, s, rel_poses, c->Mcum, c->range, d.T, c->status);
    const int HW = d.H * d.W;
    hipLaunchKernelGGL(k_gauge_theta, dim3((HW + 255) / 256), dim3(256), 0, s, theta, HW, c->range, c->status);
    return hipGetLastError() == hipSuccess ? 0 : VOLDOR_EDEVICE;
}

int launch_cumulative(voldor_ctx *c, const double *rel_poses, int T, hipStream_t s)
{
    hipLaunchKernelGGL(k_cumulative, dim3(1), dim3(64), 0, s, rel_poses, c->Mcum, T);
    return hipGetLastError() == hipSuccess ? 0 : VOLDOR_EDEVICE;
}

}  // namespace vo
