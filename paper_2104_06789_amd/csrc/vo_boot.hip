// vo_boot.hip -- FP64 bootstrap of a window (Sec. 5.3, Table 1):
//   k_boot_hyp     8-point essential-matrix hypotheses from random
//                  correspondences x <-> x + X_1(x) (null vector of the 8x9
//                  epipolar system by fully pivoted elimination), projected
//                  onto the essential manifold U diag(1,1,0) V^T;
//   k_boot_score   least median of squares: exact lower median of the
//                  pixel-space Sampson distances over a fixed pixel subset,
//                  by radix selection on the residuals held in registers;
//   k_boot_pick    best hypothesis, its four (R, +-t) decompositions and the
//                  cheirality vote -> T_1 with |t_1| = 1;
//   k_boot_tri     two-view triangulation of every pixel along its frame-0 ray;
//   k_hist/_pick   radix selection of the 1st, 50th and 99th percentile depth;
//   k_boot_final   invalid depths -> median, clamp to [0.5 P1, 2 P99].
#include <algorithm>

#include "vo_internal.hpp"

namespace vo {

__device__ __forceinline__ bool flow_present(const float2 *X1, int64_t j)
{
    const float2 f = X1[j];
    return isfinite(f.x) && isfinite(f.y);
}

// symmetric 3x3 eigen-decomposition by cyclic Jacobi rotations; columns of V
__device__ void eig3_sym(const double *S_in, double *w, double *V)
{
    double S[9];
    for (int i = 0; i < 9; ++i) { S[i] = S_in[i]; V[i] = (i == 0 || i == 4 || i == 8) ? 1.0 : 0.0; }
    for (int sweep = 0; sweep < 30; ++sweep) {
        const double off = S[1] * S[1] + S[2] * S[2] + S[5] * S[5];
        const double dia = S[0] * S[0] + S[4] * S[4] + S[8] * S[8];
        if (off <= 1e-32 * dia || off == 0.0) break;
        for (int pq = 0; pq < 3; ++pq) {
            const int p = pq == 2 ? 1 : 0, q = pq == 0 ? 1 : 2;
            const double spq = S[3 * p + q];
            if (spq == 0.0) continue;
            const double tau = (S[3 * q + q] - S[3 * p + p]) / (2.0 * spq);
            const double tt = (tau >= 0 ? 1.0 : -1.0) / (fabs(tau) + sqrt(1.0 + tau * tau));
            const double cs = 1.0 / sqrt(1.0 + tt * tt), sn = tt * cs;
            for (int k = 0; k < 3; ++k) {  // columns p, q of S
                const double a = S[3 * k + p], b = S[3 * k + q];
                S[3 * k + p] = cs * a - sn * b;
                S[3 * k + q] = sn * a + cs * b;
            }
            for (int k = 0; k < 3; ++k) {  // rows p, q of S
                const double a = S[3 * p + k], b = S[3 * q + k];
                S[3 * p + k] = cs * a - sn * b;
                S[3 * q + k] = sn * a + cs * b;
            }
            for (int k = 0; k < 3; ++k) {
                const double a = V[3 * k + p], b = V[3 * k + q];
                V[3 * k + p] = cs * a - sn * b;
                V[3 * k + q] = sn * a + cs * b;
            }
        }
    }
    w[0] = S[0];
    w[1] = S[4];
    w[2] = S[8];
}

// Rank-2 factors of E: E ~ u1 v1^T s1 + u2 v2^T s2 with proper rotations
// U = [u1 u2 u1xu2], V = [v1 v2 v1xv2] (columns, row-major storage).
__device__ void essential_factors(const double *E, double *U, double *V)
{
    double EtE[9];
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j)
            EtE[3 * i + j] = E[i] * E[j] + E[3 + i] * E[3 + j] + E[6 + i] * E[6 + j];
    double w[3], Q[9];
    eig3_sym(EtE, w, Q);
    // order eigen-pairs by decreasing eigenvalue
    int o[3] = {0, 1, 2};
    for (int a = 0; a < 3; ++a)
        for (int b = a + 1; b < 3; ++b)
            if (w[o[b]] > w[o[a]]) { const int t = o[a]; o[a] = o[b]; o[b] = t; }
    double v[3][3], u[3][3];
    for (int c = 0; c < 2; ++c)
        for (int k = 0; k < 3; ++k) v[c][k] = Q[3 * k + o[c]];
    cross3d(v[0], v[1], v[2]);
    for (int c = 0; c < 2; ++c) {
        mv3(E, v[c], u[c]);
        const double n = sqrt(dot3d(u[c], u[c]));
        for (int k = 0; k < 3; ++k) u[c][k] /= (n > 0 ? n : 1.0);
    }
    const double dd = dot3d(u[0], u[1]);
    for (int k = 0; k < 3; ++k) u[1][k] -= dd * u[0][k];
    const double n1 = sqrt(dot3d(u[1], u[1]));
    for (int k = 0; k < 3; ++k) u[1][k] /= (n1 > 0 ? n1 : 1.0);
    cross3d(u[0], u[1], u[2]);
    for (int r = 0; r < 3; ++r)
        for (int c = 0; c < 3; ++c) {
            U[3 * r + c] = u[c][r];
            V[3 * r + c] = v[c][r];
        }
}

struct HypArgs {
    const float2 *X1;
    double *hyp;
    double *score;
    float4 *sub;        // [Ne] scoring subset: x, y, X_1(x) (NaN flow if missing)
    int H, W, M, Ne;
    double fx, fy, cx, cy;
    uint64_t seed;
};

__device__ __forceinline__ void boot_hyp_body(const HypArgs &a)
{
    const int nhb = (a.M + 63) / 64;
    if ((int)blockIdx.x >= nhb) {
        // trailing blocks: the pixel subset j_i = floor(i HW / Ne) of the median
        const int i = (blockIdx.x - nhb) * 64 + threadIdx.x;
        if (i < a.Ne) {
            const int j = (int)(((int64_t)i * ((int64_t)a.H * a.W)) / a.Ne);
            const int y = j / a.W, x = j - y * a.W;
            float2 f = a.X1[j];
            if (!(isfinite(f.x) && isfinite(f.y))) f.x = f.y = __int_as_float(0x7fc00000);
            a.sub[i] = make_float4((float)x, (float)y, f.x, f.y);
        }
        return;
    }
    const int h = blockIdx.x * blockDim.x + threadIdx.x;
    if (h >= a.M) return;
    const int64_t HW = (int64_t)a.H * a.W;
    int64_t idx[8];
    bool ok = false;
    for (int att = 0; att < 16 && !ok; ++att) {
        uint64_t c[4] = {(uint64_t)h, (uint64_t)att, 0ull, 0ull};
        philox4x64_10(c, a.seed, kBootStream);
        ok = true;
#pragma unroll
        for (int k = 0; k < 8; ++k) {
            const uint32_t u = (k & 1) ? (uint32_t)(c[k >> 1] >> 32) : (uint32_t)c[k >> 1];
            idx[k] = u32_to_index(u, HW);
            ok = ok && flow_present(a.X1, idx[k]);
#pragma unroll
            for (int m = 0; m < k; ++m) ok = ok && idx[m] != idx[k];
        }
    }
    a.score[h] = __longlong_as_double(0x7ff0000000000000ll);  // +inf until scored
    double *out = a.hyp + 18 * h;
    if (!ok) {
        out[0] = __longlong_as_double(0x7ff8000000000000ll);
        return;
    }
    // epipolar rows: b^T E a = 0 with a = K^-1 x, b = K^-1 (x + X_1(x))
    double A[8][9];
#pragma unroll
    for (int k = 0; k < 8; ++k) {
        const int jk = (int)idx[k], y = jk / a.W, x = jk - y * a.W;
        const float2 f = a.X1[idx[k]];
        const double av[3] = {(x - a.cx) / a.fx, (y - a.cy) / a.fy, 1.0};
        const double bv[3] = {(x + (double)f.x - a.cx) / a.fx, (y + (double)f.y - a.cy) / a.fy, 1.0};
        for (int i = 0; i < 3; ++i)
            for (int l = 0; l < 3; ++l) A[k][3 * i + l] = bv[i] * av[l];
    }
    // null vector by Gaussian elimination with full pivoting; every index is
    // static (row and column exchanges by selects) so the system stays in
    // registers
    int perm[9];
#pragma unroll
    for (int i = 0; i < 9; ++i) perm[i] = i;
    bool degenerate = false;
#pragma unroll
    for (int r = 0; r < 8; ++r) {
        int pr = r, pc = r;
        double best = 0.0;
#pragma unroll
        for (int i = r; i < 8; ++i)
#pragma unroll
            for (int j = r; j < 9; ++j) {
                const double v = fabs(A[i][j]);
                const bool gt = v > best;
                best = gt ? v : best;
                pr = gt ? i : pr;
                pc = gt ? j : pc;
            }
        degenerate = degenerate || best == 0.0;
#pragma unroll
        for (int i = r + 1; i < 8; ++i) {
            const bool sw = pr == i;
#pragma unroll
            for (int j = 0; j < 9; ++j) {
                const double x = A[r][j], y = A[i][j];
                A[r][j] = sw ? y : x;
                A[i][j] = sw ? x : y;
            }
        }
#pragma unroll
        for (int j = r + 1; j < 9; ++j) {
            const bool sw = pc == j;
#pragma unroll
            for (int i = 0; i < 8; ++i) {
                const double x = A[i][r], y = A[i][j];
                A[i][r] = sw ? y : x;
                A[i][j] = sw ? x : y;
            }
            const int x = perm[r], y = perm[j];
            perm[r] = sw ? y : x;
            perm[j] = sw ? x : y;
        }
#pragma unroll
        for (int i = r + 1; i < 8; ++i) {
            const double f = A[i][r] / A[r][r];
#pragma unroll
            for (int j = r; j < 9; ++j) A[i][j] -= f * A[r][j];
        }
    }
    if (degenerate) {
        out[0] = __longlong_as_double(0x7ff8000000000000ll);
        return;
    }
    double xp[9];
    xp[8] = 1.0;
#pragma unroll
    for (int r = 7; r >= 0; --r) {
        double s = 0.0;
#pragma unroll
        for (int j = r + 1; j < 9; ++j) s += A[r][j] * xp[j];
        xp[r] = -s / A[r][r];
    }
    double e[9], nrm = 0.0;
#pragma unroll
    for (int q = 0; q < 9; ++q) {
        double v = 0.0;
#pragma unroll
        for (int j = 0; j < 9; ++j) v = perm[j] == q ? xp[j] : v;
        e[q] = v;
    }
    for (int j = 0; j < 9; ++j) nrm += e[j] * e[j];
    nrm = sqrt(nrm);
    for (int j = 0; j < 9; ++j) e[j] /= nrm;
    double U[9], V[9], E[9];
    essential_factors(e, U, V);
    for (int i = 0; i < 3; ++i)
        for (int l = 0; l < 3; ++l) E[3 * i + l] = U[3 * i] * V[3 * l] + U[3 * i + 1] * V[3 * l + 1];
    // F = K^-T E K^-1
    const double Ki[9] = {1.0 / a.fx, 0, -a.cx / a.fx, 0, 1.0 / a.fy, -a.cy / a.fy, 0, 0, 1};
    double KiT[9], T1[9], F[9];
    for (int i = 0; i < 3; ++i)
        for (int l = 0; l < 3; ++l) KiT[3 * i + l] = Ki[3 * l + i];
    mm3(KiT, E, T1);
    mm3(T1, Ki, F);
    bool fin = true;
    for (int i = 0; i < 9; ++i) fin = fin && isfinite(E[i]) && isfinite(F[i]);
    if (!fin) {
        out[0] = __longlong_as_double(0x7ff8000000000000ll);
        return;
    }
    for (int i = 0; i < 9; ++i) { out[i] = E[i]; out[9 + i] = F[i]; }
}

__global__ void __launch_bounds__(64) k_boot_hyp(HypArgs a) { boot_hyp_body(a); }

// Bin of a 256-bin histogram (counts h, read by threads 0..255) that holds
// the element of rank `rank`: the unique thread with excl <= rank < incl
// writes the bin and the rank within it.  Called by the whole workgroup.
__device__ __forceinline__ void select_bin(uint32_t h, uint32_t rank, uint32_t *wtot, uint32_t *bin,
                                           uint32_t *rank_in_bin)
{
    const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
    uint32_t incl = h;
    for (int off = 1; off < 64; off <<= 1) {
        const uint32_t v = __shfl_up(incl, off, 64);
        if (lane >= off) incl += v;
    }
    if (tid < 256 && lane == 63) wtot[wv] = incl;
    __syncthreads();
    if (tid < 256) {
        for (int w = 0; w < wv; ++w) incl += wtot[w];
        const uint32_t excl = incl - h;
        if (rank >= excl && rank < incl) {
            *bin = (uint32_t)tid;
            *rank_in_bin = rank - excl;
        }
    }
    __syncthreads();
}

struct ScoreArgs {
    const float4 *sub;
    const double *hyp;
    double *score;
    int Ne;
};

__device__ __forceinline__ uint64_t shfl_xor_u64(uint64_t v, int o)
{
    const uint32_t lo = __shfl_xor((uint32_t)v, o, 64), hi = __shfl_xor((uint32_t)(v >> 32), o, 64);
    return ((uint64_t)hi << 32) | lo;
}

// Lower median of the Sampson distances of one hypothesis over the fixed
// pixel subset, exactly: the distances are held as order-preserving 64-bit
// keys (non-negative FP64 bit patterns), 32 per thread.  The bits shared by
// the smallest and the largest key are skipped; radix passes below them
// narrow the median's bucket until it holds at most one key per thread, and
// those candidates are ranked against each other directly.  Wide digits keep
// the lanes of one atomic on distinct histogram bins.
constexpr int kEvalCand = kEvalThreads;
constexpr int kDigitBits = 12;   // 4096 bins = 8 per thread

__device__ __forceinline__ void boot_score_body(const ScoreArgs &a)
{
    __shared__ uint32_t hist[1 << kDigitBits];
    __shared__ int cnt_red[kEvalThreads / 64];
    __shared__ uint64_t kmin_red[kEvalThreads / 64], kmax_red[kEvalThreads / 64];
    __shared__ uint64_t cand[kEvalCand];
    __shared__ uint32_t s_wtot[kEvalThreads / 64], s_bin, s_rib, s_inb, s_nc;
    const int h = blockIdx.x, tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
    const double *hp = a.hyp + 18 * h;
    if (isnan(hp[0])) return;  // invalid hypothesis keeps +inf
    double F[9];
    for (int i = 0; i < 9; ++i) F[i] = hp[9 + i];
    uint64_t key[kEvalPerThread];
    uint32_t valid = 0;
    uint64_t kmin = ~0ull, kmax = 0;
#pragma unroll
    for (int m = 0; m < kEvalPerThread; ++m) {
        const int i = tid + m * kEvalThreads;
        uint64_t kk = 0;
        if (i < a.Ne) {
            const float4 sp = a.sub[i];
            if (isfinite(sp.z) && isfinite(sp.w)) {
                const double x = (double)sp.x, y = (double)sp.y;
                const double x2 = x + sp.z, y2 = y + sp.w;
                const double Fx0 = F[0] * x + F[1] * y + F[2];
                const double Fx1 = F[3] * x + F[4] * y + F[5];
                const double Fx2 = F[6] * x + F[7] * y + F[8];
                const double Ft0 = F[0] * x2 + F[3] * y2 + F[6];
                const double Ft1 = F[1] * x2 + F[4] * y2 + F[7];
                const double e = x2 * Fx0 + y2 * Fx1 + Fx2;
                const double r = e * e / (Fx0 * Fx0 + Fx1 * Fx1 + Ft0 * Ft0 + Ft1 * Ft1);
                kk = (uint64_t)__double_as_longlong(r);
                valid |= 1u << m;
                kmin = kk < kmin ? kk : kmin;
                kmax = kk > kmax ? kk : kmax;
            }
        }
        key[m] = kk;
    }
    // present pixels and the key range over the workgroup
    int c = __popc(valid);
    for (int o = 32; o > 0; o >>= 1) {
        c += __shfl_xor(c, o, 64);
        const uint64_t mn = shfl_xor_u64(kmin, o), mx = shfl_xor_u64(kmax, o);
        kmin = mn < kmin ? mn : kmin;
        kmax = mx > kmax ? mx : kmax;
    }
    if (lane == 0) {
        cnt_red[wv] = c;
        kmin_red[wv] = kmin;
        kmax_red[wv] = kmax;
    }
    if (tid == 0) s_nc = 0;
    __syncthreads();
    int tot = 0;
    for (int w = 0; w < kEvalThreads / 64; ++w) {
        tot += cnt_red[w];
        kmin = kmin_red[w] < kmin ? kmin_red[w] : kmin;
        kmax = kmax_red[w] > kmax ? kmax_red[w] : kmax;
    }
    if (tot == 0) return;  // no usable pixel: the hypothesis keeps +inf
    uint32_t rank = (uint32_t)((tot - 1) / 2);
    uint64_t prefix = kmin;
    if (kmin != kmax) {
        // bits below the common prefix of all keys
        int shift = 64 - __clzll((long long)(kmin ^ kmax));   // number of varying low bits
        prefix = (kmin >> shift) << shift;
        uint32_t inbin = (uint32_t)tot;
        while (shift > 0 && inbin > (uint32_t)kEvalCand) {
            const int ds = shift > kDigitBits ? shift - kDigitBits : 0;   // digit = bits [ds, shift)
            const int nbin = 1 << (shift - ds);
            for (int q = tid; q < nbin; q += kEvalThreads) hist[q] = 0;
            __syncthreads();
#pragma unroll
            for (int m = 0; m < kEvalPerThread; ++m)
                if (((valid >> m) & 1u) && (key[m] >> shift) == (prefix >> shift))
                    atomicAdd(&hist[(uint32_t)(key[m] >> ds) & (uint32_t)(nbin - 1)], 1u);
            __syncthreads();
            // bins [8 tid, 8 tid + 8) per thread; the thread whose range holds the rank finds the bin
            uint32_t c8[8], loc = 0;
#pragma unroll
            for (int q = 0; q < 8; ++q) {
                c8[q] = 8 * tid + q < nbin ? hist[8 * tid + q] : 0u;
                loc += c8[q];
            }
            uint32_t incl = loc;
            for (int o = 1; o < 64; o <<= 1) {
                const uint32_t v = __shfl_up(incl, o, 64);
                if (lane >= o) incl += v;
            }
            if (lane == 63) s_wtot[wv] = incl;
            __syncthreads();
            for (int w = 0; w < wv; ++w) incl += s_wtot[w];
            uint32_t ex = incl - loc;
            if (ex <= rank && rank < incl) {
#pragma unroll
                for (int q = 0; q < 8; ++q) {
                    if (ex <= rank && rank < ex + c8[q]) {
                        s_bin = 8 * tid + q;
                        s_rib = rank - ex;
                        s_inb = c8[q];
                    }
                    ex += c8[q];
                }
            }
            __syncthreads();
            rank = s_rib;
            inbin = s_inb;
            prefix |= (uint64_t)s_bin << ds;
            shift = ds;
            __syncthreads();   // hist, s_wtot and s_bin are reused by the next pass
        }
        if (shift > 0) {
            // at most kEvalCand keys share the bucket: gather them (one atomic per
            // wave and key slot) and rank them against each other
#pragma unroll
            for (int m = 0; m < kEvalPerThread; ++m) {
                const bool take = ((valid >> m) & 1u) && (key[m] >> shift) == (prefix >> shift);
                const uint64_t bal = __ballot(take);
                if (bal) {
                    const int leader = __ffsll((long long)bal) - 1;
                    uint32_t base = 0;
                    if (lane == leader) base = atomicAdd(&s_nc, (uint32_t)__popcll(bal));
                    base = __shfl(base, leader, 64);
                    if (take) cand[base + __popcll(bal & __lanemask_lt())] = key[m];
                }
            }
            __syncthreads();
            const uint32_t nc = s_nc;
            if ((uint32_t)tid < nc) {
                const uint64_t v = cand[tid];
                uint32_t less = 0, eq = 0;
                for (uint32_t q = 0; q < nc; ++q) {
                    const uint64_t u = cand[q];
                    less += u < v;
                    eq += u == v;
                }
                if (less <= rank && rank < less + eq) a.score[h] = __longlong_as_double((long long)v);
            }
            return;
        }
    }
    if (tid == 0) a.score[h] = __longlong_as_double((long long)prefix);
}

__global__ void __launch_bounds__(kEvalThreads) k_boot_score(ScoreArgs a) { boot_score_body(a); }

// sel layout: [0..2] prefix, [3..5] rank, [8..11] cheirality votes, [12] valid count
constexpr int kSelVotes = 8;

struct PickArgs {
    const double *hyp;
    const double *score;
    double *cand;       // [21]: R of both decompositions (2 x 9), t up to sign (3)
    double *info;       // [4]
    int *status;
    int M;
};

__device__ __forceinline__ double tri_depth(const double *R, const double *t, double xn, double yn,
                                            double bx, double by, bool &ok)
{
    const double r[3] = {xn, yn, 1.0};
    double av[3];
    mv3(R, r, av);
    const double c0 = av[0] - bx * av[2], c1 = av[1] - by * av[2];
    const double e0 = t[0] - bx * t[2], e1 = t[1] - by * t[2];
    const double cc = c0 * c0 + c1 * c1;
    const double th = -(c0 * e0 + c1 * e1) / cc;
    ok = cc >= 1e-12 && th > 0 && isfinite(th);
    return th;
}

// least median of squares: lowest finite score, lowest index on ties; the
// two rotations and the translation direction of its essential matrix
__device__ __forceinline__ void boot_pick_body(const PickArgs &a)
{
    __shared__ double s_rs[4];
    __shared__ int s_rh[4];
    const int tid = threadIdx.x;
    double bs = __longlong_as_double(0x7ff0000000000000ll);
    int best = 0x7fffffff;
    for (int h = tid; h < a.M; h += 256) {
        const double sc = a.score[h];
        if (isfinite(sc) && (sc < bs || (sc == bs && h < best))) { bs = sc; best = h; }
    }
    for (int o = 32; o > 0; o >>= 1) {
        const double so = __shfl_down(bs, o, 64);
        const int ho = __shfl_down(best, o, 64);
        if (so < bs || (so == bs && ho < best)) { bs = so; best = ho; }
    }
    if ((tid & 63) == 0) { s_rs[tid >> 6] = bs; s_rh[tid >> 6] = best; }
    __syncthreads();
    if (tid != 0) return;
    for (int w = 1; w < 4; ++w)
        if (s_rs[w] < bs || (s_rs[w] == bs && s_rh[w] < best)) { bs = s_rs[w]; best = s_rh[w]; }
    if (!isfinite(bs)) {
        *a.status = kStatusDegenerate;
        return;
    }
    double U[9], V[9];
    essential_factors(a.hyp + 18 * best, U, V);
    const double Wm[9] = {0, -1, 0, 1, 0, 0, 0, 0, 1};
    const double WmT[9] = {0, 1, 0, -1, 0, 0, 0, 0, 1};
    double VT[9], T1[9];
    for (int i = 0; i < 3; ++i)
        for (int l = 0; l < 3; ++l) VT[3 * i + l] = V[3 * l + i];
    mm3(U, Wm, T1);
    mm3(T1, VT, a.cand);
    mm3(U, WmT, T1);
    mm3(T1, VT, a.cand + 9);
    a.cand[18] = U[2];
    a.cand[19] = U[5];
    a.cand[20] = U[8];
    a.info[0] = best;
    a.info[1] = bs;
}

__global__ void __launch_bounds__(256) k_boot_pick(PickArgs a) { boot_pick_body(a); }

struct VoteArgs {
    const float2 *X1;
    const double *cand;
    uint32_t *sel;
    const int *status;
    int H, W, Ne;
    double fx, fy, cx, cy;
};

// cheirality vote of the four decompositions (R_a, +t), (R_a, -t), (R_b, +t),
// (R_b, -t) over the pixel subset
__device__ __forceinline__ void boot_vote_body(const VoteArgs &a)
{
    if (*a.status != kStatusOk) return;
    __shared__ int red[4][4];
    const int tid = threadIdx.x;
    double Rc[2][9], tc[3];
    for (int k = 0; k < 9; ++k) {
        Rc[0][k] = a.cand[k];
        Rc[1][k] = a.cand[9 + k];
    }
    for (int k = 0; k < 3; ++k) tc[k] = a.cand[18 + k];
    const int64_t HW = (int64_t)a.H * a.W;
    int cnt[4] = {0, 0, 0, 0};
    for (int i = blockIdx.x * 256 + tid; i < a.Ne; i += gridDim.x * 256) {
        const int j = (int)(((int64_t)i * HW) / a.Ne);
        const float2 f = a.X1[j];
        if (!(isfinite(f.x) && isfinite(f.y))) continue;
        const int y = j / a.W, x = j - y * a.W;
        const double xn = (x - a.cx) / a.fx, yn = (y - a.cy) / a.fy;
        const double bx = (x + (double)f.x - a.cx) / a.fx, by = (y + (double)f.y - a.cy) / a.fy;
#pragma unroll
        for (int c = 0; c < 4; ++c) {
            const double *R = Rc[c >> 1];
            const double sg = (c & 1) ? -1.0 : 1.0;
            const double t[3] = {sg * tc[0], sg * tc[1], sg * tc[2]};
            bool ok;
            const double th = tri_depth(R, t, xn, yn, bx, by, ok);
            if (!ok) continue;
            const double z1 = th * (R[6] * xn + R[7] * yn + R[8]) + t[2];
            if (z1 > 0) ++cnt[c];
        }
    }
    for (int c = 0; c < 4; ++c) {
        int v = cnt[c];
        for (int off = 32; off > 0; off >>= 1) v += __shfl_down(v, off, 64);
        if ((tid & 63) == 0) red[c][tid >> 6] = v;
    }
    __syncthreads();
    if (tid < 4) {
        const int v = red[tid][0] + red[tid][1] + red[tid][2] + red[tid][3];
        if (v) atomicAdd(&a.sel[kSelVotes + tid], (uint32_t)v);
    }
}

__global__ void __launch_bounds__(256) k_boot_vote(VoteArgs a) { boot_vote_body(a); }

struct TriArgs {
    const float2 *X1;
    const double *cand;
    double *rel;         // [T][12]
    double *Mcum;        // [T+1][12]
    double *info;
    float *theta;
    uint32_t *keys;
    uint32_t *sel;       // votes in; sel[12] accumulates the valid count
    const int *status;
    int H, W, T;
    double fx, fy, cx, cy;
};

// the decomposition with most points in front of both cameras (first on
// ties) -> T_1 with |t_1| = 1; two-view depth of every pixel along its ray
__device__ __forceinline__ void boot_tri_body(const TriArgs &a)
{
    if (*a.status != kStatusOk) return;
    __shared__ int red[4];
    int bc = 0;
    uint32_t bn = 0;
    for (int c = 0; c < 4; ++c) {
        const uint32_t v = a.sel[kSelVotes + c];
        if (c == 0 || v > bn) { bn = v; bc = c; }
    }
    double R[9], t[3];
    for (int k = 0; k < 9; ++k) R[k] = a.cand[9 * (bc >> 1) + k];
    {
        const double sg = (bc & 1) ? -1.0 : 1.0;
        for (int k = 0; k < 3; ++k) t[k] = sg * a.cand[18 + k];
        const double tn = sqrt(t[0] * t[0] + t[1] * t[1] + t[2] * t[2]);
        for (int k = 0; k < 3; ++k) t[k] /= tn;
    }
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        for (int k = 0; k < 9; ++k) a.rel[k] = R[k];
        for (int k = 0; k < 3; ++k) a.rel[9 + k] = t[k];
        for (int tt = 1; tt < a.T; ++tt)
            for (int k = 0; k < 12; ++k) a.rel[12 * tt + k] = (k == 0 || k == 4 || k == 8) ? 1.0 : 0.0;
        for (int k = 0; k < 12; ++k) a.Mcum[k] = (k == 0 || k == 4 || k == 8) ? 1.0 : 0.0;
        for (int k = 0; k < 9; ++k) a.Mcum[12 + k] = R[k];
        for (int k = 0; k < 3; ++k) a.Mcum[21 + k] = t[k];
        a.info[3] = bn;
    }
    const int HW = a.H * a.W;
    const int j = blockIdx.x * blockDim.x + threadIdx.x;
    int valid = 0;
    if (j < HW) {
        const float2 f = a.X1[j];
        uint32_t key = 0xffffffffu;
        float th32 = 0.0f;
        if (isfinite(f.x) && isfinite(f.y)) {
            const int y = j / a.W, x = j - y * a.W;
            bool ok;
            const double th = tri_depth(R, t, (x - a.cx) / a.fx, (y - a.cy) / a.fy,
                                        (x + (double)f.x - a.cx) / a.fx, (y + (double)f.y - a.cy) / a.fy, ok);
            if (ok) {
                th32 = (float)th;
                key = __float_as_uint(th32);
                valid = 1;
            }
        }
        a.theta[j] = th32;
        a.keys[j] = key;
    }
    for (int off = 32; off > 0; off >>= 1) valid += __shfl_down(valid, off, 64);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = valid;
    __syncthreads();
    if (threadIdx.x == 0) {
        const int tot = red[0] + red[1] + red[2] + red[3];
        if (tot) atomicAdd(&a.sel[12], (uint32_t)tot);
    }
}

__global__ void __launch_bounds__(256) k_boot_tri(TriArgs a) { boot_tri_body(a); }

__device__ __forceinline__ void sel_init_body(uint32_t *sel, uint32_t *hist, int *status)
{
    const int tid = threadIdx.x;
    for (int i = tid; i < 3 * 256; i += blockDim.x) hist[i] = 0;
    if (tid == 0) {
        if (*status != kStatusOk) return;
        const uint32_t n = sel[12];
        if (n == 0) { *status = kStatusDegenerate; return; }
        const double q[3] = {0.01, 0.50, 0.99};
        for (int i = 0; i < 3; ++i) {
            sel[i] = 0;
            sel[3 + i] = (uint32_t)floor(q[i] * (double)(n - 1));
        }
    }
}

__global__ void k_sel_init(uint32_t *sel, uint32_t *hist, int *status) { sel_init_body(sel, hist, status); }

__device__ __forceinline__ void hist_body(const uint32_t *keys, int64_t n, const uint32_t *sel, uint32_t *hist,
                                          int pass, const int *status)
{
    if (*status != kStatusOk) return;
    __shared__ uint32_t lh[3][256];
    for (int i = threadIdx.x; i < 768; i += 256) (&lh[0][0])[i] = 0;
    __syncthreads();
    const int shift = 8 * pass;
    const uint32_t mask = pass == 3 ? 0u : (0xffffffffu << (shift + 8));
    const uint32_t p0 = sel[0], p1 = sel[1], p2 = sel[2];
    for (int64_t j = (int64_t)blockIdx.x * 256 + threadIdx.x; j < n; j += (int64_t)gridDim.x * 256) {
        const uint32_t k = keys[j];
        if (k == 0xffffffffu) continue;
        const uint32_t dgt = (k >> shift) & 255u;
        const uint32_t km = k & mask;
        if (km == p0) atomicAdd(&lh[0][dgt], 1u);
        if (km == p1) atomicAdd(&lh[1][dgt], 1u);
        if (km == p2) atomicAdd(&lh[2][dgt], 1u);
    }
    __syncthreads();
    for (int i = threadIdx.x; i < 768; i += 256) {
        const uint32_t v = (&lh[0][0])[i];
        if (v) atomicAdd(&hist[i], v);
    }
}

__global__ void __launch_bounds__(256) k_hist(const uint32_t *keys, int64_t n, const uint32_t *sel,
                                              uint32_t *hist, int pass, const int *status)
{
    hist_body(keys, n, sel, hist, pass, status);
}

__device__ __forceinline__ void hist_pick_body(uint32_t *sel, uint32_t *hist, int pass, const int *status)
{
    if (*status != kStatusOk) return;
    __shared__ uint32_t s_wtot[4], s_bin, s_rib;
    const int shift = 8 * pass;
    for (int q = 0; q < 3; ++q) {
        if (threadIdx.x == 0) {
            s_bin = 255;
            s_rib = 0;
        }
        const uint32_t rank = sel[3 + q];
        __syncthreads();
        select_bin(hist[256 * q + threadIdx.x], rank, s_wtot, &s_bin, &s_rib);
        if (threadIdx.x == 0) {
            sel[3 + q] = s_rib;
            sel[q] |= s_bin << shift;
        }
        __syncthreads();
    }
    for (int i = threadIdx.x; i < 768; i += blockDim.x) hist[i] = 0;
}

__global__ void __launch_bounds__(256) k_hist_pick(uint32_t *sel, uint32_t *hist, int pass, const int *status)
{
    hist_pick_body(sel, hist, pass, status);
}

__device__ __forceinline__ void boot_final_body(float *theta, const uint32_t *keys, int64_t n, const uint32_t *sel,
                                                double *range, double *info, double depth_lo, double depth_hi,
                                                const int *status)
{
    if (*status != kStatusOk) return;
    const float P1 = __uint_as_float(sel[0]), P50 = __uint_as_float(sel[1]), P99 = __uint_as_float(sel[2]);
    const double dlo = depth_lo > 0 ? depth_lo : 0.5 * (double)P1;
    const double dhi = depth_hi > 0 ? depth_hi : 2.0 * (double)P99;
    const float flo = (float)dlo, fhi = (float)dhi;
    const int64_t j = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (j == 0) {
        range[0] = dlo;
        range[1] = dhi;
        range[2] = 1.0;
        info[2] = (double)sel[12];
    }
    if (j < n) {
        float th = keys[j] == 0xffffffffu ? P50 : theta[j];
        th = fminf(fmaxf(th, flo), fhi);
        theta[j] = th;
    }
}

__global__ void __launch_bounds__(256) k_boot_final(float *theta, const uint32_t *keys, int64_t n,
                                                    const uint32_t *sel, double *range, double *info,
                                                    double depth_lo, double depth_hi, const int *status)
{
    boot_final_body(theta, keys, n, sel, range, info, depth_lo, depth_hi, status);
}

__device__ __forceinline__ void boot_init_body(int *status, uint32_t *sel)
{
    if (threadIdx.x == 0) *status = kStatusOk;
    if (threadIdx.x < 16) sel[threadIdx.x] = 0;
}

__global__ void k_boot_init(int *status, uint32_t *sel) { boot_init_body(status, sel); }

// T_1 given instead of estimated (overlapping consecutive batches, Sec. 5.3):
// the pose becomes decomposition candidate 0 with the only vote, so that the
// triangulation and depth-range passes run unchanged (k_boot_tri rescales its
// translation to unit length); a non-finite pose or a zero translation is
// degenerate
__global__ void k_boot_seed(const double *T1, double *cand, uint32_t *sel, double *info, int *status)
{
    if (threadIdx.x != 0 || *status != kStatusOk) return;
    bool fin = true;
    for (int k = 0; k < 12; ++k) fin = fin && isfinite(T1[k]);
    const double tn = sqrt(T1[9] * T1[9] + T1[10] * T1[10] + T1[11] * T1[11]);
    if (!fin || !(tn > 0.0)) {
        *status = kStatusDegenerate;
        return;
    }
    for (int k = 0; k < 9; ++k) cand[k] = T1[k];
    for (int k = 0; k < 3; ++k) cand[18 + k] = T1[9 + k];
    sel[kSelVotes] = 1;
    info[0] = -1.0;
    info[1] = 0.0;
}

// ---------------------------------------------------------------------------
// The bootstrap of several windows at once (a lockstep batch lane): each
// kernel is one launch whose blockIdx.y selects a window's arguments, those
// of its launch_bootstrap; counts gathered by atomics are integers, so the
// windows' grid strides may differ from a single window's without changing
// any result.
struct BootWin {
    HypArgs h;
    ScoreArgs sc;
    PickArgs pk;
    VoteArgs va;
    TriArgs tr;
    uint32_t *sel, *hist, *keys;
    int *status;
    float *theta;
    double *range, *info;
    int64_t HW;
    double depth_lo, depth_hi;
};

// A window's arguments with their pointers in the global address space
// (global_ptr): the kernels below read them from the array in device memory
__device__ __forceinline__ HypArgs to_global(HypArgs a)
{
    a.X1 = global_ptr(a.X1);
    a.hyp = global_ptr(a.hyp);
    a.score = global_ptr(a.score);
    a.sub = global_ptr(a.sub);
    return a;
}

__device__ __forceinline__ ScoreArgs to_global(ScoreArgs a)
{
    a.sub = global_ptr(a.sub);
    a.hyp = global_ptr(a.hyp);
    a.score = global_ptr(a.score);
    return a;
}

__device__ __forceinline__ PickArgs to_global(PickArgs a)
{
    a.hyp = global_ptr(a.hyp);
    a.score = global_ptr(a.score);
    a.cand = global_ptr(a.cand);
    a.info = global_ptr(a.info);
    a.status = global_ptr(a.status);
    return a;
}

__device__ __forceinline__ VoteArgs to_global(VoteArgs a)
{
    a.X1 = global_ptr(a.X1);
    a.cand = global_ptr(a.cand);
    a.sel = global_ptr(a.sel);
    a.status = global_ptr(a.status);
    return a;
}

__device__ __forceinline__ TriArgs to_global(TriArgs a)
{
    a.X1 = global_ptr(a.X1);
    a.cand = global_ptr(a.cand);
    a.rel = global_ptr(a.rel);
    a.Mcum = global_ptr(a.Mcum);
    a.info = global_ptr(a.info);
    a.theta = global_ptr(a.theta);
    a.keys = global_ptr(a.keys);
    a.sel = global_ptr(a.sel);
    a.status = global_ptr(a.status);
    return a;
}

__global__ void k_boot_init_multi(const BootWin *w)
{
    const BootWin &b = w[blockIdx.y];
    boot_init_body(global_ptr(b.status), global_ptr(b.sel));
}

__global__ void __launch_bounds__(64) k_boot_hyp_multi(const BootWin *w)
{
    const BootWin &b = w[blockIdx.y];
    if ((int)blockIdx.x >= (b.h.M + 63) / 64 + (b.h.Ne + 63) / 64) return;
    boot_hyp_body(to_global(b.h));
}

__global__ void __launch_bounds__(kEvalThreads) k_boot_score_multi(const BootWin *w)
{
    boot_score_body(to_global(w[blockIdx.y].sc));
}

__global__ void __launch_bounds__(256) k_boot_pick_multi(const BootWin *w)
{
    boot_pick_body(to_global(w[blockIdx.y].pk));
}

__global__ void __launch_bounds__(256) k_boot_vote_multi(const BootWin *w)
{
    boot_vote_body(to_global(w[blockIdx.y].va));
}

__global__ void __launch_bounds__(256) k_boot_tri_multi(const BootWin *w)
{
    const BootWin &b = w[blockIdx.y];
    if ((int64_t)blockIdx.x * 256 >= b.HW) return;   // past this window's pixels
    boot_tri_body(to_global(b.tr));
}

__global__ void __launch_bounds__(256) k_sel_init_multi(const BootWin *w)
{
    const BootWin &b = w[blockIdx.y];
    sel_init_body(global_ptr(b.sel), global_ptr(b.hist), global_ptr(b.status));
}

__global__ void __launch_bounds__(256) k_hist_multi(const BootWin *w, int pass)
{
    const BootWin &b = w[blockIdx.y];
    hist_body(global_ptr(b.keys), b.HW, global_ptr(b.sel), global_ptr(b.hist), pass, global_ptr(b.status));
}

__global__ void __launch_bounds__(256) k_hist_pick_multi(const BootWin *w, int pass)
{
    const BootWin &b = w[blockIdx.y];
    hist_pick_body(global_ptr(b.sel), global_ptr(b.hist), pass, global_ptr(b.status));
}

__global__ void __launch_bounds__(256) k_boot_final_multi(const BootWin *w)
{
    const BootWin &b = w[blockIdx.y];
    boot_final_body(global_ptr(b.theta), global_ptr(b.keys), b.HW, global_ptr(b.sel), global_ptr(b.range),
                    global_ptr(b.info), b.depth_lo, b.depth_hi, global_ptr(b.status));
}

void plan_bootstrap(Plan &p, std::vector<MultiLaunch> &out, const std::vector<WinRef> &w,
                    const std::vector<int> &idx, int n_hyp, int n_eval, uint64_t seed, double depth_lo,
                    double depth_hi)
{
    const int n = (int)idx.size();
    std::vector<BootWin> bw(n);
    int g_hyp = 0, g_vote = 0, g_px = 0, g_hist = 0;
    for (int k = 0; k < n; ++k) {
        const WinRef &r = w[idx[k]];
        voldor_ctx *c = r.c;
        const WinDims &d = r.d;
        const int64_t HW = (int64_t)d.H * d.W;
        const int Ne = (int)(n_eval < HW ? n_eval : HW);
        BootWin &b = bw[k];
        b.h = HypArgs{r.X, c->hyp, c->hyp_score, c->boot_sub, d.H, d.W, n_hyp, Ne, d.fx, d.fy, d.cx, d.cy, seed};
        b.sc = ScoreArgs{c->boot_sub, c->hyp, c->hyp_score, Ne};
        b.pk = PickArgs{c->hyp, c->hyp_score, c->boot_cand, c->boot_info, c->status, n_hyp};
        b.va = VoteArgs{r.X, c->boot_cand, c->sel, c->status, d.H, d.W, Ne, d.fx, d.fy, d.cx, d.cy};
        b.tr = TriArgs{r.X, c->boot_cand, r.poses, c->Mcum, c->boot_info, r.depth, c->dkeys, c->sel, c->status,
                       d.H, d.W, d.T, d.fx, d.fy, d.cx, d.cy};
        b.sel = c->sel;
        b.hist = c->hist;
        b.keys = c->dkeys;
        b.status = c->status;
        b.theta = r.depth;
        b.range = c->range;
        b.info = c->boot_info;
        b.HW = HW;
        b.depth_lo = depth_lo;
        b.depth_hi = depth_hi;
        g_hyp = std::max(g_hyp, (n_hyp + 63) / 64 + (Ne + 63) / 64);
        g_vote = std::max(g_vote, (Ne + 255) / 256);
        g_px = std::max(g_px, (int)((HW + 255) / 256));
        g_hist = std::max(g_hist, (int)std::min<int64_t>((HW + 255) / 256, 1024));
    }
    MultiLaunch l = {};
    l.nwin = n;
    l.off = p.put(bw.data(), n);
    auto emit = [&](int kind, int gx, int variant) {
        l.kind = kind;
        l.gx = gx;
        l.variant = variant;
        out.push_back(l);
    };
    emit(kMultiBootInit, 1, 0);
    emit(kMultiBootHyp, g_hyp, 0);
    emit(kMultiBootScore, n_hyp, 0);
    emit(kMultiBootPick, 1, 0);
    emit(kMultiBootVote, g_vote, 0);
    emit(kMultiBootTri, g_px, 0);
    emit(kMultiSelInit, 1, 0);
    for (int pass = 3; pass >= 0; --pass) {
        emit(kMultiHist, g_hist, pass);
        emit(kMultiHistPick, 1, pass);
    }
    emit(kMultiBootFinal, g_px, 0);
}

int launch_boot_multi(const MultiLaunch &m, const unsigned char *dev, hipStream_t s)
{
    if (m.nwin < 1) return 0;
    const BootWin *w = (const BootWin *)(dev + m.off);
    const dim3 grid(m.gx, m.nwin);
    switch (m.kind) {
    case kMultiBootInit: hipLaunchKernelGGL(k_boot_init_multi, grid, dim3(64), 0, s, w); break;
    case kMultiBootHyp: hipLaunchKernelGGL(k_boot_hyp_multi, grid, dim3(64), 0, s, w); break;
    case kMultiBootScore: hipLaunchKernelGGL(k_boot_score_multi, grid, dim3(kEvalThreads), 0, s, w); break;
    case kMultiBootPick: hipLaunchKernelGGL(k_boot_pick_multi, grid, dim3(256), 0, s, w); break;
    case kMultiBootVote: hipLaunchKernelGGL(k_boot_vote_multi, grid, dim3(256), 0, s, w); break;
    case kMultiBootTri: hipLaunchKernelGGL(k_boot_tri_multi, grid, dim3(256), 0, s, w); break;
    case kMultiSelInit: hipLaunchKernelGGL(k_sel_init_multi, grid, dim3(256), 0, s, w); break;
    case kMultiHist: hipLaunchKernelGGL(k_hist_multi, grid, dim3(256), 0, s, w, m.variant); break;
    case kMultiHistPick: hipLaunchKernelGGL(k_hist_pick_multi, grid, dim3(256), 0, s, w, m.variant); break;
    case kMultiBootFinal: hipLaunchKernelGGL(k_boot_final_multi, grid, dim3(256), 0, s, w); break;
    default: return VOLDOR_EINVAL;
    }
    return hipGetLastError() == hipSuccess ? 0 : VOLDOR_EDEVICE;
}

int launch_bootstrap(voldor_ctx *c, const float2 *flows, const WinDims &d, int n_hyp, int n_eval,
                     uint64_t seed, double depth_lo, double depth_hi, double *rel_poses,
                     float *theta, hipStream_t s, const double *T1_seed)
{
    const int64_t HW = (int64_t)d.H * d.W;
    const int Ne = (int)(n_eval < HW ? n_eval : HW);
    hipLaunchKernelGGL(k_boot_init, dim3(1), dim3(64), 0, s, c->status, c->sel);
    if (T1_seed) {
        hipLaunchKernelGGL(k_boot_seed, dim3(1), dim3(64), 0, s, T1_seed, c->boot_cand, c->sel, c->boot_info,
                           c->status);
    } else {
        HypArgs h{flows, c->hyp, c->hyp_score, c->boot_sub, d.H, d.W, n_hyp, Ne, d.fx, d.fy, d.cx, d.cy, seed};
        hipLaunchKernelGGL(k_boot_hyp, dim3((n_hyp + 63) / 64 + (Ne + 63) / 64), dim3(64), 0, s, h);
        ScoreArgs sc{c->boot_sub, c->hyp, c->hyp_score, Ne};
        hipLaunchKernelGGL(k_boot_score, dim3(n_hyp), dim3(kEvalThreads), 0, s, sc);
        PickArgs pk{c->hyp, c->hyp_score, c->boot_cand, c->boot_info, c->status, n_hyp};
        hipLaunchKernelGGL(k_boot_pick, dim3(1), dim3(256), 0, s, pk);
        VoteArgs va{flows, c->boot_cand, c->sel, c->status, d.H, d.W, Ne, d.fx, d.fy, d.cx, d.cy};
        hipLaunchKernelGGL(k_boot_vote, dim3((Ne + 255) / 256), dim3(256), 0, s, va);
    }
    TriArgs tr{flows, c->boot_cand, rel_poses, c->Mcum, c->boot_info, theta, c->dkeys, c->sel, c->status,
               d.H, d.W, d.T, d.fx, d.fy, d.cx, d.cy};
    hipLaunchKernelGGL(k_boot_tri, dim3((unsigned)((HW + 255) / 256)), dim3(256), 0, s, tr);
    hipLaunchKernelGGL(k_sel_init, dim3(1), dim3(256), 0, s, c->sel, c->hist, c->status);
    int blocks = (int)((HW + 255) / 256);
    if (blocks > 1024) blocks = 1024;
    for (int pass = 3; pass >= 0; --pass) {
        hipLaunchKernelGGL(k_hist, dim3(blocks), dim3(256), 0, s, c->dkeys, HW, c->sel, c->hist, pass, c->status);
        hipLaunchKernelGGL(k_hist_pick, dim3(1), dim3(256), 0, s, c->sel, c->hist, pass, c->status);
    }
    hipLaunchKernelGGL(k_boot_final, dim3((unsigned)((HW + 255) / 256)), dim3(256), 0, s, theta, c->dkeys,
                       HW, c->sel, c->range, c->boot_info, depth_lo, depth_hi, c->status);
    return hipGetLastError() == hipSuccess ? 0 : VOLDOR_EDEVICE;
}

}  // namespace vo
