// vo_pose.hip -- pose step of one frame (Sec. 5.2, Eq. 15-19):
//   k_pose_groups  S random pixel triples -> 3-D points in camera t-1 and
//                  bearings in camera t through the flow X_t -> P3P roots in
//                  front of both cameras -> se(3) samples weighted by the
//                  product of the three rigidness values (FP64);
//   k_pose_seed    kernel density of each start candidate (previous pose and
//                  the first samples in group order) over all samples (FP64);
//   k_pose_ms      densest candidate, Gaussian mean-shift to the mode,
//                  T_t = exp(p*), M_t = T_t o M_{t-1};
// plus the scale gauge |t_1| = 1.
#include <algorithm>

#include "vo_internal.hpp"


namespace vo {

// P3P groups are solved by 4 lanes each (one lane per quartic root slot), 16
// groups to a 64-lane workgroup.  The valid samples of one workgroup are
// stored contiguously in (group, root) order at slots [64 b, 64 b + bcnt[b]),
// so that the dense sample order of the paper's description is the block
// order followed by the order inside each block.
constexpr int kGrpLanes = 4;
constexpr int kGrpPerBlk = 64 / kGrpLanes;
constexpr int kSlotsPerBlk = 64;
constexpr int kMaxPoseBlks = kMaxGroups / kGrpPerBlk;

struct GroupArgs {
    const float *theta;
    const float *rig;
    const float2 *flows;
    const double *Mprev;   // M_{t-1}
    double *samples;       // SoA [7][ns]: p (6), weight
    int *gcnt;             // [S] samples of each group
    int *gpre;             // [S] first sample of each group inside its block
    int *bcnt;             // [nb][2] samples of each block, groups with a valid setup
    double *bws;           // [nb] weight sum of each block's samples
    float *sampf;          // SoA [7][ns]: whitened p (p_c s_c), log2 weight (FP32)
    const int *status;
    WinDims d;
    int S, t, it, ns;
    uint64_t seed;
    double wt, wr;         // whitening scales s_c of translation and rotation
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

__device__ __forceinline__ void pose_groups_body(const GroupArgs &a)
{
    if (a.status && *a.status != kStatusOk) return;
    const int lane = threadIdx.x, r = lane & (kGrpLanes - 1), base = lane & ~(kGrpLanes - 1);
    const int g = blockIdx.x * kGrpPerBlk + (lane >> 2);
    const int H = a.d.H, W = a.d.W;
    const int64_t HW = (int64_t)H * W;
    // the three pixels of the group (every lane of the group draws the same)
    bool ok = g < a.S;
    int64_t j0 = 0, j1 = 0, j2 = 0;
    if (ok) {
        bool drawn = false;
        for (int att = 0; att < 8 && !drawn; ++att) {
            uint64_t c[4] = {(uint64_t)a.it, (uint64_t)a.t, (uint64_t)g, (uint64_t)att};
            philox4x64_10(c, a.seed, kPoseStream);
            j0 = u32_to_index((uint32_t)(c[0] >> 32), HW);
            j1 = u32_to_index((uint32_t)(c[1] >> 32), HW);
            j2 = u32_to_index((uint32_t)(c[2] >> 32), HW);
            drawn = j0 != j1 && j0 != j2 && j1 != j2;
        }
        ok = drawn;
    }
    // lane r < 3 of the group: point r in camera t-1 and its bearing in camera t
    double Pk[3] = {0.0, 0.0, 0.0}, fk[3] = {0.0, 0.0, 1.0}, wk = 1.0;
    int okk = 1;
    if (ok && r < 3) {
        const int64_t jj = r == 0 ? j0 : (r == 1 ? j1 : j2);
        const int x = (int)(jj % W), y = (int)(jj / W);
        const double th = (double)a.theta[jj];
        const double ray[3] = {(x - a.d.cx) / a.d.fx, (y - a.d.cy) / a.d.fy, 1.0};
        const double *M = a.Mprev;
        mv3(M, ray, Pk);
        for (int c = 0; c < 3; ++c) Pk[c] = th * Pk[c] + M[9 + c];
        okk = Pk[2] > 0;
        double fu = 0.0, fv = 0.0;
        if (okk) {
            double u0 = a.d.fx * Pk[0] / Pk[2] + a.d.cx, v0 = a.d.fy * Pk[1] / Pk[2] + a.d.cy;
            if (a.t == 1) { u0 = x; v0 = y; }   // pi_0 is the pixel itself
            okk = flow_bilinear_d(a.flows + (size_t)(a.t - 1) * HW, H, W, u0, v0, fu, fv);
            if (okk) {
                const double bx = (u0 + fu - a.d.cx) / a.d.fx, by = (v0 + fv - a.d.cy) / a.d.fy;
                const double nb = sqrt(bx * bx + by * by + 1.0);
                fk[0] = bx / nb;
                fk[1] = by / nb;
                fk[2] = 1.0 / nb;
            }
        }
        if (a.rig) wk = (double)a.rig[(size_t)(a.t - 1) * HW + jj];
    }
    // every lane of the group gathers the three points
    double P[9], f[9], w = 1.0;
    bool gok = ok;
#pragma unroll
    for (int k = 0; k < 3; ++k) {
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            P[3 * k + c] = __shfl(Pk[c], base + k, 64);
            f[3 * k + c] = __shfl(fk[c], base + k, 64);
        }
        w *= __shfl(wk, base + k, 64);
        gok = gok && __shfl(okk, base + k, 64) != 0;
    }
    // root slot r: pose, then all three points in front of camera t
    double R[9], tv[3];
    bool val = gok && p3p_root(P, f, r, R, tv);
    if (val)
        for (int k = 0; k < 3; ++k)
            val = val && R[6] * P[3 * k] + R[7] * P[3 * k + 1] + R[8] * P[3 * k + 2] + tv[2] > 0;
    // se(3) log of the root (its rotation angle is the first sort key)
    double key[4] = {0.0, 0.0, 0.0, 0.0};
    double p[6] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
    if (val) {
        se3_log(R, tv, p, &key[0]);
        key[1] = tv[0];
        key[2] = tv[1];
        key[3] = tv[2];
    }
    // canonical order among the group's roots: rotation angle, then t_x, t_y, t_z
    int rank = 0;
#pragma unroll
    for (int q = 0; q < kGrpLanes; ++q) {
        double kq[4];
#pragma unroll
        for (int c = 0; c < 4; ++c) kq[c] = __shfl(key[c], base + q, 64);
        const int vq = __shfl((int)val, base + q, 64);
        int cmp = 0;   // -1: root q precedes this lane's root, +1: follows
#pragma unroll
        for (int c = 3; c >= 0; --c) cmp = kq[c] < key[c] ? -1 : (kq[c] > key[c] ? 1 : cmp);
        if (q != r && vq && (cmp < 0 || (cmp == 0 && q < r))) ++rank;
    }
    if (val)
        for (int c = 0; c < 6; ++c) val = val && isfinite(p[c]);
    // valid samples fill the group's positions without gaps, in canonical order
    const unsigned long long vm = __ballot(val);
    int pos = 0;
#pragma unroll
    for (int q = 0; q < kGrpLanes; ++q) {
        const int rq = __shfl(rank, base + q, 64);
        if (((vm >> (base + q)) & 1ull) && rq < rank) ++pos;
    }
    const int excl = __popcll(vm & ((1ull << base) - 1ull));
    const unsigned long long gm = __ballot(gok && r == 0);
    if (r == 0 && g < a.S) {
        a.gcnt[g] = __popcll((vm >> base) & 0xFull);
        a.gpre[g] = excl;
    }
    double wv_sum = val ? w : 0.0;
    for (int off = 32; off > 0; off >>= 1) wv_sum += __shfl_xor(wv_sum, off, 64);
    if (lane == 0) {
        a.bcnt[2 * blockIdx.x] = __popcll(vm);
        a.bcnt[2 * blockIdx.x + 1] = __popcll(gm);
        a.bws[blockIdx.x] = wv_sum;
    }
    if (val) {
        const size_t sl = (size_t)kSlotsPerBlk * blockIdx.x + excl + pos;
        double *o = a.samples + sl;
        float *of = a.sampf + sl;
        for (int c = 0; c < 6; ++c) {
            o[(size_t)c * a.ns] = p[c];
            of[(size_t)c * a.ns] = (float)(p[c] * (c < 3 ? a.wt : a.wr));
        }
        o[(size_t)6 * a.ns] = w;
        int e;
        const double mt = frexp(w, &e);
        of[(size_t)6 * a.ns] = (float)e + __builtin_amdgcn_logf((float)mt);   // log2 w
    }
}

__global__ void __launch_bounds__(64) k_pose_groups(GroupArgs a) { pose_groups_body(a); }

// the kernels of a pose step over several windows at once (a lockstep batch
// lane): blockIdx.y selects a window's arguments, which are those of a single
// window's launch, so every window gets exactly its own result
// their pointers in the global address space (global_ptr)
__device__ __forceinline__ GroupArgs to_global(GroupArgs a)
{
    a.theta = global_ptr(a.theta);
    a.rig = global_ptr(a.rig);
    a.flows = global_ptr(a.flows);
    a.Mprev = global_ptr(a.Mprev);
    a.samples = global_ptr(a.samples);
    a.gcnt = global_ptr(a.gcnt);
    a.gpre = global_ptr(a.gpre);
    a.bcnt = global_ptr(a.bcnt);
    a.bws = global_ptr(a.bws);
    a.sampf = global_ptr(a.sampf);
    a.status = global_ptr(a.status);
    return a;
}

__global__ void __launch_bounds__(64) k_pose_groups_multi(const GroupArgs *args)
{
    const GroupArgs a = to_global(args[blockIdx.y]);
    if ((int)blockIdx.x * kGrpPerBlk >= a.S) return;   // past this window's blocks
    pose_groups_body(a);
}

// AoS copy [4S][8] of the samples in per-group slots 4g + r (p, weight, valid;
// zero where a group has fewer samples): test hook of the pose step
__global__ void k_samples_aos(const double *soa, const int *gcnt, const int *gpre, int S, int ns,
                              double *aos)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= 4 * S) return;
    const int g = i >> 2, r = i & 3;
    double *o = aos + (size_t)8 * i;
    if (r < gcnt[g]) {
        const size_t src = (size_t)kSlotsPerBlk * (g / kGrpPerBlk) + gpre[g] + r;
        for (int c = 0; c < 7; ++c) o[c] = soa[(size_t)c * ns + src];
        o[7] = 1.0;
    } else {
        for (int c = 0; c < 8; ++c) o[c] = 0.0;
    }
}

__device__ __forceinline__ double mahal2(const double *a, const double *b, double is2t, double is2r)
{
    const double d0 = a[0] - b[0], d1 = a[1] - b[1], d2 = a[2] - b[2];
    const double d3 = a[3] - b[3], d4 = a[4] - b[4], d5 = a[5] - b[5];
    return (d0 * d0 + d1 * d1 + d2 * d2) * is2t + (d3 * d3 + d4 * d4 + d5 * d5) * is2r;
}

__device__ __forceinline__ double wave_sum_d(double v)
{
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
    return v;
}

__device__ __forceinline__ int wave_incl_scan(int v, int lane)
{
    for (int off = 1; off < 64; off <<= 1) {
        const int u = __shfl_up(v, off, 64);
        if (lane >= off) v += u;
    }
    return v;
}

struct SeedArgs {
    const double *samples; // SoA [7][ns], block-compacted
    const int *bcnt;       // [nb][2]
    double *seed_score;    // [n_seeds + 1][8]: p (6), unused, valid
    double *seed_part;     // [n_seeds + 1][kSeedParts] partial densities
    const double *prev;    // previous relative pose T_t
    const double *start_p; // or NULL: candidate 0 is this se(3) point instead (p (6), valid)
    const int *status;
    int ns, nb, have_prev;
    double is2t, is2r;
};

constexpr int kSeedThreads = 256;
constexpr int kSeedParts = 8;                                  // workgroups per candidate
constexpr int kSeedWaves = kSeedParts * kSeedThreads / 64;     // waves sharing one candidate
constexpr int kSeedBatch = 4;                                  // sample blocks in flight per wave

// Partial kernel density of one start candidate (candidate 0: the previous
// pose; candidate k: the (k-1)-th sample in group order) over the sample
// blocks b = w, w + 32, ... of wave w of the candidate's eight workgroups,
// FP64 throughout.  The partials are added in a fixed order by the mean-shift.
__device__ __forceinline__ void pose_seed_body(const SeedArgs &a)
{
    if (a.status && *a.status != kStatusOk) return;
    __shared__ double seed[8];
    __shared__ double red[kSeedThreads / 64];
    const int cand = blockIdx.x / kSeedParts, part = blockIdx.x % kSeedParts;
    const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
    const int gw = part * (kSeedThreads / 64) + wv;
    const int nbw = a.nb > gw ? (a.nb - gw + kSeedWaves - 1) / kSeedWaves : 0;   // blocks of this wave
    // first batch of this wave's samples, in flight while the candidate is found
    double raw[kSeedBatch][7];
    bool ok[kSeedBatch];
    // the slots of a block are loaded whatever its count (they lie inside the
    // buffer; unused ones are masked), so counts and samples travel together
    auto load_batch = [&](int j0) {
#pragma unroll
        for (int u = 0; u < kSeedBatch; ++u) {
            const int j = j0 + u;
            const int b = gw + kSeedWaves * j;
            const int cnt = j < nbw ? a.bcnt[2 * b] : 0;
            ok[u] = lane < cnt;
            const size_t sl = j < nbw ? (size_t)kSlotsPerBlk * b + lane : 0;
#pragma unroll
            for (int c = 0; c < 7; ++c) raw[u][c] = a.samples[(size_t)c * a.ns + sl];
        }
    };
    load_batch(0);
    if (tid < 64) {
        if (cand == 0 && a.start_p) {
            if (tid < 7) seed[tid] = a.start_p[tid];
        } else if (cand == 0) {
            if (tid == 0) {
                seed[6] = a.have_prev ? 1.0 : 0.0;
                if (a.have_prev) {
                    double p[6];
                    se3_log(a.prev, a.prev + 9, p);
                    for (int c = 0; c < 6; ++c) seed[c] = p[c];
                }
            }
        } else {
            // dense index cand - 1: scan the block counts 64 blocks at a time
            const int target = cand - 1;
            int base = 0;
            bool found = false;
            for (int q = 0; q * 64 < a.nb && !found; ++q) {
                const int b = 64 * q + lane;
                const int cnt = b < a.nb ? a.bcnt[2 * b] : 0;
                const int incl = wave_incl_scan(cnt, lane);
                const int tot = __shfl(incl, 63, 64);
                if (target < base + tot) {
                    found = true;
                    const int ex = base + incl - cnt;
                    if (ex <= target && target < ex + cnt) {
                        const size_t sl = (size_t)kSlotsPerBlk * b + (target - ex);
                        for (int c = 0; c < 6; ++c) seed[c] = a.samples[(size_t)c * a.ns + sl];
                    }
                }
                base += tot;
            }
            if (lane == 0) seed[6] = found ? 1.0 : 0.0;
        }
    }
    __syncthreads();
    if (seed[6] == 0.0) {
        if (part == 0 && tid == 0) a.seed_score[8 * cand + 7] = 0.0;
        return;
    }
    double sd[6];
    for (int c = 0; c < 6; ++c) sd[c] = seed[c];
    double s = 0.0;
    for (int j0 = 0; j0 < nbw; j0 += kSeedBatch) {
        if (j0 > 0) load_batch(j0);
#pragma unroll
        for (int u = 0; u < kSeedBatch; ++u)
            if (ok[u]) s += raw[u][6] * exp_nonpos(-0.5 * mahal2(sd, raw[u], a.is2t, a.is2r));
    }
    s = wave_sum_d(s);
    if (lane == 0) red[wv] = s;
    __syncthreads();
    if (tid == 0) {
        double D = 0.0;
        for (int w = 0; w < kSeedThreads / 64; ++w) D += red[w];
        a.seed_part[kSeedParts * cand + part] = D;
        if (part == 0) {
            for (int c = 0; c < 6; ++c) a.seed_score[8 * cand + c] = sd[c];
            a.seed_score[8 * cand + 7] = 1.0;
        }
    }
}

__global__ void __launch_bounds__(kSeedThreads) k_pose_seed(SeedArgs a) { pose_seed_body(a); }

__device__ __forceinline__ SeedArgs to_global(SeedArgs a)
{
    a.samples = global_ptr(a.samples);
    a.bcnt = global_ptr(a.bcnt);
    a.seed_score = global_ptr(a.seed_score);
    a.seed_part = global_ptr(a.seed_part);
    a.prev = global_ptr(a.prev);
    a.start_p = global_ptr(a.start_p);
    a.status = global_ptr(a.status);
    return a;
}

__global__ void __launch_bounds__(kSeedThreads) k_pose_seed_multi(const SeedArgs *args)
{
    const SeedArgs a = to_global(args[blockIdx.y]);
    pose_seed_body(a);
}

struct MsArgs {
    const float *sampf;     // SoA [7][ns], block-compacted: whitened p, log2 weight
    const int *bcnt;        // [nb][2]
    const double *bws;      // [nb] weight sum of each block's samples
    const double *seed_score;
    const double *seed_part;
    double *rel;            // relative poses [T][12]; T_t written at t-1
    double *Mcum;           // cumulative poses [T+1][12]; M_t written
    int *diag;              // [4]
    const int *status;
    int ns, nb, n_seeds, t, max_iters, fallback_prev_frame;
    double wt, wr, tol;     // whitening scales s_c, stop tolerance (Mahalanobis)
};

constexpr int kMsThreads = 512;
constexpr int kMsWaves = kMsThreads / 64;
constexpr int kMsRegs = 16;                         // samples held in registers per lane
constexpr int kMsWaveCap = 64 * kMsRegs;            // register samples per wave
constexpr int kMsListCap = kSlotsPerBlk * (kMaxPoseBlks / kMsWaves);   // samples per wave, at most

// Cross-lane sums without the LDS crossbar.  swap32_sum: lane l gets
// a[l] + a[l + 32] in the lower half and b[l - 32] + b[l] in the upper half
// (gfx950 lane-half swap); swap16_sum: the same between rows 2k and 2k + 1 of
// 16 lanes; dpp: row-local permutations (ror:8 = xor 8, half-mirror, quad xor).
__device__ __forceinline__ float swap32_sum(float a, float b)
{
    const auto r = __builtin_amdgcn_permlane32_swap(__float_as_uint(a), __float_as_uint(b), false, false);
    return __uint_as_float(r[0]) + __uint_as_float(r[1]);
}
__device__ __forceinline__ float swap16_sum(float a, float b)
{
    const auto r = __builtin_amdgcn_permlane16_swap(__float_as_uint(a), __float_as_uint(b), false, false);
    return __uint_as_float(r[0]) + __uint_as_float(r[1]);
}
constexpr int kDppRowRor8 = 0x128, kDppHalfMirror = 0x141, kDppQuadXor1 = 0xB1, kDppQuadXor2 = 0x4E;
template <int CTRL>
__device__ __forceinline__ float dpp(float v)
{
    return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), CTRL, 0xf, 0xf, true));
}
// sum over the 8 lanes of each aligned group of 8
__device__ __forceinline__ float group8_sum(float x)
{
    x += dpp<kDppHalfMirror>(x);
    x += dpp<kDppQuadXor1>(x);
    x += dpp<kDppQuadXor2>(x);
    return x;
}

// Sum of v[0..7] over the wave, transposed: on return every lane l holds the
// wave total of component l >> 3.  Seven exchanges instead of 48 shuffles.
__device__ __forceinline__ float wave_sum8_t(const float *v, int lane)
{
    float a4[4], b2[2];
#pragma unroll
    for (int j = 0; j < 4; ++j) a4[j] = swap32_sum(v[j], v[j + 4]);       // component 4 h1 + j
#pragma unroll
    for (int j = 0; j < 2; ++j) b2[j] = swap16_sum(a4[j], a4[j + 2]);     // 4 h1 + 2 h2 + j
    const bool h3 = lane & 8;
    const float x = (h3 ? b2[1] : b2[0]) + dpp<kDppRowRor8>(h3 ? b2[0] : b2[1]);
    return group8_sum(x);
}

// Gaussian mean-shift from the densest start candidate in one workgroup.
// Wave w owns the sample blocks b = w, w + 8, ...; it lists their samples in
// LDS and holds them as FP32 offsets from the start point P0 in whitened
// coordinates (o_c = (p_c - P0_c) s_c with s_c^2 = log2(e) / (2 sigma_c^2), so
// that the kernel weight at mean m is 2^(-|o - m|^2)), together with
// log2 w - |o|^2: the exponent at m is then that plus 2 o.m - |m|^2, six FMAs
// per sample and no re-centring.  A running log2 density c2 keeps every
// weight in FP32 range.  The mean itself is kept in FP64.  Every wave
// evaluates the same totals, so the stop decision is uniform with one barrier
// per step.
__device__ __forceinline__ void pose_ms_body(const MsArgs &a)
{
    if (a.status && *a.status != kStatusOk) return;
    __shared__ unsigned short widx[kMsWaves][kMsListCap];
    __shared__ double wbest[kMsWaves][8];   // p (6), density, id
    __shared__ double wtot[kMsWaves][4];    // samples, valid groups, weight sum
    __shared__ float red[2][64];
    const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
    double *Tt = a.rel + 12 * (a.t - 1);

    // this wave's sample list (lane j: block wv + 8 j)
    const int b = wv + kMsWaves * lane;
    const bool hb = b < a.nb;
    const int cnt = hb ? a.bcnt[2 * b] : 0;
    const int gv = hb ? a.bcnt[2 * b + 1] : 0;
    const double bw = hb ? a.bws[b] : 0.0;
    // start candidates: lane-parallel densities (partials added in order)
    double dens = -1.0;
    double cp[6] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
    int id = 1 << 30;
    if (tid <= a.n_seeds) {   // all loads issued together, selected afterwards
        double part[kSeedParts], cc[6];
        for (int p = 0; p < kSeedParts; ++p) part[p] = a.seed_part[kSeedParts * tid + p];
        for (int c = 0; c < 6; ++c) cc[c] = a.seed_score[8 * tid + c];
        if (a.seed_score[8 * tid + 7] != 0.0) {
            double D = 0.0;
            for (int p = 0; p < kSeedParts; ++p) D += part[p];
            dens = D;
            id = tid;
            for (int c = 0; c < 6; ++c) cp[c] = cc[c];
        }
    }
    const int incl = wave_incl_scan(cnt, lane);
    const int Nw = __shfl(incl, 63, 64);
    const int ex = incl - cnt;
    const int nbw = a.nb > wv ? (a.nb - wv + kMsWaves - 1) / kMsWaves : 0;   // blocks of this wave
    for (int j = 0; j < nbw; ++j) {
        const int cj = __builtin_amdgcn_readlane(cnt, j), ej = __builtin_amdgcn_readlane(ex, j);
        if (lane < cj) widx[wv][ej + lane] = (unsigned short)(kSlotsPerBlk * (wv + kMsWaves * j) + lane);
    }
    // wave arg-max of the candidates, earliest on ties
    double bd = dens;
    int bi = id;
    for (int o = 32; o > 0; o >>= 1) {
        const double so = __shfl_xor(bd, o, 64);
        const int io = __shfl_xor(bi, o, 64);
        if (so > bd || (so == bd && io < bi)) { bd = so; bi = io; }
    }
    const int gsum = wave_incl_scan(gv, lane);
    const double wsum = wave_sum_d(bw);
    if (id == bi && bi < (1 << 30))
        for (int c = 0; c < 6; ++c) wbest[wv][c] = cp[c];
    if (lane == 0) {
        wbest[wv][6] = bd;
        wbest[wv][7] = (double)bi;
        wtot[wv][0] = (double)Nw;
        wtot[wv][2] = wsum;
    }
    if (lane == 63) wtot[wv][1] = (double)gsum;
    __syncthreads();
    // workgroup totals and the densest candidate (every thread, same order)
    int N = 0, groups = 0, bw_ = 0;
    double WS = 0.0, D0 = -1.0, bid = (double)(1 << 30);
    for (int w = 0; w < kMsWaves; ++w) {
        N += (int)wtot[w][0];
        groups += (int)wtot[w][1];
        WS += wtot[w][2];
        const double so = wbest[w][6], io = wbest[w][7];
        if (so > D0 || (so == D0 && io < bid)) { D0 = so; bid = io; bw_ = w; }
    }
    if (N == 0 || !(WS > 0.0) || !(bid < (double)(1 << 30))) {
        if (tid == 0) {
            if (a.fallback_prev_frame)
                for (int k = 0; k < 12; ++k) Tt[k] = a.rel[12 * (a.t - 2) + k];
            pose_mul(Tt, a.Mcum + 12 * (a.t - 1), a.Mcum + 12 * a.t);
            a.diag[0] = N;
            a.diag[1] = groups;
            a.diag[2] = 0;
            a.diag[3] = 1;
        }
        return;
    }
    // start: the candidate in whitened coordinates, rounded to FP32 (the
    // register frame is centred on that exactly representable point)
    double sc[6], P0[6];
    for (int c = 0; c < 6; ++c) {
        sc[c] = c < 3 ? a.wt : a.wr;
        P0[c] = (double)(float)(wbest[bw_][c] * sc[c]);
    }
    const int nreg = min(Nw, kMsWaveCap);

    float o[kMsRegs][6], lw[kMsRegs];
    // register samples: every load in flight at once, straight into place
#pragma unroll
    for (int m = 0; m < kMsRegs; ++m) {
        const int i = lane + 64 * m;
        const bool in = i < nreg;
        const int sl = in ? widx[wv][i] : 0;
#pragma unroll
        for (int c = 0; c < 6; ++c) o[m][c] = in ? a.sampf[(size_t)c * a.ns + sl] : 0.0f;
        lw[m] = in ? a.sampf[(size_t)6 * a.ns + sl] : -INFINITY;
    }
    // o: offset from the start point; lw becomes log2 w - |o|^2, so that the
    // exponent at mean m is lw - |o|^2 + 2 o.m - |m|^2 with no re-centring
#pragma unroll
    for (int m = 0; m < kMsRegs; ++m) {
        float n2 = 0.0f;
#pragma unroll
        for (int c = 0; c < 6; ++c) {
            o[m][c] -= (float)P0[c];
            n2 = fmaf(o[m][c], o[m][c], n2);
        }
        lw[m] -= n2;
    }
    // c2: log2 of the density at the current mean (starts at the candidate's)
    float c2 = D0 > 0.0 ? (float)log2(D0) : 0.0f;
    double cen[6] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0};   // whitened mean - P0
    const double tol2 = a.tol * a.tol * 0.72134752044448170;
    int it = 0;
    for (; it < a.max_iters && D0 > 0.0; ++it) {
        float cf[6], tc[6], cn2 = 0.0f;
#pragma unroll
        for (int c = 0; c < 6; ++c) {
            cf[c] = (float)cen[c];
            tc[c] = 2.0f * cf[c];
            cn2 = fmaf(cf[c], cf[c], cn2);
        }
        const float bias = -c2 - cn2;
        float acc[8] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
#pragma unroll
        for (int m = 0; m < kMsRegs; ++m) {
            if (lane + 64 * m < nreg) {
                float e = lw[m] + bias;
#pragma unroll
                for (int c = 0; c < 6; ++c) e = fmaf(tc[c], o[m][c], e);
                const float k = __builtin_amdgcn_exp2f(e);
                acc[6] += k;
#pragma unroll
                for (int c = 0; c < 6; ++c) acc[c] = fmaf(k, o[m][c], acc[c]);
            }
        }
        if (Nw > kMsWaveCap) {
            // the rest from memory: offsets from the start, centred distance
            for (int i = kMsWaveCap + lane; i < Nw; i += 64) {
                const int sl = widx[wv][i];
                float d[6], q2 = 0.0f;
                for (int c = 0; c < 6; ++c) {
                    d[c] = a.sampf[(size_t)c * a.ns + sl] - (float)P0[c];
                    const float dc = d[c] - cf[c];
                    q2 = fmaf(dc, dc, q2);
                }
                const float k = __builtin_amdgcn_exp2f(a.sampf[(size_t)6 * a.ns + sl] - c2 - q2);
                acc[6] += k;
                for (int c = 0; c < 6; ++c) acc[c] = fmaf(k, d[c], acc[c]);
            }
        }
        const float x = wave_sum8_t(acc, lane);
        float *rb = red[it & 1];
        if ((lane & 7) == 0) rb[8 * (lane >> 3) + wv] = x;   // [component][wave]
        __syncthreads();
        const float y = group8_sum(rb[lane]);   // lanes 8c .. 8c + 7: total of component c
        const double den = (double)__int_as_float(__builtin_amdgcn_readlane(__float_as_int(y), 48));
        if (!(den > 0.0)) break;
        const double iden = 1.0 / den;
        double step2 = 0.0;
#pragma unroll
        for (int c = 0; c < 6; ++c) {
            const double mc = (double)__int_as_float(__builtin_amdgcn_readlane(__float_as_int(y), 8 * c)) * iden;
            const double sh = mc - cen[c];
            cen[c] = mc;
            step2 += sh * sh;
        }
        c2 += __builtin_amdgcn_logf((float)den);
        if (step2 < tol2) { ++it; break; }
    }
    if (tid == 0) {
        double pp[6], R[9], tv[3];
        for (int c = 0; c < 6; ++c) pp[c] = (P0[c] + cen[c]) / sc[c];
        se3_exp(pp, R, tv);
        for (int k = 0; k < 9; ++k) Tt[k] = R[k];
        for (int k = 0; k < 3; ++k) Tt[9 + k] = tv[k];
        pose_mul(Tt, a.Mcum + 12 * (a.t - 1), a.Mcum + 12 * a.t);
        a.diag[0] = N;
        a.diag[1] = groups;
        a.diag[2] = it;
        a.diag[3] = 0;
    }
}

__global__ void __launch_bounds__(kMsThreads) k_pose_ms(MsArgs a) { pose_ms_body(a); }

__device__ __forceinline__ MsArgs to_global(MsArgs a)
{
    a.sampf = global_ptr(a.sampf);
    a.bcnt = global_ptr(a.bcnt);
    a.bws = global_ptr(a.bws);
    a.seed_score = global_ptr(a.seed_score);
    a.seed_part = global_ptr(a.seed_part);
    a.rel = global_ptr(a.rel);
    a.Mcum = global_ptr(a.Mcum);
    a.diag = global_ptr(a.diag);
    a.status = global_ptr(a.status);
    return a;
}

__global__ void __launch_bounds__(kMsThreads) k_pose_ms_multi(const MsArgs *args)
{
    const MsArgs a = to_global(args[blockIdx.y]);
    pose_ms_body(a);
}

// ---------------------------------------------------------------------------
// All-pixel start (pose_start = 1): every candidate -- the previous pose, then
// each valid sample in (group, root) order -- is scored by sum_j W_t^j ell_t^j
// over every pixel with M_t = T_c o M_{t-1} (a missing item counts log 1/2);
// the first maximum starts the mean-shift.  The flow lookup at pi_{t-1}(theta)
// and the terms that depend only on the observed flow do not depend on the
// candidate: they are computed once per pixel and block, and the candidate
// loop is arithmetic only.
// ---------------------------------------------------------------------------
constexpr int kCandChunk = 64;     // candidates per scoring workgroup
constexpr float kLogHalfF = -0.69314718055994531f;
constexpr int kCandThreads = 256;
constexpr int kCandPix = 4;        // pixels per thread per pass

struct CandFrameArgs {
    const double *samples;   // SoA [7][ns] block-compacted
    const int *bcnt;         // [nb][2]
    const double *prev;      // previous relative pose T_t (if have_prev)
    const double *Mprev;     // M_{t-1}
    float *cF;               // [n][12] FP32 frames (R - I, t) of M_t = T_c o M_{t-1}
    int *cslot;              // [n] sample slot; -1 previous pose; -2 no candidate
    int *cn;                 // candidates 1 + valid samples
    const int *status;
    int nb, ns, have_prev;
};

// block 0: the previous pose and the count; block b + 1: the samples of
// sample block b at dense indices 1 + (samples of blocks before b) + lane
__global__ void __launch_bounds__(64) k_cand_frames(CandFrameArgs a)
{
    if (a.status && *a.status != kStatusOk) return;
    const int lane = threadIdx.x;
    const int b = (int)blockIdx.x - 1;
    int pre = 0;
    for (int q = lane; q < (b < 0 ? a.nb : b); q += 64) pre += a.bcnt[2 * q];
    for (int o = 32; o > 0; o >>= 1) pre += __shfl_xor(pre, o, 64);
    double T[12];
    int dense = -1, slot = -2;
    if (b < 0) {
        if (lane == 0) {
            *a.cn = 1 + pre;
            dense = 0;
            slot = a.have_prev ? -1 : -2;
            for (int k = 0; k < 12; ++k) T[k] = a.have_prev ? a.prev[k] : ((k == 0 || k == 4 || k == 8) ? 1.0 : 0.0);
        }
    } else if (lane < a.bcnt[2 * b]) {
        slot = kSlotsPerBlk * b + lane;
        dense = 1 + pre + lane;
        double pv[6];
        for (int c = 0; c < 6; ++c) pv[c] = a.samples[(size_t)c * a.ns + slot];
        se3_exp(pv, T, T + 9);
    }
    if (dense < 0) return;
    double Mt[12];
    pose_mul(T, a.Mprev, Mt);
    float *f = a.cF + (size_t)12 * dense;
    for (int i = 0; i < 9; ++i) f[i] = (float)(Mt[i] - ((i == 0 || i == 4 || i == 8) ? 1.0 : 0.0));
    for (int i = 0; i < 3; ++i) f[9 + i] = (float)Mt[9 + i];
    a.cslot[dense] = slot;
}

struct CandScoreArgs {
    const float *theta;
    const float *rig;        // W_t of frame t (or NULL: 1)
    const float2 *flows;
    const double *Mprev;     // M_{t-1}
    const float *cF;
    const int *cslot;
    const int *cn;
    float *part;             // [candidate][kCandTiles] partial scores
    const int *status;
    EmisParams e;
    int T, H, W, t;
};

// grid (kCandTiles pixel ranges, candidate chunks of kCandChunk); MODEL 0 Fisk
// residual model (Eq. 5), 1 Gaussian flow error
template <int MODEL>
__global__ void __launch_bounds__(kCandThreads) k_cand_score(CandScoreArgs a)
{
    if (a.status && *a.status != kStatusOk) return;
    const int n = *a.cn;
    const int c0 = blockIdx.y * kCandChunk;
    if (c0 >= n) return;
    __shared__ FrameF hf[kCandChunk];
    __shared__ int hv[kCandChunk];
    __shared__ FrameF pf;
    __shared__ float ws[kCandThreads / 64][kCandChunk];
    const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
    const int m = min(kCandChunk, n - c0);
    for (int i = tid; i < m * 12; i += kCandThreads) (&hf[0].D[0])[i] = a.cF[(size_t)12 * c0 + i];
    if (tid < kCandChunk) hv[tid] = tid < m && a.cslot[c0 + tid] != -2;
    for (int i = tid; i < (kCandThreads / 64) * kCandChunk; i += kCandThreads) (&ws[0][0])[i] = 0.0f;
    if (tid == 0) {
        for (int i = 0; i < 9; ++i) pf.D[i] = (float)(a.Mprev[i] - ((i == 0 || i == 4 || i == 8) ? 1.0 : 0.0));
        for (int i = 0; i < 3; ++i) pf.t[i] = (float)a.Mprev[9 + i];
    }
    __syncthreads();
    const EmisParams &e = a.e;
    const int64_t HW = (int64_t)a.H * a.W;
    const int64_t j0 = HW * blockIdx.x / kCandTiles, j1 = HW * (blockIdx.x + 1) / kCandTiles;
    const float2 *X = a.flows + (size_t)(a.t - 1) * HW;
    for (int64_t pb = j0; pb < j1; pb += kCandThreads * kCandPix) {
        // the pixels' candidate-free terms
        float xh[kCandPix], yh[kCandPix], th[kCandPix], w[kCandPix], dx0[kCandPix], dy0[kCandPix];
        float vu[kCandPix], vv[kCandPix], la[kCandPix], beta[kCandPix], k0[kCandPix];
        bool ok[kCandPix];
#pragma unroll
        for (int k = 0; k < kCandPix; ++k) {
            const int64_t j = pb + tid + (int64_t)k * kCandThreads;
            const bool in = j < j1;
            const int jj = in ? (int)j : 0;
            const int y = jj / a.W, x = jj - y * a.W;
            xh[k] = ((float)x - e.cx) * e.ifx;
            yh[k] = ((float)y - e.cy) * e.ify;
            th[k] = a.theta[jj];
            w[k] = in ? (a.rig ? a.rig[(size_t)(a.t - 1) * HW + jj] : 1.0f) : 0.0f;
            dx0[k] = 0.0f;
            dy0[k] = 0.0f;
            bool v = in && th[k] > 0.0f;
            if (a.t > 1) v = v && displacement(pf, xh[k], yh[k], th[k], e.fx, e.fy, dx0[k], dy0[k]);
            float fu = 0.0f, fv = 0.0f;
            v = v && sample_flow(X, a.H, a.W, add_nc((float)x, dx0[k]), add_nc((float)y, dy0[k]), fu, fv);
            ok[k] = v;
            vu[k] = fu;
            vv[k] = fv;
            const float vn2 = fmaf(fu, fu, fv * fv);
            const float vn = __builtin_amdgcn_sqrtf(vn2);
            la[k] = fmaf(e.a2, vn, e.log_a1);
            if constexpr (MODEL == 1) {
                // d = log(mu/rho) = (x - m) / s: k0 = m, beta = 1 / s = ln 2 / alpha
                k0[k] = fmaxf(e.lam2 * vn2, e.x_floor);
                beta[k] = kLn2F * fast_exp(-la[k]);
            } else {
                beta[k] = fmaxf(fmaf(e.b1, vn, e.b2), e.beta_min);
                const float lm = fast_log(fmaxf(e.lam2 * vn2, e.x_floor));
                // d = log(mu/rho) = k0 - (beta - 1) log x + 2 softplus(beta (log x - log alpha))
                k0[k] = (beta[k] - 1.0f) * lm - 2.0f * softplus(beta[k] * (lm - la[k]));
            }
        }
        for (int h0 = 0; h0 < kCandChunk; h0 += 8) {
            float acc[8];
#pragma unroll
            for (int u = 0; u < 8; ++u) {
                acc[u] = 0.0f;
                if (!hv[h0 + u]) continue;
                const FrameF f = hf[h0 + u];
#pragma unroll
                for (int k = 0; k < kCandPix; ++k) {
                    float ell = kLogHalfF;
                    float dx1, dy1;
                    if (ok[k] && displacement(f, xh[k], yh[k], th[k], e.fx, e.fy, dx1, dy1)) {
                        const float rx = sub_nc(sub_nc(dx1, dx0[k]), vu[k]), ry = sub_nc(sub_nc(dy1, dy0[k]), vv[k]);
                        const float x2 = fminf(fmaxf(fmaf(rx, rx, ry * ry), e.x_floor), 1e30f);
                        float d;
                        if constexpr (MODEL == 1) {
                            d = (x2 - k0[k]) * beta[k];
                        } else {
                            const float lx = fast_log(x2);
                            d = k0[k] - (beta[k] - 1.0f) * lx + 2.0f * softplus(beta[k] * (lx - la[k]));
                        }
                        ell = emis_from_d(d).ell;
                    }
                    acc[u] = fmaf(w[k], ell, acc[u]);
                }
            }
            // lanes 8u .. 8u + 7 get the wave total of candidate h0 + u
            const float tot = wave_sum8_t(acc, lane);
            if ((lane & 7) == 0) ws[wv][h0 + (lane >> 3)] += tot;
        }
    }
    __syncthreads();
    if (tid < m) {
        float sum = 0.0f;
        for (int q = 0; q < kCandThreads / 64; ++q) sum += ws[q][tid];
        a.part[(size_t)(c0 + tid) * kCandTiles + blockIdx.x] = sum;
    }
}

// one wave per candidate: FP64 total of its tile partials in a fixed order
__global__ void __launch_bounds__(256) k_cand_sum(const float *part, const int *cslot, const int *cn,
                                                  double *score, const int *status)
{
    if (status && *status != kStatusOk) return;
    const int c = blockIdx.x * 4 + (threadIdx.x >> 6), lane = threadIdx.x & 63;
    if (c >= *cn) return;
    double s = 0.0;
    for (int q = lane; q < kCandTiles; q += 64) s += (double)part[(size_t)c * kCandTiles + q];
    s = wave_sum_d(s);
    if (lane == 0) score[c] = cslot[c] == -2 ? -INFINITY : s;
}

// first maximum over the candidates -> the start's se(3) point (p (6), valid)
__global__ void __launch_bounds__(1024) k_cand_pick(const double *score, const int *cslot, const int *cn,
                                                    const double *samples, int ns, const double *prev,
                                                    double *start_p, const int *status)
{
    if (status && *status != kStatusOk) return;
    __shared__ double bs[16];
    __shared__ int bi[16];
    const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
    const int n = *cn;
    double best = -INFINITY;
    int idx = 1 << 30;
    for (int c = tid; c < n; c += 1024) {
        const double v = score[c];
        if (v > best) { best = v; idx = c; }   // ascending c: the first maximum stays
    }
    for (int o = 32; o > 0; o >>= 1) {
        const double so = __shfl_xor(best, o, 64);
        const int io = __shfl_xor(idx, o, 64);
        if (so > best || (so == best && io < idx)) { best = so; idx = io; }
    }
    if (lane == 0) { bs[wv] = best; bi[wv] = idx; }
    __syncthreads();
    if (tid == 0) {
        best = bs[0];
        idx = bi[0];
        for (int q = 1; q < 16; ++q)
            if (bs[q] > best || (bs[q] == best && bi[q] < idx)) { best = bs[q]; idx = bi[q]; }
        const bool ok = idx < n && best > -INFINITY;
        start_p[6] = ok ? 1.0 : 0.0;
        if (ok) {
            const int sl = cslot[idx];
            if (sl == -1) {
                se3_log(prev, prev + 9, start_p);
            } else {
                for (int c = 0; c < 6; ++c) start_p[c] = samples[(size_t)c * ns + sl];
            }
        }
    }
}

// scale gauge |t_1| = 1: translations, depth range, cumulative poses (the
// depth map is rescaled by the rigidness pass that precedes this kernel)
__device__ __forceinline__ void gauge_poses_body(double *rel, double *Mcum, double *range, int T, const int *status)
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

__global__ void k_gauge_poses(double *rel, double *Mcum, double *range, int T, const int *status)
{
    gauge_poses_body(rel, Mcum, range, T, status);
}

struct GaugeArgs {
    double *rel, *Mcum, *range;
    const int *status;
    int T;
};

__global__ void k_gauge_poses_multi(const GaugeArgs *args)
{
    const GaugeArgs a = args[blockIdx.y];
    gauge_poses_body(global_ptr(a.rel), global_ptr(a.Mcum), global_ptr(a.range), a.T, global_ptr(a.status));
}

__global__ void k_cumulative(const double *rel, double *Mcum, int T)
{
    if (threadIdx.x != 0) return;
    for (int k = 0; k < 12; ++k) Mcum[k] = (k == 0 || k == 4 || k == 8) ? 1.0 : 0.0;
    for (int t = 1; t <= T; ++t) pose_mul(rel + 12 * (t - 1), Mcum + 12 * (t - 1), Mcum + 12 * t);
}

// ---------------------------------------------------------------------------
// Arguments of the three kernels of a pose step (the start candidates of the
// KDE start; the all-pixel start replaces candidate 0 and drops the others)
static void pose_step_args(voldor_ctx *c, const float *theta, const float *rig, const float2 *flows,
                           const WinDims &d, const PoseParams &pp, int t, int it, int have_prev,
                           double *rel_poses, GroupArgs &g, SeedArgs &sa, MsArgs &m)
{
    const int nb = (pp.S + kGrpPerBlk - 1) / kGrpPerBlk;
    const int ns = kSlotsPerBlk * nb;
    g.theta = theta;
    g.rig = d.use_w ? rig : nullptr;
    g.flows = flows;
    g.Mprev = c->Mcum + 12 * (t - 1);
    g.samples = c->samples;
    g.gcnt = c->gcnt;
    g.gpre = c->gpre;
    g.bcnt = c->bcnt;
    g.bws = c->bws;
    g.sampf = c->sampf;
    g.wt = sqrt(0.72134752044448170 / pp.s2t);   // s_c^2 = log2(e) / (2 sigma_c^2)
    g.wr = sqrt(0.72134752044448170 / pp.s2r);
    g.status = c->status;
    g.d = d;
    g.S = pp.S;
    g.t = t;
    g.it = it;
    g.ns = ns;
    g.seed = pp.seed;
    sa.samples = c->samples;
    sa.bcnt = c->bcnt;
    sa.seed_score = c->seed_score;
    sa.seed_part = c->seed_part;
    sa.prev = rel_poses + 12 * (t - 1);
    sa.start_p = nullptr;
    sa.status = c->status;
    sa.ns = ns;
    sa.nb = nb;
    sa.have_prev = have_prev;
    sa.is2t = 1.0 / pp.s2t;
    sa.is2r = 1.0 / pp.s2r;
    m.sampf = c->sampf;
    m.bcnt = c->bcnt;
    m.bws = c->bws;
    m.seed_score = c->seed_score;
    m.seed_part = c->seed_part;
    m.rel = rel_poses;
    m.Mcum = c->Mcum;
    m.diag = c->pose_diag + 4 * (t - 1);
    m.status = c->status;
    m.ns = ns;
    m.nb = nb;
    m.n_seeds = pp.n_seeds;
    m.t = t;
    m.max_iters = pp.ms_max_iters;
    m.fallback_prev_frame = (!have_prev && t >= 2) ? 1 : 0;
    m.wt = g.wt;
    m.wr = g.wr;
    m.tol = pp.ms_tol;
}

int launch_pose_step(voldor_ctx *c, const float *theta, const float *rig, const float2 *flows,
                     const WinDims &d, const EmisParams &e, const PoseParams &pp, int t, int it,
                     int have_prev, double *rel_poses, hipStream_t s)
{
    GroupArgs g;
    SeedArgs sa;
    MsArgs m;
    pose_step_args(c, theta, rig, flows, d, pp, t, it, have_prev, rel_poses, g, sa, m);
    const int nb = sa.nb, ns = sa.ns;
    hipLaunchKernelGGL(k_pose_groups, dim3(nb), dim3(64), 0, s, g);
    const bool allpix = pp.pose_start == 1;
    if (allpix) {
        CandFrameArgs cf;
        cf.samples = c->samples;
        cf.bcnt = c->bcnt;
        cf.prev = rel_poses + 12 * (t - 1);
        cf.Mprev = c->Mcum + 12 * (t - 1);
        cf.cF = c->cand_F;
        cf.cslot = c->cand_slot;
        cf.cn = c->cand_n;
        cf.status = c->status;
        cf.nb = nb;
        cf.ns = ns;
        cf.have_prev = have_prev;
        hipLaunchKernelGGL(k_cand_frames, dim3(nb + 1), dim3(64), 0, s, cf);
        CandScoreArgs cs;
        cs.theta = theta;
        cs.rig = d.use_w ? rig : nullptr;
        cs.flows = flows;
        cs.Mprev = c->Mcum + 12 * (t - 1);
        cs.cF = c->cand_F;
        cs.cslot = c->cand_slot;
        cs.cn = c->cand_n;
        cs.part = c->cand_part;
        cs.status = c->status;
        cs.e = e;
        cs.T = d.T;
        cs.H = d.H;
        cs.W = d.W;
        cs.t = t;
        const int ncand = 1 + ns;   // upper bound; chunks past the count exit
        const dim3 cgrid(kCandTiles, (ncand + kCandChunk - 1) / kCandChunk);
        if (e.model)
            hipLaunchKernelGGL(k_cand_score<1>, cgrid, dim3(kCandThreads), 0, s, cs);
        else
            hipLaunchKernelGGL(k_cand_score<0>, cgrid, dim3(kCandThreads), 0, s, cs);
        hipLaunchKernelGGL(k_cand_sum, dim3((ncand + 3) / 4), dim3(256), 0, s, c->cand_part, c->cand_slot,
                           c->cand_n, c->cand_score, c->status);
        hipLaunchKernelGGL(k_cand_pick, dim3(1), dim3(1024), 0, s, c->cand_score, c->cand_slot, c->cand_n,
                           c->samples, ns, rel_poses + 12 * (t - 1), c->cand_start, c->status);
        sa.start_p = c->cand_start;
        m.n_seeds = 0;
    }
    hipLaunchKernelGGL(k_pose_seed, dim3((m.n_seeds + 1) * kSeedParts), dim3(kSeedThreads), 0, s, sa);
    hipLaunchKernelGGL(k_pose_ms, dim3(1), dim3(kMsThreads), 0, s, m);
    return hipGetLastError() == hipSuccess ? 0 : VOLDOR_EDEVICE;
}

void plan_pose_step(Plan &p, std::vector<MultiLaunch> &out, const std::vector<WinRef> &w,
                    const std::vector<int> &idx, int t, int it)
{
    const int n = (int)idx.size();
    std::vector<GroupArgs> g(n);
    std::vector<SeedArgs> sa(n);
    std::vector<MsArgs> m(n);
    int nb_max = 0;
    for (int k = 0; k < n; ++k) {
        const WinRef &r = w[idx[k]];
        WinDims d = r.d;
        d.use_w = it > 0 ? 1 : 0;
        pose_step_args(r.c, r.depth, r.rig, r.X, d, r.pp, t, it, (it > 0 || t == 1) ? 1 : 0, r.poses, g[k],
                       sa[k], m[k]);
        nb_max = std::max(nb_max, sa[k].nb);
    }
    // every window of a batch has the same number of start candidates
    const int n_seeds = n ? m[0].n_seeds : 0;
    MultiLaunch l = {};
    l.nwin = n;
    l.kind = kMultiPoseGroups;
    l.off = p.put(g.data(), n);
    l.gx = nb_max;
    out.push_back(l);
    l.kind = kMultiPoseSeed;
    l.off = p.put(sa.data(), n);
    l.gx = (n_seeds + 1) * kSeedParts;
    out.push_back(l);
    l.kind = kMultiPoseMs;
    l.off = p.put(m.data(), n);
    l.gx = 1;
    out.push_back(l);
}

void plan_gauge_poses(Plan &p, std::vector<MultiLaunch> &out, const std::vector<WinRef> &w,
                      const std::vector<int> &idx)
{
    const int n = (int)idx.size();
    std::vector<GaugeArgs> g(n);
    for (int k = 0; k < n; ++k) {
        const WinRef &r = w[idx[k]];
        g[k].rel = r.poses;
        g[k].Mcum = r.c->Mcum;
        g[k].range = r.c->range;
        g[k].status = r.c->status;
        g[k].T = r.d.T;
    }
    MultiLaunch l = {};
    l.kind = kMultiGauge;
    l.nwin = n;
    l.off = p.put(g.data(), n);
    l.gx = 1;
    out.push_back(l);
}

int launch_pose_multi(const MultiLaunch &m, const unsigned char *dev, hipStream_t s)
{
    if (m.nwin < 1) return 0;
    const dim3 grid(m.gx, m.nwin);
    switch (m.kind) {
    case kMultiPoseGroups:
        hipLaunchKernelGGL(k_pose_groups_multi, grid, dim3(64), 0, s, (const GroupArgs *)(dev + m.off));
        break;
    case kMultiPoseSeed:
        hipLaunchKernelGGL(k_pose_seed_multi, grid, dim3(kSeedThreads), 0, s, (const SeedArgs *)(dev + m.off));
        break;
    case kMultiPoseMs:
        hipLaunchKernelGGL(k_pose_ms_multi, grid, dim3(kMsThreads), 0, s, (const MsArgs *)(dev + m.off));
        break;
    case kMultiGauge:
        hipLaunchKernelGGL(k_gauge_poses_multi, grid, dim3(64), 0, s, (const GaugeArgs *)(dev + m.off));
        break;
    default:
        return VOLDOR_EINVAL;
    }
    return hipGetLastError() == hipSuccess ? 0 : VOLDOR_EDEVICE;
}

int launch_samples_aos(voldor_ctx *c, int S, double *out, hipStream_t s)
{
    const int ns = kSlotsPerBlk * ((S + kGrpPerBlk - 1) / kGrpPerBlk);
    hipLaunchKernelGGL(k_samples_aos, dim3((4 * S + 255) / 256), dim3(256), 0, s, c->samples, c->gcnt,
                       c->gpre, S, ns, out);
    return hipGetLastError() == hipSuccess ? 0 : VOLDOR_EDEVICE;
}

size_t pose_seed_parts() { return kSeedParts; }

size_t pose_sample_slots(int S_max)
{
    return (size_t)kSlotsPerBlk * ((S_max + kGrpPerBlk - 1) / kGrpPerBlk);
}

int launch_gauge_poses(voldor_ctx *c, double *rel_poses, const WinDims &d, hipStream_t s)
{
    hipLaunchKernelGGL(k_gauge_poses, dim3(1), dim3(64), 0, s, rel_poses, c->Mcum, c->range, d.T, c->status);
    return hipGetLastError() == hipSuccess ? 0 : VOLDOR_EDEVICE;
}

int launch_cumulative(voldor_ctx *c, const double *rel_poses, int T, hipStream_t s)
{
    hipLaunchKernelGGL(k_cumulative, dim3(1), dim3(64), 0, s, rel_poses, c->Mcum, T);
    return hipGetLastError() == hipSuccess ? 0 : VOLDOR_EDEVICE;
}

}  // namespace vo
