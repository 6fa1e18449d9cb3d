// vo_api.hip -- the C ABI (include/voldor.h): argument checking, context
// workspace, and the launch sequence of one window (Table 1):
//   bootstrap; for each iteration: pose of frames 1..T in order, the
//   directional sweeps, the unsmoothed rigidness, the scale gauge;
//   finally the log-likelihood.
// All launches go to the caller's stream; only voldor_window's final status
// read and the host outputs of the step entry points synchronise.
#include <math.h>
#include <stdlib.h>
#include <string.h>

#include "vo_internal.hpp"

using namespace vo;

namespace {

__global__ void k_reset_status(int *status)
{
    if (threadIdx.x == 0) *status = kStatusOk;
}

bool params_ok(const voldor_params *p)
{
    if (!p || p->struct_size != sizeof(voldor_params)) return false;
    if (p->n_iters < 1 || p->sweeps_per_iter < 1) return false;
    if (p->n_pose_groups < 1 || p->n_pose_groups > kMaxGroups) return false;
    if (p->n_seeds < 1 || p->n_seeds > kMaxSeeds || p->ms_max_iters < 0) return false;
    if (p->lmeds_hypotheses < 1 || p->lmeds_hypotheses > kMaxHyp) return false;
    if (p->lmeds_eval_pixels < 8 || p->lmeds_eval_pixels > kEvalThreads * kEvalPerThread) return false;
    if (!(p->gamma >= 0.5 && p->gamma < 1.0) || !(p->lambda > 0) || !(p->a1 > 0)) return false;
    if (!isfinite(p->a2) || !isfinite(p->b1) || !isfinite(p->b2)) return false;
    if (!(p->sigma2_trans > 0) || !(p->sigma2_rot > 0)) return false;
    if (!(p->beta_min > 0) || !(p->x_floor > 0) || !(p->ms_tol >= 0)) return false;
    if (!(p->depth_lo >= 0) || !(p->depth_hi >= 0)) return false;
    if (p->depth_lo > 0 && p->depth_hi > 0 && !(p->depth_hi > p->depth_lo)) return false;
    if (p->criterion != VOLDOR_CRITERION_MIE && p->criterion != VOLDOR_CRITERION_MLE) return false;
    if (p->pose_start != 0 && p->pose_start != 1) return false;
    if (p->residual_model != VOLDOR_RESIDUAL_FISK && p->residual_model != VOLDOR_RESIDUAL_GAUSS) return false;
    return true;
}

// a window fits the context, and a chain of either direction fits the LDS of
// one workgroup under the depth criterion in use
bool dims_ok(const voldor_ctx *c, int T, int H, int W, int criterion)
{
    if (!c) return false;
    if (T < 1 || T > c->T_max || H < 16 || W < 16 || H > c->H_max || W > c->W_max) return false;
    int ntr = 512, ntc = 512, la = 0;
    sweep_cfg_for(c, 0, W, T, criterion, &ntr, &la);
    sweep_cfg_for(c, 1, H, T, criterion, &ntc, &la);
    if ((int)sweep_lds_bytes(T, W, criterion, ntr) > c->max_lds ||
        (int)sweep_lds_bytes(T, H, criterion, ntc) > c->max_lds)
        return false;
    return true;
}

bool K_ok(const double *K)
{
    return K && K[0] > 0 && K[1] > 0 && isfinite(K[0]) && isfinite(K[1]) && isfinite(K[2]) &&
           isfinite(K[3]);
}

WinDims dims(int T, int H, int W, const double *K)
{
    WinDims d;
    d.T = T;
    d.H = H;
    d.W = W;
    d.use_w = 0;
    d.fx = K[0];
    d.fy = K[1];
    d.cx = K[2];
    d.cy = K[3];
    return d;
}

EmisParams emis(const double *K, const voldor_params *p)
{
    EmisParams e;
    e.fx = (float)K[0];
    e.fy = (float)K[1];
    e.cx = (float)K[2];
    e.cy = (float)K[3];
    e.log_a1 = (float)log(p->a1);
    e.a2 = (float)p->a2;
    e.b1 = (float)p->b1;
    e.b2 = (float)p->b2;
    e.lam2 = (float)(p->lambda * p->lambda);
    e.beta_min = (float)p->beta_min;
    e.x_floor = (float)p->x_floor;
    e.model = p->residual_model;
    e.ifx = (float)(1.0 / K[0]);
    e.ify = (float)(1.0 / K[1]);
    e.l2a1 = (float)log2(p->a1);
    e.a2l = (float)(p->a2 * 1.4426950408889634);
    return e;
}

PoseParams pose_params(const voldor_params *p)
{
    PoseParams pp;
    pp.S = p->n_pose_groups;
    pp.n_seeds = p->n_seeds;
    pp.ms_max_iters = p->ms_max_iters;
    pp.pose_start = p->pose_start;
    pp.ms_tol = p->ms_tol;
    pp.s2t = p->sigma2_trans;
    pp.s2r = p->sigma2_rot;
    pp.seed = p->seed;
    return pp;
}

template <typename T>
hipError_t dalloc(T **p, size_t n)
{
    return hipMalloc((void **)p, n * sizeof(T) + 16);
}

// phase timing: a timestamp after each phase, written on the window's stream
// by a one-thread kernel reading the GPU's constant-rate real-time counter
// (s_memrealtime); the interval ending at stamp i belongs to ev_phase[i] and,
// for the sweeps, holds ev_launches[i] launches.  Unlike HIP events these
// stamps keep working when the window is captured into a HIP graph: every
// replay rewrites them.  The sweeps of one iteration share one interval: its
// mean is the time per launch.

__global__ void k_stamp(unsigned long long *slot)
{
    if (threadIdx.x == 0) *slot = wall_clock64();
}

void mark(voldor_ctx *c, hipStream_t s, int phase, int launches = 0)
{
    if (!c->timing) return;
    // a full slot moves its last stamp forward: the whole-window time stays exact
    const int i = c->n_ev < kEvPerWin ? c->n_ev : kEvPerWin - 1;
    hipLaunchKernelGGL(k_stamp, dim3(1), dim3(64), 0, s, c->stamps + c->tw_cur * kEvPerWin + i);
    if (hipGetLastError() != hipSuccess) return;
    c->ev_phase[c->tw_cur][i] = phase;
    c->ev_launches[c->tw_cur][i] = launches;
    c->n_ev = i + 1;
}

// phases of the window in ring slot w (its stamps complete and copied to the
// host copy):
// [0] bootstrap, [1] pose steps, [2] sweeps, [3] sweep launches,
// [4] rigidness + gauge, [5] log-likelihood, [6] whole window
void slot_timing(const voldor_ctx *c, int w, double *ms8)
{
    for (int i = 0; i < 8; ++i) ms8[i] = 0.0;
    const unsigned long long *st = c->stamps_host + w * kEvPerWin;
    const int n = c->ev_n[w];
    const double ms_per_tick = 1.0 / c->stamp_khz;
    for (int i = 1; i < n; ++i) {
        const double ms = (double)(long long)(st[i] - st[i - 1]) * ms_per_tick;
        const int ph = c->ev_phase[w][i];
        if (ph >= 0 && ph < 6) ms8[ph] += ms;
        if (ph == kPhaseSweep) ms8[3] += c->ev_launches[w][i];
    }
    if (n > 1) ms8[6] = (double)(long long)(st[n - 1] - st[0]) * ms_per_tick;
}

// the stamps of every ring slot to the host copy (the stream is complete)
int fetch_stamps(voldor_ctx *c)
{
    return hipMemcpy(c->stamps_host, c->stamps, sizeof(unsigned long long) * kTimingRing * kEvPerWin,
                     hipMemcpyDeviceToHost) == hipSuccess ? VOLDOR_OK : VOLDOR_EDEVICE;
}

__global__ void k_copy_status(const int *status, int32_t *out)
{
    if (threadIdx.x == 0) *out = *status;
}

// a proposed initial state against the bootstrap's: ll[0] and ll[2] are the
// window log-likelihoods (Eq. 3 at the posterior rigidness) after each state's
// first pass of pose steps; the proposal's poses are in rel, the bootstrap
// state's in rel_a.  The proposal wins on a strictly higher likelihood: its
// depth replaces the bootstrap's; otherwise the bootstrap state's poses return.
__global__ void __launch_bounds__(256) k_init_select(const double *ll, const float *prop_depth, float *depth,
                                                     const double *rel_a, double *rel, int HW, int T,
                                                     int32_t *choice, const int *status)
{
    if (status && *status != kStatusOk) return;
    const bool use = ll[2] > ll[0];
    const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (choice && j == 0) *choice = use ? 1 : 0;
    if (!use && j < 12 * T) rel[j] = rel_a[j];
    if (use && j < HW) depth[j] = prop_depth[j];
}

__global__ void k_copy_d(const double *src, double *dst, int n, const int *status)
{
    if (status && *status != kStatusOk) return;
    for (int i = threadIdx.x; i < n; i += blockDim.x) dst[i] = src[i];
}

int upload_M(voldor_ctx *c, const double *M, int T, hipStream_t s)
{
    if (hipMemcpyAsync(c->Mcum, M, sizeof(double) * 12 * (T + 1), hipMemcpyHostToDevice, s) != hipSuccess)
        return VOLDOR_EDEVICE;
    return 0;
}

}  // namespace

extern "C" {

void voldor_params_default(voldor_params *p)
{
    if (!p) return;
    memset(p, 0, sizeof *p);
    p->struct_size = sizeof(voldor_params);
    p->n_iters = 3;
    p->sweeps_per_iter = 4;
    p->n_pose_groups = 256;
    p->n_seeds = 64;
    p->ms_max_iters = 100;
    p->lmeds_hypotheses = 512;
    p->lmeds_eval_pixels = 16384;
    p->ms_tol = 1e-5;
    p->a1 = 0.01;
    p->a2 = 0.09;
    p->b1 = -0.0022;
    p->b2 = 1.0;
    p->lambda = 0.15;
    p->gamma = 0.9;
    p->sigma2_trans = 0.1;
    p->sigma2_rot = 0.004;
    p->beta_min = 0.01;
    p->x_floor = 1e-12;
    p->depth_lo = 0.0;
    p->depth_hi = 0.0;
    p->seed = 0;
    p->criterion = VOLDOR_CRITERION_MIE;
    p->pose_start = 0;
    p->residual_model = VOLDOR_RESIDUAL_FISK;
    p->pad = 0;
}

const char *voldor_status_str(int status)
{
    switch (status) {
    case VOLDOR_OK: return "ok";
    case VOLDOR_EINVAL: return "invalid argument";
    case VOLDOR_ENOMEM: return "device allocation failed";
    case VOLDOR_EDEVICE: return "HIP runtime error";
    case VOLDOR_EDEGENERATE: return "degenerate bootstrap";
    default: return "unknown status";
    }
}

int voldor_create(voldor_ctx **out, int T_max, int H_max, int W_max, int S_max)
{
    if (!out) return VOLDOR_EINVAL;
    *out = nullptr;
    if (T_max < 1 || T_max > kTMax || H_max < 16 || W_max < 16 || H_max > 4096 || W_max > 4096 ||
        S_max < 1 || S_max > kMaxGroups)
        return VOLDOR_EINVAL;
    voldor_ctx *c = (voldor_ctx *)calloc(1, sizeof(voldor_ctx));
    if (!c) return VOLDOR_ENOMEM;
    if (hipGetDevice(&c->device) != hipSuccess) { free(c); return VOLDOR_EDEVICE; }
    int lds = 0;
    if (hipDeviceGetAttribute(&lds, hipDeviceAttributeMaxSharedMemoryPerBlock, c->device) != hipSuccess) {
        free(c);
        return VOLDOR_EDEVICE;
    }
    // static LDS of the sweep kernel (frames, list counters) comes off the top
    c->max_lds = lds - (int)(sizeof(FrameF) * (kTMax + 1)) - 256;
    c->sweep_nt[0] = c->sweep_nt[1] = 512;
    c->T_max = T_max;
    c->H_max = H_max;
    c->W_max = W_max;
    c->S_max = S_max;
    const size_t HW = (size_t)H_max * W_max;
    bool ok = true;
    ok = ok && dalloc(&c->Mcum, 12 * (T_max + 1)) == hipSuccess;
    ok = ok && dalloc(&c->range, 4) == hipSuccess;
    ok = ok && dalloc(&c->status, 8) == hipSuccess;
    ok = ok && dalloc(&c->samples, (size_t)7 * pose_sample_slots(S_max)) == hipSuccess;
    ok = ok && dalloc(&c->seed_score, (size_t)8 * (kMaxSeeds + 1)) == hipSuccess;
    ok = ok && dalloc(&c->pose_diag, 4 * T_max) == hipSuccess;
    ok = ok && dalloc(&c->hyp, (size_t)18 * kMaxHyp) == hipSuccess;
    ok = ok && dalloc(&c->hyp_score, kMaxHyp) == hipSuccess;
    ok = ok && dalloc(&c->boot_info, 4) == hipSuccess;
    ok = ok && dalloc(&c->boot_cand, 24) == hipSuccess;
    ok = ok && dalloc(&c->boot_sub, (size_t)kEvalThreads * kEvalPerThread) == hipSuccess;
    ok = ok && dalloc(&c->dkeys, HW) == hipSuccess;
    ok = ok && dalloc(&c->hist, 3 * 256) == hipSuccess;
    ok = ok && dalloc(&c->sel, 16) == hipSuccess;
    ok = ok && dalloc(&c->ll_part, 2 * kLLBlocks) == hipSuccess;
    ok = ok && dalloc(&c->init_ll, 4) == hipSuccess;
    ok = ok && dalloc(&c->init_rel, 24 * T_max) == hipSuccess;
    ok = ok && dalloc(&c->sampf, (size_t)7 * pose_sample_slots(S_max)) == hipSuccess;
    ok = ok && dalloc(&c->gcnt, S_max) == hipSuccess;
    ok = ok && dalloc(&c->gpre, S_max) == hipSuccess;
    ok = ok && dalloc(&c->bcnt, 2 * (S_max / 16 + 1)) == hipSuccess;
    ok = ok && dalloc(&c->bws, S_max / 16 + 1) == hipSuccess;
    ok = ok && dalloc(&c->seed_part, (kMaxSeeds + 1) * pose_seed_parts()) == hipSuccess;
    ok = ok && dalloc(&c->prev_pose, 12) == hipSuccess;
    ok = ok && dalloc(&c->pose_tmp, 16) == hipSuccess;
    ok = ok && dalloc(&c->rel_tmp, 12 * T_max) == hipSuccess;
    ok = ok && dalloc(&c->theta_tmp, HW) == hipSuccess;
    ok = ok && dalloc(&c->flows_t, (size_t)T_max * HW) == hipSuccess;
    const size_t ncand = 1 + pose_sample_slots(S_max);
    ok = ok && dalloc(&c->cand_F, 12 * ncand) == hipSuccess;
    ok = ok && dalloc(&c->cand_slot, ncand) == hipSuccess;
    ok = ok && dalloc(&c->cand_n, 4) == hipSuccess;
    ok = ok && dalloc(&c->cand_part, ncand * kCandTiles) == hipSuccess;
    ok = ok && dalloc(&c->cand_score, ncand) == hipSuccess;
    ok = ok && dalloc(&c->cand_start, 8) == hipSuccess;
    if (!ok) {
        voldor_destroy(c);
        return VOLDOR_ENOMEM;
    }
    if (hipMemset(c->status, 0, 8 * sizeof(int)) != hipSuccess ||
        hipMemset(c->pose_diag, 0, 4 * T_max * sizeof(int)) != hipSuccess ||
        hipDeviceSynchronize() != hipSuccess) {
        voldor_destroy(c);
        return VOLDOR_EDEVICE;
    }
    *out = c;
    return VOLDOR_OK;
}

void voldor_destroy(voldor_ctx *c)
{
    if (!c) return;
    voldor_set_timing(c, 0);
    void *bufs[] = {c->Mcum, c->range, c->status, c->samples, c->seed_score,
                    c->pose_diag, c->hyp, c->hyp_score, c->boot_info, c->boot_cand, c->boot_sub, c->dkeys, c->hist,
                    c->sel, c->ll_part, c->init_ll, c->init_rel, c->sampf, c->gcnt, c->gpre, c->bcnt, c->bws, c->seed_part, c->prev_pose, c->pose_tmp, c->rel_tmp, c->theta_tmp, c->flows_t,
                    c->cand_F, c->cand_slot, c->cand_n, c->cand_part, c->cand_score, c->cand_start};
    for (void *b : bufs)
        if (b) (void)hipFree(b);
    free(c);
}

}  // extern "C"

namespace vo {

bool window_args_ok(const voldor_ctx *c, const float *flows, int T, int H, int W, const double *K,
                    const voldor_params *p, const double *poses, const float *depth,
                    const float *rigidness)
{
    if (!c || !flows || !poses || !depth || !rigidness) return false;
    if (((uintptr_t)flows & 7) != 0) return false;
    if (!params_ok(p) || !K_ok(K) || !dims_ok(c, T, H, W, p->criterion)) return false;
    return p->n_pose_groups <= c->S_max;
}

// enqueue one window on s; host-side argument errors are returned at once,
// device-side ones end up in c->status (and in *status_out if given)
int window_enqueue(voldor_ctx *c, const float *flows, int T, int H, int W, const double *K,
                   const voldor_params *p, double *poses, float *depth, float *rigidness,
                   double *loglik, int32_t *status_out, hipStream_t s, const WindowInit *init)
{
    if (!window_args_ok(c, flows, T, H, W, K, p, poses, depth, rigidness)) return VOLDOR_EINVAL;
    const float2 *X = (const float2 *)flows;
    WinDims d = dims(T, H, W, K);
    const EmisParams e = emis(K, p);
    const PoseParams pp = pose_params(p);
    c->last_stream = s;
    c->tw_cur = (int)(c->tw_count % kTimingRing);
    c->n_ev = 0;
    mark(c, s, kPhaseNone);
    int rc = launch_transpose_flows(c, X, T, H, W, s);
    if (rc == 0)
        rc = launch_bootstrap(c, X, d, p->lmeds_hypotheses, p->lmeds_eval_pixels, p->seed, p->depth_lo,
                              p->depth_hi, poses, depth, s, init ? init->T1 : nullptr);
    mark(c, s, kPhaseBoot);
    const bool proposed = init && init->depth && init->rig;
    if (proposed && (!c->init_rel || !c->init_ll)) return VOLDOR_EDEVICE;
    if (rc == 0 && proposed) {
        // the bootstrap's state (its depth, W = 1) and the proposal's each get the
        // first pass of pose steps from the bootstrap's T_1; the window
        // log-likelihood after it picks one, poses included
        double *rel_boot = c->init_rel, *rel_a = c->init_rel + 12 * c->T_max;
        hipLaunchKernelGGL(k_copy_d, dim3(1), dim3(256), 0, s, poses, rel_boot, 12 * T, c->status);
        d.use_w = 0;
        for (int t = 1; t <= T && rc == 0; ++t)
            rc = launch_pose_step(c, depth, rigidness, X, d, e, pp, t, 0, t == 1 ? 1 : 0, poses, s);
        if (rc == 0) rc = launch_rigidness(c, depth, X, d, e, nullptr, nullptr, nullptr, nullptr, c->init_ll, s);
        if (rc == 0) {
            hipLaunchKernelGGL(k_copy_d, dim3(1), dim3(256), 0, s, poses, rel_a, 12 * T, c->status);
            hipLaunchKernelGGL(k_copy_d, dim3(1), dim3(256), 0, s, rel_boot, poses, 12 * T, c->status);
        }
        d.use_w = 1;
        for (int t = 1; t <= T && rc == 0; ++t)
            rc = launch_pose_step(c, init->depth, init->rig, X, d, e, pp, t, 0, t == 1 ? 1 : 0, poses, s);
        if (rc == 0)
            rc = launch_rigidness(c, init->depth, X, d, e, nullptr, nullptr, nullptr, nullptr, c->init_ll + 2, s);
        if (rc == 0) {
            const int n = H * W > 12 * T ? H * W : 12 * T;
            hipLaunchKernelGGL(k_init_select, dim3((n + 255) / 256), dim3(256), 0, s, c->init_ll, init->depth, depth,
                               rel_a, poses, H * W, T, init->choice, c->status);
            rc = hipGetLastError() == hipSuccess ? 0 : VOLDOR_EDEVICE;
        }
        if (rc == 0) rc = launch_cumulative(c, poses, T, s);
        mark(c, s, kPhasePose);
    }
    for (int it = 0; it < p->n_iters && rc == 0; ++it) {
        d.use_w = it > 0 ? 1 : 0;
        if (!(it == 0 && proposed)) {
            for (int t = 1; t <= T && rc == 0; ++t)
                rc = launch_pose_step(c, depth, rigidness, X, d, e, pp, t, it, (it > 0 || t == 1) ? 1 : 0, poses, s);
            mark(c, s, kPhasePose);
        }
        int swn = 0;
        for (int sw = 0; sw < p->sweeps_per_iter && rc == 0; ++sw, ++swn) {
            const int64_t gs = (int64_t)it * p->sweeps_per_iter + sw;
            rc = launch_sweep(c, depth, depth, X, d, e, (float)p->gamma, p->seed, gs, (int)(gs % 4),
                              c->range, nullptr, s, p->criterion);
        }
        mark(c, s, kPhaseSweep, swn);
        // unsmoothed W, then the scale gauge: depth rescaled in the same pass
        if (rc == 0)
            rc = launch_rigidness(c, depth, X, d, e, rigidness, nullptr, nullptr, nullptr, nullptr, s, depth, poses);
        if (rc == 0) rc = launch_gauge_poses(c, poses, d, s);
        mark(c, s, kPhaseRig);
    }
    if (rc == 0 && loglik) {
        rc = launch_rigidness(c, depth, X, d, e, nullptr, nullptr, nullptr, nullptr, loglik, s);
        mark(c, s, kPhaseLL);
    }
    if (rc == 0 && status_out) {
        hipLaunchKernelGGL(k_copy_status, dim3(1), dim3(64), 0, s, c->status, status_out);
        if (hipGetLastError() != hipSuccess) rc = VOLDOR_EDEVICE;
    }
    if (c->timing) {
        c->ev_n[c->tw_cur] = c->n_ev;
        ++c->tw_count;
    }
    return rc;
}

// Lockstep lane: the window_enqueue sequence of several windows at once.  The
// bootstraps run one after another; then per iteration one pose step per
// frame index over the windows that have that frame, the sweeps over all
// chains of all windows, the rigidness pass with the gauge; finally the
// log-likelihood.  Each window sees the launches, arguments and order of its
// own window_enqueue, so its results are the same bit for bit.
void lockstep_plan(voldor_ctx *const *wc, const voldor_window_desc *w, const std::vector<int> &idx,
                   const voldor_params *p, Plan &plan, std::vector<WinRef> &refs, std::vector<LockStep> &steps)
{
    const int n = (int)idx.size();
    refs.resize(n);
    int Tmax = 0;
    for (int k = 0; k < n; ++k) {
        const voldor_window_desc &d = w[idx[k]];
        voldor_params pw = *p;
        if (d.n_pose_groups > 0) pw.n_pose_groups = d.n_pose_groups;
        WinRef &r = refs[k];
        r.c = wc[k];
        r.X = (const float2 *)d.flows;
        r.d = dims(d.T, d.H, d.W, d.K);
        r.e = emis(d.K, &pw);
        r.pp = pose_params(&pw);
        r.depth = d.depth;
        r.rig = d.rigidness;
        r.poses = d.poses;
        Tmax = d.T > Tmax ? d.T : Tmax;
    }
    auto stamp = [&](int phase, int launches) {
        LockStep st = {};
        st.kind = kStepStamp;
        st.phase = phase;
        st.launches = launches;
        steps.push_back(st);
    };
    auto multi = [&](const std::vector<MultiLaunch> &ms) {
        for (const MultiLaunch &m : ms) {
            LockStep st = {};
            st.kind = kStepMulti;
            st.m = m;
            steps.push_back(st);
        }
    };
    std::vector<int> all(n);
    for (int k = 0; k < n; ++k) all[k] = k;
    for (int k = 0; k < n; ++k) {
        LockStep st = {};
        st.kind = kStepTranspose;
        st.win = k;
        steps.push_back(st);
    }
    std::vector<MultiLaunch> ms;
    plan_bootstrap(plan, ms, refs, all, p->lmeds_hypotheses, p->lmeds_eval_pixels, p->seed, p->depth_lo,
                   p->depth_hi);
    multi(ms);
    stamp(kPhaseBoot, 0);
    for (int it = 0; it < p->n_iters; ++it) {
        for (int t = 1; t <= Tmax; ++t) {
            std::vector<int> act;
            for (int k = 0; k < n; ++k)
                if (refs[k].d.T >= t) act.push_back(k);
            ms.clear();
            plan_pose_step(plan, ms, refs, act, t, it);
            multi(ms);
        }
        stamp(kPhasePose, 0);
        for (int sw = 0; sw < p->sweeps_per_iter; ++sw) {
            const int64_t gs = (int64_t)it * p->sweeps_per_iter + sw;
            ms.clear();
            plan_sweep(plan, ms, refs, all, (float)p->gamma, p->seed, gs, (int)(gs % 4), p->criterion);
            multi(ms);
        }
        stamp(kPhaseSweep, p->sweeps_per_iter * n);
        ms.clear();
        plan_rigidness(plan, ms, refs, all, true, std::vector<double *>());
        plan_gauge_poses(plan, ms, refs, all);
        multi(ms);
        stamp(kPhaseRig, 0);
    }
    std::vector<int> with_ll;
    std::vector<double *> ll;
    for (int k = 0; k < n; ++k)
        if (w[idx[k]].loglik) {
            with_ll.push_back(k);
            ll.push_back(w[idx[k]].loglik);
        }
    if (!with_ll.empty()) {
        ms.clear();
        plan_rigidness(plan, ms, refs, with_ll, false, ll);
        multi(ms);
        stamp(kPhaseLL, 0);
    }
    for (int k = 0; k < n; ++k) {
        LockStep st = {};
        st.kind = kStepStatus;
        st.win = k;
        steps.push_back(st);
    }
}

int lockstep_run(voldor_ctx *lane, const std::vector<WinRef> &refs, const std::vector<LockStep> &steps,
                 const voldor_window_desc *w, const std::vector<int> &idx, const voldor_params *p,
                 const unsigned char *plan_dev, int32_t *status_out, hipStream_t s)
{
    lane->last_stream = s;
    lane->tw_cur = (int)(lane->tw_count % kTimingRing);
    lane->n_ev = 0;
    mark(lane, s, kPhaseNone);
    int rc = 0;
    for (const LockStep &st : steps) {
        if (rc) break;
        switch (st.kind) {
        case kStepBoot: {
            const WinRef &r = refs[st.win];
            r.c->last_stream = s;
            rc = launch_transpose_flows(r.c, r.X, r.d.T, r.d.H, r.d.W, s);
            if (rc == 0)
                rc = launch_bootstrap(r.c, r.X, r.d, p->lmeds_hypotheses, p->lmeds_eval_pixels, p->seed,
                                      p->depth_lo, p->depth_hi, r.poses, r.depth, s, nullptr);
            break;
        }
        case kStepTranspose: {
            const WinRef &r = refs[st.win];
            r.c->last_stream = s;
            rc = launch_transpose_flows(r.c, r.X, r.d.T, r.d.H, r.d.W, s);
            break;
        }
        case kStepMulti:
            if (st.m.kind == kMultiSweep || st.m.kind == kMultiRig || st.m.kind == kMultiLL)
                rc = launch_sweep_multi(st.m, plan_dev, s);
            else if (st.m.kind >= kMultiBootInit)
                rc = launch_boot_multi(st.m, plan_dev, s);
            else
                rc = launch_pose_multi(st.m, plan_dev, s);
            break;
        case kStepStamp:
            mark(lane, s, st.phase, st.launches);
            break;
        case kStepStatus:
            hipLaunchKernelGGL(k_copy_status, dim3(1), dim3(64), 0, s, refs[st.win].c->status,
                               status_out + idx[st.win]);
            rc = hipGetLastError() == hipSuccess ? 0 : VOLDOR_EDEVICE;
            break;
        default:
            rc = VOLDOR_EINVAL;
        }
    }
    (void)w;
    if (lane->timing) {
        lane->ev_n[lane->tw_cur] = lane->n_ev;
        ++lane->tw_count;
    }
    return rc;
}

}  // namespace vo

extern "C" {

int voldor_window(voldor_ctx *c, const float *flows, int T, int H, int W, const double *K,
                  const voldor_params *p, double *poses, float *depth, float *rigidness,
                  double *loglik, void *stream)
{
    hipStream_t s = (hipStream_t)stream;
    const int rc = window_enqueue(c, flows, T, H, W, K, p, poses, depth, rigidness, loglik, nullptr, s);
    if (rc != 0) return rc;
    if (hipStreamSynchronize(s) != hipSuccess) return VOLDOR_EDEVICE;
    if (c->timing && fetch_stamps(c) == VOLDOR_OK) slot_timing(c, c->tw_cur, c->last_ms);
    int st = 0;
    if (hipMemcpy(&st, c->status, sizeof(int), hipMemcpyDeviceToHost) != hipSuccess) return VOLDOR_EDEVICE;
    return st;
}

int voldor_window_async(voldor_ctx *c, const float *flows, int T, int H, int W, const double *K,
                        const voldor_params *p, double *poses, float *depth, float *rigidness,
                        double *loglik, int32_t *status_out, void *stream)
{
    if (!status_out || ((uintptr_t)status_out & 3) != 0) return VOLDOR_EINVAL;
    return window_enqueue(c, flows, T, H, W, K, p, poses, depth, rigidness, loglik, status_out,
                          (hipStream_t)stream);
}

int voldor_window_init(voldor_ctx *c, const float *flows, int T, int H, int W, const double *K,
                       const voldor_params *p, const float *init_depth, const float *init_rig, double *poses,
                       float *depth, float *rigidness, double *loglik, int32_t *status_out, int32_t *choice_out,
                       void *stream)
{
    if (!status_out || ((uintptr_t)status_out & 3) != 0 || !init_depth || !init_rig) return VOLDOR_EINVAL;
    if (choice_out && ((uintptr_t)choice_out & 3) != 0) return VOLDOR_EINVAL;
    const WindowInit in = {init_depth, init_rig, choice_out, nullptr};
    return window_enqueue(c, flows, T, H, W, K, p, poses, depth, rigidness, loglik, status_out,
                          (hipStream_t)stream, &in);
}

int voldor_window_seeded(voldor_ctx *c, const float *flows, int T, int H, int W, const double *K,
                         const voldor_params *p, const double *T1, double *poses, float *depth, float *rigidness,
                         double *loglik, int32_t *status_out, void *stream)
{
    if (!T1 || ((uintptr_t)T1 & 7) != 0) return VOLDOR_EINVAL;
    if (!status_out || ((uintptr_t)status_out & 3) != 0) return VOLDOR_EINVAL;
    const WindowInit in = {nullptr, nullptr, nullptr, T1};
    return window_enqueue(c, flows, T, H, W, K, p, poses, depth, rigidness, loglik, status_out,
                          (hipStream_t)stream, &in);
}

// first frames of the windows of a sequence of N flows: 0, stride, ..., and a
// last one ending at flow N
static int vo_starts(int N, int T, int stride, int *out, int cap)
{
    int n = 0, s = 0;
    if (cap > 0) out[0] = 0;
    n = 1;
    while (s + T < N) {
        s = s + stride < N - T ? s + stride : N - T;
        if (n < cap) out[n] = s;
        ++n;
    }
    return n;
}

int voldor_vo_windows(int N, int T, int stride)
{
    if (T < 2 || T > 16 || N < T || stride < 1 || stride >= T) return VOLDOR_EINVAL;
    return vo_starts(N, T, stride, nullptr, 0);
}

// one thread: the trajectory of the sequence from the windows' relative poses
// (every window in its own gauge |t_1| = 1).  Window i's scale relative to
// window i - 1 is the length, in window i - 1's units, of the frame pair that
// seeded window i's T_1; the pose of frame pair (k, k + 1) comes from the
// latest window starting at or before k.  Any failed window: all NaN.
__global__ void k_vo_chain(const double *wposes, const int32_t *wstatus, int nwin, int N, int T, int stride,
                           double *traj)
{
    if (threadIdx.x != 0) return;
    bool ok = true;
    for (int i = 0; i < nwin; ++i) ok = ok && wstatus[i] == kStatusOk;
    if (!ok) {
        for (int k = 0; k < 12 * (N + 1); ++k) traj[k] = __longlong_as_double(0x7ff8000000000000ll);
        return;
    }
    for (int k = 0; k < 12; ++k) traj[k] = (k == 0 || k == 4 || k == 8) ? 1.0 : 0.0;
    int i = 0, s_i = 0, s_next = T < N ? (stride < N - T ? stride : N - T) : N;
    double scale = 1.0;
    for (int k = 0; k < N; ++k) {
        while (i + 1 < nwin && s_next <= k) {
            // window i + 1 starts at s_next: its T_1 is window i's pair s_next
            const double *tp = wposes + (size_t)12 * ((size_t)i * T + (s_next - s_i)) + 9;
            scale *= sqrt(tp[0] * tp[0] + tp[1] * tp[1] + tp[2] * tp[2]);
            ++i;
            s_i = s_next;
            s_next = s_i + stride < N - T ? s_i + stride : N - T;
        }
        const double *r = wposes + (size_t)12 * ((size_t)i * T + (k - s_i));
        double step[12];
        for (int q = 0; q < 9; ++q) step[q] = r[q];
        for (int q = 0; q < 3; ++q) step[9 + q] = r[9 + q] * scale;
        pose_mul(step, traj + 12 * k, traj + 12 * (k + 1));
    }
}

int voldor_vo_sequence(voldor_ctx *c, const float *flows, int N, int H, int W, const double *K,
                       const voldor_params *p, int T, int stride, double *wposes, float *depth, float *rigidness,
                       int32_t *wstatus, double *traj, void *stream)
{
    const int nwin = voldor_vo_windows(N, T, stride);
    if (nwin < 1 || !flows || !wposes || !depth || !rigidness || !wstatus || !traj) return VOLDOR_EINVAL;
    if (((uintptr_t)wstatus & 3) != 0 || ((uintptr_t)wposes & 7) != 0 || ((uintptr_t)traj & 7) != 0)
        return VOLDOR_EINVAL;
    if (!window_args_ok(c, flows, T, H, W, K, p, wposes, depth, rigidness)) return VOLDOR_EINVAL;
    hipStream_t s = (hipStream_t)stream;
    int starts[4096];
    if (nwin > 4096) return VOLDOR_EINVAL;
    vo_starts(N, T, stride, starts, nwin);
    const size_t fstride = (size_t)H * W * 2;
    for (int i = 0; i < nwin; ++i) {
        const WindowInit in = {nullptr, nullptr, nullptr,
                               i == 0 ? nullptr : wposes + (size_t)12 * ((size_t)(i - 1) * T + (starts[i] - starts[i - 1]))};
        const int rc = window_enqueue(c, flows + fstride * starts[i], T, H, W, K, p, wposes + (size_t)12 * T * i,
                                      depth, rigidness, nullptr, wstatus + i, s, i == 0 ? nullptr : &in);
        if (rc) return rc;
    }
    hipLaunchKernelGGL(k_vo_chain, dim3(1), dim3(64), 0, s, wposes, wstatus, nwin, N, T, stride, traj);
    return hipGetLastError() == hipSuccess ? VOLDOR_OK : VOLDOR_EDEVICE;
}

int voldor_set_sweep_threads(voldor_ctx *c, int rows, int cols)
{
    if (!c) return VOLDOR_EINVAL;
    const int v[2] = {rows ? rows : 512, cols ? cols : 512};
    for (int a = 0; a < 2; ++a)
        if (v[a] != 256 && v[a] != 512 && v[a] != 768 && v[a] != 1024) return VOLDOR_EINVAL;
    c->sweep_nt[0] = v[0];
    c->sweep_nt[1] = v[1];
    c->n_sweep_tab = 0;   // an explicit setting replaces the tuned ones
    return VOLDOR_OK;
}

int voldor_get_sweep_threads(const voldor_ctx *c, int *rows, int *cols)
{
    if (!c || !rows || !cols) return VOLDOR_EINVAL;
    *rows = c->sweep_nt[0];
    *cols = c->sweep_nt[1];
    return VOLDOR_OK;
}

int voldor_set_sweep_lookahead(voldor_ctx *c, int rows, int cols)
{
    if (!c || rows < 0 || cols < 0 || rows > 4096 || cols > 4096) return VOLDOR_EINVAL;
    c->sweep_la[0] = rows;
    c->sweep_la[1] = cols;
    c->n_sweep_tab = 0;   // an explicit setting replaces the tuned ones
    return VOLDOR_OK;
}

int voldor_get_sweep_lookahead(const voldor_ctx *c, int *rows, int *cols)
{
    if (!c || !rows || !cols) return VOLDOR_EINVAL;
    *rows = c->sweep_la[0];
    *cols = c->sweep_la[1];
    return VOLDOR_OK;
}

// Times the sweeps of this window's shape at every setting of the two tuning
// axes, threads per chain (256, 512, 768, 1024 where the chain fits the LDS) and
// look-ahead cap of the propagation rounds (none, 32, 16, 8, 4, 2), row and column
// sweeps apart, from the state the window ends in, and keeps the fastest of
// each axis for this chain class (length, frames, criterion) in the context.
// No setting changes the result.
int voldor_autotune(voldor_ctx *c, const float *flows, int T, int H, int W, const double *K,
                    const voldor_params *p, int *rows_out, int *cols_out, void *stream)
{
    if (!c || !flows || ((uintptr_t)flows & 7) != 0) return VOLDOR_EINVAL;
    if (!params_ok(p) || !K_ok(K) || T < 1 || T > c->T_max || H < 16 || W < 16 || H > c->H_max || W > c->W_max)
        return VOLDOR_EINVAL;
    hipStream_t s = (hipStream_t)stream;
    const float2 *X = (const float2 *)flows;
    WinDims d = dims(T, H, W, K);
    const EmisParams e = emis(K, p);
    // the state the timed sweeps start from: the window solved once with the
    // current settings (its later iterations, three in four, are where the
    // sweeps spend their time; from the bootstrap's noisier depth the
    // propagation runs are shorter and favour small look-aheads)
    float *rig_tmp = nullptr;
    if (hipMalloc((void **)&rig_tmp, sizeof(float) * (size_t)T * H * W) != hipSuccess) return VOLDOR_ENOMEM;
    int rc = window_enqueue(c, flows, T, H, W, K, p, c->rel_tmp, c->theta_tmp, rig_tmp, nullptr, nullptr, s);
    int st = 0;
    // the end state is kept (in the rigidness buffer, no longer needed) and
    // every setting is timed from it: timed sweeps move the depth on, and
    // settings timed later would otherwise start from later states
    float *theta_keep = rig_tmp;
    const size_t HW = (size_t)H * W;
    if (rc == 0 && (hipStreamSynchronize(s) != hipSuccess ||
                    hipMemcpy(&st, c->status, sizeof st, hipMemcpyDeviceToHost) != hipSuccess ||
                    hipMemcpy(theta_keep, c->theta_tmp, HW * sizeof(float), hipMemcpyDeviceToDevice) != hipSuccess))
        rc = VOLDOR_EDEVICE;
    if (rc == 0 && st != kStatusOk) rc = st;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    if (rc == 0 && hipEventCreate(&e0) != hipSuccess) rc = VOLDOR_EDEVICE;
    if (rc == 0 && hipEventCreate(&e1) != hipSuccess) rc = VOLDOR_EDEVICE;
    if (rc) {
        if (e0) (void)hipEventDestroy(e0);
        (void)hipFree(rig_tmp);
        return rc;
    }
    const int widths[4] = {256, 512, 768, 1024};
    const int caps[6] = {0, 32, 16, 8, 4, 2};
    // the defaults are the fallback while timing: clear any tuned entry of
    // these classes by timing through a temporary default instead
    const int keep_nt[2] = {c->sweep_nt[0], c->sweep_nt[1]}, keep_la[2] = {c->sweep_la[0], c->sweep_la[1]};
    const int keep_n = c->n_sweep_tab;
    SweepCfg keep_tab[kSweepTab];
    for (int i = 0; i < keep_n; ++i) keep_tab[i] = c->sweep_tab[i];
    c->n_sweep_tab = 0;
    int best_nt[2] = {512, 512}, best_la[2] = {0, 0};
    for (int axis = 0; axis < 2 && rc == 0; ++axis) {
        const int L = axis ? H : W;
        float best_ms = 1e30f;
        for (int wi = 0; wi < 4 && rc == 0; ++wi) {
            const int nt = widths[wi];
            if ((int)sweep_lds_bytes(T, L, p->criterion, nt) > c->max_lds) continue;
            for (int ci = 0; ci < 6 && rc == 0; ++ci) {
                c->sweep_nt[axis] = nt;
                c->sweep_la[axis] = caps[ci];
                if (hipMemcpyAsync(c->theta_tmp, theta_keep, HW * sizeof(float), hipMemcpyDeviceToDevice, s) !=
                    hipSuccess)
                    rc = VOLDOR_EDEVICE;
                float ms = 0.0f;
                for (int rep = 0; rep < 5 && rc == 0; ++rep) {   // the first sweep warms up
                    if (rep == 1 && hipEventRecord(e0, s) != hipSuccess) rc = VOLDOR_EDEVICE;
                    const int64_t gs = (int64_t)p->n_iters * p->sweeps_per_iter + rep;
                    if (rc == 0)
                        rc = launch_sweep(c, c->theta_tmp, c->theta_tmp, X, d, e, (float)p->gamma, p->seed, gs,
                                          axis + 2 * (rep & 1), c->range, nullptr, s, p->criterion);
                }
                if (rc == 0 && (hipEventRecord(e1, s) != hipSuccess || hipEventSynchronize(e1) != hipSuccess ||
                                hipEventElapsedTime(&ms, e0, e1) != hipSuccess))
                    rc = VOLDOR_EDEVICE;
                if (rc == 0 && ms < best_ms) {
                    best_ms = ms;
                    best_nt[axis] = nt;
                    best_la[axis] = caps[ci];
                }
            }
        }
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (hipStreamSynchronize(s) != hipSuccess && rc == 0) rc = VOLDOR_EDEVICE;
    (void)hipFree(rig_tmp);
    c->sweep_nt[0] = keep_nt[0];
    c->sweep_nt[1] = keep_nt[1];
    c->sweep_la[0] = keep_la[0];
    c->sweep_la[1] = keep_la[1];
    for (int i = 0; i < keep_n; ++i) c->sweep_tab[i] = keep_tab[i];
    c->n_sweep_tab = keep_n;
    if (rc == 0) {
        sweep_cfg_store(c, W, T, p->criterion, best_nt[0], best_la[0]);
        sweep_cfg_store(c, H, T, p->criterion, best_nt[1], best_la[1]);
    }
    int r = 512, la = 0, cc = 512;
    sweep_cfg_for(c, 0, W, T, p->criterion, &r, &la);
    sweep_cfg_for(c, 1, H, T, p->criterion, &cc, &la);
    if (rows_out) *rows_out = r;
    if (cols_out) *cols_out = cc;
    return rc;
}

// The tuned settings of this context's chain classes: out[4 i + 0..3] = (chain
// length, frames, threads, look-ahead cap) of entry i (criterion MIE and MLE
// entries alike); returns the number of entries (at most max_n).
int voldor_sweep_tuning(const voldor_ctx *c, int *out, int max_n)
{
    if (!c || (!out && max_n > 0) || max_n < 0) return VOLDOR_EINVAL;
    const int n = c->n_sweep_tab < max_n ? c->n_sweep_tab : max_n;
    for (int i = 0; i < n; ++i) {
        out[4 * i] = c->sweep_tab[i].L;
        out[4 * i + 1] = c->sweep_tab[i].T;
        out[4 * i + 2] = c->sweep_tab[i].nt;
        out[4 * i + 3] = c->sweep_tab[i].la;
    }
    return n;
}

int voldor_set_timing(voldor_ctx *c, int enable)
{
    if (!c) return VOLDOR_EINVAL;
    if (enable && !c->timing) {
        int khz = 0;
        if (hipDeviceGetAttribute(&khz, hipDeviceAttributeWallClockRate, c->device) != hipSuccess || khz <= 0)
            return VOLDOR_EDEVICE;
        c->stamp_khz = (double)khz;
        c->stamps_host = (unsigned long long *)calloc((size_t)kTimingRing * kEvPerWin, sizeof(unsigned long long));
        if (!c->stamps_host) return VOLDOR_ENOMEM;
        if (hipMalloc((void **)&c->stamps, sizeof(unsigned long long) * kTimingRing * kEvPerWin) != hipSuccess) {
            free(c->stamps_host);
            c->stamps_host = nullptr;
            return VOLDOR_ENOMEM;
        }
        for (int w = 0; w < kTimingRing; ++w) c->ev_n[w] = 0;
        c->tw_count = 0;
        c->timing = 1;
    } else if (!enable && c->timing) {
        (void)hipDeviceSynchronize();
        (void)hipFree(c->stamps);
        free(c->stamps_host);
        c->stamps = nullptr;
        c->stamps_host = nullptr;
        c->timing = 0;
    }
    return VOLDOR_OK;
}

int voldor_last_timing(voldor_ctx *c, double *out)
{
    if (!c || !out) return VOLDOR_EINVAL;
    for (int i = 0; i < 8; ++i) out[i] = c->last_ms[i];
    return VOLDOR_OK;
}

int voldor_timing_summary(voldor_ctx *c, double *out, int *n_windows)
{
    if (!c || !out) return VOLDOR_EINVAL;
    for (int i = 0; i < 8; ++i) out[i] = 0.0;
    if (n_windows) *n_windows = 0;
    if (!c->timing) return VOLDOR_EINVAL;
    if (c->tw_count == 0) return VOLDOR_OK;
    if (hipStreamSynchronize(c->last_stream) != hipSuccess) return VOLDOR_EDEVICE;
    if (fetch_stamps(c) != VOLDOR_OK) return VOLDOR_EDEVICE;
    const long long n = c->tw_count < kTimingRing ? c->tw_count : kTimingRing;
    for (long long k = c->tw_count - n; k < c->tw_count; ++k) {
        double ms8[8];
        slot_timing(c, (int)(k % kTimingRing), ms8);
        for (int i = 0; i < 8; ++i) out[i] += ms8[i] / (double)n;
    }
    slot_timing(c, (int)((c->tw_count - 1) % kTimingRing), c->last_ms);
    if (n_windows) *n_windows = (int)n;
    c->tw_count = 0;
    return VOLDOR_OK;
}

int voldor_philox(const uint64_t *ctr, uint64_t key0, uint64_t key1, uint64_t *out, int n, void *stream)
{
    if (!ctr || !out || n < 0) return VOLDOR_EINVAL;
    const int rc = launch_philox(ctr, key0, key1, out, n, (hipStream_t)stream);
    if (rc) return rc;
    return hipStreamSynchronize((hipStream_t)stream) == hipSuccess ? VOLDOR_OK : VOLDOR_EDEVICE;
}

int voldor_emission(voldor_ctx *c, const float *theta, const float *flows, int T, int H, int W,
                    const double *K, const voldor_params *p, const double *M, float *r, float *ell,
                    float *logrho, float *logmu, void *stream)
{
    if (!c || !theta || !flows || !M) return VOLDOR_EINVAL;
    if (!params_ok(p) || !K_ok(K) || !dims_ok(c, T, H, W, p->criterion)) return VOLDOR_EINVAL;
    hipStream_t s = (hipStream_t)stream;
    hipLaunchKernelGGL(k_reset_status, dim3(1), dim3(64), 0, s, c->status);
    int rc = upload_M(c, M, T, s);
    if (rc == 0)
        rc = launch_rigidness(c, theta, (const float2 *)flows, dims(T, H, W, K), emis(K, p), r, ell,
                              logrho, logmu, nullptr, s);
    if (rc) return rc;
    return hipStreamSynchronize(s) == hipSuccess ? VOLDOR_OK : VOLDOR_EDEVICE;
}

int voldor_sweep(voldor_ctx *c, const float *theta_in, float *theta_out, const float *flows, int T,
                 int H, int W, const double *K, const voldor_params *p, const double *M, double d_lo,
                 double d_hi, int64_t global_sweep, int dir, float *q_out, void *stream)
{
    if (!c || !theta_in || !theta_out || !flows || !M) return VOLDOR_EINVAL;
    if (!params_ok(p) || !K_ok(K) || !dims_ok(c, T, H, W, p->criterion)) return VOLDOR_EINVAL;
    if (dir < 0 || dir > 3 || !(d_lo > 0) || !(d_hi > d_lo) || global_sweep < 0) return VOLDOR_EINVAL;
    hipStream_t s = (hipStream_t)stream;
    double rng[4] = {d_lo, d_hi, 1.0, 0.0};
    hipLaunchKernelGGL(k_reset_status, dim3(1), dim3(64), 0, s, c->status);
    if (hipMemcpyAsync(c->range, rng, sizeof rng, hipMemcpyHostToDevice, s) != hipSuccess) return VOLDOR_EDEVICE;
    int rc = upload_M(c, M, T, s);
    if (rc == 0) rc = launch_transpose_flows(c, (const float2 *)flows, T, H, W, s);
    if (rc == 0)
        rc = launch_sweep(c, theta_in, theta_out, (const float2 *)flows, dims(T, H, W, K), emis(K, p),
                          (float)p->gamma, p->seed, global_sweep, dir, c->range, q_out, s, p->criterion);
    if (rc) return rc;
    return hipStreamSynchronize(s) == hipSuccess ? VOLDOR_OK : VOLDOR_EDEVICE;
}

int voldor_last_range(voldor_ctx *c, double *range2)
{
    if (!c || !range2) return VOLDOR_EINVAL;
    if (hipDeviceSynchronize() != hipSuccess) return VOLDOR_EDEVICE;
    return hipMemcpy(range2, c->range, sizeof(double) * 2, hipMemcpyDeviceToHost) == hipSuccess ? VOLDOR_OK
                                                                                                 : VOLDOR_EDEVICE;
}

int voldor_pose_scores(voldor_ctx *c, double *scores, int max_n, int *n_out)
{
    if (!c || !scores || !n_out || max_n < 1) return VOLDOR_EINVAL;
    int n = 0;
    if (hipDeviceSynchronize() != hipSuccess) return VOLDOR_EDEVICE;
    if (hipMemcpy(&n, c->cand_n, sizeof n, hipMemcpyDeviceToHost) != hipSuccess) return VOLDOR_EDEVICE;
    if (n < 1 || n > max_n) return VOLDOR_EINVAL;
    if (hipMemcpy(scores, c->cand_score, sizeof(double) * n, hipMemcpyDeviceToHost) != hipSuccess)
        return VOLDOR_EDEVICE;
    *n_out = n;
    return VOLDOR_OK;
}

int voldor_pose_step(voldor_ctx *c, const float *theta, const float *rig, const float *flows, int T,
                     int H, int W, const double *K, const voldor_params *p, const double *M, int t,
                     int it, const double *prevT, double *T_out, double *samples, int *diag,
                     void *stream)
{
    if (!c || !theta || !flows || !M || !T_out) return VOLDOR_EINVAL;
    if (!params_ok(p) || !K_ok(K) || !dims_ok(c, T, H, W, p->criterion)) return VOLDOR_EINVAL;
    if (t < 1 || t > T || it < 0 || p->n_pose_groups > c->S_max) return VOLDOR_EINVAL;
    hipStream_t s = (hipStream_t)stream;
    hipLaunchKernelGGL(k_reset_status, dim3(1), dim3(64), 0, s, c->status);
    if (hipMemcpyAsync(c->Mcum, M, sizeof(double) * 12 * (T + 1), hipMemcpyHostToDevice, s) != hipSuccess)
        return VOLDOR_EDEVICE;
    // previous estimate of T_t (or identity as the fallback of the frame before)
    double ident[12] = {1, 0, 0, 0, 1, 0, 0, 0, 1, 0, 0, 0};
    const double *pv = prevT ? prevT : ident;
    if (hipMemcpyAsync(c->rel_tmp + 12 * (t - 1), pv, sizeof ident, hipMemcpyHostToDevice, s) != hipSuccess)
        return VOLDOR_EDEVICE;
    if (t >= 2 && hipMemcpyAsync(c->rel_tmp + 12 * (t - 2), ident, sizeof ident, hipMemcpyHostToDevice, s) != hipSuccess)
        return VOLDOR_EDEVICE;
    WinDims d = dims(T, H, W, K);
    d.use_w = rig ? 1 : 0;
    int rc = launch_pose_step(c, theta, rig, (const float2 *)flows, d, emis(K, p), pose_params(p), t, it,
                              prevT ? 1 : 0, c->rel_tmp, s);
    if (rc) return rc;
    if (samples && launch_samples_aos(c, p->n_pose_groups, samples, s) != 0) return VOLDOR_EDEVICE;
    if (hipStreamSynchronize(s) != hipSuccess) return VOLDOR_EDEVICE;
    if (hipMemcpy(T_out, c->rel_tmp + 12 * (t - 1), sizeof(double) * 12, hipMemcpyDeviceToHost) != hipSuccess)
        return VOLDOR_EDEVICE;
    if (diag && hipMemcpy(diag, c->pose_diag + 4 * (t - 1), sizeof(int) * 4, hipMemcpyDeviceToHost) != hipSuccess)
        return VOLDOR_EDEVICE;
    return VOLDOR_OK;
}

int voldor_bootstrap(voldor_ctx *c, const float *flows, int T, int H, int W, const double *K,
                     const voldor_params *p, double *relT, float *theta, double *range, double *info,
                     void *stream)
{
    if (!c || !flows || !relT || !theta || !range) return VOLDOR_EINVAL;
    if (!params_ok(p) || !K_ok(K) || !dims_ok(c, T, H, W, p->criterion)) return VOLDOR_EINVAL;
    hipStream_t s = (hipStream_t)stream;
    int rc = launch_bootstrap(c, (const float2 *)flows, dims(T, H, W, K), p->lmeds_hypotheses,
                              p->lmeds_eval_pixels, p->seed, p->depth_lo, p->depth_hi, c->rel_tmp, theta, s);
    if (rc) return rc;
    if (hipStreamSynchronize(s) != hipSuccess) return VOLDOR_EDEVICE;
    int st = 0;
    if (hipMemcpy(&st, c->status, sizeof(int), hipMemcpyDeviceToHost) != hipSuccess) return VOLDOR_EDEVICE;
    if (st != VOLDOR_OK) return st;
    if (hipMemcpy(relT, c->rel_tmp, sizeof(double) * 12, hipMemcpyDeviceToHost) != hipSuccess ||
        hipMemcpy(range, c->range, sizeof(double) * 2, hipMemcpyDeviceToHost) != hipSuccess)
        return VOLDOR_EDEVICE;
    if (info && hipMemcpy(info, c->boot_info, sizeof(double) * 4, hipMemcpyDeviceToHost) != hipSuccess)
        return VOLDOR_EDEVICE;
    return VOLDOR_OK;
}

}  // extern "C"
