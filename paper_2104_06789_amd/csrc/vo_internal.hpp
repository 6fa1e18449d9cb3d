// vo_internal.hpp -- context layout and kernel launchers shared by the
// translation units of the gfx950 library (not part of the public ABI).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>
#include <string.h>

#include <vector>

#include "voldor.h"
#include "vo_device.hpp"

namespace vo {

constexpr int kMaxSeeds = 255;      // mean-shift start candidates drawn from samples
constexpr int kMaxHyp = 4096;       // bootstrap hypotheses
constexpr int kEvalThreads = 512;   // threads of the bootstrap scoring kernel
constexpr int kEvalPerThread = 32;  // residuals held per thread (16384 max)
constexpr int kMaxGroups = 8192;    // P3P groups per frame
constexpr int kLLBlocks = 1024;     // partial sums of the log-likelihood
constexpr int kCandTiles = 256;     // pixel ranges of the all-pixel candidate scores

// Device status word values (mirror voldor_status).
enum : int { kStatusOk = 0, kStatusDegenerate = -4 };
// phase of a timing interval (the interval that ends at a stamp)
enum : int { kPhaseNone = -1, kPhaseBoot = 0, kPhasePose = 1, kPhaseSweep = 2, kPhaseRig = 4, kPhaseLL = 5 };
constexpr int kTimingRing = 32;   // windows whose phase events are kept
constexpr int kEvPerWin = 128;    // events per window, at most

// Tuned launch settings of the sweeps for one chain class (chain length,
// frames, depth criterion): threads per chain and look-ahead cap.
struct SweepCfg {
    int L, T, crit, nt, la;
};
constexpr int kSweepTab = 16;

// Window-level device parameters shared by all kernels of one call.
struct WinDims {
    int T, H, W;
    int use_w;          // pose weights from the rigidness buffer (else all 1)
    double fx, fy, cx, cy;
};

struct PoseParams {
    int S, n_seeds, ms_max_iters, pose_start;
    double ms_tol, s2t, s2r;
    uint64_t seed;
};

}  // namespace vo

struct voldor_ctx {
    int device;
    int T_max, H_max, W_max, S_max;
    int max_lds;           // bytes of LDS one workgroup may allocate
    int sweep_nt[2];       // threads per chain of row (directions 0/2) and column (1/3) sweeps
    int sweep_la[2];       // look-ahead cap of the propagation rounds (0: none), rows and columns
    // autotuned settings per chain class (override the two defaults above)
    vo::SweepCfg sweep_tab[vo::kSweepTab];
    int n_sweep_tab;
    // persistent device state
    double *Mcum;          // [(T_max+1)][12] cumulative poses M_0..M_T
    double *range;         // [4]: d_lo, d_hi, gauge scale, spare
    int *status;           // [8]: status word, pose diagnostics scratch
    double *samples;       // SoA [7][slots] pose samples (p, weight), compacted per block of groups
    double *seed_score;    // [kMaxSeeds + 1][8] (p, unused, valid)
    int *pose_diag;        // [T_max][4]
    double *hyp;           // [kMaxHyp][18]: essential E (9), fundamental F (9)
    double *hyp_score;     // [kMaxHyp] median Sampson residual
    double *boot_info;     // [4]
    double *boot_cand;     // [24] rotations and translation of the best essential matrix
    float4 *boot_sub;      // [kEvalThreads kEvalPerThread] pixel subset of the median (x, y, flow)
    uint32_t *dkeys;       // [H_max W_max] order-preserving keys of triangulated depths
    uint32_t *hist;        // [3][256] radix histograms
    uint32_t *sel;         // [16] radix-select state (prefix, rank) x 3, valid count
    double *ll_part;       // [kLLBlocks][2] log-likelihood partial sums
    double *init_ll;       // [4] window log-likelihoods (and L1 masses) of the bootstrap and a proposed state
    double *init_rel;      // [2][T_max][12] bootstrap poses, first-pass poses of the bootstrap's state
    float *sampf;          // SoA [7][slots] whitened pose samples (FP32) for the mean-shift
    int *gcnt;             // [S_max] valid samples per group
    int *gpre;             // [S_max] first sample of each group inside its block
    int *bcnt;             // [S_max / 16 + 1][2] samples and valid groups per block
    double *bws;           // [S_max / 16 + 1] weight sum per block
    double *seed_part;     // [kMaxSeeds + 1][seed parts] partial densities of the start candidates
    double *prev_pose;     // [12] staging of a host-provided previous pose
    double *pose_tmp;      // [16]
    double *rel_tmp;       // [T_max][12] poses for step entry points
    float *theta_tmp;      // [H_max W_max]
    float2 *flows_t;       // [T_max][W_max][H_max]: the window's flows transposed, for the column sweeps
    // all-pixel start candidates (pose_start = 1), n = 1 + sample slots at most
    float *cand_F;         // [n][12] FP32 frames of M_t = T_c o M_{t-1}
    int *cand_slot;        // [n] sample slot, -1 previous pose, -2 none
    int *cand_n;           // [4] candidate count
    float *cand_part;      // [n][kCandTiles] partial scores
    double *cand_score;    // [n] scores, dense order
    double *cand_start;    // [8] start point p (6), valid
    // optional phase timing of windows: device timestamps written on the
    // window's stream, one ring slot per window so that windows enqueued back
    // to back keep theirs
    int timing;
    int n_ev;              // stamps of the window being recorded
    int tw_cur;            // its ring slot
    long long tw_count;    // windows recorded since the last summary
    unsigned long long *stamps;        // device [kTimingRing][kEvPerWin]
    unsigned long long *stamps_host;   // host copy
    double stamp_khz;                  // rate of the real-time counter
    int ev_phase[vo::kTimingRing][vo::kEvPerWin];   // phase of the interval that ends at a stamp
    int ev_launches[vo::kTimingRing][vo::kEvPerWin];   // kernel launches of a sweep interval
    int ev_n[vo::kTimingRing];
    double last_ms[8];
    hipStream_t last_stream;
};

namespace vo {

// ---- whole window (vo_api.hip)
bool window_args_ok(const voldor_ctx *c, const float *flows, int T, int H, int W, const double *K,
                    const voldor_params *p, const double *poses, const float *depth,
                    const float *rigidness);
// optional initial state proposed for a window (depth [H][W], rigidness [T][H][W]);
// choice (device int, may be NULL) receives 1 when it replaced the bootstrap's
// T1 (device double[12], may be NULL): T_1 given instead of the bootstrap's
// estimate (overlapping consecutive windows)
struct WindowInit {
    const float *depth;
    const float *rig;
    int32_t *choice;
    const double *T1;
};
int window_enqueue(voldor_ctx *c, const float *flows, int T, int H, int W, const double *K,
                   const voldor_params *p, double *poses, float *depth, float *rigidness,
                   double *loglik, int32_t *status_out, hipStream_t s, const WindowInit *init = nullptr);

// ---- sweep / emission (vo_sweep.hip)
int launch_sweep(voldor_ctx *c, const float *theta_in, float *theta_out, const float2 *flows,
                 const WinDims &d, const EmisParams &e, float gamma, uint64_t seed,
                 int64_t gsweep, int dir, const double *range_dev, float *q_out, hipStream_t s,
                 int criterion);
// theta_gauge (with rel_poses): also writes theta / |t_1| there, after use
int launch_rigidness(voldor_ctx *c, const float *theta, const float2 *flows, const WinDims &d,
                     const EmisParams &e, float *r, float *ell, float *logrho, float *logmu,
                     double *ll_out, hipStream_t s, float *theta_gauge = nullptr,
                     const double *rel_poses = nullptr);
int launch_philox(const uint64_t *ctr, uint64_t k0, uint64_t k1, uint64_t *out, int n,
                  hipStream_t s);
// the window's flows transposed into c->flows_t; every sweep of columns reads
// that copy, so it runs before a window's (or a step entry point's) sweeps
int launch_transpose_flows(voldor_ctx *c, const float2 *flows, int T, int H, int W, hipStream_t s);
// LDS bytes of one chain of length L with nt threads (256, 512, 768 or 1024)
size_t sweep_lds_bytes(int T, int L, int criterion, int nt);
// threads per chain and look-ahead cap of chains of length L (axis 0 rows, 1
// columns): the tuned entry of this class, else the axis default
void sweep_cfg_for(const voldor_ctx *c, int axis, int L, int T, int crit, int *nt, int *la);
void sweep_cfg_store(voldor_ctx *c, int L, int T, int crit, int nt, int la);

// ---- pose (vo_pose.hip)
int launch_pose_step(voldor_ctx *c, const float *theta, const float *rig, const float2 *flows,
                     const WinDims &d, const EmisParams &e, const PoseParams &pp, int t, int it,
                     int have_prev, double *rel_poses, hipStream_t s);
int launch_samples_aos(voldor_ctx *c, int S, double *out, hipStream_t s);
size_t pose_sample_slots(int S_max);
size_t pose_seed_parts();
int launch_gauge_poses(voldor_ctx *c, double *rel_poses, const WinDims &d, hipStream_t s);
int launch_cumulative(voldor_ctx *c, const double *rel_poses, int T, hipStream_t s);

// ---- bootstrap (vo_boot.hip)
// T1_seed (device double[12], or NULL): T_1 given instead of estimated
int launch_bootstrap(voldor_ctx *c, const float2 *flows, const WinDims &d, int n_hyp, int n_eval,
                     uint64_t seed, double depth_lo, double depth_hi, double *rel_poses,
                     float *theta, hipStream_t s, const double *T1_seed = nullptr);

// ---- lockstep batches: the windows of one batch lane advance together, and
// each pose-step kernel, sweep and rigidness pass is one launch over the
// (window, frame) or (window, chain) items of all of them.  A plan holds the
// argument arrays of those launches, built on the host once per distinct
// batch call and uploaded to device memory; the launches read their window's
// arguments from it.
struct WinRef {
    voldor_ctx *c;          // the window's own workspace
    const float2 *X;
    WinDims d;
    EmisParams e;
    PoseParams pp;
    float *depth, *rig;
    double *poses;
};

struct MultiLaunch {
    int kind;          // kernel (kMulti*)
    int variant;       // template variant of a sweep: ((nt / 256) * 2 + criterion) * 2 + model
    size_t off, off2;  // byte offsets of its argument arrays in the plan
    int nwin;          // windows (grid y; a sweep's window count)
    int gx;            // grid x
    size_t lds;        // dynamic LDS bytes
};
enum : int {
    kMultiPoseGroups = 1, kMultiPoseSeed, kMultiPoseMs, kMultiGauge, kMultiSweep, kMultiRig, kMultiLL,
    kMultiBootInit, kMultiBootHyp, kMultiBootScore, kMultiBootPick, kMultiBootVote, kMultiBootTri, kMultiSelInit,
    kMultiHist, kMultiHistPick, kMultiBootFinal
};

struct Plan {
    std::vector<unsigned char> host;
    // append n records, 256-byte aligned; returns their byte offset
    template <typename A>
    size_t put(const A *a, size_t n)
    {
        const size_t off = (host.size() + 255) & ~(size_t)255;
        host.resize(off + sizeof(A) * n);
        memcpy(host.data() + off, a, sizeof(A) * n);
        return off;
    }
};

// the pose step of frame t, iteration it, for windows w[idx[k]] (every one has
// T >= t): its three kernels, arguments as launch_pose_step (KDE start only)
void plan_pose_step(Plan &p, std::vector<MultiLaunch> &out, const std::vector<WinRef> &w,
                    const std::vector<int> &idx, int t, int it);
void plan_gauge_poses(Plan &p, std::vector<MultiLaunch> &out, const std::vector<WinRef> &w,
                      const std::vector<int> &idx);
int launch_pose_multi(const MultiLaunch &m, const unsigned char *dev, hipStream_t s);
// one sweep (direction dir, global sweep index gsweep) of every chain of the
// windows: one launch per class of threads per chain and LDS bytes
void plan_sweep(Plan &p, std::vector<MultiLaunch> &out, const std::vector<WinRef> &w,
                const std::vector<int> &idx, float gamma, uint64_t seed, int64_t gsweep, int dir,
                int criterion);
// the rigidness pass of the windows: W and the scale gauge (gauge), or the
// log-likelihood into ll[k] (device double[2] per window) through ll_part
void plan_rigidness(Plan &p, std::vector<MultiLaunch> &out, const std::vector<WinRef> &w,
                    const std::vector<int> &idx, bool gauge, const std::vector<double *> &ll);
int launch_sweep_multi(const MultiLaunch &m, const unsigned char *dev, hipStream_t s);

// the bootstraps of the windows (no T_1 given): their kernels, one launch each
void plan_bootstrap(Plan &p, std::vector<MultiLaunch> &out, const std::vector<WinRef> &w,
                    const std::vector<int> &idx, int n_hyp, int n_eval, uint64_t seed, double depth_lo,
                    double depth_hi);
int launch_boot_multi(const MultiLaunch &m, const unsigned char *dev, hipStream_t s);

// the steps of one lockstep lane, in stream order
struct LockStep {
    int kind;          // kStep*
    MultiLaunch m;     // kStepMulti
    int win;           // window (index into the lane's WinRef list) of a transpose, bootstrap or status copy
    int phase, launches;   // timing stamp
};
enum : int { kStepMulti = 0, kStepBoot, kStepStamp, kStepStatus, kStepTranspose };
// plans the lockstep schedule of windows w[idx[k]] (contexts wc[k]) under
// parameters p: the lane's WinRef list, its steps, the argument arrays in plan
void lockstep_plan(voldor_ctx *const *wc, const voldor_window_desc *w, const std::vector<int> &idx,
                   const voldor_params *p, Plan &plan, std::vector<WinRef> &refs, std::vector<LockStep> &steps);
// enqueues a planned lane on s (plan_dev: the uploaded plan; timing stamps on lane)
int lockstep_run(voldor_ctx *lane, const std::vector<WinRef> &refs, const std::vector<LockStep> &steps,
                 const voldor_window_desc *w, const std::vector<int> &idx, const voldor_params *p,
                 const unsigned char *plan_dev, int32_t *status_out, hipStream_t s);

}  // namespace vo
