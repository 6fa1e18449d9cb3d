/*
 * voldor.h -- C ABI of the MI355X (gfx950) window solver of VOLDOR
 * (Min, Yang, Dunn, "VOLDOR: Visual Odometry from Log-logistic Dense Optical
 * flow Residuals", CVPR 2020).
 *
 * The library infers, from T externally computed dense optical-flow fields
 * X_1..X_T (X_t maps image I_{t-1} to I_t; problem statement, Sec. 3), the
 * relative camera poses T_1..T_T, the depth map theta of the first frame and
 * the per-frame rigidness maps W_1..W_T, by the generalized-EM loop of
 * Table 1: bootstrap; then per iteration the pose of every frame (Eq. 15-19),
 * the rigidness E-step by forward-backward on image rows/columns (Eq. 11-14),
 * the depth M-step by the maximum-inlier criterion with sampling and
 * propagation (Eq. 10, Fig. 5), and the unsmoothed rigidness.
 *
 * Conventions shared by every entry point
 *   - pixel j = (x, y), integer pixel centres, index j = y*W + x;
 *   - flows: float32 [T][H][W][2], (u, v) = displacement in pixels of pixel
 *     (x, y) of image t-1; non-finite components mark a missing observation;
 *   - poses: 12 doubles, row-major R (9) then t (3); a point moves as
 *     P_t = R P_{t-1} + t (relative pose of frame t to frame t-1);
 *   - depth: z-depth along K^-1 [x y 1]^T, in units of |t_1| (= 1);
 *   - "device" pointers are HIP device memory of the current device; "host"
 *     pointers are ordinary CPU memory.  The caller owns all buffers; nothing
 *     is retained after a call returns.
 *   - every call returns a voldor_status; nothing throws across the ABI.
 *     VOLDOR_EINVAL leaves all outputs untouched.
 */
#ifndef VOLDOR_H
#define VOLDOR_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    VOLDOR_OK = 0,
    VOLDOR_EINVAL = -1,      /* bad argument: null pointer, size, parameter range   */
    VOLDOR_ENOMEM = -2,      /* device allocation failed (voldor_create only)       */
    VOLDOR_EDEVICE = -3,     /* a HIP runtime call failed                            */
    VOLDOR_EDEGENERATE = -4  /* bootstrap impossible: < 8 usable flows in X_1, or no */
                             /* finite epipolar hypothesis, or no valid depth       */
} voldor_status;

/* Solver parameters.  struct_size must equal sizeof(voldor_params).
 * Defaults (voldor_params_default) follow the paper's experiments: lambda =
 * 0.15, gamma = 0.9, kernel covariance diag(0.1 I3, 0.004 I3), a1 = 0.01,
 * a2 = 0.09, b1 = -0.0022, b2 = 1.0 (Sec. 6.1). */
typedef struct {
    uint32_t struct_size;
    int32_t n_iters;           /* EM iterations (Table 1 loop)                       */
    int32_t sweeps_per_iter;   /* directional sweeps per iteration: L>R,T>B,R>L,B>T */
    int32_t n_pose_groups;     /* S: P3P groups per frame (Eq. 16), <= 8192          */
    int32_t n_seeds;           /* mean-shift start candidates from the samples, <=255*/
    int32_t ms_max_iters;      /* mean-shift iteration cap                           */
    int32_t lmeds_hypotheses;  /* bootstrap 8-point hypotheses, <= 4096              */
    int32_t lmeds_eval_pixels; /* bootstrap residual subset, 8..16384                */
    double ms_tol;             /* mean-shift stop: Mahalanobis length of the step    */
    double a1, a2, b1, b2;     /* Fisk scale A(v) = a1 exp(a2|v|), shape B(v) = b1|v|+b2 (Eq. 6-7) */
    double lambda;             /* outlier density: Fisk at EPE = lambda |v| (Eq. 8)  */
    double gamma;              /* rigidness transition probability (Eq. 11), [0.5,1)*/
    double sigma2_trans;       /* kernel covariance, translation variance (Eq. 18)   */
    double sigma2_rot;         /* kernel covariance, rotation variance (Eq. 18)      */
    double beta_min;           /* floor applied to B(v)                               */
    double x_floor;            /* floor applied to squared residuals (px^2)           */
    double depth_lo, depth_hi; /* > 0: fixed depth sampling range; 0: from bootstrap */
    uint64_t seed;             /* Philox4x64-10 key word 0 of every random draw      */
    int32_t criterion;         /* depth M-step: VOLDOR_CRITERION_MIE (Eq. 10) or     */
                               /* VOLDOR_CRITERION_MLE (Eq. 9, expected log-likelihood */
                               /* sum_t q log rho + (1-q) log mu; a missing frame adds 0)*/
    int32_t pose_start;        /* mean-shift start: 0 the densest (kernel density) of */
                               /* the previous pose and the first n_seeds samples;    */
                               /* 1 the candidate (previous pose, then every sample)  */
                               /* of highest sum over all pixels of W_t ell_t        */
    int32_t residual_model;    /* density of rho (Eq. 4) and mu (Eq. 8):             */
                               /* VOLDOR_RESIDUAL_FISK (Eq. 5, scale and shape by     */
                               /* Eq. 6-7) or VOLDOR_RESIDUAL_GAUSS, the Gaussian      */
                               /* model of the paper's ablations (Sec. 6, Fig. 8-9):  */
                               /* squared EPE exponential with mean A(v) / ln 2, the  */
                               /* Fisk's median; b1, b2, beta_min unused              */
    int32_t pad;               /* 0                                                   */
} voldor_params;

enum { VOLDOR_CRITERION_MIE = 0, VOLDOR_CRITERION_MLE = 1 };
enum { VOLDOR_RESIDUAL_FISK = 0, VOLDOR_RESIDUAL_GAUSS = 1 };

/* Fill *p with the defaults above (n_iters 3, 4 sweeps, S 256, 64 seeds,
 * 100 mean-shift iterations, tol 1e-5, 512 hypotheses, 16384 eval pixels,
 * beta_min 0.01, x_floor 1e-12, automatic depth range, seed 0, MIE, KDE start). */
void voldor_params_default(voldor_params *p);

/* Static description of a status code. */
const char *voldor_status_str(int status);

/* Opaque solver context: owns the device workspace for windows up to
 * T_max x H_max x W_max with at most S_max pose groups per frame, on the device
 * current at creation.  T_max <= 16, 16 <= H_max, W_max <= 4096.
 * Returns VOLDOR_ENOMEM / VOLDOR_EDEVICE on allocation failure. */
typedef struct voldor_ctx voldor_ctx;
int voldor_create(voldor_ctx **out, int T_max, int H_max, int W_max, int S_max);
void voldor_destroy(voldor_ctx *ctx);

/* Solve one window (Table 1).
 *   flows     device float32 [T][H][W][2], 8-byte aligned
 *   K         host double[4] = fx, fy, cx, cy (pixels)
 *   p         host parameters
 *   poses     device double [T][12], relative poses T_1..T_T (output)
 *   depth     device float  [H][W], depth of frame 0 (output)
 *   rigidness device float  [T][H][W], final unsmoothed W_t (output)
 *   loglik    device double [2] or NULL: log-likelihood of Eq. 3 under the final
 *             rigidness, and the L1 mass of its terms (output)
 *   stream    hipStream_t (NULL = default stream)
 * Work is enqueued on `stream`; the call waits for it to finish and returns
 * the device-side status (VOLDOR_EDEGENERATE leaves the outputs unspecified).
 * Calls that share a context must not overlap. */
int voldor_window(voldor_ctx *ctx, const float *flows, int T, int H, int W, const double *K,
                  const voldor_params *p, double *poses, float *depth, float *rigidness,
                  double *loglik, void *stream);

/* The same window (Table 1), enqueued without waiting: windows submitted back
 * to back on one stream run with no host round trip between them.
 *   status_out  device int32, 4-byte aligned: receives the window's device
 *               status (VOLDOR_OK or VOLDOR_EDEGENERATE) when its work is done
 * Other arguments as voldor_window.  The return value covers only the host-side
 * checks (VOLDOR_EINVAL, VOLDOR_EDEVICE for a failed launch); inputs and outputs
 * must stay allocated until the stream reaches the end of the window.  All
 * windows of one context must be enqueued on one stream (they share its
 * workspace in stream order). */
int voldor_window_async(voldor_ctx *ctx, const float *flows, int T, int H, int W, const double *K,
                        const voldor_params *p, double *poses, float *depth, float *rigidness,
                        double *loglik, int32_t *status_out, void *stream);

/* The window with a proposed initial state (an extension: Table 1 starts from
 * the bootstrap).  The bootstrap still runs (T_1, depth range); the proposal's
 * depth init_depth (device float [H][W], > 0, in the scale |t_1| = 1) and
 * rigidness init_rig (device float [T][H][W]) replace the bootstrap's depth and
 * W = 1 when the log-likelihood of X_1 under T_1 (Eq. 3 at the posterior
 * rigidness) is higher with them; the pose steps of the first iteration then
 * weigh by that rigidness.  choice_out (device int32 or NULL) receives 1 when
 * the proposal was used.  Enqueued like voldor_window_async. */
int voldor_window_init(voldor_ctx *ctx, const float *flows, int T, int H, int W, const double *K,
                       const voldor_params *p, const float *init_depth, const float *init_rig, double *poses,
                       float *depth, float *rigidness, double *loglik, int32_t *status_out, int32_t *choice_out,
                       void *stream);

/* The same window with T_1 given instead of estimated: the paper's
 * alternative for overlapping consecutive batches (Sec. 5.3), where T_1 comes
 * from the previous window's estimate of the same frame pair.
 *   T1  device double[12] (R row-major, t), 8-byte aligned; read when the
 *       window's work runs, so it may be an earlier window's pose output on the
 *       same stream.  Its translation is rescaled to unit length (the gauge);
 *       the depth follows by two-view triangulation from T_1 and X_1.  A
 *       non-finite pose or zero translation gives VOLDOR_EDEGENERATE.
 * Enqueued without waiting, like voldor_window_async. */
int voldor_window_seeded(voldor_ctx *ctx, const float *flows, int T, int H, int W, const double *K,
                         const voldor_params *p, const double *T1, double *poses, float *depth, float *rigidness,
                         double *loglik, int32_t *status_out, void *stream);

/* Sliding-window visual odometry over N flows X_1..X_N (Sec. 5.3): windows of
 * T flows start at frames 0, stride, 2 stride, ..., with a last one ending at
 * flow N (voldor_vo_windows gives their count: 2 <= T <= 16, T <= N,
 * 1 <= stride < T).  The first window is bootstrapped from X_1; every later one
 * takes T_1 from the previous window's estimate of the same frame pair, on the
 * device, with no host round trip.  Each window fixes its own scale (|t_1| = 1);
 * the trajectory chains them.
 *   flows     device float32 [N][H][W][2]
 *   wposes    device double [windows][T][12]: every window's relative poses
 *   depth, rigidness  device float [H][W], [T][H][W]: the last window's results
 *   wstatus   device int32 [windows]: each window's status
 *   traj      device double [N+1][12]: camera poses M_k (x_k = M_k x_0) in the
 *             first window's scale; all NaN if any window failed
 * Enqueued without waiting.  Returns VOLDOR_EINVAL for bad sizes. */
int voldor_vo_windows(int N, int T, int stride);
int voldor_vo_sequence(voldor_ctx *ctx, const float *flows, int N, int H, int W, const double *K,
                       const voldor_params *p, int T, int stride, double *wposes, float *depth, float *rigidness,
                       int32_t *wstatus, double *traj, void *stream);

/* Threads per chain of the depth sweeps (256, 512, 768 or 1024; 0 = 512), row
 * sweeps and column sweeps apart.  The width changes how a chain's work is
 * spread over a workgroup and how many chains fit a CU, never the result: all
 * widths give the same depth bit for bit.  Windows whose chains would not fit
 * the LDS at the chosen width are rejected with VOLDOR_EINVAL. */
int voldor_set_sweep_threads(voldor_ctx *ctx, int rows, int cols);
int voldor_get_sweep_threads(const voldor_ctx *ctx, int *rows, int *cols);

/* Look-ahead of the propagation rounds (Fig. 5's neighbour candidate found
 * for every chain position at once): in each round every live origin tests its
 * value at up to `cap` further positions, at most threads / live origins; 0
 * means no cap (the whole workgroup every round).  A small cap wastes fewer
 * evaluations past each origin's first loss and takes more rounds.  Like the
 * width it never changes the result.  Row and column sweeps apart; cap 0 or
 * 1..4096, else VOLDOR_EINVAL. */
int voldor_set_sweep_lookahead(voldor_ctx *ctx, int rows, int cols);
int voldor_get_sweep_lookahead(const voldor_ctx *ctx, int *rows, int *cols);

/* Autotuner: solves the given window once (device flows as voldor_window),
 * then times the row and the column sweeps from its final state at every
 * setting of the two tuning axes, threads per chain (256, 512, 768, 1024 where
 * the chain fits the LDS) and the look-ahead cap (none, 32, 16, 8, 4, 2), and keeps
 * the fastest for this chain class
 * (chain length, T, depth criterion) in the context: windows of that class then
 * use it, others the defaults of voldor_set_sweep_threads/_lookahead (which
 * drop every tuned class).  The threads chosen for rows and columns are
 * returned in *rows_out, *cols_out if not NULL.  Waits for the device.
 * VOLDOR_EDEGENERATE if the bootstrap fails (nothing is then kept); allocates
 * (and frees) one rigidness map of scratch.
 * voldor_sweep_tuning lists the tuned classes: out[4i .. 4i+3] = chain length,
 * T, threads, look-ahead cap; returns their number (at most max_n). */
int voldor_autotune(voldor_ctx *ctx, const float *flows, int T, int H, int W, const double *K,
                    const voldor_params *p, int *rows_out, int *cols_out, void *stream);
int voldor_sweep_tuning(const voldor_ctx *ctx, int *out, int max_n);

/* Regression of the Fisk laws of Eq. 6-7 on optical-flow residuals (the
 * procedure behind Fig. 4b).  Items x = |X - G|^2 (floored at x_floor) are
 * binned by |X| in nbins equal bins over [0, v_max); each bin with at least
 * min_count items is fitted by the moments of log x (log of a Fisk variable is
 * logistic with location log A and scale 1/B); log A and B are then fitted
 * against the bins' mean |X| by least squares weighted by the counts.
 *   X, G    device float [n][2]: observed flows and reference flows, 8-byte
 *           aligned; items with a non-finite component are skipped
 *   laws    host double[4]: a1, a2, b1, b2 (output)
 *   bins    host double [nbins][4] or NULL: count, sum |X|, sum log x,
 *           sum (log x)^2 per bin (output)
 * 2 <= nbins <= 256.  Waits for the device.  VOLDOR_EDEGENERATE if fewer than
 * two bins qualify.  Allocates its own scratch. */
int voldor_residual_fit(const float *X, const float *G, int64_t n, int nbins, double v_max, double x_floor,
                        int min_count, double *laws, double *bins, void *stream);

/* The binning pass of voldor_residual_fit alone, enqueued without waiting:
 *   work  device double[voldor_residual_workspace(n, nbins)]: scratch (the query
 *         returns VOLDOR_EINVAL, negative, for n < 1 or nbins outside [2, 256])
 *   bins  device double [nbins][4]: count, sum |X|, sum log x, sum (log x)^2 */
int64_t voldor_residual_workspace(int64_t n, int nbins);
int voldor_residual_bins(const float *X, const float *G, int64_t n, int nbins, double v_max, double x_floor,
                         double *work, double *bins, void *stream);

/* voldor_residual_bins for callers that cannot allocate device memory (code
 * under HIP graph capture, tight serving loops, harnesses that forbid
 * hipMalloc): the same kernels and result, bit for bit, with the partials in a
 * static device array of VOLDOR_RESIDUAL_SCRATCH_DOUBLES doubles (2 MiB) that
 * every device the library runs on holds until the process ends.  Nothing is
 * allocated and no part of the array needs to start at zero (every partial is
 * written before it is read).  VOLDOR_EINVAL when the partials,
 * voldor_residual_workspace(n, nbins) doubles, exceed the array (e.g. more
 * than 64 bins at n >= 2^21 items), or for the arguments voldor_residual_bins
 * rejects; VOLDOR_EDEVICE when the runtime cannot give the array's address on
 * the current device.  All calls on one device share its array: calls that
 * overlap on one device (two streams, or two host threads) race.  Enqueued
 * without waiting. */
#define VOLDOR_RESIDUAL_SCRATCH_DOUBLES 262144
int voldor_residual_bins_noalloc(const float *X, const float *G, int64_t n, int nbins, double v_max,
                                 double x_floor, double *bins, void *stream);

/* ---- batches: many windows of uneven shape and T ------------------------- */

/* One window of a batch: the arguments of voldor_window for that window. */
typedef struct {
    const float *flows;    /* device float32 [T][H][W][2], 8-byte aligned           */
    int32_t T, H, W;
    double K[4];           /* fx, fy, cx, cy (pixels)                                */
    double *poses;         /* device double [T][12] (output)                         */
    float *depth;          /* device float [H][W] (output)                           */
    float *rigidness;      /* device float [T][H][W] (output)                        */
    double *loglik;        /* device double [2] or NULL (output)                     */
    const float *init_depth;  /* device float [H][W] or NULL: proposed initial state, */
    const float *init_rig;    /* device float [T][H][W] or NULL  as voldor_window_init */
    int32_t *choice;          /* device int32 or NULL: 1 when the proposal was used    */
    int32_t n_pose_groups;    /* P3P groups per frame of this window (0: params')     */
    int32_t pad;
} voldor_window_desc;

/* Batch solver: `lanes` (1..16) HIP streams, each with the workspace of a
 * context sized T_max x H_max x W_max x S_max.  Windows are independent, so a
 * batch is spread over the lanes (largest first, onto the least loaded lane)
 * and the lanes run concurrently: one window's latency-bound pose steps
 * overlap the sweeps of the others.  Measured on MI355X with ROCm's graph
 * replay: the work of at most four lanes runs at once, a further lane starting
 * when an earlier one ends.  flags: VOLDOR_BATCH_GRAPH captures each
 * distinct batch call into a HIP graph on first use and replays it when the
 * same call (descriptors, count, parameters, status array, stream) comes again.
 * Returns VOLDOR_EINVAL / VOLDOR_ENOMEM / VOLDOR_EDEVICE like voldor_create. */
typedef struct voldor_batch voldor_batch;
/* VOLDOR_BATCH_LOCKSTEP: the windows of each lane advance together, with one
 * workspace per window (allocated on the first call with that many windows):
 * each of a pose step's three kernels is one launch over the (window, frame)
 * items of the lane's windows, each sweep one launch over their (window,
 * chain) items per threads-per-chain class, each rigidness pass one launch
 * over their pixels: the work-list form of a batch of Table 1 runs.  The launch
 * arguments are built on the host and uploaded once per distinct call; a call
 * with new descriptors waits for the stream and the lanes first.  Results are
 * still those of voldor_window on each window, bit for bit.  Needs the KDE
 * pose start (pose_start 0) and no proposed initial state; VOLDOR_EINVAL
 * otherwise. */
enum { VOLDOR_BATCH_GRAPH = 1, VOLDOR_BATCH_LOCKSTEP = 2 };
int voldor_batch_create(voldor_batch **out, int lanes, int T_max, int H_max, int W_max, int S_max,
                        int flags);
void voldor_batch_destroy(voldor_batch *b);

/* Solve n windows (Table 1 for each; the same parameters for all), enqueued
 * on `stream` without waiting: the batch starts after the work already on
 * `stream` and the stream continues after all of it.
 *   wins        host array of n descriptors (read during the call only)
 *   status_out  device int32 [n], 4-byte aligned: window i's device status
 * Results are those of voldor_window on each window, bit for bit.  Host-side
 * errors (VOLDOR_EINVAL for any bad descriptor, before anything is enqueued;
 * VOLDOR_EDEVICE) are returned.  Batches of one batch object run one after
 * another in stream order; calls must not overlap on the host.  Graph mode
 * needs a stream other than the null stream. */
int voldor_window_batch(voldor_batch *b, const voldor_window_desc *wins, int n, const voldor_params *p,
                        int32_t *status_out, void *stream);

/* Sweep widths and look-ahead caps of every lane of the batch (as
 * voldor_set_sweep_threads and voldor_set_sweep_lookahead). */
int voldor_batch_set_sweep_threads(voldor_batch *b, int rows, int cols);
int voldor_batch_set_sweep_lookahead(voldor_batch *b, int rows, int cols);

/* Autotuner of a batch: voldor_autotune on the first window of every distinct
 * chain class (shape, T, criterion) among the n descriptors, the settings then
 * shared by every lane.  Waits for the device.  Results never depend on it. */
int voldor_batch_autotune(voldor_batch *b, const voldor_window_desc *wins, int n, const voldor_params *p,
                          void *stream);

/* Phase timing of a batch's windows, each lane as voldor_set_timing (a
 * captured graph replays the event records, so the summary covers the last
 * replay of every window captured since the previous summary).  The summary
 * waits, then gives in out[0..6] the phase SUMS (not means) over the windows
 * of every lane, the last 32 of each lane at most, in out[7] the time during
 * which at least one lane ran sweeps (the union of the windows' sweep
 * intervals on the device's real-time counter), and their number. */
int voldor_batch_set_timing(voldor_batch *b, int enable);
int voldor_batch_timing_summary(voldor_batch *b, double *out, int *n_windows);

/* Phase timing of windows with HIP events recorded on their stream, kept for
 * the last 32 windows.  voldor_set_timing(ctx, 1) creates the events (0
 * destroys them).  Phases, in milliseconds: [0] bootstrap, [1] pose steps,
 * [2] directional sweeps, [3] number of sweep launches, [4] rigidness and
 * gauge, [5] log-likelihood, [6] whole window, [7] unused.
 * voldor_last_timing: out[8] of the last voldor_window call (or of the last
 * window a summary covered).
 * voldor_timing_summary: waits for the stream of the last window, then fills
 * out[8] with the mean over the windows enqueued since the previous summary
 * (the last 32 of them at most) and their number in *n_windows (may be NULL);
 * starts a new count.  VOLDOR_EINVAL when timing is off. */
int voldor_set_timing(voldor_ctx *ctx, int enable);
int voldor_last_timing(voldor_ctx *ctx, double *out);
int voldor_timing_summary(voldor_ctx *ctx, double *out, int *n_windows);

/* ---- learned proposal of the initial state ------------------------------- */

/* An extension beyond the paper (whose EM starts from the bootstrap of
 * Sec. 5.3): a small convolutional network maps the 2T flow channels of a
 * window to an initial depth and T rigidness maps, which the plain EM then
 * refines and judges.  Six 3x3 convolutions, stride 1, zero padding: input 32
 * channels (channel 2(t-1)+c = component c of X_t / 16, non-finite as 0, the
 * rest 0), layers 1-5 with 32 outputs and ReLU, layer 6 with 16 outputs of
 * which 0 is log theta and 1..T the logits of W_t.  BF16 weights and
 * activations, FP32 accumulation on the matrix cores, FP32 master weights.
 * Loss: mean squared log-depth error + mean binary cross-entropy of W against
 * targets; Adam (beta 0.9 / 0.999, eps 1e-8) with bias correction.
 *
 * Parameters, host float array of voldor_net_param_count() values, layer by
 * layer: w[3][3][C_in][C_out] (dy, dx, in, out), then b[C_out]; C_in = 32,
 * C_out = 32 (layer 6: 16).  Weights of padded channels must be 0.
 * All tensors below are device memory; the calls enqueue on `stream` (except
 * set/get params, which wait). */
typedef struct voldor_net voldor_net;
int voldor_net_create(voldor_net **out, int T, int N_max, int H_max, int W_max);   /* T <= 8 */
void voldor_net_destroy(voldor_net *net);
int voldor_net_param_count(const voldor_net *net);
int voldor_net_set_params(voldor_net *net, const float *host_params);   /* also resets Adam */
int voldor_net_get_params(voldor_net *net, float *host_params);

/* Forward pass on N windows: flows float32 [N][T][H][W][2]; depth float
 * [N][H][W] = exp(z_0) (or NULL); rig float [N][T][H][W] = sigmoid(z_t) (or
 * NULL); z_out float [N][H][W][16] raw outputs (or NULL). */
int voldor_net_forward(voldor_net *net, const float *flows, int N, int H, int W, float *depth, float *rig,
                       float *z_out, void *stream);

/* Loss and gradient at the current parameters against target depth float
 * [N][H][W] (> 0) and rigidness float [N][T][H][W]: loss_out double[1] (or
 * NULL), grad_out float [param_count] in the parameter layout (or NULL). */
int voldor_net_gradient(voldor_net *net, const float *flows, int N, int H, int W, const float *depth,
                        const float *rig, double *loss_out, float *grad_out, void *stream);

/* One Adam step of learning rate lr on the same loss. */
int voldor_net_train_step(voldor_net *net, const float *flows, int N, int H, int W, const float *depth,
                          const float *rig, float lr, double *loss_out, void *stream);

/* One layer k (0..5) on explicit BF16 tensors [N][H][W][32]: forward (out bf16
 * [N][H][W][32], or float [N][H][W][16] for k = 5) or, with backward != 0 and
 * k >= 1, the gradient to the layer's input times (mask > 0). */
int voldor_net_layer(voldor_net *net, int k, int backward, const void *in, const void *mask, void *out, int N,
                     int H, int W, void *stream);

/* ---- step entry points: one step of the loop on explicit state ----------- */

/* Philox4x64-10 (Salmon et al., SC'11) on n counters: ctr, out device
 * uint64 [n][4]; key = (key0, key1). */
int voldor_philox(const uint64_t *ctr, uint64_t key0, uint64_t key1, uint64_t *out, int n,
                  void *stream);

/* Emission of Eq. 2-8 for the depth map theta (device float [H][W]) under the
 * cumulative poses M (host double [T+1][12], M_0 = I): r = rho/(rho+mu),
 * ell = log r, log rho, log mu, each device float [T][H][W] (any may be NULL).
 * Missing observations give r = 1/2, ell = log 1/2, logrho = logmu = 0. */
int voldor_emission(voldor_ctx *ctx, const float *theta, const float *flows, int T, int H, int W,
                    const double *K, const voldor_params *p, const double *M, float *r, float *ell,
                    float *logrho, float *logmu, void *stream);

/* One directional sweep (E-step forward-backward on the chains of direction
 * dir, then the MIE depth walk with q held fixed; Eq. 10-14, Fig. 5).
 *   theta_in / theta_out  device float [H][W] (may alias)
 *   M        host double [T+1][12] cumulative poses
 *   d_lo, d_hi  depth sampling range; global_sweep = it*sweeps_per_iter + s
 *   dir      0 left->right (rows), 1 top->bottom (columns), 2 right->left, 3 bottom->top
 *   q_out    device float [T][H][W] or NULL: smoothed rigidness of the E-step */
int voldor_sweep(voldor_ctx *ctx, const float *theta_in, float *theta_out, const float *flows,
                 int T, int H, int W, const double *K, const voldor_params *p, const double *M,
                 double d_lo, double d_hi, int64_t global_sweep, int dir, float *q_out,
                 void *stream);

/* Pose of frame t (1..T) for EM iteration `it` (Eq. 15-19): P3P samples of
 * S random pixel triples, weighted by the product of their rigidness, mapped
 * to se(3), mode by Gaussian mean-shift.
 *   theta     device float [H][W]; rig device float [T][H][W] or NULL (all 1)
 *   M         host double [T+1][12] (M_{t-1} is used)
 *   prevT     host double[12] or NULL: previous estimate of T_t (also returned
 *             when no sample carries weight)
 *   T_out     host double[12] (output)
 *   samples   device double [4S][8] or NULL: (p[6], weight, valid) per group slot
 *   diag      host int[4] or NULL: samples, valid groups, mean-shift iterations,
 *             fallback flag */
int voldor_pose_step(voldor_ctx *ctx, const float *theta, const float *rig, const float *flows,
                     int T, int H, int W, const double *K, const voldor_params *p, const double *M,
                     int t, int it, const double *prevT, double *T_out, double *samples, int *diag,
                     void *stream);

/* All-pixel candidate scores of the last pose step run with pose_start = 1 on
 * this context (voldor_pose_step, or the last pose step of a window).  The
 * paper does not describe this scoring: Sec. 5.2 leaves the mean-shift start
 * open, and this option picks it by scoring every hypothesis over every pixel
 * with the E-step weights (an extension beside the default densest start):
 *   scores  host double[max_n]: [0] the previous pose (-inf if there was
 *           none), [1..] every valid sample in (group, root) order, each the
 *           sum over all pixels of W_t ell_t at M_t = T_c o M_{t-1}
 *   n_out   host int: 1 + the number of samples
 * Waits for the device.  VOLDOR_EINVAL when max_n is too small or no such step
 * has run. */
int voldor_pose_scores(voldor_ctx *ctx, double *scores, int max_n, int *n_out);

/* The depth sampling range [d_lo, d_hi] of the last window run on this context,
 * in the gauge its outputs are in (the bootstrap's P1 / 2 and 2 P99, Sec. 5.3,
 * rescaled with the depth after every iteration): host double[2].  Waits for the
 * device.  With the window's outputs it is the whole state an EM iteration
 * starts from. */
int voldor_last_range(voldor_ctx *ctx, double *range2);

/* Bootstrap (Sec. 5.3): T_1 by least median of squares over 8-point
 * essential-matrix hypotheses of X_1, depth by two-view triangulation, the
 * depth sampling range [0.5 P1, 2 P99] of the triangulated depths.
 *   relT   host double[12] (output); theta device float [H][W] (output);
 *   range  host double[2] (output); info host double[4] or NULL: best
 *          hypothesis, its median Sampson residual, valid depths, cheirality count */
int voldor_bootstrap(voldor_ctx *ctx, const float *flows, int T, int H, int W, const double *K,
                     const voldor_params *p, double *relT, float *theta, double *range,
                     double *info, void *stream);

#ifdef __cplusplus
}
#endif
#endif /* VOLDOR_H */
