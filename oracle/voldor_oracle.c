/*
 * voldor_oracle.c -- plain, slow FP64 CPU oracle of VOLDOR's window solver.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product path may call, link or
 * load this file: it exists so that tests, the smoke check and the CPU
 * baseline of the benchmark can compare the HIP library against an
 * independent, obviously-correct statement of the method.  It shares no code,
 * header, table or helper with the HIP library.
 *
 * Paper: Min, Yang, Dunn, "VOLDOR: Visual Odometry from Log-logistic Dense
 * Optical flow Residuals", CVPR 2020 (arXiv 2104.06789).
 *
 * Every step follows the paper in the order it gives (Table 1):
 *   bootstrap   - W := 1, T_1 from epipolar geometry of X_1 by least median
 *                 of squares, depth by two-view triangulation (Sec. 5.3);
 *   per iter    - pose of every frame in turn from P3P samples + mean-shift
 *                 (Sec. 5.2, Eq. 15-19); rigidness E-step by forward-backward
 *                 on 1-D chains (Eq. 11-14); depth M-step by the maximum-
 *                 inlier criterion with sampling + propagation (Eq. 10,
 *                 Fig. 5) or, as a variant, the maximum-likelihood criterion
 *                 it relaxes (Eq. 9); rigidness without smoothing.
 * The residual model is the Fisk (log-logistic) density of the squared
 * end-point error with flow-dependent scale/shape (Eq. 4-8), or, as the
 * variant of the paper's ablations, the density of the squared error under
 * an isotropic Gaussian flow error with the same median.
 *
 * All floating point is double.  Flows arrive as float32 [T][H][W][2].
 * Readings of points the paper leaves open are listed at each function.
 *
 * Parity status: every function below is pinned by CPU tests against closed
 * forms, library routines, brute force or invariants, except the end-to-end
 * outputs on noisy inputs, which the paper gives no worked example for.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

/* ------------------------------------------------------------------------ */
/* parameters (layout mirrored by the Python ctypes wrapper)                */
/* ------------------------------------------------------------------------ */
typedef struct {
    uint32_t struct_size;
    int32_t n_iters;           /* EM iterations                                  */
    int32_t sweeps_per_iter;   /* directional sweeps per iteration               */
    int32_t n_pose_groups;     /* S: P3P groups per frame                        */
    int32_t n_seeds;           /* mean-shift start candidates taken from samples */
    int32_t ms_max_iters;      /* mean-shift iteration cap                       */
    int32_t lmeds_hypotheses;  /* bootstrap 8-point hypotheses                   */
    int32_t lmeds_eval_pixels; /* bootstrap residual subset size                 */
    double ms_tol;             /* mean-shift stop: Mahalanobis step length       */
    double a1, a2, b1, b2;     /* Fisk scale/shape laws, Eq. 6-7                 */
    double lambda;             /* outlier density parameter, Eq. 8               */
    double gamma;              /* HMM transition, Eq. 11                         */
    double sigma2_trans, sigma2_rot; /* kernel covariance diagonal, Eq. 18       */
    double beta_min;           /* floor of the shape B(v)                        */
    double x_floor;            /* floor of the squared residual                  */
    double depth_lo, depth_hi; /* >0: caller-fixed sampling range                */
    uint64_t seed;
    int32_t criterion;         /* depth M-step: 0 MIE (Eq. 10), 1 MLE (Eq. 9)    */
    int32_t pose_start;        /* mean-shift start: 0 densest of n_seeds samples */
                               /* and the previous pose, 1 best all-pixel score  */
    int32_t residual_model;    /* density of rho (Eq. 4) and mu (Eq. 8): 0 Fisk  */
                               /* (Eq. 5), 1 Gaussian flow error (or_gauss_logpdf)*/
    int32_t pad;
} or_params;

enum { OR_OK = 0, OR_EINVAL = -1, OR_EDEGENERATE = -4 };

/* Philox stream purposes (key word 1). */
enum { PURPOSE_DEPTH = 1, PURPOSE_POSE = 2, PURPOSE_BOOT = 3 };

int or_params_size(void) { return (int)sizeof(or_params); }

/* ------------------------------------------------------------------------ */
/* Philox4x64-10 (Salmon, Moraes, Dror, Shaw, SC'11)                        */
/* ------------------------------------------------------------------------ */
void or_philox4x64(const uint64_t ctr_in[4], const uint64_t key_in[2], uint64_t out[4])
{
    const uint64_t M0 = 0xD2E7470EE14C6C93ULL, M1 = 0xCA5A826395121157ULL;
    const uint64_t W0 = 0x9E3779B97F4A7C15ULL, W1 = 0xBB67AE8584CAA73BULL;
    uint64_t c0 = ctr_in[0], c1 = ctr_in[1], c2 = ctr_in[2], c3 = ctr_in[3];
    uint64_t k0 = key_in[0], k1 = key_in[1];
    for (int round = 0; round < 10; ++round) {
        if (round > 0) { k0 += W0; k1 += W1; }
        unsigned __int128 p0 = (unsigned __int128)M0 * c0;
        unsigned __int128 p1 = (unsigned __int128)M1 * c2;
        uint64_t hi0 = (uint64_t)(p0 >> 64), lo0 = (uint64_t)p0;
        uint64_t hi1 = (uint64_t)(p1 >> 64), lo1 = (uint64_t)p1;
        uint64_t n0 = hi1 ^ c1 ^ k0, n1 = lo1, n2 = hi0 ^ c3 ^ k1, n3 = lo0;
        c0 = n0; c1 = n1; c2 = n2; c3 = n3;
    }
    out[0] = c0; out[1] = c1; out[2] = c2; out[3] = c3;
}

static void philox_draw(uint64_t seed, uint64_t purpose, uint64_t a, uint64_t b,
                        uint64_t c, uint64_t d, uint64_t out[4])
{
    uint64_t ctr[4] = {a, b, c, d};
    uint64_t key[2] = {seed, purpose};
    or_philox4x64(ctr, key, out);
}

/* uniform integer in [0, n) from the high 32 bits of a 64-bit word */
static int64_t index_from_u32(uint32_t u, int64_t n)
{
    return (int64_t)(((uint64_t)u * (uint64_t)n) >> 32);
}

/* Random depth candidate (Sec. 5.1, sampling-propagation): log-uniform on
 * [d_lo, d_hi], one draw per pixel per sweep.  The pixel's coordinate along
 * the sweep axis a (x for horizontal sweeps, dir 0/2; y for vertical ones)
 * and across it b select the Philox block with counter (gsweep, b, a / 8, 0)
 * and its 32-bit word a mod 8, words in the order hi(o0), lo(o0), hi(o1), ...;
 * u = (word + 1/2) 2^-32. */
double or_depth_sample(uint64_t seed, int64_t global_sweep, int dir, int x, int y,
                       double d_lo, double d_hi)
{
    uint64_t o[4];
    const int a = (dir & 1) ? y : x, b = (dir & 1) ? x : y;
    philox_draw(seed, PURPOSE_DEPTH, (uint64_t)global_sweep, (uint64_t)b, (uint64_t)(a / 8), 0, o);
    const int m = a % 8;
    const uint64_t v = o[m / 2];
    const uint32_t word = (m % 2 == 0) ? (uint32_t)(v >> 32) : (uint32_t)v;
    double u = ((double)word + 0.5) * (1.0 / 4294967296.0);
    return exp(log(d_lo) + u * (log(d_hi) - log(d_lo)));
}

/* ------------------------------------------------------------------------ */
/* Fisk (log-logistic) density, Eq. 5, in log form                          */
/*   F(x;a,b) = (b/a)(x/a)^(b-1) / (1 + (x/a)^b)^2                           */
/* ------------------------------------------------------------------------ */
static double log1pexp(double z) { return z > 0 ? z + log1p(exp(-z)) : log1p(exp(z)); }

double or_fisk_logpdf(double x, double log_alpha, double beta)
{
    double lx = log(x) - log_alpha;           /* log(x/alpha) */
    return log(beta) - log_alpha + (beta - 1.0) * lx - 2.0 * log1pexp(beta * lx);
}

/* The Gaussian residual model of the paper's ablations (Sec. 6, Fig. 8):
 * an isotropic two-dimensional Gaussian flow error makes the squared EPE x
 * exponential, density exp(-x/s)/s.  Reading: its mean s is tied to the Fisk
 * scale law A(v) of Eq. 6 by equal medians, s ln 2 = alpha (the Fisk median
 * is alpha), so the same a1, a2 parameterise both models and b1, b2 are
 * unused. */
double or_gauss_logpdf(double x, double log_alpha)
{
    double log_s = log_alpha - log(log(2.0));
    return -x * exp(-log_s) - log_s;
}

/* ------------------------------------------------------------------------ */
/* small dense linear algebra                                               */
/* ------------------------------------------------------------------------ */
static void mat3_mul(const double *A, const double *B, double *C)
{
    double T[9];
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) {
            double s = 0;
            for (int k = 0; k < 3; ++k) s += A[3 * i + k] * B[3 * k + j];
            T[3 * i + j] = s;
        }
    memcpy(C, T, sizeof T);
}
static void mat3_vec(const double *A, const double *x, double *y)
{
    double t[3];
    for (int i = 0; i < 3; ++i) t[i] = A[3 * i] * x[0] + A[3 * i + 1] * x[1] + A[3 * i + 2] * x[2];
    memcpy(y, t, sizeof t);
}
static double dot3(const double *a, const double *b) { return a[0] * b[0] + a[1] * b[1] + a[2] * b[2]; }
static void cross3(const double *a, const double *b, double *c)
{
    double t[3] = {a[1] * b[2] - a[2] * b[1], a[2] * b[0] - a[0] * b[2], a[0] * b[1] - a[1] * b[0]};
    memcpy(c, t, sizeof t);
}
static double norm3(const double *a) { return sqrt(dot3(a, a)); }

/* Cyclic Jacobi eigen-decomposition of a symmetric n x n matrix (row-major).
 * Eigenvalues ascending in w; eigenvectors as COLUMNS of V. */
void or_sym_eig(int n, const double *A_in, double *w, double *V)
{
    double A[81];
    memcpy(A, A_in, sizeof(double) * n * n);
    for (int i = 0; i < n; ++i)
        for (int j = 0; j < n; ++j) V[i * n + j] = (i == j);
    for (int sweep = 0; sweep < 100; ++sweep) {
        double off = 0, tot = 0;
        for (int i = 0; i < n; ++i)
            for (int j = 0; j < n; ++j) {
                tot += A[i * n + j] * A[i * n + j];
                if (i != j) off += A[i * n + j] * A[i * n + j];
            }
        if (off <= 1e-30 * tot || off == 0) break;
        for (int p = 0; p < n - 1; ++p)
            for (int q = p + 1; q < n; ++q) {
                double apq = A[p * n + q];
                if (apq == 0) continue;
                double app = A[p * n + p], aqq = A[q * n + q];
                double tau = (aqq - app) / (2 * apq);
                double t = (tau >= 0 ? 1.0 : -1.0) / (fabs(tau) + sqrt(1 + tau * tau));
                double c = 1 / sqrt(1 + t * t), s = t * c;
                for (int k = 0; k < n; ++k) { /* A <- A J */
                    double akp = A[k * n + p], akq = A[k * n + q];
                    A[k * n + p] = c * akp - s * akq;
                    A[k * n + q] = s * akp + c * akq;
                }
                for (int k = 0; k < n; ++k) { /* A <- J^T A */
                    double apk = A[p * n + k], aqk = A[q * n + k];
                    A[p * n + k] = c * apk - s * aqk;
                    A[q * n + k] = s * apk + c * aqk;
                }
                for (int k = 0; k < n; ++k) {
                    double vkp = V[k * n + p], vkq = V[k * n + q];
                    V[k * n + p] = c * vkp - s * vkq;
                    V[k * n + q] = s * vkp + c * vkq;
                }
            }
    }
    /* sort ascending (selection sort, columns move with values) */
    for (int i = 0; i < n; ++i) w[i] = A[i * n + i];
    for (int i = 0; i < n; ++i) {
        int m = i;
        for (int j = i + 1; j < n; ++j) if (w[j] < w[m]) m = j;
        if (m != i) {
            double tw = w[i]; w[i] = w[m]; w[m] = tw;
            for (int k = 0; k < n; ++k) { double tv = V[k * n + i]; V[k * n + i] = V[k * n + m]; V[k * n + m] = tv; }
        }
    }
}

/* SVD of a 3x3 matrix from the eigen-decomposition of A^T A.
 * Singular values descending; U, V proper rotations with third columns
 * u1 x u2 and v1 x v2 (adequate for the rank-2 essential matrices used here). */
void or_svd3(const double *A, double *U, double *S, double *V)
{
    double AtA[9], w[3], E[9];
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) {
            double s = 0;
            for (int k = 0; k < 3; ++k) s += A[3 * k + i] * A[3 * k + j];
            AtA[3 * i + j] = s;
        }
    or_sym_eig(3, AtA, w, E);
    double v[3][3];
    for (int c = 0; c < 3; ++c) { /* descending */
        int src = 2 - c;
        for (int k = 0; k < 3; ++k) v[c][k] = E[3 * k + src];
        S[c] = sqrt(w[src] > 0 ? w[src] : 0);
    }
    cross3(v[0], v[1], v[2]);
    double u[3][3];
    for (int c = 0; c < 2; ++c) {
        mat3_vec(A, v[c], u[c]);
        double nn = norm3(u[c]);
        for (int k = 0; k < 3; ++k) u[c][k] /= (nn > 0 ? nn : 1);
    }
    /* re-orthogonalise u2 against u1 */
    double d = dot3(u[0], u[1]);
    for (int k = 0; k < 3; ++k) u[1][k] -= d * u[0][k];
    double nn = norm3(u[1]);
    for (int k = 0; k < 3; ++k) u[1][k] /= (nn > 0 ? nn : 1);
    cross3(u[0], u[1], u[2]);
    for (int r = 0; r < 3; ++r)
        for (int c = 0; c < 3; ++c) { U[3 * r + c] = u[c][r]; V[3 * r + c] = v[c][r]; }
}

/* solve 3x3 A x = b by Gaussian elimination with partial pivoting */
static int solve3(const double *A_in, const double *b_in, double *x)
{
    double A[3][4];
    for (int i = 0; i < 3; ++i) { for (int j = 0; j < 3; ++j) A[i][j] = A_in[3 * i + j]; A[i][3] = b_in[i]; }
    for (int c = 0; c < 3; ++c) {
        int p = c;
        for (int r = c + 1; r < 3; ++r) if (fabs(A[r][c]) > fabs(A[p][c])) p = r;
        if (A[p][c] == 0) return 0;
        if (p != c) for (int j = 0; j < 4; ++j) { double t = A[c][j]; A[c][j] = A[p][j]; A[p][j] = t; }
        for (int r = c + 1; r < 3; ++r) {
            double f = A[r][c] / A[c][c];
            for (int j = c; j < 4; ++j) A[r][j] -= f * A[c][j];
        }
    }
    for (int i = 2; i >= 0; --i) {
        double s = A[i][3];
        for (int j = i + 1; j < 3; ++j) s -= A[i][j] * x[j];
        x[i] = s / A[i][i];
    }
    return 1;
}

/* ------------------------------------------------------------------------ */
/* SE(3) exponential / logarithm (se(3) 6-vector ordered (rho, phi))        */
/* ------------------------------------------------------------------------ */
static void hat3(const double *w, double *W)
{
    W[0] = 0;     W[1] = -w[2]; W[2] = w[1];
    W[3] = w[2];  W[4] = 0;     W[5] = -w[0];
    W[6] = -w[1]; W[7] = w[0];  W[8] = 0;
}

/* V(phi) = I + B [phi]x + C [phi]x^2 and R = I + A [phi]x + B [phi]x^2 */
static void se3_RV(const double *phi, double *R, double *V)
{
    double th2 = dot3(phi, phi), th = sqrt(th2), A, B, C;
    if (th < 1e-6) {
        A = 1 - th2 / 6 + th2 * th2 / 120;
        B = 0.5 - th2 / 24 + th2 * th2 / 720;
        C = 1.0 / 6 - th2 / 120 + th2 * th2 / 5040;
    } else {
        A = sin(th) / th;
        B = (1 - cos(th)) / th2;
        C = (th - sin(th)) / (th2 * th);
    }
    double P[9], P2[9];
    hat3(phi, P);
    mat3_mul(P, P, P2);
    for (int i = 0; i < 9; ++i) {
        double I = (i % 4 == 0);
        if (R) R[i] = I + A * P[i] + B * P2[i];
        if (V) V[i] = I + B * P[i] + C * P2[i];
    }
}

void or_se3_exp(const double *p, double *R, double *t)
{
    double V[9];
    se3_RV(p + 3, R, V);
    mat3_vec(V, p, t);
}

/* rotation log: phi with |phi| in [0, pi] */
static void so3_log(const double *R, double *phi)
{
    double w[3] = {R[7] - R[5], R[2] - R[6], R[3] - R[1]};
    double s = 0.5 * norm3(w);
    double c = 0.5 * (R[0] + R[4] + R[8] - 1);
    double th = atan2(s, c);
    if (th < 1e-6) {
        double f = 0.5 * (1 + th * th / 6);
        for (int k = 0; k < 3; ++k) phi[k] = f * w[k];
    } else if (th < M_PI - 1e-3) {
        double f = th / (2 * sin(th));
        for (int k = 0; k < 3; ++k) phi[k] = f * w[k];
    } else {
        /* near pi: R + R^T = 2 cos(th) I + 2 (1 - cos(th)) n n^T */
        double oc = 1 - c, n[3];
        int m = 0;
        double d[3] = {R[0], R[4], R[8]};
        for (int k = 1; k < 3; ++k) if (d[k] > d[m]) m = k;
        n[m] = sqrt(fmax(0.0, (d[m] - c) / oc));
        for (int k = 0; k < 3; ++k)
            if (k != m) n[k] = (R[3 * m + k] + R[3 * k + m]) / (2 * oc * n[m]);
        double nn = norm3(n);
        for (int k = 0; k < 3; ++k) n[k] /= nn;
        if (dot3(n, w) < 0) for (int k = 0; k < 3; ++k) n[k] = -n[k];
        for (int k = 0; k < 3; ++k) phi[k] = th * n[k];
    }
}

void or_se3_log(const double *R, const double *t, double *p)
{
    double V[9];
    so3_log(R, p + 3);
    se3_RV(p + 3, NULL, V);
    if (!solve3(V, t, p)) { p[0] = p[1] = p[2] = NAN; }
}

/* ------------------------------------------------------------------------ */
/* poses: 12 doubles = R row-major (9) + t (3); P_cam = R P + t             */
/* ------------------------------------------------------------------------ */
static void pose_compose(const double *A, const double *B, double *C) /* C = A o B */
{
    double R[9], t[3];
    mat3_mul(A, B, R);
    mat3_vec(A, B + 9, t);
    for (int k = 0; k < 3; ++k) t[k] += A[9 + k];
    memcpy(C, R, sizeof R);
    memcpy(C + 9, t, sizeof t);
}

static void pose_identity(double *P)
{
    memset(P, 0, 12 * sizeof(double));
    P[0] = P[4] = P[8] = 1;
}

/* cumulative M_0 = I, M_t = T_t o M_{t-1} (Eq. 1: product of relative poses) */
static void cumulative(const double *rel, int T, double *M)
{
    pose_identity(M);
    for (int t = 1; t <= T; ++t) pose_compose(rel + 12 * (t - 1), M + 12 * (t - 1), M + 12 * t);
}

/* ------------------------------------------------------------------------ */
/* geometry: projection (Eq. 1), bilinear flow lookup                       */
/* ------------------------------------------------------------------------ */
typedef struct {
    const float *flows;
    int T, H, W;
    double fx, fy, cx, cy;
} or_frame_set;

/* P = M (theta K^-1 [x y 1]^T); returns 0 if the point is not in front. */
static int project(const or_frame_set *F, const double *M, int x, int y, double theta,
                   double *u, double *v)
{
    double r[3] = {(x - F->cx) / F->fx, (y - F->cy) / F->fy, 1.0}, P[3];
    mat3_vec(M, r, P);
    for (int k = 0; k < 3; ++k) P[k] = theta * P[k] + M[9 + k];
    if (!(P[2] > 0)) return 0;
    *u = F->fx * P[0] / P[2] + F->cx;
    *v = F->fy * P[1] / P[2] + F->cy;
    return isfinite(*u) && isfinite(*v);
}

/* Bilinear sample of flow X_t (t = 1..T) at a sub-pixel location of image
 * I_{t-1}.  Domain [0, W-1] x [0, H-1]; all four taps must be finite. */
static int flow_at(const or_frame_set *F, int t, double px, double py, double *fu, double *fv)
{
    if (!(px >= 0 && px <= F->W - 1 && py >= 0 && py <= F->H - 1)) return 0;
    int x0 = (int)floor(px), y0 = (int)floor(py);
    if (x0 > F->W - 2) x0 = F->W - 2;
    if (y0 > F->H - 2) y0 = F->H - 2;
    double ax = px - x0, ay = py - y0;
    const float *X = F->flows + (size_t)(t - 1) * F->H * F->W * 2;
    double wts[4] = {(1 - ax) * (1 - ay), ax * (1 - ay), (1 - ax) * ay, ax * ay};
    int xs[4] = {x0, x0 + 1, x0, x0 + 1}, ys[4] = {y0, y0, y0 + 1, y0 + 1};
    double su = 0, sv = 0;
    for (int k = 0; k < 4; ++k) {
        const float *p = X + ((size_t)ys[k] * F->W + xs[k]) * 2;
        if (!isfinite(p[0]) || !isfinite(p[1])) return 0;
        su += wts[k] * p[0];
        sv += wts[k] * p[1];
    }
    *fu = su;
    *fv = sv;
    return 1;
}

/* test hook: bilinear flow at (px, py) of X_t; returns 0 when missing */
int or_lookup(const float *flows, int T, int H, int W, int t, double px, double py, double *out)
{
    or_frame_set F = {flows, T, H, W, 1, 1, 0, 0};
    return flow_at(&F, t, px, py, out, out + 1);
}

/* ------------------------------------------------------------------------ */
/* emission (Eq. 2, 4-8): for candidate depth theta at pixel (x,y), frame t  */
/* ------------------------------------------------------------------------ */
typedef struct {
    int observed;
    double r;       /* rho / (rho + mu): posterior of W=1 with equal priors  */
    double ell;     /* log r, the MIE term of Eq. 10                          */
    double logrho, logmu;
} or_emis;

/* Test hook: when on, a posterior r below the smallest normal FP32 number
 * (2^-126) is 0.  Where floating point decides the depth M-step's argmax, both
 * sides then take it with the posterior in FP32's range: under the light-tailed
 * Gaussian residual model an outlier observation has r = e^-d with d up to
 * several hundred, and FP64 still orders the depth candidates of pixels that
 * are outliers in every frame by such posteriors, where FP32 holds exact
 * zeros.  Off by default; no other part of the arithmetic changes. */
static int g_f32_range = 0;
void or_set_f32_range(int on) { g_f32_range = on ? 1 : 0; }

static or_emis emission(const or_frame_set *F, const or_params *p, const double *M,
                        int t, int x, int y, double theta)
{
    or_emis e = {0, 0.5, log(0.5), 0, 0};
    double u0, v0, u1, v1, fu, fv;
    if (t == 1) {          /* pi_0 = K theta K^-1 x = x exactly (T_0 = I) */
        if (!(theta > 0)) return e;
        u0 = x;
        v0 = y;
    } else if (!project(F, M + 12 * (t - 1), x, y, theta, &u0, &v0)) return e;
    if (!project(F, M + 12 * t, x, y, theta, &u1, &v1)) return e;
    if (!flow_at(F, t, u0, v0, &fu, &fv)) return e;
    /* rigid flow xi_t = pi_t - pi_{t-1}; residual against observed flow */
    double du = (u1 - u0) - fu, dv = (v1 - v0) - fv;
    double x2 = du * du + dv * dv;
    if (x2 < p->x_floor) x2 = p->x_floor;
    double vn2 = fu * fu + fv * fv, vn = sqrt(vn2);
    double log_alpha = log(p->a1) + p->a2 * vn;          /* Eq. 6 */
    double beta = p->b1 * vn + p->b2;                     /* Eq. 7 */
    if (beta < p->beta_min) beta = p->beta_min;
    double m = p->lambda * p->lambda * vn2;               /* Eq. 8 argument */
    if (m < p->x_floor) m = p->x_floor;
    e.observed = 1;
    if (p->residual_model == 1) {
        e.logrho = or_gauss_logpdf(x2, log_alpha);        /* Eq. 4, Gaussian model */
        e.logmu = or_gauss_logpdf(m, log_alpha);          /* Eq. 8, same density */
    } else {
        e.logrho = or_fisk_logpdf(x2, log_alpha, beta);   /* Eq. 4 */
        e.logmu = or_fisk_logpdf(m, log_alpha, beta);     /* Eq. 8 */
    }
    double d = e.logmu - e.logrho;                        /* log(mu/rho) */
    e.r = 1.0 / (1.0 + exp(d));
    if (g_f32_range && e.r < 1.1754943508222875e-38) e.r = 0.0;
    e.ell = -log1pexp(d);
    return e;
}

/* Dense emission maps for one depth map (test hook). */
void or_emission_map(const double *theta, const float *flows, int T, int H, int W,
                     const double *K, const or_params *p, const double *M,
                     double *r, double *ell, double *logrho, double *logmu, uint8_t *obs)
{
    or_frame_set F = {flows, T, H, W, K[0], K[1], K[2], K[3]};
    for (int t = 1; t <= T; ++t)
        for (int y = 0; y < H; ++y)
            for (int x = 0; x < W; ++x) {
                size_t j = (size_t)y * W + x, o = (size_t)(t - 1) * H * W + j;
                or_emis e = emission(&F, p, M, t, x, y, theta[j]);
                if (r) r[o] = e.r;
                if (ell) ell[o] = e.ell;
                if (logrho) logrho[o] = e.logrho;
                if (logmu) logmu[o] = e.logmu;
                if (obs) obs[o] = (uint8_t)e.observed;
            }
}

/* ------------------------------------------------------------------------ */
/* forward-backward on one chain (Eq. 11-14)                                */
/* r[k] is the normalised emission of state W=1 at chain position k; state  */
/* W=0 has 1-r[k].  Uniform prior at the chain start, unit end message.     */
/* Messages are normalised to sum 1 at every step.                          */
/* ------------------------------------------------------------------------ */
void or_fb_chain(const double *r, int L, double gamma, double *q)
{
    double *f1 = (double *)malloc(sizeof(double) * L * 2);
    double *f0 = f1 + L;
    double p1 = 0.5, p0 = 0.5; /* predicted prior at position 0 */
    for (int k = 0; k < L; ++k) {
        if (k > 0) {
            p1 = gamma * f1[k - 1] + (1 - gamma) * f0[k - 1];
            p0 = (1 - gamma) * f1[k - 1] + gamma * f0[k - 1];
        }
        double a = r[k] * p1, b = (1 - r[k]) * p0, s = a + b;
        f1[k] = a / s;
        f0[k] = b / s;
    }
    double b1 = 0.5, b0 = 0.5; /* m_b at the last position */
    for (int k = L - 1; k >= 0; --k) {
        if (k < L - 1) {
            double e1 = r[k + 1] * b1, e0 = (1 - r[k + 1]) * b0;
            double n1 = gamma * e1 + (1 - gamma) * e0;
            double n0 = (1 - gamma) * e1 + gamma * e0;
            double s = n1 + n0;
            b1 = n1 / s;
            b0 = n0 / s;
        }
        double a = f1[k] * b1, b = f0[k] * b0;
        q[k] = a / (a + b);
    }
    free(f1);
}

/* chain geometry of a sweep direction: 0 L->R, 1 T->B, 2 R->L, 3 B->T */
static int chain_count(int dir, int H, int W) { return (dir & 1) ? W : H; }
static int chain_len(int dir, int H, int W) { return (dir & 1) ? H : W; }
static int chain_pixel(int dir, int H, int W, int c, int k)
{
    switch (dir) {
    case 0: return c * W + k;
    case 1: return k * W + c;
    case 2: return c * W + (W - 1 - k);
    default: return (H - 1 - k) * W + c;
    }
}

/* q for every frame along the chains of one direction (rows for 0/2,
 * columns for 1/3); r is [T][H][W]. */
void or_fb_map(const double *r, int T, int H, int W, int dir, double gamma, double *q)
{
    int L = chain_len(dir, H, W), C = chain_count(dir, H, W);
    double *rc = (double *)malloc(sizeof(double) * L * 2), *qc = rc + L;
    for (int t = 0; t < T; ++t)
        for (int c = 0; c < C; ++c) {
            for (int k = 0; k < L; ++k) rc[k] = r[(size_t)t * H * W + chain_pixel(dir, H, W, c, k)];
            or_fb_chain(rc, L, gamma, qc);
            for (int k = 0; k < L; ++k) q[(size_t)t * H * W + chain_pixel(dir, H, W, c, k)] = qc[k];
        }
    free(rc);
}

/* ------------------------------------------------------------------------ */
/* one directional sweep: E-step (FB on the chains with the current depth)   */
/* then M-step (MIE, Eq. 10) by sampling + propagation along the chain       */
/* (Fig. 5).  q is held fixed during the walk.  Candidates at position k:   */
/* the previous depth, the neighbour's new depth (k>0), a random sample.    */
/* Ties prefer previous, then neighbour, then sample.                       */
/* ------------------------------------------------------------------------ */
/* Term of frame t in the depth M-step objective at a candidate depth, given
 * the E-step's q = q(W_t = 1):
 *   MIE (Eq. 10): q log(rho / (rho + mu)) = q ell; a missing observation has
 *                 ell = log 1/2 (r = 1/2, no evidence either way);
 *   MLE (Eq. 9, the estimator that Eq. 10 relaxes): the expectation over
 *                 W_t of log P(X_t | theta, W_t), q log rho + (1 - q) log mu.
 *                 mu depends on theta through the flow it is evaluated on
 *                 (sampled at pi_{t-1}(theta)), so the W = 0 term stays.  A
 *                 missing observation has no likelihood factor: term 0. */
static double depth_term(const or_params *p, const or_emis *e, double q)
{
    if (p->criterion == 1) return e->observed ? q * e->logrho + (1 - q) * e->logmu : 0.0;
    return q * e->ell;
}

static double mie_score(const or_frame_set *F, const or_params *p, const double *M,
                        const double *q, int x, int y, double theta)
{
    double s = 0;
    size_t j = (size_t)y * F->W + x;
    for (int t = 1; t <= F->T; ++t) {
        or_emis e = emission(F, p, M, t, x, y, theta);
        s += depth_term(p, &e, q[(size_t)(t - 1) * F->H * F->W + j]);
    }
    return s;
}

static double mie_mass(const or_frame_set *F, const or_params *p, const double *M,
                       const double *q, int x, int y, double theta)
{
    double s = 0;
    size_t j = (size_t)y * F->W + x;
    for (int t = 1; t <= F->T; ++t) {
        or_emis e = emission(F, p, M, t, x, y, theta);
        const double qt = q[(size_t)(t - 1) * F->H * F->W + j];
        /* per-item magnitude of the objective's terms (the near-tie scale) */
        s += p->criterion == 1 ? (e.observed ? qt * fabs(e.logrho) + (1 - qt) * fabs(e.logmu) : 0.0)
                               : fabs(qt * e.ell);
    }
    return s;
}

/* test hook: the depth M-step objective sum_t term_t at pixel (x, y) */
double or_depth_score(const double *q, const float *flows, int T, int H, int W, const double *K,
                      const or_params *p, const double *M, int x, int y, double theta)
{
    or_frame_set F = {flows, T, H, W, K[0], K[1], K[2], K[3]};
    return mie_score(&F, p, M, q, x, y, theta);
}

/* theta_in -> theta_out (may alias); q_out [T][H][W] optional;
 * choice_out [H][W] optional: 0 previous, 1 neighbour, 2 sample. */
void or_sweep(const double *theta_in, double *theta_out, const float *flows, int T, int H,
              int W, const double *K, const or_params *p, const double *M, double d_lo,
              double d_hi, int64_t global_sweep, int dir, double *q_out, int8_t *choice_out)
{
    or_frame_set F = {flows, T, H, W, K[0], K[1], K[2], K[3]};
    size_t HW = (size_t)H * W;
    double *r = (double *)malloc(sizeof(double) * HW * T * 2);
    double *q = r + HW * T;
    double *prev = (double *)malloc(sizeof(double) * HW);
    memcpy(prev, theta_in, sizeof(double) * HW);
    for (int t = 1; t <= T; ++t)
        for (int y = 0; y < H; ++y)
            for (int x = 0; x < W; ++x)
                r[(size_t)(t - 1) * HW + (size_t)y * W + x] =
                    emission(&F, p, M, t, x, y, prev[(size_t)y * W + x]).r;
    or_fb_map(r, T, H, W, dir, p->gamma, q);
    int L = chain_len(dir, H, W), C = chain_count(dir, H, W);
    for (int c = 0; c < C; ++c) {
        double carried = 0;
        for (int k = 0; k < L; ++k) {
            int j = chain_pixel(dir, H, W, c, k), x = j % W, y = j / W;
            double s_prev = mie_score(&F, p, M, q, x, y, prev[j]);
            double smp = or_depth_sample(p->seed, global_sweep, dir, x, y, d_lo, d_hi);
            double s_smp = mie_score(&F, p, M, q, x, y, smp);
            double best = prev[j], s_best = s_prev;
            int ch = 0;
            if (k > 0) {
                double s_nbr = mie_score(&F, p, M, q, x, y, carried);
                if (s_nbr > s_best) { best = carried; s_best = s_nbr; ch = 1; }
            }
            if (s_smp > s_best) { best = smp; s_best = s_smp; ch = 2; }
            theta_out[j] = best;
            if (choice_out) choice_out[j] = (int8_t)ch;
            carried = best;
        }
    }
    if (q_out) memcpy(q_out, q, sizeof(double) * HW * T);
    free(prev);
    free(r);
}

/* Validity check of a sweep result produced elsewhere (test hook).
 * For every pixel, the candidate result must be one of {previous depth,
 * the candidate result at the preceding chain position, the random sample}
 * (relative tolerance vtol), and must be the maximum-score choice under the
 * tie rule, up to a near-tie margin: score gap <= stol * sum_t |q ell|.
 * status: 0 exact decision, 1 accepted near tie, 2 wrong value, 3 wrong decision. */
void or_sweep_check(const double *theta_in, const double *theta_cand, const float *flows,
                    int T, int H, int W, const double *K, const or_params *p, const double *M,
                    double d_lo, double d_hi, int64_t global_sweep, int dir, double vtol,
                    double stol, int8_t *status, double *gap_out)
{
    or_frame_set F = {flows, T, H, W, K[0], K[1], K[2], K[3]};
    size_t HW = (size_t)H * W;
    double *r = (double *)malloc(sizeof(double) * HW * T * 2);
    double *q = r + HW * T;
    for (int t = 1; t <= T; ++t)
        for (int y = 0; y < H; ++y)
            for (int x = 0; x < W; ++x)
                r[(size_t)(t - 1) * HW + (size_t)y * W + x] =
                    emission(&F, p, M, t, x, y, theta_in[(size_t)y * W + x]).r;
    or_fb_map(r, T, H, W, dir, p->gamma, q);
    int L = chain_len(dir, H, W), C = chain_count(dir, H, W);
    for (int c = 0; c < C; ++c) {
        for (int k = 0; k < L; ++k) {
            int j = chain_pixel(dir, H, W, c, k), x = j % W, y = j / W;
            double cand[3], sc[3];
            int have[3] = {1, k > 0, 1};
            cand[0] = theta_in[j];
            cand[1] = k > 0 ? theta_cand[chain_pixel(dir, H, W, c, k - 1)] : 0;
            cand[2] = or_depth_sample(p->seed, global_sweep, dir, x, y, d_lo, d_hi);
            double mass = 0;
            for (int i = 0; i < 3; ++i)
                if (have[i]) {
                    sc[i] = mie_score(&F, p, M, q, x, y, cand[i]);
                    double mm = mie_mass(&F, p, M, q, x, y, cand[i]);
                    if (mm > mass) mass = mm;
                }
            int best = 0;
            for (int i = 1; i < 3; ++i)
                if (have[i] && sc[i] > sc[best]) best = i;
            double got = theta_cand[j];
            int which = -1;
            for (int i = 0; i < 3; ++i)
                if (have[i] && fabs(got - cand[i]) <= vtol * fabs(cand[i])) {
                    if (which < 0 || i == best) which = i;
                }
            double gap = 0;
            int8_t st;
            if (which < 0) st = 2;
            else if (which == best) st = 0;
            else {
                gap = sc[best] - sc[which];
                st = (gap <= stol * (mass > 0 ? mass : 1e-300)) ? 1 : 3;
            }
            status[j] = st;
            if (gap_out) gap_out[j] = gap;
        }
    }
    free(r);
}

/* ------------------------------------------------------------------------ */
/* P3P (Grunert's distance formulation as reviewed by Haralick et al. 1994). */
/* 3-D points Pw (3x3, one point per row) and unit bearings f (one per row); */
/* returns up to 4 (R, t) with f_i ~ R Pw_i + t.                              */
/* Quartic in v = s3/s1 built by explicit polynomial arithmetic; real roots  */
/* isolated through the roots of the derivative and refined by bisection.   */
/* ------------------------------------------------------------------------ */
static double poly_eval(const double *c, int n, double x) /* c[0] + c[1] x + ... */
{
    double s = 0;
    for (int i = n; i >= 0; --i) s = s * x + c[i];
    return s;
}

static double bisect(const double *c, int n, double lo, double hi)
{
    double flo = poly_eval(c, n, lo);
    for (int it = 0; it < 200; ++it) {
        double mid = 0.5 * (lo + hi);
        if (mid == lo || mid == hi) break;
        double fm = poly_eval(c, n, mid);
        if (fm == 0) return mid;
        if ((fm < 0) == (flo < 0)) { lo = mid; flo = fm; } else hi = mid;
    }
    return 0.5 * (lo + hi);
}

/* real roots of a degree-n polynomial (n <= 4), ascending */
static int real_roots(const double *c_in, int n, double *roots)
{
    double c[5];
    memcpy(c, c_in, sizeof(double) * (n + 1));
    while (n > 0 && c[n] == 0) --n;
    if (n == 0) return 0;
    if (n == 1) { roots[0] = -c[0] / c[1]; return 1; }
    /* Cauchy bound */
    double bound = 0;
    for (int i = 0; i < n; ++i) bound = fmax(bound, fabs(c[i] / c[n]));
    bound += 1;
    double d[4], crit[4];
    for (int i = 1; i <= n; ++i) d[i - 1] = i * c[i];
    int nc = real_roots(d, n - 1, crit);
    double pts[6];
    int np = 0;
    pts[np++] = -bound;
    for (int i = 0; i < nc; ++i)
        if (crit[i] > -bound && crit[i] < bound) pts[np++] = crit[i];
    pts[np++] = bound;
    int nr = 0;
    for (int i = 0; i + 1 < np; ++i) {
        double a = pts[i], b = pts[i + 1];
        double fa = poly_eval(c, n, a), fb = poly_eval(c, n, b);
        if (fa == 0) { if (nr == 0 || roots[nr - 1] != a) roots[nr++] = a; continue; }
        if ((fa < 0) != (fb < 0)) roots[nr++] = bisect(c, n, a, b);
    }
    double fl = poly_eval(c, n, pts[np - 1]);
    if (fl == 0 && (nr == 0 || roots[nr - 1] != pts[np - 1])) roots[nr++] = pts[np - 1];
    return nr;
}

static void poly_mul(const double *a, int na, const double *b, int nb, double *c)
{
    for (int i = 0; i <= na + nb; ++i) c[i] = 0;
    for (int i = 0; i <= na; ++i)
        for (int j = 0; j <= nb; ++j) c[i + j] += a[i] * b[j];
}

/* rigid transform taking triangle P (rows) onto congruent triangle Q (rows) */
static void triangle_align(const double *P, const double *Q, double *R, double *t)
{
    double FP[9], FQ[9];
    const double *src[2] = {P, Q};
    double *dst[2] = {FP, FQ};
    for (int s = 0; s < 2; ++s) {
        const double *X = src[s];
        double e1[3], e2[3], e3[3], d2[3];
        for (int k = 0; k < 3; ++k) { e1[k] = X[3 + k] - X[k]; d2[k] = X[6 + k] - X[k]; }
        double n1 = norm3(e1);
        for (int k = 0; k < 3; ++k) e1[k] /= n1;
        cross3(e1, d2, e3);
        double n3 = norm3(e3);
        for (int k = 0; k < 3; ++k) e3[k] /= n3;
        cross3(e3, e1, e2);
        for (int k = 0; k < 3; ++k) { dst[s][3 * k] = e1[k]; dst[s][3 * k + 1] = e2[k]; dst[s][3 * k + 2] = e3[k]; }
    }
    /* R = FQ FP^T */
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) {
            double s = 0;
            for (int k = 0; k < 3; ++k) s += FQ[3 * i + k] * FP[3 * j + k];
            R[3 * i + j] = s;
        }
    double rp[3];
    mat3_vec(R, P, rp);
    for (int k = 0; k < 3; ++k) t[k] = Q[k] - rp[k];
}

/* Newton's method on the three law-of-cosines equations of P3P,
 *   s2^2 + s3^2 - 2 s2 s3 ca = a2,  s1^2 + s3^2 - 2 s1 s3 cb = b2,
 *   s1^2 + s2^2 - 2 s1 s2 cg = c2,
 * from the distances one root of the quartic gives.  Where two solutions
 * share (nearly) one value of v the quartic has a (near) double root, which
 * a root finder resolves only to about half the digits; the distances are
 * then brought to the solution of the equations themselves.  A step is kept
 * only while it lowers the residual. */
static void p3p_refine(double *s, double a2, double b2, double c2, double ca, double cb, double cg)
{
    double F[3], r0 = 0;
    for (int it = 0; it < 8; ++it) {
        F[0] = s[1] * s[1] + s[2] * s[2] - 2 * s[1] * s[2] * ca - a2;
        F[1] = s[0] * s[0] + s[2] * s[2] - 2 * s[0] * s[2] * cb - b2;
        F[2] = s[0] * s[0] + s[1] * s[1] - 2 * s[0] * s[1] * cg - c2;
        double r = fabs(F[0]) + fabs(F[1]) + fabs(F[2]);
        if (it == 0) r0 = r;
        if (r == 0) return;
        double J[9] = {0, 2 * (s[1] - s[2] * ca), 2 * (s[2] - s[1] * ca),
                       2 * (s[0] - s[2] * cb), 0, 2 * (s[2] - s[0] * cb),
                       2 * (s[0] - s[1] * cg), 2 * (s[1] - s[0] * cg), 0};
        double mF[3] = {-F[0], -F[1], -F[2]}, d[3];
        if (!solve3(J, mF, d)) return;
        double sn[3] = {s[0] + d[0], s[1] + d[1], s[2] + d[2]};
        double G0 = sn[1] * sn[1] + sn[2] * sn[2] - 2 * sn[1] * sn[2] * ca - a2;
        double G1 = sn[0] * sn[0] + sn[2] * sn[2] - 2 * sn[0] * sn[2] * cb - b2;
        double G2 = sn[0] * sn[0] + sn[1] * sn[1] - 2 * sn[0] * sn[1] * cg - c2;
        double rn = fabs(G0) + fabs(G1) + fabs(G2);
        if (!(rn < r) || !(sn[0] > 0 && sn[1] > 0 && sn[2] > 0)) return;
        s[0] = sn[0];
        s[1] = sn[1];
        s[2] = sn[2];
        if (fabs(d[0]) + fabs(d[1]) + fabs(d[2]) <= 1e-16 * (s[0] + s[1] + s[2])) return;
    }
    (void)r0;
}

int or_p3p(const double *Pw, const double *f_in, double *Rs, double *ts)
{
    double f[9];
    for (int i = 0; i < 3; ++i) {
        double n = norm3(f_in + 3 * i);
        for (int k = 0; k < 3; ++k) f[3 * i + k] = f_in[3 * i + k] / n;
    }
    double d23[3], d13[3], d12[3];
    for (int k = 0; k < 3; ++k) {
        d23[k] = Pw[3 + k] - Pw[6 + k];
        d13[k] = Pw[k] - Pw[6 + k];
        d12[k] = Pw[k] - Pw[3 + k];
    }
    double a2 = dot3(d23, d23), b2 = dot3(d13, d13), c2 = dot3(d12, d12);
    double ca = dot3(f + 3, f + 6), cb = dot3(f, f + 6), cg = dot3(f, f + 3);
    if (!(b2 > 0) || !(a2 > 0) || !(c2 > 0)) return 0;
    /* Q(v) = 1 + v^2 - 2 v cb ; N(v) = b2 (v^2 - 1) + (c2 - a2) Q(v) ; D(v) = 2 b2 (v ca - cg) */
    double Qp[3] = {1, -2 * cb, 1};
    double Np[3] = {-b2 + (c2 - a2), (c2 - a2) * (-2 * cb), b2 + (c2 - a2)};
    double Dp[2] = {-2 * b2 * cg, 2 * b2 * ca};
    /* b2 N^2 - 2 b2 cg N D + (b2 - c2 Q) D^2 = 0 */
    double N2[5], ND[4], D2[3], QD2[5], quart[5];
    poly_mul(Np, 2, Np, 2, N2);
    poly_mul(Np, 2, Dp, 1, ND);
    poly_mul(Dp, 1, Dp, 1, D2);
    double BQ[3] = {b2 - c2 * Qp[0], -c2 * Qp[1], -c2 * Qp[2]};
    poly_mul(BQ, 2, D2, 2, QD2);
    for (int i = 0; i <= 4; ++i) {
        quart[i] = b2 * N2[i] + QD2[i];
        if (i <= 3) quart[i] += -2 * b2 * cg * ND[i];
    }
    double roots[4];
    int nr = real_roots(quart, 4, roots);
    int n = 0;
    for (int i = 0; i < nr; ++i) {
        double v = roots[i];
        double D = poly_eval(Dp, 1, v), Q = poly_eval(Qp, 2, v);
        if (!(v > 0) || fabs(D) < 1e-14 * b2 || !(Q > 0)) continue;
        double u = poly_eval(Np, 2, v) / D;
        if (!(u > 0)) continue;
        double sd[3] = {sqrt(b2 / Q), 0, 0};
        sd[1] = u * sd[0];
        sd[2] = v * sd[0];
        p3p_refine(sd, a2, b2, c2, ca, cb, cg);
        double s1 = sd[0], s2 = sd[1], s3 = sd[2];
        double Qc[9];
        for (int k = 0; k < 3; ++k) { Qc[k] = s1 * f[k]; Qc[3 + k] = s2 * f[3 + k]; Qc[6 + k] = s3 * f[6 + k]; }
        double R[9], t[3];
        triangle_align(Pw, Qc, R, t);
        int ok = 1;
        for (int k = 0; k < 9; ++k) ok &= isfinite(R[k]);
        for (int k = 0; k < 3; ++k) ok &= isfinite(t[k]);
        if (!ok) continue;
        memcpy(Rs + 9 * n, R, sizeof R);
        memcpy(ts + 3 * n, t, sizeof t);
        ++n;
    }
    return n;
}

/* ------------------------------------------------------------------------ */
/* mean-shift in se(3) with Gaussian kernel exp(-d^2/2),                     */
/* d^2 = (p-q)^T Sigma^-1 (p-q), Sigma = diag(s2t I3, s2r I3) (Eq. 18-19)   */
/* ------------------------------------------------------------------------ */
static double mdist2(const double *a, const double *b, double s2t, double s2r)
{
    double d = 0;
    for (int k = 0; k < 3; ++k) d += (a[k] - b[k]) * (a[k] - b[k]) / s2t;
    for (int k = 3; k < 6; ++k) d += (a[k] - b[k]) * (a[k] - b[k]) / s2r;
    return d;
}

double or_kde(const double *samples, const double *w, int n, const double *at, double s2t, double s2r)
{
    double s = 0;
    for (int i = 0; i < n; ++i) s += w[i] * exp(-0.5 * mdist2(at, samples + 6 * i, s2t, s2r));
    return s;
}

int or_meanshift(const double *samples, const double *w, int n, const double *start,
                 double s2t, double s2r, double tol, int max_iters, double *out)
{
    double p[6];
    memcpy(p, start, sizeof p);
    int it = 0;
    for (; it < max_iters; ++it) {
        double num[6] = {0, 0, 0, 0, 0, 0}, den = 0;
        for (int i = 0; i < n; ++i) {
            double k = w[i] * exp(-0.5 * mdist2(p, samples + 6 * i, s2t, s2r));
            den += k;
            for (int c = 0; c < 6; ++c) num[c] += k * samples[6 * i + c];
        }
        if (!(den > 0)) break;
        double np_[6];
        for (int c = 0; c < 6; ++c) np_[c] = num[c] / den;
        double step = sqrt(mdist2(np_, p, s2t, s2r));
        memcpy(p, np_, sizeof p);
        if (step < tol) { ++it; break; }
    }
    memcpy(out, p, sizeof p);
    return it;
}

/* ------------------------------------------------------------------------ */
/* pose step for frame t (Sec. 5.2)                                          */
/* ------------------------------------------------------------------------ */
static double rot_angle(const double *R)
{
    double w[3] = {R[7] - R[5], R[2] - R[6], R[3] - R[1]};
    return atan2(0.5 * norm3(w), 0.5 * (R[0] + R[4] + R[8] - 1));
}

typedef struct {
    int n_samples, n_valid_groups, ms_iters, fallback;
} or_pose_diag;

/* Draw group g's three pixels (all distinct); returns 0 if 8 attempts fail. */
static int pose_group_pixels(uint64_t seed, int it, int t, int g, int64_t HW, int64_t *j)
{
    for (int a = 0; a < 8; ++a) {
        uint64_t o[4];
        philox_draw(seed, PURPOSE_POSE, (uint64_t)it, (uint64_t)t, (uint64_t)g, (uint64_t)a, o);
        for (int k = 0; k < 3; ++k) j[k] = index_from_u32((uint32_t)(o[k] >> 32), HW);
        if (j[0] != j[1] && j[0] != j[2] && j[1] != j[2]) return 1;
    }
    return 0;
}

/* theta [H][W]; Wmap [T][H][W] or NULL (all ones); M cumulative [T+1][12]
 * (M[t-1] used); prevT [12] or NULL; T_out [12].
 * samples_out optional [4S][8]: p(6), w, valid. */
/* All-pixel score of a candidate relative pose Tc of frame t: the sum over
 * every pixel j of W_t^j ell_t^j(theta_j) with M_t = Tc o M_{t-1} (W = 1 when
 * no rigidness is given; a missing item has ell = log 1/2, as in Eq. 10's
 * criterion).  Mtmp: scratch of T+1 poses. */
static double allpix_score(const or_frame_set *F, const or_params *p, const double *M, int t,
                           const double *theta, const double *Wmap, const double *Tc, double *Mtmp)
{
    memcpy(Mtmp, M, sizeof(double) * 12 * t);
    pose_compose(Tc, M + 12 * (t - 1), Mtmp + 12 * t);
    const int64_t HW = (int64_t)F->H * F->W;
    double s = 0;
    for (int y = 0; y < F->H; ++y)
        for (int x = 0; x < F->W; ++x) {
            const int64_t j = (int64_t)y * F->W + x;
            const or_emis e = emission(F, p, Mtmp, t, x, y, theta[j]);
            s += (Wmap ? Wmap[(int64_t)(t - 1) * HW + j] : 1.0) * e.ell;
        }
    return s;
}

static int pose_step_core(const double *theta, const double *Wmap, const float *flows, int T, int H,
                          int W, const double *K, const or_params *p, const double *M, int t, int it,
                          const double *prevT, double *T_out, double *samples_out, int *diag,
                          double *scores_out, int *n_scores);

int or_pose_step(const double *theta, const double *Wmap, const float *flows, int T, int H,
                 int W, const double *K, const or_params *p, const double *M, int t, int it,
                 const double *prevT, double *T_out, double *samples_out, int *diag)
{
    return pose_step_core(theta, Wmap, flows, T, H, W, K, p, M, t, it, prevT, T_out, samples_out, diag,
                          NULL, NULL);
}

/* test hook: the pose step with p->pose_start = 1, also returning the
 * all-pixel scores: [0] the previous pose (-inf if none), [1..n] the valid
 * samples in (group, root) order; *n_scores = 1 + n. */
int or_pose_step_scores(const double *theta, const double *Wmap, const float *flows, int T, int H,
                        int W, const double *K, const or_params *p, const double *M, int t, int it,
                        const double *prevT, double *T_out, double *scores_out, int *n_scores)
{
    return pose_step_core(theta, Wmap, flows, T, H, W, K, p, M, t, it, prevT, T_out, NULL, NULL,
                          scores_out, n_scores);
}

static int pose_step_core(const double *theta, const double *Wmap, const float *flows, int T, int H,
                          int W, const double *K, const or_params *p, const double *M, int t, int it,
                          const double *prevT, double *T_out, double *samples_out, int *diag,
                          double *scores_out, int *n_scores)
{
    or_frame_set F = {flows, T, H, W, K[0], K[1], K[2], K[3]};
    int S = p->n_pose_groups;
    int64_t HW = (int64_t)H * W;
    double *smp = (double *)malloc(sizeof(double) * 6 * 4 * S);
    double *wts = (double *)malloc(sizeof(double) * 4 * S);
    int n = 0, nvalid = 0;
    const double *Mp = M + 12 * (t - 1);
    if (samples_out) memset(samples_out, 0, sizeof(double) * 8 * 4 * S);
    for (int g = 0; g < S; ++g) {
        int64_t j[3];
        if (!pose_group_pixels(p->seed, it, t, g, HW, j)) continue;
        double Pw[9], fb[9], wgt = 1;
        int ok = 1;
        for (int k = 0; k < 3 && ok; ++k) {
            int x = (int)(j[k] % W), y = (int)(j[k] / W);
            double th = theta[j[k]];
            double r[3] = {(x - F.cx) / F.fx, (y - F.cy) / F.fy, 1.0}, P[3];
            mat3_vec(Mp, r, P);
            for (int c = 0; c < 3; ++c) P[c] = th * P[c] + Mp[9 + c];
            if (!(P[2] > 0)) { ok = 0; break; }
            double u0 = F.fx * P[0] / P[2] + F.cx, v0 = F.fy * P[1] / P[2] + F.cy, fu, fv;
            if (t == 1) { u0 = x; v0 = y; }   /* pi_0 is the pixel itself */
            if (!flow_at(&F, t, u0, v0, &fu, &fv)) { ok = 0; break; }
            double yx = u0 + fu, yy = v0 + fv;
            double b[3] = {(yx - F.cx) / F.fx, (yy - F.cy) / F.fy, 1.0};
            double nb = norm3(b);
            for (int c = 0; c < 3; ++c) { Pw[3 * k + c] = P[c]; fb[3 * k + c] = b[c] / nb; }
            if (Wmap) wgt *= Wmap[(size_t)(t - 1) * HW + j[k]];
        }
        if (!ok) continue;
        ++nvalid;
        double Rs[36], ts[12];
        int nr = or_p3p(Pw, fb, Rs, ts);
        /* keep roots with all three points in front of camera t */
        int keep[4], nk = 0;
        for (int i = 0; i < nr; ++i) {
            int front = 1;
            for (int k = 0; k < 3; ++k) {
                double z = Rs[9 * i + 6] * Pw[3 * k] + Rs[9 * i + 7] * Pw[3 * k + 1] +
                           Rs[9 * i + 8] * Pw[3 * k + 2] + ts[3 * i + 2];
                front &= z > 0;
            }
            if (front) keep[nk++] = i;
        }
        /* canonical order: rotation angle, then t_x, t_y, t_z */
        for (int a = 0; a < nk; ++a)
            for (int b = a + 1; b < nk; ++b) {
                int ia = keep[a], ib = keep[b];
                double ka[4] = {rot_angle(Rs + 9 * ia), ts[3 * ia], ts[3 * ia + 1], ts[3 * ia + 2]};
                double kb[4] = {rot_angle(Rs + 9 * ib), ts[3 * ib], ts[3 * ib + 1], ts[3 * ib + 2]};
                int less = 0;
                for (int c = 0; c < 4; ++c) {
                    if (kb[c] < ka[c]) { less = 1; break; }
                    if (kb[c] > ka[c]) break;
                }
                if (less) { keep[a] = ib; keep[b] = ia; }
            }
        int slot = 0; /* valid samples fill the group's slots without gaps */
        for (int a = 0; a < nk; ++a) {
            int i = keep[a];
            double pv[6];
            or_se3_log(Rs + 9 * i, ts + 3 * i, pv);
            int fin = 1;
            for (int c = 0; c < 6; ++c) fin &= isfinite(pv[c]);
            if (!fin) continue;
            memcpy(smp + 6 * n, pv, sizeof pv);
            wts[n] = wgt;
            if (samples_out) {
                double *so = samples_out + 8 * (4 * g + slot);
                memcpy(so, pv, sizeof pv);
                so[6] = wgt;
                so[7] = 1;
            }
            ++slot;
            ++n;
        }
    }
    double wsum = 0;
    for (int i = 0; i < n; ++i) wsum += wts[i];
    int ms_iters = 0, fallback = 0;
    if (scores_out) {
        /* every candidate's all-pixel score, whether or not the step uses it */
        double *Mtmp = (double *)malloc(sizeof(double) * 12 * (t + 1));
        scores_out[0] = prevT ? allpix_score(&F, p, M, t, theta, Wmap, prevT, Mtmp) : -INFINITY;
        for (int i = 0; i < n; ++i) {
            double Tc[12];
            or_se3_exp(smp + 6 * i, Tc, Tc + 9);
            scores_out[1 + i] = allpix_score(&F, p, M, t, theta, Wmap, Tc, Mtmp);
        }
        free(Mtmp);
        if (n_scores) *n_scores = 1 + n;
    }
    if (n == 0 || !(wsum > 0)) {
        fallback = 1;
        if (prevT) memcpy(T_out, prevT, 12 * sizeof(double));
        else pose_identity(T_out);
    } else {
        /* start: the candidate of highest kernel density among the previous
         * pose (if any) and the first n_seeds samples in (group, root) order */
        double best_p[6], best_d = -1;
        int have = 0;
        if (p->pose_start == 1) {
            /* the literal reading of scoring every hypothesis over all pixels:
             * the start is the candidate (previous pose first, then every
             * sample in (group, root) order) of highest all-pixel score, the
             * first on ties */
            double *Mtmp = (double *)malloc(sizeof(double) * 12 * (t + 1));
            if (prevT) {
                or_se3_log(prevT, prevT + 9, best_p);
                best_d = allpix_score(&F, p, M, t, theta, Wmap, prevT, Mtmp);
                have = 1;
            }
            for (int i = 0; i < n; ++i) {
                double Tc[12];
                or_se3_exp(smp + 6 * i, Tc, Tc + 9);
                const double dd = allpix_score(&F, p, M, t, theta, Wmap, Tc, Mtmp);
                if (!have || dd > best_d) { best_d = dd; memcpy(best_p, smp + 6 * i, sizeof best_p); have = 1; }
            }
            free(Mtmp);
        } else if (prevT) {
            double pp[6];
            or_se3_log(prevT, prevT + 9, pp);
            double dd = or_kde(smp, wts, n, pp, p->sigma2_trans, p->sigma2_rot);
            memcpy(best_p, pp, sizeof pp);
            best_d = dd;
            have = 1;
        }
        int ns = p->pose_start == 1 ? 0 : (n < p->n_seeds ? n : p->n_seeds);
        for (int i = 0; i < ns; ++i) {
            double dd = or_kde(smp, wts, n, smp + 6 * i, p->sigma2_trans, p->sigma2_rot);
            if (!have || dd > best_d) { best_d = dd; memcpy(best_p, smp + 6 * i, sizeof best_p); have = 1; }
        }
        double mode[6];
        ms_iters = or_meanshift(smp, wts, n, best_p, p->sigma2_trans, p->sigma2_rot, p->ms_tol,
                                p->ms_max_iters, mode);
        or_se3_exp(mode, T_out, T_out + 9);
    }
    if (diag) { diag[0] = n; diag[1] = nvalid; diag[2] = ms_iters; diag[3] = fallback; }
    free(smp);
    free(wts);
    return OR_OK;
}

/* ------------------------------------------------------------------------ */
/* bootstrap (Sec. 5.3, Table 1): T_1 by least-median-of-squares over       */
/* 8-point essential-matrix hypotheses from X_1, depth by triangulation      */
/* ------------------------------------------------------------------------ */
static int present(const float *X1, int64_t j)
{
    return isfinite(X1[2 * j]) && isfinite(X1[2 * j + 1]);
}

static int cmp_double(const void *a, const void *b)
{
    double x = *(const double *)a, y = *(const double *)b;
    return x < y ? -1 : x > y;
}

/* Unit null vector of the 8x9 epipolar system (rows of A): with exactly eight
 * correspondences the least-squares solution of the 8-point method is the
 * null vector of A.  It is the last column of Q in the Householder QR
 * factorisation A^T = Q R (9x9 Q). */
void or_null_vector_8x9(const double *A, double *e)
{
    double M[9][8], V[8][9], beta[8];
    for (int i = 0; i < 9; ++i)
        for (int k = 0; k < 8; ++k) M[i][k] = A[9 * k + i];
    for (int k = 0; k < 8; ++k) {
        double nrm = 0;
        for (int i = k; i < 9; ++i) nrm += M[i][k] * M[i][k];
        nrm = sqrt(nrm);
        double alpha = M[k][k] > 0 ? -nrm : nrm;
        double vn = 0;
        for (int i = 0; i < 9; ++i) V[k][i] = i < k ? 0 : M[i][k];
        V[k][k] -= alpha;
        for (int i = k; i < 9; ++i) vn += V[k][i] * V[k][i];
        beta[k] = vn > 0 ? 2.0 / vn : 0.0;
        for (int j = k; j < 8; ++j) {
            double s = 0;
            for (int i = k; i < 9; ++i) s += V[k][i] * M[i][j];
            for (int i = k; i < 9; ++i) M[i][j] -= beta[k] * s * V[k][i];
        }
    }
    for (int i = 0; i < 9; ++i) e[i] = (i == 8);
    for (int k = 7; k >= 0; --k) {   /* Q e_9 = H_0 H_1 ... H_7 e_9 */
        double s = 0;
        for (int i = k; i < 9; ++i) s += V[k][i] * e[i];
        for (int i = k; i < 9; ++i) e[i] -= beta[k] * s * V[k][i];
    }
    double n = 0;
    for (int i = 0; i < 9; ++i) n += e[i] * e[i];
    n = sqrt(n);
    for (int i = 0; i < 9; ++i) e[i] /= n;
}

/* triangulated z-depth along the frame-0 ray from relative pose (R, t) */
static double triangulate(const double *R, const double *t, double xn, double yn, double bx,
                          double by, int *ok)
{
    double r[3] = {xn, yn, 1}, a[3];
    mat3_vec(R, r, a);
    double c0 = a[0] - bx * a[2], c1 = a[1] - by * a[2];
    double e0 = t[0] - bx * t[2], e1 = t[1] - by * t[2];
    double cc = c0 * c0 + c1 * c1;
    double th = -(c0 * e0 + c1 * e1) / cc;
    *ok = cc >= 1e-12 && th > 0 && isfinite(th);
    return th;
}

/* relT_out [12]; theta_out [H][W]; range_out [2] = d_lo, d_hi;
 * info_out optional [4]: best hypothesis, its median, valid pixels, cheirality count */
static int depth_from_T1(const float *X1, int H, int W, const double *K, const or_params *p,
                         const double *R1, const double *t1, double *theta_out, double *range_out, double *nv_out);

int or_bootstrap(const float *flows, int T, int H, int W, const double *K, const or_params *p,
                 double *relT_out, double *theta_out, double *range_out, double *info_out)
{
    (void)T;
    int64_t HW = (int64_t)H * W;
    const float *X1 = flows;
    double fx = K[0], fy = K[1], cx = K[2], cy = K[3];
    int64_t n_present = 0;
    for (int64_t j = 0; j < HW; ++j) n_present += present(X1, j);
    if (n_present < 8) return OR_EDEGENERATE;
    /* evaluation subset: pixels floor(i HW / Ne), i < Ne, that are present */
    int64_t Ne = p->lmeds_eval_pixels < HW ? p->lmeds_eval_pixels : HW;
    int64_t *ev = (int64_t *)malloc(sizeof(int64_t) * Ne);
    int64_t nev = 0;
    for (int64_t i = 0; i < Ne; ++i) {
        int64_t j = (i * HW) / Ne;
        if (present(X1, j)) ev[nev++] = j;
    }
    if (nev < 8) { free(ev); return OR_EDEGENERATE; }
    double *res = (double *)malloc(sizeof(double) * nev);
    int M = p->lmeds_hypotheses;
    double best_score = INFINITY, bestE[9];
    int best_h = -1;
    for (int h = 0; h < M; ++h) {
        int64_t idx[8];
        int got = 0;
        for (int a = 0; a < 16 && !got; ++a) {
            uint64_t o[4];
            philox_draw(p->seed, PURPOSE_BOOT, (uint64_t)h, (uint64_t)a, 0, 0, o);
            got = 1;
            for (int k = 0; k < 8; ++k) {
                uint32_t u = (k & 1) ? (uint32_t)(o[k >> 1] >> 32) : (uint32_t)o[k >> 1];
                idx[k] = index_from_u32(u, HW);
                if (!present(X1, idx[k])) got = 0;
                for (int m = 0; m < k; ++m) if (idx[m] == idx[k]) got = 0;
            }
        }
        if (!got) continue;
        /* 8-point system b^T E a = 0 in normalised coordinates */
        double A[72];
        for (int k = 0; k < 8; ++k) {
            int x = (int)(idx[k] % W), y = (int)(idx[k] / W);
            double a[3] = {(x - cx) / fx, (y - cy) / fy, 1};
            double b[3] = {(x + (double)X1[2 * idx[k]] - cx) / fx, (y + (double)X1[2 * idx[k] + 1] - cy) / fy, 1};
            for (int i = 0; i < 3; ++i)
                for (int l = 0; l < 3; ++l) A[9 * k + 3 * i + l] = b[i] * a[l];
        }
        double E0[9], U[9], Sg[3], Vv[9], E[9];
        or_null_vector_8x9(A, E0);
        /* projection onto the essential manifold: U diag(1,1,0) V^T */
        or_svd3(E0, U, Sg, Vv);
        for (int i = 0; i < 3; ++i)
            for (int l = 0; l < 3; ++l) E[3 * i + l] = U[3 * i] * Vv[3 * l] + U[3 * i + 1] * Vv[3 * l + 1];
        /* F = K^-T E K^-1 ; Sampson distance^2 in pixels */
        double Ki[9] = {1 / fx, 0, -cx / fx, 0, 1 / fy, -cy / fy, 0, 0, 1}, KiT[9], Fm[9];
        for (int i = 0; i < 3; ++i) for (int l = 0; l < 3; ++l) KiT[3 * i + l] = Ki[3 * l + i];
        mat3_mul(KiT, E, Fm);
        mat3_mul(Fm, Ki, Fm);
        for (int64_t i = 0; i < nev; ++i) {
            int64_t j = ev[i];
            int x = (int)(j % W), y = (int)(j / W);
            double x1[3] = {x, y, 1}, x2[3] = {x + (double)X1[2 * j], y + (double)X1[2 * j + 1], 1}, Fx[3], Ftx[3];
            mat3_vec(Fm, x1, Fx);
            for (int c = 0; c < 3; ++c) Ftx[c] = Fm[c] * x2[0] + Fm[3 + c] * x2[1] + Fm[6 + c] * x2[2];
            double e = dot3(x2, Fx);
            res[i] = e * e / (Fx[0] * Fx[0] + Fx[1] * Fx[1] + Ftx[0] * Ftx[0] + Ftx[1] * Ftx[1]);
        }
        qsort(res, nev, sizeof(double), cmp_double);
        double med = res[(nev - 1) / 2];
        if (isfinite(med) && med < best_score) { best_score = med; best_h = h; memcpy(bestE, E, sizeof E); }
    }
    if (best_h < 0) { free(ev); free(res); return OR_EDEGENERATE; }
    /* decomposition into (R, +-t) pairs; cheirality vote over the subset */
    double U[9], Sg[3], Vv[9];
    or_svd3(bestE, U, Sg, Vv);
    double Wm[9] = {0, -1, 0, 1, 0, 0, 0, 0, 1}, WmT[9] = {0, 1, 0, -1, 0, 0, 0, 0, 1}, VT[9];
    for (int i = 0; i < 3; ++i) for (int l = 0; l < 3; ++l) VT[3 * i + l] = Vv[3 * l + i];
    double Rc[2][9], tc[3] = {U[2], U[5], U[8]};
    mat3_mul(U, Wm, Rc[0]);
    mat3_mul(Rc[0], VT, Rc[0]);
    mat3_mul(U, WmT, Rc[1]);
    mat3_mul(Rc[1], VT, Rc[1]);
    int best_c = -1, best_cnt = -1;
    for (int c = 0; c < 4; ++c) {
        const double *R = Rc[c >> 1];
        double t[3], sg = (c & 1) ? -1 : 1;
        for (int k = 0; k < 3; ++k) t[k] = sg * tc[k];
        int cnt = 0;
        for (int64_t i = 0; i < nev; ++i) {
            int64_t j = ev[i];
            int x = (int)(j % W), y = (int)(j / W), ok;
            double xn = (x - cx) / fx, yn = (y - cy) / fy;
            double bx = (x + (double)X1[2 * j] - cx) / fx, by = (y + (double)X1[2 * j + 1] - cy) / fy;
            double th = triangulate(R, t, xn, yn, bx, by, &ok);
            if (!ok) continue;
            double r[3] = {xn, yn, 1}, P[3];
            mat3_vec(R, r, P);
            if (th * P[2] + t[2] > 0) ++cnt;
        }
        if (cnt > best_cnt) { best_cnt = cnt; best_c = c; }
    }
    double R1[9], t1[3], sg = (best_c & 1) ? -1 : 1;
    memcpy(R1, Rc[best_c >> 1], sizeof R1);
    for (int k = 0; k < 3; ++k) t1[k] = sg * tc[k];
    double tn = norm3(t1);
    for (int k = 0; k < 3; ++k) t1[k] /= tn;
    memcpy(relT_out, R1, sizeof R1);
    memcpy(relT_out + 9, t1, sizeof t1);
    double nvd = 0;
    const int st = depth_from_T1(X1, H, W, K, p, R1, t1, theta_out, range_out, &nvd);
    if (info_out) { info_out[0] = best_h; info_out[1] = best_score; info_out[2] = nvd; info_out[3] = best_cnt; }
    free(ev); free(res);
    return st;
}

/* Depth of frame 0 by two-view triangulation from T_1 = (R1, t1) and X_1
 * (Table 1, third row): every pixel with a present flow; the sampling range
 * [d_lo, d_hi] = [P1 / 2, 2 P99] of the valid depths (unless fixed by p);
 * invalid pixels take the median, and all depths are clamped to the range. */
static int depth_from_T1(const float *X1, int H, int W, const double *K, const or_params *p,
                         const double *R1, const double *t1, double *theta_out, double *range_out, double *nv_out)
{
    int64_t HW = (int64_t)H * W;
    double fx = K[0], fy = K[1], cx = K[2], cy = K[3];
    /* triangulation of every pixel; percentiles of the valid depths */
    double *vals = (double *)malloc(sizeof(double) * HW);
    uint8_t *val = (uint8_t *)malloc(HW);
    int64_t nv = 0;
    for (int64_t j = 0; j < HW; ++j) {
        int x = (int)(j % W), y = (int)(j / W), ok = 0;
        double th = 0;
        if (present(X1, j))
            th = triangulate(R1, t1, (x - cx) / fx, (y - cy) / fy, (x + (double)X1[2 * j] - cx) / fx,
                             (y + (double)X1[2 * j + 1] - cy) / fy, &ok);
        val[j] = (uint8_t)ok;
        theta_out[j] = th;
        if (ok) vals[nv++] = th;
    }
    *nv_out = (double)nv;
    if (nv == 0) { free(vals); free(val); return OR_EDEGENERATE; }
    qsort(vals, nv, sizeof(double), cmp_double);
    double P1 = vals[(int64_t)floor(0.01 * (nv - 1))], P50 = vals[(int64_t)floor(0.50 * (nv - 1))],
           P99 = vals[(int64_t)floor(0.99 * (nv - 1))];
    double d_lo = p->depth_lo > 0 ? p->depth_lo : 0.5 * P1;
    double d_hi = p->depth_hi > 0 ? p->depth_hi : 2.0 * P99;
    for (int64_t j = 0; j < HW; ++j) {
        double th = val[j] ? theta_out[j] : P50;
        if (th < d_lo) th = d_lo;
        if (th > d_hi) th = d_hi;
        theta_out[j] = th;
    }
    range_out[0] = d_lo;
    range_out[1] = d_hi;
    free(vals); free(val);
    return OR_OK;
}

/* The bootstrap with T_1 given instead of estimated: the paper's alternative
 * for overlapping consecutive batches (Sec. 5.3), T_1 from the previous
 * window's estimate.  Its translation is rescaled to unit length (the gauge);
 * the depth follows by triangulation as above.  A zero translation is
 * degenerate. */
int or_bootstrap_seeded(const float *flows, int T, int H, int W, const double *K, const or_params *p,
                        const double *T1, double *relT_out, double *theta_out, double *range_out)
{
    (void)T;
    const double tn = norm3(T1 + 9);
    if (!(tn > 0) || !isfinite(tn)) return OR_EDEGENERATE;
    double R1[9], t1[3];
    memcpy(R1, T1, sizeof R1);
    for (int k = 0; k < 3; ++k) t1[k] = T1[9 + k] / tn;
    memcpy(relT_out, R1, sizeof R1);
    memcpy(relT_out + 9, t1, sizeof t1);
    double nv = 0;
    return depth_from_T1(flows, H, W, K, p, R1, t1, theta_out, range_out, &nv);
}

/* ------------------------------------------------------------------------ */
/* whole window (Table 1)                                                   */
/* ------------------------------------------------------------------------ */
static int params_ok(const or_params *p, int T, int H, int W, const double *K)
{
    if (p->struct_size != sizeof(or_params)) return 0;
    if (T < 1 || H < 16 || W < 16) return 0;
    if (!(K[0] > 0) || !(K[1] > 0) || !isfinite(K[2]) || !isfinite(K[3])) return 0;
    if (!(p->gamma >= 0.5 && p->gamma < 1) || !(p->lambda > 0) || !(p->a1 > 0)) return 0;
    if (p->n_pose_groups < 1 || p->n_iters < 1 || p->sweeps_per_iter < 1) return 0;
    if (p->lmeds_hypotheses < 1 || p->lmeds_eval_pixels < 8 || p->n_seeds < 0) return 0;
    if (!(p->sigma2_trans > 0) || !(p->sigma2_rot > 0) || !(p->beta_min > 0) || !(p->x_floor > 0)) return 0;
    if (p->criterion != 0 && p->criterion != 1) return 0;
    if (p->pose_start != 0 && p->pose_start != 1) return 0;
    if (p->residual_model != 0 && p->residual_model != 1) return 0;
    return 1;
}

/* poses_out [T][12] relative; depth_out [H][W]; rig_out [T][H][W];
 * loglik_out [2] = L and its L1 mass; diag_out optional [8]. */
/* Log-likelihood of the window under relative poses rel (Eq. 3 with the
 * posterior rigidness r of every observed pixel and frame): the score by which
 * a proposed initial state is compared with the bootstrap's. */
static double window_loglik(const or_frame_set *F, const or_params *p, const double *rel,
                            const double *theta)
{
    double *M = (double *)malloc(sizeof(double) * 12 * (F->T + 1));
    cumulative(rel, F->T, M);
    double L = 0, Lc = 0;
    for (int t = 1; t <= F->T; ++t)
        for (int y = 0; y < F->H; ++y)
            for (int x = 0; x < F->W; ++x) {
                or_emis e = emission(F, p, M, t, x, y, theta[(size_t)y * F->W + x]);
                if (!e.observed) continue;
                double term = e.r * e.logrho + (1 - e.r) * e.logmu;
                double yk = term - Lc, tk = L + yk;
                Lc = (tk - L) - yk;
                L = tk;
            }
    free(M);
    return L;
}

/* One pass of pose steps t = 1..T of iteration `it` (Sec. 5.2) on the depth
 * theta and rigidness rig (NULL: W = 1); rel is updated in place, M rebuilt. */
static void pose_pass(const float *flows, int T, int H, int W, const double *K, const or_params *p,
                      const double *theta, const double *rig, int it, double *rel, double *M,
                      int *fallbacks, int *ms_total)
{
    pose_identity(M);
    for (int t = 1; t <= T; ++t) {
        const double *prevT = NULL;
        if (it > 0 || t == 1) prevT = rel + 12 * (t - 1);
        else prevT = rel + 12 * (t - 2); /* first pass: previous frame's motion as fallback */
        double Tn[12], prevcopy[12];
        memcpy(prevcopy, prevT, sizeof prevcopy);
        int dg[4];
        or_pose_step(theta, rig, flows, T, H, W, K, p, M, t, it, (it > 0 || t == 1) ? prevcopy : NULL, Tn,
                     NULL, dg);
        if (dg[3]) memcpy(Tn, prevcopy, sizeof Tn);
        *fallbacks += dg[3];
        *ms_total += dg[2];
        memcpy(rel + 12 * (t - 1), Tn, sizeof Tn);
        pose_compose(rel + 12 * (t - 1), M + 12 * (t - 1), M + 12 * t);
    }
}

/* One EM iteration of Table 1 (iteration index `it`, which sets the random
 * draws): the pose of every frame (unless with_pose is 0), the directional
 * sweeps, the unsmoothed rigidness, then the scale gauge |t_1| = 1 applied to
 * the depth, the translations and the depth range. */
static void em_iteration(const float *flows, int T, int H, int W, const double *K, const or_params *p, int it,
                         int with_pose, double *rel, double *M, double *depth, double *rig, int have_w,
                         double *range, int *fallbacks, int *ms_total)
{
    size_t HW = (size_t)H * W;
    or_frame_set F = {flows, T, H, W, K[0], K[1], K[2], K[3]};
    if (with_pose) pose_pass(flows, T, H, W, K, p, depth, have_w ? rig : NULL, it, rel, M, fallbacks, ms_total);
    for (int s = 0; s < p->sweeps_per_iter; ++s) {
        int64_t gs = (int64_t)it * p->sweeps_per_iter + s;
        or_sweep(depth, depth, flows, T, H, W, K, p, M, range[0], range[1], gs, (int)(gs % 4), NULL, NULL);
    }
    /* rigidness without smoothing (last row of Table 1) */
    for (int t = 1; t <= T; ++t)
        for (int y = 0; y < H; ++y)
            for (int x = 0; x < W; ++x)
                rig[(size_t)(t - 1) * HW + (size_t)y * W + x] = emission(&F, p, M, t, x, y, depth[(size_t)y * W + x]).r;
    /* scale gauge: |t_1| = 1 */
    double sc = norm3(rel + 9);
    if (sc > 0) {
        for (size_t j = 0; j < HW; ++j) depth[j] /= sc;
        for (int t = 1; t <= T; ++t)
            for (int k = 0; k < 3; ++k) rel[12 * (t - 1) + 9 + k] /= sc;
        range[0] /= sc;
        range[1] /= sc;
    }
}

/* Log-likelihood of Eq. 3 under the final rigidness (Kahan sums), and its L1
 * mass: loglik_out[0], loglik_out[1] (if loglik_out). */
static void final_loglik(const or_frame_set *F, const or_params *p, const double *rel, double *M,
                         const double *depth, const double *rig, double *loglik_out)
{
    const int T = F->T, H = F->H, W = F->W;
    const size_t HW = (size_t)H * W;
    cumulative(rel, T, M);
    double L = 0, Lc = 0, A = 0, Ac = 0;
    for (int t = 1; t <= T; ++t)
        for (int y = 0; y < H; ++y)
            for (int x = 0; x < W; ++x) {
                size_t j = (size_t)y * W + x;
                or_emis e = emission(F, p, M, t, x, y, depth[j]);
                if (!e.observed) continue;
                double w = rig[(size_t)(t - 1) * HW + j];
                double term = w * e.logrho + (1 - w) * e.logmu;
                double yk = term - Lc, tk = L + yk;
                Lc = (tk - L) - yk;
                L = tk;
                double ya = fabs(term) - Ac, ta = A + ya;
                Ac = (ta - A) - ya;
                A = ta;
            }
    if (loglik_out) { loglik_out[0] = L; loglik_out[1] = A; }
}

static int window_core(const float *flows, int T, int H, int W, const double *K, const or_params *p,
                       const double *init_depth, const double *init_rig, double *poses_out,
                       double *depth_out, double *rig_out, double *loglik_out, double *diag_out,
                       int *choice_out, const double *T1_seed)
{
    if (!flows || !K || !p || !poses_out || !depth_out || !rig_out) return OR_EINVAL;
    if (!params_ok(p, T, H, W, K)) return OR_EINVAL;
    size_t HW = (size_t)H * W;
    or_frame_set F = {flows, T, H, W, K[0], K[1], K[2], K[3]};
    double *rel = poses_out;
    double *M = (double *)malloc(sizeof(double) * 12 * (T + 1));
    double range[2], binfo[4];
    int st;
    if (T1_seed) {
        st = or_bootstrap_seeded(flows, T, H, W, K, p, T1_seed, rel, depth_out, range);
        binfo[0] = -1; binfo[1] = 0; binfo[2] = 0; binfo[3] = 0;
    } else {
        st = or_bootstrap(flows, T, H, W, K, p, rel, depth_out, range, binfo);
    }
    if (st != OR_OK) { free(M); return st; }
    for (int t = 2; t <= T; ++t) pose_identity(rel + 12 * (t - 1));
    int have_w = 0; /* W == 1 until the first unsmoothed update */
    int fallbacks = 0, ms_total = 0, first_pass_done = 0;
    if (init_depth && init_rig) {
        /* a proposed initial state (depth, W) against the bootstrap's (depth,
         * W = 1): each gets the first pass of pose steps, and the one whose
         * window log-likelihood is higher is kept, poses included */
        double *rel_boot = (double *)malloc(sizeof(double) * 12 * T);
        double *rel_a = (double *)malloc(sizeof(double) * 12 * T);
        memcpy(rel_boot, rel, sizeof(double) * 12 * T);
        pose_pass(flows, T, H, W, K, p, depth_out, NULL, 0, rel, M, &fallbacks, &ms_total);
        const double La = window_loglik(&F, p, rel, depth_out);
        memcpy(rel_a, rel, sizeof(double) * 12 * T);
        memcpy(rel, rel_boot, sizeof(double) * 12 * T);
        pose_pass(flows, T, H, W, K, p, init_depth, init_rig, 0, rel, M, &fallbacks, &ms_total);
        const double Lb = window_loglik(&F, p, rel, init_depth);
        const int use = Lb > La;
        if (use) memcpy(depth_out, init_depth, HW * sizeof(double));
        else memcpy(rel, rel_a, sizeof(double) * 12 * T);
        cumulative(rel, T, M);
        if (choice_out) *choice_out = use;
        free(rel_boot);
        free(rel_a);
        first_pass_done = 1;
    }
    for (int it = 0; it < p->n_iters; ++it) {
        em_iteration(flows, T, H, W, K, p, it, !(it == 0 && first_pass_done), rel, M, depth_out, rig_out,
                     have_w, range, &fallbacks, &ms_total);
        have_w = 1;
    }
    final_loglik(&F, p, rel, M, depth_out, rig_out, loglik_out);
    if (diag_out) {
        diag_out[0] = binfo[0]; diag_out[1] = binfo[1]; diag_out[2] = range[0]; diag_out[3] = range[1];
        diag_out[4] = fallbacks; diag_out[5] = ms_total; diag_out[6] = binfo[2]; diag_out[7] = binfo[3];
    }
    free(M);
    return OR_OK;
}

int or_window(const float *flows, int T, int H, int W, const double *K, const or_params *p,
              double *poses_out, double *depth_out, double *rig_out, double *loglik_out,
              double *diag_out)
{
    return window_core(flows, T, H, W, K, p, NULL, NULL, poses_out, depth_out, rig_out, loglik_out,
                       diag_out, NULL, NULL);
}

/* One window whose T_1 is given (overlapping consecutive batches, Sec. 5.3). */
int or_window_seeded(const float *flows, int T, int H, int W, const double *K, const or_params *p,
                     const double *T1, double *poses_out, double *depth_out, double *rig_out,
                     double *loglik_out, double *diag_out)
{
    if (!T1) return OR_EINVAL;
    return window_core(flows, T, H, W, K, p, NULL, NULL, poses_out, depth_out, rig_out, loglik_out,
                       diag_out, NULL, T1);
}

/* The window from a proposed initial state (depth [H][W] > 0, rigidness
 * [T][H][W]), used where it beats the bootstrap on X_1; *choice_out = 1 then. */
int or_window_init(const float *flows, int T, int H, int W, const double *K, const or_params *p,
                   const double *init_depth, const double *init_rig, double *poses_out,
                   double *depth_out, double *rig_out, double *loglik_out, double *diag_out,
                   int *choice_out)
{
    if (!init_depth || !init_rig) return OR_EINVAL;
    return window_core(flows, T, H, W, K, p, init_depth, init_rig, poses_out, depth_out, rig_out,
                       loglik_out, diag_out, choice_out, NULL);
}

/* Test hook: the iterations it0 .. n_iters - 1 of a window from a given state
 * at the start of iteration it0 (relative poses rel_in [T][12] in the gauge
 * |t_1| = 1, depth_in [H][W], the rigidness rig_in [T][H][W] of the previous
 * iteration, which weights the pose samples, and the depth range
 * range_in[2]), then the log-likelihood: the EM from another implementation's
 * state, one iteration at a time.  Outputs as or_window. */
int or_window_from_state(const float *flows, int T, int H, int W, const double *K, const or_params *p, int it0,
                         const double *rel_in, const double *depth_in, const double *rig_in,
                         const double *range_in, double *poses_out, double *depth_out, double *rig_out,
                         double *loglik_out)
{
    if (!flows || !K || !p || !rel_in || !depth_in || !rig_in || !range_in || !poses_out || !depth_out || !rig_out)
        return OR_EINVAL;
    if (!params_ok(p, T, H, W, K) || it0 < 1 || it0 >= p->n_iters) return OR_EINVAL;
    size_t HW = (size_t)H * W;
    or_frame_set F = {flows, T, H, W, K[0], K[1], K[2], K[3]};
    double *M = (double *)malloc(sizeof(double) * 12 * (T + 1));
    double range[2] = {range_in[0], range_in[1]};
    memcpy(poses_out, rel_in, sizeof(double) * 12 * T);
    memcpy(depth_out, depth_in, sizeof(double) * HW);
    memcpy(rig_out, rig_in, sizeof(double) * HW * T);
    cumulative(poses_out, T, M);
    int fallbacks = 0, ms_total = 0;
    for (int it = it0; it < p->n_iters; ++it)
        em_iteration(flows, T, H, W, K, p, it, 1, poses_out, M, depth_out, rig_out, 1, range, &fallbacks, &ms_total);
    final_loglik(&F, p, poses_out, M, depth_out, rig_out, loglik_out);
    free(M);
    return OR_OK;
}
