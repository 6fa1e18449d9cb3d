// vo_resfit.hip -- regression of the Fisk laws of Eq. 6-7 on optical-flow
// residuals (the procedure behind the paper's Fig. 4b): squared end-point
// errors x = |X - G|^2 binned by the observed flow magnitude |X|, a Fisk fit
// per bin by the moments of log x (the log of a Fisk variable is logistic with
// location log(alpha) and scale 1/beta), and count-weighted least squares of
// log(alpha) = log(a1) + a2 v and beta = b1 v + b2 over the bins.
//
// k_resid_bins streams the two flow fields once (16 bytes per item) and
// accumulates per-bin count, sum |v|, sum log x and sum (log x)^2 in FP64;
// its cost is the VALU work of the per-bin row reductions and of the log, not
// HBM.  Per-workgroup partials are then summed over workgroups in a fixed
// order, so the result does not depend on scheduling.
#include "vo_internal.hpp"

#include <math.h>
#include <string.h>

#include <algorithm>
#include <mutex>

namespace vo {

constexpr int kFitThreads = 512;
constexpr int kFitMaxBins = 256;
constexpr int kFitBlocks = 1024;
constexpr int kFitK = 4;   // items per lane and round

// FP64 cross-lane moves without the LDS crossbar, on the two 32-bit halves:
// DPP row rotation within 16 lanes, and the gfx950 lane-half swaps, which give
// every lane the value of lane l ^ 16 (rows 2k, 2k + 1) or l ^ 32
template <int CTRL>
__device__ __forceinline__ double dpp_d(double v)
{
    const unsigned long long u = (unsigned long long)__double_as_longlong(v);
    const unsigned lo = (unsigned)__builtin_amdgcn_update_dpp(0, (int)(unsigned)u, CTRL, 0xf, 0xf, true);
    const unsigned hi = (unsigned)__builtin_amdgcn_update_dpp(0, (int)(unsigned)(u >> 32), CTRL, 0xf, 0xf, true);
    return __longlong_as_double((long long)(((unsigned long long)hi << 32) | lo));
}

__device__ __forceinline__ double partner16_d(double v, int lane)
{
    const unsigned long long u = (unsigned long long)__double_as_longlong(v);
    const auto lo = __builtin_amdgcn_permlane16_swap((unsigned)u, (unsigned)u, false, false);
    const auto hi = __builtin_amdgcn_permlane16_swap((unsigned)(u >> 32), (unsigned)(u >> 32), false, false);
    const int k = (lane & 16) ? 0 : 1;
    return __longlong_as_double((long long)(((unsigned long long)hi[k] << 32) | lo[k]));
}

__device__ __forceinline__ double partner32_d(double v, int lane)
{
    const unsigned long long u = (unsigned long long)__double_as_longlong(v);
    const auto lo = __builtin_amdgcn_permlane32_swap((unsigned)u, (unsigned)u, false, false);
    const auto hi = __builtin_amdgcn_permlane32_swap((unsigned)(u >> 32), (unsigned)(u >> 32), false, false);
    const int k = (lane & 32) ? 0 : 1;
    return __longlong_as_double((long long)(((unsigned long long)hi[k] << 32) | lo[k]));
}

// Natural log of a positive finite x to a few ulp: x = m 2^e with m in
// [sqrt(1/2), sqrt(2)), and log m = 2 atanh(s) = 2 (s + s^3/3 + s^5/5 + ...)
// with s = (m - 1) / (m + 1), |s| <= 0.1716; eleven terms leave a remainder
// below 1e-20.  The log only enters sums (no bin decision depends on it).
__device__ __forceinline__ double fit_log(double x)
{
    int e;
    double m = frexp(x, &e);   // m in [0.5, 1)
    if (m < 0.70710678118654752) {
        m *= 2.0;
        e -= 1;
    }
    const double s = (m - 1.0) / (m + 1.0), s2 = s * s;
    double p = 1.0 / 23.0;
#pragma unroll
    for (int k = 21; k >= 3; k -= 2) p = fma(p, s2, 1.0 / k);
    const double t = 2.0 * s;
    return fma((double)e, 0.69314718055994530942, fma(t * s2, p, t));
}

// total over the 16 lanes of a row, in every lane of the row
__device__ __forceinline__ double fit_row_sum(double v)
{
    v += dpp_d<0x128>(v);   // row_ror:8
    v += dpp_d<0x124>(v);   // row_ror:4
    v += dpp_d<0x122>(v);   // row_ror:2
    v += dpp_d<0x121>(v);   // row_ror:1
    return v;
}

__device__ __forceinline__ int fit_row_sum_i(int v)
{
    v += __builtin_amdgcn_update_dpp(0, v, 0x128, 0xf, 0xf, true);
    v += __builtin_amdgcn_update_dpp(0, v, 0x124, 0xf, 0xf, true);
    v += __builtin_amdgcn_update_dpp(0, v, 0x122, 0xf, 0xf, true);
    v += __builtin_amdgcn_update_dpp(0, v, 0x121, 0xf, 0xf, true);
    return v;
}

// A wave takes kFitK x 64 consecutive items at a time (item k of lane l is
// l + 64 k: coalesced loads).  Flows are smooth, so the items fall in few bins;
// for each bin present, every lane adds its items in it, the four sums are
// reduced over each 16-lane row, and in every row the lane that owns the bin
// (lane b % 16 of the row, register slot b / 16) adds them to its running
// sums.  No atomics and no shared-memory traffic in the loop, a fixed order.
// At the end the four rows are added (rows 0 + 1, 2 + 3, then the halves),
// each wave writes its sums to LDS, and the waves are added in wave order.
template <int NS>
__global__ void __launch_bounds__(kFitThreads) k_resid_bins(const float2 *X, const float2 *G, int64_t n, int nbins,
                                                            double inv_width, double x_floor, double *part)
{
    extern __shared__ double hist[];   // [waves][nbins][4]
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    int cnt[NS];
    double sv[NS], sy[NS], syy[NS];
#pragma unroll
    for (int k = 0; k < NS; ++k) {
        cnt[k] = 0;
        sv[k] = sy[k] = syy[k] = 0.0;
    }
    const int64_t stride = (int64_t)gridDim.x * kFitThreads * kFitK;
    for (int64_t j0 = ((int64_t)blockIdx.x * (kFitThreads / 64) + wv) * 64 * kFitK; j0 < n; j0 += stride) {
        int b[kFitK];
        double v[kFitK], y[kFitK];
        float2 xs[kFitK], gs[kFitK];
#pragma unroll
        for (int k = 0; k < kFitK; ++k) {   // all loads first (index clamped, n >= 1)
            const int64_t j = min(j0 + lane + 64 * k, n - 1);
            xs[k] = X[j];
            gs[k] = G[j];
        }
#pragma unroll
        for (int k = 0; k < kFitK; ++k) {
            b[k] = -1;
            v[k] = y[k] = 0.0;
            if (j0 + lane + 64 * k < n) {
                const float2 x = xs[k], g = gs[k];
                if (isfinite(x.x + x.y + g.x + g.y)) {
                    const double vx = x.x, vy = x.y;
                    const double m = sqrt(vx * vx + vy * vy);
                    const int bb = (int)floor(m * inv_width);
                    if (bb >= 0 && bb < nbins) {
                        const double dx = vx - (double)g.x, dy = vy - (double)g.y;
                        y[k] = fit_log(fmax(dx * dx + dy * dy, x_floor));
                        v[k] = m;
                        b[k] = bb;
                    }
                }
            }
        }
        int first = b[kFitK - 1];
#pragma unroll
        for (int k = kFitK - 2; k >= 0; --k) first = b[k] >= 0 ? b[k] : first;
        uint64_t pending = __ballot(first >= 0);
        while (pending) {
            const int bin = __builtin_amdgcn_readlane(first, (int)__builtin_ctzll(pending));
            int c = 0;
            double tv = 0.0, ty = 0.0, tyy = 0.0;
#pragma unroll
            for (int k = 0; k < kFitK; ++k) {
                const bool m = b[k] == bin;
                const double mv = m ? v[k] : 0.0, my = m ? y[k] : 0.0;
                c += m ? 1 : 0;
                tv += mv;
                ty += my;
                tyy = fma(my, my, tyy);
                b[k] = m ? -1 : b[k];
            }
            c = fit_row_sum_i(c);
            tv = fit_row_sum(tv);
            ty = fit_row_sum(ty);
            tyy = fit_row_sum(tyy);
            const bool own = (lane & 15) == (bin & 15);
#pragma unroll
            for (int k = 0; k < NS; ++k)
                if (own && (bin >> 4) == k) {
                    cnt[k] += c;
                    sv[k] += tv;
                    sy[k] += ty;
                    syy[k] += tyy;
                }
            first = b[kFitK - 1];
#pragma unroll
            for (int k = kFitK - 2; k >= 0; --k) first = b[k] >= 0 ? b[k] : first;
            pending = __ballot(first >= 0);
        }
    }
    double *h = hist + (size_t)wv * nbins * 4;
#pragma unroll
    for (int k = 0; k < NS; ++k) {
        // rows: lane l and l ^ 16 first, then l and l ^ 32 (the same order in every lane)
        double c = (double)cnt[k], a = sv[k], e = sy[k], f = syy[k];
        c += partner16_d(c, lane);
        a += partner16_d(a, lane);
        e += partner16_d(e, lane);
        f += partner16_d(f, lane);
        c += partner32_d(c, lane);
        a += partner32_d(a, lane);
        e += partner32_d(e, lane);
        f += partner32_d(f, lane);
        const int bin = lane + 16 * k;
        if (lane < 16 && bin < nbins) {
            h[4 * bin + 0] = c;
            h[4 * bin + 1] = a;
            h[4 * bin + 2] = e;
            h[4 * bin + 3] = f;
        }
    }
    __syncthreads();
    for (int i = threadIdx.x; i < nbins * 4; i += kFitThreads) {
        double t = 0.0;
        for (int w = 0; w < kFitThreads / 64; ++w) t += hist[(size_t)w * nbins * 4 + i];
        part[(size_t)blockIdx.x * nbins * 4 + i] = t;
    }
}

// Sum of the workgroup partials, one workgroup per 8 consecutive (bin,
// statistic) columns, so that the 8 threads reading a partial row take one
// whole 64-byte line.  Thread t takes column c0 + (t & 7) of the rows
// g = t / 8, g + 128, g + 256, ... into two running sums (rows g + 256 k and
// g + 128 + 256 k, so that two loads are in flight), added in a fixed order;
// then a fixed tree over the 128 row groups.
constexpr int kRedThreads = 1024;
constexpr int kRedGroups = kRedThreads / 8;
__global__ void __launch_bounds__(kRedThreads) k_resid_reduce(const double *part, int nblocks, int ncol, double *out)
{
    __shared__ double red[kRedThreads];
    const int t = threadIdx.x, c = blockIdx.x * 8 + (t & 7);
    double s0 = 0.0, s1 = 0.0;
    if (c < ncol) {
        int b = t >> 3;
        for (; b + kRedGroups < nblocks; b += 2 * kRedGroups) {
            s0 += part[(size_t)b * ncol + c];
            s1 += part[(size_t)(b + kRedGroups) * ncol + c];
        }
        if (b < nblocks) s0 += part[(size_t)b * ncol + c];
    }
    red[t] = s0 + s1;
    __syncthreads();
    for (int h = kRedThreads / 2; h >= 8; h >>= 1) {   // h is a multiple of 8: t and t + h share a column
        if (t < h) red[t] += red[t + h];
        __syncthreads();
    }
    if (t < 8 && c < ncol) out[c] = red[t];
}

// The binning pass into the partials buffer `work` (blocks x nbins x 4
// doubles, every entry written by its workgroup before the reduction reads
// it), then the fixed-order reduction into bins.
static int resid_bins_launch(const float *X, const float *G, int64_t n, int nbins, double v_max, double x_floor,
                             double *work, double *bins, hipStream_t s)
{
    const int blocks = (int)std::min<int64_t>(kFitBlocks, (n + kFitThreads * kFitK - 1) / (kFitThreads * kFitK));
    const size_t lds = sizeof(double) * (kFitThreads / 64) * nbins * 4;
    const auto *x2 = (const float2 *)X, *g2 = (const float2 *)G;
    const double iw = nbins / v_max;
    const int ns = (nbins + 15) / 16;
#define FIT_LAUNCH(NS) hipLaunchKernelGGL(k_resid_bins<NS>, dim3(blocks), dim3(kFitThreads), lds, s, x2, g2, n, nbins, iw, x_floor, work)
    if (ns <= 1) FIT_LAUNCH(1);
    else if (ns <= 2) FIT_LAUNCH(2);
    else if (ns <= 3) FIT_LAUNCH(3);
    else if (ns <= 4) FIT_LAUNCH(4);
    else if (ns <= 8) FIT_LAUNCH(8);
    else FIT_LAUNCH(16);
#undef FIT_LAUNCH
    hipLaunchKernelGGL(k_resid_reduce, dim3((nbins * 4 + 7) / 8), dim3(kRedThreads), 0, s, work, blocks, nbins * 4,
                       bins);
    return hipGetLastError() == hipSuccess ? VOLDOR_OK : VOLDOR_EDEVICE;
}

static bool resid_args_ok(const float *X, const float *G, int64_t n, int nbins, double v_max, double x_floor,
                          const double *bins)
{
    return X && G && bins && n >= 1 && nbins >= 2 && nbins <= kFitMaxBins && v_max > 0.0 && x_floor > 0.0 &&
           ((uintptr_t)X & 7) == 0 && ((uintptr_t)G & 7) == 0 && ((uintptr_t)bins & 7) == 0;
}

// Partials of the binning pass for callers that cannot allocate: one
// file-scope device array, VOLDOR_RESIDUAL_SCRATCH_DOUBLES doubles (2 MiB),
// held by every device the library runs on until the process ends.  Host code
// never passes the array's name to a kernel (on the host it is a stand-in, not
// a device address): its address on each device comes from
// hipGetSymbolAddress, taken once per device with that device current.
static __device__ __align__(256) double scratch[VOLDOR_RESIDUAL_SCRATCH_DOUBLES];
constexpr int kScratchDevices = 64;
static std::mutex g_scratch_mu;
static double *g_scratch_ptr[kScratchDevices];

// the device address of `scratch` on the current device; VOLDOR_EDEVICE if the
// runtime cannot give it
static int scratch_on_current_device(double **out)
{
    int dev = -1;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kScratchDevices) return VOLDOR_EDEVICE;
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void *p = nullptr;
        if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || !p) return VOLDOR_EDEVICE;
        g_scratch_ptr[dev] = (double *)p;
    }
    *out = g_scratch_ptr[dev];
    return VOLDOR_OK;
}

}  // namespace vo

extern "C" {

int64_t voldor_residual_workspace(int64_t n, int nbins)
{
    if (n < 1 || nbins < 2 || nbins > vo::kFitMaxBins) return VOLDOR_EINVAL;
    const int64_t blocks = std::min<int64_t>(vo::kFitBlocks, (n + vo::kFitThreads * vo::kFitK - 1) / (vo::kFitThreads * vo::kFitK));
    return blocks * nbins * 4;
}

int voldor_residual_bins(const float *X, const float *G, int64_t n, int nbins, double v_max, double x_floor,
                         double *work, double *bins, void *stream)
{
    using namespace vo;
    if (!resid_args_ok(X, G, n, nbins, v_max, x_floor, bins) || !work || ((uintptr_t)work & 7) != 0)
        return VOLDOR_EINVAL;
    return resid_bins_launch(X, G, n, nbins, v_max, x_floor, work, bins, (hipStream_t)stream);
}

int voldor_residual_bins_noalloc(const float *X, const float *G, int64_t n, int nbins, double v_max,
                                 double x_floor, double *bins, void *stream)
{
    using namespace vo;
    if (!resid_args_ok(X, G, n, nbins, v_max, x_floor, bins)) return VOLDOR_EINVAL;
    const int64_t need = voldor_residual_workspace(n, nbins);
    if (need < 1 || need > VOLDOR_RESIDUAL_SCRATCH_DOUBLES) return VOLDOR_EINVAL;
    double *work = nullptr;
    const int rc = scratch_on_current_device(&work);
    if (rc) return rc;
    return resid_bins_launch(X, G, n, nbins, v_max, x_floor, work, bins, (hipStream_t)stream);
}

int voldor_residual_fit(const float *X, const float *G, int64_t n, int nbins, double v_max, double x_floor,
                        int min_count, double *laws, double *bins, void *stream)
{
    using namespace vo;
    if (!X || !G || !laws || n < 1 || nbins < 2 || nbins > kFitMaxBins || !(v_max > 0.0) || !(x_floor > 0.0) ||
        min_count < 2 || ((uintptr_t)X & 7) != 0 || ((uintptr_t)G & 7) != 0)
        return VOLDOR_EINVAL;
    hipStream_t s = (hipStream_t)stream;
    double *part = nullptr, *out = nullptr;
    if (hipMalloc((void **)&part, sizeof(double) * (size_t)voldor_residual_workspace(n, nbins)) != hipSuccess)
        return VOLDOR_ENOMEM;
    if (hipMalloc((void **)&out, sizeof(double) * nbins * 4) != hipSuccess) {
        (void)hipFree(part);
        return VOLDOR_ENOMEM;
    }
    double st[kFitMaxBins * 4];
    int rc = voldor_residual_bins(X, G, n, nbins, v_max, x_floor, part, out, stream);
    if (rc == 0 && (hipStreamSynchronize(s) != hipSuccess ||
                    hipMemcpy(st, out, sizeof(double) * nbins * 4, hipMemcpyDeviceToHost) != hipSuccess))
        rc = VOLDOR_EDEVICE;
    (void)hipFree(part);
    (void)hipFree(out);
    if (rc) return rc;
    if (bins) memcpy(bins, st, sizeof(double) * nbins * 4);
    // weighted least squares (weights = counts) of y_b = c0 + c1 vbar_b for
    // y = log(alpha) and y = beta, over the bins with enough items
    double S = 0, Sv = 0, Svv = 0, Sa = 0, Sva = 0, Sb = 0, Svb = 0;
    int used = 0;
    for (int k = 0; k < nbins; ++k) {
        const double c = st[4 * k];
        if (c < min_count) continue;
        const double vbar = st[4 * k + 1] / c, mean = st[4 * k + 2] / c;
        const double var = st[4 * k + 3] / c - mean * mean;
        if (!(var > 0.0)) continue;
        const double beta = M_PI / sqrt(3.0 * var);
        S += c;
        Sv += c * vbar;
        Svv += c * vbar * vbar;
        Sa += c * mean;
        Sva += c * vbar * mean;
        Sb += c * beta;
        Svb += c * vbar * beta;
        ++used;
    }
    const double det = S * Svv - Sv * Sv;
    if (used < 2 || !(det > 0.0)) return VOLDOR_EDEGENERATE;
    const double a2 = (S * Sva - Sv * Sa) / det, la1 = (Sa - a2 * Sv) / S;
    const double b1 = (S * Svb - Sv * Sb) / det, b2 = (Sb - b1 * Sv) / S;
    laws[0] = exp(la1);
    laws[1] = a2;
    laws[2] = b1;
    laws[3] = b2;
    return VOLDOR_OK;
}

}  // extern "C"
