// vo_resfit.hip -- regression of the Fisk laws of Eq. 6-7 on optical-flow
// residuals (the procedure behind the paper's Fig. 4b): squared end-point
// errors x = |X - G|^2 binned by the observed flow magnitude |X|, a Fisk fit
// per bin by the moments of log x (the log of a Fisk variable is logistic with
// location log(alpha) and scale 1/beta), and count-weighted least squares of
// log(alpha) = log(a1) + a2 v and beta = b1 v + b2 over the bins.
//
// k_resid_bins streams the two flow fields once (16 bytes per item, HBM
// bound) and accumulates per-bin count, sum |v|, sum log x and sum (log x)^2
// in FP64; per-workgroup partials are then summed over workgroups in a fixed
// order, so the result does not depend on scheduling.
#include "vo_internal.hpp"

#include <math.h>
#include <string.h>

#include <algorithm>

namespace vo {

constexpr int kFitThreads = 256;
constexpr int kFitMaxBins = 256;
constexpr int kFitBlocks = 1024;

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

// wave total (every lane; lane 0's is the one used, in a fixed order)
__device__ __forceinline__ double fit_wave_sum(double v, int lane)
{
    v += dpp_d<0x128>(v);   // row_ror:8
    v += dpp_d<0x124>(v);   // row_ror:4
    v += dpp_d<0x122>(v);   // row_ror:2
    v += dpp_d<0x121>(v);   // row_ror:1
    v += partner16_d(v, lane);
    v += partner32_d(v, lane);
    return v;
}

// Each wave keeps its own histogram in LDS.  A wave takes 64 consecutive
// items at a time; flows are smooth, so its lanes fall in few bins: for each
// bin present, the four sums over the lanes in it are wave reductions, and
// lane 0 adds them to the wave's histogram (no atomics, a fixed order).  The
// four waves' histograms are added in wave order at the end.
__global__ void __launch_bounds__(kFitThreads) k_resid_bins(const float2 *X, const float2 *G, int64_t n, int nbins,
                                                            double inv_width, double x_floor, double *part)
{
    __shared__ double hist[kFitThreads / 64][kFitMaxBins * 4];
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    double *h = hist[wv];
    for (int i = lane; i < nbins * 4; i += 64) h[i] = 0.0;
    const int64_t stride = (int64_t)gridDim.x * kFitThreads;
    for (int64_t j0 = (int64_t)blockIdx.x * kFitThreads + 64 * wv; j0 < n; j0 += stride) {
        const int64_t j = j0 + lane;
        int b = -1;
        double v = 0.0, y = 0.0;
        if (j < n) {
            const float2 x = X[j], g = G[j];
            if (isfinite(x.x + x.y + g.x + g.y)) {
                const double vx = x.x, vy = x.y;
                v = sqrt(vx * vx + vy * vy);
                const int bb = (int)floor(v * inv_width);
                if (bb >= 0 && bb < nbins) {
                    const double dx = vx - (double)g.x, dy = vy - (double)g.y;
                    y = log(fmax(dx * dx + dy * dy, x_floor));
                    b = bb;
                }
            }
        }
        uint64_t pending = __ballot(b >= 0);
        while (pending) {
            const int leader = __ffsll((unsigned long long)pending) - 1;
            const int bin = __shfl(b, leader, 64);
            const bool mine = b == bin;
            const double c = fit_wave_sum(mine ? 1.0 : 0.0, lane), sv = fit_wave_sum(mine ? v : 0.0, lane);
            const double sy = fit_wave_sum(mine ? y : 0.0, lane), syy = fit_wave_sum(mine ? y * y : 0.0, lane);
            if (lane == 0) {
                h[4 * bin + 0] += c;
                h[4 * bin + 1] += sv;
                h[4 * bin + 2] += sy;
                h[4 * bin + 3] += syy;
            }
            pending &= ~__ballot(mine);
        }
    }
    __syncthreads();
    for (int i = threadIdx.x; i < nbins * 4; i += kFitThreads) {
        double t = 0.0;
        for (int w = 0; w < kFitThreads / 64; ++w) t += hist[w][i];
        part[(size_t)blockIdx.x * nbins * 4 + i] = t;
    }
}

// one workgroup per (bin, statistic): thread t adds the partials of
// workgroups t, t + 256, ... in order, then a fixed tree over the threads
__global__ void __launch_bounds__(256) k_resid_reduce(const double *part, int nblocks, int nbins, double *out)
{
    __shared__ double red[256];
    const int i = blockIdx.x, t = threadIdx.x;
    double s = 0.0;
    for (int b = t; b < nblocks; b += 256) s += part[(size_t)b * nbins * 4 + i];
    red[t] = s;
    __syncthreads();
    for (int h = 128; h > 0; h >>= 1) {
        if (t < h) red[t] += red[t + h];
        __syncthreads();
    }
    if (t == 0) out[i] = red[0];
}

}  // namespace vo

extern "C" {

int64_t voldor_residual_workspace(int64_t n, int nbins)
{
    if (n < 1 || nbins < 2 || nbins > vo::kFitMaxBins) return VOLDOR_EINVAL;
    const int64_t blocks = std::min<int64_t>(vo::kFitBlocks, (n + vo::kFitThreads - 1) / vo::kFitThreads);
    return blocks * nbins * 4;
}

int voldor_residual_bins(const float *X, const float *G, int64_t n, int nbins, double v_max, double x_floor,
                         double *work, double *bins, void *stream)
{
    using namespace vo;
    if (!X || !G || !work || !bins || n < 1 || nbins < 2 || nbins > kFitMaxBins || !(v_max > 0.0) ||
        !(x_floor > 0.0) || ((uintptr_t)X & 7) != 0 || ((uintptr_t)G & 7) != 0 || ((uintptr_t)work & 7) != 0 ||
        ((uintptr_t)bins & 7) != 0)
        return VOLDOR_EINVAL;
    hipStream_t s = (hipStream_t)stream;
    const int blocks = (int)std::min<int64_t>(kFitBlocks, (n + kFitThreads - 1) / kFitThreads);
    hipLaunchKernelGGL(k_resid_bins, dim3(blocks), dim3(kFitThreads), 0, s, (const float2 *)X, (const float2 *)G, n,
                       nbins, nbins / v_max, x_floor, work);
    hipLaunchKernelGGL(k_resid_reduce, dim3(nbins * 4), dim3(256), 0, s, work, blocks, nbins, bins);
    return hipGetLastError() == hipSuccess ? VOLDOR_OK : VOLDOR_EDEVICE;
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
