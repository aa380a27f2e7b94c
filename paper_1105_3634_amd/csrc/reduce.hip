// Float64 global sums on the GPU.
//
//  - conserved quantities: sum_r n_a and sum_r j_a (the species continuity
//    and momentum balances of Sec. 2, eqs. continuity and momentcomponent);
//  - the composition-mode amplitude |sum_r (n_a - n_b) exp(-i k x)| whose
//    decay 1/tau = D q^2 gives the mutual diffusion coefficient (Sec. 5.1),
//    or the amplitude |sum_r n_a exp(-i k x)| of one species (a tracer band,
//    whose section-averaged modes decay at D_eff q^2, Sec. 5.2);
//  - the x-variance of a tracer band (Taylor dispersion, Sec. 5.2);
//  - a least-squares fit of a recorded time series.
// Two passes: each block reduces a grid-strided slice (wave shuffles, then
// LDS across the block's waves) into a partial row; one block then sums the
// partial rows in a fixed order, so results do not depend on timing.
#include <hip/hip_runtime.h>

#include "mlb_internal.h"

namespace mlb {

constexpr int kRedThreads = 256;
constexpr int kMaxRed = 16;   // values reduced per site (4 + 12 for M = 4)

__device__ inline double wave_sum(double v)
{
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
    return v;
}

// Sum `nv` per-thread values over the block; result valid in thread 0.
__device__ inline void block_sum(double *vals, int nv, double *lds /* [nv][4] */)
{
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    for (int k = 0; k < nv; ++k) {
        const double w = wave_sum(vals[k]);
        if (lane == 0) lds[k * 4 + wid] = w;
    }
    __syncthreads();
    if (threadIdx.x == 0)
        for (int k = 0; k < nv; ++k) vals[k] = ((lds[k * 4 + 0] + lds[k * 4 + 1]) + lds[k * 4 + 2]) + lds[k * 4 + 3];
}

template <typename T>
__global__ void __launch_bounds__(kRedThreads) k_conserved_partial(const T *__restrict__ n, const T *__restrict__ j,
                                                                   int M, long long N, double *__restrict__ partials)
{
    __shared__ double lds[kMaxRed * 4];
    double acc[kMaxRed];
    const int nv = 4 * M;
    for (int k = 0; k < nv; ++k) acc[k] = 0.0;
    for (long long s = (long long)blockIdx.x * kRedThreads + threadIdx.x; s < N;
         s += (long long)gridDim.x * kRedThreads) {
        for (int a = 0; a < M; ++a) {
            acc[a] += (double)n[(long long)a * N + s];
            for (int d = 0; d < 3; ++d) acc[M + 3 * a + d] += (double)j[((long long)a * 3 + d) * N + s];
        }
    }
    block_sum(acc, nv, lds);
    if (threadIdx.x == 0)
        for (int k = 0; k < nv; ++k) partials[(long long)blockIdx.x * nv + k] = acc[k];
}

__global__ void k_sum_partials(const double *__restrict__ partials, int nparts, int nv, double *__restrict__ out)
{
    // thread k sums column k in block order
    const int k = threadIdx.x;
    if (k >= nv) return;
    double s = 0.0;
    for (int p = 0; p < nparts; ++p) s += partials[(long long)p * nv + k];
    out[k] = s;
}

void launch_conserved(const void *n, const void *j, int prec, int M, long long N, double *partials, int nparts,
                      double *out, hipStream_t st)
{
    if (prec == 64)
        hipLaunchKernelGGL(k_conserved_partial<double>, dim3(nparts), dim3(kRedThreads), 0, st, (const double *)n,
                           (const double *)j, M, N, partials);
    else
        hipLaunchKernelGGL(k_conserved_partial<float>, dim3(nparts), dim3(kRedThreads), 0, st, (const float *)n,
                           (const float *)j, M, N, partials);
    hipLaunchKernelGGL(k_sum_partials, dim3(1), dim3(64), 0, st, partials, nparts, 4 * M, out);
}

// -------------------------------------------------------------- mode / spread
template <typename T>
__global__ void __launch_bounds__(kRedThreads) k_mode_partial(const T *__restrict__ n, int a, int b, int nx,
                                                              long long N, double *__restrict__ partials)
{
    __shared__ double lds[2 * 4];
    double acc[2] = {0.0, 0.0};
    const double k = 2.0 * M_PI / (double)nx;
    for (long long s = (long long)blockIdx.x * kRedThreads + threadIdx.x; s < N;
         s += (long long)gridDim.x * kRedThreads) {
        const int x = (int)(s % nx);
        const double dn = b >= 0 ? (double)n[(long long)a * N + s] - (double)n[(long long)b * N + s]
                                 : (double)n[(long long)a * N + s];
        double sn, cs;
        sincos(k * (double)x, &sn, &cs);
        acc[0] += dn * cs;
        acc[1] += dn * sn;
    }
    block_sum(acc, 2, lds);
    if (threadIdx.x == 0) {
        partials[2 * blockIdx.x + 0] = acc[0];
        partials[2 * blockIdx.x + 1] = acc[1];
    }
}

template <typename T>
__global__ void __launch_bounds__(kRedThreads) k_spread_partial(const T *__restrict__ n, int a, int nx, long long N,
                                                                double *__restrict__ partials)
{
    __shared__ double lds[3 * 4];
    double acc[3] = {0.0, 0.0, 0.0};
    const double c = 0.5 * (double)nx;
    for (long long s = (long long)blockIdx.x * kRedThreads + threadIdx.x; s < N;
         s += (long long)gridDim.x * kRedThreads) {
        const double x = (double)(s % nx) - c;
        const double v = (double)n[(long long)a * N + s];
        acc[0] += v;
        acc[1] += v * x;
        acc[2] += v * x * x;
    }
    block_sum(acc, 3, lds);
    if (threadIdx.x == 0)
        for (int k = 0; k < 3; ++k) partials[3 * blockIdx.x + k] = acc[k];
}

// kind 0: amplitude sqrt(c^2 + s^2) from 2 columns; kind 1: variance from 3 columns.
// Thread t sums the partial rows t, t + 256, ... in order; the block sum then
// adds the threads in a fixed tree, so the result does not depend on timing.
__global__ void __launch_bounds__(kRedThreads) k_append_series(const double *__restrict__ partials, int nparts,
                                                               int kind, double *series, int *count, int cap, double t)
{
    __shared__ double lds[3 * 4];
    const int nv = kind == 0 ? 2 : 3;
    double acc[3] = {0.0, 0.0, 0.0};
    for (int p = threadIdx.x; p < nparts; p += kRedThreads)
        for (int k = 0; k < nv; ++k) acc[k] += partials[(long long)p * nv + k];
    block_sum(acc, nv, lds);
    if (threadIdx.x != 0) return;
    double v;
    if (kind == 0) {
        v = sqrt(acc[0] * acc[0] + acc[1] * acc[1]);
    } else {
        const double m1 = acc[1] / acc[0];
        v = acc[2] / acc[0] - m1 * m1;
    }
    const int c = *count;
    if (c < cap) {
        series[2 * c + 0] = t;
        series[2 * c + 1] = v;
        *count = c + 1;
    }
}

void launch_mode(const void *n, int prec, int a, int b, int nx, long long N, double *partials, int nparts,
                 double *series, int *count, int cap, double t, hipStream_t st)
{
    if (prec == 64)
        hipLaunchKernelGGL(k_mode_partial<double>, dim3(nparts), dim3(kRedThreads), 0, st, (const double *)n, a, b,
                           nx, N, partials);
    else
        hipLaunchKernelGGL(k_mode_partial<float>, dim3(nparts), dim3(kRedThreads), 0, st, (const float *)n, a, b,
                           nx, N, partials);
    hipLaunchKernelGGL(k_append_series, dim3(1), dim3(kRedThreads), 0, st, partials, nparts, 0, series, count, cap,
                       t);
}

void launch_spread(const void *n, int prec, int a, int nx, long long N, double *partials, int nparts,
                   double *series, int *count, int cap, double t, hipStream_t st)
{
    if (prec == 64)
        hipLaunchKernelGGL(k_spread_partial<double>, dim3(nparts), dim3(kRedThreads), 0, st, (const double *)n, a,
                           nx, N, partials);
    else
        hipLaunchKernelGGL(k_spread_partial<float>, dim3(nparts), dim3(kRedThreads), 0, st, (const float *)n, a,
                           nx, N, partials);
    hipLaunchKernelGGL(k_append_series, dim3(1), dim3(kRedThreads), 0, st, partials, nparts, 1, series, count, cap,
                       t);
}

// ---------------------------------------------------------------------- fit
// Ordinary least squares y = alpha + beta t over samples with t >= t_min.
// kind 0: y = ln(v), D = -beta / k2;  kind 1: y = v, D = beta / 2.
// Mode fits (kind 0) use the samples from t_lo = min(t_min, the first time
// the amplitude is at most a tenth of the first sample's) on, as long as
// the amplitude stays at least 1e-6 of the first sample's: a fast mode has
// reached the float32 rounding floor of the densities long before a t_min
// chosen for slow ones, and a slow mode never reaches either bound.
constexpr double kFitStart = 0.1, kFitFloor = 1e-6;
constexpr double kFitGoodR2 = 0.98, kFitGoodFloor = 1e-4;

__device__ inline bool fit_sample(const double *series, int i, int kind, double t_lo, double a0)
{
    if (series[2 * i] < t_lo) return false;
    return kind != 0 || series[2 * i + 1] >= kFitFloor * a0;
}

__global__ void k_fit(const double *__restrict__ series, const int *__restrict__ count, int cap, int kind,
                      double t_min, double k2, double *out)
{
    if (threadIdx.x != 0) return;
    const int c = min(*count, cap);
    double t_lo = t_min, a0 = 0.0;
    if (kind == 0 && c > 0) {
        a0 = series[1];
        for (int i = 0; i < c; ++i)
            if (series[2 * i + 1] <= kFitStart * a0) {
                t_lo = fmin(t_min, series[2 * i]);
                break;
            }
    }
    double n = 0.0, st = 0.0, sy = 0.0;
    for (int i = 0; i < c; ++i) {
        if (!fit_sample(series, i, kind, t_lo, a0)) continue;
        const double t = series[2 * i];
        const double y = kind == 0 ? log(series[2 * i + 1]) : series[2 * i + 1];
        n += 1.0;
        st += t;
        sy += y;
    }
    if (n < 2.0) {
        out[0] = nan("");
        out[1] = nan("");
        out[2] = n;
        out[3] = 0.0;
        out[4] = 0.0;
        return;
    }
    const double tm = st / n, ym = sy / n;
    double stt = 0.0, sty = 0.0;
    for (int i = 0; i < c; ++i) {
        if (!fit_sample(series, i, kind, t_lo, a0)) continue;
        const double t = series[2 * i];
        const double y = kind == 0 ? log(series[2 * i + 1]) : series[2 * i + 1];
        stt += (t - tm) * (t - tm);
        sty += (t - tm) * (y - ym);
    }
    const double beta = sty / stt;
    // coefficient of determination and the smallest amplitude of the window
    double syy = 0.0, sres = 0.0, vmin = INFINITY;
    for (int i = 0; i < c; ++i) {
        if (!fit_sample(series, i, kind, t_lo, a0)) continue;
        const double t = series[2 * i];
        const double y = kind == 0 ? log(series[2 * i + 1]) : series[2 * i + 1];
        const double r = y - (ym + beta * (t - tm));
        syy += (y - ym) * (y - ym);
        sres += r * r;
        vmin = fmin(vmin, series[2 * i + 1]);
    }
    const double r2 = syy > 0.0 ? 1.0 - sres / syy : 0.0;
    out[0] = kind == 0 ? -beta / k2 : 0.5 * beta;
    out[1] = beta;
    out[2] = n;
    out[3] = r2;
    // well conditioned: a straight line (R^2 >= 0.98) through at least five
    // samples; a mode fit also keeps its window above 1e-4 of the first
    // amplitude, clear of the rounding floor of float32 densities
    out[4] = (n >= 5.0 && r2 >= kFitGoodR2 && (kind != 0 || vmin >= kFitGoodFloor * a0)) ? 1.0 : 0.0;
}

void launch_fit(const double *series, const int *count, int cap, int kind, double t_min, double k2, double *out,
                hipStream_t st)
{
    hipLaunchKernelGGL(k_fit, dim3(1), dim3(64), 0, st, series, count, cap, kind, t_min, k2, out);
}

__global__ void k_zero_i32(int *p, int n)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = 0;
}

void launch_zero_i32(int *p, int n, hipStream_t st)
{
    hipLaunchKernelGGL(k_zero_i32, dim3((n + 255) / 256), dim3(256), 0, st, p, n);
}

}  // namespace mlb
