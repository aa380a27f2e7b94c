// Attractive molecular field by spectral convolution (float32, MFMA).
//
// The RPA field of Sec. 3 (below eq. potmeanforce) acting on species a is
//   C_a(r) = sum_b sum_{e in T_ab} w_ab(e) n_b(r + e),   w_ab(e) = 6 eps sigma^6 / |e|^7 e_hat,
// a circular convolution on the periodic box.  In Fourier space
//   C^_a(k) = i sum_b S_ab(k) n^_b(k),   S_ab(k) = -Im F[w_ab](k)     (w_ab is odd),
// so each step runs: a real-to-complex DFT of the M density fields, the
// spectral product, and a complex-to-real inverse DFT of the 3M output
// components.  Every 1-D DFT along an axis is a dense contraction with the
// DFT matrix, executed as a batched float32 GEMM on the matrix cores
// (v_mfma_f32_16x16x4f32):
//   x (innermost):  rows = lines, C = A W          (W: nx x 2nkx, or 2nkx x nx)
//   y, z:           C = W B                         (W: 2L x 2L real block form
//                                                    of the complex DFT matrix)
// Complex data live as split real/imaginary planes:
//   spec[field][plane][z][y][kx],  kx < nkx = nx/2 + 1.
// The spectrum S_ab is obtained once at init by the same forward stages
// applied to the kernels w_ab placed on the grid, scaled by 1/N so the
// inverse stages need no normalisation.
#include <hip/hip_runtime.h>

#include <cmath>

#include "spectral.h"

namespace mlb {

typedef float v4f __attribute__((ext_vector_type(4)));

constexpr int kTM = 64, kTN = 64, kTK = 16;
constexpr int kGemmThreads = 256;

__device__ inline long long part_t(const MatAddr &m, int t)
{
    const int h = t / m.t_div;
    return (long long)h * m.s_thi + (long long)(t - h * m.t_div) * m.s_tlo;
}
__device__ inline long long part_r(const MatAddr &m, int r)
{
    const int h = r / m.r_div;
    return (long long)h * m.s_rhi + (long long)(r - h * m.r_div) * m.s_rlo;
}
__device__ inline long long part_c(const MatAddr &m, int c)
{
    const int h = c / m.c_div;
    return (long long)h * m.s_chi + (long long)(c - h * m.c_div) * m.s_clo;
}

// C(t) [M x N] = A(t) [M x K] * B(t) [K x N], all float32, general strided
// addressing (separable: batch part + row part + column part).  Workgroup:
// 4 waves, 64x64 output tile, each wave a 32x32 quadrant made of 2x2 MFMA
// 16x16 blocks; K staged through LDS 16 at a time, the next K slice held in
// registers while the current one is consumed.  Each thread loads a fixed
// tile column of A (4 rows) and a fixed tile column of B (4 K-rows), so
// row/column address parts are computed once per workgroup.
// Lane layout of v_mfma_f32_16x16x4f32: A[i][k] from lane i + 16k,
// B[k][j] from lane j + 16k, D[4q + v][j] in lane j + 16q, element v.
__global__ void __launch_bounds__(kGemmThreads) k_gemm_f32(GemmDesc g)
{
    __shared__ float As[kTM][kTK + 1];
    __shared__ float Bs[kTK][kTN + 1];
    const int t = blockIdx.z;
    const int m0 = blockIdx.y * kTM, n0 = blockIdx.x * kTN;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int wm = (wave >> 1) * 32, wn = (wave & 1) * 32;
    const float *__restrict__ A = g.A.base + part_t(g.A, t);
    const float *__restrict__ B = g.B.base + part_t(g.B, t);
    // A loads: rows ar + 16 i, K column ak
    const int ar = tid / kTK, ak = tid % kTK;
    long long arow[4];
    bool arok[4];
    for (int i = 0; i < 4; ++i) {
        const int r = m0 + ar + 16 * i;
        arok[i] = r < g.M;
        arow[i] = arok[i] ? part_r(g.A, r) : 0;
    }
    // B loads: K rows bk + 4 i, column bc
    const int bk = tid / kTN, bc = tid % kTN;
    const bool bcok = n0 + bc < g.N;
    const long long bcol = bcok ? part_c(g.B, n0 + bc) : 0;
    float ra[4], rb[4];
    auto load = [&](int k0) {
        const int ka = k0 + ak;
        const long long acol = ka < g.K ? part_c(g.A, ka) : 0;
        for (int i = 0; i < 4; ++i) ra[i] = (arok[i] && ka < g.K) ? A[arow[i] + acol] : 0.f;
        for (int i = 0; i < 4; ++i) {
            const int kb = k0 + bk + 4 * i;
            rb[i] = (bcok && kb < g.K) ? B[part_r(g.B, kb) + bcol] : 0.f;
        }
    };
    v4f acc[2][2];
    for (int i = 0; i < 2; ++i)
        for (int j = 0; j < 2; ++j) acc[i][j] = v4f{0.f, 0.f, 0.f, 0.f};
    load(0);
    for (int k0 = 0; k0 < g.K; k0 += kTK) {
        for (int i = 0; i < 4; ++i) As[ar + 16 * i][ak] = ra[i];
        for (int i = 0; i < 4; ++i) Bs[bk + 4 * i][bc] = rb[i];
        __syncthreads();
        if (k0 + kTK < g.K) load(k0 + kTK);
#pragma unroll
        for (int kk = 0; kk < kTK; kk += 4) {
            const int ka = kk + (lane >> 4), li = lane & 15;
            float a[2], b[2];
            for (int i = 0; i < 2; ++i) a[i] = As[wm + 16 * i + li][ka];
            for (int j = 0; j < 2; ++j) b[j] = Bs[ka][wn + 16 * j + li];
            for (int i = 0; i < 2; ++i)
                for (int j = 0; j < 2; ++j)
                    acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x4f32(a[i], b[j], acc[i][j], 0, 0, 0);
        }
        __syncthreads();
    }
    float *__restrict__ C = g.C.base + part_t(g.C, t);
    const int j = lane & 15, q = lane >> 4;
    for (int bj = 0; bj < 2; ++bj) {
        const int c = n0 + wn + 16 * bj + j;
        if (c >= g.N) continue;
        const long long cc = part_c(g.C, c);
        for (int bi = 0; bi < 2; ++bi)
            for (int v = 0; v < 4; ++v) {
                const int r = m0 + wm + 16 * bi + 4 * q + v;
                if (r < g.M) C[part_r(g.C, r) + cc] = acc[bi][bj][v];
            }
    }
}

void launch_gemm(const GemmDesc &g, hipStream_t st)
{
    dim3 grid((g.N + kTN - 1) / kTN, (g.M + kTM - 1) / kTM, g.batch);
    hipLaunchKernelGGL(k_gemm_f32, grid, dim3(kGemmThreads), 0, st, g);
}

// Spectral product: out(a,d) = i sum_b S_{p(a,b), d} n^_b.
//   re_out = -sum_b S n^_b,im,  im_out = sum_b S n^_b,re
__global__ void k_spec_mul(const float *__restrict__ in, const float *__restrict__ S, float *__restrict__ out,
                           int M, long long Sp)
{
    const long long k = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= Sp) return;
    const int a = blockIdx.y / 3, d = blockIdx.y % 3;
    float re = 0.f, im = 0.f;
    for (int b = 0; b < M; ++b) {
        const int lo = a < b ? a : b, hi = a < b ? b : a;
        const int p = lo * M - (lo * (lo - 1)) / 2 + (hi - lo);
        const float s = S[((long long)p * 3 + d) * Sp + k];
        const float nr = in[(long long)b * 2 * Sp + k], ni = in[(long long)b * 2 * Sp + Sp + k];
        re -= s * ni;
        im += s * nr;
    }
    out[(long long)blockIdx.y * 2 * Sp + k] = re;
    out[(long long)blockIdx.y * 2 * Sp + Sp + k] = im;
}

// S = -Im(F[w]) / Ntot from the forward spectrum of the placed kernels.
__global__ void k_spec_extract(const float *__restrict__ spec, float *__restrict__ S, int nfields, long long Sp,
                               float scale)
{
    const long long k = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= Sp) return;
    const int f = blockIdx.y;
    S[(long long)f * Sp + k] = -spec[(long long)f * 2 * Sp + Sp + k] * scale;
}

// ------------------------------------------------------------------ plan
namespace {

MatAddr dense(const float *base, long long ld)
{
    MatAddr m{};
    m.base = const_cast<float *>(base);
    m.t_div = 1 << 30; m.r_div = 1 << 30; m.c_div = 1 << 30;
    m.s_rlo = ld; m.s_clo = 1;
    return m;
}

}  // namespace

void SpectralPlan::forward_stages(const float *real_in, int nfields, float *s1, float *s2, hipStream_t st) const
{
    // x: rows (z, y) of each field; output columns (plane, kx)
    GemmDesc gx{};
    gx.M = nz * ny; gx.N = 2 * nkx; gx.K = nx; gx.batch = nfields;
    gx.A = dense(real_in, nx); gx.A.t_div = 1 << 30; gx.A.s_tlo = (long long)nx * ny * nz;
    gx.B = dense(wxf, 2 * nkx);
    gx.C = dense(s1, nkx); gx.C.s_tlo = 2 * Sp; gx.C.c_div = nkx; gx.C.s_chi = Sp; gx.C.s_clo = 1;
    launch_gemm(gx, st);
    // y: per field, rows (plane, ky), K (plane, y), columns (z, kx)
    GemmDesc gy{};
    gy.M = 2 * ny; gy.N = nz * nkx; gy.K = 2 * ny; gy.batch = nfields;
    gy.A = dense(wyf, 2 * ny);
    gy.B = dense(s1, 0); gy.B.s_tlo = 2 * Sp; gy.B.r_div = ny; gy.B.s_rhi = Sp; gy.B.s_rlo = nkx;
    gy.B.c_div = nkx; gy.B.s_chi = Sz; gy.B.s_clo = 1;
    gy.C = gy.B; gy.C.base = s2;
    launch_gemm(gy, st);
    // z: per field, rows (plane, kz), K (plane, z), columns (y, kx) contiguous
    GemmDesc gz{};
    gz.M = 2 * nz; gz.N = ny * nkx; gz.K = 2 * nz; gz.batch = nfields;
    gz.A = dense(wzf, 2 * nz);
    gz.B = dense(s2, 0); gz.B.s_tlo = 2 * Sp; gz.B.r_div = nz; gz.B.s_rhi = Sp; gz.B.s_rlo = Sz; gz.B.s_clo = 1;
    gz.C = gz.B; gz.C.base = s1;
    launch_gemm(gz, st);
}

void SpectralPlan::inverse_stages(float *s1, float *s2, int nfields, float *real_out, hipStream_t st) const
{
    GemmDesc gz{};
    gz.M = 2 * nz; gz.N = ny * nkx; gz.K = 2 * nz; gz.batch = nfields;
    gz.A = dense(wzi, 2 * nz);
    gz.B = dense(s2, 0); gz.B.s_tlo = 2 * Sp; gz.B.r_div = nz; gz.B.s_rhi = Sp; gz.B.s_rlo = Sz; gz.B.s_clo = 1;
    gz.C = gz.B; gz.C.base = s1;
    launch_gemm(gz, st);
    GemmDesc gy{};
    gy.M = 2 * ny; gy.N = nz * nkx; gy.K = 2 * ny; gy.batch = nfields;
    gy.A = dense(wyi, 2 * ny);
    gy.B = dense(s1, 0); gy.B.s_tlo = 2 * Sp; gy.B.r_div = ny; gy.B.s_rhi = Sp; gy.B.s_rlo = nkx;
    gy.B.c_div = nkx; gy.B.s_chi = Sz; gy.B.s_clo = 1;
    gy.C = gy.B; gy.C.base = s2;
    launch_gemm(gy, st);
    // x: complex-to-real; K (plane, kx)
    GemmDesc gx{};
    gx.M = nz * ny; gx.N = nx; gx.K = 2 * nkx; gx.batch = nfields;
    gx.A = dense(s2, nkx); gx.A.s_tlo = 2 * Sp; gx.A.c_div = nkx; gx.A.s_chi = Sp; gx.A.s_clo = 1;
    gx.B = dense(wxi, nx);
    gx.C = dense(real_out, nx); gx.C.s_tlo = (long long)nx * ny * nz;
    launch_gemm(gx, st);
}

void SpectralPlan::build_spectrum(const float *placed, float *s1, float *s2, hipStream_t st) const
{
    const int nf = 3 * P;
    forward_stages(placed, nf, s1, s2, st);
    const float scale = 1.0f / (float)((double)nx * ny * nz);
    hipLaunchKernelGGL(k_spec_extract, dim3((unsigned)((Sp + 255) / 256), nf), dim3(256), 0, st, s1, S, nf, Sp,
                       scale);
}

void SpectralPlan::apply(const float *n, float *s1, float *s2, float *tail, hipStream_t st) const
{
    forward_stages(n, M, s1, s2, st);
    hipLaunchKernelGGL(k_spec_mul, dim3((unsigned)((Sp + 255) / 256), 3 * M), dim3(256), 0, st, s1, S, s2, M, Sp);
    inverse_stages(s1, s2, 3 * M, tail, st);
}

}  // namespace mlb

// ---------------------------------------------------------------- host side
namespace mlb {

namespace {
double angle(long long k, long long x, int L)
{
    return 2.0 * M_PI * (double)((k * x) % L) / (double)L;
}
}  // namespace

std::vector<float> SpectralPlan::dft_x_forward(int nx)
{
    const int nkx = nx / 2 + 1;
    std::vector<float> w((size_t)nx * 2 * nkx);
    for (int x = 0; x < nx; ++x)
        for (int k = 0; k < nkx; ++k) {
            const double th = angle(k, x, nx);
            w[(size_t)x * 2 * nkx + k] = (float)std::cos(th);
            w[(size_t)x * 2 * nkx + nkx + k] = (float)(-std::sin(th));
        }
    return w;
}

std::vector<float> SpectralPlan::dft_x_inverse(int nx)
{
    const int nkx = nx / 2 + 1;
    std::vector<float> w((size_t)2 * nkx * nx);
    for (int k = 0; k < nkx; ++k) {
        const double ck = (k == 0 || (nx % 2 == 0 && k == nx / 2)) ? 1.0 : 2.0;
        for (int x = 0; x < nx; ++x) {
            const double th = angle(k, x, nx);
            w[(size_t)k * nx + x] = (float)(ck * std::cos(th));
            w[(size_t)(nkx + k) * nx + x] = (float)(-ck * std::sin(th));
        }
    }
    return w;
}

std::vector<float> SpectralPlan::dft_block(int L, bool inverse)
{
    // rows (plane_out, k), columns (plane_in, l); forward exp(-i th), inverse exp(+i th)
    std::vector<float> w((size_t)4 * L * L);
    const double sg = inverse ? -1.0 : 1.0;
    const size_t ld = 2 * (size_t)L;
    for (int k = 0; k < L; ++k)
        for (int l = 0; l < L; ++l) {
            const double th = angle(k, l, L);
            const float c = (float)std::cos(th), s = (float)(sg * std::sin(th));
            w[(size_t)k * ld + l] = c;            // re <- re
            w[(size_t)k * ld + L + l] = s;        // re <- im
            w[(size_t)(L + k) * ld + l] = -s;     // im <- re
            w[(size_t)(L + k) * ld + L + l] = c;  // im <- im
        }
    return w;
}

}  // namespace mlb
