// Attractive molecular field by spectral convolution (float32, MFMA).
//
// The RPA field of Sec. 3 (below eq. potmeanforce) acting on species a is
//   C_a(r) = sum_b sum_{e in T_ab} w_ab(e) n_b(r + e),   w_ab(e) = 6 eps sigma^6 / |e|^7 e_hat,
// a circular convolution on the periodic box.  In Fourier space
//   C^_a(k) = i sum_b S_ab(k) n^_b(k),   S_ab(k) = -Im F[w_ab](k)     (w_ab is odd),
// so each step runs: a real-to-complex DFT of the M density fields, the
// spectral product, and a complex-to-real inverse DFT of the 3M output
// components.  Every 1-D DFT along an axis is a dense contraction with the
// DFT matrix on the matrix cores (v_mfma_f32_16x16x4f32):
//   x (innermost):  batched GEMM over lines, C = A W  (W: nx x 2nkx, or 2nkx x nx)
//   y and z:        one workgroup per (kx plane, field) holds the plane in
//                   LDS and applies the 2L x 2L real block form of the
//                   complex DFT matrix along y, then along z; a second
//                   kernel forms the spectral products and runs the
//                   inverse y/z transforms, one workgroup per (kx, component).
// Complex data live as split real/imaginary parts, kx-major:
//   spec[field][kx][re|im][z][y],  kx < nkx = nx/2 + 1.
// The spectrum S_ab is obtained once at init by the same forward stages
// applied to the kernels w_ab placed on the grid, scaled by 1/N so the
// inverse stages need no normalisation.
#include <hip/hip_runtime.h>

#include <cmath>

#include "spectral.h"

namespace mlb {

typedef float v4f __attribute__((ext_vector_type(4)));

constexpr int kTK = 16;

// A divisor of kPlain or more marks a plain stride (no split); the test is
// uniform across the launch, so it costs a scalar branch, not a division.
constexpr int kPlain = 1 << 30;

__device__ inline long long part_t(const MatAddr &m, int t)
{
    if (m.t_div >= kPlain) return (long long)t * m.s_tlo;
    const int h = t / m.t_div;
    return (long long)h * m.s_thi + (long long)(t - h * m.t_div) * m.s_tlo;
}
__device__ inline long long part_r(const MatAddr &m, int r)
{
    if (m.r_div >= kPlain) return (long long)r * m.s_rlo;
    const int h = r / m.r_div;
    return (long long)h * m.s_rhi + (long long)(r - h * m.r_div) * m.s_rlo;
}
__device__ inline long long part_c(const MatAddr &m, int c)
{
    if (m.c_div >= kPlain) return (long long)c * m.s_clo;
    const int h = c / m.c_div;
    return (long long)h * m.s_chi + (long long)(c - h * m.c_div) * m.s_clo;
}

// C(t) [M x N] = A(t) [M x K] * B(t) [K x N], all float32, general strided
// addressing (separable: batch part + row part + column part).  Workgroup:
// W waves (W = 4: 64x64 output tile; W = 1: 32x32), each wave a 32x32
// block made of 2x2 MFMA 16x16 blocks; K staged through LDS 16 at a time,
// the next K slice held in registers while the current one is consumed.
// Each thread loads a fixed tile column of A and of B, so row/column
// address parts are computed once per workgroup.
// Lane layout of v_mfma_f32_16x16x4f32: A[i][k] from lane i + 16k,
// B[k][j] from lane j + 16k, D[4q + v][j] in lane j + 16q, element v.
template <int W>
__global__ void __launch_bounds__(64 * W) k_gemm_f32(GemmDesc g)
{
    constexpr int kTM = W == 4 ? 64 : 32, kTN = kTM, NT = 64 * W;
    constexpr int RA = kTM * kTK / NT, RB = kTK * kTN / NT;   // loads per thread
    __shared__ float As[kTM][kTK + 1];
    __shared__ float Bs[kTK][kTN + 1];
    const int t = blockIdx.z;
    const int m0 = blockIdx.y * kTM, n0 = blockIdx.x * kTN;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int wm = W == 4 ? (wave >> 1) * 32 : 0, wn = W == 4 ? (wave & 1) * 32 : 0;
    const float *__restrict__ A = g.A.base + part_t(g.A, t);
    const float *__restrict__ B = g.B.base + part_t(g.B, t);
    // A loads: rows ar + (NT / kTK) i, K column ak
    const int ar = tid / kTK, ak = tid % kTK;
    long long arow[RA];
    bool arok[RA];
    for (int i = 0; i < RA; ++i) {
        const int r = m0 + ar + (NT / kTK) * i;
        arok[i] = r < g.M;
        arow[i] = arok[i] ? part_r(g.A, r) : 0;
    }
    // B loads: K rows bk + (NT / kTN) i, column bc
    const int bk = tid / kTN, bc = tid % kTN;
    const bool bcok = n0 + bc < g.N;
    const long long bcol = bcok ? part_c(g.B, n0 + bc) : 0;
    float ra[RA], rb[RB];
    auto load = [&](int k0) {
        const int ka = k0 + ak;
        const long long acol = ka < g.K ? part_c(g.A, ka) : 0;
        for (int i = 0; i < RA; ++i) ra[i] = (arok[i] && ka < g.K) ? A[arow[i] + acol] : 0.f;
        for (int i = 0; i < RB; ++i) {
            const int kb = k0 + bk + (NT / kTN) * i;
            rb[i] = (bcok && kb < g.K) ? B[part_r(g.B, kb) + bcol] : 0.f;
        }
    };
    v4f acc[2][2];
    for (int i = 0; i < 2; ++i)
        for (int j = 0; j < 2; ++j) acc[i][j] = v4f{0.f, 0.f, 0.f, 0.f};
    load(0);
    for (int k0 = 0; k0 < g.K; k0 += kTK) {
        for (int i = 0; i < RA; ++i) As[ar + (NT / kTK) * i][ak] = ra[i];
        for (int i = 0; i < RB; ++i) Bs[bk + (NT / kTN) * i][bc] = rb[i];
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

// 64x64 tiles when they give the chip enough workgroups, else 32x32.
void launch_gemm(const GemmDesc &g, hipStream_t st)
{
    const long long big = (long long)((g.N + 63) / 64) * ((g.M + 63) / 64) * g.batch;
    if (big >= 48) {
        dim3 grid((g.N + 63) / 64, (g.M + 63) / 64, g.batch);
        hipLaunchKernelGGL(k_gemm_f32<4>, grid, dim3(256), 0, st, g);
    } else {
        dim3 grid((g.N + 31) / 32, (g.M + 31) / 32, g.batch);
        hipLaunchKernelGGL(k_gemm_f32<1>, grid, dim3(64), 0, st, g);
    }
}

// ------------------------------------------------------- y/z stages (LDS)
// Two kernels per application of the field:
//   forward:  workgroup (kx, f) transforms the kx plane of input field f
//             along y, then z, and writes its spectrum;
//   inverse:  workgroup (kx, g) forms output component g's spectral product
//             from the M input spectra and transforms it back along z, then y.
// A complex plane lives in LDS as two real parts, rows padded to odd
// strides against bank conflicts:
//   X[p][z][y]  (row stride RY = ny + 1)      T[p][ky][z]  (row stride RZ = nz + 1)
// Each 1-D transform is a dense contraction on the matrix cores
// (v_mfma_f32_16x16x4f32, 16x16 output blocks dealt to the 4 waves):
//   y stage:  T[(p',ky)][z]  = sum_{(p,y)} Wy[(p',ky)][(p,y)] X[p][z][y]
//   z stage:  X[p'][kz][ky] = sum_{(p,z)} T[p][ky][z] Wz[(p',kz)][(p,z)]
// with Wy, Wz the real 2L x 2L block form of the complex DFT matrix, read
// from global memory (a few KB, resident in every L2).  The K loop runs per
// real/imaginary block so lane indices need no division; plane indices use
// a multiply-shift division by ny prepared on the host.
struct FastDiv {
    unsigned m;
    int l;   // q = (umulhi(n, m) + n) >> l, exact for n < 2^31
};

__device__ inline int fdiv(int n, FastDiv d)
{
    const unsigned un = (unsigned)n;
    return (int)((__umulhi(un, d.m) + un) >> d.l);
}

struct YZArgs {
    int ny, nz, M, mode;          // mode 0: forward -> sine spectra of the kernels; 1: forward -> spectra
    int ny_real;                  // lattice rows of a plane; rows ny_real.. are zero-padding (mode 1)
    int PS;                       // ny * nz (one real part of a plane)
    long long Sp, FSTR;           // per-field spectrum part size, field stride in the spectra buffers
    FastDiv div_ny;
    const float *in;
    float *out;
    const float *S;
    float scale;
    const float *wy, *wz;         // forward or inverse DFT matrices (2L x 2L, row-major)
};

struct YZLds {
    int ny, nz, RY, RZ, PX, PT, ty, tz;   // PX, PT: padded part sizes of X and T planes
};

__device__ inline YZLds yz_geometry(const YZArgs &a)
{
    YZLds g;
    g.ny = a.ny; g.nz = a.nz; g.RY = a.ny + 1; g.RZ = a.nz + 1;
    g.PX = a.nz * g.RY; g.PT = a.ny * g.RZ; g.ty = 2 * a.ny; g.tz = 2 * a.nz;
    return g;
}

__device__ inline void yz_stage_y(const YZLds &g, const float *__restrict__ Wy, const float *X, float *T)
{
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, li = lane & 15, q = lane >> 4;
    const int bm = (g.ty + 15) / 16, bn = (g.nz + 15) / 16;
    for (int blk = wave; blk < bm * bn; blk += 4) {
        const int i0 = (blk / bn) * 16, j0 = (blk % bn) * 16;
        const int ia = i0 + li, jb = j0 + li;
        v4f acc = v4f{0.f, 0.f, 0.f, 0.f};
        for (int p = 0; p < 2; ++p)
            for (int y0 = 0; y0 < g.ny; y0 += 4) {
                const int yy = y0 + q;
                const float a = (ia < g.ty && yy < g.ny) ? Wy[ia * g.ty + p * g.ny + yy] : 0.f;
                const float b = (jb < g.nz && yy < g.ny) ? X[p * g.PX + jb * g.RY + yy] : 0.f;
                acc = __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, acc, 0, 0, 0);
            }
        for (int v = 0; v < 4; ++v) {
            const int i = i0 + 4 * q + v;
            if (i < g.ty && jb < g.nz) {
                const int pp = i >= g.ny ? 1 : 0;
                T[pp * g.PT + (i - pp * g.ny) * g.RZ + jb] = acc[v];
            }
        }
    }
}

__device__ inline void yz_stage_z(const YZLds &g, const float *__restrict__ Wz, const float *T, float *X)
{
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, li = lane & 15, q = lane >> 4;
    const int bm = (g.ny + 15) / 16, bn = (g.tz + 15) / 16;
    for (int blk = wave; blk < bm * bn; blk += 4) {
        const int i0 = (blk / bn) * 16, j0 = (blk % bn) * 16;
        const int ia = i0 + li, jb = j0 + li;
        v4f acc = v4f{0.f, 0.f, 0.f, 0.f};
        for (int p = 0; p < 2; ++p)
            for (int z0 = 0; z0 < g.nz; z0 += 4) {
                const int zz = z0 + q;
                const float a = (ia < g.ny && zz < g.nz) ? T[p * g.PT + ia * g.RZ + zz] : 0.f;
                const float b = (jb < g.tz && zz < g.nz) ? Wz[jb * g.tz + p * g.nz + zz] : 0.f;
                acc = __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, acc, 0, 0, 0);
            }
        for (int v = 0; v < 4; ++v) {
            const int i = i0 + 4 * q + v;
            if (i < g.ny && jb < g.tz) {
                const int pp = jb >= g.nz ? 1 : 0;
                X[pp * g.PX + (jb - pp * g.nz) * g.RY + i] = acc[v];
            }
        }
    }
}

// grid (nkx, nfields): spectrum of the kx plane of field f
__global__ void __launch_bounds__(256) k_yz_forward(YZArgs a)
{
    extern __shared__ float L[];
    const YZLds g = yz_geometry(a);
    const int kx = blockIdx.x, f = blockIdx.y;
    const int PL = 2 * (g.PX > g.PT ? g.PX : g.PT);
    float *X = L, *T = L + PL;
    const int P2 = 2 * a.PS;
    const float *__restrict__ src = a.in + f * a.FSTR + (long long)kx * P2;
    for (int i = threadIdx.x; i < P2; i += blockDim.x) {
        const int p = i >= a.PS ? 1 : 0;
        const int r = i - p * a.PS, z = fdiv(r, a.div_ny), y = r - z * a.ny;
        X[p * g.PX + z * g.RY + y] = (a.mode == 0 || y < a.ny_real) ? src[i] : 0.f;
    }
    __syncthreads();
    yz_stage_y(g, a.wy, X, T);
    __syncthreads();
    yz_stage_z(g, a.wz, T, X);
    __syncthreads();
    if (a.mode == 0) {
        // sine spectra of the odd kernels: S = -Im F[w] / N, layout [f][kx][kz][ky]
        float *__restrict__ dst = a.out + f * a.Sp + (long long)kx * a.PS;
        for (int i = threadIdx.x; i < a.PS; i += blockDim.x) {
            const int z = fdiv(i, a.div_ny), y = i - z * a.ny;
            dst[i] = -X[g.PX + z * g.RY + y] * a.scale;
        }
        return;
    }
    float *__restrict__ dst = a.out + f * a.FSTR + (long long)kx * P2;
    for (int i = threadIdx.x; i < P2; i += blockDim.x) {
        const int p = i >= a.PS ? 1 : 0;
        const int r = i - p * a.PS, z = fdiv(r, a.div_ny), y = r - z * a.ny;
        dst[i] = X[p * g.PX + z * g.RY + y];
    }
}

// grid (nkx, 3M): output component (species aa, direction d) of the field:
// C^ = i sum_b S_{aa b, d} n^_b, then the inverse y/z stages
__global__ void __launch_bounds__(256) k_yz_inverse(YZArgs a)
{
    extern __shared__ float L[];
    const YZLds g = yz_geometry(a);
    const int kx = blockIdx.x, gout = blockIdx.y;
    const int PL = 2 * (g.PX > g.PT ? g.PX : g.PT);
    float *X = L, *T = L + PL;
    const int P2 = 2 * a.PS;
    const int M = a.M, aa = gout / 3, d = gout % 3;
    for (int i = threadIdx.x; i < a.PS; i += blockDim.x) {
        const int z = fdiv(i, a.div_ny), y = i - z * a.ny;
        const int o = z * g.RY + y;
        float re = 0.f, im = 0.f;
        for (int b = 0; b < M; ++b) {
            const int lo = aa < b ? aa : b, hi = aa < b ? b : aa;
            const int pr = lo * M - (lo * (lo - 1)) / 2 + (hi - lo);
            const float sv = a.S[(long long)(pr * 3 + d) * a.Sp + (long long)kx * a.PS + i];
            const float *__restrict__ F = a.in + b * a.FSTR + (long long)kx * P2;
            re -= sv * F[a.PS + i];
            im += sv * F[i];
        }
        X[o] = re;
        X[g.PX + o] = im;
    }
    __syncthreads();
    yz_stage_y(g, a.wy, X, T);
    __syncthreads();
    yz_stage_z(g, a.wz, T, X);
    __syncthreads();
    float *__restrict__ dst = a.out + gout * a.FSTR + (long long)kx * P2;
    for (int i = threadIdx.x; i < P2; i += blockDim.x) {
        const int p = i >= a.PS ? 1 : 0;
        const int r = i - p * a.PS, z = fdiv(r, a.div_ny), y = r - z * a.ny;
        dst[i] = X[p * g.PX + z * g.RY + y];
    }
}

// LDS bytes of the y/z kernels: two padded complex planes.  They run beside
// the first gather's tiles and must fit in what those leave of a CU's LDS,
// so the DFT matrices stay in global memory (L2-resident): copied into LDS
// they tripled the footprint and the overlapped step took 16 % longer.
constexpr size_t kYZLdsMax = 150 * 1024;

size_t yz_lds_bytes(int ny, int nz)
{
    const size_t PX = (size_t)nz * (ny + 1), PT = (size_t)ny * (nz + 1);
    const size_t PL = 2 * (PX > PT ? PX : PT);
    return sizeof(float) * 2 * PL;
}

bool SpectralPlan::fused_fits(int ny, int nz, int M)
{
    (void)M;
    return yz_lds_bytes(ny, nz) <= kYZLdsMax && (long long)ny * nz < (1LL << 30);
}

// ------------------------------------------------------------------ plan
namespace {

MatAddr dense(const float *base, long long ld)
{
    MatAddr m{};
    m.base = const_cast<float *>(base);
    m.t_div = kPlain; m.r_div = kPlain; m.c_div = kPlain;
    m.s_rlo = ld; m.s_clo = 1;
    return m;
}

}  // namespace

void SpectralPlan::x_forward(const float *real_in, int nfields, float *s1, hipStream_t st, bool on_transform_grid) const
{
    // rows (z, y) of each field; output columns (plane, kx) into [f][kx][p][z][y]
    const int rows_y = on_transform_grid ? ny : nyr;
    GemmDesc gx{};
    gx.M = nz * rows_y; gx.N = 2 * nkx; gx.K = nx; gx.batch = nfields;
    gx.A = dense(real_in, nx); gx.A.s_tlo = (long long)nx * rows_y * nz;
    gx.B = dense(wxf, 2 * nkx);
    gx.C = dense(s1, 1); gx.C.s_tlo = 2 * Sp; gx.C.c_div = nkx; gx.C.s_chi = (long long)ny * nz;
    gx.C.s_clo = 2LL * ny * nz;
    if (rows_y != ny) {   // row (z, y) of the lattice -> z ny + y of the padded plane
        gx.C.r_div = rows_y; gx.C.s_rhi = ny; gx.C.s_rlo = 1;
    }
    launch_gemm(gx, st);
}

void SpectralPlan::x_inverse(const float *s2, int nfields, float *real_out, hipStream_t st) const
{
    // lattice rows only: row (z, y) reads z ny + y of the padded plane
    GemmDesc gx{};
    gx.M = nz * nyr; gx.N = nx; gx.K = 2 * nkx; gx.batch = nfields;
    gx.A = dense(s2, 1); gx.A.s_tlo = 2 * Sp; gx.A.c_div = nkx; gx.A.s_chi = (long long)ny * nz;
    gx.A.s_clo = 2LL * ny * nz;
    if (nyr != ny) {
        gx.A.r_div = nyr; gx.A.s_rhi = ny; gx.A.s_rlo = 1;
    }
    gx.B = dense(wxi, nx);
    gx.C = dense(real_out, nx); gx.C.s_tlo = (long long)nx * nyr * nz;
    launch_gemm(gx, st);
}

namespace {
FastDiv make_fastdiv(int d)
{
    int l = 0;
    while ((1LL << l) < d) ++l;
    const unsigned long long two32 = 1ULL << 32;
    FastDiv f;
    f.l = l;
    f.m = (unsigned)((two32 * ((1ULL << l) - (unsigned long long)d)) / (unsigned long long)d + 1);
    return f;
}
}  // namespace

void SpectralPlan::launch_yz(int mode, int nfields, const float *in, float *out, hipStream_t st) const
{
    YZArgs a{};
    a.ny = ny; a.nz = nz; a.M = M; a.mode = mode;
    a.ny_real = nyr;
    a.PS = ny * nz; a.Sp = Sp; a.FSTR = 2 * Sp;
    a.div_ny = make_fastdiv(ny);
    a.in = in; a.out = out; a.S = S;
    a.scale = 1.0f / (float)((double)nx * ny * nz);
    const size_t lds = yz_lds_bytes(ny, nz);
    if (mode == 2) {
        a.wy = wyi; a.wz = wzi;
        hipLaunchKernelGGL(k_yz_inverse, dim3(nkx, 3 * M), dim3(256), lds, st, a);
    } else {
        a.wy = wyf; a.wz = wzf;
        hipLaunchKernelGGL(k_yz_forward, dim3(nkx, nfields), dim3(256), lds, st, a);
    }
}

bool SpectralPlan::prepare(int ny, int nz, int M)
{
    (void)ny;
    (void)nz;
    (void)M;
    // the largest dynamic LDS any plan may ask for: plans of other sizes in
    // the same process then never find a smaller limit set by this one
    const int bytes = (int)kYZLdsMax;
    for (const void *fn : {(const void *)k_yz_forward, (const void *)k_yz_inverse})
        if (hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, bytes) != hipSuccess) return false;
    return true;
}

void SpectralPlan::build_spectrum(const float *placed, float *s1, float *s2, hipStream_t st) const
{
    (void)s2;
    const int nf = 3 * P;
    x_forward(placed, nf, s1, st, true);
    launch_yz(0, nf, s1, S, st);
}

void SpectralPlan::apply(const float *n, float *s1, float *s2, float *tail, hipStream_t st) const
{
    x_forward(n, M, s1, st);
    launch_yz(1, M, s1, s2, st);        // spectra of the M densities
    launch_yz(2, 3 * M, s2, s1, st);    // products and inverse y/z stages, 3M components
    x_inverse(s1, 3 * M, tail, st);
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
