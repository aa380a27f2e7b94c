// Spectral evaluation of the attractive field (see spectral.hip).
// Applicable when two (y, z) planes of the box fit the LDS budget
// (SpectralPlan::fused_fits); otherwise the field is summed directly.
#pragma once

#include <hip/hip_runtime.h>

#include <vector>

namespace mlb {

// Element (r, c) of batch t lives at
//   base + (t / t_div) s_thi + (t % t_div) s_tlo + (r / r_div) s_rhi + (r % r_div) s_rlo
//        + (c / c_div) s_chi + (c % c_div) s_clo
struct MatAddr {
    float *base;
    int t_div, r_div, c_div;
    long long s_thi, s_tlo, s_rhi, s_rlo, s_chi, s_clo;
};

struct GemmDesc {
    int M, N, K, batch;
    MatAddr A, B, C;
};

void launch_gemm(const GemmDesc &g, hipStream_t st);

struct SpectralPlan {
    int nx = 0, ny = 0, nz = 0, nkx = 0, M = 0, P = 0;
    int nyr = 0;                  // lattice ny; ny is the transform length (zero-padded past walls)
    long long Sz = 0, Sp = 0;     // ny * nkx,  nz * ny * nkx
    // device matrices (row-major)
    const float *wxf = nullptr;   // nx x 2nkx        [cos | -sin]
    const float *wxi = nullptr;   // 2nkx x nx        complex-to-real
    const float *wyf = nullptr, *wyi = nullptr;   // 2ny x 2ny
    const float *wzf = nullptr, *wzi = nullptr;   // 2nz x 2nz
    float *S = nullptr;           // [P][3][Sp] kernel sine spectra / N

    // Host tables: DFT matrices in the order wxf, wxi, wyf, wyi, wzf, wzi.
    static std::vector<float> dft_x_forward(int nx);
    static std::vector<float> dft_x_inverse(int nx);
    static std::vector<float> dft_block(int L, bool inverse);

    // x stage as batched GEMMs; spectra in [field][kx][re|im][z][y], y < ny;
    // lattice fields fill y < nyr (the rest is zero-padding), the placed
    // kernels (on_transform_grid) every y < ny
    void x_forward(const float *real_in, int nfields, float *s1, hipStream_t st, bool on_transform_grid = false) const;
    void x_inverse(const float *s2, int nfields, float *real_out, hipStream_t st) const;
    // y/z stages, one workgroup per kx plane and field: mode 0 forward -> sine
    // spectra of the kernels, 1 forward -> spectra, 2 products + inverse (3M outputs)
    void launch_yz(int mode, int nfields, const float *in, float *out, hipStream_t st) const;
    static bool fused_fits(int ny, int nz, int M);
    static bool prepare(int ny, int nz, int M);
    // placed: [P][3][N] kernels w_ab on the periodic grid (sum over wrapped offsets)
    void build_spectrum(const float *placed, float *s1, float *s2, hipStream_t st) const;
    // tail [M][3][N] = sum_b K_ab * n_b for density fields n [M][N]
    void apply(const float *n, float *s1, float *s2, float *tail, hipStream_t st) const;
};

}  // namespace mlb
