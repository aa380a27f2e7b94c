// Internal launch interface of the closure network kernels (cnn.hip).
// Activations are channel-last bfloat16 [site][C]; C padded to 16 or 32.
#pragma once

#include <hip/hip_runtime.h>

namespace mlb {

struct CnnShape {
    int nx, ny, nz;
    long long N;
};

// Layer l (0..3) has packed (in, out) channels (16, 32), (32, 32), (32, 32), (32, 16);
// layer 0's 16 input slots hold its 14 inputs, then zeros.
constexpr int kNetLayers = 4;
constexpr int kNetIn = 14, kNetHidden = 32, kNetOut = 6;
constexpr int kNetInSlots = 16;
inline int net_cip(int l) { return l == 0 ? kNetInSlots : 32; }
inline int net_cop(int l) { return l == 3 ? 16 : 32; }
inline int net_cin(int l) { return l == 0 ? kNetIn : kNetHidden; }
inline int net_cout(int l) { return l == 3 ? kNetOut : kNetHidden; }

// raise the dynamic-LDS limit of the convolution kernels (once per process)
bool cnn_prepare();
// z (float32, may be null) = conv(in) + b; a (bf16, may be null) = act ? silu(z) : z
void cnn_conv_fwd(int layer, const CnnShape &sh, const unsigned short *in, const unsigned short *W, const float *b,
                  float *z, unsigned short *a, int act, hipStream_t st);
// last layer straight into lattice fields: Nf [6][N] = (conv(in) + b) * scale
void cnn_conv_out_fields(const CnnShape &sh, const unsigned short *in, const unsigned short *W, const float *b,
                         float scale, float *Nf, hipStream_t st);
// gin = conv^T(gout) * silu'(zin)   (layers 1..3)
void cnn_conv_dgrad(int layer, const CnnShape &sh, const unsigned short *gout, const unsigned short *WT,
                    const float *zin, unsigned short *gin, hipStream_t st);
// writes 27 COP CIP + COP floats at gw: the weight gradient [27][COP][CIP]
// followed by the bias gradient [COP]; part holds ceil(N / 256) partial rows
void cnn_conv_wgrad(int layer, const CnnShape &sh, const unsigned short *gout, const unsigned short *ain, float *part,
                    float *gw, hipStream_t st);
size_t cnn_wgrad_part_floats(int layer, long long N);
// wgt * MSE over N x 6 outputs: gout [N][16] bf16, loss_part [ceil(N / 256)]
void cnn_mse(const CnnShape &sh, float wgt, const float *y, const float *tg, unsigned short *gout, float *loss_part,
             hipStream_t st);
// one Adam step (1-based `step`); the decay constants enter in float64 so
// that 1 - b and 1 - b^t carry no float32 rounding of b
void cnn_adam(int n, int cop, int cip, int cout, int cin, float *w, const float *gw, float *m, float *v, float lr,
              double b1, double b2, double eps, int step, unsigned short *wb, unsigned short *wt, float *b,
              const float *gb, float *mb, float *vb, hipStream_t st);
void cnn_cast(int n, int cop, int cip, const float *w, unsigned short *wb, unsigned short *wt, hipStream_t st);
// lattice fields -> network input: (n_a / n_ref - 1, j_a / j_ref, c_s^2 grad n_a / f_ref)
// (central differences on the periodic grid, c_s^2 = 1/3)
void cnn_pack_input(const CnnShape &sh, const float *n, const float *j, float n_ref, float j_ref, float f_ref,
                    unsigned short *x, hipStream_t st);
// channel-first float32 [14][N] -> packed input [N][16]
void cnn_pack_x(const CnnShape &sh, const float *xf, unsigned short *x, hipStream_t st);
// channel-first float32 input [14][N] and target [6][N] = Nf / f_ref from lattice fields
void cnn_fields_x(const CnnShape &sh, const float *n, const float *j, float n_ref, float j_ref, const float *Nf,
                  float f_ref, float *xf, float *tf, hipStream_t st);
// channel-first [6][N] / f_ref -> [N][6]
void cnn_pack_target(const CnnShape &sh, const float *Nf, float f_ref, float *tg, hipStream_t st);
// y [N][16] -> channel-first [6][N] * f_ref
void cnn_unpack_output(const CnnShape &sh, const float *y, float f_ref, float *Nf, hipStream_t st);
// squared-error partials: part[2w] = sum (a - b)^2, part[2w + 1] = sum b^2
void cnn_err_partial(long long n, const float *a, const float *b, double *part, int nparts, hipStream_t st);
// training pool of `count` samples: part[s * nparts + p] = partial sums of
// squares of the `len` floats at base + s stride (float64)
void cnn_pool_sumsq(const float *base, long long stride, long long len, int count, double *part, int nparts,
                    hipStream_t st);
// base + s stride, len floats, times mul, for every sample s
void cnn_pool_scale(float *base, long long stride, long long len, int count, float mul, hipStream_t st);

}  // namespace mlb
