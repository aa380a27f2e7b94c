// Learned force closure: a 3D convolutional network on the lattice.
//
// It maps the local state of a binary mixture (densities n_a and momentum
// densities j_a, scaled) to the force densities N_a = n_a Phi_a of the
// kinetic equation (Sec. 2, eq. evolution; the field of Sec. 3,
// eq. splitforce).  Four 3x3x3 convolutions on the periodic lattice,
// channels 8 -> 32 -> 32 -> 32 -> 6, SiLU after the first three.
//
// Layout: activations channel-last [site][C] (C padded to a multiple of
// 16), weights [tap][C_out][C_in] in bfloat16, accumulation in float32 on
// the matrix cores (v_mfma_f32_16x16x16bf16_1k: 16 x 16 x 16 per wave).
//
// The first layer runs in split bfloat16: every input value x is carried as
// hi = bf16(x) and lo = bf16(x - hi), every weight w as hi and lo the same
// way, and the 32 packed input channels [x_hi | x_lo | x_hi | 0] meet the
// weight row [w_hi | w_hi | w_lo | 0], so one contraction gives
// w_hi x_hi + w_hi x_lo + w_lo x_hi, about 16 significant bits.  The
// force is a spatial derivative of fields whose local values it barely
// changes; with 8-bit inputs or first-layer weights the rounding of the
// undifferentiated part would swamp it.
// Lane layout (one block): A[i][4g .. 4g+3] in lane i + 16g, B[4g .. 4g+3][j]
// in lane j + 16g, D[4g + v][j] in lane j + 16g, element v.
//
// Kernels: convolution forward (bias, optional SiLU, stores the
// pre-activation for the backward pass), data gradient (transposed
// weights, times SiLU' of the previous pre-activation), weight and bias
// gradients (per-workgroup partial sums in fixed order, then a second
// reduction pass), MSE loss gradient, Adam on float32 master weights, and
// the packing of lattice fields into network inputs and outputs.
#include <hip/hip_runtime.h>

#include <cmath>

#include "cnn.h"

namespace mlb {

typedef short v4s __attribute__((ext_vector_type(4)));
typedef float v4f __attribute__((ext_vector_type(4)));

__device__ inline unsigned short f2bf(float f)
{
    // round to nearest even
    unsigned int u = __float_as_uint(f);
    if ((u & 0x7f800000u) == 0x7f800000u) return (unsigned short)(u >> 16);   // inf / nan
    u += 0x7fffu + ((u >> 16) & 1u);
    return (unsigned short)(u >> 16);
}
__device__ inline float bf2f(unsigned short h) { return __uint_as_float(((unsigned int)h) << 16); }

__device__ inline float sigm(float z) { return 1.f / (1.f + __expf(-z)); }

struct Grid3 {
    int nx, ny, nz;
};

__device__ inline long long shift_site(const Grid3 &g, int x, int y, int z, int dx, int dy, int dz)
{
    int xx = x + dx, yy = y + dy, zz = z + dz;
    xx = xx < 0 ? xx + g.nx : (xx >= g.nx ? xx - g.nx : xx);
    yy = yy < 0 ? yy + g.ny : (yy >= g.ny ? yy - g.ny : yy);
    zz = zz < 0 ? zz + g.nz : (zz >= g.nz ? zz - g.nz : zz);
    return ((long long)zz * g.ny + yy) * g.nx + xx;
}

// ------------------------------------------------------------ forward
// out[s][co] = b[co] + sum_t sum_ci W[t][co][ci] in[s + d_t][ci]
// Block: 4 waves x 64 sites; each wave: COP/16 channel blocks x 4 site blocks.
template <int CIP, int COP>
__global__ void __launch_bounds__(256) k_conv_fwd(Grid3 g, long long N, const unsigned short *__restrict__ in,
                                                 const unsigned short *__restrict__ W, const float *__restrict__ bias,
                                                 float *__restrict__ zout, unsigned short *__restrict__ aout, int act)
{
    constexpr int CB = COP / 16, KB = CIP / 16;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, li = lane & 15, gq = lane >> 4;
    const long long s0 = (long long)blockIdx.x * 256 + wave * 64;
    int sx[4], sy[4], sz[4];
    bool ok[4];
    for (int sb = 0; sb < 4; ++sb) {
        const long long s = s0 + sb * 16 + li;
        ok[sb] = s < N;
        const long long ss = ok[sb] ? s : 0;
        sx[sb] = (int)(ss % g.nx);
        sy[sb] = (int)((ss / g.nx) % g.ny);
        sz[sb] = (int)(ss / ((long long)g.nx * g.ny));
    }
    v4f acc[CB][4];
    for (int c = 0; c < CB; ++c)
        for (int sb = 0; sb < 4; ++sb) acc[c][sb] = v4f{0.f, 0.f, 0.f, 0.f};
    for (int t = 0; t < 27; ++t) {
        const int dz = t / 9 - 1, dy = (t / 3) % 3 - 1, dx = t % 3 - 1;
        long long nb[4];
        for (int sb = 0; sb < 4; ++sb) nb[sb] = shift_site(g, sx[sb], sy[sb], sz[sb], dx, dy, dz);
        for (int kb = 0; kb < KB; ++kb) {
            v4s a[CB], b[4];
            for (int c = 0; c < CB; ++c)
                a[c] = *reinterpret_cast<const v4s *>(W + ((long long)t * COP + c * 16 + li) * CIP + kb * 16 + 4 * gq);
            for (int sb = 0; sb < 4; ++sb)
                b[sb] = *reinterpret_cast<const v4s *>(in + nb[sb] * CIP + kb * 16 + 4 * gq);
            for (int c = 0; c < CB; ++c)
                for (int sb = 0; sb < 4; ++sb)
                    acc[c][sb] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a[c], b[sb], acc[c][sb], 0, 0, 0);
        }
    }
    for (int c = 0; c < CB; ++c)
        for (int sb = 0; sb < 4; ++sb) {
            if (!ok[sb]) continue;
            const long long s = s0 + sb * 16 + li;
            for (int v = 0; v < 4; ++v) {
                const int co = c * 16 + 4 * gq + v;
                const float z = acc[c][sb][v] + bias[co];
                if (zout) zout[s * COP + co] = z;
                const float av = act ? z * sigm(z) : z;
                if (aout) aout[s * COP + co] = f2bf(av);
            }
        }
}

// ------------------------------------------------------- data gradient
// gin[s][ci] = (sum_t sum_co W[t][co][ci] gout[s - d_t][co]) * silu'(zin[s][ci])
// WT = weights transposed to [t][ci][co].
template <int CIP, int COP>
__global__ void __launch_bounds__(256) k_conv_dgrad(Grid3 g, long long N, const unsigned short *__restrict__ gout,
                                                   const unsigned short *__restrict__ WT,
                                                   const float *__restrict__ zin, unsigned short *__restrict__ gin)
{
    constexpr int CB = CIP / 16, KB = COP / 16;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, li = lane & 15, gq = lane >> 4;
    const long long s0 = (long long)blockIdx.x * 256 + wave * 64;
    int sx[4], sy[4], sz[4];
    bool ok[4];
    for (int sb = 0; sb < 4; ++sb) {
        const long long s = s0 + sb * 16 + li;
        ok[sb] = s < N;
        const long long ss = ok[sb] ? s : 0;
        sx[sb] = (int)(ss % g.nx);
        sy[sb] = (int)((ss / g.nx) % g.ny);
        sz[sb] = (int)(ss / ((long long)g.nx * g.ny));
    }
    v4f acc[CB][4];
    for (int c = 0; c < CB; ++c)
        for (int sb = 0; sb < 4; ++sb) acc[c][sb] = v4f{0.f, 0.f, 0.f, 0.f};
    for (int t = 0; t < 27; ++t) {
        const int dz = t / 9 - 1, dy = (t / 3) % 3 - 1, dx = t % 3 - 1;
        long long nb[4];
        for (int sb = 0; sb < 4; ++sb) nb[sb] = shift_site(g, sx[sb], sy[sb], sz[sb], -dx, -dy, -dz);
        for (int kb = 0; kb < KB; ++kb) {
            v4s a[CB], b[4];
            for (int c = 0; c < CB; ++c)
                a[c] = *reinterpret_cast<const v4s *>(WT + ((long long)t * CIP + c * 16 + li) * COP + kb * 16 + 4 * gq);
            for (int sb = 0; sb < 4; ++sb)
                b[sb] = *reinterpret_cast<const v4s *>(gout + nb[sb] * COP + kb * 16 + 4 * gq);
            for (int c = 0; c < CB; ++c)
                for (int sb = 0; sb < 4; ++sb)
                    acc[c][sb] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a[c], b[sb], acc[c][sb], 0, 0, 0);
        }
    }
    for (int c = 0; c < CB; ++c)
        for (int sb = 0; sb < 4; ++sb) {
            if (!ok[sb]) continue;
            const long long s = s0 + sb * 16 + li;
            for (int v = 0; v < 4; ++v) {
                const int ci = c * 16 + 4 * gq + v;
                const float z = zin[s * CIP + ci];
                const float sg = sigm(z);
                gin[s * CIP + ci] = f2bf(acc[c][sb][v] * (sg * (1.f + z * (1.f - sg))));
            }
        }
}

// ----------------------------------------------------- weight gradient
// part[wg][t][co][ci] = sum_{s in chunk} gout[s][co] ain[s + d_t][ci], plus
// bias part[wg][bias][co] = sum_s gout[s][co].  Chunk = 256 consecutive
// sites per workgroup, staged in LDS as [co][site] and [ci][site] so the
// MFMA operands (4 consecutive sites per lane) are contiguous.
template <int CIP, int COP>
__global__ void __launch_bounds__(256) k_conv_wgrad(Grid3 g, long long N, const unsigned short *__restrict__ gout,
                                                   const unsigned short *__restrict__ ain, float *__restrict__ part)
{
    __shared__ unsigned short Gs[COP][256 + 8];
    __shared__ unsigned short As[CIP][256 + 8];
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6, li = lane & 15, gq = lane >> 4;
    const long long s0 = (long long)blockIdx.x * 256;
    const long long me = s0 + tid;
    const bool ok = me < N;
    int mx = 0, my = 0, mz = 0;
    if (ok) {
        mx = (int)(me % g.nx);
        my = (int)((me / g.nx) % g.ny);
        mz = (int)(me / ((long long)g.nx * g.ny));
    }
    for (int c = 0; c < COP; ++c) Gs[c][tid] = ok ? gout[me * COP + c] : (unsigned short)0;
    constexpr int BM = COP / 16, BN = CIP / 16, NBLK = BM * BN;
    float *out = part + (long long)blockIdx.x * (27 * COP * CIP + COP);
    for (int t = 0; t < 27; ++t) {
        const int dz = t / 9 - 1, dy = (t / 3) % 3 - 1, dx = t % 3 - 1;
        __syncthreads();
        if (ok) {
            const long long nb = shift_site(g, mx, my, mz, dx, dy, dz);
            for (int c = 0; c < CIP; ++c) As[c][tid] = ain[nb * CIP + c];
        } else {
            for (int c = 0; c < CIP; ++c) As[c][tid] = 0;
        }
        __syncthreads();
        for (int blk = wave; blk < NBLK; blk += 4) {
            const int bi = blk / BN, bj = blk % BN;
            v4f acc = v4f{0.f, 0.f, 0.f, 0.f};
            for (int k0 = 0; k0 < 256; k0 += 16) {
                v4s a, b;
                for (int e = 0; e < 4; ++e) {
                    a[e] = (short)Gs[bi * 16 + li][k0 + 4 * gq + e];
                    b[e] = (short)As[bj * 16 + li][k0 + 4 * gq + e];
                }
                acc = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a, b, acc, 0, 0, 0);
            }
            for (int v = 0; v < 4; ++v) {
                const int co = bi * 16 + 4 * gq + v, ci = bj * 16 + li;
                out[((long long)t * COP + co) * CIP + ci] = acc[v];
            }
        }
    }
    __syncthreads();
    if (tid < COP) {
        float sb = 0.f;
        for (int k = 0; k < 256; ++k) sb += bf2f(Gs[tid][k]);
        out[27 * COP * CIP + tid] = sb;
    }
}

// sum the per-workgroup partial rows in order: out[i] = sum_w part[w][i]
__global__ void k_sum_rows(const float *__restrict__ part, int nrows, int len, float *__restrict__ out)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= len) return;
    float s = 0.f;
    for (int w = 0; w < nrows; ++w) s += part[(long long)w * len + i];
    out[i] = s;
}

// ------------------------------------------------------------- loss
// y [s][COP] (float32 pre-activation of the last layer), target [s][NOUT];
// loss = wgt * mean (y - t)^2; g = wgt 2 (y - t) / (N NOUT) as bf16 [s][COP];
// loss partials per block.
__global__ void k_mse(long long N, int COP, int NOUT, float wgt, const float *__restrict__ y,
                      const float *__restrict__ tg, unsigned short *__restrict__ gout, float *__restrict__ loss_part)
{
    __shared__ float red[256];
    const long long s = (long long)blockIdx.x * 256 + threadIdx.x;
    float l = 0.f;
    if (s < N) {
        const float inv = wgt * 2.f / ((float)N * (float)NOUT);
        for (int c = 0; c < COP; ++c) {
            float gv = 0.f;
            if (c < NOUT) {
                const float d = y[s * COP + c] - tg[s * NOUT + c];
                l += d * d;
                gv = inv * d;
            }
            gout[s * COP + c] = f2bf(gv);
        }
    }
    red[threadIdx.x] = l;
    __syncthreads();
    for (int o = 128; o > 0; o >>= 1) {
        if (threadIdx.x < o) red[threadIdx.x] += red[threadIdx.x + o];
        __syncthreads();
    }
    if (threadIdx.x == 0) loss_part[blockIdx.x] = wgt * red[0];
}

// ------------------------------------------------------------- Adam
// master [t][co][ci] float32 (padded layout), grads same layout; refreshes
// the bf16 copies W [t][co][ci] and WT [t][ci][co].  Padded entries stay 0.
// split (first layer, CIP = 4 cin): master entries ci < cin; the gradient of
// w is that of its x_hi and x_lo slots, and the bf16 row gets w_hi, w_hi,
// w_lo, 0 in slots ci, ci + cin, ci + 2 cin, ci + 3 cin.
struct AdamConst {
    float lr, b1, b2, omb1, omb2, c1, c2, eps;   // omb = 1 - b, c = 1 - b^t (formed in float64)
};

__device__ inline void store_split(unsigned short *wb, int i, int cin, float w)
{
    const unsigned short hi = f2bf(w);
    wb[i] = hi;
    wb[i + cin] = hi;
    wb[i + 2 * cin] = f2bf(w - bf2f(hi));
    wb[i + 3 * cin] = 0;
}

__global__ void k_adam(int n, int COP, int CIP, int cout, int cin, int split, float *__restrict__ w,
                       const float *__restrict__ gw, float *__restrict__ m, float *__restrict__ v, AdamConst k,
                       unsigned short *__restrict__ wb, unsigned short *__restrict__ wt)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const int t = i / (COP * CIP), r = i - t * COP * CIP, co = r / CIP, ci = r - co * CIP;
    if (split && ci >= cin) return;                // written by the owner of slot ci % cin
    if (co >= cout || ci >= cin) {
        wb[i] = 0;
        wt[((long long)t * CIP + ci) * COP + co] = 0;
        return;
    }
    const float gi = split ? gw[i] + gw[i + cin] : gw[i];
    const float mi = k.b1 * m[i] + k.omb1 * gi;
    const float vi = k.b2 * v[i] + k.omb2 * gi * gi;
    m[i] = mi;
    v[i] = vi;
    const float wi = w[i] - k.lr * (mi / k.c1) / (sqrtf(vi / k.c2) + k.eps);
    w[i] = wi;
    if (split) {
        store_split(wb, i, cin, wi);
        return;
    }
    wb[i] = f2bf(wi);
    wt[((long long)t * CIP + ci) * COP + co] = f2bf(wi);
}

__global__ void k_adam_bias(int n, float *__restrict__ b, const float *__restrict__ gb, float *__restrict__ m,
                            float *__restrict__ v, AdamConst k)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const float mi = k.b1 * m[i] + k.omb1 * gb[i];
    const float vi = k.b2 * v[i] + k.omb2 * gb[i] * gb[i];
    m[i] = mi;
    v[i] = vi;
    b[i] = b[i] - k.lr * (mi / k.c1) / (sqrtf(vi / k.c2) + k.eps);
}

// refresh bf16 copies from float32 masters (after loading weights)
__global__ void k_cast_weights(int n, int COP, int CIP, int cin, int split, const float *__restrict__ w,
                               unsigned short *__restrict__ wb, unsigned short *__restrict__ wt)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const int t = i / (COP * CIP), r = i - t * COP * CIP, co = r / CIP, ci = r - co * CIP;
    if (split) {
        if (ci < cin) store_split(wb, i, cin, w[i]);
        return;
    }
    wb[i] = f2bf(w[i]);
    wt[((long long)t * CIP + ci) * COP + co] = f2bf(w[i]);
}

// ---------------------------------------------------------- packing
// split first-layer input of one site: x[0..31] = [hi(v) | lo(v) | hi(v) | 0]
__device__ inline void store_input(unsigned short *__restrict__ x, const float v[8])
{
    for (int c = 0; c < 8; ++c) {
        const unsigned short hi = f2bf(v[c]);
        x[c] = hi;
        x[8 + c] = f2bf(v[c] - bf2f(hi));
        x[16 + c] = hi;
        x[24 + c] = 0;
    }
}

// network input of site s: (n_0, n_1) / n_ref - 1, (j_0, j_1) / j_ref
__global__ void k_pack_input(long long N, const float *__restrict__ n, const float *__restrict__ j, float n_ref,
                             float j_ref, unsigned short *__restrict__ x)
{
    const long long s = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= N) return;
    float v[8];
    v[0] = n[s] / n_ref - 1.f;
    v[1] = n[N + s] / n_ref - 1.f;
    for (int d = 0; d < 3; ++d) {
        v[2 + d] = j[d * N + s] / j_ref;
        v[5 + d] = j[(3 + d) * N + s] / j_ref;
    }
    store_input(x + s * 32, v);
}

// input from channel-first float32 xf [8][N]
__global__ void k_pack_x(long long N, const float *__restrict__ xf, unsigned short *__restrict__ x)
{
    const long long s = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= N) return;
    float v[8];
    for (int c = 0; c < 8; ++c) v[c] = xf[c * N + s];
    store_input(x + s * 32, v);
}

// channel-first float32 network input and target from lattice fields:
// xf[c][s] as in k_pack_input, tf[c][s] = N_c(s) / f_ref
__global__ void k_fields_x(long long N, const float *__restrict__ n, const float *__restrict__ j, float n_ref,
                           float j_ref, const float *__restrict__ Nf, float f_ref, float *__restrict__ xf,
                           float *__restrict__ tf)
{
    const long long s = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= N) return;
    xf[s] = n[s] / n_ref - 1.f;
    xf[N + s] = n[N + s] / n_ref - 1.f;
    for (int d = 0; d < 3; ++d) {
        xf[(2 + d) * N + s] = j[d * N + s] / j_ref;
        xf[(5 + d) * N + s] = j[(3 + d) * N + s] / j_ref;
    }
    for (int c = 0; c < 6; ++c) tf[c * N + s] = Nf[c * N + s] / f_ref;
}

// target[s][3a + d] = N_a,d(s) / f_ref
__global__ void k_pack_target(long long N, const float *__restrict__ Nf, float f_ref, float *__restrict__ tg)
{
    const long long s = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= N) return;
    for (int c = 0; c < 6; ++c) tg[s * 6 + c] = Nf[c * N + s] / f_ref;
}

// Nf[c][s] = y[s][c] f_ref  (c = 3a + d)
__global__ void k_unpack_output(long long N, int COP, const float *__restrict__ y, float f_ref, float *__restrict__ Nf)
{
    const long long s = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= N) return;
    for (int c = 0; c < 6; ++c) Nf[c * N + s] = y[s * COP + c] * f_ref;
}

// ||a - b||^2 and ||b||^2 partials over n floats (closure error check)
__global__ void k_err_partial(long long n, const float *__restrict__ a, const float *__restrict__ b,
                              double *__restrict__ part)
{
    __shared__ double r0[256], r1[256];
    double e = 0.0, w = 0.0;
    for (long long i = (long long)blockIdx.x * 256 + threadIdx.x; i < n; i += (long long)gridDim.x * 256) {
        const double d = (double)a[i] - (double)b[i];
        e += d * d;
        w += (double)b[i] * (double)b[i];
    }
    r0[threadIdx.x] = e;
    r1[threadIdx.x] = w;
    __syncthreads();
    for (int o = 128; o > 0; o >>= 1) {
        if (threadIdx.x < o) {
            r0[threadIdx.x] += r0[threadIdx.x + o];
            r1[threadIdx.x] += r1[threadIdx.x + o];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        part[2 * blockIdx.x] = r0[0];
        part[2 * blockIdx.x + 1] = r1[0];
    }
}

// ------------------------------------------------------------ launches
namespace {
inline unsigned nblocks(long long n, int b = 256) { return (unsigned)((n + b - 1) / b); }
}

void cnn_conv_fwd(int layer, const CnnShape &sh, const unsigned short *in, const unsigned short *W, const float *b,
                  float *z, unsigned short *a, int act, hipStream_t st)
{
    const Grid3 g{sh.nx, sh.ny, sh.nz};
    const unsigned nb = nblocks(sh.N);
    switch (layer) {
    case 3: hipLaunchKernelGGL((k_conv_fwd<32, 16>), dim3(nb), dim3(256), 0, st, g, sh.N, in, W, b, z, a, act); break;
    default: hipLaunchKernelGGL((k_conv_fwd<32, 32>), dim3(nb), dim3(256), 0, st, g, sh.N, in, W, b, z, a, act); break;
    }
}

void cnn_conv_dgrad(int layer, const CnnShape &sh, const unsigned short *gout, const unsigned short *WT, const float *zin,
                    unsigned short *gin, hipStream_t st)
{
    const Grid3 g{sh.nx, sh.ny, sh.nz};
    const unsigned nb = nblocks(sh.N);
    if (layer == 3) hipLaunchKernelGGL((k_conv_dgrad<32, 16>), dim3(nb), dim3(256), 0, st, g, sh.N, gout, WT, zin, gin);
    else hipLaunchKernelGGL((k_conv_dgrad<32, 32>), dim3(nb), dim3(256), 0, st, g, sh.N, gout, WT, zin, gin);
}

void cnn_conv_wgrad(int layer, const CnnShape &sh, const unsigned short *gout, const unsigned short *ain, float *part,
                    float *gw, hipStream_t st)
{
    const Grid3 g{sh.nx, sh.ny, sh.nz};
    const unsigned nb = nblocks(sh.N);
    int cip = 32, cop = 32;
    switch (layer) {
    case 3: cop = 16; hipLaunchKernelGGL((k_conv_wgrad<32, 16>), dim3(nb), dim3(256), 0, st, g, sh.N, gout, ain, part); break;
    default: hipLaunchKernelGGL((k_conv_wgrad<32, 32>), dim3(nb), dim3(256), 0, st, g, sh.N, gout, ain, part); break;
    }
    const int len = 27 * cop * cip + cop;
    hipLaunchKernelGGL(k_sum_rows, dim3(nblocks(len)), dim3(256), 0, st, part, (int)nb, len, gw);
}

size_t cnn_wgrad_part_floats(int layer, long long N)
{
    return (size_t)nblocks(N) * (size_t)(27 * net_cop(layer) * net_cip(layer) + net_cop(layer));
}

void cnn_mse(const CnnShape &sh, float wgt, const float *y, const float *tg, unsigned short *gout, float *loss_part,
             hipStream_t st)
{
    hipLaunchKernelGGL(k_mse, dim3(nblocks(sh.N)), dim3(256), 0, st, sh.N, 16, 6, wgt, y, tg, gout, loss_part);
}

void cnn_adam(int n, int cop, int cip, int cout, int cin, int split, float *w, const float *gw, float *m, float *v, float lr,
              double b1, double b2, double eps, int step, unsigned short *wb, unsigned short *wt, float *b,
              const float *gb, float *mb, float *vb, hipStream_t st)
{
    const AdamConst k{lr, (float)b1, (float)b2, (float)(1.0 - b1), (float)(1.0 - b2),
                      (float)(1.0 - std::pow(b1, step)), (float)(1.0 - std::pow(b2, step)), (float)eps};
    hipLaunchKernelGGL(k_adam, dim3(nblocks(n)), dim3(256), 0, st, n, cop, cip, cout, cin, split, w, gw, m, v, k, wb,
                       wt);
    hipLaunchKernelGGL(k_adam_bias, dim3(1), dim3(64), 0, st, cop, b, gb, mb, vb, k);
}

void cnn_cast(int n, int cop, int cip, int cin, int split, const float *w, unsigned short *wb, unsigned short *wt,
              hipStream_t st)
{
    hipLaunchKernelGGL(k_cast_weights, dim3(nblocks(n)), dim3(256), 0, st, n, cop, cip, cin, split, w, wb, wt);
}

void cnn_pack_input(const CnnShape &sh, const float *n, const float *j, float n_ref, float j_ref, unsigned short *x,
                    hipStream_t st)
{
    hipLaunchKernelGGL(k_pack_input, dim3(nblocks(sh.N)), dim3(256), 0, st, sh.N, n, j, n_ref, j_ref, x);
}

void cnn_pack_x(const CnnShape &sh, const float *xf, unsigned short *x, hipStream_t st)
{
    hipLaunchKernelGGL(k_pack_x, dim3(nblocks(sh.N)), dim3(256), 0, st, sh.N, xf, x);
}

void cnn_fields_x(const CnnShape &sh, const float *n, const float *j, float n_ref, float j_ref, const float *Nf,
                  float f_ref, float *xf, float *tf, hipStream_t st)
{
    hipLaunchKernelGGL(k_fields_x, dim3(nblocks(sh.N)), dim3(256), 0, st, sh.N, n, j, n_ref, j_ref, Nf, f_ref, xf,
                       tf);
}

void cnn_pack_target(const CnnShape &sh, const float *Nf, float f_ref, float *tg, hipStream_t st)
{
    hipLaunchKernelGGL(k_pack_target, dim3(nblocks(sh.N)), dim3(256), 0, st, sh.N, Nf, f_ref, tg);
}

void cnn_unpack_output(const CnnShape &sh, const float *y, float f_ref, float *Nf, hipStream_t st)
{
    hipLaunchKernelGGL(k_unpack_output, dim3(nblocks(sh.N)), dim3(256), 0, st, sh.N, 16, y, f_ref, Nf);
}

void cnn_err_partial(long long n, const float *a, const float *b, double *part, int nparts, hipStream_t st)
{
    hipLaunchKernelGGL(k_err_partial, dim3(nparts), dim3(256), 0, st, n, a, b, part);
}

}  // namespace mlb
