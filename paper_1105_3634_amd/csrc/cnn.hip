// Learned force closure: a 3D convolutional network on the lattice.
//
// It maps the local state of a binary mixture to the force densities
// N_a = n_a Phi_a of the kinetic equation (Sec. 2, eq. evolution; the field
// of Sec. 3, eq. splitforce).  Four 3x3x3 convolutions on the periodic
// lattice, channels 14 -> 32 -> 32 -> 32 -> 6, SiLU after the first three.
// The 14 inputs of a site are its scaled densities n_a / n_ref - 1, its
// momentum densities j_a / j_ref and the lattice pressure gradients
// c_s^2 grad n_a / f_ref (central differences, c_s^2 = 1/3).  The force is
// dominated by derivatives of the densities; given as inputs at the scale
// of the force they need no more than bfloat16's 8 bits, where a network
// that had to difference the densities itself would lose them to the
// rounding of the undifferentiated values.
//
// Layout: activations channel-last [site][C] (C padded to a multiple of
// 16), weights [tap][C_out][C_in] in bfloat16, accumulation in float32 on
// the matrix cores.  Forward and data-gradient convolutions run on LDS
// tiles with v_mfma_f32_16x16x32_bf16 (k_conv_tile); the weight gradient
// contracts over sites with v_mfma_f32_16x16x16bf16_1k (k_conv_wgrad).
// 16 x 16 output blocks: D[4g + v][j] in lane j + 16g, element v.
//
// Kernels: convolution forward (bias, optional SiLU, stores the
// pre-activation for the backward pass), data gradient (transposed
// weights, times SiLU' of the previous pre-activation), weight and bias
// gradients (per-workgroup partial sums in fixed order, then a second
// reduction pass), MSE loss gradient, Adam on float32 master weights, and
// the packing of lattice fields into network inputs and outputs.
#include <hip/hip_runtime.h>

#include <cmath>
#include <type_traits>

#include "cnn.h"

namespace mlb {

typedef short v4s __attribute__((ext_vector_type(4)));
typedef float v4f __attribute__((ext_vector_type(4)));

// float -> bfloat16, round to nearest even (v_cvt_pk_bf16_f32)
__device__ inline unsigned short f2bf(float f) { return __builtin_bit_cast(unsigned short, (__bf16)f); }
__device__ inline float bf2f(unsigned short h) { return __uint_as_float(((unsigned int)h) << 16); }

// logistic function with the hardware reciprocal (v_rcp_f32, about 1 ulp):
// its results are rounded to bfloat16 or feed bfloat16 products, so the
// correctly rounded division sequence would buy nothing
__device__ inline float sigm(float z) { return __builtin_amdgcn_rcpf(1.f + __expf(-z)); }

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

// --------------------------------------------- tiled convolution (LDS)
// out[s][o] = sum_t sum_k W[t][o][k] in[s + SGN d_t][k]   (k < KIN, o < OUT)
//   forward (SGN = +1, EPI 0): W = weights [t][co][ci]; z = acc + b -> zout
//     (float32, optional), aout = act ? silu(z) : z (bf16, optional)
//   data gradient (SGN = -1, EPI 1): W = transposed weights [t][ci][co];
//     gin = acc * silu'(zin) (bf16)
//   output layer into lattice fields (SGN = +1, EPI 2): zout[o][s] =
//     (acc + b) * scale for the kNetOut channels, channel-first float32
// Persistent blocks (one per CU) walk 16 x 8 x 4 tiles; within a tile each
// wave owns kWaveRows rows of 16 consecutive x in one z plane (one MFMA site
// block per row) and all OUT channels (2 kWaveRows independent accumulators
// for OUT = 32).
// The layer's weights are staged in LDS once per block; each tile with a
// one-cell halo (18 x 10 x 6 sites) is loaded into registers while the
// previous tile computes, then stored to LDS.  Both are chunk-major: [channel chunk][site] and
// [channel chunk][weight row], a chunk being the CW = KIN / 2 bytes one lane
// feeds to one MFMA, so the 16 lanes of a site block read 16 consecutive
// chunks.
// KIN = 32: v_mfma_f32_16x16x32_bf16, lane j + 16 g holds channels
// 8g..8g+7 of both operands (any fixed lane -> channel assignment shared by
// the two operands gives the same sum); KIN = 16: v_mfma_f32_16x16x16bf16_1k
// with channels 4g..4g+3.
typedef __bf16 v8bf __attribute__((ext_vector_type(8)));

constexpr int kCTX = 16, kCTY = 8, kCTZ = 4;
// Waves per tile block: each wave owns kWaveRows rows of 16 sites in one z
// plane (all rows with 4 waves; half of them with 8, two waves per SIMD so
// that one wave's LDS waits overlap the other's MFMAs).
#ifndef MLB_CONV_WAVES
#define MLB_CONV_WAVES 8
#endif
constexpr int kConvWaves = MLB_CONV_WAVES, kConvThreads = 64 * kConvWaves;
constexpr int kWaveRows = kCTY * kCTZ / kConvWaves, kRowBlocks = kCTY / kWaveRows;
static_assert(kWaveRows * kRowBlocks == kCTY && kRowBlocks * kCTZ == kConvWaves, "waves tile the block");
constexpr int kCHX = kCTX + 2, kCHY = kCTY + 2, kCHZ = kCTZ + 2;
constexpr int kCHS = kCHX * kCHY * kCHZ;
constexpr int kCRows = kCHY * kCHZ;

// Byte stride between the channel-chunk planes of the staged tile.  A
// 16-byte LDS read serves 16 lanes per clock, and consecutive 8-lane blocks
// must fall on opposite halves of the 64 banks (measured): the site block of
// chunk g + 1 (lanes 16 (g + 1) ..) has to start on the same bank as that of
// chunk g, so 16-byte chunk planes are padded to a multiple of 256 bytes
// (1080 sites x 16 bytes = 17280 would put them 128 bytes off).
__host__ __device__ constexpr int conv_plane(int cw) { return cw == 16 ? (kCHS * cw + 255) / 256 * 256 : kCHS * cw; }

__host__ __device__ constexpr int conv_lds(int kin, int out)
{
    return 4 * conv_plane(kin / 2) + 4 * 27 * out * (kin / 2) + 2 * 4 * kCRows + 4 * out;
}

__device__ inline int wrap_cell(int v, int n)
{
    v %= n;
    return v < 0 ? v + n : v;
}

// native vector types (arrays of them stay in registers)
typedef unsigned v4u __attribute__((ext_vector_type(4)));
typedef unsigned v2u __attribute__((ext_vector_type(2)));
template <int CW>
struct Chunk;
template <>
struct Chunk<16> {
    typedef v4u T;
};
template <>
struct Chunk<8> {
    typedef v2u T;
};

// Chunks (chunk chk of halo column gx, rows row0 + k RSTEP, k = K0 .. K0 +
// H - 1) of a tile whose halo rows start at the site offsets RowOff[].  The
// prefetch buffer is kept as halves of H chunks: the compiler keeps arrays
// of this size in registers.
template <int KIN, int H, int K0, int RSTEP>
__device__ __forceinline__ void conv_fetch(const int *RowOff, unsigned gx, int row0, int chk,
                                           const unsigned short *__restrict__ in,
                                           typename Chunk<KIN / 2>::T (&pre)[H])
{
    typedef typename Chunk<KIN / 2>::T CT;
#pragma unroll
    for (int k = 0; k < H; ++k) {
        const unsigned site = (unsigned)RowOff[row0 + (K0 + k) * RSTEP] + gx;
        // KIN / 4 channels per chunk; the element offset in 64 bits (site KIN exceeds 2^32 from 2^27 sites)
        pre[k] = *reinterpret_cast<const CT *>(in + (size_t)site * KIN + chk * (KIN / 4));
    }
}

// Site offsets (wrapped z and y, x = 0) of the halo rows of a tile.
__device__ inline void conv_rows(const Grid3 &g, int ntx, int nty, int tile, int *RowOff)
{
    const int y0 = ((tile / ntx) % nty) * kCTY, z0 = (tile / (ntx * nty)) * kCTZ;
    const int r = threadIdx.x;
    if (r < kCRows) {
        const int hy = r % kCHY, hz = r / kCHY;
        RowOff[r] = (wrap_cell(z0 - 1 + hz, g.nz) * g.ny + wrap_cell(y0 - 1 + hy, g.ny)) * g.nx;
    }
}

template <int KIN, int OUT, int SGN, int EPI>
__global__ void __launch_bounds__(kConvThreads) k_conv_tile(Grid3 g, long long N, const unsigned short *__restrict__ in,
                                                  const unsigned short *__restrict__ W,
                                                  const float *__restrict__ bias, const float *__restrict__ zin,
                                                  float *__restrict__ zout, unsigned short *__restrict__ aout, int act,
                                                  float scale)
{
    extern __shared__ __align__(16) unsigned char Ls[];
    constexpr int CW = KIN / 2, NCH = 4, CB = OUT / 16;       // chunk bytes; 4 chunks per site or weight row
    constexpr int WROWS = 27 * OUT;
    constexpr int RSTEP = 256 / (kCHX * NCH);                 // halo rows staged per pass (threads < 256)
    constexpr int MAXK = kCRows / RSTEP;                      // rows per staging thread
    static_assert(RSTEP * MAXK == kCRows, "staging threads cover the halo rows evenly");
    typedef typename Chunk<CW>::T CT;
    constexpr int PI = conv_plane(CW), PW = WROWS * CW;        // chunk-plane strides (bytes)
    unsigned char *Lin = Ls;                                  // [NCH][kCHS][CW]
    unsigned char *Lwt = Ls + NCH * PI;                       // [NCH][WROWS][CW]
    int *RowOff = reinterpret_cast<int *>(Lwt + NCH * PW);    // [2][kCRows], by tile parity
    float *Lbias = reinterpret_cast<float *>(RowOff + 2 * kCRows);   // [OUT]
    const int tid = threadIdx.x;
    const int ntx = (g.nx + kCTX - 1) / kCTX, nty = (g.ny + kCTY - 1) / kCTY, ntz = (g.nz + kCTZ - 1) / kCTZ;
    const int ntiles = ntx * nty * ntz;
    // weights once per block
    {
        constexpr int WCH = WROWS * NCH;
#pragma unroll 4
        for (int i = tid; i < WCH; i += kConvThreads)
            *reinterpret_cast<CT *>(Lwt + (i % NCH) * PW + (i / NCH) * CW) =
                *reinterpret_cast<const CT *>(W + (long long)i * (CW / 2));
    }
    // staging thread = (chunk, halo column), x fastest; rows row0 + k RSTEP
    const int ch = tid / kCHX, hx = tid % kCHX;
    const int row0 = ch / NCH, chk = ch % NCH;
    const bool stager = row0 < RSTEP;
    auto column = [&](int tile) { return (unsigned)wrap_cell((tile % ntx) * kCTX - 1 + hx, g.nx); };
    // the next tile's chunks, loaded while the current tile computes
    constexpr int H = MAXK / 2;
    static_assert(2 * H == MAXK, "two prefetch halves");
    CT preA[H], preB[H];
    // Tile walk.  Workgroup b runs on XCD b mod 8; with a multiple of 8
    // blocks and at least one tile each, the blocks of one XCD take one
    // contiguous eighth of the tiles (tile lo + w, lo + w + blocks/8, ...), so
    // the halos that neighbouring tiles share come from that XCD's L2.
    int t0 = blockIdx.x, tstep = gridDim.x, tend = ntiles;
    if (gridDim.x % 8 == 0 && ntiles >= (int)gridDim.x) {
        const int xcd = blockIdx.x % 8;
        tstep = gridDim.x / 8;
        t0 = (int)((long long)xcd * ntiles / 8) + (int)blockIdx.x / 8;
        tend = (int)((long long)(xcd + 1) * ntiles / 8);
    }
    if (t0 < tend) conv_rows(g, ntx, nty, t0, RowOff);
    if (tid < OUT) Lbias[tid] = EPI == 1 ? 0.f : bias[tid];
    __syncthreads();
    if (stager && t0 < tend) {
        const unsigned gx = column(t0);
        conv_fetch<KIN, H, 0, RSTEP>(RowOff, gx, row0, chk, in, preA);
        conv_fetch<KIN, H, H, RSTEP>(RowOff, gx, row0, chk, in, preB);
    }

    const int lane = tid & 63, wave = tid >> 6, li = lane & 15, gq = lane >> 4;
    const int wz = wave / kRowBlocks, wy = (wave % kRowBlocks) * kWaveRows;   // the wave's plane and first row
    // halo index of the wave's site (x0 + li, y0 + wy + sb, z0 + wz) is
    // (li + 1) + (wy + sb + 1) kCHX + (wz + 1) kCHX kCHY; Lb points at sb = 0
    const unsigned char *Lb = Lin + gq * PI + ((li + 1) + (wy + 1) * kCHX + (wz + 1) * kCHX * kCHY) * CW;
    // weight row co = c 16 + li of tap t is chunk row t OUT + co
    const unsigned char *Wl = Lwt + gq * PW + li * CW;
    typedef typename std::conditional<KIN == 32, v8bf, v4s>::type OP;

    // the lane's bias values, read once through LDS: a global load in the
    // epilogue would wait (vmcnt) for the next tile's prefetch as well
    float bl[CB][4];
#pragma unroll
    for (int c = 0; c < CB; ++c)
#pragma unroll
        for (int v = 0; v < 4; ++v) bl[c][v] = Lbias[c * 16 + 4 * gq + v];

    for (int tile = t0, it = 0; tile < tend; tile += tstep, ++it) {
        __syncthreads();   // the previous tile's reads of Lin are done
        const int next = tile + tstep;
        int *RowNext = RowOff + ((it + 1) & 1) * kCRows;
        if (next < tend) conv_rows(g, ntx, nty, next, RowNext);
        if (stager) {
#pragma unroll
            for (int k = 0; k < H; ++k) {
                *reinterpret_cast<CT *>(Lin + chk * PI + (hx + (row0 + k * RSTEP) * kCHX) * CW) = preA[k];
                *reinterpret_cast<CT *>(Lin + chk * PI + (hx + (row0 + (H + k) * RSTEP) * kCHX) * CW) = preB[k];
            }
        }
        __syncthreads();
        if (stager && next < tend) {
            const unsigned gx = column(next);
            conv_fetch<KIN, H, 0, RSTEP>(RowNext, gx, row0, chk, in, preA);
            conv_fetch<KIN, H, H, RSTEP>(RowNext, gx, row0, chk, in, preB);
        }

        v4f acc[CB][kWaveRows];
#pragma unroll
        for (int c = 0; c < CB; ++c)
#pragma unroll
            for (int sb = 0; sb < kWaveRows; ++sb) acc[c][sb] = v4f{0.f, 0.f, 0.f, 0.f};
        OP a[CB], an[CB];
#pragma unroll
        for (int c = 0; c < CB; ++c) a[c] = *reinterpret_cast<const OP *>(Wl + c * 16 * CW);
#pragma unroll
        for (int t = 0; t < 27; ++t) {
            const int dz = t / 9 - 1, dy = (t / 3) % 3 - 1, dx = t % 3 - 1;
            const int off = SGN * (dx + dy * kCHX + dz * kCHX * kCHY);
            if (t + 1 < 27)
#pragma unroll
                for (int c = 0; c < CB; ++c)
                    an[c] = *reinterpret_cast<const OP *>(Wl + ((t + 1) * OUT + c * 16) * CW);
            OP b[kWaveRows];
#pragma unroll
            for (int sb = 0; sb < kWaveRows; ++sb) b[sb] = *reinterpret_cast<const OP *>(Lb + (off + sb * kCHX) * CW);
#pragma unroll
            for (int sb = 0; sb < kWaveRows; ++sb)
#pragma unroll
                for (int c = 0; c < CB; ++c) {
                    if constexpr (KIN == 32)
                        acc[c][sb] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[c], b[sb], acc[c][sb], 0, 0, 0);
                    else
                        acc[c][sb] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a[c], b[sb], acc[c][sb], 0, 0, 0);
                }
            if (t + 1 < 27)
#pragma unroll
                for (int c = 0; c < CB; ++c) a[c] = an[c];
        }

        const int x0 = (tile % ntx) * kCTX, y0 = ((tile / ntx) % nty) * kCTY, z0 = (tile / (ntx * nty)) * kCTZ;
        const int x = x0 + li, z = z0 + wz;
        if (x >= g.nx || z >= g.nz) continue;
#pragma unroll
        for (int sb = 0; sb < kWaveRows; ++sb) {
            const int y = y0 + wy + sb;
            if (y >= g.ny) break;
            const long long s = ((long long)z * g.ny + y) * g.nx + x;
#pragma unroll
            for (int c = 0; c < CB; ++c) {
                const int o0 = c * 16 + 4 * gq;
                if constexpr (EPI == 0) {
                    float zv[4];
                    unsigned short av[4];
                    for (int v = 0; v < 4; ++v) {
                        zv[v] = acc[c][sb][v] + bl[c][v];
                        av[v] = f2bf(act ? zv[v] * sigm(zv[v]) : zv[v]);
                    }
                    if (zout)
                        *reinterpret_cast<float4 *>(zout + s * OUT + o0) = make_float4(zv[0], zv[1], zv[2], zv[3]);
                    if (aout) {
                        const uint2 pk = make_uint2((unsigned)av[0] | ((unsigned)av[1] << 16),
                                                    (unsigned)av[2] | ((unsigned)av[3] << 16));
                        *reinterpret_cast<uint2 *>(aout + s * OUT + o0) = pk;
                    }
                } else if constexpr (EPI == 2) {
                    for (int v = 0; v < 4; ++v)
                        if (o0 + v < kNetOut) zout[(long long)(o0 + v) * N + s] = (acc[c][sb][v] + bl[c][v]) * scale;
                } else {
                    const float4 zz = *reinterpret_cast<const float4 *>(zin + s * OUT + o0);
                    const float zi[4] = {zz.x, zz.y, zz.z, zz.w};
                    unsigned short gv[4];
                    for (int v = 0; v < 4; ++v) {
                        const float sg = sigm(zi[v]);
                        gv[v] = f2bf(acc[c][sb][v] * (sg * (1.f + zi[v] * (1.f - sg))));
                    }
                    const uint2 pk = make_uint2((unsigned)gv[0] | ((unsigned)gv[1] << 16),
                                                (unsigned)gv[2] | ((unsigned)gv[3] << 16));
                    *reinterpret_cast<uint2 *>(aout + s * OUT + o0) = pk;
                }
            }
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
    // blockIdx.y picks a third of the taps (one dz plane): three workgroups
    // per chunk fill disjoint parts of the chunk's partial row
    for (int t = 9 * (int)blockIdx.y; t < 9 * (int)blockIdx.y + 9; ++t) {
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
    if (blockIdx.y == 0 && tid < COP) {
        float sb = 0.f;
        for (int k = 0; k < 256; ++k) sb += bf2f(Gs[tid][k]);
        out[27 * COP * CIP + tid] = sb;
    }
}

// out[i] = sum_w part[w][i] in a fixed order: the rows are split into four
// contiguous quarters, each summed in order by its own thread (64 columns
// per block), and the quarter sums are added in quarter order
__global__ void __launch_bounds__(256) k_sum_rows(const float *__restrict__ part, int nrows, int len,
                                                  float *__restrict__ out)
{
    __shared__ float red[4][64];
    const int c = threadIdx.x % 64, q = threadIdx.x / 64;
    const int i = blockIdx.x * 64 + c;
    const int per = (nrows + 3) / 4, w0 = min(nrows, q * per), w1 = min(nrows, w0 + per);
    float s = 0.f;
    if (i < len) {
#pragma unroll 8
        for (int w = w0; w < w1; ++w) s += part[(long long)w * len + i];
    }
    red[q][c] = s;
    __syncthreads();
    if (q == 0 && i < len) out[i] = ((red[0][c] + red[1][c]) + red[2][c]) + red[3][c];
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
struct AdamConst {
    float lr, b1, b2, omb1, omb2, c1, c2, eps;   // omb = 1 - b, c = 1 - b^t (formed in float64)
};

__global__ void k_adam(int n, int COP, int CIP, int cout, int cin, float *__restrict__ w, const float *__restrict__ gw,
                       float *__restrict__ m, float *__restrict__ v, AdamConst k, unsigned short *__restrict__ wb,
                       unsigned short *__restrict__ wt)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const int t = i / (COP * CIP), r = i - t * COP * CIP, co = r / CIP, ci = r - co * CIP;
    if (co >= cout || ci >= cin) {
        wb[i] = 0;
        wt[((long long)t * CIP + ci) * COP + co] = 0;
        return;
    }
    const float gi = gw[i];
    const float mi = k.b1 * m[i] + k.omb1 * gi;
    const float vi = k.b2 * v[i] + k.omb2 * gi * gi;
    m[i] = mi;
    v[i] = vi;
    const float wi = w[i] - k.lr * (mi / k.c1) / (sqrtf(vi / k.c2) + k.eps);
    w[i] = wi;
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
__global__ void k_cast_weights(int n, int COP, int CIP, const float *__restrict__ w, unsigned short *__restrict__ wb,
                               unsigned short *__restrict__ wt)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const int t = i / (COP * CIP), r = i - t * COP * CIP, co = r / CIP, ci = r - co * CIP;
    wb[i] = f2bf(w[i]);
    wt[((long long)t * CIP + ci) * COP + co] = f2bf(w[i]);
}

// ---------------------------------------------------------- packing
// first-layer input of one site: x[0..15] = [bf16(v[0..13]) | 0], written as
// two 16-byte stores (a site's 32 bytes are 16-byte aligned)
__device__ inline void store_input(unsigned short *__restrict__ x, const float v[kNetIn])
{
    static_assert(kNetIn <= kNetInSlots && kNetInSlots == 16, "two 16-byte stores per site");
    unsigned p[8];
#pragma unroll
    for (int c = 0; c < 8; ++c) {
        const unsigned short a = 2 * c < kNetIn ? f2bf(v[2 * c]) : 0, b = 2 * c + 1 < kNetIn ? f2bf(v[2 * c + 1]) : 0;
        p[c] = (unsigned)a | ((unsigned)b << 16);
    }
    uint4 *o = reinterpret_cast<uint4 *>(x);
    o[0] = make_uint4(p[0], p[1], p[2], p[3]);
    o[1] = make_uint4(p[4], p[5], p[6], p[7]);
}

// The 14 inputs of site s: v[0..1] = n_a / n_ref - 1, v[2..7] = j_a,d / j_ref
// (index 2 + 3a + d), v[8..13] = c_s^2 (n_a(s + e_d) - n_a(s - e_d)) / 2 / f_ref
// (index 8 + 3a + d), neighbours with periodic wrap.
__device__ inline void site_inputs(const CnnShape &sh, long long s, const float *__restrict__ n,
                                   const float *__restrict__ j, float n_ref, float j_ref, float f_ref, float v[kNetIn])
{
    const long long N = sh.N;
    const int nx = sh.nx, ny = sh.ny, nz = sh.nz;
    const long long nxy = (long long)nx * ny;
    const int x = (int)(s % nx), y = (int)((s / nx) % ny), z = (int)(s / nxy);
    const long long dxp = x == nx - 1 ? 1 - nx : 1, dxm = x == 0 ? nx - 1 : -1;
    const long long dyp = y == ny - 1 ? nx - nxy : nx, dym = y == 0 ? nxy - nx : -nx;
    const long long dzp = z == nz - 1 ? nxy - N : nxy, dzm = z == 0 ? N - nxy : -nxy;
    const long long dp[3] = {dxp, dyp, dzp}, dm[3] = {dxm, dym, dzm};
    const float gsc = (1.f / 6.f) / f_ref;   // c_s^2 / 2 / f_ref
#pragma unroll
    for (int a = 0; a < 2; ++a) {
        const float *na = n + a * N;
        v[a] = na[s] / n_ref - 1.f;
#pragma unroll
        for (int d = 0; d < 3; ++d) {
            v[2 + 3 * a + d] = j[(3 * a + d) * N + s] / j_ref;
            v[8 + 3 * a + d] = (na[s + dp[d]] - na[s + dm[d]]) * gsc;
        }
    }
}

__global__ void k_pack_input(CnnShape sh, const float *__restrict__ n, const float *__restrict__ j, float n_ref,
                             float j_ref, float f_ref, unsigned short *__restrict__ x)
{
    const long long s = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= sh.N) return;
    float v[kNetIn];
    site_inputs(sh, s, n, j, n_ref, j_ref, f_ref, v);
    store_input(x + s * kNetInSlots, v);
}

// input from channel-first float32 xf [14][N]
__global__ void k_pack_x(long long N, const float *__restrict__ xf, unsigned short *__restrict__ x)
{
    const long long s = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= N) return;
    float v[kNetIn];
    for (int c = 0; c < kNetIn; ++c) v[c] = xf[c * N + s];
    store_input(x + s * kNetInSlots, v);
}

// channel-first float32 network input and target from lattice fields:
// xf[c][s] = the inputs of site_inputs, tf[c][s] = N_c(s) / f_ref
__global__ void k_fields_x(CnnShape sh, const float *__restrict__ n, const float *__restrict__ j, float n_ref,
                           float j_ref, const float *__restrict__ Nf, float f_ref, float *__restrict__ xf,
                           float *__restrict__ tf)
{
    const long long s = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    const long long N = sh.N;
    if (s >= N) return;
    float v[kNetIn];
    site_inputs(sh, s, n, j, n_ref, j_ref, f_ref, v);
    for (int c = 0; c < kNetIn; ++c) xf[c * N + s] = v[c];
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

namespace {
// persistent grid: one block per compute unit (the LDS footprint allows one)
unsigned conv_tiles(const CnnShape &sh)
{
    static int cus = 0;
    if (cus == 0) {
        int dev = 0, n = 0;
        if (hipGetDevice(&dev) == hipSuccess &&
            hipDeviceGetAttribute(&n, hipDeviceAttributeMultiprocessorCount, dev) == hipSuccess && n > 0)
            cus = n;
        else
            cus = 256;
    }
    const long long tiles =
        (long long)((sh.nx + kCTX - 1) / kCTX) * ((sh.ny + kCTY - 1) / kCTY) * ((sh.nz + kCTZ - 1) / kCTZ);
    return (unsigned)(tiles < cus ? tiles : cus);
}
}  // namespace

bool cnn_prepare()
{
    return hipFuncSetAttribute((const void *)k_conv_tile<32, 32, 1, 0>, hipFuncAttributeMaxDynamicSharedMemorySize,
                               conv_lds(32, 32)) == hipSuccess &&
           hipFuncSetAttribute((const void *)k_conv_tile<32, 16, 1, 0>, hipFuncAttributeMaxDynamicSharedMemorySize,
                               conv_lds(32, 16)) == hipSuccess &&
           hipFuncSetAttribute((const void *)k_conv_tile<32, 16, 1, 2>, hipFuncAttributeMaxDynamicSharedMemorySize,
                               conv_lds(32, 16)) == hipSuccess &&
           hipFuncSetAttribute((const void *)k_conv_tile<32, 32, -1, 1>, hipFuncAttributeMaxDynamicSharedMemorySize,
                               conv_lds(32, 32)) == hipSuccess &&
           hipFuncSetAttribute((const void *)k_conv_tile<16, 32, -1, 1>, hipFuncAttributeMaxDynamicSharedMemorySize,
                               conv_lds(16, 32)) == hipSuccess &&
           hipFuncSetAttribute((const void *)k_conv_tile<16, 32, 1, 0>, hipFuncAttributeMaxDynamicSharedMemorySize,
                               conv_lds(16, 32)) == hipSuccess;
}

void cnn_conv_fwd(int layer, const CnnShape &sh, const unsigned short *in, const unsigned short *W, const float *b,
                  float *z, unsigned short *a, int act, hipStream_t st)
{
    const Grid3 g{sh.nx, sh.ny, sh.nz};
    const unsigned nb = conv_tiles(sh);
    if (net_cop(layer) == 16)
        hipLaunchKernelGGL((k_conv_tile<32, 16, 1, 0>), dim3(nb), dim3(kConvThreads), conv_lds(32, 16), st, g, sh.N, in, W, b,
                           nullptr, z, a, act, 1.f);
    else if (net_cip(layer) == 16)
        hipLaunchKernelGGL((k_conv_tile<16, 32, 1, 0>), dim3(nb), dim3(kConvThreads), conv_lds(16, 32), st, g, sh.N, in, W, b,
                           nullptr, z, a, act, 1.f);
    else
        hipLaunchKernelGGL((k_conv_tile<32, 32, 1, 0>), dim3(nb), dim3(kConvThreads), conv_lds(32, 32), st, g, sh.N, in, W, b,
                           nullptr, z, a, act, 1.f);
}

void cnn_conv_out_fields(const CnnShape &sh, const unsigned short *in, const unsigned short *W, const float *b,
                         float scale, float *Nf, hipStream_t st)
{
    const Grid3 g{sh.nx, sh.ny, sh.nz};
    hipLaunchKernelGGL((k_conv_tile<32, 16, 1, 2>), dim3(conv_tiles(sh)), dim3(kConvThreads), conv_lds(32, 16), st, g,
                       sh.N, in, W, b, nullptr, Nf, nullptr, 0, scale);
}

void cnn_conv_dgrad(int layer, const CnnShape &sh, const unsigned short *gout, const unsigned short *WT, const float *zin,
                    unsigned short *gin, hipStream_t st)
{
    const Grid3 g{sh.nx, sh.ny, sh.nz};
    const unsigned nb = conv_tiles(sh);
    if (net_cop(layer) == 16)
        hipLaunchKernelGGL((k_conv_tile<16, 32, -1, 1>), dim3(nb), dim3(kConvThreads), conv_lds(16, 32), st, g, sh.N, gout, WT,
                           nullptr, zin, nullptr, gin, 0, 1.f);
    else
        hipLaunchKernelGGL((k_conv_tile<32, 32, -1, 1>), dim3(nb), dim3(kConvThreads), conv_lds(32, 32), st, g, sh.N, gout, WT,
                           nullptr, zin, nullptr, gin, 0, 1.f);
}

void cnn_conv_wgrad(int layer, const CnnShape &sh, const unsigned short *gout, const unsigned short *ain, float *part,
                    float *gw, hipStream_t st)
{
    const Grid3 g{sh.nx, sh.ny, sh.nz};
    const unsigned nb = nblocks(sh.N);
    int cip = 32, cop = 32;
    switch (layer) {
    case 0: cip = 16; hipLaunchKernelGGL((k_conv_wgrad<16, 32>), dim3(nb, 3), dim3(256), 0, st, g, sh.N, gout, ain, part); break;
    case 3: cop = 16; hipLaunchKernelGGL((k_conv_wgrad<32, 16>), dim3(nb, 3), dim3(256), 0, st, g, sh.N, gout, ain, part); break;
    default: hipLaunchKernelGGL((k_conv_wgrad<32, 32>), dim3(nb, 3), dim3(256), 0, st, g, sh.N, gout, ain, part); break;
    }
    const int len = 27 * cop * cip + cop;
    hipLaunchKernelGGL(k_sum_rows, dim3((len + 63) / 64), dim3(256), 0, st, part, (int)nb, len, gw);
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

void cnn_adam(int n, int cop, int cip, int cout, int cin, float *w, const float *gw, float *m, float *v, float lr,
              double b1, double b2, double eps, int step, unsigned short *wb, unsigned short *wt, float *b,
              const float *gb, float *mb, float *vb, hipStream_t st)
{
    const AdamConst k{lr, (float)b1, (float)b2, (float)(1.0 - b1), (float)(1.0 - b2),
                      (float)(1.0 - std::pow(b1, step)), (float)(1.0 - std::pow(b2, step)), (float)eps};
    hipLaunchKernelGGL(k_adam, dim3(nblocks(n)), dim3(256), 0, st, n, cop, cip, cout, cin, w, gw, m, v, k, wb, wt);
    hipLaunchKernelGGL(k_adam_bias, dim3(1), dim3(64), 0, st, cop, b, gb, mb, vb, k);
}

void cnn_cast(int n, int cop, int cip, const float *w, unsigned short *wb, unsigned short *wt, hipStream_t st)
{
    hipLaunchKernelGGL(k_cast_weights, dim3(nblocks(n)), dim3(256), 0, st, n, cop, cip, w, wb, wt);
}

void cnn_pack_input(const CnnShape &sh, const float *n, const float *j, float n_ref, float j_ref, float f_ref,
                    unsigned short *x, hipStream_t st)
{
    hipLaunchKernelGGL(k_pack_input, dim3(nblocks(sh.N)), dim3(256), 0, st, sh, n, j, n_ref, j_ref, f_ref, x);
}

void cnn_pack_x(const CnnShape &sh, const float *xf, unsigned short *x, hipStream_t st)
{
    hipLaunchKernelGGL(k_pack_x, dim3(nblocks(sh.N)), dim3(256), 0, st, sh.N, xf, x);
}

void cnn_fields_x(const CnnShape &sh, const float *n, const float *j, float n_ref, float j_ref, const float *Nf,
                  float f_ref, float *xf, float *tf, hipStream_t st)
{
    hipLaunchKernelGGL(k_fields_x, dim3(nblocks(sh.N)), dim3(256), 0, st, sh, n, j, n_ref, j_ref, Nf, f_ref, xf, tf);
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

// Sums of squares of `len` floats at base + s stride for every sample s of a
// training pool (float64): block (p, s) writes part[s * nparts + p].
__global__ void __launch_bounds__(256) k_pool_sumsq(const float *__restrict__ base, long long stride, long long len,
                                                    double *__restrict__ part)
{
    __shared__ double r[256];
    const float *x = base + (long long)blockIdx.y * stride;
    double acc = 0.0;
    for (long long i = (long long)blockIdx.x * 256 + threadIdx.x; i < len; i += (long long)gridDim.x * 256) {
        const double v = (double)x[i];
        acc += v * v;
    }
    r[threadIdx.x] = acc;
    __syncthreads();
    for (int o = 128; o > 0; o >>= 1) {
        if (threadIdx.x < o) r[threadIdx.x] += r[threadIdx.x + o];
        __syncthreads();
    }
    if (threadIdx.x == 0) part[(long long)blockIdx.y * gridDim.x + blockIdx.x] = r[0];
}

__global__ void k_pool_scale(float *__restrict__ base, long long stride, long long len, float mul)
{
    float *x = base + (long long)blockIdx.y * stride;
    for (long long i = (long long)blockIdx.x * 256 + threadIdx.x; i < len; i += (long long)gridDim.x * 256)
        x[i] *= mul;
}

void cnn_pool_sumsq(const float *base, long long stride, long long len, int count, double *part, int nparts,
                    hipStream_t st)
{
    hipLaunchKernelGGL(k_pool_sumsq, dim3(nparts, count), dim3(256), 0, st, base, stride, len, part);
}

void cnn_pool_scale(float *base, long long stride, long long len, int count, float mul, hipStream_t st)
{
    hipLaunchKernelGGL(k_pool_scale, dim3(64, count), dim3(256), 0, st, base, stride, len, mul);
}

}  // namespace mlb
