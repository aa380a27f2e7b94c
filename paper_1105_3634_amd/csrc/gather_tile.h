// Float32 gathers on LDS-staged halo tiles.
//
// Same fields as the ordered per-site kernels of step_kernels.h (which the
// float64 build uses), with the arithmetic regrouped for throughput:
//
// For species a at r and partner b, over the half-shell pairs (+e, -e),
//   G+- = g_ab(r) + g_ab(r+-e),   t+- = G+- n_b(r+-e)
//   mean field   Smf_b = sum e_hat (t+ - t-)                       eq. (potmeanforce)
//   tensor       Ts_b  = sum (t+ + t-) e_hat e_hat^T              eqs. (tensorgamma)
//   current      Sv_b  = sum e_hat e_hat.(G+ j_b(r+e) + G- j_b(r-e))
// and, with cm, ck, cg the pair constants,
//   Nmf   = n_a sum_b cm Smf_b
//   T_a   = sum_b ck Ts_b,   Gam_a = sum_b cg trace(Ts_b)
//   D_a[u_old] = n_a sum_b ck Sv_b - T_a j_a        (pair form of eqs. gammaab +
//                                                    viscousforce, Newton-3 antisymmetric)
// The second gather needs only
//   D_a[V] = n_a ( sum_b ck sum e_hat e_hat.(t+ V_b(r+e) + t- V_b(r-e)) - T_a V_a )
// because T_a (stored by the first gather) already holds the local part.
//
// Tile: TX x TY x TZ = 256 sites (a template parameter; the autotuner picks
// among the built shapes), one thread per site; per partner species the
// block stages n_b, the three components of j_b and g_ab (first gather) or
// n_b V_b and g_ab (second gather) for the tile plus a halo of R cells (R = largest stencil component of the
// system) into LDS; periodic wrap and walls are resolved while filling, so
// the inner loop is address arithmetic on a uniform offset and LDS loads.
#pragma once

#include <algorithm>

#include "step_kernels.h"

namespace mlb {


// The gathers run several threads per tile site: thread group h (the waves
// of threads h * 256 ... h * 256 + 255) takes the h-th part of every shell
// list, and the parts are added in group order at the end.  More waves per
// CU at the same LDS footprint hide the LDS and scalar-load latencies of the
// inner loop.  Split factor, shell-loop unrolling and the register budget
// (waves per SIMD) per kernel:
#ifndef MLB_G1_UNROLL
#define MLB_G1_UNROLL 4
#endif
#ifndef MLB_G1_WAVES
#define MLB_G1_WAVES 6
#endif
#ifndef MLB_S2_SPLIT
#define MLB_S2_SPLIT 3
#endif
#ifndef MLB_S2_UNROLL
#define MLB_S2_UNROLL 4
#endif
#ifndef MLB_S2_WAVES
#define MLB_S2_WAVES 6
#endif
// Bank-aware lane layouts (below) allowed in the first / second gather, a
// bit mask: 1 = z-paired (8-wide tiles), 2 = z-major (16-wide tiles)
#ifndef MLB_G1_LAYOUTS
#define MLB_G1_LAYOUTS 2
#endif
#ifndef MLB_S2_LAYOUTS
#define MLB_S2_LAYOUTS 3
#endif
// The first gather runs with 2 or 3 thread groups per tile site (a launch
// parameter the autotuner picks: fewer groups leave LDS and wave slots to
// the spectral field that runs beside it); the second with kSplitS2.
constexpr int kSplitG1Max = 3, kSplitS2 = MLB_S2_SPLIT;
constexpr int kStep2Threads = kSplitS2 * kBlock;

// shell entries [kb, ke) of group h of SPLIT
template <int SPLIT>
__device__ inline void split_range(int kn, int h, int &kb, int &ke)
{
    const int part = (kn + SPLIT - 1) / SPLIT;
    kb = min(kn, h * part);
    ke = min(kn, kb + part);
}

// Every group ends with the sum of all groups' partial sums, added in group
// order (the same bits in every group); the LDS staging area is reused after
// a barrier, V floats per site and group.  The groups then share the
// epilogue's stores.
template <int SPLIT, int V>
__device__ inline void split_allreduce(float4 *lds, float (&v)[V])
{
    if (SPLIT == 1) return;
    float *R = reinterpret_cast<float *>(lds);
    const int i = threadIdx.x % kBlock, h = threadIdx.x / kBlock;
    __syncthreads();
#pragma unroll
    for (int j = 0; j < V; ++j) R[(h * V + j) * kBlock + i] = v[j];
    __syncthreads();
#pragma unroll
    for (int j = 0; j < V; ++j) {
        float acc = R[j * kBlock + i];
        for (int g = 1; g < SPLIT; ++g) acc += R[(g * V + j) * kBlock + i];
        v[j] = acc;
    }
}

// Field pointers cast to the global address space: loads and stores then
// compile to global_* instructions, which count only against the vector
// memory counter (flat ones also hold the LDS counter, so a wait on LDS
// data would wait for outstanding field loads as well).
typedef __attribute__((address_space(1))) float gfloat;
__device__ inline gfloat *glb(float *p) { return (gfloat *)p; }

struct TileGeo {
    int x0, y0, z0;       // tile origin
    int R, HX, HY, HZ;    // halo width and staged extents
    int PXY;              // z-plane pitch of the staged arrays (sites)
    int FS;               // floats per staged field
};

// Bank layouts of the gathers' staged tiles.  LDS has 64 banks of 4 bytes;
// one clock of a 16-byte read serves 16 consecutive lanes, consecutive
// 8-lane blocks must lie on opposite 128-byte halves (mod 256), and the
// 16-lane runs of a read must start at the same offset mod 256 (measured).
// The plain order (x, then y, then z) breaks this wherever a halo row is a
// multiple of 256 bytes (8-wide tiles, rows of 16 sites) or 128 mod 256
// (16-wide tiles, rows of 24 sites): every shell-loop read then takes two
// clocks.  Two layouts avoid it:
// - z-paired (8-wide tiles, TZ even): z planes padded to a pitch of 8 mod 16
//   sites, lanes 8..15 of every 16 on the next plane instead of the next
//   row; the two 8-lane halves lie 128 bytes apart mod 256, and the 4-byte g
//   reads of a wave (4 rows x 2 planes x 8 x) fall on distinct banks too.
// - z-major (16-wide tiles): z planes padded to a multiple of 16 sites
//   (none at halo 4: 24 x 12 sites), the 16-lane runs on consecutive planes,
//   all starting at the same offset mod 256.
// Layout 0 keeps unpadded planes and the plain order.
__host__ __device__ constexpr int lane_layout(int TX, int TZ, int allowed)
{
    return (TX == 8 && TZ % 2 == 0 && (allowed & 1)) ? 1 : (TX == 16 && (allowed & 2)) ? 2 : 0;
}

__host__ __device__ inline int plane_pitch(int LM, int plane)
{
    return LM == 1 ? plane + ((24 - plane % 16) % 16) : LM == 2 ? (plane + 15) / 16 * 16 : plane;
}

template <int TX, int TY, int TZ, int LM = 0>
__device__ inline TileGeo tile_geo(const SysDesc<float> &S, int local, int R)
{
    TileGeo t;
    const int tx = (S.nx + TX - 1) / TX, ty = (S.ny + TY - 1) / TY;
    const int bx = local % tx, by = (local / tx) % ty, bz = local / (tx * ty);
    t.x0 = bx * TX; t.y0 = by * TY; t.z0 = bz * TZ;
    t.R = R;
    t.HX = TX + 2 * t.R; t.HY = TY + 2 * t.R; t.HZ = TZ + 2 * t.R;
    t.PXY = plane_pitch(LM, t.HX * t.HY);
    t.FS = t.PXY * t.HZ;
    return t;
}

// Staging of the halo tile.  Rows (hy, hz) of the tile are numbered
// row = hy + HY hz; RowOff[row] holds the global site offset of the row's
// x = 0 site ((gz ny + gy) nx after periodic wrap) in its low 29 bits and,
// in bits 29-30, 0 for a fluid row or 1 / 2 for a row beyond the y = 0 /
// y = ny - 1 wall: the hard-core stencils see there the mirror image of the
// fluid across the wall plane (y = 1/2 or ny - 3/2), so the offset is that
// of the mirrored fluid row, and the image moves with the wall (the staging
// replaces its momentum or velocity by the wall's).  Sites number below
// 2^29 (checked on the host).  Thread t owns the halo column hx = t % HX (its wrapped global
// x computed once) and the rows t / HX, t / HX + NT / HX, ... (NT threads per
// block); consecutive
// threads read consecutive x, so global loads coalesce, and the per-element
// work is a table read, an add and the loads.
constexpr int kRowImgShift = 29, kRowOffMask = (1 << kRowImgShift) - 1;

__device__ inline int wrap_mod(int v, int n)
{
    v %= n;
    return v < 0 ? v + n : v;
}

struct StageLane {
    int hx, row0, rstep;   // rstep = 0: the thread stages nothing
    int gx;
};

template <int NT = kBlock>
__device__ inline StageLane stage_lane(const SysDesc<float> &S, const TileGeo &t)
{
    StageLane l;
    l.rstep = NT / t.HX;
    l.hx = threadIdx.x % t.HX;
    l.row0 = threadIdx.x / t.HX;
    if (l.row0 >= l.rstep) l.rstep = 0;          // left-over threads of the last partial column set
    l.gx = wrap_mod(t.x0 - t.R + l.hx, S.nx);
    return l;
}

// RowL (may be null) receives the row's LDS base, hy HX + hz PXY.
template <int NT = kBlock>
__device__ inline void fill_rows(const SysDesc<float> &S, const TileGeo &t, int *RowOff, int *RowL = nullptr)
{
    const int rows = t.HY * t.HZ;
    for (int r = threadIdx.x; r < rows; r += NT) {
        const int hz = r / t.HY, hy = r - hz * t.HY;
        if (RowL) RowL[r] = hy * t.HX + hz * t.PXY;
        int gy = t.y0 - t.R + hy;
        const int gz = wrap_mod(t.z0 - t.R + hz, S.nz);
        int img = 0;
        if (S.walls) {
            if (gy <= 0) {
                gy = 1 - gy;
                img = 1;
            } else if (gy >= S.ny - 1) {
                gy = 2 * S.ny - 3 - gy;
                img = 2;
            }
        } else {
            gy = wrap_mod(gy, S.ny);
        }
        RowOff[r] = (gz * S.ny + gy) * S.nx | img << kRowImgShift;
    }
}

// Padded layouts (LM != 0) take each row's LDS base from RowL, the plain one
// uses row HX.
template <int LM>
__device__ inline void stage(const SysDesc<float> &S, const TileGeo &t, const StageLane &l, const int *RowOff,
                             const int *RowL, float4 *lds4, float *ldsg, const gfloat *__restrict__ nb,
                             const gfloat *__restrict__ vb, const gfloat *__restrict__ gp)
{
    const unsigned N = (unsigned)S.N;
    const int rows = t.HY * t.HZ;
    if (l.rstep == 0) return;
    for (int row = l.row0; row < rows; row += l.rstep) {
        const int ro = RowOff[row];
        const int img = ro >> kRowImgShift;
        const int i = l.hx + (LM ? RowL[row] : row * t.HX);
        const unsigned so = (unsigned)((ro & kRowOffMask) + l.gx);
        const float n = nb[so];
        // an image's momentum density: its density times the wall's velocity
        const float4 v = img ? make_float4(n, n * S.wall_ux[img - 1], 0.f, 0.f)
                             : make_float4(n, vb[so], vb[N + so], vb[2 * N + so]);
        lds4[i] = v;
        ldsg[i] = gp[so];
    }
}

// Second gather: one float4 per halo site, (n_b V_b, g_ab); the shell loop
// then needs no separate g reads and no product with n_b.
template <int LM>
__device__ inline void stage_nv(const SysDesc<float> &S, const TileGeo &t, const StageLane &l, const int *RowOff,
                                const int *RowL, float4 *lds4, const gfloat *__restrict__ nb,
                                const gfloat *__restrict__ vb, const gfloat *__restrict__ gp)
{
    const unsigned N = (unsigned)S.N;
    const int rows = t.HY * t.HZ;
    if (l.rstep == 0) return;
    for (int row = l.row0; row < rows; row += l.rstep) {
        const int ro = RowOff[row];
        const int img = ro >> kRowImgShift;
        const int i = l.hx + (LM ? RowL[row] : row * t.HX);
        const unsigned so = (unsigned)((ro & kRowOffMask) + l.gx);
        const float n = nb[so];
        // an image moves with the wall: n (u_wall, 0, 0)
        lds4[i] = img ? make_float4(n * S.wall_ux[img - 1], 0.f, 0.f, gp[so])
                      : make_float4(n * vb[so], n * vb[N + so], n * vb[2 * N + so], gp[so]);
    }
}

// One scalar field of the halo tile (rows beyond a wall take the mirrored
// fluid row; unpadded planes).  The thread's rows go in batches of 8 whose
// loads are all issued before the first store to LDS (one wait for memory
// per batch).
__device__ inline void stage1(const TileGeo &t, const StageLane &l, const int *RowOff, float *dst,
                              const gfloat *__restrict__ src)
{
    const int rows = t.HY * t.HZ;
    if (l.rstep == 0) return;
    constexpr int B = 8;
    for (int row0 = l.row0; row0 < rows; row0 += B * l.rstep) {
        float v[B];
#pragma unroll
        for (int k = 0; k < B; ++k) {
            const int row = row0 + k * l.rstep;
            v[k] = src[row < rows ? (unsigned)((RowOff[row] & kRowOffMask) + l.gx) : 0u];
        }
#pragma unroll
        for (int k = 0; k < B; ++k) {
            const int row = row0 + k * l.rstep;
            if (row < rows) dst[l.hx + row * t.HX] = v[k];
        }
    }
}

// The (a,b) half-shell is read straight from the float4 table sh_q
// (packed offset bits, e_hat): the index is wave-uniform, so the entries
// arrive through scalar loads into SGPRs and the offset arithmetic runs on
// the scalar unit.  LDS bandwidth, the binding resource of the gathers,
// then carries only the staged fields.  shell_off returns the byte offset of
// e in the float4 field array; the g array's offset is a quarter of it.
typedef float ShellEntry __attribute__((ext_vector_type(4)));
typedef const __attribute__((address_space(4))) ShellEntry *ConstF4;   // read-only for the kernel's lifetime

__device__ inline ConstF4 shell_list(const Tables<float> &tb, int k0)
{
    return (ConstF4)(tb.sh_q + k0);
}


__device__ inline int shell_off(float packed, int HX, int HXY)
{
    int ex, ey, ez;
    unpack_offset(__float_as_int(packed), ex, ey, ez);
    return 16 * (ex + ey * HX + ez * HXY);
}

// field reads at a byte offset from the site's own address
__device__ inline float4 ld4(const char *base, int byte) { return *reinterpret_cast<const float4 *>(base + byte); }
__device__ inline float ld1(const char *base, int byte) { return *reinterpret_cast<const float *>(base + byte); }

// ---- sign-grouped first gather
// Points of a half-shell that differ only in the signs of their y and z
// components share |e_hat|: their contributions to the friction tensor,
// the mean field and the current are summed as +- combinations of the
// members' scalars, with the products of |e_hat| components taken once per
// group (22.5 instead of 29 arithmetic operations per point in a four-point
// group, 17.5 in a two-point one).  The sums associate differently from the
// plain loop, so the two forms agree to float32 rounding, not bit for bit.

// one member of a group: t+- = G+- n_b(r +- e), dt = t+ - t-, st = t+ + t-,
// w = G+ j_b(r + e) + G- j_b(r - e)
struct G1Pt {
    float dt, st, w[3];
};
__device__ inline G1Pt g1_point(const char *c4, const char *cg, float g0, float packed, int HX, int HXY)
{
    const int o4 = shell_off(packed, HX, HXY), o1 = o4 >> 2;
    const float4 Ap = ld4(c4, o4), Am = ld4(c4, -o4);
    const float Gp = g0 + ld1(cg, o1), Gm = g0 + ld1(cg, -o1);
    const float tp = Gp * Ap.x, tm = Gm * Am.x;
    G1Pt r;
    r.dt = tp - tm;
    r.st = tp + tm;
    r.w[0] = Gp * Ap.y + Gm * Am.y;
    r.w[1] = Gp * Ap.z + Gm * Am.z;
    r.w[2] = Gp * Ap.w + Gm * Am.w;
    return r;
}
// symmetric tensor element (i, j) in the order xx, xy, xz, yy, yz, zz
__host__ __device__ constexpr int tix(int i, int j)
{
    return i > j ? tix(j, i) : i == 0 ? j : i == 1 ? 2 + j : 5;
}
// two-point groups: shared axis SA (component A), flipped axis SB (+-B)
template <int SA, int SB>
__device__ inline void g1_pair(const ShellEntry E0, const ShellEntry E1, const char *c4, const char *cg, float g0,
                               int HX, int HXY, float (&sv)[3], float (&tv)[6], float (&vv)[3])
{
    const G1Pt m0 = g1_point(c4, cg, g0, E0.x, HX, HXY), m1 = g1_point(c4, cg, g0, E0.y, HX, HXY);
    const float A = E0.z, B = E0.w;
    const float pr0 = A * m0.w[SA] + B * m0.w[SB], pr1 = A * m1.w[SA] - B * m1.w[SB];
    sv[SA] += A * (m0.dt + m1.dt);
    sv[SB] += B * (m0.dt - m1.dt);
    const float sum = m0.st + m1.st, dif = m0.st - m1.st;
    tv[tix(SA, SA)] += E1.x * sum;
    tv[tix(SB, SB)] += E1.y * sum;
    tv[tix(SA, SB)] += E1.z * dif;
    vv[SA] += A * (pr0 + pr1);
    vv[SB] += B * (pr0 - pr1);
}

struct TileSite {
    int tx, ty, tz, x, y, z;
    bool active;
    long long s;
    int c;   // LDS offset of the site
};

// Site of this thread: x fastest, then y, then z; z-paired tiles (LM 1)
// take x, then one bit of z, then y, then the rest of z; z-major tiles
// (LM 2) x, then z, then y.
template <int TX, int TY, int TZ, int LM = 0>
__device__ inline TileSite tile_site(const SysDesc<float> &S, const TileGeo &t)
{
    TileSite q;
    const int i = threadIdx.x % (TX * TY * TZ);
    q.tx = i % TX;
    if (LM == 1) {
        const int j = i / (2 * TX);
        q.ty = j % TY;
        q.tz = 2 * (j / TY) + (i / TX) % 2;
    } else if (LM == 2) {
        const int j = i / TX;
        q.tz = j % TZ;
        q.ty = j / TZ;
    } else {
        q.ty = (i / TX) % TY;
        q.tz = i / (TX * TY);
    }
    q.x = t.x0 + q.tx; q.y = t.y0 + q.ty; q.z = t.z0 + q.tz;
    q.active = q.x < S.nx && q.y < S.ny && q.z < S.nz;
    q.s = ((long long)q.z * S.ny + q.y) * S.nx + q.x;
    q.c = (q.tx + t.R) + (q.ty + t.R) * t.HX + (q.tz + t.R) * t.PXY;
    return q;
}

// ------------------------------------------------------------ first gather
template <int TX, int TY, int TZ, int SPLIT, bool GROUPED>
__global__ void __launch_bounds__(SPLIT * kBlock) __attribute__((amdgpu_waves_per_eu(MLB_G1_WAVES)))
k_gather1_tile(const SysDesc<float> *__restrict__ sys,
                                                         const int2 *__restrict__ bmap, Tables<float> tb)
{
    extern __shared__ float4 lds[];
    static_assert(TX * TY * TZ == kBlock && SPLIT >= 2 && SPLIT <= kSplitG1Max, "SPLIT threads per tile site");
    const int2 bm = bmap[blockIdx.x];
    if (bm.x < 0) return;
    const SysDesc<float> &S = sys[bm.x];
    const int a = blockIdx.y;
    if (a >= S.M) return;
    constexpr int LM = lane_layout(TX, TZ, MLB_G1_LAYOUTS);
    const TileGeo t = tile_geo<TX, TY, TZ, LM>(S, bm.y, S.reach);
    const TileSite q = tile_site<TX, TY, TZ, LM>(S, t);
    const int h = __builtin_amdgcn_readfirstlane(threadIdx.x / kBlock);   // wave-uniform
    const long long N = S.N;
    const long long o3 = (long long)a * 3 * N;
    float4 *L4 = lds;
    float *Lg = reinterpret_cast<float *>(lds + t.FS);
    int *RowOff = reinterpret_cast<int *>(lds + t.FS + (t.FS + 3) / 4);
    int *RowL = RowOff + t.HY * t.HZ;
    const int HXY = t.PXY;
    const StageLane sl = stage_lane<SPLIT * kBlock>(S, t);
    fill_rows<SPLIT * kBlock>(S, t, RowOff, LM ? RowL : nullptr);
    const char *c4 = reinterpret_cast<const char *>(L4 + q.c);
    const char *cg = reinterpret_cast<const char *>(Lg + q.c);
    const bool solid = q.active && S.walls && (q.y == 0 || q.y == S.ny - 1);
    // group 0 stores H and V-hat, group 1 the friction tensor and
    // (1/m_a) / (1 + Gamma / (2 m_a))
    const bool do_hv = h == 0, do_t = h == 1;
    const long long sc = q.active && (do_hv || do_t) ? q.s : 0;
    const float na = glb(S.n)[(long long)a * N + sc];
    const float ja0 = glb(S.j)[o3 + sc], ja1 = glb(S.j)[o3 + N + sc], ja2 = glb(S.j)[o3 + 2 * N + sc];
    float mf0 = 0.f, mf1 = 0.f, mf2 = 0.f, dj0 = 0.f, dj1 = 0.f, dj2 = 0.f, gam = 0.f;
    float T00 = 0.f, T01 = 0.f, T02 = 0.f, T11 = 0.f, T12 = 0.f, T22 = 0.f;
    for (int b = 0; b < S.M; ++b) {
        const gfloat *__restrict__ gpair = glb(S.g) + (long long)pidx(S.M, a, b) * N;
        int kb, ke;
        split_range<SPLIT>(S.sh_cnt[a][b], h, kb, ke);
        __syncthreads();
        stage<LM>(S, t, sl, RowOff, RowL, L4, Lg, glb(S.n) + (long long)b * N, glb(S.j) + (long long)b * 3 * N, gpair);
        __syncthreads();
        const float g0 = Lg[q.c];
        float s0 = 0.f, s1 = 0.f, s2 = 0.f, v0 = 0.f, v1 = 0.f, v2 = 0.f;
        float t00 = 0.f, t01 = 0.f, t02 = 0.f, t11 = 0.f, t12 = 0.f, t22 = 0.f;
        ConstF4 Q;
        if constexpr (GROUPED) {
            float sv[3] = {0.f, 0.f, 0.f}, tv[6] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f}, vv[3] = {0.f, 0.f, 0.f};
            // four-point groups: members (+y,+z), (-y,+z), (+y,-z), (-y,-z)
            {
                const ConstF4 Q = (ConstF4)(tb.sg_q + S.sg_start[a][b][0]);
                split_range<SPLIT>(S.sg_cnt[a][b][0], h, kb, ke);
#pragma unroll 1
                for (int k = kb; k < ke; ++k) {
                    const ShellEntry E0 = Q[4 * k], E1 = Q[4 * k + 1], E2 = Q[4 * k + 2], E3 = Q[4 * k + 3];
                    const G1Pt m0 = g1_point(c4, cg, g0, E0.x, t.HX, HXY), m1 = g1_point(c4, cg, g0, E0.y, t.HX, HXY);
                    const G1Pt m2 = g1_point(c4, cg, g0, E0.z, t.HX, HXY), m3 = g1_point(c4, cg, g0, E0.w, t.HX, HXY);
                    const float p = E1.x, qq = E1.y, r = E1.z;
                    const float pr0 = p * m0.w[0] + qq * m0.w[1] + r * m0.w[2];
                    const float pr1 = p * m1.w[0] - qq * m1.w[1] + r * m1.w[2];
                    const float pr2 = p * m2.w[0] + qq * m2.w[1] - r * m2.w[2];
                    const float pr3 = p * m3.w[0] - qq * m3.w[1] - r * m3.w[2];
                    const float dA = m0.dt + m2.dt, dB = m1.dt + m3.dt, dC = m0.dt - m2.dt, dD = m1.dt - m3.dt;
                    sv[0] += p * (dA + dB); sv[1] += qq * (dA - dB); sv[2] += r * (dC + dD);
                    const float sA = m0.st + m2.st, sB = m1.st + m3.st, sC = m0.st - m2.st, sD = m1.st - m3.st;
                    const float ss = sA + sB;
                    tv[0] += E2.x * ss; tv[3] += E2.y * ss; tv[5] += E2.z * ss;
                    tv[1] += E3.x * (sA - sB); tv[2] += E3.y * (sC + sD); tv[4] += E3.z * (sC - sD);
                    const float pA = pr0 + pr2, pB = pr1 + pr3, pC = pr0 - pr2, pD = pr1 - pr3;
                    vv[0] += p * (pA + pB); vv[1] += qq * (pA - pB); vv[2] += r * (pC + pD);
                }
            }
            // two-point groups
            {
                const ConstF4 Q = (ConstF4)(tb.sg_q + S.sg_start[a][b][1]);
                split_range<SPLIT>(S.sg_cnt[a][b][1], h, kb, ke);
#pragma unroll 2
                for (int k = kb; k < ke; ++k) g1_pair<0, 1>(Q[2 * k], Q[2 * k + 1], c4, cg, g0, t.HX, HXY, sv, tv, vv);
            }
            {
                const ConstF4 Q = (ConstF4)(tb.sg_q + S.sg_start[a][b][2]);
                split_range<SPLIT>(S.sg_cnt[a][b][2], h, kb, ke);
#pragma unroll 2
                for (int k = kb; k < ke; ++k) g1_pair<0, 2>(Q[2 * k], Q[2 * k + 1], c4, cg, g0, t.HX, HXY, sv, tv, vv);
            }
            {
                const ConstF4 Q = (ConstF4)(tb.sg_q + S.sg_start[a][b][3]);
                split_range<SPLIT>(S.sg_cnt[a][b][3], h, kb, ke);
#pragma unroll 2
                for (int k = kb; k < ke; ++k) g1_pair<1, 2>(Q[2 * k], Q[2 * k + 1], c4, cg, g0, t.HX, HXY, sv, tv, vv);
            }
            s0 = sv[0]; s1 = sv[1]; s2 = sv[2]; v0 = vv[0]; v1 = vv[1]; v2 = vv[2];
            t00 = tv[0]; t01 = tv[1]; t02 = tv[2]; t11 = tv[3]; t12 = tv[4]; t22 = tv[5];
            // single points on an axis: the plain form below
            split_range<SPLIT>(S.sg_cnt[a][b][4], h, kb, ke);
            Q = (ConstF4)(tb.sg_q + S.sg_start[a][b][4]);
        } else {
            Q = shell_list(tb, S.sh_start[a][b]);
        }
#pragma unroll MLB_G1_UNROLL
        for (int k = kb; k < ke; ++k) {
            const ShellEntry ta = Q[k];
            const int o4 = shell_off(ta.x, t.HX, HXY), o1 = o4 >> 2;
            const float e0 = ta.y, e1 = ta.z, e2 = ta.w;
            const float4 Ap = ld4(c4, o4), Am = ld4(c4, -o4);
            const float Gp = g0 + ld1(cg, o1), Gm = g0 + ld1(cg, -o1);
            const float tp = Gp * Ap.x, tm = Gm * Am.x;
            const float dt = tp - tm, st = tp + tm;
            s0 += e0 * dt; s1 += e1 * dt; s2 += e2 * dt;
            const float se0 = st * e0, se1 = st * e1, se2 = st * e2;
            t00 += se0 * e0; t01 += se0 * e1; t02 += se0 * e2;
            t11 += se1 * e1; t12 += se1 * e2; t22 += se2 * e2;
            const float w0 = Gp * Ap.y + Gm * Am.y;
            const float w1 = Gp * Ap.z + Gm * Am.z;
            const float w2 = Gp * Ap.w + Gm * Am.w;
            const float pr = e0 * w0 + e1 * w1 + e2 * w2;
            v0 += e0 * pr; v1 += e1 * pr; v2 += e2 * pr;
        }
        const float cm = S.cm[a][b], ck = S.ck[a][b];
        mf0 += cm * s0; mf1 += cm * s1; mf2 += cm * s2;
        dj0 += ck * v0; dj1 += ck * v1; dj2 += ck * v2;
        T00 += ck * t00; T01 += ck * t01; T02 += ck * t02;
        T11 += ck * t11; T12 += ck * t12; T22 += ck * t22;
        gam += S.cg[a][b] * (t00 + t11 + t22);
    }
    float part[13] = {mf0, mf1, mf2, dj0, dj1, dj2, gam, T00, T01, T02, T11, T12, T22};
    split_allreduce<SPLIT>(lds, part);
    mf0 = part[0]; mf1 = part[1]; mf2 = part[2]; dj0 = part[3]; dj1 = part[4]; dj2 = part[5]; gam = part[6];
    T00 = part[7]; T01 = part[8]; T02 = part[9]; T11 = part[10]; T12 = part[11]; T22 = part[12];
    if (!q.active || !(do_hv || do_t)) return;
    const long long s = q.s;
    gfloat *__restrict__ Tout = glb(S.Tloc) + (long long)a * 6 * N;
    if (solid) {
        if (do_hv)
            for (int d = 0; d < 3; ++d) {
                glb(S.vh)[o3 + d * N + s] = 0.f;
                glb(S.H)[o3 + d * N + s] = 0.f;
                if (S.parts) glb(S.parts)[o3 + d * N + s] = 0.f;
            }
        if (do_t) {
            for (int d = 0; d < 6; ++d) Tout[d * N + s] = 0.f;
            if (S.tail_deferred) glb(S.gfac)[(long long)a * N + s] = 0.f;
        }
        return;
    }
    // a force density changes the number flux at the rate 1/m_a
    const float im = S.im[a];
    const float hg = (0.5f * gam) * im;
    if (do_t) {
        // the deferred spectral field enters V-hat as (1/m_a) C_a / (1 + hg)
        if (S.tail_deferred) glb(S.gfac)[(long long)a * N + s] = (na != 0.f) ? im / (1.f + hg) : 0.f;
        Tout[0 * N + s] = T00; Tout[1 * N + s] = T01; Tout[2 * N + s] = T02;
        Tout[3 * N + s] = T11; Tout[4 * N + s] = T12; Tout[5 * N + s] = T22;
    }
    if (!do_hv) return;
    float tl0 = 0.f, tl1 = 0.f, tl2 = 0.f;
    if (S.tail && !S.tail_deferred) {
        tl0 = glb(S.tail)[o3 + s]; tl1 = glb(S.tail)[o3 + N + s]; tl2 = glb(S.tail)[o3 + 2 * N + s];
    }
    const float mfv[3] = {mf0, mf1, mf2}, tlv[3] = {tl0, tl1, tl2}, jav[3] = {ja0, ja1, ja2};
    const float djv[3] = {dj0, dj1, dj2};
    const float Tj[3] = {T00 * ja0 + T01 * ja1 + T02 * ja2, T01 * ja0 + T11 * ja1 + T12 * ja2,
                         T02 * ja0 + T12 * ja1 + T22 * ja2};
#pragma unroll
    for (int d = 0; d < 3; ++d) {
        const float fe = S.fprof ? glb(const_cast<float *>(S.fprof))[((long long)a * 3 + d) * S.ny + q.y]
                                 : S.fext[a][d];
        const float Nmf = na * mfv[d], Ntl = na * tlv[d], Nex = na * fe;
        const float Nc = Nmf + Ntl + Nex;
        const float Dd = na * djv[d] - Tj[d];
        if (S.scheme == 1) {
            glb(S.H)[o3 + d * N + s] = Nc + Dd;
            glb(S.vh)[o3 + d * N + s] = 0.f;
        } else {
            glb(S.H)[o3 + d * N + s] = Nc + 0.5f * Dd;
            glb(S.vh)[o3 + d * N + s] =
                (na != 0.f) ? ((jav[d] + im * Nc) + im * Dd + hg * jav[d]) / (na * (1.f + hg)) : 0.f;
        }
        if (S.parts) {
            float acc = 0.f;
            if (S.parts_mask & 1u) acc += Nmf;
            if (S.parts_mask & 2u) acc += Ntl;
            if (S.parts_mask & 8u) acc += Nex;
            if (S.parts_mask & 4u) acc += (S.scheme == 1 ? Dd : 0.5f * Dd);
            glb(S.parts)[o3 + d * N + s] = acc;
        }
    }
}

// c.v for a lattice velocity c (components -1, 0, 1): signed sums of the
// components, no products; -0 is the exact identity of the first addition
__device__ inline float cdot(int cx, int cy, int cz, const float v[3])
{
    float acc = -0.f;
    if (cx) acc += cx > 0 ? v[0] : -v[0];
    if (cy) acc += cy > 0 ? v[1] : -v[1];
    if (cz) acc += cz > 0 ? v[2] : -v[2];
    return acc;
}

// ------------------------------- second gather + collision + push streaming
template <int TX, int TY, int TZ>
__global__ void __launch_bounds__(kStep2Threads) __attribute__((amdgpu_waves_per_eu(MLB_S2_WAVES)))
k_step2_tile(const SysDesc<float> *__restrict__ sys,
                                                       const int2 *__restrict__ bmap, Tables<float> tb, int parity,
                                                       int write_force_only)
{
    extern __shared__ float4 lds[];
    static_assert(TX * TY * TZ == kBlock, "kSplitS2 threads per tile site");
    const int2 bm = bmap[blockIdx.x];
    if (bm.x < 0) return;
    const SysDesc<float> &S = sys[bm.x];
    const int a = blockIdx.y;
    if (a >= S.M) return;
    constexpr int LM = lane_layout(TX, TZ, MLB_S2_LAYOUTS);
    const TileGeo t = tile_geo<TX, TY, TZ, LM>(S, bm.y, S.reach);
    const TileSite q = tile_site<TX, TY, TZ, LM>(S, t);
    const long long N = S.N;
    const long long o3 = (long long)a * 3 * N;
    float4 *L4 = lds;
    int *RowOff = reinterpret_cast<int *>(lds + t.FS);
    int *RowL = RowOff + t.HY * t.HZ;
    const int HXY = t.PXY;
    const int h = __builtin_amdgcn_readfirstlane(threadIdx.x / kBlock);   // wave-uniform
    // The collision's inputs are loaded before the gathers, so that their
    // latency hides behind the shell loops.  Every group forms the total
    // force; group h collides and streams populations [ib, ie).
    constexpr int kPer = (kQ + kSplitS2 - 1) / kSplitS2;
    const int ib = min(kQ, h * kPer), ie = min(kQ, ib + kPer);
    const bool fluid = q.active && !(S.walls && (q.y == 0 || q.y == S.ny - 1));
    const bool epi = fluid && (ib < ie || (h == 0 && write_force_only));
    const bool need_f = epi && !write_force_only && S.omega_is_one == 0;
    const long long s = q.s;
    float na = 0.f, Na[3] = {0.f, 0.f, 0.f}, Tl[6] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f}, va[3] = {0.f, 0.f, 0.f};
    float ja[3] = {0.f, 0.f, 0.f}, u[3] = {0.f, 0.f, 0.f}, fi[kQ];
    if (epi) {
        na = glb(S.n)[(long long)a * N + s];
#pragma unroll
        for (int d = 0; d < 3; ++d) Na[d] = glb(S.H)[o3 + d * N + s];
        if (S.scheme != 1) {
            const gfloat *__restrict__ Tg = glb(S.Tloc) + (long long)a * 6 * N;
#pragma unroll
            for (int d = 0; d < 6; ++d) Tl[d] = Tg[d * N + s];
#pragma unroll
            for (int d = 0; d < 3; ++d) va[d] = glb(S.vh)[o3 + d * N + s];
        }
        if (!write_force_only) {
#pragma unroll
            for (int d = 0; d < 3; ++d) {
                ja[d] = glb(S.j)[o3 + d * N + s];
                u[d] = glb(S.u)[d * N + s];
            }
        }
    }
    {
        const gfloat *__restrict__ fin = glb(S.f[parity]) + (long long)a * kQ * N;
#pragma unroll
        for (int i = 0; i < kQ; ++i) fi[i] = (need_f && i >= ib && i < ie) ? fin[(long long)i * N + s] : 0.f;
    }
    float acc0 = 0.f, acc1 = 0.f, acc2 = 0.f;
    if (S.scheme != 1) {
        const StageLane sl = stage_lane<kStep2Threads>(S, t);
        fill_rows<kStep2Threads>(S, t, RowOff, LM ? RowL : nullptr);
        const char *c4 = reinterpret_cast<const char *>(L4 + q.c);
        for (int b = 0; b < S.M; ++b) {
            const gfloat *__restrict__ gpair = glb(S.g) + (long long)pidx(S.M, a, b) * N;
            int kb, ke;
            split_range<kSplitS2>(S.sh_cnt[a][b], h, kb, ke);
            __syncthreads();
            stage_nv<LM>(S, t, sl, RowOff, RowL, L4, glb(S.n) + (long long)b * N, glb(S.vh) + (long long)b * 3 * N,
                         gpair);
            __syncthreads();
            const ConstF4 Q = shell_list(tb, S.sh_start[a][b]);
            const float g0 = L4[q.c].w;
            float v0 = 0.f, v1 = 0.f, v2 = 0.f;
#pragma unroll MLB_S2_UNROLL
            for (int k = kb; k < ke; ++k) {
                const ShellEntry ta = Q[k];
                const int o4 = shell_off(ta.x, t.HX, HXY);
                const float e0 = ta.y, e1 = ta.z, e2 = ta.w;
                const float4 Ap = ld4(c4, o4), Am = ld4(c4, -o4);
                const float Gp = g0 + Ap.w, Gm = g0 + Am.w;
                const float w0 = Gp * Ap.x + Gm * Am.x;
                const float w1 = Gp * Ap.y + Gm * Am.y;
                const float w2 = Gp * Ap.z + Gm * Am.z;
                const float pr = e0 * w0 + e1 * w1 + e2 * w2;
                v0 += e0 * pr; v1 += e1 * pr; v2 += e2 * pr;
            }
            const float ck = S.ck[a][b];
            acc0 += ck * v0; acc1 += ck * v1; acc2 += ck * v2;
        }
        float part[3] = {acc0, acc1, acc2};
        split_allreduce<kSplitS2>(lds, part);
        acc0 = part[0]; acc1 = part[1]; acc2 = part[2];
    }
    if (!q.active) return;
    if (!fluid) {
        if (write_force_only && h == 0)
            for (int d = 0; d < 3; ++d) glb(S.Nf)[o3 + d * N + s] = 0.f;
        return;
    }
    if (!epi) return;
    if (S.scheme != 1) {
        const float T00 = Tl[0], T01 = Tl[1], T02 = Tl[2], T11 = Tl[3], T12 = Tl[4], T22 = Tl[5];
        const float va0 = va[0], va1 = va[1], va2 = va[2];
        const float Dn[3] = {na * (acc0 - (T00 * va0 + T01 * va1 + T02 * va2)),
                             na * (acc1 - (T01 * va0 + T11 * va1 + T12 * va2)),
                             na * (acc2 - (T02 * va0 + T12 * va1 + T22 * va2))};
#pragma unroll
        for (int d = 0; d < 3; ++d) {
            Na[d] += 0.5f * Dn[d];
            if (h == 0 && S.parts && (S.parts_mask & 4u)) glb(S.parts)[o3 + d * N + s] += 0.5f * Dn[d];
        }
    }
    if (write_force_only) {
        if (h == 0)
            for (int d = 0; d < 3; ++d) glb(S.Nf)[o3 + d * N + s] = Na[d];
        return;
    }
    gfloat *__restrict__ fout = glb(S.f[parity ^ 1]) + (long long)a * kQ * N;
    // The collision of eq. (evolution) with the force term, regrouped so that
    // only the parts that depend on c_i stay inside the population loop:
    //   omega psi_i + src_i = w_i E_i (A + 3 c_i.P),
    //   E_i = (1 - 3/2 u.u) + c_i.u (3 + 9/2 c_i.u) [+ dth (c_i.c_i - 1)],
    //   P = omega m_a (j - n u) + N,  A = omega n - 3 u.P
    // (psi_i = w_i E_i (n + (m_a/kT) (j - n u).(c_i - u)), src_i = 3 w_i E_i
    // (c_i - u).N, with m_a/kT = 3 m_a; dth = (9/2)(kT/m_a - 1/3)).
    const bool w1 = S.omega_is_one != 0;
    const float om = w1 ? 1.f : S.omega;
    const float uu = (u[0] * u[0] + u[1] * u[1]) + u[2] * u[2];
    const float B = 1.f - 1.5f * uu;
    const float omm = om * S.mass[a], dth = S.dth[a];
    float P[3];
#pragma unroll
    for (int d = 0; d < 3; ++d) P[d] = omm * (ja[d] - na * u[d]) + Na[d];
    const float A = om * na - 3.f * ((u[0] * P[0] + u[1] * P[1]) + u[2] * P[2]);
    // neighbour offsets with periodic wrap (32-bit: sites number below 2^29);
    // beyond a wall the population bounces back instead
    const int nx = S.nx, nxy = S.nx * S.ny, s32 = (int)s;
    const int ox[2] = {q.x == 0 ? nx - 1 : -1, q.x == nx - 1 ? 1 - nx : 1};
    const int oy[2] = {q.y == 0 ? nxy - nx : -nx, q.y == S.ny - 1 ? nx - nxy : nx};
    const int nall = (int)S.N;
    const int oz[2] = {q.z == 0 ? nall - nxy : -nxy, q.z == S.nz - 1 ? nxy - nall : nxy};
    const bool wlo = S.walls && q.y == 1, whi = S.walls && q.y == S.ny - 2;
#pragma unroll
    for (int i = 0; i < kQ; ++i) {
        if (i < ib || i >= ie) continue;
        const int cx = kC[i][0], cy = kC[i][1], cz = kC[i][2];
        const float cu = cdot(cx, cy, cz, u), cP = cdot(cx, cy, cz, P);
        float E = B + cu * (3.f + 4.5f * cu);
        if (!S.unit_mass) E += dth * (float)(cx * cx + cy * cy + cz * cz - 1);
        float fs = (lattice_weight<float>(i) * E) * (A + 3.f * cP);
        if (!w1) fs += S.om1 * fi[i];
        if ((cy < 0 && wlo) || (cy > 0 && whi)) {
            const float uw = cy < 0 ? S.wall_ux[0] : S.wall_ux[1];
            fout[(long long)opposite(i) * N + s] = fs - ((6.f * lattice_weight<float>(i)) * na) * ((float)cx * uw);
        } else {
            int o = s32;
            if (cx) o += ox[cx > 0];
            if (cy) o += oy[cy > 0];
            if (cz) o += oz[cz > 0];
            fout[(long long)i * N + o] = fs;
        }
    }
}

// ---------------------------------------------------------- contact values
// Same fields as k_contact (ball-smoothed densities -> BMCSL contact values,
// ball sums in the same order: centre, then each (+e, -e) pair of the
// half-list); the densities of every species are staged for the tile plus a
// halo of the ball reach.  LDS: M float arrays, the ball half-lists of all
// species (index offsets), the row-offset table.
template <int TX, int TY, int TZ>
__global__ void __launch_bounds__(kBlock) k_contact_tile(const SysDesc<float> *__restrict__ sys,
                                                         const int2 *__restrict__ bmap, Tables<float> tb)
{
    extern __shared__ float4 lds[];
    static_assert(TX * TY * TZ == kBlock, "one thread per tile site");
    const int2 bm = bmap[blockIdx.x];
    if (bm.x < 0) return;
    const SysDesc<float> &S = sys[bm.x];
    const TileGeo t = tile_geo<TX, TY, TZ>(S, bm.y, S.ball_reach);
    const TileSite q = tile_site<TX, TY, TZ>(S, t);
    const long long N = S.N;
    float *Ln = reinterpret_cast<float *>(lds);
    int *Off = reinterpret_cast<int *>(Ln + S.M * t.FS);
    int *RowOff = Off + S.ball_total;
    const StageLane sl = stage_lane(S, t);
    fill_rows(S, t, RowOff);
    const int kb = S.bl_start[0];
    for (int k = threadIdx.x; k < S.ball_total; k += kBlock) {
        int ex, ey, ez;
        unpack_offset(tb.bl_e[kb + k], ex, ey, ez);
        Off[k] = ex + ey * t.HX + ez * t.HX * t.HY;
    }
    __syncthreads();
    for (int c = 0; c < S.M; ++c) stage1(t, sl, RowOff, Ln + c * t.FS, glb(S.n) + (long long)c * N);
    __syncthreads();
    if (!q.active) return;
    const long long s = q.s;
    if (S.walls && (q.y == 0 || q.y == S.ny - 1)) {
        for (int p = 0; p < S.P; ++p) glb(S.g)[(long long)p * N + s] = 0.f;
        return;
    }
    float nb[kMaxS];
    for (int c = 0; c < S.M; ++c) {
        const float *L = Ln + c * t.FS + q.c;
        float acc = L[0];
        const int k0 = S.bl_start[c] - kb, kn = S.bl_cnt[c];
        for (int k = 0; k < kn; ++k) {
            const int o = Off[k0 + k];
            acc = acc + (L[o] + L[-o]);
        }
        nb[c] = acc / (float)S.bl_full[c];
    }
    float x2 = S.s2[0] * nb[0], x3 = S.s3[0] * nb[0];
    for (int c = 1; c < S.M; ++c) {
        x2 = x2 + S.s2[c] * nb[c];
        x3 = x3 + S.s3[c] * nb[c];
    }
    const float qf = 1.f / (1.f - x3);
    for (int a = 0; a < S.M; ++a)
        for (int b = a; b < S.M; ++b) {
            const float z = (S.dd[a][b] * x2) * qf;
            glb(S.g)[(long long)pidx(S.M, a, b) * N + s] = qf * ((1.f + z) * (1.f + 2.f * z));
        }
}

inline size_t contact_lds_bytes(int TX, int TY, int TZ, int R, int ball_total, int maxM)
{
    const size_t FS = (size_t)(TX + 2 * R) * (TY + 2 * R) * (TZ + 2 * R);
    const size_t rows = (size_t)(TY + 2 * R) * (TZ + 2 * R);
    return 4 * ((size_t)maxM * FS + (size_t)ball_total + rows);
}

// float4 + float per staged site in the first gather, one float4 in the
// second (z planes padded on z-paired shapes), then the row-offset table
// and, z-paired, the row-base table (one int each per halo row); at least
// the partial sums of the split reductions (13 floats per site and group in
// the first gather, 3 in the second)
inline size_t tile_lds_bytes(int TX, int TY, int TZ, int R, int layouts, bool second)
{
    const int plane = (TX + 2 * R) * (TY + 2 * R);
    const int LM = lane_layout(TX, TZ, layouts);
    const bool zp = LM != 0;
    const size_t FS = (size_t)plane_pitch(LM, plane) * (TZ + 2 * R);
    const size_t rows = (size_t)(TY + 2 * R) * (TZ + 2 * R);
    const size_t reduce = (second ? (size_t)kSplitS2 * 3 : (size_t)kSplitG1Max * 13) * kBlock * 4;
    return std::max(16 * FS + (second ? 0 : 16 * ((FS + 3) / 4)) + (zp ? 8 : 4) * rows, reduce);
}

}  // namespace mlb
