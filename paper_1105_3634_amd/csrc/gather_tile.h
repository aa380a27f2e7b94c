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
// block stages n_b, the three components of j_b (or V_b) and g_ab for the
// tile plus a halo of R cells (R = largest stencil component of the
// system) into LDS; periodic wrap and walls are resolved while filling, so
// the inner loop is address arithmetic on a uniform offset and LDS loads.
#pragma once

#include "step_kernels.h"

namespace mlb {

constexpr int kTileFields = 5;   // n, v0, v1, v2, g

struct TileGeo {
    int x0, y0, z0;       // tile origin
    int R, HX, HY, HZ;    // halo width and staged extents
    int FS;               // floats per staged field
};

template <int TX, int TY, int TZ>
__device__ inline TileGeo tile_geo(const SysDesc<float> &S, int local, int R)
{
    TileGeo t;
    const int tx = (S.nx + TX - 1) / TX, ty = (S.ny + TY - 1) / TY;
    const int bx = local % tx, by = (local / tx) % ty, bz = local / (tx * ty);
    t.x0 = bx * TX; t.y0 = by * TY; t.z0 = bz * TZ;
    t.R = R;
    t.HX = TX + 2 * t.R; t.HY = TY + 2 * t.R; t.HZ = TZ + 2 * t.R;
    t.FS = t.HX * t.HY * t.HZ;
    return t;
}

// Staging of the halo tile.  Rows (hy, hz) of the tile are numbered
// row = hy + HY hz; RowOff[row] holds the global site offset of the row's
// x = 0 site ((gz ny + gy) nx after periodic wrap), or -1 for a row outside
// the walls.  Thread t owns the halo column hx = t % HX (its wrapped global
// x computed once) and the rows t / HX, t / HX + 256 / HX, ...; consecutive
// threads read consecutive x, so global loads coalesce, and the per-element
// work is a table read, an add and the loads.
__device__ inline int wrap_mod(int v, int n)
{
    v %= n;
    return v < 0 ? v + n : v;
}

struct StageLane {
    int hx, row0, rstep;   // rstep = 0: the thread stages nothing
    int gx;
};

__device__ inline StageLane stage_lane(const SysDesc<float> &S, const TileGeo &t)
{
    StageLane l;
    l.rstep = kBlock / t.HX;
    l.hx = threadIdx.x % t.HX;
    l.row0 = threadIdx.x / t.HX;
    if (l.row0 >= l.rstep) l.rstep = 0;          // left-over threads of the last partial column set
    l.gx = wrap_mod(t.x0 - t.R + l.hx, S.nx);
    return l;
}

__device__ inline void fill_rows(const SysDesc<float> &S, const TileGeo &t, int *RowOff)
{
    const int rows = t.HY * t.HZ;
    for (int r = threadIdx.x; r < rows; r += kBlock) {
        const int hz = r / t.HY, hy = r - hz * t.HY;
        int gy = t.y0 - t.R + hy;
        const int gz = wrap_mod(t.z0 - t.R + hz, S.nz);
        if (S.walls) {
            RowOff[r] = (gy >= 0 && gy < S.ny) ? (gz * S.ny + gy) * S.nx : -1;
        } else {
            gy = wrap_mod(gy, S.ny);
            RowOff[r] = (gz * S.ny + gy) * S.nx;
        }
    }
}

__device__ inline void stage(const SysDesc<float> &S, const TileGeo &t, const StageLane &l, const int *RowOff,
                             float4 *lds4, float *ldsg, const float *__restrict__ nb, const float *__restrict__ vb,
                             const float *__restrict__ gp)
{
    const unsigned N = (unsigned)S.N;
    const int rows = t.HY * t.HZ;
    if (l.rstep == 0) return;
    for (int row = l.row0; row < rows; row += l.rstep) {
        const int ro = RowOff[row];
        const int i = l.hx + row * t.HX;
        float4 v = make_float4(0.f, 0.f, 0.f, 0.f);
        float g = 0.f;
        if (ro >= 0) {
            const unsigned so = (unsigned)(ro + l.gx);
            v = make_float4(nb[so], vb[so], vb[N + so], vb[2 * N + so]);
            g = gp[so];
        }
        lds4[i] = v;
        ldsg[i] = g;
    }
}

// One scalar field of the halo tile (zero outside the walls).
__device__ inline void stage1(const TileGeo &t, const StageLane &l, const int *RowOff, float *dst,
                              const float *__restrict__ src)
{
    const int rows = t.HY * t.HZ;
    if (l.rstep == 0) return;
    for (int row = l.row0; row < rows; row += l.rstep) {
        const int ro = RowOff[row];
        dst[l.hx + row * t.HX] = ro >= 0 ? src[(unsigned)(ro + l.gx)] : 0.f;
    }
}

// Copy the (a,b) half-shell into LDS: TA[k] = (byte offset of e in the
// float4 field array, e_hat); the g array's offset is a quarter of it and
// the tensor e_hat e_hat^T is formed in registers.  Reads of TA are
// wave-uniform broadcasts; every LDS read costs bandwidth, so the table
// holds no more than this.
__device__ inline void stage_table(const Tables<float> &tb, int k0, int kn, const TileGeo &t, float4 *TA)
{
    const int HXY = t.HX * t.HY;
    for (int k = threadIdx.x; k < kn; k += kBlock) {
        int ex, ey, ez;
        unpack_offset(tb.sh_e[k0 + k], ex, ey, ez);
        const int off = ex + ey * t.HX + ez * HXY;
        const float *u = tb.sh_u + 3 * (k0 + k);
        TA[k] = make_float4(__int_as_float(16 * off), u[0], u[1], u[2]);
    }
}

// field reads at a byte offset from the site's own address
__device__ inline float4 ld4(const char *base, int byte) { return *reinterpret_cast<const float4 *>(base + byte); }
__device__ inline float ld1(const char *base, int byte) { return *reinterpret_cast<const float *>(base + byte); }

struct TileSite {
    int tx, ty, tz, x, y, z;
    bool active;
    long long s;
    int c;   // LDS offset of the site
};

template <int TX, int TY, int TZ>
__device__ inline TileSite tile_site(const SysDesc<float> &S, const TileGeo &t)
{
    TileSite q;
    q.tx = threadIdx.x % TX;
    q.ty = (threadIdx.x / TX) % TY;
    q.tz = threadIdx.x / (TX * TY);
    q.x = t.x0 + q.tx; q.y = t.y0 + q.ty; q.z = t.z0 + q.tz;
    q.active = q.x < S.nx && q.y < S.ny && q.z < S.nz;
    q.s = ((long long)q.z * S.ny + q.y) * S.nx + q.x;
    q.c = (q.tx + t.R) + (q.ty + t.R) * t.HX + (q.tz + t.R) * t.HX * t.HY;
    return q;
}

// ------------------------------------------------------------ first gather
template <int TX, int TY, int TZ>
__global__ void __launch_bounds__(kBlock) k_gather1_tile(const SysDesc<float> *__restrict__ sys,
                                                         const int2 *__restrict__ bmap, Tables<float> tb)
{
    extern __shared__ float4 lds[];
    static_assert(TX * TY * TZ == kBlock, "one thread per tile site");
    const int2 bm = bmap[blockIdx.x];
    if (bm.x < 0) return;
    const SysDesc<float> &S = sys[bm.x];
    const int a = blockIdx.y;
    if (a >= S.M) return;
    const TileGeo t = tile_geo<TX, TY, TZ>(S, bm.y, S.reach);
    const TileSite q = tile_site<TX, TY, TZ>(S, t);
    const long long N = S.N;
    const long long o3 = (long long)a * 3 * N;
    float4 *L4 = lds;
    float *Lg = reinterpret_cast<float *>(lds + t.FS);
    float4 *TA = lds + t.FS + (t.FS + 3) / 4;
    int *RowOff = reinterpret_cast<int *>(TA + S.sh_max);
    const StageLane sl = stage_lane(S, t);
    fill_rows(S, t, RowOff);
    const char *c4 = reinterpret_cast<const char *>(L4 + q.c);
    const char *cg = reinterpret_cast<const char *>(Lg + q.c);
    const bool solid = q.active && S.walls && (q.y == 0 || q.y == S.ny - 1);
    const long long sc = q.active ? q.s : 0;
    const float na = S.n[(long long)a * N + sc];
    const float ja0 = S.j[o3 + sc], ja1 = S.j[o3 + N + sc], ja2 = S.j[o3 + 2 * N + sc];
    float mf0 = 0.f, mf1 = 0.f, mf2 = 0.f, dj0 = 0.f, dj1 = 0.f, dj2 = 0.f, gam = 0.f;
    float T00 = 0.f, T01 = 0.f, T02 = 0.f, T11 = 0.f, T12 = 0.f, T22 = 0.f;
    for (int b = 0; b < S.M; ++b) {
        const float *__restrict__ gpair = S.g + (long long)pidx(S.M, a, b) * N;
        const int k0 = S.sh_start[a][b], kn = S.sh_cnt[a][b];
        __syncthreads();
        stage(S, t, sl, RowOff, L4, Lg, S.n + (long long)b * N, S.j + (long long)b * 3 * N, gpair);
        stage_table(tb, k0, kn, t, TA);
        __syncthreads();
        const float g0 = Lg[q.c];
        float s0 = 0.f, s1 = 0.f, s2 = 0.f, v0 = 0.f, v1 = 0.f, v2 = 0.f;
        float t00 = 0.f, t01 = 0.f, t02 = 0.f, t11 = 0.f, t12 = 0.f, t22 = 0.f;
#pragma unroll 4
        for (int k = 0; k < kn; ++k) {
            const float4 ta = TA[k];
            const int o4 = __float_as_int(ta.x), o1 = o4 >> 2;
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
    if (!q.active) return;
    const long long s = q.s;
    float *__restrict__ Tout = S.Tloc + (long long)a * 6 * N;
    if (solid) {
        for (int d = 0; d < 3; ++d) {
            S.vh[o3 + d * N + s] = 0.f;
            S.H[o3 + d * N + s] = 0.f;
            if (S.parts) S.parts[o3 + d * N + s] = 0.f;
        }
        for (int d = 0; d < 6; ++d) Tout[d * N + s] = 0.f;
        if (S.tail_deferred) S.gfac[(long long)a * N + s] = 0.f;
        return;
    }
    float tl0 = 0.f, tl1 = 0.f, tl2 = 0.f;
    if (S.tail && !S.tail_deferred) {
        tl0 = S.tail[o3 + s]; tl1 = S.tail[o3 + N + s]; tl2 = S.tail[o3 + 2 * N + s];
    }
    const float mfv[3] = {mf0, mf1, mf2}, tlv[3] = {tl0, tl1, tl2}, jav[3] = {ja0, ja1, ja2};
    const float djv[3] = {dj0, dj1, dj2};
    const float Tj[3] = {T00 * ja0 + T01 * ja1 + T02 * ja2, T01 * ja0 + T11 * ja1 + T12 * ja2,
                         T02 * ja0 + T12 * ja1 + T22 * ja2};
    const float hg = 0.5f * gam;
    if (S.tail_deferred) S.gfac[(long long)a * N + s] = (na != 0.f) ? 1.f / (1.f + hg) : 0.f;
#pragma unroll
    for (int d = 0; d < 3; ++d) {
        const float Nmf = na * mfv[d], Ntl = na * tlv[d], Nex = na * S.fext[a][d];
        const float Nc = Nmf + Ntl + Nex;
        const float Dd = na * djv[d] - Tj[d];
        if (S.scheme == 1) {
            S.H[o3 + d * N + s] = Nc + Dd;
            S.vh[o3 + d * N + s] = 0.f;
        } else {
            S.H[o3 + d * N + s] = Nc + 0.5f * Dd;
            S.vh[o3 + d * N + s] = (na != 0.f) ? (jav[d] + Nc + Dd + hg * jav[d]) / (na * (1.f + hg)) : 0.f;
        }
        if (S.parts) {
            float acc = 0.f;
            if (S.parts_mask & 1u) acc += Nmf;
            if (S.parts_mask & 2u) acc += Ntl;
            if (S.parts_mask & 8u) acc += Nex;
            if (S.parts_mask & 4u) acc += (S.scheme == 1 ? Dd : 0.5f * Dd);
            S.parts[o3 + d * N + s] = acc;
        }
    }
    Tout[0 * N + s] = T00; Tout[1 * N + s] = T01; Tout[2 * N + s] = T02;
    Tout[3 * N + s] = T11; Tout[4 * N + s] = T12; Tout[5 * N + s] = T22;
}

// ------------------------------- second gather + collision + push streaming
template <int TX, int TY, int TZ>
__global__ void __launch_bounds__(kBlock) k_step2_tile(const SysDesc<float> *__restrict__ sys,
                                                       const int2 *__restrict__ bmap, Tables<float> tb, int parity,
                                                       int write_force_only)
{
    extern __shared__ float4 lds[];
    static_assert(TX * TY * TZ == kBlock, "one thread per tile site");
    const int2 bm = bmap[blockIdx.x];
    if (bm.x < 0) return;
    const SysDesc<float> &S = sys[bm.x];
    const int a = blockIdx.y;
    if (a >= S.M) return;
    const TileGeo t = tile_geo<TX, TY, TZ>(S, bm.y, S.reach);
    const TileSite q = tile_site<TX, TY, TZ>(S, t);
    const long long N = S.N;
    const long long o3 = (long long)a * 3 * N;
    float4 *L4 = lds;
    float *Lg = reinterpret_cast<float *>(lds + t.FS);
    float4 *TA = lds + t.FS + (t.FS + 3) / 4;
    int *RowOff = reinterpret_cast<int *>(TA + S.sh_max);
    float acc0 = 0.f, acc1 = 0.f, acc2 = 0.f;
    if (S.scheme != 1) {
        const StageLane sl = stage_lane(S, t);
        fill_rows(S, t, RowOff);
        const char *c4 = reinterpret_cast<const char *>(L4 + q.c);
        const char *cg = reinterpret_cast<const char *>(Lg + q.c);
        for (int b = 0; b < S.M; ++b) {
            const float *__restrict__ gpair = S.g + (long long)pidx(S.M, a, b) * N;
            const int k0 = S.sh_start[a][b], kn = S.sh_cnt[a][b];
            __syncthreads();
            stage(S, t, sl, RowOff, L4, Lg, S.n + (long long)b * N, S.vh + (long long)b * 3 * N, gpair);
            stage_table(tb, k0, kn, t, TA);
            __syncthreads();
            const float g0 = Lg[q.c];
            float v0 = 0.f, v1 = 0.f, v2 = 0.f;
#pragma unroll 4
            for (int k = 0; k < kn; ++k) {
                const float4 ta = TA[k];
                const int o4 = __float_as_int(ta.x), o1 = o4 >> 2;
                const float e0 = ta.y, e1 = ta.z, e2 = ta.w;
                const float4 Ap = ld4(c4, o4), Am = ld4(c4, -o4);
                const float tp = (g0 + ld1(cg, o1)) * Ap.x, tm = (g0 + ld1(cg, -o1)) * Am.x;
                const float w0 = tp * Ap.y + tm * Am.y;
                const float w1 = tp * Ap.z + tm * Am.z;
                const float w2 = tp * Ap.w + tm * Am.w;
                const float pr = e0 * w0 + e1 * w1 + e2 * w2;
                v0 += e0 * pr; v1 += e1 * pr; v2 += e2 * pr;
            }
            const float ck = S.ck[a][b];
            acc0 += ck * v0; acc1 += ck * v1; acc2 += ck * v2;
        }
    }
    if (!q.active) return;
    const long long s = q.s;
    if (S.walls && (q.y == 0 || q.y == S.ny - 1)) {
        if (write_force_only)
            for (int d = 0; d < 3; ++d) S.Nf[o3 + d * N + s] = 0.f;
        return;
    }
    const float na = S.n[(long long)a * N + s];
    float Na[3] = {S.H[o3 + s], S.H[o3 + N + s], S.H[o3 + 2 * N + s]};
    if (S.scheme != 1) {
        const float *__restrict__ Tl = S.Tloc + (long long)a * 6 * N;
        const float T00 = Tl[s], T01 = Tl[N + s], T02 = Tl[2 * N + s], T11 = Tl[3 * N + s], T12 = Tl[4 * N + s],
                    T22 = Tl[5 * N + s];
        const float va0 = S.vh[o3 + s], va1 = S.vh[o3 + N + s], va2 = S.vh[o3 + 2 * N + s];
        const float Dn[3] = {na * (acc0 - (T00 * va0 + T01 * va1 + T02 * va2)),
                             na * (acc1 - (T01 * va0 + T11 * va1 + T12 * va2)),
                             na * (acc2 - (T02 * va0 + T12 * va1 + T22 * va2))};
#pragma unroll
        for (int d = 0; d < 3; ++d) {
            Na[d] += 0.5f * Dn[d];
            if (S.parts && (S.parts_mask & 4u)) S.parts[o3 + d * N + s] += 0.5f * Dn[d];
        }
    }
    if (write_force_only) {
        for (int d = 0; d < 3; ++d) S.Nf[o3 + d * N + s] = Na[d];
        return;
    }
    const float ja[3] = {S.j[o3 + s], S.j[o3 + N + s], S.j[o3 + 2 * N + s]};
    const float u[3] = {S.u[s], S.u[N + s], S.u[2 * N + s]};
    const float *__restrict__ fin = S.f[parity] + (long long)a * kQ * N;
    float *__restrict__ fout = S.f[parity ^ 1] + (long long)a * kQ * N;
    const bool w1 = S.omega_is_one != 0;
    const Site r{q.x, q.y, q.z};
#pragma unroll
    for (int i = 0; i < kQ; ++i) {
        const float fi = w1 ? 0.f : fin[(long long)i * N + s];
        const float fs = post_collision<float>(i, fi, w1, S.omega, S.om1, na, ja, u, Na);
        const int yy = q.y + kC[i][1];
        if (S.walls && (yy == 0 || yy == S.ny - 1)) {
            const float uw = (yy == 0) ? S.wall_ux[0] : S.wall_ux[1];
            fout[(long long)opposite(i) * N + s] = fs - ((6.f * lattice_weight<float>(i)) * na) * ((float)kC[i][0] * uw);
        } else {
            fout[(long long)i * N + nbr(S, r, kC[i][0], kC[i][1], kC[i][2])] = fs;
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
    for (int c = 0; c < S.M; ++c) stage1(t, sl, RowOff, Ln + c * t.FS, S.n + (long long)c * N);
    __syncthreads();
    if (!q.active) return;
    const long long s = q.s;
    if (S.walls && (q.y == 0 || q.y == S.ny - 1)) {
        for (int p = 0; p < S.P; ++p) S.g[(long long)p * N + s] = 0.f;
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
            S.g[(long long)pidx(S.M, a, b) * N + s] = qf * ((1.f + z) * (1.f + 2.f * z));
        }
}

inline size_t contact_lds_bytes(int TX, int TY, int TZ, int R, int ball_total, int maxM)
{
    const size_t FS = (size_t)(TX + 2 * R) * (TY + 2 * R) * (TZ + 2 * R);
    const size_t rows = (size_t)(TY + 2 * R) * (TZ + 2 * R);
    return 4 * ((size_t)maxM * FS + (size_t)ball_total + rows);
}

// float4 + float per staged site, the shell table (16 bytes per entry),
// then the row-offset table (one int per halo row)
inline size_t tile_lds_bytes(int TX, int TY, int TZ, int R, int sh_max)
{
    const size_t FS = (size_t)(TX + 2 * R) * (TY + 2 * R) * (TZ + 2 * R);
    const size_t rows = (size_t)(TY + 2 * R) * (TZ + 2 * R);
    return 16 * FS + 16 * ((FS + 3) / 4) + 16 * (size_t)sh_max + 4 * rows;
}

}  // namespace mlb
