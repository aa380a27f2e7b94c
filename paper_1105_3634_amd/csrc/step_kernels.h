// Per-site passes of one lattice step (templated on the float type).
//
// One step  t -> t+1  of the kinetic equation of Sec. 2, eq. (evolution):
//   moments    n_a, j_a, barycentric u                         eq. (colonna)
//   contact    ball-smoothed packing fractions -> BMCSL g_ab   (Sec. 2: g at
//              contact depends on the densities through a smoothing)
//   gather1    hard-core mean field (eq. potmeanforce), attractive RPA field,
//              external force, dissipative pair form at the old velocities
//              (eqs. gammaab, tensorgamma, viscousforce), friction rate,
//              velocity predictor V and predictor-time force H
//   step2      dissipative pair form at V, total force N = n_a Phi_a,
//              orthogonalised BGK collision (eq. prefactor) with the field
//              term, push streaming, halfway bounce-back at moving walls
//
// Every arithmetic expression is written in one fixed order (velocities in
// canonical order, stencil half-lists with each +e/-e pair combined first,
// species ascending).  The float64 build compiles these kernels without
// contraction, which makes the float64 results independent of the launch
// shape and reproducible bit for bit.
#pragma once

#include "mlb_internal.h"

namespace mlb {

__device__ constexpr int kC[kQ][3] = {
    {0, 0, 0},
    {1, 0, 0}, {-1, 0, 0}, {0, 1, 0}, {0, -1, 0}, {0, 0, 1}, {0, 0, -1},
    {1, 1, 0}, {-1, -1, 0}, {1, -1, 0}, {-1, 1, 0},
    {1, 0, 1}, {-1, 0, -1}, {1, 0, -1}, {-1, 0, 1},
    {0, 1, 1}, {0, -1, -1}, {0, 1, -1}, {0, -1, 1}};

template <typename T>
__device__ inline T lattice_weight(int i)
{
    return i == 0 ? T(1.0) / T(3.0) : (i <= 6 ? T(1.0) / T(18.0) : T(1.0) / T(36.0));
}

__device__ constexpr int opposite(int i) { return i == 0 ? 0 : ((i & 1) ? i + 1 : i - 1); }

struct Site {
    int x, y, z;
};

template <typename T>
__device__ inline Site site_of(const SysDesc<T> &S, long long s)
{
    Site r;
    r.x = (int)(s % S.nx);
    long long q = s / S.nx;
    r.y = (int)(q % S.ny);
    r.z = (int)(q / S.ny);
    return r;
}

template <typename T>
__device__ inline bool is_solid(const SysDesc<T> &S, int y)
{
    return S.walls && (y == 0 || y == S.ny - 1);
}

// Index of r + e, or -1 outside a walled box.  Offsets are smaller than the
// box edge in every periodic direction (checked on the host).
template <typename T>
__device__ inline long long nbr(const SysDesc<T> &S, const Site &r, int ex, int ey, int ez)
{
    int xx = r.x + ex;
    xx = xx < 0 ? xx + S.nx : (xx >= S.nx ? xx - S.nx : xx);
    int zz = r.z + ez;
    zz = zz < 0 ? zz + S.nz : (zz >= S.nz ? zz - S.nz : zz);
    int yy = r.y + ey;
    if (S.walls) {
        if (yy < 0 || yy >= S.ny) return -1;
    } else {
        yy = yy < 0 ? yy + S.ny : (yy >= S.ny ? yy - S.ny : yy);
    }
    return ((long long)zz * S.ny + yy) * S.nx + xx;
}

template <typename T>
__device__ inline T ld(const T *__restrict__ F, long long s)
{
    return s < 0 ? T(0) : F[s];
}

// r + e as the hard-core stencils (smoothing balls, mean-field and friction
// shells) see it: the site itself in a periodic box and inside the fluid
// rows; beyond a wall (y + e_y <= 0 or >= ny - 1) the mirror image of the
// fluid across the nearer wall plane (y = 1/2 or y = ny - 3/2, where halfway
// bounce-back puts the walls), which carries that fluid site's density and
// contact value and moves with the wall.  img: 0 fluid, 1 image beyond the
// y = 0 wall, 2 beyond the y = ny - 1 wall.  The host checks that the shell
// reach stays inside the fluid rows, so one reflection suffices.
template <typename T>
__device__ inline long long hc_nbr(const SysDesc<T> &S, const Site &r, int ex, int ey, int ez, int &img)
{
    int xx = r.x + ex;
    xx = xx < 0 ? xx + S.nx : (xx >= S.nx ? xx - S.nx : xx);
    int zz = r.z + ez;
    zz = zz < 0 ? zz + S.nz : (zz >= S.nz ? zz - S.nz : zz);
    int yy = r.y + ey;
    img = 0;
    if (S.walls) {
        if (yy <= 0) {
            yy = 1 - yy;
            img = 1;
        } else if (yy >= S.ny - 1) {
            yy = 2 * S.ny - 3 - yy;
            img = 2;
        }
    } else {
        yy = yy < 0 ? yy + S.ny : (yy >= S.ny ? yy - S.ny : yy);
    }
    return ((long long)zz * S.ny + yy) * S.nx + xx;
}

__device__ inline int pidx(int M, int a, int b)
{
    const int lo = a < b ? a : b, hi = a < b ? b : a;
    return lo * M - (lo * (lo - 1)) / 2 + (hi - lo);
}

// ------------------------------------------------------------------ moments
template <typename T>
__global__ void __launch_bounds__(kBlock) k_moments(const SysDesc<T> *__restrict__ sys,
                                                    const int2 *__restrict__ bmap, int parity)
{
    const int2 bm = bmap[blockIdx.x];
    if (bm.x < 0) return;
    const SysDesc<T> &S = sys[bm.x];
    const long long s = (long long)bm.y * kBlock + threadIdx.x;
    if (s >= S.N) return;
    const long long N = S.N;
    const T *__restrict__ f = S.f[parity];
    T nt = T(0), jt[3] = {T(0), T(0), T(0)};
    for (int a = 0; a < S.M; ++a) {
        T fi[kQ];
#pragma unroll
        for (int i = 0; i < kQ; ++i) fi[i] = f[((long long)a * kQ + i) * N + s];
        T na = fi[0];
#pragma unroll
        for (int i = 1; i < kQ; ++i) na = na + fi[i];
        T ja[3];
#pragma unroll
        for (int d = 0; d < 3; ++d) {
            T acc = T(0);
#pragma unroll
            for (int i = 1; i < kQ; ++i) {
                if (kC[i][d] == 1) acc = acc + fi[i];
                else if (kC[i][d] == -1) acc = acc - fi[i];
            }
            ja[d] = acc;
        }
        S.n[(long long)a * N + s] = na;
#pragma unroll
        for (int d = 0; d < 3; ++d) S.j[((long long)a * 3 + d) * N + s] = ja[d];
        // barycentric velocity: mass-weighted (Sec. 2, eq. massdensity and below)
        const T ma = S.mass[a];
        if (a == 0) {
            nt = ma * na;
            jt[0] = ma * ja[0]; jt[1] = ma * ja[1]; jt[2] = ma * ja[2];
        } else {
            nt = nt + ma * na;
            jt[0] = jt[0] + ma * ja[0]; jt[1] = jt[1] + ma * ja[1]; jt[2] = jt[2] + ma * ja[2];
        }
    }
#pragma unroll
    for (int d = 0; d < 3; ++d) S.u[(long long)d * N + s] = (nt != T(0)) ? jt[d] / nt : T(0);
}

// ------------------------------------------------- contact values (BMCSL)
//   g_ab = 1/(1-xi3) + 3 d xi2/(1-xi3)^2 + 2 d^2 xi2^2/(1-xi3)^3 = q (1+z)(1+2z)
//   q = 1/(1-xi3), z = d xi2 q, xi_k = (pi/6) sum_c sigma_c^k nbar_c.
template <typename T>
__global__ void __launch_bounds__(kBlock) k_contact(const SysDesc<T> *__restrict__ sys,
                                                    const int2 *__restrict__ bmap, Tables<T> tb)
{
    const int2 bm = bmap[blockIdx.x];
    if (bm.x < 0) return;
    const SysDesc<T> &S = sys[bm.x];
    const long long s = (long long)bm.y * kBlock + threadIdx.x;
    if (s >= S.N) return;
    const long long N = S.N;
    const Site r = site_of(S, s);
    if (is_solid(S, r.y)) {
        for (int p = 0; p < S.P; ++p) S.g[(long long)p * N + s] = T(0);
        return;
    }
    T nb[kMaxS];
    for (int c = 0; c < S.M; ++c) {
        const T *__restrict__ nc = S.n + (long long)c * N;
        T acc = nc[s];
        const int b0 = S.bl_start[c], bn = S.bl_cnt[c];
        for (int k = 0; k < bn; ++k) {
            int ex, ey, ez;
            unpack_offset(tb.bl_e[b0 + k], ex, ey, ez);
            int ip, im;
            const long long sp = hc_nbr(S, r, ex, ey, ez, ip), sm = hc_nbr(S, r, -ex, -ey, -ez, im);
            acc = acc + (nc[sp] + nc[sm]);
        }
        nb[c] = acc / (T)S.bl_full[c];
    }
    T x2 = S.s2[0] * nb[0], x3 = S.s3[0] * nb[0];
    for (int c = 1; c < S.M; ++c) {
        x2 = x2 + S.s2[c] * nb[c];
        x3 = x3 + S.s3[c] * nb[c];
    }
    const T q = T(1) / (T(1) - x3);
    for (int a = 0; a < S.M; ++a)
        for (int b = a; b < S.M; ++b) {
            const T z = (S.dd[a][b] * x2) * q;
            S.g[(long long)pidx(S.M, a, b) * N + s] = q * ((T(1) + z) * (T(1) + T(2) * z));
        }
}

// ----------------------------------------------------------------- gather 1
// Thread = (site, species a).  For each partner b over the half-shell S_ab:
//   G+- = g_ab(r) + g_ab(r+-e),  t+- = G+- n_b(r+-e)
//   mean field  sum e_hat (t+ - t-)
//   friction    sum (t+ + t-)
//   pair form   sum e_hat (G+ e_hat.X+ + G- e_hat.X-),  X = n_a(r) j_b(r') - n_b(r') j_a(r)
// then scaled by the pair constants; the attractive tail (direct mode) sums
// w(e) (n_b(r+e) - n_b(r-e)) over its half-list.
template <typename T>
__global__ void __launch_bounds__(kBlock) k_gather1(const SysDesc<T> *__restrict__ sys,
                                                    const int2 *__restrict__ bmap, Tables<T> tb)
{
    const int2 bm = bmap[blockIdx.x];
    if (bm.x < 0) return;
    const SysDesc<T> &S = sys[bm.x];
    const int a = blockIdx.y;
    if (a >= S.M) return;
    const long long s = (long long)bm.y * kBlock + threadIdx.x;
    if (s >= S.N) return;
    const long long N = S.N;
    const Site r = site_of(S, s);
    const long long o3 = (long long)a * 3 * N;
    if (is_solid(S, r.y)) {
        for (int d = 0; d < 3; ++d) {
            S.vh[o3 + d * N + s] = T(0);
            S.H[o3 + d * N + s] = T(0);
            if (S.parts) S.parts[o3 + d * N + s] = T(0);
        }
        return;
    }
    const T na = S.n[(long long)a * N + s];
    const T ja[3] = {S.j[o3 + s], S.j[o3 + N + s], S.j[o3 + 2 * N + s]};
    T mf[3] = {T(0), T(0), T(0)}, tl[3] = {T(0), T(0), T(0)}, dv[3] = {T(0), T(0), T(0)};
    T gam = T(0);
    for (int b = 0; b < S.M; ++b) {
        const T *__restrict__ nb = S.n + (long long)b * N;
        const T *__restrict__ jb = S.j + (long long)b * 3 * N;
        const T *__restrict__ gp = S.g + (long long)pidx(S.M, a, b) * N;
        const T g0 = gp[s];
        T smf[3] = {T(0), T(0), T(0)}, sdv[3] = {T(0), T(0), T(0)}, sg = T(0);
        const int k0 = S.sh_start[a][b], kn = S.sh_cnt[a][b];
        for (int k = 0; k < kn; ++k) {
            int ex, ey, ez;
            unpack_offset(tb.sh_e[k0 + k], ex, ey, ez);
            const T e0 = tb.sh_u[3 * (k0 + k) + 0], e1 = tb.sh_u[3 * (k0 + k) + 1],
                    e2 = tb.sh_u[3 * (k0 + k) + 2];
            int ip, im;
            const long long sp = hc_nbr(S, r, ex, ey, ez, ip), sm = hc_nbr(S, r, -ex, -ey, -ez, im);
            const T Gp = g0 + gp[sp], Gm = g0 + gp[sm];
            const T np_ = nb[sp], nm_ = nb[sm];
            const T tp = Gp * np_, tm = Gm * nm_;
            const T dt = tp - tm;
            smf[0] = smf[0] + e0 * dt;
            smf[1] = smf[1] + e1 * dt;
            smf[2] = smf[2] + e2 * dt;
            sg = sg + (tp + tm);
            // an image's momentum density: its density times the wall's velocity
            const T jp0 = ip ? np_ * S.wall_ux[ip - 1] : jb[sp];
            const T jp1 = ip ? np_ * T(0) : jb[N + sp];
            const T jp2 = ip ? np_ * T(0) : jb[2 * N + sp];
            const T jm0 = im ? nm_ * S.wall_ux[im - 1] : jb[sm];
            const T jm1 = im ? nm_ * T(0) : jb[N + sm];
            const T jm2 = im ? nm_ * T(0) : jb[2 * N + sm];
            const T Xp0 = na * jp0 - np_ * ja[0];
            const T Xp1 = na * jp1 - np_ * ja[1];
            const T Xp2 = na * jp2 - np_ * ja[2];
            const T Xm0 = na * jm0 - nm_ * ja[0];
            const T Xm1 = na * jm1 - nm_ * ja[1];
            const T Xm2 = na * jm2 - nm_ * ja[2];
            const T pp = Gp * ((e0 * Xp0 + e1 * Xp1) + e2 * Xp2);
            const T pm = Gm * ((e0 * Xm0 + e1 * Xm1) + e2 * Xm2);
            const T pq = pp + pm;
            sdv[0] = sdv[0] + e0 * pq;
            sdv[1] = sdv[1] + e1 * pq;
            sdv[2] = sdv[2] + e2 * pq;
        }
        const T cm = S.cm[a][b], ck = S.ck[a][b];
        mf[0] = mf[0] + cm * smf[0]; mf[1] = mf[1] + cm * smf[1]; mf[2] = mf[2] + cm * smf[2];
        dv[0] = dv[0] + ck * sdv[0]; dv[1] = dv[1] + ck * sdv[1]; dv[2] = dv[2] + ck * sdv[2];
        gam = gam + S.cg[a][b] * sg;
        if (S.tail_direct && S.tl_cnt[a][b] > 0) {
            T st[3] = {T(0), T(0), T(0)};
            const int t0 = S.tl_start[a][b], tn = S.tl_cnt[a][b];
            for (int k = 0; k < tn; ++k) {
                int ex, ey, ez;
                unpack_offset(tb.tl_e[t0 + k], ex, ey, ez);
                const long long sp = nbr(S, r, ex, ey, ez), sm = nbr(S, r, -ex, -ey, -ez);
                const T dn = ld(nb, sp) - ld(nb, sm);
                st[0] = st[0] + tb.tl_w[3 * (t0 + k) + 0] * dn;
                st[1] = st[1] + tb.tl_w[3 * (t0 + k) + 1] * dn;
                st[2] = st[2] + tb.tl_w[3 * (t0 + k) + 2] * dn;
            }
            tl[0] = tl[0] + st[0]; tl[1] = tl[1] + st[1]; tl[2] = tl[2] + st[2];
        }
    }
    if (!S.tail_direct && S.tail) {
        // spectral mode: sum_b (K_ab * n_b) precomputed for this species
        tl[0] = S.tail[o3 + s]; tl[1] = S.tail[o3 + N + s]; tl[2] = S.tail[o3 + 2 * N + s];
    }
    // a force density changes the number flux at the rate 1/m_a
    const T im = S.im[a];
    const T hg = (T(0.5) * gam) * im;
#pragma unroll
    for (int d = 0; d < 3; ++d) {
        const T Nmf = na * mf[d];
        const T Ntl = na * tl[d];
        const T fe = S.fprof ? S.fprof[((long long)a * 3 + d) * S.ny + r.y] : S.fext[a][d];
        const T Nex = na * fe;
        const T Nc = (Nmf + Ntl) + Nex;
        const T Dd = dv[d];
        if (S.scheme == 1) {
            S.H[o3 + d * N + s] = Nc + Dd;
            S.vh[o3 + d * N + s] = T(0);
        } else {
            S.H[o3 + d * N + s] = Nc + T(0.5) * Dd;
            S.vh[o3 + d * N + s] =
                (na != T(0)) ? (((ja[d] + im * Nc) + im * Dd) + hg * ja[d]) / (na * (T(1) + hg)) : T(0);
        }
        if (S.parts) {
            T acc = T(0);
            if (S.parts_mask & 1u) acc = acc + Nmf;
            if (S.parts_mask & 2u) acc = acc + Ntl;
            if (S.parts_mask & 8u) acc = acc + Nex;
            if (S.parts_mask & 4u) acc = acc + (S.scheme == 1 ? Dd : T(0.5) * Dd);
            S.parts[o3 + d * N + s] = acc;
        }
    }
}

// ------------------------------------------------------------------ step 2
// Orthogonalised BGK collision with the field term (eq. evolution), the
// Maxwellian of eq. (psia) with thermal speed^2 theta_a = kT/m_a in
// second-order Hermite form on the lattice (c_s^2 = 1/3):
//   E_i = 1 + 3 c.u + 9/2 (c.u)^2 - 3/2 u.u + (9/2)(theta_a - 1/3)(c.c - 1)
//   psi_perp_i = w_i E_i [n_a + (m_a/kT) (j_a - n_a u).(c_i - u)]     eq. (prefactor)
//   S_i = w_i E_i (c_i - u).N_a / kT
//   f*_i = (1 - omega) f_i + omega psi_perp_i + S_i
// ith = m_a/kT, dth = (9/2)(theta_a - 1/3) (0 for unit masses: no term).
template <typename T>
__device__ inline T post_collision(int i, T fi, bool omega_one, T omega, T om1, T na, const T ja[3],
                                   const T u[3], const T Na[3], T ith, T dth)
{
    const T uu = (u[0] * u[0] + u[1] * u[1]) + u[2] * u[2];
    const T cx = (T)kC[i][0], cy = (T)kC[i][1], cz = (T)kC[i][2];
    const T cu = (cx * u[0] + cy * u[1]) + cz * u[2];
    T E = ((T(1) + T(3) * cu) + (T(4.5) * cu) * cu) - T(1.5) * uu;
    if (dth != T(0)) {
        const int c2 = kC[i][0] * kC[i][0] + kC[i][1] * kC[i][1] + kC[i][2] * kC[i][2];
        E = E + dth * (T)(c2 - 1);
    }
    const T wE = lattice_weight<T>(i) * E;
    const T m0 = cx - u[0], m1 = cy - u[1], m2 = cz - u[2];
    const T v0 = ja[0] - na * u[0], v1 = ja[1] - na * u[1], v2 = ja[2] - na * u[2];
    const T dotv = (v0 * m0 + v1 * m1) + v2 * m2;
    const T dotN = (m0 * Na[0] + m1 * Na[1]) + m2 * Na[2];
    const T psi = wE * (na + ith * dotv);
    const T src = wE * (T(3) * dotN);   // 3 = 1/kT
    if (omega_one) return psi + src;
    return (om1 * fi + omega * psi) + src;
}

// Thread = (site, species a): second gather (pair form at the predicted
// velocities), total force, collision and push streaming.  With
// write_force_only the force is stored and no population is touched.
template <typename T>
__global__ void __launch_bounds__(kBlock) k_step2(const SysDesc<T> *__restrict__ sys,
                                                  const int2 *__restrict__ bmap, Tables<T> tb,
                                                  int parity, int write_force_only)
{
    const int2 bm = bmap[blockIdx.x];
    if (bm.x < 0) return;
    const SysDesc<T> &S = sys[bm.x];
    const int a = blockIdx.y;
    if (a >= S.M) return;
    const long long s = (long long)bm.y * kBlock + threadIdx.x;
    if (s >= S.N) return;
    const long long N = S.N;
    const Site r = site_of(S, s);
    const long long o3 = (long long)a * 3 * N;
    if (is_solid(S, r.y)) {
        if (write_force_only)
            for (int d = 0; d < 3; ++d) S.Nf[o3 + d * N + s] = T(0);
        return;
    }
    const T na = S.n[(long long)a * N + s];
    T Na[3];
    if (S.scheme == 1) {
        Na[0] = S.H[o3 + s]; Na[1] = S.H[o3 + N + s]; Na[2] = S.H[o3 + 2 * N + s];
    } else {
        const T va[3] = {S.vh[o3 + s], S.vh[o3 + N + s], S.vh[o3 + 2 * N + s]};
        T dv[3] = {T(0), T(0), T(0)};
        for (int b = 0; b < S.M; ++b) {
            const T *__restrict__ nb = S.n + (long long)b * N;
            const T *__restrict__ vb = S.vh + (long long)b * 3 * N;
            const T *__restrict__ gp = S.g + (long long)pidx(S.M, a, b) * N;
            const T g0 = gp[s];
            T sdv[3] = {T(0), T(0), T(0)};
            const int k0 = S.sh_start[a][b], kn = S.sh_cnt[a][b];
            for (int k = 0; k < kn; ++k) {
                int ex, ey, ez;
                unpack_offset(tb.sh_e[k0 + k], ex, ey, ez);
                const T e0 = tb.sh_u[3 * (k0 + k) + 0], e1 = tb.sh_u[3 * (k0 + k) + 1],
                        e2 = tb.sh_u[3 * (k0 + k) + 2];
                int ip, im;
                const long long sp = hc_nbr(S, r, ex, ey, ez, ip), sm = hc_nbr(S, r, -ex, -ey, -ez, im);
                const T tp = (g0 + gp[sp]) * nb[sp];
                const T tm = (g0 + gp[sm]) * nb[sm];
                // an image moves with the wall: (u_wall, 0, 0)
                const T Yp0 = (ip ? S.wall_ux[ip - 1] : vb[sp]) - va[0];
                const T Yp1 = (ip ? T(0) : vb[N + sp]) - va[1];
                const T Yp2 = (ip ? T(0) : vb[2 * N + sp]) - va[2];
                const T Ym0 = (im ? S.wall_ux[im - 1] : vb[sm]) - va[0];
                const T Ym1 = (im ? T(0) : vb[N + sm]) - va[1];
                const T Ym2 = (im ? T(0) : vb[2 * N + sm]) - va[2];
                const T pp = tp * ((e0 * Yp0 + e1 * Yp1) + e2 * Yp2);
                const T pm = tm * ((e0 * Ym0 + e1 * Ym1) + e2 * Ym2);
                const T pq = pp + pm;
                sdv[0] = sdv[0] + e0 * pq;
                sdv[1] = sdv[1] + e1 * pq;
                sdv[2] = sdv[2] + e2 * pq;
            }
            const T ck = S.ck[a][b];
            dv[0] = dv[0] + ck * sdv[0]; dv[1] = dv[1] + ck * sdv[1]; dv[2] = dv[2] + ck * sdv[2];
        }
#pragma unroll
        for (int d = 0; d < 3; ++d) {
            const T Dn = na * dv[d];
            Na[d] = S.H[o3 + d * N + s] + T(0.5) * Dn;
            if (S.parts && (S.parts_mask & 4u)) S.parts[o3 + d * N + s] = S.parts[o3 + d * N + s] + T(0.5) * Dn;
        }
    }
    if (write_force_only) {
        for (int d = 0; d < 3; ++d) S.Nf[o3 + d * N + s] = Na[d];
        return;
    }
    const T ja[3] = {S.j[o3 + s], S.j[o3 + N + s], S.j[o3 + 2 * N + s]};
    const T u[3] = {S.u[s], S.u[N + s], S.u[2 * N + s]};
    const T *__restrict__ fin = S.f[parity] + (long long)a * kQ * N;
    T *__restrict__ fout = S.f[parity ^ 1] + (long long)a * kQ * N;
    const bool w1 = S.omega_is_one != 0;
#pragma unroll
    for (int i = 0; i < kQ; ++i) {
        const T fi = w1 ? T(0) : fin[(long long)i * N + s];
        const T fs = post_collision<T>(i, fi, w1, S.omega, S.om1, na, ja, u, Na, S.ith[a], S.dth[a]);
        const int yy = r.y + kC[i][1];
        if (S.walls && (yy == 0 || yy == S.ny - 1)) {
            const T uw = (yy == 0) ? S.wall_ux[0] : S.wall_ux[1];
            const T cux = (T)kC[i][0] * uw;
            fout[(long long)opposite(i) * N + s] = fs - ((T(6) * lattice_weight<T>(i)) * na) * cux;
        } else {
            fout[(long long)i * N + nbr(S, r, kC[i][0], kC[i][1], kC[i][2])] = fs;
        }
    }
}

// The attractive field computed beside the first gather (tiled float32
// path): its contribution N_tail = n_a C_a enters the predictor-time force
// H and, through N^c, the predictor V-hat = (... + N^c / m_a ...) / (n_a (1 + Gamma_a / (2 m_a))).
template <typename T>
__global__ void __launch_bounds__(kBlock) k_add_tail(const SysDesc<T> *__restrict__ sys,
                                                     const int2 *__restrict__ bmap)
{
    const int2 bm = bmap[blockIdx.x];
    if (bm.x < 0) return;
    const SysDesc<T> &S = sys[bm.x];
    const int a = blockIdx.y;
    if (a >= S.M || !S.tail_deferred) return;
    const long long s = (long long)bm.y * kBlock + threadIdx.x;
    if (s >= S.N) return;
    const long long N = S.N;
    const Site r = site_of(S, s);
    if (is_solid(S, r.y)) return;
    const long long o3 = (long long)a * 3 * N;
    const T na = S.n[(long long)a * N + s], gf = S.gfac[(long long)a * N + s];
    // all loads first: the stores could alias them as far as the compiler
    // knows, which would serialise the three components
    const bool fe = S.scheme == 1, pt = S.parts && (S.parts_mask & 2u);
    T c[3], h[3], v[3], pp[3];
#pragma unroll
    for (int d = 0; d < 3; ++d) {
        c[d] = S.tail[o3 + d * N + s];
        h[d] = S.H[o3 + d * N + s];
        v[d] = fe ? T(0) : S.vh[o3 + d * N + s];
        pp[d] = pt ? S.parts[o3 + d * N + s] : T(0);
    }
#pragma unroll
    for (int d = 0; d < 3; ++d) {
        const T ntl = na * c[d];
        S.H[o3 + d * N + s] = h[d] + ntl;
        if (!fe) S.vh[o3 + d * N + s] = v[d] + c[d] * gf;
        if (pt) S.parts[o3 + d * N + s] = pp[d] + ntl;
    }
}

// ------------------------------------------------------- initial populations
// f = psi_perp(n0, n0 u0, u) at fluid sites (float64 inputs), zero on walls.
template <typename T>
__global__ void __launch_bounds__(kBlock) k_init_pop(const SysDesc<T> *__restrict__ sys,
                                                     const int2 *__restrict__ bmap,
                                                     const double *__restrict__ n0,
                                                     const double *__restrict__ u0)
{
    const int2 bm = bmap[blockIdx.x];
    if (bm.x < 0) return;
    const SysDesc<T> &S = sys[bm.x];
    const long long s = (long long)bm.y * kBlock + threadIdx.x;
    if (s >= S.N) return;
    const long long N = S.N;
    const Site r = site_of(S, s);
    T *__restrict__ f = S.f[0];
    if (is_solid(S, r.y)) {
        for (int a = 0; a < S.M; ++a)
            for (int i = 0; i < kQ; ++i) {
                f[((long long)a * kQ + i) * N + s] = T(0);
                S.f[1][((long long)a * kQ + i) * N + s] = T(0);
            }
        return;
    }
    T nt = T(0), jt[3] = {T(0), T(0), T(0)};
    T jj[kMaxS][3];
    for (int a = 0; a < S.M; ++a) {
        const T na = (T)n0[(long long)a * N + s];
        const T ma = S.mass[a];
        for (int d = 0; d < 3; ++d) jj[a][d] = na * (T)u0[((long long)a * 3 + d) * N + s];
        if (a == 0) {
            nt = ma * na; jt[0] = ma * jj[a][0]; jt[1] = ma * jj[a][1]; jt[2] = ma * jj[a][2];
        } else {
            nt = nt + ma * na;
            jt[0] = jt[0] + ma * jj[a][0]; jt[1] = jt[1] + ma * jj[a][1]; jt[2] = jt[2] + ma * jj[a][2];
        }
    }
    T u[3];
    for (int d = 0; d < 3; ++d) u[d] = (nt != T(0)) ? jt[d] / nt : T(0);
    const T zero3[3] = {T(0), T(0), T(0)};
    for (int a = 0; a < S.M; ++a) {
        const T na = (T)n0[(long long)a * N + s];
#pragma unroll
        for (int i = 0; i < kQ; ++i)
            f[((long long)a * kQ + i) * N + s] =
                post_collision<T>(i, T(0), true, T(1), T(0), na, jj[a], u, zero3, S.ith[a], S.dth[a]);
    }
}

// ----------------------------------------------------------------- launches
template <typename T>
void Launch<T>::moments(const SysDesc<T> *sys, const int2 *map, int nblk, int parity, hipStream_t st)
{
    hipLaunchKernelGGL(k_moments<T>, dim3(nblk), dim3(kBlock), 0, st, sys, map, parity);
}
template <typename T>
void Launch<T>::contact(const SysDesc<T> *sys, const int2 *map, int nblk, Tables<T> tb, hipStream_t st)
{
    hipLaunchKernelGGL(k_contact<T>, dim3(nblk), dim3(kBlock), 0, st, sys, map, tb);
}
template <typename T>
void Launch<T>::gather1(const SysDesc<T> *sys, const int2 *map, int nblk, int maxM, Tables<T> tb,
                        hipStream_t st)
{
    hipLaunchKernelGGL(k_gather1<T>, dim3(nblk, maxM), dim3(kBlock), 0, st, sys, map, tb);
}
template <typename T>
void Launch<T>::step2(const SysDesc<T> *sys, const int2 *map, int nblk, int maxM, Tables<T> tb,
                      int parity, int write_force_only, hipStream_t st)
{
    hipLaunchKernelGGL(k_step2<T>, dim3(nblk, maxM), dim3(kBlock), 0, st, sys, map, tb, parity,
                       write_force_only);
}
template <typename T>
void Launch<T>::add_tail(const SysDesc<T> *sys, const int2 *map, int nblk, int maxM, hipStream_t st)
{
    hipLaunchKernelGGL(k_add_tail<T>, dim3(nblk, maxM), dim3(kBlock), 0, st, sys, map);
}
template <typename T>
void Launch<T>::init_pop(const SysDesc<T> *sys, const int2 *map, int nblk, const double *n0,
                         const double *u0, hipStream_t st)
{
    hipLaunchKernelGGL(k_init_pop<T>, dim3(nblk), dim3(kBlock), 0, st, sys, map, n0, u0);
}

}  // namespace mlb
