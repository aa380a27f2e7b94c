// Float32 collision and push streaming with a given force, for the steps a
// closure network drives.  The collision of eq. (evolution) with the force
// term, regrouped as in the tiled second gather's epilogue so that only the
// parts that depend on c_i stay inside the population loop:
//   f*_i = w_i E_i (A + 3 c_i.P) [+ (1 - omega) f_i],
//   E_i = (1 - 3/2 u.u) + c_i.u (3 + 9/2 c_i.u) [+ dth (c_i.c_i - 1)],
//   P = omega m_a (j - n u) + N,  A = omega n - 3 u.P
// (kT = 1/3, so m_a / kT = 3 m_a; dth = (9/2)(kT/m_a - 1/3)).  Beyond a
// wall the population bounces back with the wall's momentum.
#include "collide_f32.h"
#include "gather_tile.h"

namespace mlb {
namespace {

__global__ void __launch_bounds__(kBlock) k_collide_f32(const SysDesc<float> *__restrict__ sys,
                                                        const int2 *__restrict__ bmap, int parity)
{
    const int2 bm = bmap[blockIdx.x];
    if (bm.x < 0) return;
    const SysDesc<float> &S = sys[bm.x];
    const int a = blockIdx.y;
    if (a >= S.M) return;
    const long long s = (long long)bm.y * kBlock + threadIdx.x;
    if (s >= S.N) return;
    const long long N = S.N;
    const Site r = site_of(S, s);
    if (is_solid(S, r.y)) return;
    const long long o3 = (long long)a * 3 * N;
    const float na = glb(S.n)[(long long)a * N + s];
    const bool w1 = S.omega_is_one != 0;
    const float om = w1 ? 1.f : S.omega;
    const float omm = om * S.mass[a], dth = S.dth[a];
    float u[3], P[3];
#pragma unroll
    for (int d = 0; d < 3; ++d) {
        u[d] = glb(S.u)[d * N + s];
        P[d] = omm * (glb(S.j)[o3 + d * N + s] - na * u[d]) + glb(S.Nf)[o3 + d * N + s];
    }
    const float uu = (u[0] * u[0] + u[1] * u[1]) + u[2] * u[2];
    const float B = 1.f - 1.5f * uu;
    const float A = om * na - 3.f * ((u[0] * P[0] + u[1] * P[1]) + u[2] * P[2]);
    // neighbour offsets with periodic wrap (32-bit: sites number below 2^29)
    const int nx = S.nx, nxy = S.nx * S.ny, s32 = (int)s, nall = (int)N;
    const int ox[2] = {r.x == 0 ? nx - 1 : -1, r.x == nx - 1 ? 1 - nx : 1};
    const int oy[2] = {r.y == 0 ? nxy - nx : -nx, r.y == S.ny - 1 ? nx - nxy : nx};
    const int oz[2] = {r.z == 0 ? nall - nxy : -nxy, r.z == S.nz - 1 ? nxy - nall : nxy};
    const bool wlo = S.walls && r.y == 1, whi = S.walls && r.y == S.ny - 2;
    const gfloat *__restrict__ fin = glb(S.f[parity]) + (long long)a * kQ * N;
    gfloat *__restrict__ fout = glb(S.f[parity ^ 1]) + (long long)a * kQ * N;
#pragma unroll
    for (int i = 0; i < kQ; ++i) {
        const int cx = kC[i][0], cy = kC[i][1], cz = kC[i][2];
        const float cu = cdot(cx, cy, cz, u), cP = cdot(cx, cy, cz, P);
        float E = B + cu * (3.f + 4.5f * cu);
        if (!S.unit_mass) E += dth * (float)(cx * cx + cy * cy + cz * cz - 1);
        float fs = (lattice_weight<float>(i) * E) * (A + 3.f * cP);
        if (!w1) fs += S.om1 * fin[(long long)i * N + s];
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

}  // namespace

void launch_collide_f32(const SysDesc<float> *sys, const int2 *map, int nblk, int maxM, int parity, hipStream_t st)
{
    hipLaunchKernelGGL(k_collide_f32, dim3(nblk, maxM), dim3(kBlock), 0, st, sys, map, parity);
}

}  // namespace mlb
