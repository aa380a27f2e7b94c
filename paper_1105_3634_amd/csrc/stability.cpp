// Linear stability of the lattice step at a uniform state (host only).
//
// Around uniform species densities n_a at rest, a perturbation of the
// populations proportional to exp(i k.r) is mapped by one step onto the
// same wavevector, so the step is a (19 M)-dimensional complex linear map
// per k.  Its pieces, linearised:
//   contact values  dg_ab = sum_c (dg_ab/dn_c) B_c(k) dn_c, B_c the ball
//                   average of cos(k.e), dg/dn of the BMCSL form
//   mean field      -kT n_a sum_b s_ab^2 w_hat i SV_ab (g_ab dn_b + n_b dg_ab / 2),
//                   SV = sum_e e_hat sin(k.e) over the shell (eq. potmeanforce,
//                   pair value (g(r) + g(r+e)) / 2)
//   attractive      n_a sum_b i TV_ab dn_b, TV = sum_e w(e) sin(k.e)
//   pair form       D_a[V] = sum_b kappa_ab g_ab (n_a ST_ab V_b n_b - n_b ST0_ab n_a V_a)
//                   (eqs. gammaab, tensorgamma, viscousforce), ST = sum e e^T cos(k.e)
//   time scheme     forward Euler, or Crank-Nicolson with one Jacobi
//                   predictor as the step applies it (forces over m_a)
//   collision       f* = (1 - omega) f + omega psi + 3 w h c.N, with
//                   psi = w h (dn + (m_a/kT) c.(dj - n du)) + 3 w n c.du,
//                   h = 1 + (9/2)(kT/m_a - 1/3)(c.c - 1), du the mass-weighted
//                   barycentric velocity (unit masses: psi = w (dn + 3 c.dj))
//   streaming       f' = exp(-i k.c) f*
// The spectral radius over a grid of k (k = 0 excluded: its conserved
// modes sit at 1) comes from power iteration.  The forward-Euler treatment
// of the friction is unstable once the friction rate per step is of order
// one, which is what the guard reports.
#include <cmath>
#include <complex>
#include <random>
#include <vector>

#include "../../include/mlb.h"
#include "mlb_internal.h"

namespace mlb {
namespace {

using cd = std::complex<double>;

constexpr int kCx[kQ][3] = {{0, 0, 0},  {1, 0, 0},  {-1, 0, 0}, {0, 1, 0},  {0, -1, 0}, {0, 0, 1},  {0, 0, -1},
                            {1, 1, 0},  {-1, -1, 0}, {1, -1, 0}, {-1, 1, 0}, {1, 0, 1},  {-1, 0, -1}, {1, 0, -1},
                            {-1, 0, 1}, {0, 1, 1},  {0, -1, -1}, {0, 1, -1}, {0, -1, 1}};

double wq(int i) { return i == 0 ? 1.0 / 3.0 : (i <= 6 ? 1.0 / 18.0 : 1.0 / 36.0); }

// BMCSL contact values of uniform densities
void bmcsl(const mlb_params *p, const double *n, double g[kMaxS][kMaxS])
{
    const int M = p->nspecies;
    double x2 = 0.0, x3 = 0.0;
    for (int c = 0; c < M; ++c) {
        const double s = p->sigma[c];
        x2 += M_PI / 6.0 * s * s * n[c];
        x3 += M_PI / 6.0 * s * s * s * n[c];
    }
    for (int a = 0; a < M; ++a)
        for (int b = 0; b < M; ++b) {
            const double d = p->sigma[a] * p->sigma[b] / (p->sigma[a] + p->sigma[b]);
            const double q = 1.0 / (1.0 - x3), z = d * x2 * q;
            g[a][b] = q * (1.0 + z) * (1.0 + 2.0 * z);
        }
}

struct PairSums {
    double SV[3] = {0, 0, 0}, ST[3][3] = {}, ST0 = 0.0, TV[3] = {0, 0, 0};
};

}  // namespace

double stability_radius(const mlb_params *p, const double *n0, int kgrid)
{
    const int M = p->nspecies;
    const double kT = p->kT, omega = 1.0 / p->tau;
    double g[kMaxS][kMaxS], dg[kMaxS][kMaxS][kMaxS];
    bmcsl(p, n0, g);
    for (int c = 0; c < M; ++c) {
        double up[kMaxS], dn[kMaxS], gu[kMaxS][kMaxS], gd[kMaxS][kMaxS];
        for (int i = 0; i < M; ++i) up[i] = dn[i] = n0[i];
        const double h = 1e-7 * std::max(n0[c], 1e-4);
        up[c] += h;
        dn[c] -= h;
        bmcsl(p, up, gu);
        bmcsl(p, dn, gd);
        for (int a = 0; a < M; ++a)
            for (int b = 0; b < M; ++b) dg[a][b][c] = (gu[a][b] - gd[a][b]) / (2.0 * h);
    }
    HostStencil shell[kMaxS][kMaxS], tail[kMaxS][kMaxS], ball[kMaxS];
    double what[kMaxS][kMaxS], kap[kMaxS][kMaxS];
    for (int c = 0; c < M; ++c) ball[c] = build_stencil(kBall, p->sigma[c], 0.0);
    for (int a = 0; a < M; ++a)
        for (int b = 0; b < M; ++b) {
            const double sab = 0.5 * (p->sigma[a] + p->sigma[b]);
            shell[a][b] = build_stencil(kShell, sab, 0.0);
            what[a][b] = 4.0 * M_PI / (double)shell[a][b].full;
            const double mu = (p->mass[a] * p->mass[b]) / (p->mass[a] + p->mass[b]);
            kap[a][b] = 2.0 * sab * sab * std::sqrt(2.0 * mu * kT / M_PI) * what[a][b];
            if (p->eps[a * MLB_MAX_SPECIES + b] > 0.0) tail[a][b] = build_stencil(kTail, sab, p->rc_factor);
        }
    std::mt19937_64 rng(12345);
    std::normal_distribution<double> nd(0.0, 1.0);
    const int dim = kQ * M;
    double worst = 0.0;
    // the lattice, its weights and the stencils are invariant under permutations
    // of the axes, so k with kx >= ky >= kz cover the grid
    for (int ix = 0; ix <= kgrid; ++ix)
        for (int iy = 0; iy <= ix; ++iy)
            for (int iz = 0; iz <= iy; ++iz) {
                if (ix == 0 && iy == 0 && iz == 0) continue;
                const double k[3] = {M_PI * ix / kgrid, M_PI * iy / kgrid, M_PI * iz / kgrid};
                double Bf[kMaxS];
                for (int c = 0; c < M; ++c) {
                    double acc = 1.0;   // centre
                    for (size_t q = 0; q < ball[c].e.size(); ++q) {
                        int ex, ey, ez;
                        unpack_offset(ball[c].e[q], ex, ey, ez);
                        acc += 2.0 * std::cos(k[0] * ex + k[1] * ey + k[2] * ez);
                    }
                    Bf[c] = acc / (double)ball[c].full;
                }
                PairSums P[kMaxS][kMaxS];
                for (int a = 0; a < M; ++a)
                    for (int b = 0; b < M; ++b) {
                        PairSums &s = P[a][b];
                        const HostStencil &S = shell[a][b];
                        for (size_t q = 0; q < S.e.size(); ++q) {
                            int ex, ey, ez;
                            unpack_offset(S.e[q], ex, ey, ez);
                            const double ph = k[0] * ex + k[1] * ey + k[2] * ez;
                            const double *u = &S.v[3 * q];
                            for (int d = 0; d < 3; ++d) {
                                s.SV[d] += 2.0 * u[d] * std::sin(ph);          // +e and -e
                                for (int d2 = 0; d2 < 3; ++d2) s.ST[d][d2] += 2.0 * u[d] * u[d2] * std::cos(ph);
                            }
                        }
                        s.ST0 = (double)S.full / 3.0;
                        const double eps = p->eps[a * MLB_MAX_SPECIES + b];
                        if (eps > 0.0) {
                            const double sab = 0.5 * (p->sigma[a] + p->sigma[b]);
                            const double s6 = sab * sab * sab * sab * sab * sab;
                            const HostStencil &T = tail[a][b];
                            for (size_t q = 0; q < T.e.size(); ++q) {
                                int ex, ey, ez;
                                unpack_offset(T.e[q], ex, ey, ez);
                                const double r2 = (double)(ex * ex + ey * ey + ez * ez);
                                const double coef = 6.0 * eps * s6 / (r2 * r2 * r2 * std::sqrt(r2));
                                const double ph = k[0] * ex + k[1] * ey + k[2] * ez;
                                for (int d = 0; d < 3; ++d) s.TV[d] += 2.0 * coef * T.v[3 * q + d] * std::sin(ph);
                            }
                        }
                    }
                cd shift[kQ];
                for (int i = 0; i < kQ; ++i)
                    shift[i] = std::exp(cd(0.0, -(k[0] * kCx[i][0] + k[1] * kCx[i][1] + k[2] * kCx[i][2])));
                // one step of the linearised map
                auto apply = [&](const std::vector<cd> &f, std::vector<cd> &out) {
                    cd dn[kMaxS], dj[kMaxS][3], Nc[kMaxS][3], Dold[kMaxS][3], V[kMaxS][3], Nf[kMaxS][3];
                    double Gam[kMaxS];
                    for (int a = 0; a < M; ++a) {
                        dn[a] = 0.0;
                        for (int d = 0; d < 3; ++d) dj[a][d] = 0.0;
                        for (int i = 0; i < kQ; ++i) {
                            const cd fi = f[(size_t)a * kQ + i];
                            dn[a] += fi;
                            for (int d = 0; d < 3; ++d) dj[a][d] += (double)kCx[i][d] * fi;
                        }
                    }
                    for (int a = 0; a < M; ++a) {
                        Gam[a] = 0.0;
                        for (int d = 0; d < 3; ++d) Nc[a][d] = Dold[a][d] = 0.0;
                        for (int b = 0; b < M; ++b) {
                            cd dgab = 0.0;
                            for (int c = 0; c < M; ++c) dgab += dg[a][b][c] * Bf[c] * dn[c];
                            const double sab = 0.5 * (p->sigma[a] + p->sigma[b]);
                            const cd amp = g[a][b] * dn[b] + 0.5 * n0[b] * dgab;
                            const double kg = kap[a][b] * g[a][b];
                            for (int d = 0; d < 3; ++d) {
                                Nc[a][d] += -kT * n0[a] * sab * sab * what[a][b] * cd(0.0, P[a][b].SV[d]) * amp;
                                Nc[a][d] += n0[a] * cd(0.0, P[a][b].TV[d]) * dn[b];
                                cd st = 0.0;
                                for (int d2 = 0; d2 < 3; ++d2) st += P[a][b].ST[d][d2] * dj[b][d2];
                                Dold[a][d] += kg * (n0[a] * st - n0[b] * P[a][b].ST0 * dj[a][d]);
                            }
                            Gam[a] += kg * n0[b] * P[a][b].ST0;
                        }
                    }
                    for (int a = 0; a < M; ++a) {
                        const double im = 1.0 / p->mass[a], hg = 0.5 * Gam[a] * im;
                        for (int d = 0; d < 3; ++d) {
                            V[a][d] = n0[a] > 0.0 ? (dj[a][d] + im * (Nc[a][d] + Dold[a][d]) + hg * dj[a][d]) /
                                                        (n0[a] * (1.0 + hg))
                                                  : cd(0.0);
                        }
                    }
                    for (int a = 0; a < M; ++a)
                        for (int d = 0; d < 3; ++d) {
                            if (p->scheme == MLB_SCHEME_FE) {
                                Nf[a][d] = Nc[a][d] + Dold[a][d];
                                continue;
                            }
                            cd dnew = 0.0;
                            for (int b = 0; b < M; ++b) {
                                cd st = 0.0;
                                for (int d2 = 0; d2 < 3; ++d2) st += P[a][b].ST[d][d2] * V[b][d2];
                                dnew += kap[a][b] * g[a][b] * n0[b] * (st - P[a][b].ST0 * V[a][d]);
                            }
                            Nf[a][d] = Nc[a][d] + 0.5 * Dold[a][d] + 0.5 * n0[a] * dnew;
                        }
                    // barycentric velocity (mass-weighted) of the perturbation
                    cd du[3] = {0.0, 0.0, 0.0};
                    double rho0 = 0.0;
                    for (int a = 0; a < M; ++a) {
                        rho0 += p->mass[a] * n0[a];
                        for (int d = 0; d < 3; ++d) du[d] += p->mass[a] * dj[a][d];
                    }
                    for (int d = 0; d < 3; ++d) du[d] = rho0 > 0.0 ? du[d] / rho0 : cd(0.0);
                    // linearised collision at rest with theta_a = kT/m_a:
                    //   psi_perp_i = w_i h_i [dn + (m_a/kT) c.(dj - n du)] + 3 w_i n c.du
                    //   S_i = 3 w_i h_i c.N,  h_i = 1 + (9/2)(theta_a - 1/3)(c.c - 1)
                    for (int a = 0; a < M; ++a) {
                        const double ith = p->mass[a] / kT, dth = 4.5 * (kT / p->mass[a] - 1.0 / 3.0);
                        for (int i = 0; i < kQ; ++i) {
                            cd cv = 0.0, cN = 0.0, cu = 0.0;
                            for (int d = 0; d < 3; ++d) {
                                cv += (double)kCx[i][d] * (dj[a][d] - n0[a] * du[d]);
                                cN += (double)kCx[i][d] * Nf[a][d];
                                cu += (double)kCx[i][d] * du[d];
                            }
                            const int c2 = kCx[i][0] * kCx[i][0] + kCx[i][1] * kCx[i][1] + kCx[i][2] * kCx[i][2];
                            const double h = 1.0 + dth * (double)(c2 - 1);
                            const cd psi = wq(i) * (h * (dn[a] + ith * cv) + 3.0 * n0[a] * cu);
                            const cd fs = (1.0 - omega) * f[(size_t)a * kQ + i] + omega * psi + 3.0 * wq(i) * h * cN;
                            out[(size_t)a * kQ + i] = shift[i] * fs;
                        }
                    }
                };
                std::vector<cd> x((size_t)dim), y((size_t)dim);
                for (auto &v : x) v = cd(nd(rng), nd(rng));
                double logsum = 0.0;
                const int burn = 200, keep = 200;
                for (int it = 0; it < burn + keep; ++it) {
                    apply(x, y);
                    double nrm = 0.0;
                    for (auto &v : y) nrm += std::norm(v);
                    nrm = std::sqrt(nrm);
                    if (!(nrm > 0.0) || !std::isfinite(nrm)) {
                        nrm = nrm > 0.0 ? nrm : 0.0;
                        if (!std::isfinite(nrm)) return INFINITY;
                        break;
                    }
                    for (size_t q = 0; q < x.size(); ++q) x[q] = y[q] / nrm;
                    if (it >= burn) logsum += std::log(nrm);
                }
                worst = std::max(worst, std::exp(logsum / keep));
            }
    return worst;
}

}  // namespace mlb
