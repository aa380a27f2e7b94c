/*
 * FP64 CPU oracle for the multicomponent Enskog lattice-Boltzmann step.
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test suite, the smoke check and the
 * CPU-baseline leg of the benchmark may load this library.  It shares no
 * code, header, table generator or constant generator with the GPU library.
 *
 * What it computes (Marini Bettolo Marconi & Melchionna, "Multicomponent
 * diffusion in nanosystems"):
 *   - the kinetic equation of Sec. 2, eq. (evolution), with the local
 *     Maxwellian eq. (psia) and its orthogonalised form eq. (prefactor),
 *     discretised on D3Q19 with a second-order Hermite equilibrium;
 *   - the moments of eq. (colonna) and the barycentric velocity (Sec. 2);
 *   - the self-consistent field of Sec. 3, eq. (splitforce): the hard-core
 *     mean field eq. (potmeanforce), the RPA attractive molecular field
 *     below it, and the drag eq. (gammaab)/(tensorgamma) plus viscous
 *     eq. (viscousforce) forces, merged into one pair form (their sum only
 *     involves u_b(r+sigma s) - u_a(r)).
 * The paper leaves the lattice discretisation to another paper; the
 * readings taken here (lattice shells, BMCSL contact values of ball-smoothed
 * packing fractions, Crank-Nicolson friction with one Jacobi predictor
 * sweep, halfway bounce-back walls beyond which the hard-core stencils see
 * the mirrored fluid moving with the wall) are the ones listed in the design
 * notes of the repository, and every arithmetic step below is written in the
 * fixed order that a bit-exact FP64 comparison relies on:
 *   velocities in canonical order, stencil half-lists sorted by
 *   (|e|^2, ex, ey, ez) with each (+e,-e) pair combined first, species
 *   ascending, no fused multiply-add (build with -ffp-contract=off).
 *
 * Sites are processed in parallel with OpenMP; per-site arithmetic does not
 * depend on the thread count, so results are identical for any count.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define OR_MAXS 4
#define OR_Q 19

/* ---------------------------------------------------------------- params */
typedef struct {
    int32_t nx, ny, nz, M;
    double tau, kT;
    double sigma[OR_MAXS];           /* sigma_aa in lattice units          */
    double eps[OR_MAXS * OR_MAXS];   /* attraction depth eps_ab (0 = off)  */
    double rc_factor;                /* tail cutoff in units of sigma_ab   */
    double fext[OR_MAXS * 3];        /* uniform external force F^a         */
    int32_t walls_y;                 /* 1: solid layers at y=0 and y=ny-1  */
    double wall_ux[2];               /* x velocity of the y=0 / y=ny-1 wall */
    int32_t scheme;                  /* 0: CN-J1, 1: forward Euler         */
    double mass[OR_MAXS];            /* species masses m_a (> 0)           */
} or_params;

/* D3Q19 in canonical order: rest, +-x, +-y, +-z, then the xy, xz, yz edges.
 * Odd index i has its opposite at i+1. */
static const int C[OR_Q][3] = {
    {0, 0, 0},
    {1, 0, 0}, {-1, 0, 0}, {0, 1, 0}, {0, -1, 0}, {0, 0, 1}, {0, 0, -1},
    {1, 1, 0}, {-1, -1, 0}, {1, -1, 0}, {-1, 1, 0},
    {1, 0, 1}, {-1, 0, -1}, {1, 0, -1}, {-1, 0, 1},
    {0, 1, 1}, {0, -1, -1}, {0, 1, -1}, {0, -1, 1}};

static double weight_of(int i)
{
    if (i == 0) return 1.0 / 3.0;
    if (i <= 6) return 1.0 / 18.0;
    return 1.0 / 36.0;
}

static int opposite_of(int i)
{
    if (i == 0) return 0;
    return (i % 2 == 1) ? i + 1 : i - 1;
}

/* ------------------------------------------------------------- stencils */
/* A half list: offsets with a positive first non-zero component, sorted by
 * (|e|^2, ex, ey, ez).  unit[] holds e/|e|, vec[] an optional vector weight
 * (tail), full = size of the symmetric set (2 * n, plus 1 for a ball). */
typedef struct {
    int n, full;
    int *e;
    double *unit;
    double *vec;
} or_list;

typedef struct {
    int ex, ey, ez, r2;
} or_off;

static int cmp_off(const void *pa, const void *pb)
{
    const or_off *a = (const or_off *)pa, *b = (const or_off *)pb;
    if (a->r2 != b->r2) return a->r2 < b->r2 ? -1 : 1;
    if (a->ex != b->ex) return a->ex < b->ex ? -1 : 1;
    if (a->ey != b->ey) return a->ey < b->ey ? -1 : 1;
    if (a->ez != b->ez) return a->ez < b->ez ? -1 : 1;
    return 0;
}

static int positive_half(int x, int y, int z)
{
    return x > 0 || (x == 0 && y > 0) || (x == 0 && y == 0 && z > 0);
}

/* kind 0: shell (s-1/2)^2 <= |e|^2 < (s+1/2)^2      (lattice sphere of
 *         radius s, the surface integrals of eqs. potmeanforce,
 *         tensorgamma, viscousforce)
 * kind 1: ball  |e|^2 <= (s/2)^2                     (smoothing volume)
 * kind 2: tail  s^2 < |e|^2 <= (rc*s)^2              (r > sigma_ab) */
static void build_list(or_list *L, int kind, double s, double rc)
{
    double lo, hi;
    int R, cap, n = 0;
    if (kind == 0) {
        lo = (s - 0.5) * (s - 0.5);
        hi = (s + 0.5) * (s + 0.5);
    } else if (kind == 1) {
        lo = 0.0;
        hi = (0.5 * s) * (0.5 * s);
    } else {
        lo = s * s;
        hi = (rc * s) * (rc * s);
    }
    R = (int)ceil(sqrt(hi)) + 1;
    cap = (2 * R + 1) * (2 * R + 1) * (2 * R + 1);
    or_off *tmp = (or_off *)malloc(sizeof(or_off) * (size_t)cap);
    for (int x = -R; x <= R; ++x)
        for (int y = -R; y <= R; ++y)
            for (int z = -R; z <= R; ++z) {
                int r2 = x * x + y * y + z * z;
                double d = (double)r2;
                int in;
                if (!positive_half(x, y, z)) continue;
                if (kind == 0) in = (d >= lo) && (d < hi);
                else if (kind == 1) in = (d <= hi);
                else in = (d > lo) && (d <= hi);
                if (in) {
                    tmp[n].ex = x; tmp[n].ey = y; tmp[n].ez = z; tmp[n].r2 = r2;
                    ++n;
                }
            }
    qsort(tmp, (size_t)n, sizeof(or_off), cmp_off);
    L->n = n;
    L->full = 2 * n + (kind == 1 ? 1 : 0);
    L->e = (int *)malloc(sizeof(int) * 3 * (size_t)(n > 0 ? n : 1));
    L->unit = (double *)malloc(sizeof(double) * 3 * (size_t)(n > 0 ? n : 1));
    L->vec = NULL;
    for (int k = 0; k < n; ++k) {
        double len = sqrt((double)tmp[k].r2);
        L->e[3 * k + 0] = tmp[k].ex;
        L->e[3 * k + 1] = tmp[k].ey;
        L->e[3 * k + 2] = tmp[k].ez;
        L->unit[3 * k + 0] = (double)tmp[k].ex / len;
        L->unit[3 * k + 1] = (double)tmp[k].ey / len;
        L->unit[3 * k + 2] = (double)tmp[k].ez / len;
    }
    free(tmp);
}

static void free_list(or_list *L)
{
    free(L->e);
    free(L->unit);
    free(L->vec);
    L->e = NULL; L->unit = NULL; L->vec = NULL; L->n = 0;
}

/* --------------------------------------------------------------- context */
typedef struct {
    or_params p;
    long N;
    int M, P;
    double omega, om1;
    or_list shell[OR_MAXS][OR_MAXS];
    or_list tail[OR_MAXS][OR_MAXS];
    or_list ball[OR_MAXS];
    int has_tail[OR_MAXS][OR_MAXS];
    double cm[OR_MAXS][OR_MAXS]; /* mean field:  -kT sigma^2 w_hat / 2      */
    double cg[OR_MAXS][OR_MAXS]; /* trace/3 of the friction: kappa / 6      */
    double ck[OR_MAXS][OR_MAXS]; /* dissipative pair form: kappa / 2        */
    double dd[OR_MAXS][OR_MAXS]; /* BMCSL d_ab = s_a s_b / (s_a + s_b)      */
    double s2[OR_MAXS], s3[OR_MAXS]; /* (pi/6) sigma^2, (pi/6) sigma^3      */
    /* per species: 1/m_a; m_a/kT = 1/theta_a (theta_a = kT/m_a, the thermal
     * speed^2 of eq. psia); (9/2)(theta_a - 1/3), the weight of the Hermite
     * temperature term of the lattice equilibrium (0 when theta_a is the
     * lattice's c_s^2 = 1/3, i.e. m_a = 1 at kT = 1/3) */
    double im[OR_MAXS], ith[OR_MAXS], dth[OR_MAXS];
    /* work fields */
    double *n, *j, *u, *g, *vh, *H, *N2, *Nmf, *Ntl, *Nex, *Dold, *Dnew, *Gam;
    /* optional externally supplied attractive field sum_b (K_ab * n_b) [M][3][N] */
    const double *tail_ext;
    /* optional body force per lattice row, F^a(y) = fext[a] + profile[a][y],
     * [M][3][ny] (NULL: the uniform fext) */
    double *fy;
} or_ctx;

static int pair_index(int M, int a, int b)
{
    int lo = a < b ? a : b, hi = a < b ? b : a;
    /* packed upper triangle, row-major: (0,0),(0,1)..(0,M-1),(1,1).. */
    return lo * M - (lo * (lo - 1)) / 2 + (hi - lo);
}

or_ctx *or_create(const or_params *p)
{
    if (p->M < 1 || p->M > OR_MAXS || p->nx < 1 || p->ny < 1 || p->nz < 1) return NULL;
    for (int a = 0; a < p->M; ++a)
        if (!(p->mass[a] > 0.0)) return NULL;
    or_ctx *c = (or_ctx *)calloc(1, sizeof(or_ctx));
    c->p = *p;
    c->M = p->M;
    c->P = p->M * (p->M + 1) / 2;
    c->N = (long)p->nx * p->ny * p->nz;
    c->omega = 1.0 / p->tau;
    c->om1 = 1.0 - c->omega;
    const double kT = p->kT;
    for (int a = 0; a < c->M; ++a) {
        double ma = p->mass[a];
        c->im[a] = 1.0 / ma;
        c->ith[a] = ma / kT;
        c->dth[a] = 4.5 * (kT / ma - 1.0 / 3.0);
        double sg = p->sigma[a];
        c->s2[a] = (M_PI / 6.0) * (sg * sg);
        c->s3[a] = (M_PI / 6.0) * ((sg * sg) * sg);
        build_list(&c->ball[a], 1, sg, 0.0);
    }
    for (int a = 0; a < c->M; ++a)
        for (int b = 0; b < c->M; ++b) {
            double sa = p->sigma[a], sb = p->sigma[b];
            double sab = 0.5 * (sa + sb);
            /* reduced mass of the colliding pair (below eq. viscousforce) */
            double mu = (p->mass[a] * p->mass[b]) / (p->mass[a] + p->mass[b]);
            build_list(&c->shell[a][b], 0, sab, 0.0);
            double what = (4.0 * M_PI) / (double)c->shell[a][b].full;
            double kap = ((2.0 * (sab * sab)) * sqrt((2.0 * mu * kT) / M_PI)) * what;
            c->cm[a][b] = ((-0.5 * kT) * (sab * sab)) * what;
            c->cg[a][b] = kap / 6.0;
            c->ck[a][b] = 0.5 * kap;
            c->dd[a][b] = (sa * sb) / (sa + sb);
            double eps = p->eps[a * OR_MAXS + b];
            c->has_tail[a][b] = eps != 0.0;
            if (eps != 0.0) {
                or_list *T = &c->tail[a][b];
                build_list(T, 2, sab, p->rc_factor);
                T->vec = (double *)malloc(sizeof(double) * 3 * (size_t)(T->n > 0 ? T->n : 1));
                double s6 = ((sab * sab) * (sab * sab)) * (sab * sab);
                for (int k = 0; k < T->n; ++k) {
                    int ex = T->e[3 * k], ey = T->e[3 * k + 1], ez = T->e[3 * k + 2];
                    double r2 = (double)(ex * ex + ey * ey + ez * ez);
                    double len = sqrt(r2);
                    double r7 = ((r2 * r2) * r2) * len;
                    /* -dU/dr for U = -eps (sigma/r)^6, i.e. 6 eps sigma^6 / r^7 */
                    double coef = ((6.0 * eps) * s6) / r7;
                    T->vec[3 * k + 0] = coef * T->unit[3 * k + 0];
                    T->vec[3 * k + 1] = coef * T->unit[3 * k + 1];
                    T->vec[3 * k + 2] = coef * T->unit[3 * k + 2];
                }
            }
        }
    size_t N = (size_t)c->N, M = (size_t)c->M;
    c->n = (double *)calloc(M * N, sizeof(double));
    c->j = (double *)calloc(3 * M * N, sizeof(double));
    c->u = (double *)calloc(3 * N, sizeof(double));
    c->g = (double *)calloc((size_t)c->P * N, sizeof(double));
    c->vh = (double *)calloc(3 * M * N, sizeof(double));
    c->H = (double *)calloc(3 * M * N, sizeof(double));
    c->N2 = (double *)calloc(3 * M * N, sizeof(double));
    c->Nmf = (double *)calloc(3 * M * N, sizeof(double));
    c->Ntl = (double *)calloc(3 * M * N, sizeof(double));
    c->Nex = (double *)calloc(3 * M * N, sizeof(double));
    c->Dold = (double *)calloc(3 * M * N, sizeof(double));
    c->Dnew = (double *)calloc(3 * M * N, sizeof(double));
    c->Gam = (double *)calloc(M * N, sizeof(double));
    return c;
}

void or_destroy(or_ctx *c)
{
    if (!c) return;
    for (int a = 0; a < OR_MAXS; ++a) {
        free_list(&c->ball[a]);
        for (int b = 0; b < OR_MAXS; ++b) {
            free_list(&c->shell[a][b]);
            free_list(&c->tail[a][b]);
        }
    }
    free(c->n); free(c->j); free(c->u); free(c->g); free(c->vh); free(c->H);
    free(c->N2); free(c->Nmf); free(c->Ntl); free(c->Nex); free(c->Dold);
    free(c->Dnew); free(c->Gam); free(c->fy);
    free(c);
}

/* ------------------------------------------------------------- geometry */
static inline int is_solid(const or_ctx *c, int y)
{
    return c->p.walls_y && (y == 0 || y == c->p.ny - 1);
}

static inline int wrap(int v, int n)
{
    int r = v % n;
    return r < 0 ? r + n : r;
}

/* Linear index of r + e as the attractive field sees it; -1 when the
 * neighbour lies outside a walled box (no fluid there: the field sums zero
 * density beyond a wall). */
static inline long neighbour(const or_ctx *c, int x, int y, int z, int ex, int ey, int ez)
{
    int xx = wrap(x + ex, c->p.nx);
    int zz = wrap(z + ez, c->p.nz);
    int yy = y + ey;
    if (c->p.walls_y) {
        if (yy < 0 || yy >= c->p.ny) return -1;
    } else {
        yy = wrap(yy, c->p.ny);
    }
    return ((long)zz * c->p.ny + yy) * c->p.nx + xx;
}

static inline double fld(const double *F, long s) { return s < 0 ? 0.0 : F[s]; }

/* Neighbour of r + e as the hard-core stencils (smoothing balls and the
 * shells of the mean field and of the friction) see it.  In a periodic box
 * and inside the fluid rows it is the site itself.  Beyond a wall
 * (y + e_y <= 0 or >= ny - 1 in a walled box) it is the mirror image of the
 * fluid across the nearer wall plane, y = 1/2 or y = ny - 3/2, where halfway
 * bounce-back puts the walls: the image carries the density and contact
 * value of the mirrored fluid site and moves with the wall.  *img is 0 for
 * a fluid site, 1 for an image beyond the y = 0 wall, 2 beyond the
 * y = ny - 1 wall. */
static inline long hc_neighbour(const or_ctx *c, int x, int y, int z, int ex, int ey, int ez, int *img)
{
    int xx = wrap(x + ex, c->p.nx);
    int zz = wrap(z + ez, c->p.nz);
    int yy = y + ey;
    *img = 0;
    if (c->p.walls_y) {
        if (yy <= 0) {
            yy = 1 - yy;
            *img = 1;
        } else if (yy >= c->p.ny - 1) {
            yy = 2 * c->p.ny - 3 - yy;
            *img = 2;
        }
    } else {
        yy = wrap(yy, c->p.ny);
    }
    return ((long)zz * c->p.ny + yy) * c->p.nx + xx;
}

/* Component d of a velocity field V at a hard-core neighbour: the wall's
 * velocity (u_wall, 0, 0) for an image, else V there. */
static inline double hc_vel(const or_ctx *c, const double *V, long s, int img, int d, long N)
{
    if (img) return d == 0 ? c->p.wall_ux[img - 1] : 0.0;
    return V[(size_t)d * N + s];
}

/* --------------------------------------------------- S1: moments, eq. (colonna) */
static void moments(or_ctx *c, const double *f)
{
    const long N = c->N;
    const int M = c->M;
#pragma omp parallel for schedule(static)
    for (long s = 0; s < N; ++s) {
        double nt = 0.0, jt[3] = {0.0, 0.0, 0.0};
        for (int a = 0; a < M; ++a) {
            const double *fa = f + (size_t)a * OR_Q * N;
            double na = fa[0 * N + s];
            for (int i = 1; i < OR_Q; ++i) na = na + fa[(size_t)i * N + s];
            double ja[3];
            for (int d = 0; d < 3; ++d) {
                double acc = 0.0;
                for (int i = 1; i < OR_Q; ++i) {
                    if (C[i][d] == 1) acc = acc + fa[(size_t)i * N + s];
                    else if (C[i][d] == -1) acc = acc - fa[(size_t)i * N + s];
                }
                ja[d] = acc;
            }
            c->n[(size_t)a * N + s] = na;
            for (int d = 0; d < 3; ++d) c->j[((size_t)a * 3 + d) * N + s] = ja[d];
            /* mass densities rho_a = m_a n_a; the barycentric velocity is
             * sum_a m_a j_a / sum_a m_a n_a (Sec. 2, eq. massdensity and below) */
            const double ma = c->p.mass[a];
            if (a == 0) {
                nt = ma * na;
                jt[0] = ma * ja[0]; jt[1] = ma * ja[1]; jt[2] = ma * ja[2];
            } else {
                nt = nt + ma * na;
                jt[0] = jt[0] + ma * ja[0]; jt[1] = jt[1] + ma * ja[1]; jt[2] = jt[2] + ma * ja[2];
            }
        }
        for (int d = 0; d < 3; ++d) c->u[(size_t)d * N + s] = (nt != 0.0) ? jt[d] / nt : 0.0;
    }
}

/* ------------------------- S2: smoothed packing fractions and BMCSL contact
 * values.  The paper only says that g at contact depends on the densities
 * through a smoothing procedure (Sec. 2, discussion of eq. evolution); the
 * reading used: ball means of radius sigma_cc/2, xi_k = (pi/6) sum_c
 * sigma_cc^k nbar_c, and the Boublik-Mansoori-Carnahan-Starling-Leland
 * mixture contact value
 *   g_ab = 1/(1-xi3) + 3 d xi2/(1-xi3)^2 + 2 d^2 xi2^2/(1-xi3)^3
 *        = q (1+z)(1+2z),  q = 1/(1-xi3),  z = d xi2 q,
 * with d = s_a s_b / (s_a + s_b). */
static void contact_values(or_ctx *c)
{
    const long N = c->N;
    const int M = c->M, nx = c->p.nx, ny = c->p.ny;
#pragma omp parallel for schedule(static)
    for (long s = 0; s < N; ++s) {
        int x = (int)(s % nx), y = (int)((s / nx) % ny), z = (int)(s / ((long)nx * ny));
        if (is_solid(c, y)) {
            for (int p = 0; p < c->P; ++p) c->g[(size_t)p * N + s] = 0.0;
            continue;
        }
        double nb[OR_MAXS];
        for (int cc = 0; cc < M; ++cc) {
            const double *nc = c->n + (size_t)cc * N;
            const or_list *B = &c->ball[cc];
            double acc = nc[s];
            for (int k = 0; k < B->n; ++k) {
                int ip, im;
                long sp = hc_neighbour(c, x, y, z, B->e[3 * k], B->e[3 * k + 1], B->e[3 * k + 2], &ip);
                long sm = hc_neighbour(c, x, y, z, -B->e[3 * k], -B->e[3 * k + 1], -B->e[3 * k + 2], &im);
                acc = acc + (nc[sp] + nc[sm]);
            }
            nb[cc] = acc / (double)B->full;
        }
        double x2 = c->s2[0] * nb[0], x3 = c->s3[0] * nb[0];
        for (int cc = 1; cc < M; ++cc) {
            x2 = x2 + c->s2[cc] * nb[cc];
            x3 = x3 + c->s3[cc] * nb[cc];
        }
        double q = 1.0 / (1.0 - x3);
        for (int a = 0; a < M; ++a)
            for (int b = a; b < M; ++b) {
                double zz = (c->dd[a][b] * x2) * q;
                double gab = q * ((1.0 + zz) * (1.0 + 2.0 * zz));
                c->g[(size_t)pair_index(M, a, b) * N + s] = gab;
            }
    }
}

/* -------------------------------- S3: first gather and the velocity predictor.
 * For species a at r, partner b, shell S_ab (radius sigma_ab):
 *   hard-core mean field, eq. (potmeanforce):
 *     Nmf_a = -kT sum_b sigma_ab^2 w_hat sum_e e_hat G n_a(r) n_b(r+e)
 *   attractive field (RPA, g = 1), below eq. (potmeanforce):
 *     Ntl_a = n_a(r) sum_b sum_{e in T_ab} n_b(r+e) 6 eps sigma^6 / |e|^7 e_hat
 *   drag + viscous forces, eqs. (gammaab), (tensorgamma), (viscousforce),
 *   as one pair form evaluated at the old velocities u_c = j_c / n_c:
 *     D_a[u] = sum_b kappa_ab sum_e G e_hat (e_hat . (n_a(r) j_b(r+e) - n_b(r+e) j_a(r)))
 *     kappa_ab = 2 sigma_ab^2 sqrt(2 mu_ab kT / pi) w_hat
 *   friction rate (trace/3 of the local friction tensor):
 *     Gam_a = (1/3) sum_b kappa_ab sum_e G n_b(r+e)
 * with G = (g_ab(r) + g_ab(r+e)) / 2 and w_hat = 4 pi / |S_ab|.
 * The predictor takes the local diagonal of the velocity-dependent force
 * implicitly (one Jacobi sweep of a Crank-Nicolson step); a force density
 * changes the number flux j_a at the rate 1/m_a (eq. momentcomponent):
 *   V_a = [j_a + (Nc_a + D_a[u]) / m_a + Gam_a j_a / (2 m_a)] / [n_a (1 + Gam_a / (2 m_a))]
 *   H_a = Nc_a + D_a[u] / 2,   Nc_a = Nmf_a + Ntl_a + n_a F^a. */
static void gather_one(or_ctx *c)
{
    const long N = c->N;
    const int M = c->M, nx = c->p.nx, ny = c->p.ny;
#pragma omp parallel for schedule(static)
    for (long s = 0; s < N; ++s) {
        int x = (int)(s % nx), y = (int)((s / nx) % ny), z = (int)(s / ((long)nx * ny));
        for (int a = 0; a < M; ++a) {
            size_t o3 = (size_t)a * 3 * N;
            if (is_solid(c, y)) {
                for (int d = 0; d < 3; ++d) {
                    c->vh[o3 + d * N + s] = 0.0; c->H[o3 + d * N + s] = 0.0;
                    c->Nmf[o3 + d * N + s] = 0.0; c->Ntl[o3 + d * N + s] = 0.0;
                    c->Nex[o3 + d * N + s] = 0.0; c->Dold[o3 + d * N + s] = 0.0;
                }
                c->Gam[(size_t)a * N + s] = 0.0;
                continue;
            }
            double na = c->n[(size_t)a * N + s];
            double ja[3] = {c->j[o3 + 0 * N + s], c->j[o3 + 1 * N + s], c->j[o3 + 2 * N + s]};
            double mf[3] = {0.0, 0.0, 0.0}, tl[3] = {0.0, 0.0, 0.0}, dv[3] = {0.0, 0.0, 0.0};
            double gam = 0.0;
            for (int b = 0; b < M; ++b) {
                const double *nb = c->n + (size_t)b * N;
                const double *jb = c->j + (size_t)b * 3 * N;
                const double *gp = c->g + (size_t)pair_index(M, a, b) * N;
                const or_list *S = &c->shell[a][b];
                double g0 = gp[s];
                double smf[3] = {0.0, 0.0, 0.0}, sdv[3] = {0.0, 0.0, 0.0}, sg = 0.0;
                for (int k = 0; k < S->n; ++k) {
                    int ex = S->e[3 * k], ey = S->e[3 * k + 1], ez = S->e[3 * k + 2];
                    const double *eh = S->unit + 3 * k;
                    int ip, im;
                    long sp = hc_neighbour(c, x, y, z, ex, ey, ez, &ip);
                    long sm = hc_neighbour(c, x, y, z, -ex, -ey, -ez, &im);
                    double Gp = g0 + gp[sp], Gm = g0 + gp[sm];
                    double np_ = nb[sp], nm_ = nb[sm];
                    double tp = Gp * np_, tm = Gm * nm_;
                    double dt = tp - tm;
                    smf[0] = smf[0] + eh[0] * dt;
                    smf[1] = smf[1] + eh[1] * dt;
                    smf[2] = smf[2] + eh[2] * dt;
                    sg = sg + (tp + tm);
                    double Xp[3], Xm[3];
                    for (int d = 0; d < 3; ++d) {
                        /* an image's momentum density: its density times the wall's velocity */
                        double jp = ip ? np_ * hc_vel(c, NULL, 0, ip, d, N) : jb[(size_t)d * N + sp];
                        double jm = im ? nm_ * hc_vel(c, NULL, 0, im, d, N) : jb[(size_t)d * N + sm];
                        Xp[d] = na * jp - np_ * ja[d];
                        Xm[d] = na * jm - nm_ * ja[d];
                    }
                    double pp = Gp * ((eh[0] * Xp[0] + eh[1] * Xp[1]) + eh[2] * Xp[2]);
                    double pm = Gm * ((eh[0] * Xm[0] + eh[1] * Xm[1]) + eh[2] * Xm[2]);
                    double pq = pp + pm;
                    sdv[0] = sdv[0] + eh[0] * pq;
                    sdv[1] = sdv[1] + eh[1] * pq;
                    sdv[2] = sdv[2] + eh[2] * pq;
                }
                for (int d = 0; d < 3; ++d) {
                    mf[d] = mf[d] + c->cm[a][b] * smf[d];
                    dv[d] = dv[d] + c->ck[a][b] * sdv[d];
                }
                gam = gam + c->cg[a][b] * sg;
                if (c->has_tail[a][b] && !c->tail_ext) {
                    const or_list *T = &c->tail[a][b];
                    double st[3] = {0.0, 0.0, 0.0};
                    for (int k = 0; k < T->n; ++k) {
                        int ex = T->e[3 * k], ey = T->e[3 * k + 1], ez = T->e[3 * k + 2];
                        long sp = neighbour(c, x, y, z, ex, ey, ez);
                        long sm = neighbour(c, x, y, z, -ex, -ey, -ez);
                        double dn = fld(nb, sp) - fld(nb, sm);
                        st[0] = st[0] + T->vec[3 * k + 0] * dn;
                        st[1] = st[1] + T->vec[3 * k + 1] * dn;
                        st[2] = st[2] + T->vec[3 * k + 2] * dn;
                    }
                    tl[0] = tl[0] + st[0]; tl[1] = tl[1] + st[1]; tl[2] = tl[2] + st[2];
                }
            }
            if (c->tail_ext)
                for (int d = 0; d < 3; ++d) tl[d] = c->tail_ext[o3 + (size_t)d * N + s];
            const double im = c->im[a];
            double hg = (0.5 * gam) * im;
            for (int d = 0; d < 3; ++d) {
                double Nmf = na * mf[d];
                double Ntl = na * tl[d];
                double Fa = c->fy ? c->fy[((size_t)a * 3 + d) * ny + y] : c->p.fext[a * 3 + d];
                double Nex = na * Fa;
                double Nc = (Nmf + Ntl) + Nex;
                double Dd = dv[d];
                c->Nmf[o3 + d * N + s] = Nmf;
                c->Ntl[o3 + d * N + s] = Ntl;
                c->Nex[o3 + d * N + s] = Nex;
                c->Dold[o3 + d * N + s] = Dd;
                if (c->p.scheme == 1) {
                    /* forward Euler: the whole force at the old velocities */
                    c->H[o3 + d * N + s] = Nc + Dd;
                    c->vh[o3 + d * N + s] = 0.0;
                } else {
                    c->H[o3 + d * N + s] = Nc + 0.5 * Dd;
                    c->vh[o3 + d * N + s] =
                        (na != 0.0) ? (((ja[d] + im * Nc) + im * Dd) + hg * ja[d]) / (na * (1.0 + hg)) : 0.0;
                }
            }
            c->Gam[(size_t)a * N + s] = gam;
        }
    }
}

/* ------------------------------ S4: second gather, D_a evaluated at the
 * predicted velocities V (same pair form as above, written with V):
 *   D_a[V] = n_a(r) sum_b kappa_ab sum_e G n_b(r+e) e_hat (e_hat . (V_b(r+e) - V_a(r)))
 *   N_a = H_a + D_a[V] / 2   (the force density n_a Phi_a of eq. evolution) */
static void gather_two(or_ctx *c)
{
    const long N = c->N;
    const int M = c->M, nx = c->p.nx, ny = c->p.ny;
#pragma omp parallel for schedule(static)
    for (long s = 0; s < N; ++s) {
        int x = (int)(s % nx), y = (int)((s / nx) % ny), z = (int)(s / ((long)nx * ny));
        for (int a = 0; a < M; ++a) {
            size_t o3 = (size_t)a * 3 * N;
            if (is_solid(c, y) || c->p.scheme == 1) {
                for (int d = 0; d < 3; ++d) {
                    c->Dnew[o3 + d * N + s] = 0.0;
                    c->N2[o3 + d * N + s] = c->H[o3 + d * N + s];
                }
                continue;
            }
            double na = c->n[(size_t)a * N + s];
            double va[3] = {c->vh[o3 + 0 * N + s], c->vh[o3 + 1 * N + s], c->vh[o3 + 2 * N + s]};
            double dv[3] = {0.0, 0.0, 0.0};
            for (int b = 0; b < M; ++b) {
                const double *nb = c->n + (size_t)b * N;
                const double *vb = c->vh + (size_t)b * 3 * N;
                const double *gp = c->g + (size_t)pair_index(M, a, b) * N;
                const or_list *S = &c->shell[a][b];
                double g0 = gp[s];
                double sdv[3] = {0.0, 0.0, 0.0};
                for (int k = 0; k < S->n; ++k) {
                    int ex = S->e[3 * k], ey = S->e[3 * k + 1], ez = S->e[3 * k + 2];
                    const double *eh = S->unit + 3 * k;
                    int ip, im;
                    long sp = hc_neighbour(c, x, y, z, ex, ey, ez, &ip);
                    long sm = hc_neighbour(c, x, y, z, -ex, -ey, -ez, &im);
                    double tp = (g0 + gp[sp]) * nb[sp];
                    double tm = (g0 + gp[sm]) * nb[sm];
                    double Yp[3], Ym[3];
                    for (int d = 0; d < 3; ++d) {
                        Yp[d] = hc_vel(c, vb, sp, ip, d, N) - va[d];
                        Ym[d] = hc_vel(c, vb, sm, im, d, N) - va[d];
                    }
                    double pp = tp * ((eh[0] * Yp[0] + eh[1] * Yp[1]) + eh[2] * Yp[2]);
                    double pm = tm * ((eh[0] * Ym[0] + eh[1] * Ym[1]) + eh[2] * Ym[2]);
                    double pq = pp + pm;
                    sdv[0] = sdv[0] + eh[0] * pq;
                    sdv[1] = sdv[1] + eh[1] * pq;
                    sdv[2] = sdv[2] + eh[2] * pq;
                }
                for (int d = 0; d < 3; ++d) dv[d] = dv[d] + c->ck[a][b] * sdv[d];
            }
            for (int d = 0; d < 3; ++d) {
                double Dn = na * dv[d];
                c->Dnew[o3 + d * N + s] = Dn;
                c->N2[o3 + d * N + s] = c->H[o3 + d * N + s] + 0.5 * Dn;
            }
        }
    }
}

/* ----------------- S5: orthogonalised BGK collision plus the field term.
 * The Maxwellian of eq. (psia) at the barycentric u with thermal speed^2
 * theta_a = kT/m_a, in second-order Hermite form on the lattice
 * (c_s^2 = 1/3):
 *   E_i(u) = 1 + 3 c.u + 9/2 (c.u)^2 - 3/2 u.u + (9/2)(theta_a - 1/3)(c.c - 1)
 * (the last term gives sum_i w_i E_i c c = theta_a I + u u; it vanishes for
 * theta_a = 1/3), and
 *   psi_perp_i = w_i E_i [n_a + (m_a/kT) (j_a - n_a u).(c_i - u)]  eq. (prefactor)
 *   S_i        = w_i E_i (c_i - u).N_a / kT                      eq. (evolution)
 *   f*_i = (1 - omega) f_i + omega psi_perp_i + S_i.
 * psi_perp carries n_a and j_a; S_i adds no mass and N_a / m_a to j_a. */
static inline double hermite_E(const or_ctx *c, int a, int i, const double u[3])
{
    double uu = (u[0] * u[0] + u[1] * u[1]) + u[2] * u[2];
    double cx = (double)C[i][0], cy = (double)C[i][1], cz = (double)C[i][2];
    double cu = (cx * u[0] + cy * u[1]) + cz * u[2];
    double E = ((1.0 + 3.0 * cu) + (4.5 * cu) * cu) - 1.5 * uu;
    if (c->dth[a] != 0.0) {
        int c2 = C[i][0] * C[i][0] + C[i][1] * C[i][1] + C[i][2] * C[i][2];
        E = E + c->dth[a] * (double)(c2 - 1);
    }
    return E;
}

static inline double post_collision(const or_ctx *c, int a, int i, double fi, double na, const double ja[3],
                                    const double u[3], const double Na[3])
{
    double cx = (double)C[i][0], cy = (double)C[i][1], cz = (double)C[i][2];
    double wE = weight_of(i) * hermite_E(c, a, i, u);
    double m0 = cx - u[0], m1 = cy - u[1], m2 = cz - u[2];
    double v0 = ja[0] - na * u[0], v1 = ja[1] - na * u[1], v2 = ja[2] - na * u[2];
    double dotv = (v0 * m0 + v1 * m1) + v2 * m2;
    double dotN = (m0 * Na[0] + m1 * Na[1]) + m2 * Na[2];
    double psi = wE * (na + c->ith[a] * dotv);
    double src = wE * (3.0 * dotN);   /* 3 = 1/kT */
    return (c->om1 * fi + c->omega * psi) + src;
}

/* ---------------------------- S6: push streaming; halfway bounce-back at
 * walls moving in x: a population that would enter a solid layer returns
 * to its site reversed, f_opp = f*_i - 6 w_i n_a (c_i . u_wall). */
static void collide_stream(or_ctx *c, const double *f, double *fo)
{
    const long N = c->N;
    const int M = c->M, nx = c->p.nx, ny = c->p.ny;
    memset(fo, 0, sizeof(double) * (size_t)M * OR_Q * (size_t)N);
#pragma omp parallel for schedule(static)
    for (long s = 0; s < N; ++s) {
        int x = (int)(s % nx), y = (int)((s / nx) % ny), z = (int)(s / ((long)nx * ny));
        if (is_solid(c, y)) continue;
        double u[3] = {c->u[s], c->u[N + s], c->u[2 * N + s]};
        for (int a = 0; a < M; ++a) {
            size_t o3 = (size_t)a * 3 * N;
            const double *fa = f + (size_t)a * OR_Q * N;
            double *foa = fo + (size_t)a * OR_Q * N;
            double na = c->n[(size_t)a * N + s];
            double ja[3] = {c->j[o3 + s], c->j[o3 + N + s], c->j[o3 + 2 * N + s]};
            double Na[3] = {c->N2[o3 + s], c->N2[o3 + N + s], c->N2[o3 + 2 * N + s]};
            for (int i = 0; i < OR_Q; ++i) {
                double fs = post_collision(c, a, i, fa[(size_t)i * N + s], na, ja, u, Na);
                int yy = y + C[i][1];
                if (c->p.walls_y && (yy == 0 || yy == ny - 1)) {
                    double uw = (yy == 0) ? c->p.wall_ux[0] : c->p.wall_ux[1];
                    double cux = (double)C[i][0] * uw;
                    double bb = fs - ((6.0 * weight_of(i)) * na) * cux;
                    foa[(size_t)opposite_of(i) * N + s] = bb;
                } else {
                    long d = neighbour(c, x, y, z, C[i][0], C[i][1], C[i][2]);
                    foa[(size_t)i * N + d] = fs;
                }
            }
        }
    }
}

/* ================================================================ API */
int or_num_species(const or_ctx *c) { return c->M; }

/* f = psi_perp(n0, n0 u0, u) at fluid sites, zero on solid layers. */
void or_init(or_ctx *c, const double *n0, const double *u0, double *f)
{
    const long N = c->N;
    const int M = c->M, nx = c->p.nx, ny = c->p.ny;
    memset(f, 0, sizeof(double) * (size_t)M * OR_Q * (size_t)N);
#pragma omp parallel for schedule(static)
    for (long s = 0; s < N; ++s) {
        int y = (int)((s / nx) % ny);
        if (is_solid(c, y)) continue;
        double nt = 0.0, jt[3] = {0.0, 0.0, 0.0};
        double jj[OR_MAXS][3];
        for (int a = 0; a < M; ++a) {
            double na = n0[(size_t)a * N + s];
            const double ma = c->p.mass[a];
            for (int d = 0; d < 3; ++d) jj[a][d] = na * u0[((size_t)a * 3 + d) * N + s];
            if (a == 0) {
                nt = ma * na; jt[0] = ma * jj[a][0]; jt[1] = ma * jj[a][1]; jt[2] = ma * jj[a][2];
            } else {
                nt = nt + ma * na;
                jt[0] = jt[0] + ma * jj[a][0]; jt[1] = jt[1] + ma * jj[a][1]; jt[2] = jt[2] + ma * jj[a][2];
            }
        }
        double u[3];
        for (int d = 0; d < 3; ++d) u[d] = (nt != 0.0) ? jt[d] / nt : 0.0;
        for (int a = 0; a < M; ++a) {
            double na = n0[(size_t)a * N + s];
            for (int i = 0; i < OR_Q; ++i) {
                /* omega = 1 form of the collision with no field: psi_perp */
                double cx = (double)C[i][0], cy = (double)C[i][1], cz = (double)C[i][2];
                double wE = weight_of(i) * hermite_E(c, a, i, u);
                double m0 = cx - u[0], m1 = cy - u[1], m2 = cz - u[2];
                double v0 = jj[a][0] - na * u[0], v1 = jj[a][1] - na * u[1], v2 = jj[a][2] - na * u[2];
                double dotv = (v0 * m0 + v1 * m1) + v2 * m2;
                f[((size_t)a * OR_Q + i) * N + s] = wE * (na + c->ith[a] * dotv);
            }
        }
    }
}

/* One or more full steps: fin (t) -> fout (t + nsteps).  fin is left intact. */
void or_step(or_ctx *c, const double *fin, double *fout, int nsteps)
{
    size_t nf = (size_t)c->M * OR_Q * (size_t)c->N;
    double *a = (double *)malloc(sizeof(double) * nf);
    memcpy(a, fin, sizeof(double) * nf);
    for (int t = 0; t < nsteps; ++t) {
        moments(c, a);
        contact_values(c);
        gather_one(c);
        gather_two(c);
        collide_stream(c, a, fout);
        memcpy(a, fout, sizeof(double) * nf);
    }
    if (nsteps <= 0) memcpy(fout, a, sizeof(double) * nf);
    free(a);
}

/* External force varying with the lattice row y (the F^a of eq. evolution
 * as a function of y; Sec. 5.2 drives its modulated flow this way):
 * profile [M][3][ny] is added to the uniform fext; NULL removes it. */
void or_set_force_profile(or_ctx *c, const double *profile)
{
    const int M = c->M, ny = c->p.ny;
    free(c->fy);
    c->fy = NULL;
    if (!profile) return;
    c->fy = (double *)malloc(sizeof(double) * 3 * (size_t)M * (size_t)ny);
    for (int a = 0; a < M; ++a)
        for (int d = 0; d < 3; ++d)
            for (int y = 0; y < ny; ++y) {
                size_t i = ((size_t)a * 3 + d) * ny + y;
                c->fy[i] = c->p.fext[a * 3 + d] + profile[i];
            }
}

/* Species densities of f (S1 only), n [M][N]. */
void or_moments(or_ctx *c, const double *f, double *n)
{
    moments(c, f);
    memcpy(n, c->n, sizeof(double) * (size_t)c->M * (size_t)c->N);
}

/* One step with the attractive field supplied by the caller: tail[M][3][N]
 * = sum_b sum_{e in T_ab} w_ab(e) n_b(r + e) for the densities of fin (the
 * same convolution the direct sum evaluates, e.g. computed by FFT). */
void or_step_ext(or_ctx *c, const double *fin, double *fout, const double *tail)
{
    c->tail_ext = tail;
    moments(c, fin);
    contact_values(c);
    gather_one(c);
    gather_two(c);
    collide_stream(c, fin, fout);
    c->tail_ext = NULL;
}

/* Evaluate S1-S4 on f and expose every intermediate field.  Any output
 * pointer may be NULL.  Layouts: n [M][N], j/vh/H/N [M][3][N], u [3][N],
 * g [P][N] (packed upper triangle), parts [5][M][3][N] =
 * (Nmf, Ntail, Next, Dold, Dnew), gam [M][N]. */
void or_fields(or_ctx *c, const double *f, double *n, double *j, double *u, double *g, double *vh,
               double *H, double *Nf, double *parts, double *gam)
{
    size_t N = (size_t)c->N, M = (size_t)c->M;
    moments(c, f);
    contact_values(c);
    gather_one(c);
    gather_two(c);
    if (n) memcpy(n, c->n, sizeof(double) * M * N);
    if (j) memcpy(j, c->j, sizeof(double) * 3 * M * N);
    if (u) memcpy(u, c->u, sizeof(double) * 3 * N);
    if (g) memcpy(g, c->g, sizeof(double) * (size_t)c->P * N);
    if (vh) memcpy(vh, c->vh, sizeof(double) * 3 * M * N);
    if (H) memcpy(H, c->H, sizeof(double) * 3 * M * N);
    if (Nf) memcpy(Nf, c->N2, sizeof(double) * 3 * M * N);
    if (parts) {
        memcpy(parts + 0 * 3 * M * N, c->Nmf, sizeof(double) * 3 * M * N);
        memcpy(parts + 1 * 3 * M * N, c->Ntl, sizeof(double) * 3 * M * N);
        memcpy(parts + 2 * 3 * M * N, c->Nex, sizeof(double) * 3 * M * N);
        memcpy(parts + 3 * 3 * M * N, c->Dold, sizeof(double) * 3 * M * N);
        memcpy(parts + 4 * 3 * M * N, c->Dnew, sizeof(double) * 3 * M * N);
    }
    if (gam) memcpy(gam, c->Gam, sizeof(double) * M * N);
}

/* Collision of a single site of species a (test hook for the moment
 * identities): returns f*_i, i = 0..18, for given f_i, n_a, j_a, u and N_a. */
void or_collide_site(or_ctx *c, int a, const double *fi, double na, const double *ja, const double *u,
                     const double *Na, double *out)
{
    for (int i = 0; i < OR_Q; ++i) out[i] = post_collision(c, a, i, fi[i], na, ja, u, Na);
}

/* Stencil export (test hook).  which: 0 shell(a,b), 1 tail(a,b), 2 ball(a).
 * Returns the half-list length; fills e[3n] and w[3n] (unit vectors for
 * shells and balls, vector weights for tails) when the pointers are given. */
int or_stencil(const or_ctx *c, int which, int a, int b, int *e, double *w)
{
    const or_list *L = which == 0 ? &c->shell[a][b] : which == 1 ? &c->tail[a][b] : &c->ball[a];
    if (which == 1 && !c->has_tail[a][b]) return 0;
    if (e) memcpy(e, L->e, sizeof(int) * 3 * (size_t)L->n);
    if (w) memcpy(w, which == 1 ? L->vec : L->unit, sizeof(double) * 3 * (size_t)L->n);
    return L->n;
}

/* Host constants (test hook): out[0..3] = cm, cg, ck, d for pair (a,b). */
void or_pair_constants(const or_ctx *c, int a, int b, double *out)
{
    out[0] = c->cm[a][b];
    out[1] = c->cg[a][b];
    out[2] = c->ck[a][b];
    out[3] = c->dd[a][b];
}

int or_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

void or_set_threads(int n)
{
#ifdef _OPENMP
    if (n > 0) omp_set_num_threads(n);
#else
    (void)n;
#endif
}
