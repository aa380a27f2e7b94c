/* The float64 oracle built with AddressSanitizer and
 * UndefinedBehaviorSanitizer (one translation unit with its source) and run
 * on small cases of every geometry and option it has: a periodic binary
 * with tails, a ternary between moving walls with tails and a body-force
 * profile, the forward-Euler scheme, a single species. */
#include <math.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include "../../oracle/mlb_oracle.c"

static int run(const char *name, or_params p, int with_profile, int steps)
{
    const int M = p.M, N = p.nx * p.ny * p.nz;
    double *n0 = calloc((size_t)M * N, sizeof(double));
    double *u0 = calloc((size_t)M * 3 * N, sizeof(double));
    double *f = calloc((size_t)M * OR_Q * N, sizeof(double));
    double *g = calloc((size_t)M * OR_Q * N, sizeof(double));
    double *n = calloc((size_t)M * N, sizeof(double));
    for (int a = 0; a < M; ++a)
        for (int r = 0; r < N; ++r) {
            const int x = r % p.nx;
            n0[(size_t)a * N + r] = 0.01 * (1.0 + 0.1 * sin(2.0 * M_PI * (x + a) / p.nx));
            u0[((size_t)a * 3) * N + r] = 0.01 * cos(2.0 * M_PI * x / p.nx);
        }
    or_ctx *c = or_create(&p);
    if (!c) {
        printf("%s: or_create failed\n", name);
        return 1;
    }
    if (with_profile) {
        double *prof = calloc((size_t)M * 3 * p.ny, sizeof(double));
        for (int y = 0; y < p.ny; ++y) prof[y] = 1e-5 * cos(2.0 * M_PI * y / p.ny);
        or_set_force_profile(c, prof);
        free(prof);
    }
    or_init(c, n0, u0, f);
    or_step(c, f, g, steps);
    or_moments(c, g, n);
    double mass = 0.0;
    for (size_t i = 0; i < (size_t)M * N; ++i) mass += n[i];
    or_destroy(c);
    const int ok = isfinite(mass) && mass > 0.0;
    printf("%s: %d steps, mass %.12f %s\n", name, steps, mass, ok ? "ok" : "NOT FINITE");
    free(n0), free(u0), free(f), free(g), free(n);
    return ok ? 0 : 1;
}

static or_params base(int nx, int ny, int nz, int M)
{
    or_params p;
    memset(&p, 0, sizeof p);
    p.nx = nx, p.ny = ny, p.nz = nz, p.M = M;
    p.tau = 1.0;
    p.kT = 1.0 / 3.0;
    p.rc_factor = 2.5;
    for (int a = 0; a < M; ++a) {
        p.sigma[a] = 2.0 + a;
        p.mass[a] = 1.0;
    }
    return p;
}

int main(void)
{
    int bad = 0;
    or_params p = base(12, 10, 9, 2);
    for (int i = 0; i < 4; ++i) p.eps[i] = 0.1;
    bad |= run("periodic binary with tails", p, 0, 4);
    p = base(12, 14, 6, 3);
    for (int i = 0; i < 9; ++i) p.eps[i] = 0.1;
    p.walls_y = 1;
    p.wall_ux[0] = -0.02, p.wall_ux[1] = 0.02;
    p.mass[0] = 0.7, p.mass[1] = 1.0, p.mass[2] = 2.5;
    bad |= run("ternary between moving walls, tails, force profile, unequal masses", p, 1, 4);
    p = base(10, 10, 10, 2);
    p.scheme = 1, p.tau = 0.8;
    bad |= run("forward Euler", p, 0, 4);
    p = base(9, 9, 9, 1);
    bad |= run("single species", p, 0, 4);
    printf("oracle checks done\n");
    return bad;
}
