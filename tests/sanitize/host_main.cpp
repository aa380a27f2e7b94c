// Host-only parts of libmlb (stencil tables, pair constants, the linear
// stability radius) built with AddressSanitizer and UndefinedBehaviorSanitizer
// and run over the parameter sets the workloads use: every table of every
// diameter in the workloads' range, and the stability radius of binary and
// ternary states under both time schemes, with and without tails.
#include <cmath>
#include <cstdio>
#include <cstring>

#include "../../paper_1105_3634_amd/csrc/mlb_internal.h"

static mlb_params make(int M, const double *sigma, int scheme, double tau, double eps)
{
    mlb_params p;
    std::memset(&p, 0, sizeof p);
    p.nx = p.ny = p.nz = 32;
    p.nspecies = M;
    p.precision = 64;
    p.scheme = scheme;
    p.tau = tau;
    p.kT = 1.0 / 3.0;
    p.rc_factor = 2.5;
    for (int a = 0; a < M; ++a) {
        p.mass[a] = 1.0;
        p.sigma[a] = sigma[a];
        for (int b = 0; b < M; ++b) p.eps[a * MLB_MAX_SPECIES + b] = eps;
    }
    return p;
}

int main()
{
    long total = 0;
    for (double s = 1.0; s <= 9.0; s += 0.25) {
        for (int kind = mlb::kShell; kind <= mlb::kTail; ++kind) {
            mlb::HostStencil h = mlb::build_stencil(kind, s, 2.5);
            total += (long)h.e.size() + h.full;
            for (double v : h.v)
                if (!std::isfinite(v)) return 2;
        }
        mlb::PairConst c = mlb::pair_constants(s, 0.5 * s + 1.0, 1.0 / 3.0, 100, 0.7, 2.0);
        if (!std::isfinite(c.cm)) return 3;
    }
    const double s2[2] = {2.0, 3.0}, s3[3] = {2.0, 3.0, 4.0};
    const double n2[2] = {0.02, 0.015}, n3[3] = {0.01, 0.008, 0.004};
    for (int scheme = 0; scheme <= 1; ++scheme)
        for (double eps : {0.0, 0.1}) {
            mlb_params p = make(2, s2, scheme, scheme ? 0.8 : 1.0, eps);
            p.mass[0] = 0.7, p.mass[1] = 2.0;
            const double r2 = mlb::stability_radius(&p, n2, 4);
            p = make(3, s3, scheme, 1.0, eps);
            const double r3 = mlb::stability_radius(&p, n3, 4);
            if (!(r2 > 0.0) || !(r3 > 0.0)) return 4;
            std::printf("scheme %d eps %.1f: radius %.6f (binary) %.6f (ternary)\n", scheme, eps, r2, r3);
        }
    std::printf("stencil entries %ld\nhost checks done\n", total);
    return 0;
}
