// Host-side construction of the lattice stencils and pair constants.
//
// Shell S(s):  lattice offsets e with (s - 1/2)^2 <= |e|^2 < (s + 1/2)^2, the
//   discrete unit sphere of radius sigma_ab over which the surface integrals
//   of eqs. (potmeanforce), (tensorgamma) and (viscousforce) run, each point
//   weighted by w_hat = 4 pi / |S|.
// Ball B(s):   |e|^2 <= (s/2)^2, the smoothing volume of the packing
//   fractions that enter the contact value g_ab (Sec. 2 leaves the smoothing
//   procedure open).
// Tail T(s):   s^2 < |e|^2 <= (rc s)^2, the support of the attractive field
//   (RPA, below eq. potmeanforce), weight -dU/dr e_hat = 6 eps s^6 / r^7 e_hat.
// Each set is stored as its half with a positive first non-zero component,
// ordered by (|e|^2, ex, ey, ez); the kernels combine each +e/-e pair.
#include <algorithm>
#include <cmath>
#include <tuple>

#include "mlb_internal.h"

namespace mlb {

HostStencil build_stencil(int kind, double s, double rc)
{
    double lo = 0.0, hi = 0.0;
    if (kind == kShell) {
        lo = (s - 0.5) * (s - 0.5);
        hi = (s + 0.5) * (s + 0.5);
    } else if (kind == kBall) {
        hi = (0.5 * s) * (0.5 * s);
    } else {
        lo = s * s;
        hi = (rc * s) * (rc * s);
    }
    const int R = (int)std::ceil(std::sqrt(hi)) + 1;
    std::vector<std::tuple<int, int, int, int>> keys;  // (r2, ex, ey, ez)
    for (int ex = -R; ex <= R; ++ex)
        for (int ey = -R; ey <= R; ++ey)
            for (int ez = -R; ez <= R; ++ez) {
                const bool positive = ex > 0 || (ex == 0 && (ey > 0 || (ey == 0 && ez > 0)));
                if (!positive) continue;
                const int r2 = ex * ex + ey * ey + ez * ez;
                const double d = (double)r2;
                bool in;
                if (kind == kShell) in = d >= lo && d < hi;
                else if (kind == kBall) in = d <= hi;
                else in = d > lo && d <= hi;
                if (in) keys.emplace_back(r2, ex, ey, ez);
            }
    std::sort(keys.begin(), keys.end());
    HostStencil st;
    st.full = 2 * (int)keys.size() + (kind == kBall ? 1 : 0);
    for (auto &k : keys) {
        const int r2 = std::get<0>(k), ex = std::get<1>(k), ey = std::get<2>(k), ez = std::get<3>(k);
        st.e.push_back(pack_offset(ex, ey, ez));
        const double len = std::sqrt((double)r2);
        st.v.push_back((double)ex / len);
        st.v.push_back((double)ey / len);
        st.v.push_back((double)ez / len);
        st.max_abs[0] = std::max(st.max_abs[0], std::abs(ex));
        st.max_abs[1] = std::max(st.max_abs[1], std::abs(ey));
        st.max_abs[2] = std::max(st.max_abs[2], std::abs(ez));
    }
    return st;
}

// Pair constants for unit masses (reduced mass 1/2):
//   w_hat = 4 pi / |S_ab|
//   kappa = 2 sigma_ab^2 sqrt(2 mu kT / pi) w_hat          eq. (tensorgamma)
//   cm    = -kT sigma_ab^2 w_hat / 2     (mean field, eq. potmeanforce; the
//                                          1/2 is that of G = (g(r)+g(r'))/2)
//   cg    = kappa / 6                    (trace/3 of the friction tensor, x 1/2)
//   ck    = kappa / 2                    (pair form, x 1/2 of G)
//   dd    = s_a s_b / (s_a + s_b)        (BMCSL contact-value coefficient)
PairConst pair_constants(double sa, double sb, double kT, int shell_full, double ma, double mb)
{
    const double sab = 0.5 * (sa + sb);
    const double mu = (ma * mb) / (ma + mb);   // reduced mass of the pair (below eq. viscousforce)
    const double what = (4.0 * M_PI) / (double)shell_full;
    const double kap = ((2.0 * (sab * sab)) * std::sqrt((2.0 * mu * kT) / M_PI)) * what;
    PairConst c;
    c.cm = ((-0.5 * kT) * (sab * sab)) * what;
    c.cg = kap / 6.0;
    c.ck = 0.5 * kap;
    c.dd = (sa * sb) / (sa + sb);
    return c;
}

}  // namespace mlb
