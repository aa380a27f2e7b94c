"""Linear response of the lattice scheme around a uniform mixture at rest.

Test infrastructure.  Written from the scheme's definition (the readings of
the paper listed in the design notes) and from the paper's linear estimates,
independently of the oracle and of the GPU library: neither is imported
here, and the stencils and contact values are rebuilt from their
definitions.

A plane wave exp(i k x) on uniform densities n_a0 at rest couples, per
species a, the density and the x momentum density (longitudinal wave) or the
y momentum density alone (transverse wave).  With omega = 1 the
post-collision populations depend only on these moments, so one time step is
exactly a small complex matrix:

  contact values   delta g_ab = sum_c dg_ab/dn_c  B_c(k) delta n_c
                   (B_c the ball average of exp(i k e_x))
  mean field       Sec. 3, eq. (potmeanforce), pair value (g(r) + g(r+e))/2
  attractive field below eq. (potmeanforce), RPA, -dU/dr of -eps (s/r)^6
  friction         the pair form of eqs. (gammaab), (tensorgamma),
                   (viscousforce) at the old velocities, one Jacobi
                   predictor V, then the Crank-Nicolson average (or forward
                   Euler)
  collision        f* = w_i [dn + 3 c_i . (dj + N)]   (omega = 1, linearised
                   orthogonalised equilibrium plus field term, unit masses);
                   with masses m_a (thermal speed^2 theta_a = kT / m_a):
                   f* = w_i h_i [dn + (m_a/kT) c_i.(dj - n du) + 3 c_i.N]
                        + 3 w_i n c_i.du,  h_i = 1 + (9/2)(theta_a - 1/3)(c_i^2 - 1),
                   du = sum_b m_b dj_b / sum_b m_b n_b the barycentric
                   velocity, and the predictor's force over m_a
  streaming        f'(x) = f*(x - c_x)  ->  exp(-i k c_x)

Eigenvalues of that matrix give the decay per step of every mode: composition
diffusion, sound, shear and the relative-velocity (w) modes of Sec. 4.2.
"""
from __future__ import annotations

import math
from typing import Optional, Sequence

import numpy as np

KT = 1.0 / 3.0

# D3Q19 velocities and weights (any order: only sums over them enter)
_C = [(0, 0, 0)] + [(s * (d == 0), s * (d == 1), s * (d == 2)) for d in range(3) for s in (1, -1)]
_C += [(a, b, 0) for a in (1, -1) for b in (1, -1)] + [(a, 0, b) for a in (1, -1) for b in (1, -1)]
_C += [(0, a, b) for a in (1, -1) for b in (1, -1)]
CV = np.array(_C, dtype=float)
WV = np.array([1 / 3] + [1 / 18] * 6 + [1 / 36] * 12)


def offsets(lo2: float, hi2: float, lo_closed: bool, hi_closed: bool) -> np.ndarray:
    """All integer offsets e with lo2 <(=) |e|^2 <(=) hi2."""
    R = int(math.ceil(math.sqrt(hi2))) + 1
    r = np.arange(-R, R + 1)
    e = np.stack(np.meshgrid(r, r, r, indexing="ij"), -1).reshape(-1, 3)
    d = (e ** 2).sum(1).astype(float)
    ok = (d >= lo2) if lo_closed else (d > lo2)
    ok &= (d <= hi2) if hi_closed else (d < hi2)
    return e[ok]


def shell(s: float) -> np.ndarray:
    """Lattice sphere of radius s: (s - 1/2)^2 <= |e|^2 < (s + 1/2)^2."""
    return offsets((s - 0.5) ** 2, (s + 0.5) ** 2, True, False)


def ball(s: float) -> np.ndarray:
    """Smoothing ball of diameter s: |e|^2 <= (s/2)^2, centre included."""
    return offsets(-1.0, (0.5 * s) ** 2, False, True)


def tail(s: float, rc: float) -> np.ndarray:
    """Attractive support s^2 < |e|^2 <= (rc s)^2."""
    return offsets(s * s, (rc * s) ** 2, False, True)


def bmcsl(nbar: Sequence[float], sigma: Sequence[float]) -> np.ndarray:
    """Boublik-Mansoori-Carnahan-Starling-Leland contact values g_ab of the
    packing fractions xi_k = (pi/6) sum_c sigma_c^k nbar_c."""
    sig = np.asarray(sigma, float)
    nb = np.asarray(nbar, float)
    x2 = math.pi / 6 * float(np.sum(nb * sig ** 2))
    x3 = math.pi / 6 * float(np.sum(nb * sig ** 3))
    d = np.outer(sig, sig) / np.add.outer(sig, sig)
    return 1 / (1 - x3) + 3 * d * x2 / (1 - x3) ** 2 + 2 * (d * x2) ** 2 / (1 - x3) ** 3


class LinearScheme:
    """Uniform mixture at rest: diameters sigma_aa, densities n0, attraction
    eps_ab (cutoff rc sigma_ab), scheme "cnj1" or "fe"."""

    def __init__(self, sigma: Sequence[float], n0: Sequence[float], eps: Optional[np.ndarray] = None,
                 rc: float = 2.5, scheme: str = "cnj1", mass: Optional[Sequence[float]] = None):
        self.sig = np.asarray(sigma, float)
        self.n0 = np.asarray(n0, float)
        self.M = len(self.sig)
        self.mass = np.ones(self.M) if mass is None else np.asarray(mass, float)
        self.mu = np.outer(self.mass, self.mass) / np.add.outer(self.mass, self.mass)
        self.rho = float((self.mass * self.n0).sum())
        self.ith = self.mass / KT                       # 1 / theta_a
        self.dth = 4.5 * (KT / self.mass - 1.0 / 3.0)   # weight of the temperature term
        self.eps = np.zeros((self.M, self.M)) if eps is None else np.asarray(eps, float)
        self.rc = rc
        self.scheme = scheme
        M = self.M
        self.sab = 0.5 * np.add.outer(self.sig, self.sig)
        self.shells = [[shell(self.sab[a, b]) for b in range(M)] for a in range(M)]
        self.balls = [ball(s) for s in self.sig]
        self.tails = [[tail(self.sab[a, b], rc) if self.eps[a, b] else None for b in range(M)] for a in range(M)]
        self.g = bmcsl(self.n0, self.sig)
        # dg_ab / dn_c by central differences of the closed form
        self.dg = np.zeros((M, M, M))
        for c in range(M):
            h = 1e-6 * max(self.n0[c], 1e-3)
            up, dn = self.n0.copy(), self.n0.copy()
            up[c] += h
            dn[c] -= h
            self.dg[:, :, c] = (bmcsl(up, self.sig) - bmcsl(dn, self.sig)) / (2 * h)
        # shell weight 4 pi / |S| and kappa = 2 s^2 sqrt(2 mu kT / pi) w_hat
        self.what = np.array([[4 * math.pi / len(self.shells[a][b]) for b in range(M)] for a in range(M)])
        self.kappa = 2 * self.sab ** 2 * np.sqrt(2 * self.mu * KT / math.pi) * self.what

    # ------------------------------------------------------------ stencil sums
    def _unit(self, e):
        return e / np.sqrt((e ** 2).sum(1))[:, None]

    def ball_factor(self, c: int, k: float) -> float:
        return float(np.cos(k * self.balls[c][:, 0]).mean())

    def shell_sin(self, a, b, k):
        """sum_e e_hat_x sin(k e_x) over the full shell S_ab."""
        e = self.shells[a][b]
        return float((self._unit(e)[:, 0] * np.sin(k * e[:, 0])).sum())

    def shell_cos2(self, a, b, k, comp=0):
        """sum_e e_hat_comp^2 cos(k e_x) over the full shell S_ab."""
        e = self.shells[a][b]
        return float((self._unit(e)[:, comp] ** 2 * np.cos(k * e[:, 0])).sum())

    def tail_sin(self, a, b, k):
        """sum_e (6 eps s^6 / |e|^7) e_hat_x sin(k e_x) over T_ab."""
        e = self.tails[a][b]
        if e is None:
            return 0.0
        r = np.sqrt((e ** 2).sum(1))
        s6 = self.sab[a, b] ** 6
        return float((6 * self.eps[a, b] * s6 / r ** 7 * (e[:, 0] / r) * np.sin(k * e[:, 0])).sum())

    # ------------------------------------------------------- force responses
    def mean_field(self, k: float) -> np.ndarray:
        """K[a, b]: per-particle hard-core mean force of species a, x component,
        for delta n_b cos(k x):  F_a(x) = K[a, b] delta n_b sin(k x)."""
        M = self.M
        K = np.zeros((M, M))
        for b in range(M):           # perturbed species
            for p in range(M):       # partner of the shell sum
                for a in range(M):
                    dgab = sum(self.dg[a, p, c] * self.ball_factor(c, k) * (c == b) for c in range(M))
                    amp = self.g[a, p] * (p == b) + 0.5 * self.n0[p] * dgab
                    K[a, b] += KT * self.sab[a, p] ** 2 * self.what[a, p] * self.shell_sin(a, p, k) * amp
        return K

    def paper_mean_field_limit(self, lattice_radius: bool = True) -> np.ndarray:
        """Small-q limit of Sec. 3, eq. (diciotto), hard-core part:
        F_a = -i q exp(i q r) sum_b dn_b kT (4 pi / 3) (s_ab^3 g_ab +
        1/2 sum_c n_c s_ac^3 dg_ac/dn_b), i.e. for dn_b cos(q x) the x force
        q dn_b sin(q x) times the returned matrix.  With lattice_radius the
        continuum sphere's sigma^3 = sigma^2 x sigma becomes sigma^2 x R_ab,
        R_ab = sum_e |e| e_hat_x^2 / sum_e e_hat_x^2 of the lattice shell
        (the radius its dipole moment sees)."""
        M = self.M
        R = np.zeros((M, M))
        for a in range(M):
            for b in range(M):
                e = self.shells[a][b]
                r = np.sqrt((e ** 2).sum(1))
                u = self._unit(e)[:, 0] ** 2
                R[a, b] = (r * u).sum() / u.sum() if lattice_radius else self.sab[a, b]
        s3 = self.sab ** 2 * R
        K = np.zeros((M, M))
        for a in range(M):
            for b in range(M):
                K[a, b] = KT * 4 * math.pi / 3 * (s3[a, b] * self.g[a, b] + 0.5 * sum(
                    self.n0[c] * s3[a, c] * self.dg[a, c, b] for c in range(M)))
        return K

    def viscous(self, k: float, comp: int) -> np.ndarray:
        """Per-particle friction force of species a (component comp) for equal
        species velocities u cos(k x) e_comp (eq. viscousforce form):
        F_a = V[a] u cos(k x)."""
        M = self.M
        V = np.zeros(M)
        for a in range(M):
            for b in range(M):
                e = self.shells[a][b]
                s = (self._unit(e)[:, comp] ** 2 * (np.cos(k * e[:, 0]) - 1.0)).sum()
                V[a] += self.kappa[a, b] * self.g[a, b] * self.n0[b] * s
        return V

    def paper_viscous_limit(self, comp: int) -> np.ndarray:
        """Eqs. (viscousforce1) and (viscousforce2): F = -c q^2 u sum_b s^4 n_b g
        sqrt(2 mu kT / pi), c = 4 pi / 15 (perpendicular) or 4 pi / 5 (parallel);
        returns the coefficient of -q^2 u."""
        c = 4 * math.pi / 5 if comp == 0 else 4 * math.pi / 15
        return np.array([c * sum(self.sab[a, b] ** 4 * self.n0[b] * self.g[a, b] * math.sqrt(2 * self.mu[a, b] * KT / math.pi)
                                 for b in range(self.M)) for a in range(self.M)])

    # ------------------------------------------------------------ one step
    def _forces(self, k, dn, dj, comp, fext=0.0):
        """Force density N_a (component comp) of the scheme for the moment
        amplitudes dn, dj (complex, exp(i k x) convention) and a body force
        of amplitude fext per particle on every species."""
        M = self.M
        Nc = self.n0 * fext + 0j
        if comp == 0:
            for a in range(M):
                for p in range(M):
                    dgap = sum(self.dg[a, p, c] * self.ball_factor(c, k) * dn[c] for c in range(M))
                    Nc[a] += -KT * self.n0[a] * self.sab[a, p] ** 2 * self.what[a, p] * 1j * \
                        self.shell_sin(a, p, k) * (self.g[a, p] * dn[p] + 0.5 * self.n0[p] * dgap)
                    Nc[a] += self.n0[a] * 1j * self.tail_sin(a, p, k) * dn[p]
        Sn = np.array([[len(self.shells[a][b]) / 3.0 for b in range(M)] for a in range(M)])
        C2 = np.array([[self.shell_cos2(a, b, k, comp) for b in range(M)] for a in range(M)])
        kg = self.kappa * self.g

        def pair_form_old(j):
            return np.array([sum(kg[a, b] * (self.n0[a] * C2[a, b] * j[b] - self.n0[b] * Sn[a, b] * j[a])
                                 for b in range(M)) for a in range(M)])

        def pair_form_v(v):
            return np.array([self.n0[a] * sum(kg[a, b] * self.n0[b] * (C2[a, b] * v[b] - Sn[a, b] * v[a])
                                              for b in range(M)) for a in range(M)])

        Dold = pair_form_old(dj)
        if self.scheme == "fe":
            return Nc + Dold
        Gam = np.array([sum(kg[a, b] * self.n0[b] * Sn[a, b] for b in range(M)) for a in range(M)])
        hg = 0.5 * Gam / self.mass
        V = (dj + (Nc + Dold) / self.mass + hg * dj) / (self.n0 * (1 + hg))
        return Nc + 0.5 * Dold + 0.5 * pair_form_v(V)

    def _lattice_sums(self, k, comp):
        """sum_i w_i ph_i c^p (and with the temperature factor c^2 - 1) for
        the streaming phase ph_i = exp(-i k c_x) and c = c_comp."""
        ph = np.exp(-1j * k * CV[:, 0])
        cc = CV[:, comp]
        t = (CV ** 2).sum(1) - 1.0
        S = [(WV * cc ** p * ph).sum() for p in range(3)]
        T = [(WV * t * cc ** p * ph).sum() for p in range(3)]
        return S, T

    def _collide_stream(self, k, comp, dn, dj, N):
        """Moments (dn', dj'_comp) after the linearised collision and streaming
        of the wave exp(i k x), given the force densities N (component comp)."""
        (S0, S1, S2), (T0, T1, T2) = self._lattice_sums(k, comp)
        du = (self.mass * dj).sum() / self.rho
        X = self.ith * (dj - self.n0 * du) + 3 * N           # per species
        h = self.dth
        dn_new = (S0 + h * T0) * dn + (S1 + h * T1) * X + 3 * S1 * self.n0 * du
        dj_new = (S1 + h * T1) * dn + (S2 + h * T2) * X + 3 * S2 * self.n0 * du
        return dn_new, dj_new

    def longitudinal(self, k: float) -> np.ndarray:
        """One step on (dn_0..dn_{M-1}, dj_0,x..dj_{M-1},x)."""
        M = self.M
        T = np.zeros((2 * M, 2 * M), complex)
        for col in range(2 * M):
            v = np.zeros(2 * M, complex)
            v[col] = 1.0
            dn, dj = v[:M], v[M:]
            T[:M, col], T[M:, col] = self._collide_stream(k, 0, dn, dj, self._forces(k, dn, dj, 0))
        return T

    def transverse(self, k: float) -> np.ndarray:
        """One step on (dj_0,y .. dj_{M-1},y) for a wave along x."""
        M = self.M
        zero = np.zeros(M, complex)
        T = np.zeros((M, M), complex)
        for col in range(M):
            dj = np.zeros(M, complex)
            dj[col] = 1.0
            T[:, col] = self._collide_stream(k, 1, zero, dj, self._forces(k, zero, dj, 1))[1]
        return T

    def transverse_forced(self, k: float) -> np.ndarray:
        """Steady transverse momentum amplitudes dj_a,y under a body force
        cos(k x) e_y of unit amplitude per particle on every species (the
        Kolmogorov flow that drives the modulated shear of Sec. 5.2): the
        fixed point of j' = T j + f."""
        M = self.M
        zero = np.zeros(M, complex)
        f = self._collide_stream(k, 1, zero, zero, self._forces(k, zero, zero, 1, fext=1.0))[1]
        return np.linalg.solve(np.eye(M) - self.transverse(k), f).real

    def shear_viscosity(self, L: int) -> float:
        """Kinematic viscosity nu of the shear mode (the slowest transverse
        eigenvalue, decay exp(-nu k^2 t) of eq. dd3) at k = 2 pi / L."""
        k = 2 * math.pi / L
        lam = np.linalg.eigvals(self.transverse(k))
        return float(-math.log(np.abs(lam).max()) / k ** 2)

    def paper_viscosity(self, tau: float = 1.0, lattice: bool = True) -> float:
        """nu = (eta^K + eta^C) / rho (Sec. 4.1): eta^C = (4/15) sum_ab
        sqrt(2 pi mu kT) s^4 g n_a n_b, the sphere's s^2 (4 pi / 15) replaced
        by the lattice shell's fourth moment when `lattice`; eta^K / rho is
        the lattice BGK value (tau - 1/2) kT (the paper's continuum kT tau
        carries the -1/2 of the discrete streaming)."""
        eta = 0.0
        for a in range(self.M):
            for b in range(self.M):
                s = self.sab[a, b]
                if lattice:
                    e = self.shells[a][b]
                    r2 = (e ** 2).sum(1)
                    m4 = self.what[a, b] * (r2 * e[:, 0] ** 2 * e[:, 1] ** 2 / r2 ** 2).sum()
                else:
                    m4 = s * s * 4 * math.pi / 15
                # (4/15) sqrt(2 pi mu kT) s^4 = 2 s^2 sqrt(2 mu kT / pi) (1/2) s^2 (4 pi / 15)
                eta += 2 * s * s * math.sqrt(2 * self.mu[a, b] * KT / math.pi) * 0.5 * m4 * self.g[a, b] * self.n0[a] * self.n0[b]
        return (tau - 0.5) * KT + eta / self.n0.sum()

    # ------------------------------------------------------------- modes
    def longitudinal_modes(self, L: int) -> np.ndarray:
        """Eigenvalues of one longitudinal step at k = 2 pi / L."""
        return np.linalg.eigvals(self.longitudinal(2 * math.pi / L))

    def diffusion(self, L: int) -> float:
        """D of the slowest real (non-oscillating) longitudinal mode at k = 2 pi / L."""
        k = 2 * math.pi / L
        lam = np.linalg.eigvals(self.longitudinal(k))
        real = lam[np.abs(lam.imag) < 1e-12].real
        return float(-math.log(real.max()) / k ** 2)


def taylor_passive_scalar(D: float, U: float, Ly: float, Lx: float, nmodes: int = 64) -> float:
    """Effective axial diffusion of a passive scalar mode exp(i q x), q = 2 pi /
    Lx, in the flow u_x(y) = U cos(2 pi y / Ly) with molecular diffusion D:
    -lambda / q^2 for the slowest eigenvalue lambda of the advection-diffusion
    operator on the y Fourier modes exp(i m k y), k = 2 pi / Ly (the flow
    couples m to m +- 1 with i q U / 2).  As q -> 0 it tends to Sec. 5.2,
    eq. (taylordiff): D (1 + Pe^2 / (2 pi^2)), Pe = U Ly / (2 D)."""
    q, k = 2 * math.pi / Lx, 2 * math.pi / Ly
    m = np.arange(-nmodes, nmodes + 1)
    A = np.diag(-D * (q * q + (m * k) ** 2)).astype(complex)
    off = -0.5j * q * U
    for i in range(len(m) - 1):
        A[i, i + 1] = off
        A[i + 1, i] = off
    lam = np.linalg.eigvals(A)
    return float(-lam.real.max() / (q * q))


def hydrodynamics(lin: LinearScheme, tau: float = 1.0) -> dict:
    """The hydrodynamic coefficients of Sec. 4.2 for a binary at rest, from
    the long-wavelength forces of Sec. 3 (eq. diciotto with the lattice
    shell's radius; the attractive part from the lattice moment of the
    force kernel) and the viscosities of Sec. 4.1 (lattice fourth moments):

      chemical potentials  d mu_a / d n_b = kT delta_ab / n_a + K_ab
      pressure             d P / d n_b    = kT + sum_a n_a K_ab
      sound speed          c_s^2 = (dP/drho)_c                        (eq. cc2)
      friction             gamma = gamma^AB + gamma^BA (unit masses,
                           eq. gammasymmetrized1)
      diffusion            D_P = c (1 - c) [(dmu_D/dc)_rho - (dmu_D/drho)_c
                           (dP/dc)_rho / (dP/drho)_c] / gamma, the diffusive
                           root of the determinant of Sec. 4.2 to order q^2
                           (D_0 of the paper when (dP/dc)_rho = 0)
      sound damping        Gamma = [nu_l + c (1 - c) (dmu_D/drho)_c
                           (dP/dc)_rho / (gamma (dP/drho)_c)] / 2, the acoustic
                           root to order q^2 (eq. damping, with the factor
                           c (1 - c) / gamma its dimensions require), nu_l =
                           (4/3 eta + eta_b) / rho: kinetic part 2 (tau - 1/2) kT
                           (lattice BGK: eta_b^K = 2/3 eta^K), collisional part
                           from the parallel lattice moment (eta_b^C = 5/3 eta^C
                           for the sphere)."""
    assert lin.M == 2
    n0 = lin.n0
    K = lin.paper_mean_field_limit(lattice_radius=True)
    for a in range(2):
        for b in range(2):
            e = lin.tails[a][b]
            if e is None:
                continue
            r = np.sqrt((e ** 2).sum(1))
            K[a, b] -= (6 * lin.eps[a, b] * lin.sab[a, b] ** 6 / r ** 6 * (e[:, 0] / r) ** 2).sum()
    dmu = np.array([[KT * (a == b) / n0[a] + K[a, b] for b in range(2)] for a in range(2)])
    dP = np.array([KT + sum(n0[a] * K[a, b] for a in range(2)) for b in range(2)])
    rho = n0.sum()
    c = n0[0] / rho

    def d_rho(v):
        return c * v[0] + (1 - c) * v[1]

    def d_c(v):
        return rho * (v[0] - v[1])

    muD = dmu[0] - dmu[1]
    gam = sum(8 / 3 * math.sqrt(2 * math.pi * lin.mu[0, 1] * KT) * lin.g[0, 1] * lin.sab[0, 1] ** 2 * n0[b] for b in range(2))
    coupling = d_rho(muD) * d_c(dP) / d_rho(dP)
    nul_c = 0.0
    for a in range(2):
        for b in range(2):
            e = lin.shells[a][b]
            r2 = (e ** 2).sum(1)
            m4 = lin.what[a, b] * (r2 * (e[:, 0] ** 2 / r2) ** 2).sum()
            nul_c += n0[a] * 2 * lin.sab[a, b] ** 2 * math.sqrt(2 * lin.mu[a, b] * KT / math.pi) * lin.g[a, b] * n0[b] * 0.5 * m4
    nul = 2 * (tau - 0.5) * KT + nul_c / rho
    return {"cs": math.sqrt(d_rho(dP)), "gamma": gam, "D_P": c * (1 - c) * (d_c(muD) - coupling) / gam,
            "D_0": c * (1 - c) * d_c(muD) / gam, "Gamma": 0.5 * (nul + c * (1 - c) * coupling / gam),
            "nu": lin.paper_viscosity(tau), "Delta": c * (1 - c) * d_c(muD)}
