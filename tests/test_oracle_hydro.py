"""Hydrodynamic modes of the scheme against Sec. 4.2 (eqs. cc1-cc4, dd1-dd6,
damping) and the diffusive/oscillatory crossover of Sec. 5.1 (eqs.
gammasymmetrized, critical).

The references are the linearised scheme (linear_scheme.py, itself pinned
to the oracle's step column by column in test_oracle_linear_response.py)
and the paper's closed forms built from the long-wavelength forces of
Sec. 3 (hydrodynamics() in linear_scheme.py):

- sound: c_s = sqrt((dP/drho)_c), damping Gamma of the acoustic root;
- shear: nu = (eta^K + eta^C) / rho (eq. dd3; pinned in test_oracle_taylor.py);
- transverse w: decay at the friction rate gamma (eq. dd5), which one
  Crank-Nicolson step turns into the factor (1 - gamma/2) / (1 + gamma/2) in
  the hydrodynamic limit;
- composition diffusion: the diffusive root of the determinant, D_P (the
  paper's D_0 = c (1 - c) (dmu_D/dc) / gamma when (dP/dc)_rho = 0);
- crossover: composition fluctuations decay without oscillating below
  q_c = sqrt(gamma^2 / (4 Delta)), at Kn = lambda_mf / L_c = (4/3) (2 pi)^-3/2
  in the dilute limit; an oracle run on either side shows both behaviours.
"""
import math

import numpy as np
import pytest

import workloads as W
from linear_scheme import KT, LinearScheme, hydrodynamics

STATES = [  # (sigma, packing, x1, eps)
    ((2.0, 2.0), 0.05, 0.5, None),
    ((2.0, 3.0), 0.2, 0.5, None),            # step-binary / closure physics
    ((3.0, 4.5), 0.3, 0.5, 0.5 * KT),        # bulk-diffusion physics (tail on)
    ((2.0, 4.0), 0.1, 0.3, None),
    ((3.0, 3.0), 0.2, 0.5, None),
]


def _lin(sigma, xi, x1, eps):
    x = np.array([x1, 1 - x1])
    n0 = W.number_density(xi, x, sigma) * x
    return LinearScheme(sigma, n0, eps=None if eps is None else np.full((2, 2), eps))


def _roots(lin, L):
    k = 2 * math.pi / L
    return np.log(np.linalg.eigvals(lin.longitudinal(k))), k


@pytest.mark.parametrize("state", STATES)
def test_sound_speed_is_thermodynamic(state):
    lin = _lin(*state)
    z, k = _roots(lin, 16384)
    sound = z[np.abs(z.imag) > 1e-9]
    assert len(sound) == 2
    h = hydrodynamics(lin)
    np.testing.assert_allclose(np.abs(sound.imag) / k, h["cs"], rtol=2e-6)


@pytest.mark.parametrize("state", STATES)
def test_sound_damping(state):
    lin = _lin(*state)
    z, k = _roots(lin, 16384)
    sound = z[np.abs(z.imag) > 1e-9]
    h = hydrodynamics(lin)
    equal = state[0][0] == state[0][1]
    # exact for equal diameters ((dP/dc)_rho = 0); the interdiffusion term
    # to O(q^2) leaves 0.5 % for unequal ones
    np.testing.assert_allclose(-sound.real / k ** 2, h["Gamma"], rtol=1e-6 if equal else 6e-3)


@pytest.mark.parametrize("state", STATES)
def test_composition_diffusion_is_the_hydrodynamic_root(state):
    lin = _lin(*state)
    h = hydrodynamics(lin)
    D = lin.diffusion(16384)
    equal_or_dilute = state[0][0] == state[0][1] or state[1] <= 0.1
    assert abs(D / h["D_P"] - 1) < (1e-4 if equal_or_dilute else 6e-3), (D, h["D_P"])
    if state[0][0] == state[0][1]:
        assert abs(h["D_P"] / h["D_0"] - 1) < 1e-12       # (dP/dc)_rho = 0 for equal diameters


@pytest.mark.parametrize("state", STATES[:3])
def test_transverse_w_decays_at_the_friction_rate(state):
    """w = u_A - u_B transverse to a long wave decays by the Crank-Nicolson
    factor of the friction rate gamma (eq. dd5)."""
    lin = _lin(*state)
    h = hydrodynamics(lin)
    lam = np.linalg.eigvals(lin.transverse(2 * math.pi / 16384)).real
    lw = lam.min()
    gam = h["gamma"]
    # one Jacobi sweep of Crank-Nicolson: the uniform counter-flow factor
    n0 = lin.n0
    G = [[8 / 3 * math.sqrt(2 * math.pi * 0.5 * KT) * lin.g[a, b] * n0[b] * lin.sab[a, b] ** 2 for b in range(2)]
         for a in range(2)]
    Gam = [G[a][0] + G[a][1] for a in range(2)]
    cnj1 = 1 - 0.5 * gam * (2 - G[0][1] / (1 + 0.5 * Gam[0]) - G[1][0] / (1 + 0.5 * Gam[1]))
    assert abs(lw - cnj1) < 1e-7
    # the rate per step against the paper's gamma: Crank-Nicolson differs at O(gamma^3)
    cn = (1 - gam / 2) / (1 + gam / 2)
    assert abs(-math.log(lw) / gam - 1) < 0.12 * gam ** 2 + 1e-3, (-math.log(lw), gam, cn)


@pytest.mark.parametrize("sigma,xi", [((2.0, 2.0), 0.02), ((3.0, 3.0), 0.02), ((2.0, 2.0), 0.05)])
def test_critical_wavenumber(sigma, xi):
    """The composition-sector roots turn complex (oscillating decay) above
    q_c = gamma / (2 sqrt(Delta)) (Sec. 5.1); dilute: Delta = kT / m and
    gamma = (8/3) sqrt(kT / (2 pi m)) / lambda_mf, so Kn = lambda_mf / L_c =
    (4/3) (2 pi)^-3/2."""
    lin = _lin(sigma, xi, 0.5, None)
    h = hydrodynamics(lin)
    qc = h["gamma"] / (2 * math.sqrt(h["Delta"]))
    n, s, g = lin.n0.sum(), sigma[0], lin.g[0, 0]
    lmf = 1 / (math.sqrt(2) * math.pi * g * s * s * n)
    gam_paper = 8 / 3 * math.sqrt(KT / (2 * math.pi)) / lmf
    assert abs(gam_paper / h["gamma"] - 1) < 1e-12
    assert abs(h["Delta"] / KT - 1) < 0.05
    assert abs(lmf / (2 * math.pi / (gam_paper / (2 * math.sqrt(KT)))) - 4 / 3 * (2 * math.pi) ** -1.5) < 1e-12

    def oscillates(k):
        # the sound pair is always complex; above q_c the composition pair is too
        z = np.log(np.linalg.eigvals(lin.longitudinal(k)))
        return int(np.sum(np.abs(z.imag) > 1e-10)) == 4

    lo, hi = 0.5 * qc, 2.0 * qc
    assert not oscillates(lo) and oscillates(hi)
    for _ in range(40):
        mid = 0.5 * (lo + hi)
        lo, hi = (mid, hi) if not oscillates(mid) else (lo, mid)
    assert abs(lo / qc - 1) < 0.05, (lo, qc)


def test_oracle_composition_mode_oscillates_above_qc(oracle_lib):
    """A dilute equal-diameter binary (packing 0.02, L_c about 132 cells):
    the composition mode of wavelength 96 overshoots zero while decaying;
    the one of wavelength 192 decays monotonically."""
    sigma, xi = (2.0, 2.0), 0.02
    n = W.number_density(xi, (0.5, 0.5), sigma)
    lin = _lin(sigma, xi, 0.5, None)
    h = hydrodynamics(lin)
    Lc = 2 * math.pi / (h["gamma"] / (2 * math.sqrt(h["Delta"])))
    assert 96 < Lc < 192
    for L, osc in ((96, True), (192, False)):
        m = W.Mixture(L, 1, 1, sigma=sigma)
        o = oracle_lib.Oracle(m)
        f = o.init(*W.mode_state(m, n, 0.5, 1e-3))
        x = np.arange(L)
        proj = []
        for _ in range(80):
            d = o.densities(f)
            proj.append(float(np.sum((d[0] - d[1])[0, 0] * np.sin(2 * math.pi * x / L))))
            f = o.step(f, 5)
        proj = np.array(proj)
        assert (np.any(proj < 0)) == osc, (L, proj[:20])
