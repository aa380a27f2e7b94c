"""Pins of the oracle's body-force profile and of the periodically modulated
shear flow of Sec. 5.2 (eq. ushape), driven by a y-periodic body force
(a Kolmogorov flow), and of Taylor dispersion in it (eqs. c99, taylordiff).

- The profile enters the field as the external force n_a F^a(y).
- The steady flow amplitude under F cos(2 pi y / Ly) equals the fixed point
  of the linearised scheme, and the viscosity it implies tends to
  (eta^K + eta^C) / rho of Sec. 4.1 as the wavelength grows.
- The passive-scalar Taylor eigenvalue used as the reference tends to
  eq. (taylordiff) as the axial wavenumber goes to zero.
- A composition mode along x in that flow decays at D_eff q^2 with D_eff the
  passive-scalar value for the measured flow amplitude and the scheme's own
  mutual diffusion coefficient.
"""
import math

import numpy as np
import pytest

import workloads as W
from linear_scheme import LinearScheme, taylor_passive_scalar


def test_force_profile_is_the_external_force(oracle_lib):
    m = W.Mixture(10, 12, 8, sigma=(2.0, 3.0, 2.5), fext=np.array([[1e-4, 0, 0], [0, -2e-5, 0], [0, 0, 3e-5]]))
    n0, u0 = W.random_state(m, [0.012, 0.008, 0.005], rel=0.3, u_amp=0.02, seed=41)
    o = oracle_lib.Oracle(m)
    rng = np.random.default_rng(42)
    prof = rng.uniform(-1e-4, 1e-4, size=(3, 3, m.ny))
    o.set_force_profile(prof)
    f = o.init(n0, u0)
    d = o.fields(f)
    F = m.fext_matrix()[:, :, None] + prof                        # [M][3][ny]
    expect = d["n"][:, None, :, :, :] * F[:, :, None, :, None]
    assert np.array_equal(d["Next"], expect)
    o.set_force_profile(None)
    d2 = o.fields(f)
    assert np.array_equal(d2["Next"], d["n"][:, None] * m.fext_matrix()[:, :, None, None, None])


def kolmogorov(m, F0):
    """Body force F0 cos(2 pi y / ny) along x on every species (equal masses:
    the same acceleration, so no relative velocity is driven)."""
    prof = np.zeros((m.M, 3, m.ny))
    prof[:, 0, :] = F0 * np.cos(2 * math.pi * np.arange(m.ny) / m.ny)[None, :]
    return prof


def _state(sigma, xi, x1=0.5):
    x = np.array([x1, 1 - x1])
    return W.number_density(xi, x, sigma) * x


@pytest.mark.parametrize("sigma,xi,Ly", [((2.0, 3.0), 0.2, 64), ((3.0, 4.5), 0.3, 48)])
def test_kolmogorov_flow_amplitude(oracle_lib, sigma, xi, Ly):
    n0 = _state(sigma, xi)
    m = W.Mixture(1, Ly, 1, sigma=sigma)
    F0 = 1e-6
    o = oracle_lib.Oracle(m)
    o.set_force_profile(kolmogorov(m, F0))
    n, u = W.uniform_state(m, n0)
    lin = LinearScheme(sigma, n0)
    k = 2 * math.pi / Ly
    nu = lin.shear_viscosity(Ly)
    f = o.step(o.init(n, u), int(25 / (nu * k * k)))
    d = o.fields(f)
    jx = d["j"][:, 0, 0, :, 0]                                    # [M][ny]
    y = np.arange(Ly)
    amp = 2.0 / Ly * (jx * np.cos(k * y)[None, :]).sum(1)
    want = lin.transverse_forced(k) * F0                          # symmetric under x <-> y
    np.testing.assert_allclose(amp, want, rtol=1e-6)
    # the implied kinematic viscosity against eta^K + eta^C of Sec. 4.1 (the
    # difference is O((k sigma)^2): 0.2 % at sigma 2-3 over 64 rows, 1.2 % at
    # sigma 3-4.5 over 48)
    nu_flow = F0 / (amp.sum() / n0.sum() * k * k)
    assert abs(nu_flow / lin.paper_viscosity() - 1) < 2e-2, (nu_flow, lin.paper_viscosity())


@pytest.mark.parametrize("sigma,xi,x1", [((2.0, 3.0), 0.2, 0.5), ((3.0, 4.5), 0.3, 0.5), ((2.0, 2.0), 0.05, 0.5),
                                         ((2.0, 4.0), 0.35, 0.9)])
def test_linearised_shear_viscosity_is_eta_k_plus_eta_c(sigma, xi, x1):
    """The shear eigenvalue of the linearised scheme at long wavelength against
    (eta^K + eta^C) / rho (Sec. 4.1), with the lattice shell's fourth moment
    in eta^C and the lattice BGK kinetic part (tau - 1/2) kT."""
    lin = LinearScheme(sigma, _state(sigma, xi, x1))
    assert abs(lin.shear_viscosity(4096) / lin.paper_viscosity() - 1) < 1e-4


def test_passive_scalar_reference_tends_to_eq_taylordiff():
    D, U, Ly = 0.5, 0.05, 40.0
    Pe = U * Ly / (2 * D)
    paper = D * (1 + Pe ** 2 / (2 * math.pi ** 2))
    vals = [taylor_passive_scalar(D, U, Ly, Lx) for Lx in (160, 640, 2560, 10240)]
    err = [abs(v / paper - 1) for v in vals]
    assert err[-1] < 1e-4 and all(a > b for a, b in zip(err, err[1:]))
    assert taylor_passive_scalar(D, 0.0, Ly, 160) == pytest.approx(D, rel=1e-12)


@pytest.mark.slow
def test_taylor_dispersion_of_composition_mode(oracle_lib):
    """Composition mode along x (Sec. 5.2) in the steady modulated flow:
    D_eff from the mode decay against the passive-scalar eigenvalue for the
    measured flow amplitude and the scheme's mutual diffusion coefficient."""
    sigma, xi = (3.0, 4.5), 0.3
    n0 = _state(sigma, xi)
    Lx, Ly = 96, 32
    lin = LinearScheme(sigma, n0)
    k = 2 * math.pi / Ly
    U = 0.06
    F0 = U / lin.transverse_forced(k).sum() * n0.sum()
    m = W.Mixture(Lx, Ly, 1, sigma=sigma)
    o = oracle_lib.Oracle(m)
    o.set_force_profile(kolmogorov(m, F0))
    n, u = W.mode_state(m, n0.sum(), 0.5, 1e-3)
    u[:, 0] = U * np.cos(k * np.arange(Ly))[None, None, :, None]
    f = o.init(n, u)
    D = lin.diffusion(Lx)
    q = 2 * math.pi / Lx
    x = np.arange(Lx)
    ts, amps, us = [], [], []
    steps = 1800
    for t in range(0, steps + 1, 30):
        d = o.fields(f)
        amps.append(abs(np.sum((d["n"][0] - d["n"][1]).mean(axis=(0, 1)) * np.exp(-1j * q * x))))
        ux = d["j"][:, 0].sum(0) / d["n"].sum(0)
        us.append(2.0 / Ly * float((ux.mean(axis=(0, 2)) * np.cos(k * np.arange(Ly))).sum()))
        ts.append(t)
        f = o.step(f, 30)
    ts, amps = np.array(ts), np.array(amps)
    sel = ts >= 300
    D_eff = -np.polyfit(ts[sel], np.log(amps[sel]), 1)[0] / q ** 2
    U_meas = float(np.mean(us[len(us) // 2:]))
    assert abs(U_meas / U - 1) < 1e-2
    want = taylor_passive_scalar(D, U_meas, Ly, Lx)
    assert want / D > 1.25                                         # the flow matters
    assert abs(D_eff / want - 1) < 0.02, (D_eff, want, D)
