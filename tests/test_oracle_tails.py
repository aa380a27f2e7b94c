"""Attractive tails and the mutual diffusion coefficient (Sec. 4.1, eq.
berthelot): Lorentz-Berthelot strengths, and D(c) of an equal-diameter
binary with tails of strengths w_AA = -5 kT, w_BB = w_AA / 2 against the
hard-sphere D.

With equal diameters the hard-sphere part of the mixture is ideal, so the
tails alone set the thermodynamic factor: D_tail / D_hs = 1 + c (1 - c) n
(w_AA + w_BB - 2 w_AB) / kT in the paper's linear estimate (w = int U,
eq. diciotto), lowest at c = 1/2 and closer to 1 at larger diameters for the
same packing.  The field of the RPA reading (the force -dU/dr for r >
sigma_ab only, no contact term where the potential is cut at the core) has
twice that long-wavelength strength for a (sigma/r)^6 tail: the surface terms
of int r^3 U'(r) dr at sigma and at the cutoff add another w.
"""
import math

import numpy as np
import pytest

import workloads as W
from linear_scheme import KT, LinearScheme, hydrodynamics


def test_berthelot_strengths_are_geometric_means():
    for sigma in ((2.0, 2.0), (2.0, 3.0)):
        eps = W.berthelot_eps([-5 * KT, -2.5 * KT], sigma, 2.5)
        sab = 0.5 * np.add.outer(sigma, sigma)
        w = -(4 * math.pi / 3) * eps * sab ** 3 * (1 - 2.5 ** -3)
        assert w[0, 0] == pytest.approx(-5 * KT, rel=1e-14)
        assert w[1, 1] == pytest.approx(-2.5 * KT, rel=1e-14)
        assert w[0, 1] == pytest.approx(-math.sqrt(w[0, 0] * w[1, 1]), rel=1e-14)
        assert np.array_equal(eps, eps.T)


def _lin(sigma, x1, tails):
    m, n0, _ = W.config_tail_study(sigma, 0.3, x1, tails=tails)
    nn = np.array([n0[0].mean(), n0[1].mean()])
    return m, LinearScheme((sigma, sigma), nn, eps=m.eps_matrix() if tails else None)


@pytest.mark.parametrize("sigma", [2.0, 4.0])
def test_tail_reduction_follows_the_thermodynamic_factor(sigma):
    """Linearised scheme: D_tail / D_hs at the workload's wavelength against the
    hydrodynamic root and against the long-wavelength factor with the lattice
    force's tail strength; the reduction peaks at c = 1/2 and shrinks with the
    diameter."""
    ratios = []
    for x1 in (0.1, 0.3, 0.5, 0.7, 0.9):
        m, hs = _lin(sigma, x1, False)
        _, lb = _lin(sigma, x1, True)
        r = lb.diffusion(m.nx) / hs.diffusion(m.nx)
        r_hyd = hydrodynamics(lb)["D_P"] / hydrodynamics(hs)["D_P"]
        assert abs(r / r_hyd - 1) < 3e-4
        # the lattice force's long-wavelength tail strength (minus sum_e 6 eps s^6
        # / |e|^6 ex^2 / |e|^2): about 2 w for the (s/r)^6 tail
        n = lb.n0.sum()
        K = np.zeros((2, 2))
        for a in range(2):
            for b in range(2):
                e = lb.tails[a][b]
                rr = np.sqrt((e ** 2).sum(1))
                K[a, b] = -(6 * lb.eps[a, b] * sigma ** 6 / rr ** 6 * (e[:, 0] / rr) ** 2).sum()
        fac = 1 + x1 * (1 - x1) * n * (K[0, 0] + K[1, 1] - 2 * K[0, 1]) / KT
        assert abs(r / fac - 1) < 1.5e-3, (x1, r, fac)
        w = -(4 * math.pi / 3) * lb.eps * sigma ** 3 * (1 - 2.5 ** -3)
        paper = 1 + x1 * (1 - x1) * n * (w[0, 0] + w[1, 1] - 2 * w[0, 1]) / KT
        assert abs((fac - 1) / (paper - 1) - 2) < 0.1          # force-only reading: twice w
        ratios.append(r)
    ratios = np.array(ratios)
    assert np.all(ratios < 1) and np.argmin(ratios) == 2
    assert abs(ratios[1] - ratios[3]) < 2e-4 and abs(ratios[0] - ratios[4]) < 2e-4


def test_reduction_shrinks_with_diameter():
    r2 = _lin(2.0, 0.5, True)[1].diffusion(64) / _lin(2.0, 0.5, False)[1].diffusion(64)
    r4 = _lin(4.0, 0.5, True)[1].diffusion(128) / _lin(4.0, 0.5, False)[1].diffusion(128)
    assert 1 - r4 < 0.25 * (1 - r2)


def test_oracle_mode_decay_with_berthelot_tails(oracle_lib):
    """The composition-mode experiment at c = 1/2, sigma = 2, with the
    Lorentz-Berthelot tails, on a line of 64 sites, against the linearised D."""
    sigma = 2.0
    mfull, lb = _lin(sigma, 0.5, True)
    m = W.Mixture(64, 1, 1, sigma=(sigma, sigma), eps=mfull.eps_matrix(), rc_factor=2.5)
    o = oracle_lib.Oracle(m)
    n = lb.n0.sum()
    f = o.init(*W.mode_state(m, n, 0.5, 1e-3))
    k = 2 * math.pi / 64
    x = np.arange(64)
    D_lin = lb.diffusion(64)
    steps = int(1.5 / (D_lin * k * k))
    ts, amps = [], []
    for t in range(0, steps + 1, 20):
        d = o.densities(f)
        amps.append(abs(np.sum((d[0] - d[1])[0, 0] * np.exp(-1j * k * x))))
        ts.append(t)
        f = o.step(f, 20)
    ts, amps = np.array(ts), np.array(amps)
    sel = ts >= steps // 4
    D = -np.polyfit(ts[sel], np.log(amps[sel]), 1)[0] / k ** 2
    assert abs(D / D_lin - 1) < 2e-3, (D, D_lin)
