"""Pin of the oracle's dynamics against the paper's mutual diffusion coefficient.

For an equal-diameter, equal-mass binary hard-sphere mixture the composition
is thermodynamically ideal, so a small sinusoidal composition mode (the
experiment of Sec. 5.1, eq. perturba) decays at D q^2 with D given by
eq. (dab):  D_AB = 3/(8 n) sqrt(kT) / (sqrt(2 pi mu) sigma^2 g),
g the contact value of the one-component fluid at the total packing.
"""
import math

import numpy as np
import pytest

import workloads as W


def _cs(eta):
    return (1 - eta / 2) / (1 - eta) ** 3


def d_ab_paper(n, sigma, eta, kT=1.0 / 3.0, mu=0.5):
    return 3.0 / (8.0 * n) * math.sqrt(kT) / (math.sqrt(2 * math.pi * mu) * sigma ** 2 * _cs(eta))


def fit_mode_decay(o, f, L, steps, every, t0):
    """Amplitude of the (n_0 - n_1) Fourier mode at k = 2 pi / L versus time; D = -slope / k^2."""
    k = 2 * math.pi / L
    x = np.arange(L)
    ts, amps = [], []
    t = 0
    while t <= steps:
        d = o.fields(f)
        dn = (d["n"][0] - d["n"][1]).mean(axis=(0, 1))
        amps.append(abs(np.sum(dn * np.exp(-1j * k * x))))
        ts.append(t)
        f = o.step(f, every)
        t += every
    ts, amps = np.array(ts), np.array(amps)
    sel = ts >= t0
    slope = np.polyfit(ts[sel], np.log(amps[sel]), 1)[0]
    return -slope / k ** 2


@pytest.mark.parametrize("sigma,eta", [(3.0, 0.2), (2.0, 0.3)])
def test_equisized_mode_decay_matches_eq_dab(oracle_lib, sigma, eta):
    L = 128
    m = W.Mixture(L, 1, 1, sigma=(sigma, sigma))
    n = W.number_density(eta, (0.5, 0.5), m.sigma)
    n0, u0 = W.mode_state(m, n, 0.5, 1e-3)
    o = oracle_lib.Oracle(m)
    f = o.init(n0, u0)
    Dp = d_ab_paper(n, sigma, eta)
    steps = int(2.0 / (Dp * (2 * math.pi / L) ** 2))
    D = fit_mode_decay(o, f, L, steps, 10, steps // 5)
    assert abs(D / Dp - 1) < 0.003, (D, Dp)
