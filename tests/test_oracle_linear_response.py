"""Pins of the oracle's force fields and of its whole step against the
paper's linear estimates and against the linearised scheme.

- Hard-core mean field of a weak density wave (Sec. 3, eq. diciotto): for
  n_b = n_b0 + dn cos(q x) the oracle's field, divided by n_a, is
  q dn sin(q x) times kT (4 pi / 3) (s_ab^3 g_ab + 1/2 sum_c n_c s_ac^3
  dg_ac/dn_b) as q -> 0, with the lattice shell's own radius in place of
  the continuum sphere's (s^3 -> s^2 R_ab).  This fixes the sign, the
  s^2 w_hat normalisation, the 1/2 of the pair value (g(r) + g(r+e)) / 2,
  the density derivative of the contact values and the smoothing.
- Viscous force of a weak velocity wave with u^A = u^B (eqs. viscousforce1,
  viscousforce2): perpendicular and parallel parts at order q^2, with the
  lattice shell's fourth moment in place of the sphere's s^2 (4 pi / 15) and
  s^2 (4 pi / 5).
- One whole step, linearised around a uniform mixture at rest, against the
  independent linearisation in linear_scheme.py (column by column, at the
  wavenumbers of the workloads), and the composition-mode decay of small
  oracle runs against its diffusion eigenvalue.
- A uniform mixture at rest stays bitwise stationary for 1000 steps.
"""
import math

import numpy as np
import pytest

import workloads as W
from linear_scheme import LinearScheme, bmcsl

KT = 1.0 / 3.0


def _line(sigma, L, eps=None, rc=2.5, scheme=W.SCHEME_CN_J1):
    """An L x 1 x 1 box: every offset with the same e_x lands on the same site,
    so the lattice sums are those of an x plane wave in an infinite box."""
    e = None if eps is None else np.full((len(sigma), len(sigma)), eps)
    return W.Mixture(L, 1, 1, sigma=tuple(sigma), eps=e, rc_factor=rc, scheme=scheme)


def _proj(v, k, fn):
    L = v.shape[-1]
    x = np.arange(L)
    return 2.0 / L * float(np.sum(v * fn(k * x)))


def _field_response(oracle_lib, m, n0, b, h, key, comp=0):
    """(field(+h) - field(-h)) / 2 for n_b = n_b0 + h cos(kx): the part odd in h."""
    o = oracle_lib.Oracle(m)
    k = 2 * math.pi / m.nx
    out = []
    for sgn in (1.0, -1.0):
        n, u = W.uniform_state(m, n0)
        n[b] += sgn * h * np.cos(k * np.arange(m.nx))[None, None, :]
        out.append(o.fields(o.init(n, u))[key])
    return (out[0] - out[1])[:, comp, 0, 0, :] / 2.0


STATES = [((3.0, 4.5), W.number_density(0.3, (0.5, 0.5), (3.0, 4.5)) * np.array([0.5, 0.5])),
          ((2.0, 3.0), W.number_density(0.2, (0.5, 0.5), (2.0, 3.0)) * np.array([0.5, 0.5])),
          ((2.0, 4.0), W.number_density(0.35, (0.9, 0.1), (2.0, 4.0)) * np.array([0.9, 0.1]))]


@pytest.mark.parametrize("sigma,n0", STATES)
def test_contact_values_match_bmcsl(oracle_lib, sigma, n0):
    m = _line(sigma, 16)
    o = oracle_lib.Oracle(m)
    n, u = W.uniform_state(m, n0)
    g = o.fields(o.init(n, u))["g"][:, 0, 0, 0]
    ref = bmcsl(n0, sigma)
    np.testing.assert_allclose(g, [ref[0, 0], ref[0, 1], ref[1, 1]], rtol=1e-14)


@pytest.mark.parametrize("sigma,n0", STATES)
def test_mean_field_plane_wave_lattice_form(oracle_lib, sigma, n0):
    """The oracle's mean field of a density wave equals the linearised lattice
    sum at finite q (ball-smoothed contact values, pair average)."""
    L = 64
    k = 2 * math.pi / L
    lin = LinearScheme(sigma, n0)
    K = lin.mean_field(k)
    for b in range(2):
        h = 1e-6 * n0[b]
        r = _field_response(oracle_lib, _line(sigma, L), n0, b, h, "Nmf")
        for a in range(2):
            amp = _proj(r[a], k, np.sin) / (n0[a] * h)
            assert abs(amp / K[a, b] - 1) < 1e-8, (a, b, amp, K[a, b])
            assert abs(_proj(r[a], k, np.cos)) < 1e-12 * abs(amp) * n0[a] * h + 1e-30


@pytest.mark.parametrize("sigma,n0", STATES)
def test_mean_field_small_q_limit_is_eq_diciotto(oracle_lib, sigma, n0):
    """Sec. 3, eq. (diciotto), hard-core part, from the oracle's field at three
    wavelengths extrapolated to q -> 0 (the q^2 and q^4 terms removed)."""
    Ls = (256, 512, 1024)
    ratios = np.zeros((3, 2, 2))
    for i, L in enumerate(Ls):
        k = 2 * math.pi / L
        for b in range(2):
            h = 1e-6 * n0[b]
            r = _field_response(oracle_lib, _line(sigma, L), n0, b, h, "Nmf")
            for a in range(2):
                ratios[i, a, b] = _proj(r[a], k, np.sin) / (n0[a] * h * k)
    # Richardson on k^2 halving: R(k) = R0 + c k^2 + d k^4
    r1 = (4 * ratios[1] - ratios[0]) / 3
    r2 = (4 * ratios[2] - ratios[1]) / 3
    limit = (16 * r2 - r1) / 15
    paper = LinearScheme(sigma, n0).paper_mean_field_limit(lattice_radius=True)
    np.testing.assert_allclose(limit, paper, rtol=2e-7)
    # the force is repulsive: a density excess of either species pushes both away
    assert np.all(paper > 0)


@pytest.mark.parametrize("sigma,n0", STATES[:2])
@pytest.mark.parametrize("comp", [0, 1])
def test_viscous_force_plane_wave(oracle_lib, sigma, n0, comp):
    """Equal species velocities u cos(q x) along x (parallel) or y
    (perpendicular): the pair form at the old velocities against the lattice
    sum, and its q^2 coefficient against eqs. (viscousforce1/2) with the lattice
    shell's fourth moment."""
    lin = LinearScheme(sigma, n0)
    U = 1e-3
    coef = []
    for L in (64, 256, 512):
        k = 2 * math.pi / L
        m = _line(sigma, L)
        o = oracle_lib.Oracle(m)
        n, u = W.uniform_state(m, n0)
        u[:, comp] = U * np.cos(k * np.arange(L))[None, None, None, :]
        d = o.fields(o.init(n, u))
        V = lin.viscous(k, comp)
        for a in range(2):
            amp = _proj(d["Dold"][a, comp, 0, 0, :], k, np.cos) / (n0[a] * U)
            if L == 64:
                assert abs(amp / V[a] - 1) < 1e-9, (a, amp, V[a])
            # no other component
            assert np.abs(d["Dold"][a, 1 - comp]).max() < 1e-14 * abs(amp) * n0[a] * U
        if L > 64:
            coef.append([_proj(d["Dold"][a, comp, 0, 0, :], k, np.cos) / (n0[a] * U * k * k) for a in range(2)])
    lim = (4 * np.array(coef[1]) - np.array(coef[0])) / 3
    # lattice form of eqs. (viscousforce1/2): -q^2 u sum_b kappa_ab g n_b (1/2) sum_e |e|^2 ehat_c^2 ehat_x^2
    want = np.zeros(2)
    for a in range(2):
        for b in range(2):
            e = lin.shells[a][b]
            r2 = (e ** 2).sum(1)
            uc = e[:, comp] ** 2 / r2
            ux = e[:, 0] ** 2 / r2
            mom4 = lin.what[a, b] * (r2 * uc * ux).sum()       # continuum: s^2 (4 pi / 15) or s^2 (4 pi / 5)
            want[a] += 2 * lin.sab[a, b] ** 2 * math.sqrt(2 * 0.5 * KT / math.pi) * lin.g[a, b] * n0[b] * 0.5 * mom4
    np.testing.assert_allclose(-lim, want, rtol=1e-6)
    # with the sphere's moment the same expression is the paper's coefficient
    paper = lin.paper_viscous_limit(comp)
    sphere = np.zeros(2)
    for a in range(2):
        for b in range(2):
            s = lin.sab[a, b]
            m4 = s * s * (4 * math.pi / 5 if comp == 0 else 4 * math.pi / 15)
            sphere[a] += 2 * s * s * math.sqrt(2 * 0.5 * KT / math.pi) * lin.g[a, b] * n0[b] * 0.5 * m4
    np.testing.assert_allclose(sphere, paper, rtol=1e-14)


def _jacobian(oracle_lib, m, n0, k):
    """One oracle step linearised on (dn_a, dj_a,x) at wavenumber k (the
    step's response to cos(kx) perturbations, projected on exp(-ikx))."""
    o = oracle_lib.Oracle(m)
    M = len(n0)
    x = np.arange(m.nx)
    c = np.cos(k * x)
    J = np.zeros((2 * M, 2 * M), complex)
    for col in range(2 * M):
        outs = []
        for sgn in (1.0, -1.0):
            n, u = W.uniform_state(m, n0)
            if col < M:
                h = 1e-6 * n0[col]
                n[col] += sgn * h * c[None, None, :]
            else:
                a = col - M
                h = 1e-6 * n0[a]
                u[a, 0] += sgn * (h / n0[a]) * c[None, None, :]
            d = o.fields(o.step(o.init(n, u), 1))
            outs.append(np.concatenate([d["n"][:, 0, 0, :], d["j"][:, 0, 0, 0, :]]))
        diff = (outs[0] - outs[1]) / (2 * h)
        J[:, col] = 2.0 / m.nx * (diff * np.exp(-1j * k * x)[None, :]).sum(1)
    return J


CASES = [
    # bulk-diffusion physics: sigma 3, 4.5, packing 0.3, tail eps = kT/2, cutoff 2.5
    dict(sigma=(3.0, 4.5), xi=0.3, x1=0.5, eps=0.5 * KT, L=128),
    # step-binary / closure physics: sigma 2, 3, packing 0.2
    dict(sigma=(2.0, 3.0), xi=0.2, x1=0.5, eps=None, L=64),
    # a dense, asymmetric ensemble corner
    dict(sigma=(2.0, 4.0), xi=0.35, x1=0.9, eps=None, L=64),
]


def _state(c):
    x = np.array([c["x1"], 1 - c["x1"]])
    return W.number_density(c["xi"], x, c["sigma"]) * x


@pytest.mark.parametrize("c", CASES)
@pytest.mark.parametrize("scheme", ["cnj1", "fe"])
def test_one_step_matches_linearised_scheme(oracle_lib, c, scheme):
    n0 = _state(c)
    m = _line(c["sigma"], c["L"], eps=c["eps"], scheme=W.SCHEME_FE if scheme == "fe" else W.SCHEME_CN_J1)
    k = 2 * math.pi / c["L"]
    lin = LinearScheme(c["sigma"], n0, eps=None if c["eps"] is None else np.full((2, 2), c["eps"]), scheme=scheme)
    J = _jacobian(oracle_lib, m, n0, k)
    T = lin.longitudinal(k)
    np.testing.assert_allclose(J, T, rtol=0, atol=2e-9 * np.abs(T).max())


@pytest.mark.parametrize("c", CASES[:2])
def test_transverse_step_matches_linearised_scheme(oracle_lib, c):
    n0 = _state(c)
    m = _line(c["sigma"], c["L"], eps=c["eps"])
    k = 2 * math.pi / c["L"]
    lin = LinearScheme(c["sigma"], n0, eps=None if c["eps"] is None else np.full((2, 2), c["eps"]))
    o = oracle_lib.Oracle(m)
    x = np.arange(c["L"])
    J = np.zeros((2, 2), complex)
    for col in range(2):
        n, u = W.uniform_state(m, n0)
        U = 1e-6
        u[col, 1] = U * np.cos(k * x)[None, None, :]
        d = o.fields(o.step(o.init(n, u), 1))
        J[:, col] = 2.0 / c["L"] * (d["j"][:, 1, 0, 0, :] * np.exp(-1j * k * x)[None, :]).sum(1) / (n0[col] * U)
    np.testing.assert_allclose(J, lin.transverse(k), rtol=0, atol=1e-10)


def test_linearised_diffusion_of_equisized_mixture_is_eq_dab():
    """An ideal (equal-diameter) mixture: the diffusion eigenvalue of the
    linearised scheme against eq. (dab), D = 3/(8 n) sqrt(kT)/(sqrt(2 pi mu)
    sigma^2 g) with g the one-component Carnahan-Starling contact value."""
    for sigma, xi in ((3.0, 0.2), (2.0, 0.3)):
        n = W.number_density(xi, (0.5, 0.5), (sigma, sigma))
        lin = LinearScheme((sigma, sigma), (n / 2, n / 2))
        g = (1 - xi / 2) / (1 - xi) ** 3
        dab = 3 / (8 * n) * math.sqrt(KT) / (math.sqrt(2 * math.pi * 0.5) * sigma ** 2 * g)
        assert abs(lin.diffusion(1024) / dab - 1) < 2e-3, (sigma, xi, lin.diffusion(1024), dab)


@pytest.mark.parametrize("c", CASES[:2])
def test_small_amplitude_mode_decay_matches_linearised_d(oracle_lib, c):
    """The composition-mode experiment of Sec. 5.1 (eq. perturba) at amplitude
    1e-3 on the oracle, fitted as 1/tau = D q^2, against the diffusion
    eigenvalue of the linearised scheme."""
    n0 = _state(c)
    L = c["L"]
    m = _line(c["sigma"], L, eps=c["eps"])
    lin = LinearScheme(c["sigma"], n0, eps=None if c["eps"] is None else np.full((2, 2), c["eps"]))
    D_lin = lin.diffusion(L)
    o = oracle_lib.Oracle(m)
    n, u = W.mode_state(m, n0.sum(), c["x1"], 1e-3)
    f = o.init(n, u)
    k = 2 * math.pi / L
    x = np.arange(L)
    steps = int(1.5 / (D_lin * k * k))
    every = max(steps // 60, 1)
    ts, amps = [], []
    for t in range(0, steps + 1, every):
        d = o.densities(f)
        amps.append(abs(np.sum((d[0] - d[1])[0, 0] * np.exp(-1j * k * x))))
        ts.append(t)
        f = o.step(f, every)
    ts, amps = np.array(ts), np.array(amps)
    sel = ts >= steps // 4
    D = -np.polyfit(ts[sel], np.log(amps[sel]), 1)[0] / k ** 2
    assert abs(D / D_lin - 1) < 5e-3, (D, D_lin)


def test_uniform_mixture_stationary_for_1000_steps(oracle_lib):
    """A uniform mixture at rest stays bitwise stationary: the +-e pair sums
    cancel exactly, so no force and no momentum ever appear.  Only the
    rounding of the density sum moves n by a few ulp in the first steps, until
    it reaches a fixed point of that rounding; from there every step returns
    the same populations bit for bit."""
    m = W.Mixture(10, 9, 8, sigma=(2.0, 3.0), eps=np.full((2, 2), 0.1), rc_factor=1.5)
    o = oracle_lib.Oracle(m)
    n0, u0 = W.uniform_state(m, [0.015, 0.008])
    f0 = o.step(o.init(n0, u0), 20)
    f = o.step(f0, 1000)
    assert np.array_equal(f, f0)
    d = o.fields(f)
    assert not d["j"].any() and not d["N"].any()
    np.testing.assert_allclose(d["n"], n0, rtol=1e-14)


def test_stored_bulk_diffusion_d12_matches_linearised_d():
    """The oracle's D_12 stored for the 128x32x32 bulk-diffusion workload
    (amplitude 0.05 plus 1 % noise, 2000 steps) against the diffusion
    eigenvalue of the linearised scheme at that physics and wavelength."""
    import json
    import os
    here = os.path.dirname(os.path.abspath(__file__))
    g = json.load(open(os.path.join(here, "golden", "bulk_diffusion_128x32x32_2000.json")))
    c = CASES[0]
    lin = LinearScheme(c["sigma"], _state(c), eps=np.full((2, 2), c["eps"]))
    assert abs(g["D12"] / lin.diffusion(128) - 1) < 5e-3, (g["D12"], lin.diffusion(128))
