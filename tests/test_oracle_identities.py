"""Pins of the oracle's step against identities the paper fixes.

- Collision/forcing moments: the orthogonalised equilibrium of eq. (prefactor)
  carries the species density and momentum of f, and the field term of
  eq. (evolution) adds momentum n_a Phi_a and no mass (Sec. 2, the species
  continuity and momentum balances, eqs. continuity and momentcomponent).
- Exact conservation of species mass and of total momentum (the dissipative
  forces are pair forms, Newton's third law).
- A uniform mixture at rest feels no force.
- The friction decay of a uniform counter-flow against the homogeneous
  friction coefficient gamma_ab = (8/3) sqrt(2 pi mu kT) g n_b sigma^2 of
  Sec. 3 (end of the linear estimates) and eq. (gammasymmetrized1).
- Plane Couette flow between moving walls in the dilute limit.
- A species with no particles anywhere drops out: every sum over partner
  species (the BMCSL contact values through the packing fractions, the
  shell integrals of eqs. (potmeanforce) and (viscousforce), the attractive
  field below eq. (potmeanforce)) gets exact zeros from it, so the other
  species evolve as the mixture without it, bit for bit.
"""
import math

import numpy as np
import pytest

import workloads as W

CV = np.array([[0, 0, 0], [1, 0, 0], [-1, 0, 0], [0, 1, 0], [0, -1, 0], [0, 0, 1], [0, 0, -1],
               [1, 1, 0], [-1, -1, 0], [1, -1, 0], [-1, 1, 0], [1, 0, 1], [-1, 0, -1], [1, 0, -1],
               [-1, 0, 1], [0, 1, 1], [0, -1, -1], [0, 1, -1], [0, -1, 1]], dtype=float)


@pytest.mark.parametrize("tau", [1.0, 0.8, 1.7])
def test_collision_moments(oracle_lib, tau):
    m = W.Mixture(4, 4, 4, sigma=(2.0, 3.0), tau=tau)
    o = oracle_lib.Oracle(m)
    rng = np.random.default_rng(7)
    for _ in range(50):
        na = rng.uniform(0.001, 0.05)
        fi = rng.uniform(0.2, 1.0, 19) * na / 19 * 1.0
        na = fi.sum()
        ja = CV.T @ fi
        u = rng.uniform(-0.1, 0.1, 3)
        Na = rng.uniform(-1e-3, 1e-3, 3)
        fs = o.collide_site(fi, na, ja, u, Na)
        assert abs(fs.sum() - na) <= 1e-15 * 19 * na
        np.testing.assert_allclose(CV.T @ fs, ja + Na, rtol=0, atol=4e-16 * 19 * na)


def test_equilibrium_second_moment(oracle_lib):
    # with j_a = n_a u the equilibrium has the ideal-gas pressure n kT plus n u u
    m = W.Mixture(4, 4, 4, sigma=(2.0,), tau=1.0)
    o = oracle_lib.Oracle(m)
    na, u = 0.02, np.array([0.03, -0.02, 0.01])
    fs = o.collide_site(np.zeros(19), na, na * u, u, np.zeros(3))
    P = (CV.T * fs) @ CV
    np.testing.assert_allclose(P, na / 3 * np.eye(3) + na * np.outer(u, u), atol=1e-17)


def test_uniform_mixture_at_rest_feels_no_force(oracle_lib):
    m = W.Mixture(12, 12, 12, sigma=(2.0, 3.0, 4.0), eps=np.full((3, 3), 0.1))
    o = oracle_lib.Oracle(m)
    n0, u0 = W.uniform_state(m, [0.01, 0.006, 0.002])
    f = o.init(n0, u0)
    for _ in range(3):
        f = o.step(f, 5)
        d = o.fields(f)
        assert np.all(d["j"] == 0.0) and np.all(d["N"] == 0.0)
        for a in range(3):
            assert np.ptp(d["n"][a]) == 0.0


def _conservation_case(oracle_lib, m, n0, u0, steps=20):
    o = oracle_lib.Oracle(m)
    f = o.init(n0, u0)
    d0 = o.fields(f)
    mass0 = d0["n"].sum(axis=(1, 2, 3))
    P0 = d0["j"].sum(axis=(0, 2, 3, 4))
    for _ in range(steps):
        d = o.fields(f)
        f2 = o.step(f, 1)
        d2 = o.fields(f2)
        # species momentum gain equals the summed force density
        dj = d2["j"].sum(axis=(2, 3, 4)) - d["j"].sum(axis=(2, 3, 4))
        np.testing.assert_allclose(dj, d["N"].sum(axis=(2, 3, 4)), atol=1e-15 * m.N)
        f = f2
    d = o.fields(f)
    np.testing.assert_allclose(d["n"].sum(axis=(1, 2, 3)), mass0, rtol=1e-13)
    np.testing.assert_allclose(d["j"].sum(axis=(0, 2, 3, 4)), P0, atol=1e-15 * m.N)
    assert np.abs(d["N"].sum(axis=(0, 2, 3, 4))).max() < 1e-16 * m.N


def test_conservation_random_binary(oracle_lib):
    m = W.Mixture(10, 9, 8, sigma=(2.0, 3.0))
    n0, u0 = W.random_state(m, [0.012, 0.008], rel=0.3, u_amp=0.03, seed=3)
    _conservation_case(oracle_lib, m, n0, u0)


def test_conservation_ternary_with_tail(oracle_lib):
    m = W.Mixture(12, 12, 12, sigma=(1.5, 2.0, 2.5), eps=np.full((3, 3), 0.15), rc_factor=2.0)
    n0, u0 = W.random_state(m, [0.02, 0.01, 0.005], rel=0.3, u_amp=0.03, seed=4)
    _conservation_case(oracle_lib, m, n0, u0, steps=8)


def test_conservation_step_profile(oracle_lib):
    m, n0, u0 = W.config_step_binary(32, 8, 8)
    _conservation_case(oracle_lib, m, n0, u0)


def test_species_mass_conserved_with_moving_walls(oracle_lib):
    m = W.Mixture(10, 12, 6, sigma=(2.0, 3.0), walls_y=True, wall_ux=(-0.04, 0.05))
    n0, u0 = W.random_state(m, [0.012, 0.008], rel=0.3, u_amp=0.03, seed=5)
    o = oracle_lib.Oracle(m)
    f = o.init(n0, u0)
    mass0 = o.fields(f)["n"].sum(axis=(1, 2, 3))
    f = o.step(f, 30)
    d = o.fields(f)
    np.testing.assert_allclose(d["n"].sum(axis=(1, 2, 3)), mass0, rtol=1e-13)
    assert np.all(d["n"][:, :, 0, :] == 0) and np.all(d["n"][:, :, -1, :] == 0)


def _gamma_ab(g, nb, sab, kT=1.0 / 3.0, mu=0.5):
    # homogeneous friction coefficient of the paper's linear estimate
    return 8.0 / 3.0 * math.sqrt(2 * math.pi * mu * kT) * g * nb * sab ** 2


@pytest.mark.parametrize("sig,n", [((2.0, 3.0), (0.012, 0.008)), ((3.0, 3.0), (0.007, 0.007)),
                                   ((2.0, 4.0), (0.02, 0.002))])
def test_friction_decay_of_uniform_counterflow(oracle_lib, sig, n):
    m = W.Mixture(12, 12, 12, sigma=sig)
    o = oracle_lib.Oracle(m)
    w0 = 1e-3
    # zero barycentric velocity: n1 u1 + n2 u2 = 0
    u1 = w0 * n[1] / (n[0] + n[1])
    u2 = -w0 * n[0] / (n[0] + n[1])
    n0, u0 = W.uniform_state(m, n, [[u1, 0, 0], [u2, 0, 0]])
    f = o.init(n0, u0)
    d = o.fields(f)
    x2 = math.pi / 6 * sum(nc * s ** 2 for nc, s in zip(n, sig))
    x3 = math.pi / 6 * sum(nc * s ** 3 for nc, s in zip(n, sig))
    gfun = lambda a, b: (1 / (1 - x3) + 3 * (sig[a] * sig[b] / (sig[a] + sig[b])) * x2 / (1 - x3) ** 2
                         + 2 * (sig[a] * sig[b] / (sig[a] + sig[b]) * x2) ** 2 / (1 - x3) ** 3)
    sab = lambda a, b: 0.5 * (sig[a] + sig[b])
    G = [[_gamma_ab(gfun(a, b), n[b], sab(a, b)) for b in range(2)] for a in range(2)]
    Gam = [G[a][0] + G[a][1] for a in range(2)]
    np.testing.assert_allclose(d["gam"][0], Gam[0], rtol=1e-13)
    np.testing.assert_allclose(d["gam"][1], Gam[1], rtol=1e-13)
    gam = G[0][1] + G[1][0]            # eq. (gammasymmetrized1) with unit masses
    lam = 1 - 0.5 * gam * (2 - G[0][1] / (1 + 0.5 * Gam[0]) - G[1][0] / (1 + 0.5 * Gam[1]))
    w = w0
    for t in range(6):
        f = o.step(f, 1)
        d = o.fields(f)
        w = w * lam
        wn = d["j"][0, 0] / d["n"][0] - d["j"][1, 0] / d["n"][1]
        np.testing.assert_allclose(wn, w, rtol=1e-11)
    assert 0 < lam < 1


def test_dilute_couette_profile(oracle_lib):
    """Halfway bounce-back puts the walls half a link outside the first fluid
    layer; in the dilute limit the steady profile is linear between them."""
    U = 0.02
    m = W.Mixture(4, 10, 4, sigma=(1.0,), walls_y=True, wall_ux=(-U, U))
    o = oracle_lib.Oracle(m)
    n0, u0 = W.uniform_state(m, [1e-5])
    f = o.step(o.init(n0, u0), 3000)
    d = o.fields(f)
    ux = (d["j"][0, 0] / np.where(d["n"][0] > 0, d["n"][0], 1))[0, 1:-1, 0]
    y = np.arange(1, 9)
    expect = -U + 2 * U * (y - 0.5) / 8.0
    np.testing.assert_allclose(ux, expect, atol=2e-6)


@pytest.mark.parametrize("scheme", [W.SCHEME_CN_J1, W.SCHEME_FE])
def test_absent_species_drops_out(oracle_lib, scheme):
    """A binary whose second species is empty everywhere against the one-species
    system of the first: populations and every field of species 0 agree bit for
    bit after 5 steps (a wrong pair or diameter index in a cross-species term
    would make them differ, since sigma_11 and eps_01 differ from sigma_00 and
    eps_00)."""
    eps2 = np.array([[0.1, 0.07], [0.07, 0.05]])
    m2 = W.Mixture(10, 11, 9, sigma=(2.5, 3.5), eps=eps2, rc_factor=2.0, scheme=scheme)
    m1 = W.Mixture(10, 11, 9, sigma=(2.5,), eps=np.array([[0.1]]), rc_factor=2.0, scheme=scheme)
    n0, u0 = W.random_state(m2, [0.02, 0.01], rel=0.4, u_amp=0.03, seed=33)
    n0[1] = 0.0
    u0[1] = 0.0
    o2, o1 = oracle_lib.Oracle(m2), oracle_lib.Oracle(m1)
    f2 = o2.step(o2.init(n0, u0), 5)
    f1 = o1.step(o1.init(n0[:1], u0[:1]), 5)
    assert np.array_equal(np.asarray(f2)[:1], np.asarray(f1))
    assert not np.asarray(f2)[1].any()
    d2, d1 = o2.fields(f2), o1.fields(f1)
    assert np.array_equal(d2["u"], d1["u"])
    assert np.array_equal(d2["g"][:1], d1["g"])          # pair (0, 0) comes first
    for k in ("n", "j", "vhat", "H", "N", "gam", "Nmf", "Ntail", "Dold", "Dnew"):
        assert np.array_equal(d2[k][:1], d1[k]), k
    assert np.abs(d1["Ntail"]).max() > 0 and np.abs(d1["H"]).max() > 0
