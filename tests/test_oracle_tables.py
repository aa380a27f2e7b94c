"""Pins of the oracle's lattice tables and contact values.

Checked against number theory (counts of lattice points on spheres), cubic
symmetry of the lattice shells, and the Carnahan-Starling closed form that
the BMCSL mixture contact value must reduce to for one species or for
equal diameters.
"""
import math

import numpy as np
import pytest

import workloads as W

# Number of ways to write k as a sum of three squares (OEIS A005875), k = 0..40.
R3 = [1, 6, 12, 8, 6, 24, 24, 0, 12, 30, 24, 24, 8, 24, 48, 0, 6, 48, 36, 24, 24,
      48, 24, 0, 24, 30, 72, 32, 0, 72, 48, 0, 12, 48, 48, 48, 30, 24, 72, 0, 24]


def _mix(sig, eps=None, rc=2.5):
    M = len(sig)
    return W.Mixture(8, 8, 8, sigma=tuple(sig), eps=None if eps is None else np.full((M, M), eps),
                     rc_factor=rc)


@pytest.mark.parametrize("sab", [1.0, 2.0, 2.25, 2.5, 2.75, 3.0, 3.5, 3.75, 4.0, 4.5])
def test_shell_counts_match_sums_of_three_squares(oracle_lib, sab):
    o = oracle_lib.Oracle(_mix([sab, sab]))
    e, unit = o.stencil("shell", 0, 0)
    lo, hi = (sab - 0.5) ** 2, (sab + 0.5) ** 2
    expect = sum(R3[k] for k in range(len(R3)) if lo <= k < hi)
    assert 2 * len(e) == expect
    r2 = (e ** 2).sum(1)
    assert np.all((r2 >= lo) & (r2 < hi))


def test_shell_sizes_at_the_workload_diameters(oracle_lib):
    # shells at sigma_ab of the workloads: 62, 98, 194, 234 points
    for s, n in [(2.0, 62), (3.0, 98), (3.75, 194), (4.5, 234), (2.5, 66), (4.0, 210)]:
        o = oracle_lib.Oracle(_mix([s]))
        assert 2 * len(o.stencil("shell", 0, 0)[0]) == n


@pytest.mark.parametrize("sab", [2.0, 2.5, 3.0, 3.75, 4.5])
def test_shell_half_list_order_and_cubic_symmetry(oracle_lib, sab):
    o = oracle_lib.Oracle(_mix([sab]))
    e, unit = o.stencil("shell", 0, 0)
    # positive half: first non-zero component > 0, no (e, -e) duplicates
    for v in e:
        nz = v[np.nonzero(v)[0][0]]
        assert nz > 0
    keys = [(int((v ** 2).sum()), int(v[0]), int(v[1]), int(v[2])) for v in e]
    assert keys == sorted(keys) and len(set(keys)) == len(keys)
    # unit vectors
    np.testing.assert_allclose(np.linalg.norm(unit, axis=1), 1.0, rtol=0, atol=1e-15)
    np.testing.assert_allclose(unit * np.linalg.norm(e, axis=1)[:, None], e, rtol=0, atol=1e-14)
    full = np.concatenate([unit, -unit])
    w_hat = 4 * math.pi / len(full)
    # sum over the sphere of w_hat e e^T = (4 pi / 3) I: exact by cubic symmetry
    T = w_hat * full.T @ full
    np.testing.assert_allclose(T, (4 * math.pi / 3) * np.eye(3), atol=1e-13)
    np.testing.assert_allclose(full.sum(0), 0.0, atol=1e-13)


@pytest.mark.parametrize("s,count", [(2.0, 7), (3.0, 19), (4.0, 33), (4.5, 57)])
def test_ball_sizes(oracle_lib, s, count):
    o = oracle_lib.Oracle(_mix([s]))
    e, _ = o.stencil("ball", 0)
    assert 2 * len(e) + 1 == count
    assert np.all((e ** 2).sum(1) <= (s / 2) ** 2)


def test_tail_weights_are_minus_dU_dr(oracle_lib):
    eps = 0.17
    o = oracle_lib.Oracle(_mix([2.0, 3.0], eps=eps, rc=2.5))
    for a, b in [(0, 0), (0, 1), (1, 1)]:
        sab = 0.5 * ([2.0, 3.0][a] + [2.0, 3.0][b])
        e, w = o.stencil("tail", a, b)
        r = np.linalg.norm(e, axis=1)
        assert np.all(r > sab) and np.all(r <= 2.5 * sab + 1e-12)
        # U(r) = -eps (sigma/r)^6 ; -dU/dr = -6 eps sigma^6 / r^7 ; the field on a
        # points toward b: weight = +6 eps sigma^6 / r^7 along e_hat
        mag = 6 * eps * sab ** 6 / r ** 7
        np.testing.assert_allclose(w, mag[:, None] * e / r[:, None], rtol=1e-14)
        # counts: every lattice point of the annulus appears once (+e, -e)
        r2 = (e ** 2).sum(1)
        total = sum(R3[k] if k < len(R3) else 0 for k in range(1, len(R3)) if sab ** 2 < k <= (2.5 * sab) ** 2)
        if (2.5 * sab) ** 2 < len(R3):
            assert 2 * len(e) == total
        assert len(set(map(tuple, e))) == len(e)


def _cs(eta):
    # Carnahan-Starling contact value of a one-component hard-sphere fluid
    return (1 - eta / 2) / (1 - eta) ** 3


@pytest.mark.parametrize("sigma,n", [(2.0, 0.02), (3.0, 0.014), (4.5, 0.004)])
def test_contact_value_reduces_to_carnahan_starling(oracle_lib, sigma, n):
    m = W.Mixture(10, 10, 10, sigma=(sigma,))
    o = oracle_lib.Oracle(m)
    n0, u0 = W.uniform_state(m, [n])
    d = o.fields(o.init(n0, u0))
    eta = math.pi / 6 * n * sigma ** 3
    np.testing.assert_allclose(d["g"][0], _cs(eta), rtol=2e-14)


def test_equal_diameter_mixture_is_one_component_fluid(oracle_lib):
    m = W.Mixture(10, 10, 10, sigma=(3.0, 3.0, 3.0))
    o = oracle_lib.Oracle(m)
    n0, u0 = W.uniform_state(m, [0.004, 0.006, 0.003])
    d = o.fields(o.init(n0, u0))
    eta = math.pi / 6 * 0.013 * 27
    for p in range(6):
        np.testing.assert_allclose(d["g"][p], _cs(eta), rtol=2e-14)


def test_bmcsl_mixture_contact_values(oracle_lib):
    # Boublik / Mansoori et al. contact value written in its usual three-term form
    s = (2.0, 3.5)
    n = (0.012, 0.006)
    m = W.Mixture(10, 10, 10, sigma=s)
    o = oracle_lib.Oracle(m)
    n0, u0 = W.uniform_state(m, n)
    d = o.fields(o.init(n0, u0))
    x2 = math.pi / 6 * sum(nc * sc ** 2 for nc, sc in zip(n, s))
    x3 = math.pi / 6 * sum(nc * sc ** 3 for nc, sc in zip(n, s))
    for (a, b), p in [((0, 0), 0), ((0, 1), 1), ((1, 1), 2)]:
        dd = s[a] * s[b] / (s[a] + s[b])
        g = 1 / (1 - x3) + 3 * dd * x2 / (1 - x3) ** 2 + 2 * (dd * x2) ** 2 / (1 - x3) ** 3
        np.testing.assert_allclose(d["g"][p], g, rtol=1e-14)
    # the cross value lies between the two like-pair values
    assert d["g"][0].max() < d["g"][1].min() < d["g"][2].min()
