"""Pins of the wall reading (halfway bounce-back walls at y = 1/2 and
y = ny - 3/2; beyond a wall the hard-core stencils see the mirror image of
the fluid, moving with the wall; the attractive field sees nothing there).

- A uniform hard-sphere fluid between walls at rest is exactly at rest: the
  mirror gives every fluid row a symmetric hard-core environment, so every
  +-e pair of the shell sums cancels (as in the periodic box).
- With the attractive tail (no image) a mixture at the Taylor/Couette
  workload's packing 0.25 relaxes to a stationary, mirror-symmetric
  equilibrium profile at rest, within 15 % of uniform (the unmirrored
  attraction thins the first layer).
- At that packing the Couette flow between walls moving at -+0.05 stays
  finite over 5000 steps, conserves species mass and settles into a linear
  profile in the bulk.
"""
import numpy as np

import workloads as W


def test_uniform_fluid_between_walls_at_rest_stays_at_rest(oracle_lib):
    m = W.Mixture(6, 20, 6, sigma=(2.0, 3.0, 4.0), walls_y=True)
    n = W.number_density(0.25, (0.5, 0.5), (2.0, 3.0))
    n0, u0 = W.uniform_state(m, [0.5 * n, 0.5 * n, 0.0])
    o = oracle_lib.Oracle(m)
    f0 = o.step(o.init(n0, u0), 20)          # rounding fixed point of the density sums
    f = o.step(f0, 200)
    assert np.array_equal(f, f0)
    d = o.fields(f)
    assert not d["j"].any() and not d["N"].any()
    fluid = d["n"][:, :, 1:-1, :]
    for a in range(2):
        assert np.ptp(fluid[a]) == 0.0


def test_equilibrium_profile_between_walls(oracle_lib):
    m, n0, u0 = W.config_taylor_couette(1, 40, 1, U=0.0, packing=0.25)
    o = oracle_lib.Oracle(m)
    f = o.step(o.init(n0, u0), 3000)
    d1 = o.fields(f)
    f = o.step(f, 200)
    d2 = o.fields(f)
    n1, n2 = d1["n"][:, 0, 1:-1, 0], d2["n"][:, 0, 1:-1, 0]
    assert np.abs(n2 - n1).max() < 1e-9 * n1.max()                       # stationary
    # at rest: near the walls a steady force N balances the pressure, and the
    # moment j of the populations is the momentum half a step before it acts,
    # so the momentum at rest is j + N / 2 = 0 (j alone is -N / 2)
    assert np.abs(d2["N"]).max() > 1e-5 * n1.max()
    assert np.abs(d2["j"] + 0.5 * d2["N"]).max() < 1e-10 * n1.max()
    np.testing.assert_allclose(n2, n2[:, ::-1], rtol=1e-10, atol=0)       # mirror symmetric
    mid = n2[:, n2.shape[1] // 2]
    for a in range(2):
        # within 15 % of the bulk: the attraction, which has no image, pulls the
        # first layer (10 % for sigma = 3) towards the bulk
        assert np.abs(n2[a] / mid[a] - 1).max() < 0.15


def test_couette_at_packing_025_is_stable(oracle_lib):
    U = 0.05
    m, n0, u0 = W.config_taylor_couette(1, 64, 1, U=U, packing=0.25)
    o = oracle_lib.Oracle(m)
    f = o.init(n0, u0)
    mass0 = o.fields(f)["n"].sum(axis=(1, 2, 3))
    f = o.step(f, 5000)
    d = o.fields(f)
    assert np.all(np.isfinite(d["n"]))
    np.testing.assert_allclose(d["n"].sum(axis=(1, 2, 3)), mass0, rtol=1e-12)
    nt = d["n"].sum(0)[0, 1:-1, 0]
    ux = d["j"][:, 0].sum(0)[0, 1:-1, 0] / nt
    y = np.arange(1, m.ny - 1)
    bulk = slice(10, -10)
    slope, icpt = np.polyfit(y[bulk], ux[bulk], 1)
    assert np.abs(ux[bulk] - (icpt + slope * y[bulk])).max() < 2e-4 * U
    # antisymmetric about the centre, the fluid dragged along by the walls
    np.testing.assert_allclose(ux, -ux[::-1], atol=1e-12)
    assert ux[0] < -0.9 * U and ux[-1] > 0.9 * U
    assert slope > 0
