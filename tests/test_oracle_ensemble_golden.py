"""Pins of the stored float64 D_12 of six ensemble members
(tests/golden/ensemble_d12_members.json, written by
tests/golden/make_ensemble_d12_golden.py from the oracle alone).

- Each stored D_12 agrees with the diffusive root of the linearised scheme
  (Sec. 5.1, eqs. dd1 - dd6 at the member's uniform state and wavelength)
  within 5e-4: the mode's amplitude 0.05 leaves the decay linear.
- The golden script runs each member on nx x 1 x 1.  A state that does not
  vary across y and z gives the same mode series on any periodic
  cross-section (the amplitude scales by ny nz): checked on nx x 3 x 2.
- Re-running one stored member reproduces its stored series bit for bit.
"""
import importlib.util
import json
import math
import os

import numpy as np
import pytest

import workloads as W
from linear_scheme import LinearScheme

HERE = os.path.dirname(os.path.abspath(__file__))
GOLDEN = os.path.join(HERE, "golden", "ensemble_d12_members.json")


def _script():
    spec = importlib.util.spec_from_file_location("make_ensemble_d12_golden",
                                                  os.path.join(HERE, "golden", "make_ensemble_d12_golden.py"))
    mod = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mod)
    return mod


def _golden():
    with open(GOLDEN) as fh:
        return json.load(fh)


def test_stored_d12_matches_linearised_scheme():
    g = _golden()
    assert len(g["members"]) == 6
    for r in g["members"]:
        n = W.number_density(r["packing"], (r["x1"], 1 - r["x1"]), r["sigma"])
        D_lin = LinearScheme(r["sigma"], [n * r["x1"], n * (1 - r["x1"])]).diffusion(r["shape"][0])
        assert abs(r["d12"] / D_lin - 1) < 5e-4, (r["member"], r["d12"], D_lin)


def test_mode_series_does_not_depend_on_the_cross_section(oracle_lib):
    mem = W.config_ensemble()[3]
    m0 = mem.mixture
    series = []
    for ny, nz in ((1, 1), (3, 2)):
        m = W.Mixture(m0.nx, ny, nz, sigma=m0.sigma, tau=m0.tau)
        n0 = np.ascontiguousarray(np.broadcast_to(mem.n0[:, :1, :1, :], (m.M, nz, ny, m.nx)))
        u0 = np.ascontiguousarray(np.broadcast_to(mem.u0[:, :, :1, :1, :], (m.M, 3, nz, ny, m.nx)))
        o = oracle_lib.Oracle(m)
        f = o.step(o.init(n0, u0), 60)
        n = o.densities(f)
        k = 2 * math.pi / m.nx
        series.append(np.abs(np.sum((n[0] - n[1]).sum(axis=(0, 1)) * np.exp(-1j * k * np.arange(m.nx)))) / (ny * nz))
        assert np.ptp(n[0], axis=(0, 1)).max() == 0.0             # still uniform across the section
    assert series[1] == pytest.approx(series[0], rel=1e-13)


def test_stored_member_reproduces(oracle_lib):
    g = _golden()
    r = min(g["members"], key=lambda r: r["sites"])
    mem = W.config_ensemble()[r["member"]]
    ts, amps = _script().mode_series(mem, steps=200)
    # bit for bit: the series were stored by the same arithmetic
    np.testing.assert_array_equal(amps, np.asarray(r["amplitude"])[:len(amps)])
    np.testing.assert_array_equal(ts, np.asarray(r["t"])[:len(ts)])
