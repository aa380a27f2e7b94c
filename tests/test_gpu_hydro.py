"""GPU runs of the paper's hydrodynamic and Taylor-dispersion experiments,
through the C ABI, against the oracle and the linearised scheme.

- Body force per lattice row (the y-periodic force that drives the
  modulated shear flow of Sec. 5.2, eq. ushape): float64 bit-exact against
  the oracle, float32 densities within 1e-5 after 60 steps.
- A uniform mixture at rest stays bitwise stationary for 1000 steps.
- The single-species mode record (the tracer's section-averaged mode of
  Sec. 5.2) against numpy on the oracle's densities, and the fit quality
  the library reports against numpy's.
- Float32 runs of the modes of Sec. 4.2 (shear wave, transverse w, sound)
  against the linearised scheme's evolution of the same initial amplitudes;
  the composition mode oscillating above q_c and not below (Sec. 5.1); the
  steady modulated flow under a cosine body force; and the Taylor D_eff of a
  composition mode in that flow against the passive-scalar eigenvalue
  (eqs. c99, taylordiff).
"""
import math

import numpy as np
import pytest

import workloads as W
from linear_scheme import LinearScheme, hydrodynamics, taylor_passive_scalar

pytestmark = pytest.mark.gpu

KT = 1.0 / 3.0


def _gpu(m, n0, u0, precision, **kw):
    import paper_1105_3634_amd as mlb
    return mlb.GpuMixture(m, n0, u0, precision=precision, **kw)


def _np(t):
    return t.detach().cpu().numpy().astype(np.float64)


def _state(sigma, xi, x1=0.5):
    x = np.array([x1, 1 - x1])
    return W.number_density(xi, x, sigma) * x


def _profile_case(name):
    rng = np.random.default_rng(7)
    if name == "walled_ternary":
        m = W.Mixture(12, 14, 10, sigma=(2.0, 3.0, 2.5), eps=np.full((3, 3), 0.1), rc_factor=1.5, walls_y=True,
                      wall_ux=(-0.02, 0.03), fext=np.array([[1e-5, 0, 0], [0, 0, -1e-5], [0, 2e-5, 0]]))
        n0, u0 = W.random_state(m, [0.012, 0.008, 0.005], rel=0.3, u_amp=0.02, seed=51)
    else:
        m = W.Mixture(16, 24, 8, sigma=(2.0, 3.0))
        n0, u0 = W.random_state(m, [0.012, 0.008], rel=0.3, u_amp=0.02, seed=52)
    prof = rng.uniform(-2e-4, 2e-4, size=(m.M, 3, m.ny))
    return m, n0, u0, prof


@pytest.mark.parametrize("name", ["walled_ternary", "periodic_binary"])
def test_force_profile_parity(oracle_lib, name):
    m, n0, u0, prof = _profile_case(name)
    o = oracle_lib.Oracle(m)
    o.set_force_profile(prof)
    f_ref = o.step(o.init(n0, u0), 10)
    print(f"[profile] case={name} precision=64", flush=True)
    g = _gpu(m, n0, u0, 64)
    g.set_force_profile(prof)
    g.step(10)
    assert np.array_equal(_np(g.populations()), f_ref)
    # removing the profile returns to the uniform force: both sides again
    o.set_force_profile(None)
    g.set_force_profile(None)
    f_ref = o.step(f_ref, 4)
    g.step(4)
    assert np.array_equal(_np(g.populations()), f_ref)
    print(f"[profile] case={name} precision=32", flush=True)
    o.set_force_profile(prof)
    n_ref = o.densities(o.step(o.init(n0, u0), 60))
    g = _gpu(m, n0, u0, 32)
    g.set_force_profile(prof)
    g.step(60)
    n = _np(g.moments()[0])
    err = max(np.abs(n[a] - n_ref[a]).max() / np.abs(n_ref[a]).max() for a in range(m.M))
    print(f"  float32 density error {err:.2e}", flush=True)
    assert err < 1e-5


@pytest.mark.parametrize("precision,tail", [(64, "none"), (64, "direct"), (32, "none"), (32, "direct"),
                                            (32, "spectral")])
def test_uniform_mixture_stationary_for_1000_steps(precision, tail):
    """After the density sums reach their rounding fixed point (20 steps), 1000
    more steps return the same populations bit for bit: every +-e pair sum
    cancels exactly, so no force and no momentum appear.  Float32 with the
    spectral attractive field is the exception: its transforms leave rounding
    noise in the field of a uniform density, so there the velocity stays
    within float32 rounding of zero instead."""
    eps = None if tail == "none" else np.full((2, 2), 0.1)
    mode = {"none": 0, "direct": 1, "spectral": 2}[tail]
    m = W.Mixture(16, 12, 10, sigma=(2.0, 3.0), eps=eps, rc_factor=1.5)
    n0, u0 = W.uniform_state(m, [0.015, 0.008])
    print(f"[stationary] precision={precision} tail={tail}", flush=True)
    g = _gpu(m, n0, u0, precision, tail_mode=mode)
    g.step(20)
    f0 = _np(g.populations())
    g.step(1000)
    f = _np(g.populations())
    n, j = (_np(t) for t in g.moments())
    if tail == "spectral":
        umax = np.abs(j).max() / n.max()
        print(f"  spectral field: max |u| {umax:.2e}", flush=True)
        assert umax < 1e-6
        return
    assert np.array_equal(f, f0)
    assert not j.any()


def test_tracer_mode_record_and_fit_quality(oracle_lib):
    """|sum_r n_a exp(-i 2 pi x / nx)| of one species (b = -1) on the GPU
    against numpy on the oracle's densities; the fit's slope, sample count and
    R^2 against numpy's over the same window."""
    m, n0, u0 = W.config_taylor_couette(48, 20, 12)
    tracer, every, samples = 2, 10, 8
    k = 2 * np.pi / m.nx
    x = np.arange(m.nx)
    o = oracle_lib.Oracle(m)
    f = o.init(n0, u0)
    ref = []
    for j in range(samples):
        dn = o.densities(f)[tracer].sum(axis=(0, 1))
        ref.append(np.hypot((dn * np.cos(k * x)).sum(), (dn * np.sin(k * x)).sum()))
        if j + 1 < samples:
            f = o.step(f, every)
    ref = np.array(ref)
    for prec, tol in ((64, 1e-12), (32, 1e-5)):
        print(f"[tracer mode] precision={prec}", flush=True)
        g = _gpu(m, n0, u0, prec)
        g.reset_series()
        for j in range(samples):
            g.record_mode(tracer, -1)
            if j + 1 < samples:
                g.step(every)
        t, v = g.series()
        err = np.abs(v - ref).max() / ref[0]
        print(f"  amplitude rel err {err:.2e}", flush=True)
        assert err < tol
        q = g.fit_ex(0, 0.0)
        lv = np.log(v)
        slope, icpt = np.polyfit(t, lv, 1)
        r2 = 1 - np.sum((lv - (icpt + slope * t)) ** 2) / np.sum((lv - lv.mean()) ** 2)
        assert q["samples"] == samples
        assert abs(q["slope"] - slope) <= 1e-9 * abs(slope)
        assert abs(q["r2"] - r2) <= 1e-9
        assert q["well_conditioned"] == (r2 >= 0.98)


# ------------------------------------------------------- modes of Sec. 4.2
def _series(g, every, count, fn):
    out = []
    for i in range(count):
        n, j = (_np(t) for t in g.moments())
        out.append(fn(n, j))
        if i + 1 < count:
            g.step(every)
    return np.array(out)


def _amp(field, k):
    """exp(-i k x) amplitude of a [nz][ny][nx] field averaged over y and z."""
    prof = field.mean(axis=(0, 1))
    L = prof.shape[0]
    return 2.0 / L * np.sum(prof * np.exp(-1j * k * np.arange(L)))


CONF1 = ((2.0, 3.0), 0.2)


def test_shear_wave_decay():
    """u_y = U cos(k x) on both species: the momentum wave decays at nu k^2
    (eq. dd3), nu = (eta^K + eta^C) / rho; the float32 run follows the
    linearised scheme's evolution."""
    sigma, xi = CONF1
    n0 = _state(sigma, xi)
    L, U, every, count = 64, 1e-3, 10, 41
    k = 2 * math.pi / L
    lin = LinearScheme(sigma, n0)
    m = W.Mixture(L, 4, 4, sigma=sigma)
    n, u = W.uniform_state(m, n0)
    u[:, 1] = U * np.cos(k * np.arange(L))[None, None, None, :]
    print("[shear wave] 64x4x4 float32", flush=True)
    g = _gpu(m, n, u, 32)
    amps = _series(g, every, count, lambda n_, j: _amp(j[:, 1].sum(0), k))
    T = np.linalg.matrix_power(lin.transverse(k), every)
    v = n0 * U + 0j
    pred = []
    for _ in range(count):
        pred.append(v.sum())
        v = T @ v
    pred = np.array(pred)
    err = np.abs(amps - pred).max() / abs(pred[0])
    t = every * np.arange(count)
    nu = -np.polyfit(t[5:], np.log(np.abs(amps[5:])), 1)[0] / k ** 2
    print(f"  max deviation {err:.2e}; nu fit {nu:.5f} linear {lin.shear_viscosity(L):.5f} "
          f"paper {lin.paper_viscosity():.5f}", flush=True)
    assert err < 2e-3
    assert abs(nu / lin.shear_viscosity(L) - 1) < 3e-3


def test_transverse_w_decay():
    """u_A - u_B transverse, zero barycentric velocity: decays at the friction
    rate (eq. dd5) through the Crank-Nicolson factor."""
    sigma, xi = CONF1
    n0 = _state(sigma, xi)
    L, W0, count = 64, 1e-3, 9
    k = 2 * math.pi / L
    lin = LinearScheme(sigma, n0)
    c = n0 / n0.sum()
    m = W.Mixture(L, 4, 4, sigma=sigma)
    n, u = W.uniform_state(m, n0)
    prof = np.cos(k * np.arange(L))[None, None, :]
    u[0, 1] = W0 * c[1] * prof
    u[1, 1] = -W0 * c[0] * prof
    print("[transverse w] 64x4x4 float32", flush=True)
    g = _gpu(m, n, u, 32)
    w = _series(g, 1, count, lambda n_, j: _amp(j[0, 1] / n_[0] - j[1, 1] / n_[1], k))
    T = lin.transverse(k)
    v = np.array([n0[0] * W0 * c[1], -n0[1] * W0 * c[0]]) + 0j
    pred = []
    for _ in range(count):
        pred.append(v[0] / n0[0] - v[1] / n0[1])
        v = T @ v
    pred = np.array(pred)
    err = np.abs(w - pred).max() / abs(pred[0])
    h = hydrodynamics(lin)
    rate = -math.log(abs(w[4] / w[3]))
    print(f"  max deviation {err:.2e}; rate per step {rate:.4f}, gamma {h['gamma']:.4f}", flush=True)
    assert err < 2e-3


@pytest.mark.parametrize("sigma,xi,x1,eps", [((2.0, 3.0), 0.2, 0.5, None), ((3.0, 4.5), 0.3, 0.5, 0.5 * KT)])
def test_sound_wave(sigma, xi, x1, eps):
    """A total-density wave at fixed composition oscillates at c_s k and decays
    at Gamma k^2 (eqs. cc1-cc2, damping); float32 run against the linearised
    scheme."""
    n0 = _state(sigma, xi, x1)
    L = 128 if eps else 64
    ny = 12 if eps else 4
    k = 2 * math.pi / L
    e = None if eps is None else np.full((2, 2), eps)
    lin = LinearScheme(sigma, n0, eps=e)
    m = W.Mixture(L, ny, ny, sigma=sigma, eps=e)
    n, u = W.uniform_state(m, n0)
    d = 1e-3
    n *= 1 + d * np.cos(k * np.arange(L))[None, None, None, :]
    every, count = 2, 60
    print(f"[sound] sigma={sigma} {L}x{ny}x{ny} float32", flush=True)
    g = _gpu(m, n, u, 32)
    amps = _series(g, every, count, lambda n_, j: _amp(n_.sum(0), k))
    T = np.linalg.matrix_power(lin.longitudinal(k), every)
    v = np.concatenate([n0 * d, [0, 0]]) + 0j
    pred = []
    for _ in range(count):
        pred.append(v[0] + v[1])
        v = T @ v
    pred = np.array(pred)
    err = np.abs(amps - pred).max() / abs(pred[0])
    h = hydrodynamics(lin)
    print(f"  max deviation {err:.2e}; c_s {h['cs']:.4f}, Gamma {h['Gamma']:.4f}", flush=True)
    assert err < 3e-3


def test_composition_mode_oscillates_above_qc():
    """Dilute equal-diameter binary (packing 0.02): wavelength 96 (q > q_c)
    overshoots zero, wavelength 192 (q < q_c) decays monotonically (Sec. 5.1)."""
    sigma, xi = (2.0, 2.0), 0.02
    n = W.number_density(xi, (0.5, 0.5), sigma)
    for L, osc in ((96, True), (192, False)):
        m = W.Mixture(L, 4, 4, sigma=sigma)
        print(f"[q_c] wavelength {L}", flush=True)
        g = _gpu(m, *W.mode_state(m, n, 0.5, 1e-3), 32)
        x = np.arange(L)
        proj = _series(g, 5, 80, lambda n_, j: float(np.sum((n_[0] - n_[1]).mean(axis=(0, 1)) *
                                                             np.sin(2 * math.pi * x / L))))
        assert np.any(proj < 0) == osc


def kolmogorov(m, F0):
    prof = np.zeros((m.M, 3, m.ny))
    prof[:, 0, :] = F0 * np.cos(2 * math.pi * np.arange(m.ny) / m.ny)[None, :]
    return prof


def test_kolmogorov_flow_amplitude():
    """Steady flow under the body force F cos(2 pi y / Ly) (float32) against
    the fixed point of the linearised scheme."""
    sigma, xi = CONF1
    n0 = _state(sigma, xi)
    Ly = 64
    k = 2 * math.pi / Ly
    lin = LinearScheme(sigma, n0)
    U = 0.02
    F0 = U / lin.transverse_forced(k).sum() * n0.sum()
    m = W.Mixture(4, Ly, 4, sigma=sigma)
    n, u = W.uniform_state(m, n0)
    print("[kolmogorov] 4x64x4 float32", flush=True)
    g = _gpu(m, n, u, 32)
    g.set_force_profile(kolmogorov(m, F0))
    g.step(int(20 / (lin.shear_viscosity(Ly) * k * k)))
    nn, j = (_np(t) for t in g.moments())
    ux = j[:, 0].sum(0) / nn.sum(0)
    amp = 2.0 / Ly * float((ux.mean(axis=(0, 2)) * np.cos(k * np.arange(Ly))).sum())
    print(f"  amplitude {amp:.6e} predicted {U:.6e}", flush=True)
    assert abs(amp / U - 1) < 2e-3


def test_taylor_dispersion():
    """Composition mode along x in the steady modulated flow (Sec. 5.2):
    D_eff from the library's mode record and fit against the passive-scalar
    eigenvalue for the measured flow, and against the flow-free D."""
    sigma, xi = (3.0, 4.5), 0.3
    n0 = _state(sigma, xi)
    Lx, Ly, nz = 128, 32, 6
    lin = LinearScheme(sigma, n0)
    k = 2 * math.pi / Ly
    res = {}
    for U in (0.0, 0.06):
        m = W.Mixture(Lx, Ly, nz, sigma=sigma)
        # amplitude 0.02: float32 rounding drift of the densities (relative
        # 1e-8 per step, proportional to the local density) would bias a 1e-3
        # mode by 10 % after 3000 steps
        n, u = W.mode_state(m, n0.sum(), 0.5, 0.02)
        u[:, 0] = U * np.cos(k * np.arange(Ly))[None, None, :, None]
        print(f"[taylor] U={U} {Lx}x{Ly}x{nz} float32", flush=True)
        g = _gpu(m, n, u, 32)
        F0 = U / lin.transverse_forced(k).sum() * n0.sum()
        g.set_force_profile(kolmogorov(m, F0))
        g.reset_series()
        for t in range(0, 3001, 20):
            g.record_mode(0, 1)
            g.step(20)
        q = g.fit_ex(0, 400.0)
        res[U] = q["D"]
        assert q["well_conditioned"]
    D = lin.diffusion(Lx)
    want = taylor_passive_scalar(D, 0.06, Ly, Lx)
    print(f"  D {res[0.0]:.5f} (linear {D:.5f}); D_eff {res[0.06]:.5f} passive scalar {want:.5f}", flush=True)
    assert abs(res[0.0] / D - 1) < 5e-3
    assert abs(res[0.06] / want - 1) < 0.02
    assert (res[0.06] - res[0.0]) > 0.2 * res[0.0]
