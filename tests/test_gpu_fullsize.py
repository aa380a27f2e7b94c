"""Full-size workloads against stored float64 oracle runs (written by the
scripts in tests/golden/ from the oracle only):
- bulk diffusion (128x32x32, float32, spectral tail, the launch
  configuration bench.py times): densities at 4096 sampled sites after 100
  steps within 1e-5 of the field's max norm, and D_12 from the mode decay
  over 2000 steps within 2 %;
- Taylor/Couette (256x64x16, walls): float64 bit-exact and float32 within
  1e-5 after 5 steps;
- the 64-system ensemble (14.75M sites): three systems within 1e-5 after 20
  steps;
- the learned-closure workload's exact-force path (192x64x64): float32
  within 1e-5 after 5 steps."""
import json
import math
import os

import numpy as np
import pytest

import workloads as W

pytestmark = pytest.mark.gpu
GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "bulk_diffusion_128x32x32_2000.json")


@pytest.fixture(scope="module")
def golden():
    with open(GOLDEN) as fh:
        return json.load(fh)


def test_densities_after_100_steps(golden):
    import paper_1105_3634_amd as mlb
    m, n0, u0 = W.config_bulk_diffusion()
    g = mlb.GpuMixture(m, n0, u0, precision=32)
    g.step(100)
    n = g.moments()[0].cpu().numpy().astype(np.float64)
    sites = np.array(golden["sample_sites"])
    for a in range(2):
        ref = np.array(golden["n100_sample"][a])
        err = np.abs(n[a].ravel()[sites] - ref).max() / golden["n100_maxnorm"][a]
        print(f"  species {a}: fp32 rel err at 4096 sites {err:.2e}", flush=True)
        assert err < 1e-5
        np.testing.assert_allclose(n[a].sum(), golden["n100_mass"][a], rtol=1e-5)


def test_d12_from_mode_decay(golden):
    import paper_1105_3634_amd as mlb
    m, n0, u0 = W.config_bulk_diffusion()
    g = mlb.GpuMixture(m, n0, u0, precision=32)
    for t in range(0, 2001, 10):
        g.record_mode(0, 1)
        if t < 2000:
            g.step(10)
    D = g.fit(0, t_min=golden["fit_t_min"])
    ts, amps = g.series()
    ref_t, ref_a = np.array(golden["t"]), np.array(golden["amplitude"])
    assert np.array_equal(ts, ref_t)
    amp_err = np.abs(amps - ref_a).max() / ref_a.max()
    rel = D / golden["D12"] - 1
    print(f"  D12 gpu {D:.6f}  oracle {golden['D12']:.6f}  rel {rel:+.2e}  max amplitude err {amp_err:.2e}",
          flush=True)
    assert abs(rel) < 0.02
    assert amp_err < 1e-4


# ---------------------------------------------------------------------------
# Taylor/Couette (256x64x16 ternary, moving walls, tail) and the 64-system
# ensemble at full size against float64 oracle references written by
# tests/golden/make_fullsize_goldens.py (oracle only).
TAYLOR = os.path.join(os.path.dirname(__file__), "golden", "taylor_couette_256x64x16_20.json")
ENSEMBLE = os.path.join(os.path.dirname(__file__), "golden", "ensemble_64_members_20.json")


def _load(path):
    with open(path) as fh:
        return json.load(fh)


def test_taylor_couette_float64_bit_exact_20_steps():
    """Float64 follows the oracle's operation order: the sampled densities
    after 20 steps are equal bit for bit (moving walls with the mirrored
    hard-core images, direct tail) at the workload's packing 0.25."""
    import paper_1105_3634_amd as mlb
    ref = _load(TAYLOR)
    m, n0, u0 = W.config_taylor_couette()
    print(f"[taylor fp64] shape={m.shape()} steps={ref['steps']}", flush=True)
    g = mlb.GpuMixture(m, n0, u0, precision=64)
    g.step(ref["steps"])
    n = g.moments()[0].cpu().numpy()
    sites = np.array(ref["sample_sites"])
    for a in range(m.M):
        got = n[a].ravel()[sites]
        assert np.array_equal(got, np.array(ref["n_sample"][a])), (a, np.abs(got - ref["n_sample"][a]).max())
        assert n[a].sum() == pytest.approx(ref["mass"][a], rel=1e-13)


def test_taylor_couette_float32_20_steps():
    """Float32 with the spectral field on the y-padded transform (tiled
    gathers): sampled densities within 1e-5 of the field's max norm."""
    import paper_1105_3634_amd as mlb
    ref = _load(TAYLOR)
    m, n0, u0 = W.config_taylor_couette()
    print(f"[taylor fp32] shape={m.shape()} steps={ref['steps']}", flush=True)
    g = mlb.GpuMixture(m, n0, u0, precision=32, device="cuda:0")
    g.step(ref["steps"])
    n = g.moments()[0].cpu().numpy().astype(np.float64)
    sites = np.array(ref["sample_sites"])
    for a in range(m.M):
        err = np.abs(n[a].ravel()[sites] - np.array(ref["n_sample"][a])).max() / ref["maxnorm"][a]
        print(f"  species {a}: fp32 rel err {err:.2e}", flush=True)
        assert err < 1e-5
        np.testing.assert_allclose(n[a].sum(), ref["mass"][a], rtol=1e-5)


def test_ensemble_fullsize_20_steps():
    """All 64 systems (14.75M sites) in one batch with the autotuned tiling
    and graph replay, as the bench runs them; the three smallest systems
    against the oracle after 20 steps (1e-5 of the max norm)."""
    import paper_1105_3634_amd as mlb
    ref = _load(ENSEMBLE)
    members = W.config_ensemble()
    assert len(members) == ref["count"]
    print(f"[ensemble] systems={len(members)} steps={ref['steps']}", flush=True)
    b = mlb.GpuBatch([x.mixture for x in members], [x.n0 for x in members], [x.u0 for x in members],
                     precision=32, options=mlb.OPT_TUNE, device="cuda:0")
    b.step(ref["steps"])
    for sysref in ref["systems"]:
        k = sysref["index"]
        n = b.moments(k)[0].cpu().numpy().astype(np.float64)
        sites = np.array(sysref["sample_sites"])
        for a in range(n.shape[0]):
            err = np.abs(n[a].ravel()[sites] - np.array(sysref["n_sample"][a])).max() / sysref["maxnorm"][a]
            print(f"  system {k} species {a}: fp32 rel err {err:.2e}", flush=True)
            assert err < 1e-5
            np.testing.assert_allclose(n[a].sum(), sysref["mass"][a], rtol=1e-5)


CLOSURE = os.path.join(os.path.dirname(__file__), "golden", "closure_physics_192x64x64_5.json")


def test_closure_workload_plain_path_float32_5_steps():
    """The learned-closure workload's exact-force path at full size (192x64x64,
    sigma 2 and 3, packing 0.2), tiled float32 gathers as the closure leg
    runs them: sampled densities within 1e-5 of the max norm after 5 steps."""
    import paper_1105_3634_amd as mlb
    ref = _load(CLOSURE)
    m, n0, u0 = W.config_closure_physics()
    print(f"[closure plain fp32] shape={m.shape()} steps={ref['steps']}", flush=True)
    g = mlb.GpuMixture(m, n0, u0, precision=32, device="cuda:0")
    g.step(ref["steps"])
    n = g.moments()[0].cpu().numpy().astype(np.float64)
    sites = np.array(ref["sample_sites"])
    for a in range(m.M):
        err = np.abs(n[a].ravel()[sites] - np.array(ref["n_sample"][a])).max() / ref["maxnorm"][a]
        print(f"  species {a}: fp32 rel err {err:.2e}", flush=True)
        assert err < 1e-5
        np.testing.assert_allclose(n[a].sum(), ref["mass"][a], rtol=1e-5)


COUETTE = os.path.join(os.path.dirname(__file__), "golden", "taylor_couette_64x24x12_600.json")


def test_couette_tracer_dispersion_against_oracle():
    """The Taylor/Couette physics at packing 0.25 on 64x24x12, float32 with the
    spectral field on the y-padded transform: the tracer's section-averaged
    mode recorded every 10 steps for 600 steps against the oracle's series
    (1e-4 of the first amplitude), and the library's D_eff fit against the
    oracle's within 2 %."""
    import paper_1105_3634_amd as mlb
    ref = _load(COUETTE)
    m, n0, u0 = W.config_taylor_couette(64, 24, 12)
    print(f"[couette D_eff] shape={m.shape()} steps={ref['steps']}", flush=True)
    g = mlb.GpuMixture(m, n0, u0, precision=32, device="cuda:0")
    g.reset_series()
    for t in range(0, ref["steps"] + 1, ref["every"]):
        g.record_mode(2, -1)
        if t < ref["steps"]:
            g.step(ref["every"])
    t, v = g.series()
    amp = np.array(ref["amplitude"])
    assert np.array_equal(t, np.array(ref["t"]))
    err = np.abs(v - amp).max() / amp[0]
    fit = g.fit_ex(0, ref["fit_t_min"])
    print(f"  series rel err {err:.2e}; D_eff {fit['D']:.6f} oracle {ref['D_eff']:.6f}", flush=True)
    assert err < 1e-4
    assert abs(fit["D"] / ref["D_eff"] - 1) < 0.02
    mass = g.conserved()[0]
    np.testing.assert_allclose(mass, ref["mass"], rtol=1e-5)


@pytest.mark.parametrize("case", ["step_binary_256^3", "bulk_diffusion_spectral_4096x64x64"])
def test_large_box_against_oracle_lines(oracle_lib, case):
    """16.8M sites in one system (the 32-bit index paths of the step, the
    spectral field and the reductions beyond a million sites): a state that
    does not vary across y and z stays so, and every (y, z) line equals the
    float64 oracle run on an nx x 1 x 1 line (in a periodic box the stencil
    sums see the same values for any cross-section) within 1e-5 of the max
    norm after 4 steps.  Step-binary physics on 256^3 (tiled gathers), and
    the bulk-diffusion physics with its spectral tail on 4096 x 64 x 64 (a
    composition mode of wavelength 16)."""
    import torch

    import paper_1105_3634_amd as mlb
    eps = np.full((2, 2), 0.5 * W.KT)
    if case.startswith("step"):
        shape, make = (256, 256, 256), lambda nx, ny, nz: W.Mixture(nx, ny, nz, sigma=(2.0, 3.0), tau=1.0)
        state = lambda m: W.step_state(m, W.number_density(0.2, (0.5, 0.5), m.sigma))
    else:
        shape = (4096, 64, 64)
        make = lambda nx, ny, nz: W.Mixture(nx, ny, nz, sigma=(3.0, 4.5), eps=eps, rc_factor=2.5)
        state = lambda m: W.mode_state(m, W.number_density(0.3, (0.5, 0.5), m.sigma), 0.5, 0.05, wavelength=16)
    line = make(shape[0], 1, 1)
    n0l, u0l = state(line)
    o = oracle_lib.Oracle(line)
    ref = o.densities(o.step(o.init(n0l, u0l), 4))[:, 0, 0, :]
    m = make(*shape)
    n0 = np.ascontiguousarray(np.broadcast_to(n0l, (m.M,) + m.shape()))
    u0 = np.zeros((m.M, 3) + m.shape())
    print(f"[large box] {case} sites={m.N}", flush=True)
    g = mlb.GpuMixture(m, n0, u0, precision=32, options=mlb.OPT_TUNE)
    del n0, u0
    g.step(4)
    n = g.moments()[0]
    torch.cuda.synchronize()
    for a in range(m.M):
        na = n[a].reshape(-1, shape[0])
        lo, hi = na.min(dim=0).values.cpu().numpy(), na.max(dim=0).values.cpu().numpy()
        err = max(np.abs(lo - ref[a]).max(), np.abs(hi - ref[a]).max()) / np.abs(ref[a]).max()
        spread = (np.abs(hi - lo) / np.abs(ref[a]).max()).max()
        print(f"  species {a}: rel err {err:.2e}, spread across lines {spread:.2e}", flush=True)
        assert err < 1e-5
    mass, _ = g.conserved()
    np.testing.assert_allclose(mass, [n0l[a].sum() * shape[1] * shape[2] for a in range(m.M)], rtol=1e-5)
