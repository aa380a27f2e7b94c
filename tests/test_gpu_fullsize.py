"""Full-size bulk-diffusion workload (128x32x32, float32, spectral tail, the
launch configuration bench.py times) against the stored float64 oracle run
(tests/golden/bulk_diffusion_128x32x32_2000.json, written by
tests/golden/make_bulk_diffusion_golden.py from the oracle only):
densities at 4096 sampled sites after 100 steps within 1e-5 of the field's
max norm, and D_12 from the mode decay over 2000 steps within 2 %."""
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
